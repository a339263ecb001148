// Host-side precomputation for wfp2d (FP64).  Internal.
#pragma once

#include <cstdint>
#include <vector>

#include "wfp2d_internal.h"

namespace wfp2d {

void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w);
double bessel_i0(double x);

// The blending function phi_width of eq. KBblending with shape b, held as
// Chebyshev series of phi' and of its antiderivative phi on [0, width].
struct Blend {
    double width, b;
    std::vector<double> cd, ci;
    Blend(double width, double b, int deg = 160);
    double phi(double t) const;
    double dphi(double t) const;
    double dphi_exact(double t) const;
};

struct Params {
    double dt, tol, b, delta, Delta, A, Aplus, a, dk, K, Kf, Kmax;
    int64_t LA, R;
    int W, p, lookahead;
};

Params derive_params(double dt, int W, double tol, double Delta, double a_in, double Kf, int p,
                     int lookahead_in);

void soe_nodes(std::vector<double> &lam, std::vector<double> &q);
// Quadrature of eq. H in r (composite Gauss-Legendre, panels of width 0.02, 16 nodes): nodes r[g]
// and E[l][g] = q_l I0(lambda_l r_g) e^{-A lambda_l} phi_Delta(A - r_g) r_g w_g, so that
// H_l(kappa) = sum_g J0(kappa r_g) E[l][g] (the contraction runs on the device in a plan)
void hankel_quadrature(double A, double Delta, double b_Delta, const std::vector<double> &lam, const std::vector<double> &q,
                       std::vector<double> &r, std::vector<double> &E);
void hankel_table(const std::vector<double> &kappa, double A, double Delta, double b_Delta,
                  const std::vector<double> &lam, const std::vector<double> &q, std::vector<double> &H);

int stencil_start(int k, int p, int lev_min);

// eta_d(r) by direct quadrature (used to build and to check the tables)
struct LocalWeights {
    double dt;
    int W, p, lev_min, nlev;
    const Blend &phi;
    std::vector<double> gx, gw, bary;
    LocalWeights(double dt, int W, int p, int lev_min, const Blend &phi);
    void eta(double r, double *out /* [nlev] */) const;
};

struct LocalTable {
    int nlev = 0, dy_base = 0, n_dy = 0;
    std::vector<int32_t> panel_base, panel_l2n;
    std::vector<SubPanel> subs;
    std::vector<double> coef;   // [n_sub][nlev][kChebDeg]
    double max_err = 0.0;
};

LocalTable build_local_table(const LocalWeights &LW, int n_dy, double rel_tol);
// eta_d(r) from the table with the same sub-panel lookup as the local kernel; the regular
// sub-panels (index < dy_base) use their leading nterm_regular coefficients
void local_table_eval(const LocalTable &T, double dt, int W, double r, double *out, int nterm_regular = kChebDeg);

// Leading Chebyshev terms kept on the regular sub-panels by a mixed-precision plan: the
// smallest of 12, 14, 16 for which the dropped terms' bound (per sub-panel, the sum over the
// dropped terms of their largest magnitude over levels; the worst sub-panel) is at most
// 1e-3 tol times the largest coefficient of the table, else kChebDeg.  Since |T_c| <= 1 on
// [-1, 1], that bound also bounds the change of every eta_d.  tail_out and cmax_out (if not
// NULL) receive the bound for the returned count and the largest coefficient.
int local_table_terms(const LocalTable &T, double tol, double *tail_out = nullptr, double *cmax_out = nullptr);
// Power-basis form of a truncated Chebyshev series on [-1, 1]: a[c] (c < nt) with
// sum_{j<nt} b[j] T_j(x) = sum_{c<nt} a[c] x^c, from the integer coefficients of T_j
// (T_0 = 1, T_1 = x, T_{j+1} = 2x T_j - T_{j-1}).
void cheb_to_power(const double *b, int nt, double *a);
// eta_d(r) as the pair-list local kernel evaluates it: the regular sub-panels' series
// truncated to nterm_regular terms and summed in the power basis by Horner's rule
// (the dyadic sub-panels as local_table_eval).
void local_table_eval_power(const LocalTable &T, double dt, int W, double r, double *out, int nterm_regular);

double es_kernel(double z, int w, double beta);
void es_fourier(int w, double beta, int64_t nf, int64_t R, std::vector<double> &out);

}  // namespace wfp2d
