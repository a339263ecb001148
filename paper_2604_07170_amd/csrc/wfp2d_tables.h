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
// eta_d(r) from the table with the same sub-panel lookup as the local kernel
void local_table_eval(const LocalTable &T, double dt, int W, double r, double *out);

double es_kernel(double z, int w, double beta);
void es_fourier(int w, double beta, int64_t nf, int64_t R, std::vector<double> &out);

}  // namespace wfp2d
