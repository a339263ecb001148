// Host-side precomputation of the wfp2d plan: parameters, blending functions,
// sum-of-exponentials nodes, Hankel coefficients, far-history FIR taps, local
// singular-quadrature weight tables and NUFFT kernel tables.  FP64 throughout.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <vector>

#include "wfp2d_tables.h"

namespace wfp2d {

// ---------------------------------------------------------------------------
// Gauss-Legendre nodes/weights on [-1, 1] (Newton iteration on P_n).
// ---------------------------------------------------------------------------
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Modified Bessel I0 by its power series (all terms positive; fine to x ~ 700).
double bessel_i0(double x)
{
    const double q = 0.25 * x * x;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 2000; ++k) {
        term *= q / (double(k) * double(k));
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    return sum;
}

// ---------------------------------------------------------------------------
// Kaiser-Bessel blending function (eq. KBblending) as Chebyshev series on
// [0, width]: phi' sampled, phi obtained by integrating the series.
// ---------------------------------------------------------------------------
Blend::Blend(double width_, double b_, int deg) : width(width_), b(b_)
{
    const int n = deg;
    std::vector<double> f(n);
    for (int q = 0; q < n; ++q) {
        double x = std::cos(M_PI * (q + 0.5) / n);
        f[q] = dphi_exact(0.5 * width * (x + 1.0));
    }
    cd.assign(n, 0.0);
    for (int k = 0; k < n; ++k) {
        double s = 0.0;
        for (int q = 0; q < n; ++q) s += f[q] * std::cos(M_PI * k * (q + 0.5) / n);
        cd[k] = 2.0 * s / n;
    }
    cd[0] *= 0.5;
    // antiderivative in x (t = width (x+1)/2, dt = width/2 dx): C_k = (c_{k-1} - c_{k+1}) / (2k)
    ci.assign(n + 1, 0.0);
    for (int k = 1; k <= n; ++k) {
        double cm = (k - 1 == 0) ? 2.0 * cd[0] : cd[k - 1];
        double cp = (k + 1 < n) ? cd[k + 1] : 0.0;
        ci[k] = 0.5 * width * (cm - cp) / (2.0 * k);
    }
    // choose C_0 so that phi(0) = 0 (x = -1: T_k(-1) = (-1)^k)
    double s = 0.0;
    for (int k = 1; k <= n; ++k) s += ci[k] * ((k & 1) ? -1.0 : 1.0);
    ci[0] = -s;
}

double Blend::dphi_exact(double t) const
{
    if (t < 0.0 || t > width) return 0.0;
    double z = 2.0 * t / width - 1.0;
    double a = std::max(0.0, 1.0 - z * z);
    return b / (width * std::sinh(b)) * bessel_i0(b * std::sqrt(a));
}

static double clenshaw(const std::vector<double> &c, double x)
{
    double b1 = 0.0, b2 = 0.0;
    for (int k = (int)c.size() - 1; k >= 1; --k) {
        double b0 = 2.0 * x * b1 - b2 + c[k];
        b2 = b1;
        b1 = b0;
    }
    return x * b1 - b2 + c[0];
}

double Blend::phi(double t) const
{
    if (t <= 0.0) return 0.0;
    if (t >= width) return 1.0;
    return clenshaw(ci, 2.0 * t / width - 1.0);
}

double Blend::dphi(double t) const
{
    if (t < 0.0 || t > width) return 0.0;
    return clenshaw(cd, 2.0 * t / width - 1.0);
}

// ---------------------------------------------------------------------------
// Parameters (Sec. 2.1, eqs. W, A, Ap, dk, K; readings recorded in the design
// notes: a by the SOE-accuracy rule, A+ rounded so that (A+ - delta)/dt is an
// integer, dk = 2 pi / (A+ + 2 + delta), K = pi/dt).
// ---------------------------------------------------------------------------
Params derive_params(double dt, int W, double tol, double Delta, double a_in, double Kf, int p,
                     int lookahead_in)
{
    Params P;
    P.dt = dt;
    P.W = W;
    P.tol = tol;
    P.b = std::log(1.0 / tol);
    P.delta = W * dt;
    P.Delta = Delta;
    P.A = 2.0 * std::sqrt(2.0) + Delta;
    const double lambda_max = 36.0;
    double a = a_in > 0 ? a_in : std::max(1.0, P.delta + std::log(1e15) / lambda_max);
    P.LA = (int64_t)std::ceil((P.A + a - P.delta) / dt - 1e-9);
    P.Aplus = P.LA * dt + P.delta;
    P.a = P.Aplus - P.A;
    P.dk = 2.0 * M_PI / (P.Aplus + 2.0 + P.delta);
    P.K = M_PI / dt;
    P.Kf = Kf;
    P.Kmax = std::max(P.K, P.Kf);
    P.R = (int64_t)std::ceil(P.Kmax / P.dk - 1e-12);
    P.p = p;
    P.lookahead = lookahead_in < 0 ? ((p + 1) / 2 - 1) : lookahead_in;
    if (P.lookahead < 0) P.lookahead = 0;
    return P;
}

// ---------------------------------------------------------------------------
// Sum-of-exponentials quadrature of eq. LaplaceIntegral (Sec. 2.3): 20 panels
// [0, lmax/2^19], [lmax/2^19, lmax/2^18], ..., [lmax/2, lmax], 32 GL nodes each.
// ---------------------------------------------------------------------------
void soe_nodes(std::vector<double> &lam, std::vector<double> &q)
{
    const double lmax = 36.0;
    const int npan = 20, ng = 32;
    std::vector<double> x, w;
    gauss_legendre(ng, x, w);
    lam.clear();
    q.clear();
    std::vector<double> edges;
    edges.push_back(0.0);
    for (int k = npan - 1; k >= 0; --k) edges.push_back(lmax / std::ldexp(1.0, k));
    for (int pnl = 0; pnl < npan; ++pnl) {
        double a = edges[pnl], bb = edges[pnl + 1];
        for (int i = 0; i < ng; ++i) {
            lam.push_back(0.5 * (bb - a) * x[i] + 0.5 * (a + bb));
            q.push_back(0.5 * (bb - a) * w[i]);
        }
    }
}

// ---------------------------------------------------------------------------
// Hankel coefficients H_l(kappa; A) of eq. H for each kappa class:
//   H_l = q_l e^{-A lam_l} int_0^A J0(kappa r) I0(lam_l r) phi_Delta(A - r) r dr
// by composite Gauss-Legendre in r (panels of width 0.02, 16 nodes).
// ---------------------------------------------------------------------------
void hankel_quadrature(double A, double Delta, double b_Delta, const std::vector<double> &lam, const std::vector<double> &q,
                       std::vector<double> &r, std::vector<double> &E)
{
    Blend phiD(Delta, b_Delta, 200);
    std::vector<double> x, w;
    gauss_legendre(16, x, w);
    const int npan = (int)std::ceil(A / 0.02);
    const double h = A / npan;
    const int nr = npan * 16;
    std::vector<double> wr(nr);
    r.resize(nr);
    for (int pnl = 0; pnl < npan; ++pnl)
        for (int i = 0; i < 16; ++i) {
            r[pnl * 16 + i] = (pnl + 0.5) * h + 0.5 * h * x[i];
            wr[pnl * 16 + i] = 0.5 * h * w[i];
        }
    const int L = (int)lam.size();
    E.resize((size_t)L * nr);
#pragma omp parallel for schedule(static)
    for (int l = 0; l < L; ++l)
        for (int g = 0; g < nr; ++g)
            E[(size_t)l * nr + g] = q[l] * bessel_i0(lam[l] * r[g]) * std::exp(-A * lam[l]) *
                                    phiD.phi(A - r[g]) * r[g] * wr[g];
}

void hankel_table(const std::vector<double> &kappa, double A, double Delta, double b_Delta,
                  const std::vector<double> &lam, const std::vector<double> &q, std::vector<double> &H)
{
    std::vector<double> r, E;
    hankel_quadrature(A, Delta, b_Delta, lam, q, r, E);
    const int nr = (int)r.size(), L = (int)lam.size();
    const int64_t nk = (int64_t)kappa.size();
    H.assign((size_t)nk * L, 0.0);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t c = 0; c < nk; ++c) {
        std::vector<double> J(nr);
        for (int g = 0; g < nr; ++g) J[g] = j0(kappa[c] * r[g]);
        for (int l = 0; l < L; ++l) {
            const double *e = &E[(size_t)l * nr];
            double s = 0.0;
            for (int g = 0; g < nr; ++g) s += J[g] * e[g];
            H[(size_t)c * L + l] = s;
        }
    }
}

// ---------------------------------------------------------------------------
// Local-part weights (Sec. 6): eta_d(r) = int_r^delta L_d(tau) [1 - phi(tau)] /
// sqrt(tau^2 - r^2) dtau, where L_d is the Lagrange cardinal function of delay
// level d for the p-point stencil of the panel [k dt, (k+1) dt] holding tau.
// Each panel piece is integrated after tau = r cosh v (dtau/sqrt(tau^2-r^2) =
// dv), the substitution Sec. 6 uses for small r; here for every r.
// ---------------------------------------------------------------------------
int stencil_start(int k, int p, int lev_min)
{
    int d0 = (p % 2 == 0) ? (k - p / 2 + 1) : (k - (p - 1) / 2);
    return std::max(d0, lev_min);
}

LocalWeights::LocalWeights(double dt_, int W_, int p_, int lev_min_, const Blend &phi_)
    : dt(dt_), W(W_), p(p_), lev_min(lev_min_), phi(phi_)
{
    int dmax = lev_min;
    for (int k = 0; k < W; ++k) dmax = std::max(dmax, stencil_start(k, p, lev_min) + p - 1);
    nlev = dmax - lev_min + 1;
    gauss_legendre(24, gx, gw);
    // barycentric weights of p equispaced nodes: w_i = (-1)^i C(p-1, i) (up to a common factor)
    bary.assign(p, 0.0);
    double c = 1.0;
    for (int i = 0; i < p; ++i) {
        bary[i] = ((i & 1) ? -1.0 : 1.0) * c;
        c = c * (p - 1 - i) / (i + 1);
    }
}

void LocalWeights::eta(double r, double *out) const
{
    std::fill(out, out + nlev, 0.0);
    const double delta = W * dt;
    std::vector<double> lv(p);
    for (int k = 0; k < W; ++k) {
        double a = std::max(r, k * dt), bb = std::min((k + 1) * dt, delta);
        if (!(bb > a)) continue;
        double va = (a == r) ? 0.0 : std::acosh(a / r);
        double vb = std::acosh(bb / r);
        int nv = std::max(1, (int)std::ceil((vb - va) / 0.25));
        double hv = (vb - va) / nv;
        int d0 = stencil_start(k, p, lev_min);
        for (int iv = 0; iv < nv; ++iv) {
            for (int g = 0; g < (int)gx.size(); ++g) {
                double v = va + (iv + 0.5) * hv + 0.5 * hv * gx[g];
                double tau = r * std::cosh(v);
                double wt = 0.5 * hv * gw[g] * (1.0 - phi.phi(tau));
                // barycentric Lagrange basis at x = tau/dt over nodes d0..d0+p-1
                double x = tau / dt;
                int hit = -1;
                double den = 0.0;
                for (int i = 0; i < p; ++i) {
                    double dx = x - (d0 + i);
                    if (dx == 0.0) { hit = i; break; }
                    lv[i] = bary[i] / dx;
                    den += lv[i];
                }
                if (hit >= 0) {
                    out[d0 + hit - lev_min] += wt;
                } else {
                    for (int i = 0; i < p; ++i) out[d0 + i - lev_min] += wt * lv[i] / den;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Chebyshev tables of eta_d(r) over sub-panels (see wfp2d_tables.h).
// ---------------------------------------------------------------------------
static double subpanel_r(const SubPanel &s, double x)
{
    double v = 0.5 * (s.ua + s.ub) + 0.5 * (s.ua - s.ub) * x;   // sqrt variable: x = +1 at r = ra
    return s.c > 0.0 ? s.c - v * v : v;
}

static void fit_subpanel(const LocalWeights &LW, const SubPanel &s, double *coef /* [nlev][D] */)
{
    const int D = kChebDeg, nl = LW.nlev;
    std::vector<double> vals((size_t)D * nl);
    // the weights at the D Chebyshev nodes, one node per thread (each writes its own row)
#pragma omp parallel for schedule(dynamic, 1)
    for (int q = 0; q < D; ++q) {
        double x = std::cos(M_PI * (q + 0.5) / D);
        LW.eta(subpanel_r(s, x), &vals[(size_t)q * nl]);
    }
    for (int d = 0; d < nl; ++d)
        for (int k = 0; k < D; ++k) {
            double sum = 0.0;
            for (int q = 0; q < D; ++q) sum += vals[(size_t)q * nl + d] * std::cos(M_PI * k * (q + 0.5) / D);
            coef[(size_t)d * D + k] = (k == 0 ? 1.0 : 2.0) * sum / D;
        }
}

static double cheb_eval(const double *c, int D, double x)
{
    double b1 = 0.0, b2 = 0.0;
    for (int k = D - 1; k >= 1; --k) {
        double b0 = 2.0 * x * b1 - b2 + c[k];
        b2 = b1;
        b1 = b0;
    }
    return x * b1 - b2 + c[0];
}

static SubPanel make_sub(double ra, double rb, double c)
{
    SubPanel s{};
    s.ra = ra;
    s.rb = rb;
    s.c = c;
    if (c > 0.0) {
        s.ua = std::sqrt(std::max(0.0, c - ra));
        s.ub = std::sqrt(std::max(0.0, c - rb));
    } else {
        s.ua = rb;   // linear variable: x = (2 r - ra - rb) / (rb - ra)
        s.ub = ra;
    }
    s.inv = 1.0 / (s.ua - s.ub);
    return s;
}

LocalTable build_local_table(const LocalWeights &LW, int n_dy, double rel_tol)
{
    LocalTable T;
    const double dt = LW.dt;
    const int D = kChebDeg, nl = LW.nlev;
    T.nlev = nl;
    T.panel_base.assign(LW.W, 0);
    T.panel_l2n.assign(LW.W, 0);
    std::vector<double> coef, tmp((size_t)nl * D);
    // Fit error is judged against max(scale of the panel, 1e-2 x scale of the
    // largest weights): pairs near r = delta carry weights ~1e-5 of those at
    // small r, so their absolute accuracy, not their relative one, matters.
    double global_scale = 0.0;
    // regular panels k = 0..W-1: r in [max(k, 1/2) dt, (k+1) dt), sqrt variable about (k+1) dt
    for (int k = 0; k < LW.W; ++k) {
        double r0 = (k == 0 ? 0.5 : (double)k) * dt, r1 = (k + 1) * dt, c = (k + 1) * dt;
        int l2n = 0;
        for (;; ++l2n) {
            int ns = 1 << l2n;
            std::vector<double> cf((size_t)ns * nl * D);
            double err = 0.0, scale = 0.0;
            for (int s = 0; s < ns; ++s) {
                SubPanel sp = make_sub(r0 + (r1 - r0) * s / ns, r0 + (r1 - r0) * (s + 1) / ns, c);
                fit_subpanel(LW, sp, &cf[(size_t)s * nl * D]);
            }
            // fit error at 7 interior points of every sub-panel (maxima: the same in any order)
            static const double xs[7] = {-0.93, -0.61, -0.27, 0.05, 0.41, 0.77, 0.97};
#pragma omp parallel for schedule(dynamic, 1) reduction(max : err, scale)
            for (int sx = 0; sx < ns * 7; ++sx) {
                const int s = sx / 7;
                const double x = xs[sx % 7];
                SubPanel sp = make_sub(r0 + (r1 - r0) * s / ns, r0 + (r1 - r0) * (s + 1) / ns, c);
                std::vector<double> evs(nl);
                LW.eta(subpanel_r(sp, x), evs.data());
                for (int d = 0; d < nl; ++d) {
                    double v = cheb_eval(&cf[((size_t)s * nl + d) * D], D, x);
                    err = std::max(err, std::fabs(v - evs[d]));
                    scale = std::max(scale, std::fabs(evs[d]));
                }
            }
            global_scale = std::max(global_scale, scale);
            const double ref = std::max(scale, 1e-2 * global_scale);
            if (err <= rel_tol * ref || l2n >= 5) {
                T.panel_base[k] = (int)T.subs.size();
                T.panel_l2n[k] = l2n;
                for (int s = 0; s < ns; ++s)
                    T.subs.push_back(make_sub(r0 + (r1 - r0) * s / ns, r0 + (r1 - r0) * (s + 1) / ns, c));
                coef.insert(coef.end(), cf.begin(), cf.end());
                T.max_err = std::max(T.max_err, ref > 0 ? err / ref : 0.0);
                break;
            }
        }
    }
    // dyadic sub-panels below dt/2: [dt 2^{-i-1}, dt 2^{-i}), i = 1..n_dy, linear variable
    T.dy_base = (int)T.subs.size();
    T.n_dy = n_dy;
    for (int i = 1; i <= n_dy; ++i) {
        SubPanel sp = make_sub(dt * std::ldexp(1.0, -i - 1), dt * std::ldexp(1.0, -i), 0.0);
        fit_subpanel(LW, sp, tmp.data());
        T.subs.push_back(sp);
        coef.insert(coef.end(), tmp.begin(), tmp.end());
    }
    T.coef = coef;
    return T;
}

void local_table_eval(const LocalTable &T, double dt, int W, double r, double *out, int nterm_regular)
{
    const double rr = r / dt;
    int sub;
    if (rr >= 0.5) {
        const int k = std::min((int)rr, W - 1);
        const double lo = k == 0 ? 0.5 : (double)k, wd = k == 0 ? 0.5 : 1.0;
        const int ns = 1 << T.panel_l2n[k];
        sub = T.panel_base[k] + std::min((int)((rr - lo) / wd * ns), ns - 1);
    } else {
        int e;
        std::frexp(rr, &e);
        sub = T.dy_base + std::min(-e, T.n_dy) - 1;
    }
    const SubPanel &sp = T.subs[sub];
    const double v = sp.c > 0.0 ? std::sqrt(std::max(0.0, sp.c - r)) : r;
    const double xc = std::min(1.0, std::max(-1.0, (2.0 * v - sp.ua - sp.ub) * sp.inv));
    const int nt = sub < T.dy_base ? std::min(std::max(nterm_regular, 1), kChebDeg) : kChebDeg;
    for (int d = 0; d < T.nlev; ++d) out[d] = cheb_eval(&T.coef[((size_t)sub * T.nlev + d) * kChebDeg], nt, xc);
}

void cheb_to_power(const double *b, int nt, double *a)
{
    // rows of integer coefficients: t_prev = T_{j-1}, t_cur = T_j (exact in int64 for j < 62)
    std::vector<int64_t> t_prev(nt, 0), t_cur(nt, 0), t_next(nt, 0);
    for (int c = 0; c < nt; ++c) a[c] = 0.0;
    t_cur[0] = 1;                                   // T_0
    for (int j = 0; j < nt; ++j) {
        for (int c = 0; c <= j; ++c) a[c] += b[j] * (double)t_cur[c];
        // T_{j+1} = 2x T_j - T_{j-1} (T_1 = x)
        for (int c = 0; c < nt; ++c) {
            const int64_t up = c > 0 ? t_cur[c - 1] : 0;
            t_next[c] = (j == 0 ? 1 : 2) * up - (j == 0 ? 0 : t_prev[c]);
        }
        t_prev.swap(t_cur);
        t_cur.swap(t_next);
    }
}

void local_table_eval_power(const LocalTable &T, double dt, int W, double r, double *out, int nterm_regular)
{
    const double rr = r / dt;
    if (rr < 0.5) {
        local_table_eval(T, dt, W, r, out, nterm_regular);
        return;
    }
    const int k = std::min((int)rr, W - 1);
    const double lo = k == 0 ? 0.5 : (double)k, wd = k == 0 ? 0.5 : 1.0;
    const int ns = 1 << T.panel_l2n[k];
    const int sub = T.panel_base[k] + std::min((int)((rr - lo) / wd * ns), ns - 1);
    const SubPanel &sp = T.subs[sub];
    const double v = sp.c > 0.0 ? std::sqrt(std::max(0.0, sp.c - r)) : r;
    const double xc = std::min(1.0, std::max(-1.0, (2.0 * v - sp.ua - sp.ub) * sp.inv));
    const int nt = std::min(std::max(nterm_regular, 1), kChebDeg);
    double a[kChebDeg];
    for (int d = 0; d < T.nlev; ++d) {
        cheb_to_power(&T.coef[((size_t)sub * T.nlev + d) * kChebDeg], nt, a);
        double y = a[nt - 1];
        for (int c = nt - 2; c >= 0; --c) y = std::fma(y, xc, a[c]);
        out[d] = y;
    }
}

int local_table_terms(const LocalTable &T, double tol, double *tail_out, double *cmax_out)
{
    const int nl = T.nlev, D = kChebDeg;
    double cmax = 0.0;
    for (double v : T.coef) cmax = std::max(cmax, std::fabs(v));
    auto tail_of = [&](int nt) {
        double tail = 0.0;
        for (int k = 0; k < T.dy_base; ++k) {
            double t = 0.0;
            for (int c = nt; c < D; ++c) {
                double cm = 0.0;
                for (int d = 0; d < nl; ++d) cm = std::max(cm, std::fabs(T.coef[((size_t)k * nl + d) * D + c]));
                t += cm;
            }
            tail = std::max(tail, t);
        }
        return tail;
    };
    int terms = D;
    for (int nt : {12, 14, 16})
        if (tail_of(nt) <= 1e-3 * tol * cmax) {
            terms = nt;
            break;
        }
    if (tail_out) *tail_out = tail_of(terms);
    if (cmax_out) *cmax_out = cmax;
    return terms;
}

// ---------------------------------------------------------------------------
// Exponential-of-semicircle spreading kernel (Barnett, Magland & af Klinteberg,
// SIAM J. Sci. Comput. 2019): psi(z) = exp(beta (sqrt(1 - (2z/w)^2) - 1)), |z| <= w/2.
// ---------------------------------------------------------------------------
double es_kernel(double z, int w, double beta)
{
    double t = 2.0 * z / w;
    double a = 1.0 - t * t;
    if (a < 0.0) return 0.0;
    return std::exp(beta * (std::sqrt(a) - 1.0));
}

// psi_hat(n) = int psi(z) cos(2 pi n z / nf) dz (real, even)
void es_fourier(int w, double beta, int64_t nf, int64_t R, std::vector<double> &out)
{
    std::vector<double> x, wt;
    gauss_legendre(400, x, wt);
    out.assign(2 * R + 1, 0.0);
    for (int64_t n = -R; n <= R; ++n) {
        double s = 0.0;
        for (size_t i = 0; i < x.size(); ++i) {
            double z = 0.5 * w * x[i];
            s += wt[i] * es_kernel(z, w, beta) * std::cos(2.0 * M_PI * (double)n * z / (double)nf);
        }
        out[n + R] = 0.5 * w * s;
    }
}

}  // namespace wfp2d
