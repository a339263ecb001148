/*
 * Reference evaluator for the 2D free-space wave potential of point sources.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the GPU path.
 *
 * What it computes (Sec. 1, eqs. solnRep, Green, pointSources; Sec. 7,
 * eq. exactSol):
 *
 *   u(x, t) = sum_j (1/2pi) int_{r_j}^{t} sigma_j(t - tau) / sqrt(tau^2 - r_j^2) dtau,
 *   r_j = |x - y_j|,
 *
 * evaluated with the *analytic* signatures by composite Gauss-Legendre
 * quadrature in double precision.  The inverse square-root singularity at
 * tau = r is removed by tau = r cosh(v) (so dtau / sqrt(tau^2-r^2) = dv, the
 * same device as Sec. 6 uses for small r); beyond r + 1/omega the panels are
 * plain, graded geometrically away from the singular point and no wider than
 * half a signature period.
 *
 * Optional windowed components (eq. split, with the blending function of
 * eq. KBblending) give stage-level references:
 *   window 1 (local):   weight [1 - phi(tau)] on tau in [0, delta]           (eq. ul)
 *   window 2 (near):    weight phi(tau) phi(A+ - tau) on tau in [0, A+]      (eq. unh)
 *   window 3 (far):     weight [1 - phi(A+ - tau)] on tau >= A+ - delta      (eq. ufh;
 *                       the truncated kernel equals G inside B)
 *   window 4 (history): weight phi(tau)  (= near + far inside B)
 *
 * Coincident source and target (r == 0): the paper's exact-solution formula
 * omits the pair (eq. exactSol requires r_j != 0) and its neighbour set
 * excludes it (Sec. 3, eq. ul1).  With self_mode = 0 the pair is skipped.
 * With self_mode = 1 the pair contributes its smooth windowed history
 * (1/2pi) int_0^t sigma(t - tau) win0(tau) / tau dtau, where win0 = phi for
 * the full field and the history, the near/far windows for those components,
 * and 0 for the local part: the local part omits r = 0 while the Fourier
 * history parts do not.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TWO_PI 6.283185307179586476925286766559
#define FAM_G 0
#define FAM_E 1
#define FAM_STEP 2
#define FAM_RAMP 3

/* ------------------------------------------------------------------ */
/* Gauss-Legendre rule on [-1,1] by Newton iteration on P_n.           */
/* ------------------------------------------------------------------ */
static void gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5));
        double pp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p1 = 1.0, p2 = 0.0;
            for (int k = 1; k <= n; ++k) {
                double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * k - 1.0) * z * p2 - (k - 1.0) * p3) / k;
            }
            pp = n * (z * p1 - p2) / (z * z - 1.0);
            double dz = p1 / pp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        /* recompute derivative at the converged root */
        {
            double p1 = 1.0, p2 = 0.0;
            for (int k = 1; k <= n; ++k) {
                double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * k - 1.0) * z * p2 - (k - 1.0) * p3) / k;
            }
            pp = n * (z * p1 - p2) / (z * z - 1.0);
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

/* ------------------------------------------------------------------ */
/* Signatures (closed forms; see the workload description)             */
/* ------------------------------------------------------------------ */
typedef struct {
    int fam;
    double A, t0, w, s;
} sig_t;

static double sig_eval(const sig_t *g, double t)
{
    switch (g->fam) {
    case FAM_G: {
        if (t <= g->t0) return 0.0;
        double c = g->t0 + 8.5 * g->s;
        double d = t - c;
        return g->A * exp(-d * d / (2.0 * g->s * g->s)) * sin(g->w * d);
    }
    case FAM_E:
        if (t <= 0.0) return 0.0;
        return g->A * 0.5 * (erf(5.0 * (t - g->t0)) + 1.0) * sin(g->w * (t - g->t0));
    case FAM_STEP:
        return t > g->t0 ? g->A : 0.0;
    case FAM_RAMP:
        return t > g->t0 ? g->A * (t - g->t0) : 0.0;
    }
    return 0.0;
}

/* sigma(t) == 0 (family E: below 1e-40 |A|) for t <= sig_start */
static double sig_start(const sig_t *g)
{
    switch (g->fam) {
    case FAM_G: return g->t0;
    case FAM_E: {
        double s0 = g->t0 - 2.0; /* 0.5 erfc(10) ~ 1e-45 */
        return s0 > 0.0 ? s0 : 0.0;
    }
    default: return g->t0;
    }
}

/* sigma(t) == 0 for t >= sig_end (Gaussian envelope below 1e-40) */
static double sig_end(const sig_t *g)
{
    if (g->fam == FAM_G) return g->t0 + 8.5 * g->s + 14.0 * g->s;
    return INFINITY;
}

/* angular frequency scale used to size panels */
static double sig_wscale(const sig_t *g)
{
    switch (g->fam) {
    case FAM_G: return fabs(g->w) + 9.0 / g->s;
    case FAM_E: return fabs(g->w) + 60.0;
    default: return 1.0;
    }
}

/* ------------------------------------------------------------------ */
/* Blending function of eq. KBblending                                 */
/* ------------------------------------------------------------------ */
static double bessel_i0(double x)
{
    /* power series sum (x^2/4)^k / (k!)^2: all terms positive */
    double q = 0.25 * x * x, term = 1.0, sum = 1.0;
    for (int k = 1; k < 500; ++k) {
        term *= q / ((double)k * (double)k);
        sum += term;
        if (term < 1e-18 * sum) break;
    }
    return sum;
}

typedef struct {
    double delta, b;     /* temporal blend width and shape */
    double Aplus;
    int window;
    double glx[64], glw[64];
} win_t;

static double phi_prime(const win_t *W, double t)
{
    if (t < 0.0 || t > W->delta) return 0.0;
    double z = 2.0 * t / W->delta - 1.0;
    double a = 1.0 - z * z;
    if (a < 0.0) a = 0.0;
    return W->b / (W->delta * sinh(W->b)) * bessel_i0(W->b * sqrt(a));
}

/* phi(t) = int_0^t phi'(s) ds by 64-point Gauss-Legendre (phi' is entire) */
static double phi_val(const win_t *W, double t)
{
    if (t <= 0.0) return 0.0;
    if (t >= W->delta) return 1.0;
    double h = 0.5 * t, sum = 0.0;
    for (int i = 0; i < 64; ++i) sum += W->glw[i] * phi_prime(W, h * (W->glx[i] + 1.0));
    return sum * h;
}

/* window weight of delay tau for r > 0 */
static double win_weight(const win_t *W, double tau)
{
    switch (W->window) {
    case 0: return 1.0;
    case 1: return tau <= W->delta ? 1.0 - phi_val(W, tau) : 0.0;
    case 2: return (tau >= W->Aplus) ? 0.0 : phi_val(W, tau) * phi_val(W, W->Aplus - tau);
    case 3: return (tau < W->Aplus - W->delta) ? 0.0 : 1.0 - phi_val(W, W->Aplus - tau);
    case 4: return phi_val(W, tau);
    }
    return 0.0;
}

/* support of the window weight in tau, and its breakpoints */
static void win_support(const win_t *W, double *lo, double *hi, double *bp, int *nbp)
{
    *nbp = 0;
    switch (W->window) {
    case 0: *lo = 0.0; *hi = INFINITY; break;
    case 1: *lo = 0.0; *hi = W->delta; break;
    case 2: *lo = 0.0; *hi = W->Aplus; bp[(*nbp)++] = W->delta; bp[(*nbp)++] = W->Aplus - W->delta; break;
    case 3: *lo = W->Aplus - W->delta; *hi = INFINITY; bp[(*nbp)++] = W->Aplus; break;
    case 4: *lo = 0.0; *hi = INFINITY; bp[(*nbp)++] = W->delta; break;
    }
}

/* is tau inside a blending transition (needs finer panels)? */
static int in_transition(const win_t *W, double a, double b)
{
    if (W->window == 0) return 0;
    if (a < W->delta && W->window != 3) return 1;
    if ((W->window == 2 || W->window == 3) && b > W->Aplus - W->delta && a < W->Aplus) return 1;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Quadrature of one source's contribution                             */
/* ------------------------------------------------------------------ */
typedef struct {
    int npp;          /* nodes per panel */
    double hscale;    /* panel-width multiplier (refinement tests use 0.5) */
    const double *gx, *gw;
} rule_t;

/* int_a^b f(tau) dtau / sqrt(tau^2 - r^2), a > r, plain GL panels graded
   geometrically away from tau = r and no wider than hmax */
static double plain_segment(const sig_t *g, const win_t *W, const rule_t *R, double t, double r,
                            double a, double b, double hmax, int r0mode)
{
    double sum = 0.0, comp = 0.0;
    double x = a;
    while (x < b) {
        double dist = x - r;
        double h = hmax;
        if (!r0mode && dist < h) h = dist;
        if (r0mode && x > 0.0 && x < h) h = x;  /* 1/tau kernel: grade from tau=0 */
        if (h <= 0.0) h = hmax;
        double xe = x + h;
        if (xe > b || b - xe < 1e-3 * h) xe = b;
        double c = 0.5 * (x + xe), hw = 0.5 * (xe - x), ps = 0.0;
        for (int i = 0; i < R->npp; ++i) {
            double tau = c + hw * R->gx[i];
            double f = sig_eval(g, t - tau);
            if (f == 0.0) continue;
            double kern;
            if (r0mode) kern = win_weight(W, tau) / tau;
            else kern = win_weight(W, tau) / sqrt((tau - r) * (tau + r));
            ps += R->gw[i] * f * kern;
        }
        ps *= hw;
        /* compensated accumulation */
        double y = ps - comp, s2 = sum + y;
        comp = (s2 - sum) - y;
        sum = s2;
        x = xe;
    }
    return sum;
}

/* int_r^b f(tau) dtau/sqrt(tau^2-r^2) with tau = r cosh v, v in [0, V] */
static double cosh_segment(const sig_t *g, const win_t *W, const rule_t *R, double t, double r, double b)
{
    double x = (b - r) / r;                        /* b = r (1 + x) */
    double V = log1p(x + sqrt(x * (2.0 + x)));     /* acosh(1 + x) */
    int nv = (int)ceil(V / (0.5 * R->hscale));
    if (nv < 1) nv = 1;
    double dv = V / nv, sum = 0.0;
    for (int p = 0; p < nv; ++p) {
        double c = (p + 0.5) * dv, hw = 0.5 * dv, ps = 0.0;
        for (int i = 0; i < R->npp; ++i) {
            double v = c + hw * R->gx[i];
            double sh = sinh(0.5 * v);
            double excess = 2.0 * r * sh * sh;     /* tau - r, exactly */
            double tau = r + excess;
            double f = sig_eval(g, (t - r) - excess);
            if (f == 0.0) continue;
            ps += R->gw[i] * f * win_weight(W, tau);
        }
        sum += ps * hw;
    }
    return sum;
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* (1/2pi)-less contribution of one source at distance r, time t */
static double pair_integral(const sig_t *g, const win_t *W, const rule_t *R, double t, double r, int self_mode)
{
    int r0 = (r == 0.0);
    if (r0 && !self_mode) return 0.0;
    win_t Wl;
    if (r0) {
        /* coincident pair: no local part; the full field keeps the history
           weight phi(tau) (near + far) */
        if (W->window == 1) return 0.0;
        if (W->window == 0) {
            Wl = *W;
            Wl.window = 4;
            W = &Wl;
        }
    }
    double wlo = 0.0, whi = 0.0, bp[4];
    int nbp;
    win_support(W, &wlo, &whi, bp, &nbp);
    /* delays where sigma(t - tau) can be nonzero */
    double tau_hi = t - sig_start(g);
    double tau_lo = t - sig_end(g);
    double lo = r, hi = tau_hi;
    if (wlo > lo) lo = wlo;
    if (tau_lo > lo) lo = tau_lo;
    if (whi < hi) hi = whi;
    if (!(hi > lo)) return 0.0;

    double hsig = R->hscale * M_PI / sig_wscale(g);      /* half a period */
    double htr = R->hscale * W->delta / 12.0;            /* inside blending transitions */

    /* breakpoints inside (lo, hi) */
    double pts[8];
    int np = 0;
    pts[np++] = lo;
    for (int i = 0; i < nbp; ++i)
        if (bp[i] > lo && bp[i] < hi) pts[np++] = bp[i];
    pts[np++] = hi;
    qsort(pts, np, sizeof(double), cmp_double);

    double total = 0.0;
    for (int s = 0; s + 1 < np; ++s) {
        double a = pts[s], b = pts[s + 1];
        if (!(b > a)) continue;
        double hmax = in_transition(W, a, b) ? (htr < hsig ? htr : hsig) : hsig;
        if (r0) {
            total += plain_segment(g, W, R, t, 0.0, a, b, hmax, 1);
            continue;
        }
        if (a == r) {
            /* singular end: cosh substitution over [r, r + 1/omega] */
            double c = r + hsig / M_PI;
            if (c > b) c = b;
            total += cosh_segment(g, W, R, t, r, c);
            if (c < b) total += plain_segment(g, W, R, t, r, c, b, hmax, 0);
        } else {
            total += plain_segment(g, W, R, t, r, a, b, hmax, 0);
        }
    }
    return total;
}

/* ------------------------------------------------------------------ */
/* Public entry point                                                  */
/* ------------------------------------------------------------------ */
/*
 * out[s] = u at (xs[2s], xs[2s+1]) and time ts[s], for s < ns.
 * fam/amp/t0/om/sw: per-source signature parameters (see the header).
 * window: 0 full, 1 local, 2 near, 3 far, 4 history; delta, b, Aplus
 * parameterise the blending (unused for window 0 unless self_mode = 1).
 * npp: GL nodes per panel (16 default); hscale: panel width multiplier (1).
 * nthreads <= 0 uses the OpenMP default.  Returns 0, or -1 on bad input.
 * Summation over sources is in a fixed order (blocks of 1024 sources, each
 * compensated), so the result does not depend on the thread count.
 */
int oracle_u(int64_t M, const double *src_xy, const int32_t *fam, const double *amp, const double *t0,
             const double *om, const double *sw, int64_t ns, const double *xs, const double *ts,
             int32_t window, double delta, double b, double Aplus, int32_t self_mode, int32_t npp,
             double hscale, int32_t nthreads, double *out)
{
    if (M < 0 || ns < 0 || npp < 2 || npp > 64 || hscale <= 0.0) return -1;
    if (window < 0 || window > 4) return -1;
    if ((window != 0 || self_mode) && !(delta > 0.0 && b > 0.0)) return -1;
    const int64_t BLK = 1024;
    int64_t nblk = (M + BLK - 1) / BLK;
    if (nblk == 0) nblk = 1;
    double *part = (double *)calloc((size_t)(ns * nblk), sizeof(double));
    if (!part) return -1;

    double gx[64], gw[64];
    gauss_legendre(npp, gx, gw);
    rule_t R = {npp, hscale, gx, gw};
    win_t W0;
    memset(&W0, 0, sizeof W0);
    W0.delta = delta;
    W0.b = b;
    W0.Aplus = Aplus;
    W0.window = window;
    gauss_legendre(64, W0.glx, W0.glw);

#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int64_t nunits = ns * nblk;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t u = 0; u < nunits; ++u) {
        int64_t s = u / nblk, k = u % nblk;
        double x = xs[2 * s], y = xs[2 * s + 1], t = ts[s];
        double sum = 0.0, comp = 0.0;
        int64_t j1 = (k + 1) * BLK < M ? (k + 1) * BLK : M;
        for (int64_t j = k * BLK; j < j1; ++j) {
            sig_t g = {fam[j], amp[j], t0[j], om[j], sw ? sw[j] : 0.0};
            double dx = x - src_xy[2 * j], dy = y - src_xy[2 * j + 1];
            double r = sqrt(dx * dx + dy * dy);
            double v = pair_integral(&g, &W0, &R, t, r, self_mode);
            double yv = v - comp, s2 = sum + yv;
            comp = (s2 - sum) - yv;
            sum = s2;
        }
        part[u] = sum;
    }
    for (int64_t s = 0; s < ns; ++s) {
        double sum = 0.0, comp = 0.0;
        for (int64_t k = 0; k < nblk; ++k) {
            double yv = part[s * nblk + k] - comp, s2 = sum + yv;
            comp = (s2 - sum) - yv;
            sum = s2;
        }
        out[s] = sum / TWO_PI;
    }
    free(part);
    return 0;
}

/* The blending function phi and phi' of eq. KBblending, for tests. */
int oracle_phi(int64_t n, const double *t, double delta, double b, double *phi, double *dphi)
{
    win_t W0;
    memset(&W0, 0, sizeof W0);
    W0.delta = delta;
    W0.b = b;
    gauss_legendre(64, W0.glx, W0.glw);
    for (int64_t i = 0; i < n; ++i) {
        if (phi) phi[i] = phi_val(&W0, t[i]);
        if (dphi) dphi[i] = phi_prime(&W0, t[i]);
    }
    return 0;
}

/* The numerical support [start, end] of a signature as the quadrature uses it
 * (sigma is taken as exactly zero outside it), for tests of the cut-offs. */
int oracle_sig_support(int32_t fam, double A, double t0, double w, double s, double *start, double *end)
{
    sig_t g = {fam, A, t0, w, s};
    if (start) *start = sig_start(&g);
    if (end) *end = sig_end(&g);
    return 0;
}

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
