/*
 * wfp2d — per-time-step evaluation of 2D free-space wave potentials of many
 * point sources by truncated-kernel windowed Fourier projection (TK-WFP),
 * on one AMD Instinct MI355X (gfx950).
 *
 * Problem (Sec. 1, eqs. wave2d, solnRep, Green, pointSources): M point sources
 * y_j and Nx targets x_i in B = [-1,1]^2, wave speed 1, signatures sigma_j(t)
 * with sigma_j(t) = 0 for t <= 0, sampled at t_n = n dt.  The library returns
 *     u(x_i, t) = sum_j int_0^t G(x_i - y_j, t - tau) sigma_j(tau) dtau,
 *     G(x, t) = H(t - |x|) / (2 pi sqrt(t^2 - |x|^2)),
 * at every step to the tolerance eps, using the three-way split of eq. split:
 * a local part by singular quadrature (Sec. 6), a near history by the Fourier
 * recurrence of Sec. 4, and a far history by the sum-of-exponentials
 * recurrence of Sec. 5, with one type-1 and one type-2 non-uniform FFT per step.
 *
 * Conventions for every entry point
 *   - Return value: a wfp2d_status; WFP2D_OK (0) on success, a negative code
 *     otherwise.  Nothing crosses the ABI as an exception.  wfp2d_last_error
 *     gives a message for the most recent failure.
 *   - Device pointers (sigma, u) are borrowed for the call only and used in
 *     stream order on the plan's stream; the caller keeps them alive until that
 *     stream has passed the call.  Host pointers are read during the call only.
 *   - A plan is used by one host thread at a time; calls on different plans
 *     are independent.
 *   - Arrays of points are row-major [n][2] float64 (x then y).
 */
#ifndef WFP2D_H
#define WFP2D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wfp2d_plan_s *wfp2d_plan;

typedef enum {
    WFP2D_OK = 0,
    WFP2D_ERR_ARG = -1,         /* bad size, pointer or parameter */
    WFP2D_ERR_DOMAIN = -2,      /* a point outside B = [-1,1]^2 */
    WFP2D_ERR_INFEASIBLE = -3,  /* parameters violate eq. dt, SOE validity, or device memory */
    WFP2D_ERR_NOMEM = -4,       /* device or host allocation failed */
    WFP2D_ERR_DEVICE = -5,      /* a HIP runtime call failed */
    WFP2D_ERR_STATE = -6,       /* call out of order (e.g. on a destroyed plan) */
    WFP2D_ERR_NONFINITE = -7    /* a NaN or Inf sample was ingested while opts.check_finite was set */
} wfp2d_status;

enum { WFP2D_PREC_FP64 = 0, WFP2D_PREC_MIXED = 1 };

typedef struct {
    /* WFP2D_PREC_MIXED (default): spreading, FFTs, the Fourier-coefficient
     * history rings and interpolation in FP32; near/far recurrence state, the
     * far-history sums and the local quadrature in FP64.
     * WFP2D_PREC_FP64: everything in FP64. */
    int32_t precision;
    /* p, the order of the time interpolation of sigma in the local part
     * (Sec. 6, eq. sigInterp); default 20 (Sec. 7). */
    int32_t interp_order;
    /* Delay, in steps, between the newest ingested sample and the time at which
     * wfp2d_evaluate reports u.  -1 (default) = ceil(p/2) - 1: every stencil of
     * eq. sigInterp is the p grid samples nearest its node, which for delays
     * below p/2 steps include samples newer than t_n, so u(t_n) is reported
     * once they have arrived.  This departs from the paper's statement that
     * only levels up to t_n are kept (Sec. 6); its accuracy is the paper's.
     * 0 = report u(t_n) from past samples only, the stencils one-sided near zero
     * delay: several orders less accurate (300 wavelengths, dt = 8/7150, p = 20:
     * relative error 7e-6 .. 3.4e-5, against 1.6e-7 .. 2.6e-7 with the default). */
    int32_t lookahead;
    double Delta;     /* radial blending width of the truncated kernel (eq. TKdef); default 1 (Sec. 5) */
    double a;         /* near/far split margin, A+ = A + a (eq. Ap); 0 = rule max(1, delta + ln(1e15)/lambda_max) */
    double Kf;        /* far-history Fourier cutoff (eq. ufhApprox); default 80 (Sec. 5) */
    double b_Delta;   /* shape parameter of the radial blend; default 30 (reproduces Table 1) */
    double nufft_tol; /* 0 = default (1e-7 mixed, 1e-11 FP64), else in [1e-15, 1e-2) */
    int64_t max_steps;/* steps the plan will be run for; 0 = unchecked.  Used to check the
                         sum-of-exponentials validity range T <~ 3e4 (Sec. 2.3). */
    int32_t device;   /* HIP device ordinal */
    void *stream;     /* hipStream_t for every launch (NULL = default stream) */
    int32_t spread_tile; /* type-1 spreading tile shape, 0 = default (6); see wfp2d_set_spread_tile */
    /* Local part (Sec. 6, eq. local2): 0 (default) = store the list of source-target
     * pairs with r < delta, with each pair's time-step panel and Chebyshev coordinate,
     * once at init (8 bytes per pair; 4 bytes plus one weight per lookup level for the
     * pairs with r < dt/2) when it takes at most half of the free device memory and
     * the local tables fit the list kernel (W <= 64), and stream it at every step;
     * -1 = never (pairs are found at every step from the cell lists).  Both give the
     * same sums up to the order of additions, except that a mixed-precision plan with
     * stored pairs evaluates only the leading Chebyshev terms of each panel whose
     * dropped tail is at most 1e-3 tol of the largest coefficient (info.cheb_degree).
     * info.local_path reports the path taken. */
    int32_t local_pairs;
    /* 0 (default): sigma and u of wfp2d_step / wfp2d_evaluate / wfp2d_evaluate_noalloc
     * are device pointers, used in stream order.  1: they are host pointers; step
     * copies sigma (through a pinned staging buffer) before it returns, and evaluate
     * returns once u is written (it synchronises the plan's stream).  A plan with
     * host pointers cannot be captured in a graph or a batch, and its
     * wfp2d_evaluate_dot still takes device pointers. */
    int32_t host_pointers;
    /* 1: the ingest kernel tests every sample; a NaN or Inf is taken as 0 (so the
     * plan's state stays finite) and raises a device-side flag.  The flag is
     * reported, and cleared, by the next wfp2d_evaluate that sees it (copied back
     * after each evaluation, so it may show one evaluation late) or by
     * wfp2d_query (which synchronises the stream first), as WFP2D_ERR_NONFINITE.
     * 0 (default): samples are not tested. */
    int32_t check_finite;
} wfp2d_opts;

typedef struct {
    double dt, delta, b, A, Aplus, a, dk, K, Kf, Kmax;
    int64_t LA;            /* (A+ - delta)/dt, an integer by construction */
    int64_t R;             /* Fourier grid half-width: modes n in [-R, R]^2 */
    int64_t n_modes;       /* stored half-disk modes |n dk| <= Kmax */
    int64_t n_near;        /* of those, near-history modes |n dk| <= K */
    int64_t n_far;         /* far-history modes |n dk| <= Kf */
    int64_t n_far_classes; /* distinct |n|^2 among far modes */
    int64_t nf;            /* fine (oversampled) FFT grid size per dimension */
    int64_t band;          /* occupied rows/columns of the fine grid */
    int64_t fft_q, fft_p;  /* nf = fft_p * fft_q, fft_q a power of two */
    int32_t nufft_w;       /* spreading kernel width in grid points */
    int32_t W, p, lookahead, n_levels; /* window steps, interp order, delay, sigma levels in the local part */
    int32_t level_min;     /* most negative delay level used by the local part (= -lookahead) */
    int32_t n_subpanels;
    int32_t cheb_degree;   /* Chebyshev terms per regular sub-panel evaluated by the local kernel */
    int64_t M, Nx;
    int64_t n_local_pairs; /* source-target pairs with 0 < r < delta */
    int64_t sigma_depth;   /* slots in the sigma history ring */
    int64_t bytes_device;  /* device memory held by the plan */
    int64_t steps_ingested;/* number of wfp2d_step calls so far */
    int64_t step_reported; /* n such that wfp2d_evaluate returns u(t_n) (<= 0: zero field) */
    int32_t precision;
    int32_t n_regular_subpanels; /* local-weight sub-panels with r >= dt/2 */
    int32_t spread_tile;         /* current spreading tile shape code */
    int32_t local_path;          /* local-part kernel: 0 generic, 1 per-step pair search, 2 stored pair lists */
    int64_t local_pair_bytes;    /* device bytes of the stored pair lists (0 if none) */
    int64_t local_pair_words;    /* entries of the stored regular pair lists: pairs with r >= dt/2 and
                                    the padding that completes each (source, sub-panel) group to whole
                                    runs of 8 (0 if none) */
    double init_ms[7];           /* wall-clock ms of the plan's set-up: 0 modes and geometry
                                    (cell sort), 1 NUFFT point data (kernel origins and
                                    weights, tile lists), 2 history tables (blend, SOE nodes,
                                    Hankel coefficients of eq. H, window FIR), 3 local-weight
                                    tables and NUFFT corrections, 4 device memory and uploads,
                                    5 pair lists, power-basis table and kernel attributes;
                                    6 total */
} wfp2d_info;

/* Fill *opts with the defaults listed above.  Never fails for a valid pointer. */
wfp2d_status wfp2d_default_opts(wfp2d_opts *opts);

/*
 * Create a plan (Secs. 3-6; parameters by eqs. W, A, Ap, dk, K, dt).
 *   M, src_xy  : sources, host pointer [M][2] float64, each in [-1,1]^2.
 *   Nx, tgt_xy : targets, host pointer [Nx][2] float64, each in [-1,1]^2; may
 *                alias src_xy.  A target that coincides with a source omits
 *                that pair from the local part (eq. ul1 requires r > 0) and
 *                keeps its smooth windowed history in the Fourier part.
 *   dt         : time step (> 0).  window_W: the paper's W, delta = W dt (eq. W).
 *   tol        : eps in (1e-15, 1e-2); b = ln(1/eps) (Sec. 2.1).
 *   opts       : NULL for defaults.
 * Copies the coordinates; the caller may free them on return.  Allocates all
 * device memory of the plan (freed by wfp2d_destroy); step and evaluate never
 * allocate.  Errors: ERR_ARG (sizes, dt, tol, W), ERR_DOMAIN (a point outside
 * B), ERR_INFEASIBLE (pi - 2b/W <= 0, so no time step satisfies eq. dt; or
 * max_steps*dt beyond the SOE validity range; or not enough device memory),
 * ERR_NOMEM, ERR_DEVICE.  On error *out is set to NULL.
 */
wfp2d_status wfp2d_init(wfp2d_plan *out, int64_t M, const double *src_xy, int64_t Nx,
                        const double *tgt_xy, double dt, int32_t window_W, double tol,
                        const wfp2d_opts *opts);

/*
 * Advance one time step (Sec. 4.2, eqs. alphakEvolution, hggrid; Sec. 5,
 * eqs. betaEvolution, beta).  sigma: device pointer [M] float64,
 * sigma[j] = sigma_j(t_n) for the n-th call (n = 1, 2, ...), in the order of
 * src_xy.  Ingests the sample, then (once n > lookahead) runs the packed
 * type-1 NUFFT of the current and lagged samples, the near-history update of
 * every Fourier mode and the far-history sum-of-exponentials update, leaving
 * the combined Fourier coefficients of u_h(t_{n - lookahead}).
 * Errors: ERR_ARG (NULL), ERR_STATE, ERR_DEVICE.
 */
wfp2d_status wfp2d_step(wfp2d_plan plan, const double *sigma);

/*
 * Write u(x_i, t_m), m = (steps so far) - lookahead, into u: device pointer
 * [Nx] float64 in the order of tgt_xy.  u = u_h + u_l: the type-2 NUFFT of
 * the Fourier coefficients (eqs. uhtraptrunc, ufhApprox) plus the local part
 * (eq. ul_GL with the interpolation of eq. sigInterp).  For m <= 0 it writes
 * zeros (zero initial data, eq. wave2d).  Errors: ERR_ARG, ERR_STATE, ERR_DEVICE;
 * ERR_NONFINITE (u is still written) when opts.check_finite is set and a
 * non-finite sample has been ingested since the flag was last reported.
 */
wfp2d_status wfp2d_evaluate(wfp2d_plan plan, double *u);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * evaluation as wfp2d_evaluate (same kernels, same result up to the order of
 * floating-point sums), but its transient buffers (the type-2 FFT
 * intermediates, the real fine grid, u_h and u_l) are taken from a fixed
 * 64 MiB device workspace instead of the plan's own.  It allocates and frees
 * nothing.  The workspace is one static array per device, mapped when the
 * library is loaded, located at wfp2d_init and held until the process ends;
 * every plan on that device shares it and it keeps the last call's contents
 * (nothing in it has to start at zero).  Calls on one device that may run at
 * the same time (on different streams or host threads) race; calls ordered
 * on one stream do not.  A plan whose evaluation needs more than 64 MiB
 * (2 (R+1) band + band^2 reals plus 16 Nx bytes, each buffer rounded up to
 * 256 bytes) is rejected with ERR_ARG.  wfp2d_debug_copy(4 / 5) shows the
 * plan's own buffers, written by wfp2d_evaluate only.
 * u: device pointer [Nx] float64, as for wfp2d_evaluate.
 * Errors: ERR_ARG (NULL u, workspace too small), ERR_STATE (stage timing
 * enabled), ERR_DEVICE.
 */
wfp2d_status wfp2d_evaluate_noalloc(wfp2d_plan plan, double *u);

/* Derived parameters and sizes of a plan.  Errors: ERR_ARG; ERR_NONFINITE (with
 * *info filled) when opts.check_finite is set and a non-finite sample has been
 * ingested since the flag was last reported (the stream is synchronised first). */
wfp2d_status wfp2d_query(wfp2d_plan plan, wfp2d_info *info);

/* Release every resource of the plan (waits for its stream).  NULL is a no-op. */
wfp2d_status wfp2d_destroy(wfp2d_plan plan);

/* Message for the last failure on this plan, or of the last failed wfp2d_init
 * when plan is NULL.  The string stays valid until the next call on the plan. */
const char *wfp2d_last_error(wfp2d_plan plan);

/* Stage read-back for tests (synchronises the plan's stream).  what:
 *   1 = S(k, t_m) of the newest near-ring slot, 2 = S(k, t_{m - LA}) of the newest lag slot,
 *   3 = combined coefficients (dk/2pi)^2 (alpha + alpha_F) at t_m,
 *   (each complex, packed half-disk order of wfp2d_debug_modes, in the plan's
 *    FP32 (mixed) or FP64 precision, interleaved re/im);
 *   4 = u_h at t_m, 5 = u_l at t_m (float64 [Nx], target order);
 *   6 = the stored modes (n_x, n_y) as int32 pairs [n_modes][2];
 *   7 = per distinct |k| of the far modes (n_far_classes rows): kappa, then its 640
 *       Hankel coefficients H_l(kappa) of eq. H as the plan computed them on the
 *       device, float64 [n_far_classes][641].
 * dst: host pointer of at least *bytes bytes; on return *bytes = bytes written.
 * Errors: ERR_ARG (unknown what, short buffer), ERR_DEVICE. */
wfp2d_status wfp2d_debug_copy(wfp2d_plan plan, int32_t what, void *dst, int64_t *bytes);

/*
 * acc[i] += weights[i] * u(x_i, t_m) for the reported step m, instead of
 * writing u (same stages as wfp2d_evaluate; nothing is added while m < 1).
 * weights and acc are device pointers to Nx float64 in caller target order,
 * borrowed for the call.  The adjoint uses it to reduce d(loss)/d(sigma_j(t_l))
 * against sigma_j(t_l) = A_j s_j(t_l), giving d(loss)/dA_j without storing the
 * adjoint field.  Errors: ERR_ARG, ERR_STATE, ERR_DEVICE.
 */
wfp2d_status wfp2d_evaluate_dot(wfp2d_plan plan, const double *weights, double *acc);

/*
 * The transpose of a plan's discrete operator.  The map sigma -> u is linear;
 * its kernel between a source y_j and a target x_i depends on |x_i - y_j| only
 * (the Green's function, eq. TKdef, the local weights of eq. ul_GL) or on
 * x_i - y_j through an even Fourier multiplier (the type-1 / type-2 NUFFT
 * pair with the same even spreading kernel), and it is causal and invariant
 * under time shifts.  So the transpose is the same method with sources and
 * targets exchanged, run on time-reversed input: wfp2d_adjoint_init builds
 * that plan (sources = the forward plan's targets, targets = its sources, the
 * same dt, W, tol and options; an independent plan, to be destroyed with
 * wfp2d_destroy).  With forward reports u(t_m), m = 1..T, and input samples
 * sigma(t_l), l = 1..T + L (L = lookahead), feeding the adjoint plan
 * x(n) = g(T + L + 1 - n) for n = 1..T + 2L (zero outside 1..T) makes its
 * report after step n equal to sum_m k(m - l) g(m) at l = T + 2L + 1 - n:
 * d(loss)/d(sigma(t_l)) for g = d(loss)/du.
 * Errors: as wfp2d_init; ERR_STATE for a NULL forward plan.
 */
wfp2d_status wfp2d_adjoint_init(wfp2d_plan *out, wfp2d_plan forward);

/*
 * Checkpoints.  The evolving state of a plan (step count, the sigma history
 * ring, the Fourier rings, the near-history state, alpha_tot and the SOE
 * state) is copied to or from a caller-owned device buffer of at least
 * wfp2d_state_bytes bytes (a header, then each buffer on a 256-byte
 * boundary).  Loading requires a blob from a plan of the same geometry
 * (M, Nx, number of modes); it replaces the plan's state, including its step
 * count.  Both synchronise the plan's stream.  Errors: ERR_ARG (NULL, too
 * small, foreign blob), ERR_STATE, ERR_DEVICE.
 */
wfp2d_status wfp2d_state_bytes(wfp2d_plan plan, int64_t *bytes);
/* Back to zero initial data (eq. wave2d; sigma(t <= 0) = 0): zeroes the
 * evolving state and the step count; synchronises the plan's stream. */
wfp2d_status wfp2d_reset(wfp2d_plan plan);
wfp2d_status wfp2d_save_state(wfp2d_plan plan, void *dst, int64_t bytes);
wfp2d_status wfp2d_load_state(wfp2d_plan plan, const void *src, int64_t bytes);

/*
 * Spectral checkpoints: the same state without the sigma history ring (the
 * Fourier rings, the near-history state, alpha_tot, the SOE state and the step
 * count; at 10^6 sources 4.5 GB instead of 39 GB), in a caller-owned device
 * buffer of at least wfp2d_spectral_state_bytes bytes.  The history ring holds
 * samples the caller already has (the lagged transform of eq. sighat and the
 * local part's levels of eq. sigInterp reach back sigma_depth steps), so after
 * wfp2d_load_spectral_state, which zeroes the ring and sets the step count to
 * the blob's n, the caller puts back sigma(t_l) for every l with
 * max(1, n - sigma_depth + 1) <= l <= n with wfp2d_put_sigma before the next
 * wfp2d_step or wfp2d_evaluate.  A spectral blob is not a full blob: each load
 * accepts only its own kind.  Errors: as wfp2d_save_state / wfp2d_load_state.
 */
wfp2d_status wfp2d_spectral_state_bytes(wfp2d_plan plan, int64_t *bytes);
wfp2d_status wfp2d_save_spectral_state(wfp2d_plan plan, void *dst, int64_t bytes);
wfp2d_status wfp2d_load_spectral_state(wfp2d_plan plan, const void *src, int64_t bytes);

/*
 * Store sigma(t_l) (layout, pointer kind and non-finite check as wfp2d_step)
 * in the history ring as step l's sample, without advancing the plan; for
 * refilling the ring after wfp2d_load_spectral_state.  l must be a step the
 * ring still holds: 1 <= l <= n and l > n - sigma_depth (n = steps so far).
 * Errors: ERR_ARG (NULL sigma, l out of reach), ERR_STATE, ERR_DEVICE.
 */
wfp2d_status wfp2d_put_sigma(wfp2d_plan plan, int64_t l, const double *sigma);

/*
 * Graph replay of one plan.  wfp2d_graph_capture records one step followed by
 * one evaluation into a HIP graph, reading the samples from the fixed device
 * pointer sigma [M] and writing u into the fixed device pointer u [Nx]
 * (both borrowed for the graph's lifetime); wfp2d_graph_launch replays it on
 * the plan's stream, equivalent to wfp2d_step(sigma) + wfp2d_evaluate(u).
 * The caller writes sigma_j(t_n) into sigma before each launch.  Capturing
 * again replaces the graph.  Not allowed while stage timing is enabled.
 * Errors: ERR_ARG, ERR_STATE, ERR_DEVICE.
 */
wfp2d_status wfp2d_graph_capture(wfp2d_plan plan, const double *sigma, double *u);
wfp2d_status wfp2d_graph_launch(wfp2d_plan plan);

/*
 * Batches of independent scatterers: n plans on one device advanced together
 * by one graph launch per step.  sigma[i] / u[i] are fixed device pointers of
 * plan i (as for wfp2d_graph_capture); stream is the (non-default) hipStream_t
 * the batch is launched on.  The plans' work is captured on n_streams
 * forked capture streams (>= 1), so different plans may run concurrently.
 * The plans must outlive the batch (destroy the batch first) and must not be
 * stepped otherwise while it is in use.  Errors (message via wfp2d_last_error(NULL)): ERR_ARG, ERR_STATE,
 * ERR_DEVICE, ERR_NOMEM.
 */
typedef struct wfp2d_batch_s *wfp2d_batch;
wfp2d_status wfp2d_batch_create(wfp2d_batch *out, int32_t n, const wfp2d_plan *plans, const double *const *sigma,
                                double *const *u, int32_t n_streams, void *stream);
wfp2d_status wfp2d_batch_launch(wfp2d_batch batch);
wfp2d_status wfp2d_batch_destroy(wfp2d_batch batch);

/*
 * Spreading tile shape of the type-1 NUFFT (eq. sighat: the sources' kernel
 * contributions are summed per tile of the fine grid in on-chip memory).
 * code 1..5 = 8x8, 16x8, 16x16, 32x16, 32x32 fine-grid points summed on the
 * vector units; code 6 = 16x16 tiles summed as a contraction over the tile's
 * sources on the matrix cores (the kernel is a tensor product, so a tile's
 * grid values are the product of the sources' y-weight columns, scaled by the
 * samples, with their x-weight rows; requires w <= 16).  The result
 * does not depend on the shape (up to the order of floating-point sums); the
 * speed does, with the source density, so an autotuner picks it by timing.
 * wfp2d_set_spread_tile rebuilds the plan's per-tile source lists (it
 * synchronises the plan's stream); wfp2d_time_spread selects `code` the same
 * way and returns the mean duration in ms of `reps` spreading launches on the
 * plan's stream (it only rewrites the plan's scratch grid, so it may be called
 * between steps).  Both fail with ERR_STATE while a graph of the plan, or a
 * batch holding it, exists; ERR_ARG for a bad code.
 */
wfp2d_status wfp2d_set_spread_tile(wfp2d_plan plan, int32_t code);
wfp2d_status wfp2d_time_spread(wfp2d_plan plan, int32_t code, int32_t reps, double *ms);

/*
 * Per-stage timing with HIP events recorded on the plan's stream around every
 * launch of the hot path (for measurement; adds one event pair per launch).
 * wfp2d_set_timing(plan, 1) clears and enables the accumulators, 0 disables.
 * wfp2d_get_timing synchronises the stream and writes, for stage s < n:
 * ms[s] = total milliseconds, launches[s] = number of launches since enabling.
 * Stages: 0 ingest, 1 spread, 2 type-1 row FFT, 3 type-1 column FFT,
 * 4 Hermitian split, 5 near update, 6 far update, 7 type-2 column FFT,
 * 8 type-2 row FFT, 9 interpolation, 10 local part, 11 combine (n <= 12).
 * Errors: ERR_ARG, ERR_DEVICE. */
wfp2d_status wfp2d_set_timing(wfp2d_plan plan, int32_t enable);
wfp2d_status wfp2d_get_timing(wfp2d_plan plan, double *ms, int64_t *launches, int32_t n);

/*
 * Host-only evaluation of the plan's precomputation, without a device (for
 * tests of the set-up numerics).  All pointers are host pointers; nothing is
 * allocated on a device.  what:
 *   1 derived parameters: in = {dt, W, tol, p, lookahead, Delta, a, Kf}
 *     (n_in = 8); out = {delta, b, A, Aplus, a, dk, K, Kmax, LA, R, lookahead,
 *     N} (n_out >= 12).  Rules of eqs. W, A, Ap, dk, K.
 *   2 sum-of-exponentials nodes (Sec. 2.3): out = {lambda_1..640, q_1..640}.
 *   3 Hankel coefficients H_l(kappa; A) of eq. H: in = {A, Delta, b_Delta,
 *     kappa_1..kappa_k}; out = [k][640].
 *   4 local weights eta_d(r) by direct quadrature (Sec. 6): in = {dt, W, p,
 *     lookahead, tol, r_1..r_k}; out = [k][n_levels] (levels d = -lookahead...).
 *   5 the same weights from the plan's Chebyshev tables (as the kernels
 *     evaluate them): same in/out as 4.
 *   6 blending function (eq. KBblending): in = {width, b, t_1..t_k};
 *     out = [k][2] = (phi, phi').
 *   7 layout of the local-weight tables: in as 4; out = {sub-panels, regular
 *     sub-panels, levels, max relative fit error, log2 splits of panel 0..W-1}.
 *   8 the weights as a mixed-precision plan with stored pair lists evaluates
 *     them: in as 4; out = {terms, tail bound, largest coefficient, then
 *     [k][n_levels]}, where the regular sub-panels keep only their leading
 *     `terms` Chebyshev coefficients (the smallest of 12, 14, 16 whose dropped
 *     coefficients sum, per sub-panel over the largest magnitude per term, to at
 *     most 1e-3 tol of the largest coefficient; else all) and the tail bound is
 *     that sum for the returned count.
 *   9 Fourier transform of the spreading kernel (the NUFFT deconvolution
 *     factors, R18): in = {w, beta, nf, n_1..n_k}, |n_i| < nf/2; out[i] =
 *     int psi(z) cos(2 pi n_i z / nf) dz over |z| <= w/2, psi the
 *     exponential-of-semicircle kernel of width w and shape beta.
 * Returns ERR_ARG for an unknown what, short buffers or bad parameters; on
 * success out_count (if not NULL) receives the number of doubles written. */
wfp2d_status wfp2d_host_eval(int32_t what, const double *in, int64_t n_in, double *out, int64_t n_out,
                             int64_t *out_count);

#ifdef __cplusplus
}
#endif

#endif /* WFP2D_H */
