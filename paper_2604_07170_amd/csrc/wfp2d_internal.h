// Internal declarations shared by the host side (plan set-up, C ABI) and the
// HIP kernels of the wfp2d library.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/wfp2d.h"

namespace wfp2d {

constexpr int kTile = 32;          // spreading / interpolation tile edge (fine-grid points)
constexpr int kChunk = 256;        // modes per work chunk of the per-mode kernels
constexpr int kNsoe = 640;         // SOE terms: 20 dyadic panels x 32 Gauss-Legendre nodes (Sec. 2.3)
constexpr int kChebDeg = 20;       // Chebyshev terms per local-weight sub-panel
constexpr int kLocalThreads = 512; // local kernel: threads per workgroup (one target each)
constexpr int kLocalPsi = 4096;    //   LDS doubles for the per-source Chebyshev profiles
constexpr int kLocalSig = 640;     //   LDS doubles for the sources' sigma levels
constexpr int kLocalMaxSrc = 16;   //   sources per chunk (upper bound)
constexpr int kLocalMaxLevels = 64;
constexpr int kLocalQueue = 256;   //   queued pairs with r < dt/2 per chunk
constexpr int kLocalOwn = 2;       //   targets owned per thread (regions up to 1024 targets in one pass)
constexpr int kFastSrc = 16;       // fast local kernel: sources per chunk
constexpr int kFastRow = 512;      //   max coefficient rows (regular sub-panels x Chebyshev terms)
constexpr int kPairTB = 1024;      // pair-list local kernel: targets per batch (LDS sums)
constexpr int kPairRec = 16;       //   int32 per work-cell record
constexpr int kPairUnit = 4;       //   adjacent cells of a row per work unit
constexpr int kFastOwn = 4;        //   targets owned per thread
constexpr int kPairBlockPad = 8;   // pair-list segments are whole runs of this many pairs
constexpr int kPcMaxRows = 480;    // producer / consumer local kernel: profile rows per source
constexpr int kPcLdsRows = 256;    //   rows of the variant with the power-basis table in LDS
// producer waves of the producer / consumer local kernel and its 16-row MFMA blocks per producer
// (rb: 2 up to 384 rows, with the A operands held in registers; else 3, read from cache at each
// item), at least 4 of its 16 waves left to evaluate pairs; 0 when the profile rows do not fit it
// (rb 4: up to kPcLdsRows rows of 35 levels, 4 producers, 12 waves left for the pairs, the table
// in LDS without the levels below each row block's first panel, which must then be exactly zero:
// zero_below)
inline int pc_producers(int n_reg, int terms, int *rb = nullptr, int nlev = 0, bool zero_below = false)
{
    const int rows = n_reg * terms, nblk = (rows + 15) / 16;
    if (nlev == 35 && zero_below && rows <= kPcLdsRows && terms % 2 == 0 && terms <= 16) {
        if (rb) *rb = 4;
        return 4;
    }
    const int r = nblk <= 24 ? 2 : 3, nprod = (nblk + r - 1) / r;
    if (rb) *rb = r;
    return (terms % 2 == 0 && rows <= kPcMaxRows && (r == 2 || terms == 20) && nprod <= 12) ? nprod : 0;
}
// Profile layout in LDS: the row of (source q, panel k) starts at q psi_src + k stride doubles.
// With the table in LDS (rb 4) and 16 terms a panel's row is padded to 9 16-byte chunks, so the
// rows of one source's panels start in different 16-byte bank groups (14 terms are 7 chunks
// already; 12 terms stay unpadded).
inline int pc_panel_stride(int rb, int terms) { return rb == 4 && terms == 16 ? 18 : terms; }
inline int pc_psi_src(int rb, int n_reg, int terms) { return n_reg * pc_panel_stride(rb, terms) + 2; }
// rb 4: first MFMA k-step of the rows [64 r, 64 r + 64) (block r of every producer), and the
// doubles of the compacted table: rows of 4 (KS - kst) levels from level 4 kst on, each padded by
// 2 doubles so that the 16 rows one MFMA operand reads fall in distinct LDS banks
constexpr int pc_kst(int r, int terms) { return (64 * r / terms) / 4; }
constexpr int pc_ctab_stride(int r, int terms, int ks) { return 4 * (ks - pc_kst(r, terms)) + 2; }
constexpr int pc_ctab_doubles(int terms, int ks)
{
    return 64 * (pc_ctab_stride(0, terms, ks) + pc_ctab_stride(1, terms, ks) + pc_ctab_stride(2, terms, ks) +
                 pc_ctab_stride(3, terms, ks));
}
// dynamic LDS of the producer / consumer kernel: two profile buffers, and with rb 4 the table
constexpr size_t pc_lds_rb4(int terms)
{
    return (size_t)2 * 16 * (16 * (terms == 16 ? 18 : terms) + 2) * 8 + (size_t)pc_ctab_doubles(terms, 9) * 8;
}
constexpr size_t kPcDynLds = std::max(std::max((size_t)2 * 16 * (kPcMaxRows + 2) * 8, pc_lds_rb4(16)),
                                      std::max(pc_lds_rb4(14), pc_lds_rb4(12)));
// fixed device workspace of wfp2d_evaluate_noalloc (one per device, held until the process ends)
constexpr size_t kScratchBytes = size_t(64) << 20;

// Work chunk of a per-mode kernel: modes [off, off+cnt) of packed column nx,
// whose first mode has ny = ny0 (ny increases by one per mode).
struct ModeChunk {
    int32_t nx, ny0, off, cnt;
};

// One sub-panel of the tabulated local weights eta_d(r).
struct SubPanel {
    double ra, rb;   // r range
    double c;        // > 0: Chebyshev variable in u = sqrt(c - r); 0: linear in r
    double ua, ub;   // variable at ra and rb: sqrt(c - r) when c > 0, else r
    double inv;      // 1 / (ua - ub): Chebyshev coordinate x = (2 v - ua - ub) * inv
};

// Parameters every kernel needs (passed by value).
struct Geom {
    int64_t M, Nx;
    int32_t W, LA, nlev, lev_min;      // levels d in [lev_min, lev_min + nlev)
    int32_t lookahead;                 // reported step m = ingested step n - lookahead
    int64_t sig_depth;                 // sigma ring slots
    double dt, dk, K, Kf, Kmax, Rd2;   // Rd2 = (Kmax/dk)^2
    int32_t R, N;                      // N = 2R + 1
    int32_t nf, P, Q, lmin, Lpad, w;   // fine grid, band origin / padded size, kernel width
    int32_t ntx;                       // tiles per band dimension
};

struct Plan;

// ---- launchers (kernels file) ----
hipError_t launch_step_begin(Plan &p);
hipError_t launch_ingest(Plan &p, const double *sigma_in);   // tests samples when p.d_nonfinite is set
hipError_t launch_ingest_at(Plan &p, const double *sigma_in, int64_t n);   // sigma(t_n) into its ring slot, likewise
hipError_t launch_spread(Plan &p);
hipError_t kernel_setup(Plan &p);
hipError_t fft_setup(Plan &p);
hipError_t launch_fft_rows1(Plan &p);
hipError_t launch_fft_cols1(Plan &p);
hipError_t launch_split(Plan &p);
hipError_t launch_near(Plan &p);
hipError_t launch_far(Plan &p);
hipError_t launch_fft_cols2(Plan &p);
hipError_t launch_fft_rows2(Plan &p);
hipError_t launch_interp(Plan &p);
hipError_t launch_local(Plan &p);
hipError_t launch_pairs_build(Plan &p, bool fill, int64_t *cnt, int64_t *dcnt);
// NUFFT kernel weights of n points (2w each, grid precision; idx: optional point order)
hipError_t launch_es_weights(Plan &p, const double2 *xy, const int32_t *idx, const int2 *base, int64_t n, double gscale,
                             void *wts);
// Hankel coefficients H[c][l] = sum_g J0(kappa_c r_g) E[l][g] (device pointers)
hipError_t launch_hankel(Plan &p, const double *kappa, int64_t nk, const double *r, int nr, const double *E, int L, double *H);
hipError_t launch_zero_f64(Plan &p, double *ptr, int64_t n);
hipError_t launch_combine_dot(Plan &p, const double *wts, double *acc);
hipError_t launch_combine(Plan &p, double *u_out);
// Device address of the fixed workspace on `device` (which must be current): looked up once per
// device with hipGetSymbolAddress and kept; later calls return the kept address.
hipError_t scratch_address(int device, void **out);

// ---- the plan ----
struct Plan {
    // problem
    int64_t M = 0, Nx = 0;
    double dt = 0, tol = 0;
    int32_t W = 0, p = 20, lookahead = 0, precision = 1;
    double Delta = 1, a = 0, Kf = 80, b_Delta = 30, nufft_tol = 0;
    int32_t device = 0;
    hipStream_t stream = nullptr;

    // derived parameters
    double b = 0, delta = 0, A = 0, Aplus = 0, dk = 0, K = 0, Kmax = 0;
    int64_t LA = 0;
    Geom g{};
    double es_beta = 0;              // exponential-of-semicircle shape

    // mode tables
    int64_t n_modes = 0, n_near = 0, n_far = 0, n_classes = 0;
    std::vector<int32_t> col_off;    // packed offset of column nx (nx = 0..R), size R+2
    std::vector<int32_t> col_ny0;    // first ny of column nx
    std::vector<ModeChunk> chunks;   // near / split / alpha work list
    int64_t n_local_pairs = 0;
    int32_t n_sub = 0;
    std::vector<SubPanel> subs;

    // step counters
    int64_t steps = 0;               // samples ingested
    int64_t sizeof_real = 4;

    // ---- device memory ----
    std::vector<void *> allocs;
    std::vector<size_t> alloc_bytes;  // size of each allocation in allocs
    int64_t bytes_device = 0;
    int64_t *d_step = nullptr;        // device-resident count of ingested steps
    double *d_sig = nullptr;          // [sig_depth][M] float64, sorted source order
    int32_t *d_src_perm = nullptr;    // sorted j -> caller index
    int32_t *d_tgt_rank = nullptr;    // caller index -> sorted i
    double2 *d_src_xy = nullptr, *d_tgt_xy = nullptr;   // sorted order
    // spreading
    int2 *d_src_base = nullptr;       // band-local kernel origin per sorted source
    void *d_src_wts = nullptr;        // [M][2w] Real
    int32_t *d_tile_off = nullptr, *d_tile_src = nullptr;
    std::vector<int2> h_src_base;     // host copy, to rebuild the tile lists for another tile shape
    int32_t spread_tile = 6;          // tile shape code (see wfp2d_set_spread_tile)
    int32_t sp_tx = 32, sp_ty = 32, sp_ntx = 1, sp_nty = 1;
    void *d_grid = nullptr;           // [Lpad][Lpad] complex Real
    void *d_T1 = nullptr;             // [Lpad][N] complex Real (rows transformed)
    void *d_T1t = nullptr;            // [N][Lpad] its transpose
    void *d_F = nullptr;              // [N][N] complex Real, index [nx+R][ny+R]
    void *d_corr = nullptr;           // [N] complex Real: e^{2 pi i n lmin/nf} / psi_hat(n)
    void *d_tw = nullptr;             // [nf] complex float64: e^{2 pi i j / nf}
    // rings of Fourier coefficients
    void *d_ring_cur = nullptr;       // [W][n_modes] complex Real
    void *d_ring_lag = nullptr;       // [W][n_modes] complex Real
    ModeChunk *d_chunks = nullptr;
    int32_t *d_col_off = nullptr, *d_col_ny0 = nullptr;   // packed column tables
    int64_t n_chunks = 0;
    double2 *d_D = nullptr, *d_C = nullptr;   // near state per packed mode
    double *d_phi_in = nullptr;       // phi(l dt), l = 0..W
    void *d_atot = nullptr;           // [n_modes] complex Real
    // far history
    int32_t *d_far_pk = nullptr, *d_far_cls = nullptr;
    double *d_H = nullptr;            // [n_classes][640]
    double *d_chi = nullptr;          // [n_classes][W-1]
    double *d_dec = nullptr, *d_inj = nullptr;   // [640]
    double2 *d_B = nullptr;           // [n_far][640]
    // type 2
    void *d_T2 = nullptr;             // [R+1][Lpad] complex Real
    void *d_T2t = nullptr;            // [Lpad][R+1] its transpose
    void *d_cgrid = nullptr;          // [Lpad][Lpad] Real
    int2 *d_tgt_base = nullptr;       // interpolation origin and weights of each target, in the
                                      // processing order d_ttile_tgt (not sorted order)
    void *d_tgt_wts = nullptr;
    int32_t *d_ttile_off = nullptr, *d_ttile_tgt = nullptr;
    double *d_uh = nullptr, *d_ul = nullptr;   // sorted target order
    // local part
    int32_t ncell = 1;
    double cell_h = 2.0;
    int32_t *d_cell_start = nullptr;  // sources per cell (sorted), size ncell^2 + 1
    int32_t *d_tcell_start = nullptr; // targets per cell (sorted), size ncell^2 + 1
    SubPanel *d_subs = nullptr;
    double *d_cheb = nullptr;         // [n_sub][nlev][kChebDeg], scaled by 1/(2 pi)
    double *d_creg = nullptr;         // regular sub-panels [n_reg][kChebDeg][nlev], scaled by 1/(2 pi)
    double *d_cpow = nullptr;         //   the same, truncated to local_terms and in the power basis (pair kernel)
    int32_t n_reg = 0, local_sc = 1;  // regular sub-panels; sources per chunk in the local kernel
    bool local_fast = false;          // one sub-panel per time-step panel and a supported level count
    int32_t *d_panel_base = nullptr;  // regular panel k -> first sub-panel, and log2 count
    int32_t *d_panel_l2n = nullptr;
    int32_t dy_base = 0, n_dy = 0;
    // pair lists of the local part (built once when they fit; see k_pairs_build)
    bool local_pairs = false;
    int32_t local_terms = kChebDeg;   // leading Chebyshev terms of each regular panel used by the pair kernel
    int64_t pair_bytes = 0;
    int64_t pair_n_work = 0;          // cells with sources and with targets in their 5 x 5 block
    int32_t *d_pair_wrec = nullptr;   // their records: s0, s1, rbeg[5], rcum[6], padding (16 int32)
    int64_t *d_pair_wseg = nullptr;   // first segment of each work cell, [n_work + 1]
    int64_t *d_pair_off = nullptr, *d_pair_doff = nullptr;   // [n_seg * kFastSrc + 1]
    int64_t pair_nword = 0;           // pair words, segments padded to whole 256-pair blocks
    double *d_pair_dw = nullptr;      // eta_d(r) of each pair with r < dt/2, [n_dy_pairs][nlev]
    int32_t n_cu = 256;               // compute units of the device (persistent grids)
    void *scratch = nullptr;          // this device's fixed workspace (see scratch_address)
    // host-pointer mode: device and pinned host staging of one sample vector and one field
    double *d_sig_in = nullptr, *d_u_out = nullptr;
    double *h_sig_stage = nullptr, *h_u_stage = nullptr;   // hipHostMalloc
    hipEvent_t ev_sig_copied = nullptr;                     // the last sample copy has left h_sig_stage
    // non-finite check: device count of non-finite samples (ingest kernel), copied to pinned
    // host memory after each evaluation; counts up to `nonfinite_reported` have been reported
    unsigned long long *d_nonfinite = nullptr;
    unsigned long long *h_nonfinite = nullptr;              // hipHostMalloc, one word
    unsigned long long nonfinite_reported = 0;
    uint64_t *d_pair_pw = nullptr;    // regular pairs, one packed word each
    uint32_t *d_pair_dent = nullptr;
    int32_t *d_pair_dtg = nullptr, *d_pair_dsg = nullptr;   // pairs with r < dt/2: sorted target, source
    int64_t pair_ndy = 0;
    int32_t pc_skip = 0;              //   the regular panels' table is zero below each panel's level (MFMA k-steps skipped)
    int32_t pc_rb = 0, pc_nprod = 0;  //   its variant: MFMA row blocks per producer, producer waves
    double init_ms[7] = {};           // set-up phases (wfp2d_info.init_ms)
    std::vector<double> h_class_kappa; // |k| of each distinct far-mode class (rows of d_H)
    void *d_pc_desc = nullptr;        // producer / consumer kernel: item descriptors (32 bytes each)
    int32_t *d_pc_ioff = nullptr;     //   first item of each workgroup
    int32_t pc_grid = 0;              //   workgroups (one per CU); 0 = kernel not used

    std::string err;

    // what the plan was made from (to build its transpose) and the evolving state
    std::vector<double> h_src_xy, h_tgt_xy;          // caller order, [n][2]
    wfp2d_opts opts{};
    std::vector<std::pair<void *, size_t>> state_bufs;   // device buffers carried from step to step

    // graph replay of one step + evaluation
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int32_t batch_refs = 0;           // batches whose graphs hold this plan's buffers

    // stage timing (events recorded around launches when enabled)
    static constexpr int kStages = 12;
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;             // pairs: start, stop
    std::vector<int> ev_stage;                   // stage of each recorded pair
    double stage_ms[kStages] = {};
    int64_t stage_n[kStages] = {};

    template <class T>
    T *alloc(int64_t count);
    void release(void *ptr);          // free one allocation made by alloc
    ~Plan();
};

}  // namespace wfp2d
