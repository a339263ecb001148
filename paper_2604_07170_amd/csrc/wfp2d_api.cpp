// Plan construction, step / evaluate orchestration and the C ABI of wfp2d.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>
#include <stdexcept>
#include <string>
#include <vector>

#include "wfp2d_internal.h"
#include "wfp2d_tables.h"

struct wfp2d_plan_s {
    wfp2d::Plan p;
};

namespace wfp2d {

struct Failure {
    wfp2d_status code;
    std::string msg;
};

[[noreturn]] static void fail(wfp2d_status code, const std::string &msg) { throw Failure{code, msg}; }

static void hip_check(hipError_t e, const char *what)
{
    if (e != hipSuccess) fail(WFP2D_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

template <class T>
T *Plan::alloc(int64_t count)
{
    void *ptr = nullptr;
    size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
    hipError_t e = hipMalloc(&ptr, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(WFP2D_ERR_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    allocs.push_back(ptr);
    alloc_bytes.push_back(bytes);
    bytes_device += (int64_t)bytes;
    hip_check(hipMemset(ptr, 0, bytes), "hipMemset");
    return (T *)ptr;
}

void Plan::release(void *ptr)
{
    if (!ptr) return;
    for (size_t i = 0; i < allocs.size(); ++i)
        if (allocs[i] == ptr) {
            (void)hipFree(ptr);
            bytes_device -= (int64_t)alloc_bytes[i];
            allocs.erase(allocs.begin() + (std::ptrdiff_t)i);
            alloc_bytes.erase(alloc_bytes.begin() + (std::ptrdiff_t)i);
            return;
        }
}

Plan::~Plan()
{
    if (stream) (void)hipStreamSynchronize(stream);
    else (void)hipDeviceSynchronize();
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    if (ev_sig_copied) (void)hipEventDestroy(ev_sig_copied);
    if (h_sig_stage) (void)hipHostFree(h_sig_stage);
    if (h_u_stage) (void)hipHostFree(h_u_stage);
    if (h_nonfinite) (void)hipHostFree(h_nonfinite);
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (void *ptr : allocs) (void)hipFree(ptr);
}

// fold the elapsed times of the recorded event pairs into the accumulators
static void drain_timing(Plan &p)
{
    if (p.ev_stage.empty()) return;
    hip_check(p.stream ? hipStreamSynchronize(p.stream) : hipDeviceSynchronize(), "synchronize");
    for (size_t i = 0; i < p.ev_stage.size(); ++i) {
        float ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, p.ev_pool[2 * i], p.ev_pool[2 * i + 1]), "hipEventElapsedTime");
        p.stage_ms[p.ev_stage[i]] += ms;
        p.stage_n[p.ev_stage[i]] += 1;
    }
    p.ev_stage.clear();
}

// run one launcher, bracketed by events when timing is enabled
template <class F>
static void timed(Plan &p, int stage, const char *what, F &&launch)
{
    if (!p.timing) {
        hip_check(launch(), what);
        return;
    }
    size_t k = p.ev_stage.size();
    if (2 * k + 2 > p.ev_pool.size()) {
        if (k >= 256) {
            drain_timing(p);
            k = 0;
        }
        while (2 * k + 2 > p.ev_pool.size()) {
            hipEvent_t e;
            hip_check(hipEventCreate(&e), "hipEventCreate");
            p.ev_pool.push_back(e);
        }
    }
    hip_check(hipEventRecord(p.ev_pool[2 * k], p.stream), "hipEventRecord");
    hip_check(launch(), what);
    hip_check(hipEventRecord(p.ev_pool[2 * k + 1], p.stream), "hipEventRecord");
    p.ev_stage.push_back(stage);
}

template <class T>
static void upload(T *dst, const std::vector<T> &src)
{
    if (src.empty()) return;
    hip_check(hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy H2D");
}

static int64_t next_pow2(int64_t v)
{
    int64_t q = 1;
    while (q < v) q <<= 1;
    return q;
}

// convert a host FP64 vector to the plan's real type and upload into a fresh buffer
static void *upload_real(Plan &p, const std::vector<double> &v)
{
    if (p.precision == WFP2D_PREC_MIXED) {
        std::vector<float> f(v.begin(), v.end());
        float *d = p.alloc<float>((int64_t)f.size());
        upload(d, f);
        return d;
    }
    double *d = p.alloc<double>((int64_t)v.size());
    upload(d, v);
    return d;
}

// Spreading tile shapes: code -> tile edge in x and y (fine-grid points); code 6 is the
// 16 x 16 tile summed as a contraction on the matrix cores.
static bool spread_tile_shape(int code, int &tx, int &ty)
{
    static const int shapes[7][2] = {{0, 0}, {8, 8}, {16, 8}, {16, 16}, {32, 16}, {32, 32}, {16, 16}};
    if (code < 1 || code > 6) return false;
    tx = shapes[code][0];
    ty = shapes[code][1];
    return true;
}

// Per-tile source lists of the spreading kernel for tile shape `code`: every
// source is listed in each tile its w x w kernel support meets.
static void build_spread_tiles(Plan &p, int code)
{
    int tx, ty;
    if (!spread_tile_shape(code, tx, ty)) fail(WFP2D_ERR_ARG, "spread tile code must be in [1, 6]");
    const Geom &g = p.g;
    const int w = g.w;
    const int ntx = (g.Lpad + tx - 1) / tx, nty = (g.Lpad + ty - 1) / ty;
    const int64_t ntile = (int64_t)ntx * nty;
    const std::vector<int2> &sb = p.h_src_base;
    const int64_t M = (int64_t)sb.size();
    std::vector<int32_t> off(ntile + 1, 0);
    for (int64_t j = 0; j < M; ++j)
        for (int y = sb[j].y / ty; y <= (sb[j].y + w - 1) / ty; ++y)
            for (int x = sb[j].x / tx; x <= (sb[j].x + w - 1) / tx; ++x) off[(int64_t)y * ntx + x + 1]++;
    for (int64_t t = 0; t < ntile; ++t) off[t + 1] += off[t];
    std::vector<int32_t> pos(off.begin(), off.end() - 1), lst(off[ntile]);
    for (int64_t j = 0; j < M; ++j)
        for (int y = sb[j].y / ty; y <= (sb[j].y + w - 1) / ty; ++y)
            for (int x = sb[j].x / tx; x <= (sb[j].x + w - 1) / tx; ++x) lst[pos[(int64_t)y * ntx + x]++] = (int32_t)j;
    p.release(p.d_tile_off);
    p.release(p.d_tile_src);
    p.d_tile_off = nullptr;
    p.d_tile_src = nullptr;
    p.d_tile_off = p.alloc<int32_t>(ntile + 1);
    upload(p.d_tile_off, off);
    p.d_tile_src = p.alloc<int32_t>(off[ntile]);
    upload(p.d_tile_src, lst);
    p.spread_tile = code;
    p.sp_tx = tx;
    p.sp_ty = ty;
    p.sp_ntx = ntx;
    p.sp_nty = nty;
}

// Pair lists of the local part (layout in k_pairs_build).  Built when the plan
// can use the MFMA local kernels and the lists take at most half of the free
// device memory; otherwise the local part finds its pairs at every step.
// Segments: per work cell (sources, and targets in its 5 x 5 block),
// ceil(sources / kFastSrc) chunks times ceil(block targets / kPairTB) batches,
// numbered cell by cell.
static void build_pair_lists(Plan &p, const std::vector<int32_t> &cell_start, const std::vector<int32_t> &tcell_start)
{
    const int n = p.ncell;
    std::vector<int32_t> wrec;
    std::vector<int64_t> wseg(1, 0);
    // a work unit is kPairUnit adjacent cells of one row: their sources are contiguous in
    // the sorted order, and the union of their 5 x 5 blocks (kPairUnit + 4 cells wide) holds
    // every target within delta of any of them
    for (int c = 0; c < n * n; c += (c % n + kPairUnit <= n - 1) ? kPairUnit : n - c % n) {
        const int cx = c % n, cy = c / n, cx1 = std::min(n - 1, cx + kPairUnit - 1);
        const int32_t s0 = cell_start[c], s1 = cell_start[(size_t)cy * n + cx1 + 1];
        if (s1 == s0) continue;
        const int xa = std::max(0, cx - 2), xb = std::min(n - 1, cx1 + 2);
        int32_t rec[kPairRec] = {s0, s1};
        int32_t cum = 0;
        int r = 0;
        for (int yy = std::max(0, cy - 2); yy <= std::min(n - 1, cy + 2); ++yy, ++r) {
            const int32_t b = tcell_start[(size_t)yy * n + xa], e = tcell_start[(size_t)yy * n + xb + 1];
            rec[2 + r] = b;
            rec[7 + r] = cum;
            cum += e - b;
        }
        for (; r < 5; ++r) rec[7 + r] = cum;
        rec[12] = cum;
        if (cum == 0) continue;
        const int64_t nseg = (int64_t)(s1 - s0 + kFastSrc - 1) / kFastSrc * ((cum + kPairTB - 1) / kPairTB);
        wrec.insert(wrec.end(), rec, rec + kPairRec);
        wseg.push_back(wseg.back() + nseg);
    }
    p.pair_n_work = (int64_t)wseg.size() - 1;
    const int64_t nslot = wseg.back() * kFastSrc;
    if (nslot == 0 || p.pair_n_work > INT32_MAX) return;
    p.d_pair_wrec = p.alloc<int32_t>((int64_t)wrec.size());
    upload(p.d_pair_wrec, wrec);
    p.d_pair_wseg = p.alloc<int64_t>((int64_t)wseg.size());
    upload(p.d_pair_wseg, wseg);
    int64_t *d_cnt = p.alloc<int64_t>(nslot), *d_dcnt = p.alloc<int64_t>(nslot);
    hip_check(launch_pairs_build(p, false, d_cnt, d_dcnt), "pair count");
    hip_check(hipStreamSynchronize(p.stream), "pair count");
    std::vector<int64_t> cnt(nslot), dcnt(nslot), off(nslot + 1, 0), doff(nslot + 1, 0), seg_end(nslot / kFastSrc);
    hip_check(hipMemcpy(cnt.data(), d_cnt, nslot * sizeof(int64_t), hipMemcpyDeviceToHost), "hipMemcpy D2H");
    hip_check(hipMemcpy(dcnt.data(), d_dcnt, nslot * sizeof(int64_t), hipMemcpyDeviceToHost), "hipMemcpy D2H");
    p.release(d_cnt);
    p.release(d_dcnt);
    // regular pairs: each segment's slots back to back, each (slot, panel) group in whole runs
    int64_t npair = 0, nreal = 0;
    for (int64_t s = 0; s < nslot; ++s) {
        off[s] = npair;
        npair += cnt[s] & 0xFFFFFFFF;                 // words: pairs and the padding of each panel's run
        nreal += cnt[s] >> 32;
        if ((s + 1) % kFastSrc == 0) {
            npair = (npair + kPairBlockPad - 1) / kPairBlockPad * kPairBlockPad;
            seg_end[s / kFastSrc] = npair;
        }
        doff[s + 1] = doff[s] + dcnt[s];
    }
    off[nslot] = npair;
    const int64_t ndy = doff.back();
    const int64_t bytes = npair * (int64_t)sizeof(uint64_t) +
                          ndy * (int64_t)(3 * sizeof(uint32_t) + p.g.nlev * sizeof(double)) +
                          2 * (nslot + 1) * (int64_t)sizeof(int64_t);
    size_t free_b = 0, total_b = 0;
    hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
    if ((double)bytes > 0.5 * (double)free_b) {
        p.release(p.d_pair_wrec);
        p.release(p.d_pair_wseg);
        p.d_pair_wrec = nullptr;
        p.d_pair_wseg = nullptr;
        return;
    }
    p.d_pair_off = p.alloc<int64_t>(nslot + 1);
    p.d_pair_doff = p.alloc<int64_t>(nslot + 1);
    upload(p.d_pair_off, off);
    upload(p.d_pair_doff, doff);
    p.pair_nword = npair;
    p.d_pair_pw = p.alloc<uint64_t>(npair);
    p.d_pair_dent = p.alloc<uint32_t>(ndy);
    p.d_pair_dw = p.alloc<double>(ndy * p.g.nlev);
    p.d_pair_dtg = p.alloc<int32_t>(ndy);
    p.d_pair_dsg = p.alloc<int32_t>(ndy);
    p.pair_ndy = ndy;
    hip_check(launch_pairs_build(p, true, nullptr, nullptr), "pair fill");
    hip_check(hipStreamSynchronize(p.stream), "pair fill");
    {
        // items of the producer / consumer local kernel: workgroup g takes work units g, g + G, ...,
        // each unit batch by batch, each batch chunk by chunk (one segment per item)
        const int64_t G = std::max<int64_t>(1, std::min<int64_t>(p.pair_n_work, p.n_cu));
        struct Desc {
            int64_t p0, p1;
            int32_t sb, ns, wk, b;
        };
        static_assert(sizeof(Desc) == 32, "item descriptor layout");
        std::vector<Desc> items;
        std::vector<int32_t> ioff(1, 0);
        for (int64_t g = 0; g < G; ++g) {
            for (int64_t wk = g; wk < p.pair_n_work; wk += G) {
                const int32_t *rec = &wrec[(size_t)wk * kPairRec];
                const int s0 = rec[0], s1 = rec[1], NT = rec[12];
                const int nb = (NT + kPairTB - 1) / kPairTB, nch = (s1 - s0 + kFastSrc - 1) / kFastSrc;
                for (int b = 0; b < nb; ++b)
                    for (int c = 0; c < nch; ++c) {
                        const int64_t seg = wseg[wk] + (int64_t)c * nb + b;
                        const int sb = s0 + c * kFastSrc;
                        items.push_back(Desc{off[seg * kFastSrc], seg_end[seg], sb, std::min(kFastSrc, s1 - sb),
                                             (int32_t)wk, b});
                    }
            }
            if ((int64_t)items.size() > INT32_MAX) return;
            ioff.push_back((int32_t)items.size());
        }
        p.d_pc_desc = p.alloc<Desc>((int64_t)items.size());
        upload((Desc *)p.d_pc_desc, items);
        p.d_pc_ioff = p.alloc<int32_t>((int64_t)ioff.size());
        upload(p.d_pc_ioff, ioff);
        p.pc_grid = (int32_t)G;
    }
    p.local_pairs = true;
    p.pair_bytes = bytes;
    p.n_local_pairs = nreal + ndy;
}

static void build(Plan &p, const double *src_xy, const double *tgt_xy)
{
    // wall-clock time of the set-up phases (wfp2d_info.init_ms)
    using clk = std::chrono::steady_clock;
    const clk::time_point t_start = clk::now();
    clk::time_point t_mark = t_start;
    auto phase = [&](int k) {
        const clk::time_point now = clk::now();
        p.init_ms[k] += std::chrono::duration<double, std::milli>(now - t_mark).count();
        t_mark = now;
    };
    hip_check(hipSetDevice(p.device), "hipSetDevice");
    hip_check(scratch_address(p.device, &p.scratch), "hipGetSymbolAddress of the fixed workspace");
    {
        int ncu = 0;
        hip_check(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p.device), "hipDeviceGetAttribute");
        p.n_cu = std::max(1, ncu);
    }
    const int64_t M = p.M, Nx = p.Nx;
    p.sizeof_real = (p.precision == WFP2D_PREC_MIXED) ? 4 : 8;

    // ---------------- parameters ----------------
    Params P = derive_params(p.dt, p.W, p.tol, p.Delta, p.a, p.Kf, p.p, p.lookahead);
    if (!(M_PI - 2.0 * P.b / p.W > 0.0))
        fail(WFP2D_ERR_INFEASIBLE, "pi - 2b/W <= 0: no time step satisfies eq. dt for this W and tol");
    p.b = P.b;
    p.delta = P.delta;
    p.A = P.A;
    p.Aplus = P.Aplus;
    p.a = P.a;
    p.dk = P.dk;
    p.K = P.K;
    p.Kmax = P.Kmax;
    p.LA = P.LA;
    p.lookahead = P.lookahead;
    if (p.LA < p.W + p.p) fail(WFP2D_ERR_INFEASIBLE, "time step too large for the near-history window");
    const int64_t R = P.R, N = 2 * R + 1;

    Geom &g = p.g;
    g.M = M;
    g.Nx = Nx;
    g.W = p.W;
    g.LA = (int32_t)p.LA;
    g.dt = p.dt;
    g.dk = p.dk;
    g.K = p.K;
    g.Kf = p.Kf;
    g.Kmax = p.Kmax;
    g.Rd2 = (p.Kmax / p.dk) * (p.Kmax / p.dk);
    g.R = (int32_t)R;
    g.N = (int32_t)N;

    // ---------------- NUFFT grid ----------------
    double tol_nufft = p.nufft_tol > 0 ? p.nufft_tol : (p.precision == WFP2D_PREC_MIXED ? 1e-7 : 1e-11);
    int w = (int)std::ceil(std::log10(1.0 / tol_nufft)) + 1;
    w = std::max(4, std::min(16, w));
    p.es_beta = 2.30 * w;
    const int64_t qmax = (p.precision == WFP2D_PREC_MIXED) ? 8192 : 4096;
    int64_t best_nf = -1;
    for (int P_ = 1; P_ <= 3; ++P_) {
        int64_t Q = std::max<int64_t>(256, next_pow2((2 * N + P_ - 1) / P_));
        int64_t nf = P_ * Q;
        double gmax = p.dk * (double)nf / (2.0 * M_PI);
        int64_t lmin = (int64_t)std::ceil(-gmax - 0.5 * w);
        int64_t lmax = (int64_t)std::floor(gmax + 0.5 * w);
        int64_t Lb = lmax - lmin + 1;
        int64_t Lpad = (Lb + kTile - 1) / kTile * kTile;
        if (Lpad > Q || Q > qmax) continue;
        if (best_nf < 0 || nf < best_nf) {
            best_nf = nf;
            g.nf = (int32_t)nf;
            g.P = P_;
            g.Q = (int32_t)Q;
            g.lmin = (int32_t)lmin;
            g.Lpad = (int32_t)Lpad;
        }
    }
    if (best_nf < 0) fail(WFP2D_ERR_INFEASIBLE, "Fourier grid too large for the single-workgroup FFT");
    // Q >= 2N/P by construction; the FP32 type-1 transform's slot layout relies on it
    if (2 * (int64_t)N > (int64_t)g.P * g.Q) fail(WFP2D_ERR_INFEASIBLE, "Fourier grid shorter than the kept modes");
    g.w = w;
    g.ntx = g.Lpad / kTile;

    // ---------------- modes: packed half disk, column-major in nx ----------------
    p.col_off.assign(R + 2, 0);
    p.col_ny0.assign(R + 1, 0);
    for (int64_t nx = 0; nx <= R; ++nx) {
        double rem = g.Rd2 - (double)(nx * nx);
        int64_t h = rem >= 0 ? (int64_t)std::floor(std::sqrt(rem)) : -1;
        while (h >= 0 && (double)((h + 1) * (h + 1) + nx * nx) <= g.Rd2) ++h;
        while (h >= 0 && (double)(h * h + nx * nx) > g.Rd2) --h;
        int64_t cnt = h < 0 ? 0 : (nx == 0 ? h + 1 : 2 * h + 1);
        p.col_ny0[nx] = (int32_t)(nx == 0 ? 0 : -h);
        p.col_off[nx + 1] = p.col_off[nx] + (int32_t)cnt;
        for (int64_t off = 0; off < cnt; off += kChunk)
            p.chunks.push_back(ModeChunk{(int32_t)nx, (int32_t)(p.col_ny0[nx] + off),
                                         (int32_t)(p.col_off[nx] + off), (int32_t)std::min<int64_t>(kChunk, cnt - off)});
    }
    p.n_modes = p.col_off[R + 1];
    p.n_chunks = (int64_t)p.chunks.size();
    std::vector<int32_t> far_pk, far_key;
    const double K2 = p.K * p.K, Kf2 = p.Kf * p.Kf, dk2 = p.dk * p.dk;
    for (int64_t nx = 0; nx <= R; ++nx)
        for (int64_t i = 0; i < p.col_off[nx + 1] - p.col_off[nx]; ++i) {
            int64_t ny = p.col_ny0[nx] + i;
            int64_t key = nx * nx + ny * ny;
            if ((double)key * dk2 <= K2) ++p.n_near;
            if ((double)key * dk2 <= Kf2) {
                far_pk.push_back((int32_t)(p.col_off[nx] + i));
                far_key.push_back((int32_t)key);
            }
        }
    p.n_far = (int64_t)far_pk.size();
    std::vector<int32_t> keys(far_key);
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    p.n_classes = (int64_t)keys.size();
    std::vector<int32_t> far_cls(p.n_far);
    for (int64_t f = 0; f < p.n_far; ++f)
        far_cls[f] = (int32_t)(std::lower_bound(keys.begin(), keys.end(), far_key[f]) - keys.begin());

    // ---------------- geometry: sort by local cell ----------------
    // cells of side >= delta/2 (the 5 x 5 block then covers every pair with r < delta); larger cells are
    // also correct, so the count is capped to keep the cell tables small
    p.ncell = std::max(1, std::min(8192, (int)std::floor(4.0 / p.delta)));
    p.cell_h = 2.0 / p.ncell;
    auto cell_of = [&](double x, double y) {
        int cx = std::min(p.ncell - 1, std::max(0, (int)std::floor((x + 1.0) / p.cell_h)));
        int cy = std::min(p.ncell - 1, std::max(0, (int)std::floor((y + 1.0) / p.cell_h)));
        return cy * p.ncell + cx;
    };
    std::vector<int32_t> scell(M), sperm(M);
    for (int64_t j = 0; j < M; ++j) scell[j] = cell_of(src_xy[2 * j], src_xy[2 * j + 1]);
    std::iota(sperm.begin(), sperm.end(), 0);
    std::stable_sort(sperm.begin(), sperm.end(), [&](int32_t a, int32_t b) { return scell[a] < scell[b]; });
    std::vector<int32_t> cell_start((size_t)p.ncell * p.ncell + 1, 0);
    for (int64_t j = 0; j < M; ++j) cell_start[scell[j] + 1]++;
    for (size_t c = 1; c < cell_start.size(); ++c) cell_start[c] += cell_start[c - 1];
    std::vector<int32_t> tcell(Nx), tperm(Nx), trank(Nx);
    for (int64_t i = 0; i < Nx; ++i) tcell[i] = cell_of(tgt_xy[2 * i], tgt_xy[2 * i + 1]);
    std::iota(tperm.begin(), tperm.end(), 0);
    std::stable_sort(tperm.begin(), tperm.end(), [&](int32_t a, int32_t b) { return tcell[a] < tcell[b]; });
    for (int64_t i = 0; i < Nx; ++i) trank[tperm[i]] = (int32_t)i;
    std::vector<int32_t> tcell_start((size_t)p.ncell * p.ncell + 1, 0);
    for (int64_t i = 0; i < Nx; ++i) tcell_start[tcell[i] + 1]++;
    for (size_t c = 1; c < tcell_start.size(); ++c) tcell_start[c] += tcell_start[c - 1];
    std::vector<double2> sxy(M), txy(Nx);
    std::vector<int32_t> tcell_sorted(Nx);
    for (int64_t j = 0; j < M; ++j) sxy[j] = make_double2(src_xy[2 * sperm[j]], src_xy[2 * sperm[j] + 1]);
    for (int64_t i = 0; i < Nx; ++i) {
        txy[i] = make_double2(tgt_xy[2 * tperm[i]], tgt_xy[2 * tperm[i] + 1]);
        tcell_sorted[i] = tcell[tperm[i]];
    }

    phase(0);                                         // modes and geometry
    // spreading / interpolation kernel data, tile lists
    const double gscale = p.dk * g.nf / (2.0 * M_PI);
    auto kernel_data = [&](const std::vector<double2> &pts, std::vector<int2> &base) {
        const int64_t n = (int64_t)pts.size();
        // the origins here; the 2w kernel weights per point on the device (k_es_weights)
        base.resize(n);
        bool inside = true;
#pragma omp parallel for schedule(static) reduction(&& : inside)
        for (int64_t j = 0; j < n; ++j) {
            double gx = pts[j].x * gscale, gy = pts[j].y * gscale;
            int64_t l0x = (int64_t)std::ceil(gx - 0.5 * w), l0y = (int64_t)std::ceil(gy - 0.5 * w);
            base[j] = make_int2((int)(l0x - g.lmin), (int)(l0y - g.lmin));
            inside = inside && !(base[j].x < 0 || base[j].y < 0 || base[j].x + w > g.Lpad || base[j].y + w > g.Lpad);
        }
        if (!inside) fail(WFP2D_ERR_DOMAIN, "point outside the spreading band");
    };
    std::vector<int2> sbase, tbase;
    kernel_data(sxy, sbase);
    kernel_data(txy, tbase);
    const int ntile = g.ntx * g.ntx;
    p.h_src_base = sbase;
    build_spread_tiles(p, p.spread_tile);
    // interpolation: each target belongs to the tile holding its kernel origin
    {
        std::vector<int32_t> off(ntile + 1, 0), lst(Nx);
        for (int64_t i = 0; i < Nx; ++i) off[(tbase[i].y / kTile) * g.ntx + tbase[i].x / kTile + 1]++;
        for (int t = 0; t < ntile; ++t) off[t + 1] += off[t];
        std::vector<int32_t> pos(off.begin(), off.end() - 1);
        for (int64_t i = 0; i < Nx; ++i) lst[pos[(tbase[i].y / kTile) * g.ntx + tbase[i].x / kTile]++] = (int32_t)i;
        // origins (and, on the device, weights) in this processing order, so that the
        // interpolation kernel reads them without waiting for the target index
        std::vector<int2> tb(Nx);
        for (int64_t e = 0; e < Nx; ++e) tb[e] = tbase[lst[e]];
        tbase.swap(tb);
        p.d_ttile_off = p.alloc<int32_t>(ntile + 1);
        upload(p.d_ttile_off, off);
        p.d_ttile_tgt = p.alloc<int32_t>(Nx);
        upload(p.d_ttile_tgt, lst);
    }

    phase(1);                                         // NUFFT point data
    // ---------------- tables ----------------
    Blend phi(p.delta, p.b, 160);
    std::vector<double> phi_in(p.W + 1);
    for (int l = 0; l <= p.W; ++l) phi_in[l] = phi.phi(l * p.dt);
    phi_in[0] = 0.0;
    phi_in[p.W] = 1.0;

    std::vector<double> lam, qw;
    soe_nodes(lam, qw);
    std::vector<double> kap(p.n_classes);
    for (int64_t c = 0; c < p.n_classes; ++c) kap[c] = p.dk * std::sqrt((double)keys[c]);
    p.h_class_kappa = kap;
    // Hankel coefficients of eq. H, one row per distinct |k|^2 of the far modes: the quadrature
    // in r on the host, the contraction with J0(kappa r) on the device (k_hankel)
    std::vector<double> H((size_t)p.n_classes * kNsoe);
    p.d_H = p.alloc<double>(std::max<int64_t>(1, p.n_classes * kNsoe));
    if (p.n_classes > 0) {
        std::vector<double> hr, hE;
        hankel_quadrature(p.A, p.Delta, p.b_Delta, lam, qw, hr, hE);
        double *d_kap = p.alloc<double>(p.n_classes), *d_r = p.alloc<double>((int64_t)hr.size());
        double *d_E = p.alloc<double>((int64_t)hE.size());
        upload(d_kap, kap);
        upload(d_r, hr);
        upload(d_E, hE);
        hip_check(launch_hankel(p, d_kap, p.n_classes, d_r, (int)hr.size(), d_E, kNsoe, p.d_H), "Hankel coefficients");
        hip_check(hipMemcpyAsync(H.data(), p.d_H, H.size() * sizeof(double), hipMemcpyDeviceToHost, p.stream), "copy");
        hip_check(p.stream ? hipStreamSynchronize(p.stream) : hipDeviceSynchronize(), "synchronize");
        p.release(d_kap);
        p.release(d_r);
        p.release(d_E);
    }
    std::vector<double> dec(kNsoe), inj(kNsoe), chi((size_t)p.n_classes * (p.W - 1));
    for (int l = 0; l < kNsoe; ++l) {
        dec[l] = std::exp(-lam[l] * p.dt);
        inj[l] = p.dt * std::exp(-lam[l] * ((double)(p.LA + p.W - 1) * p.dt - p.A));
    }
    // window FIR per class: chi[c][i] = (1 - phi) sum_l H[c][l] dt e^{-lambda_l ((LA + 1 + i) dt - A)}
    std::vector<double> fir((size_t)(p.W - 1) * kNsoe);
    for (int i = 0; i < p.W - 1; ++i)
        for (int l = 0; l < kNsoe; ++l)
            fir[(size_t)i * kNsoe + l] = p.dt * std::exp(-lam[l] * ((double)(p.LA + 1 + i) * p.dt - p.A));
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < p.n_classes; ++c)
        for (int i = 0; i < p.W - 1; ++i) {
            double s = 0.0;
            for (int l = 0; l < kNsoe; ++l) s += H[(size_t)c * kNsoe + l] * fir[(size_t)i * kNsoe + l];
            chi[(size_t)c * (p.W - 1) + i] = s * (1.0 - phi_in[p.W - 1 - i]);
        }

    phase(2);                                         // history tables
    const int lev_min = -p.lookahead;
    LocalWeights LW(p.dt, p.W, p.p, lev_min, phi);
    LocalTable LT = build_local_table(LW, 40, 1e-11);
    g.nlev = LT.nlev;
    g.lev_min = lev_min;
    p.n_sub = (int32_t)LT.subs.size();
    p.subs = LT.subs;
    p.dy_base = LT.dy_base;
    p.n_dy = LT.n_dy;
    // sigma history: the lagged type-1 input reaches m - LA; the local part reaches m - dmax
    int64_t dmax = lev_min + LT.nlev - 1;
    g.sig_depth = std::max<int64_t>(p.LA, dmax) + p.lookahead + 1;


    // NUFFT correction and twiddles
    std::vector<double> psihat;
    es_fourier(w, p.es_beta, g.nf, R, psihat);
    std::vector<double> corr(2 * N), tw(2 * (size_t)g.nf);
    for (int64_t n = -R; n <= R; ++n) {
        double ang = 2.0 * M_PI * (double)(n * g.lmin % g.nf) / (double)g.nf;
        corr[2 * (n + R)] = std::cos(ang) / psihat[n + R];
        corr[2 * (n + R) + 1] = std::sin(ang) / psihat[n + R];
    }
    for (int64_t j = 0; j < g.nf; ++j) {
        tw[2 * j] = std::cos(2.0 * M_PI * (double)j / (double)g.nf);
        tw[2 * j + 1] = std::sin(2.0 * M_PI * (double)j / (double)g.nf);
    }

    phase(3);                                         // local tables, NUFFT corrections
    // ---------------- device memory ----------------
    const int64_t sr = p.sizeof_real;
    g.lookahead = p.lookahead;
    p.d_step = p.alloc<int64_t>(1);
    p.d_sig = p.alloc<double>(g.sig_depth * M);
    p.d_src_perm = p.alloc<int32_t>(M);
    upload(p.d_src_perm, sperm);
    p.d_tgt_rank = p.alloc<int32_t>(Nx);
    upload(p.d_tgt_rank, trank);
    p.d_src_xy = p.alloc<double2>(M);
    upload(p.d_src_xy, sxy);
    p.d_tgt_xy = p.alloc<double2>(Nx);
    upload(p.d_tgt_xy, txy);
    p.d_src_base = p.alloc<int2>(M);
    upload(p.d_src_base, sbase);
    p.d_tgt_base = p.alloc<int2>(Nx);
    upload(p.d_tgt_base, tbase);
    // exponential-of-semicircle weights of every source (sorted order) and target (processing
    // order), 2w per point, in the grid precision
    p.d_src_wts = p.alloc<char>(M * 2 * w * sr);
    p.d_tgt_wts = p.alloc<char>(Nx * 2 * w * sr);
    hip_check(launch_es_weights(p, p.d_src_xy, nullptr, p.d_src_base, M, gscale, p.d_src_wts), "source weights");
    hip_check(launch_es_weights(p, p.d_tgt_xy, p.d_ttile_tgt, p.d_tgt_base, Nx, gscale, p.d_tgt_wts), "target weights");
    p.d_grid = p.alloc<char>((int64_t)g.Lpad * g.Lpad * 2 * sr);
    p.d_T1 = p.alloc<char>((int64_t)g.Lpad * N * 2 * sr);
    p.d_T1t = p.alloc<char>((int64_t)g.Lpad * N * 2 * sr);
    p.d_F = p.alloc<char>(N * N * 2 * sr);
    p.d_corr = upload_real(p, corr);
    {
        double *d = p.alloc<double>((int64_t)tw.size());   // FP64 in both forms: staged into LDS tables
        upload(d, tw);
        p.d_tw = d;
    }
    p.d_ring_cur = p.alloc<char>((int64_t)p.W * p.n_modes * 2 * sr);
    p.d_ring_lag = p.alloc<char>((int64_t)p.W * p.n_modes * 2 * sr);
    p.d_chunks = p.alloc<ModeChunk>(p.n_chunks);
    upload(p.d_chunks, p.chunks);
    p.d_col_off = p.alloc<int32_t>(R + 2);
    upload(p.d_col_off, p.col_off);
    p.d_col_ny0 = p.alloc<int32_t>(R + 1);
    upload(p.d_col_ny0, p.col_ny0);
    p.d_D = p.alloc<double2>(p.n_modes);
    p.d_C = p.alloc<double2>(p.n_modes);
    p.d_phi_in = p.alloc<double>(p.W + 1);
    upload(p.d_phi_in, phi_in);
    p.d_atot = p.alloc<char>(p.n_modes * 2 * sr);
    p.d_far_pk = p.alloc<int32_t>(p.n_far);
    upload(p.d_far_pk, far_pk);
    p.d_far_cls = p.alloc<int32_t>(p.n_far);
    upload(p.d_far_cls, far_cls);
    // d_H holds the Hankel table computed above
    p.d_chi = p.alloc<double>(p.n_classes * (p.W - 1));
    upload(p.d_chi, chi);
    p.d_dec = p.alloc<double>(kNsoe);
    upload(p.d_dec, dec);
    p.d_inj = p.alloc<double>(kNsoe);
    upload(p.d_inj, inj);
    p.d_B = p.alloc<double2>(p.n_far * kNsoe);
    p.d_T2 = p.alloc<char>((R + 1) * (int64_t)g.Lpad * 2 * sr);
    p.d_T2t = p.alloc<char>((R + 1) * (int64_t)g.Lpad * 2 * sr);
    p.d_cgrid = p.alloc<char>((int64_t)g.Lpad * g.Lpad * sr);
    p.d_uh = p.alloc<double>(Nx);
    p.d_ul = p.alloc<double>(Nx);
    p.d_cell_start = p.alloc<int32_t>((int64_t)cell_start.size());
    upload(p.d_cell_start, cell_start);
    p.d_tcell_start = p.alloc<int32_t>((int64_t)tcell_start.size());
    upload(p.d_tcell_start, tcell_start);
    p.d_subs = p.alloc<SubPanel>(p.n_sub);
    upload(p.d_subs, LT.subs);
    {
        // tables scaled by 1/(2 pi) (eq. local2); regular sub-panels also in [sub][c][d] order
        const double s2pi = 0.5 / M_PI;
        std::vector<double> cheb(LT.coef);
        for (double &v : cheb) v *= s2pi;
        p.d_cheb = p.alloc<double>((int64_t)cheb.size());
        upload(p.d_cheb, cheb);
        p.n_reg = LT.dy_base;
        const int nl = LT.nlev, D = kChebDeg;
        std::vector<double> creg((size_t)p.n_reg * D * nl);
        for (int sp = 0; sp < p.n_reg; ++sp)
            for (int d = 0; d < nl; ++d)
                for (int c = 0; c < D; ++c)
                    creg[((size_t)sp * D + c) * nl + d] = s2pi * LT.coef[((size_t)sp * nl + d) * D + c];
        p.d_creg = p.alloc<double>((int64_t)creg.size());
        upload(p.d_creg, creg);
        if (nl > kLocalMaxLevels) fail(WFP2D_ERR_INFEASIBLE, "too many sigma levels for the local kernel (W + p too large)");
        p.local_sc = std::min<int>(kLocalMaxSrc, std::min(kLocalPsi / (p.n_reg * D), kLocalSig / nl));
        if (p.local_sc < 1) fail(WFP2D_ERR_INFEASIBLE, "local-weight tables too large for the local kernel");
        bool one_sub = true;
        for (int k = 0; k < p.W; ++k) one_sub = one_sub && LT.panel_l2n[k] == 0;
        p.local_fast = one_sub && p.n_reg * D <= kFastRow && (nl == 35 || nl == 43);
    }
    p.d_panel_base = p.alloc<int32_t>(p.W);
    upload(p.d_panel_base, LT.panel_base);
    p.d_panel_l2n = p.alloc<int32_t>(p.W);
    upload(p.d_panel_l2n, LT.panel_l2n);
    // Mixed precision: the pair-list kernel evaluates only the leading terms of each regular
    // panel's series when the dropped ones sum to at most 1e-3 tol, relative to the largest
    // coefficient (the scale of the fit criterion of the tables).  Measured, the field then
    // moves by about ten times that bound, two orders of magnitude below tol; FP64 plans use
    // every stored term.
    hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
    phase(4);                                         // device memory and uploads
    p.local_terms = p.precision == WFP2D_PREC_MIXED ? local_table_terms(LT, p.tol) : kChebDeg;
    {
        // every regular panel k has exactly zero coefficients on the levels d < k (its nodes lie
        // at delays >= k dt, and the centred stencils reach no further forward): the pair
        // kernel's LDS-table form then stores and multiplies only the levels from each row
        // block's first panel on
        bool zero_below = true;
        for (int sp = 0; sp < p.n_reg && zero_below; ++sp)
            for (int d = 0; d < std::min(sp, LT.nlev) && zero_below; ++d)
                for (int c = 0; c < p.local_terms; ++c)
                    if (LT.coef[((size_t)sp * LT.nlev + d) * kChebDeg + c] != 0.0) {
                        zero_below = false;
                        break;
                    }
        p.pc_skip = zero_below ? 1 : 0;
        p.pc_nprod = pc_producers(p.n_reg, p.local_terms, &p.pc_rb, LT.nlev, zero_below);
    }
    if (p.local_fast && p.W <= 64 && p.pc_nprod > 0 && p.opts.local_pairs == 0)
        build_pair_lists(p, cell_start, tcell_start);
    if (!p.local_pairs) p.local_terms = kChebDeg;
    if (p.local_pairs) {
        // the pair kernel sums each regular panel's truncated series by Horner's rule: the
        // same polynomials in the power basis, [n_reg][kChebDeg][nlev] (terms beyond
        // local_terms zero), scaled by 1/(2 pi)
        const int nl = LT.nlev, D = p.local_terms;
        const double s2pi = 0.5 / M_PI;
        std::vector<double> cpow((size_t)p.n_reg * kChebDeg * nl, 0.0), b(kChebDeg), a(kChebDeg);
        for (int sp = 0; sp < p.n_reg; ++sp)
            for (int d = 0; d < nl; ++d) {
                for (int c = 0; c < kChebDeg; ++c) b[c] = LT.coef[((size_t)sp * nl + d) * kChebDeg + c];
                cheb_to_power(b.data(), D, a.data());
                for (int c = 0; c < D; ++c) cpow[((size_t)sp * kChebDeg + c) * nl + d] = s2pi * a[c];
            }
        p.d_cpow = p.alloc<double>((int64_t)cpow.size());
        upload(p.d_cpow, cpow);
    }
    // local-pair count (reported; without pair lists the local kernel finds pairs through the cell lists)
    if (!p.local_pairs) {
        int64_t cnt = 0;
        const double d2 = p.delta * p.delta;
        for (int64_t i = 0; i < Nx; ++i) {
            int c = tcell_sorted[i], cx = c % p.ncell, cy = c / p.ncell;
            for (int yy = std::max(0, cy - 2); yy <= std::min(p.ncell - 1, cy + 2); ++yy)
                for (int xx = std::max(0, cx - 2); xx <= std::min(p.ncell - 1, cx + 2); ++xx) {
                    int cc = yy * p.ncell + xx;
                    for (int32_t j = cell_start[cc]; j < cell_start[cc + 1]; ++j) {
                        double dx = txy[i].x - sxy[j].x, dy = txy[i].y - sxy[j].y, r2 = dx * dx + dy * dy;
                        if (r2 > 0.0 && r2 < d2) ++cnt;
                    }
                }
        }
        p.n_local_pairs = cnt;
    }
    if (p.opts.host_pointers) {
        p.d_sig_in = p.alloc<double>(M);
        p.d_u_out = p.alloc<double>(Nx);
        hip_check(hipHostMalloc((void **)&p.h_sig_stage, (size_t)M * sizeof(double), hipHostMallocDefault),
                  "hipHostMalloc (sample staging)");
        hip_check(hipHostMalloc((void **)&p.h_u_stage, (size_t)Nx * sizeof(double), hipHostMallocDefault),
                  "hipHostMalloc (field staging)");
        hip_check(hipEventCreateWithFlags(&p.ev_sig_copied, hipEventDisableTiming), "hipEventCreate");
    }
    if (p.opts.check_finite) {
        p.d_nonfinite = p.alloc<unsigned long long>(1);
        hip_check(hipHostMalloc((void **)&p.h_nonfinite, sizeof(unsigned long long), hipHostMallocDefault),
                  "hipHostMalloc (non-finite count)");
        *p.h_nonfinite = 0;
    }
    p.state_bufs = {{p.d_step, sizeof(int64_t)},
                    {p.d_sig, (size_t)g.sig_depth * M * sizeof(double)},
                    {p.d_ring_cur, (size_t)p.W * p.n_modes * 2 * sr},
                    {p.d_ring_lag, (size_t)p.W * p.n_modes * 2 * sr},
                    {p.d_D, (size_t)p.n_modes * sizeof(double2)},
                    {p.d_C, (size_t)p.n_modes * sizeof(double2)},
                    {p.d_atot, (size_t)p.n_modes * 2 * sr},
                    {p.d_B, (size_t)p.n_far * kNsoe * sizeof(double2)}};
    phase(5);                                         // pair lists and the power-basis table
    hip_check(fft_setup(p), "FFT kernel attributes");
    hip_check(kernel_setup(p), "local kernel attributes");
    hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize after set-up");
    phase(5);
    p.init_ms[6] = std::chrono::duration<double, std::milli>(clk::now() - t_start).count();
}

// One step: a fixed sequence of launches whose arguments do not depend on the
// step index (the kernels read the device-resident step counter), so the
// sequence can also be captured in a graph.
static void enqueue_step(Plan &p, const double *sigma)
{
    timed(p, 0, "ingest", [&] {
        hipError_t e = launch_step_begin(p);
        return e != hipSuccess ? e : launch_ingest(p, sigma);
    });
    timed(p, 1, "spread", [&] { return launch_spread(p); });
    timed(p, 2, "fft rows (type 1)", [&] { return launch_fft_rows1(p); });
    timed(p, 3, "fft columns (type 1)", [&] { return launch_fft_cols1(p); });
    timed(p, 4, "hermitian split", [&] { return launch_split(p); });
    timed(p, 5, "near-history update", [&] { return launch_near(p); });
    timed(p, 6, "far-history update", [&] { return launch_far(p); });
}

static void enqueue_evaluate(Plan &p, double *u, const double *dot_w = nullptr, double *dot_acc = nullptr)
{
    timed(p, 7, "fft columns (type 2)", [&] { return launch_fft_cols2(p); });
    timed(p, 8, "fft rows (type 2)", [&] { return launch_fft_rows2(p); });
    timed(p, 9, "interpolation", [&] { return launch_interp(p); });
    timed(p, 10, "local part", [&] {
        hipError_t e = launch_zero_f64(p, p.d_ul, p.Nx);
        return e != hipSuccess ? e : launch_local(p);
    });
    timed(p, 11, "combine", [&] { return dot_acc ? launch_combine_dot(p, dot_w, dot_acc) : launch_combine(p, u); });
    if (p.d_nonfinite)
        hip_check(hipMemcpyAsync(p.h_nonfinite, p.d_nonfinite, sizeof(unsigned long long), hipMemcpyDeviceToHost, p.stream),
                  "non-finite count copy");
}

// true (once per new count) when the ingest kernel has counted non-finite samples
// that were not reported yet; reads the count copied back by the last finished evaluation
static bool nonfinite_news(Plan &p)
{
    if (!p.h_nonfinite) return false;
    const unsigned long long c = *(volatile unsigned long long *)p.h_nonfinite;
    if (c == p.nonfinite_reported) return false;
    p.nonfinite_reported = c;
    return true;
}

// sample vector for the kernels: the caller's device pointer, or (host-pointer plans) a
// device copy made through the pinned staging buffer; the caller's buffer is free on return
static const double *stage_sigma(Plan &p, const double *sigma)
{
    if (!p.opts.host_pointers) return sigma;
    hip_check(hipEventSynchronize(p.ev_sig_copied), "hipEventSynchronize");   // the previous copy has left the staging
    std::memcpy(p.h_sig_stage, sigma, (size_t)p.M * sizeof(double));
    hip_check(hipMemcpyAsync(p.d_sig_in, p.h_sig_stage, (size_t)p.M * sizeof(double), hipMemcpyHostToDevice, p.stream),
              "sample copy");
    hip_check(hipEventRecord(p.ev_sig_copied, p.stream), "hipEventRecord");
    return p.d_sig_in;
}

// evaluation into the caller's u (device), or into the device staging then back to the caller's
// host buffer (host-pointer plans; synchronises the stream)
template <class F>
static wfp2d_status evaluate_into(Plan &p, double *u, F &&enqueue)
{
    if (!p.opts.host_pointers) {
        enqueue(u);
        return nonfinite_news(p) ? WFP2D_ERR_NONFINITE : WFP2D_OK;
    }
    enqueue(p.d_u_out);
    hip_check(hipMemcpyAsync(p.h_u_stage, p.d_u_out, (size_t)p.Nx * sizeof(double), hipMemcpyDeviceToHost, p.stream),
              "field copy");
    hip_check(p.stream ? hipStreamSynchronize(p.stream) : hipDeviceSynchronize(), "synchronize");
    std::memcpy(u, p.h_u_stage, (size_t)p.Nx * sizeof(double));
    return nonfinite_news(p) ? WFP2D_ERR_NONFINITE : WFP2D_OK;
}

static void do_step(Plan &p, const double *sigma)
{
    hip_check(hipSetDevice(p.device), "hipSetDevice");
    const double *s = stage_sigma(p, sigma);
    p.steps += 1;
    enqueue_step(p, s);
}

// capture `body` (which enqueues on `st`) into an executable graph
template <class F>
static void capture_graph(hipStream_t st, hipGraph_t &graph, hipGraphExec_t &exec, F &&body)
{
    if (exec) {
        (void)hipGraphExecDestroy(exec);
        exec = nullptr;
    }
    if (graph) {
        (void)hipGraphDestroy(graph);
        graph = nullptr;
    }
    hip_check(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    try {
        body();
    } catch (...) {
        hipGraph_t g0 = nullptr;
        (void)hipStreamEndCapture(st, &g0);
        if (g0) (void)hipGraphDestroy(g0);
        throw;
    }
    hip_check(hipStreamEndCapture(st, &graph), "hipStreamEndCapture");
    hip_check(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
}

}  // namespace wfp2d

struct wfp2d_batch_s {
    std::vector<wfp2d_plan> plans;
    hipStream_t stream = nullptr;
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> events;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~wfp2d_batch_s()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        for (hipStream_t s : side) (void)hipStreamDestroy(s);
    }
};

using namespace wfp2d;

static std::string g_init_error;

#define WFP2D_GUARD(plan_ptr, ...)                                         \
    try {                                                                  \
        __VA_ARGS__;                                                       \
    } catch (const Failure &f) {                                           \
        if (plan_ptr) (plan_ptr)->p.err = f.msg;                           \
        else g_init_error = f.msg;                                         \
        return f.code;                                                     \
    } catch (const std::bad_alloc &) {                                     \
        if (plan_ptr) (plan_ptr)->p.err = "host allocation failed";        \
        else g_init_error = "host allocation failed";                      \
        return WFP2D_ERR_NOMEM;                                            \
    } catch (const std::exception &e) {                                    \
        if (plan_ptr) (plan_ptr)->p.err = e.what();                        \
        else g_init_error = e.what();                                      \
        return WFP2D_ERR_DEVICE;                                           \
    }

extern "C" {

wfp2d_status wfp2d_default_opts(wfp2d_opts *o)
{
    if (!o) return WFP2D_ERR_ARG;
    std::memset(o, 0, sizeof *o);
    o->precision = WFP2D_PREC_MIXED;
    o->interp_order = 20;
    o->lookahead = -1;
    o->Delta = 1.0;
    o->a = 0.0;
    o->Kf = 80.0;
    o->b_Delta = 30.0;
    o->nufft_tol = 0.0;
    o->max_steps = 0;
    o->device = 0;
    o->stream = nullptr;
    o->spread_tile = 0;
    o->local_pairs = 0;
    o->host_pointers = 0;
    o->check_finite = 0;
    return WFP2D_OK;
}

wfp2d_status wfp2d_init(wfp2d_plan *out, int64_t M, const double *src_xy, int64_t Nx, const double *tgt_xy,
                        double dt, int32_t window_W, double tol, const wfp2d_opts *opts)
{
    if (out) *out = nullptr;
    wfp2d_plan_s *h = nullptr;
    try {
        if (!out || !src_xy || !tgt_xy) fail(WFP2D_ERR_ARG, "NULL pointer argument");
        if (M <= 0 || Nx <= 0 || M > 2000000000LL || Nx > 2000000000LL) fail(WFP2D_ERR_ARG, "M and Nx must be in [1, 2e9]");
        if (!(dt > 0.0) || !std::isfinite(dt)) fail(WFP2D_ERR_ARG, "dt must be positive and finite");
        if (window_W < 2 || window_W > 4096) fail(WFP2D_ERR_ARG, "W must be in [2, 4096]");
        if (!(tol > 1e-15 && tol < 1e-2)) fail(WFP2D_ERR_ARG, "tol must be in (1e-15, 1e-2)");
        wfp2d_opts o;
        wfp2d_default_opts(&o);
        if (opts) o = *opts;
        if (o.precision != WFP2D_PREC_FP64 && o.precision != WFP2D_PREC_MIXED) fail(WFP2D_ERR_ARG, "unknown precision");
        if (o.interp_order < 2 || o.interp_order > 32) fail(WFP2D_ERR_ARG, "interp_order must be in [2, 32]");
        if (o.spread_tile < 0 || o.spread_tile > 6) fail(WFP2D_ERR_ARG, "spread_tile must be in [0, 6]");
        if (o.local_pairs != 0 && o.local_pairs != -1) fail(WFP2D_ERR_ARG, "local_pairs must be 0 (auto) or -1 (never)");
        if ((o.host_pointers != 0 && o.host_pointers != 1) || (o.check_finite != 0 && o.check_finite != 1))
            fail(WFP2D_ERR_ARG, "host_pointers and check_finite must be 0 or 1");
        if (!(o.nufft_tol == 0.0 || (o.nufft_tol >= 1e-15 && o.nufft_tol < 1e-2)))
            fail(WFP2D_ERR_ARG, "nufft_tol must be 0 or in [1e-15, 1e-2) (kernel widths up to 16)");
        if (!(o.Delta > 0.0) || !(o.Kf > 0.0) || !(o.b_Delta > 0.0) || o.a < 0.0) fail(WFP2D_ERR_ARG, "bad Delta, Kf, b_Delta or a");
        for (int64_t i = 0; i < M; ++i)
            if (!(std::fabs(src_xy[2 * i]) <= 1.0 && std::fabs(src_xy[2 * i + 1]) <= 1.0))
                fail(WFP2D_ERR_DOMAIN, "source " + std::to_string(i) + " outside [-1,1]^2");
        for (int64_t i = 0; i < Nx; ++i)
            if (!(std::fabs(tgt_xy[2 * i]) <= 1.0 && std::fabs(tgt_xy[2 * i + 1]) <= 1.0))
                fail(WFP2D_ERR_DOMAIN, "target " + std::to_string(i) + " outside [-1,1]^2");
        if (!(M_PI - 2.0 * std::log(1.0 / tol) / window_W > 0.0))
            fail(WFP2D_ERR_INFEASIBLE, "pi - 2b/W <= 0: no time step satisfies eq. dt for this W and tol");
        if (o.max_steps > 0 && (double)o.max_steps * dt > 3.0e4)
            fail(WFP2D_ERR_INFEASIBLE, "max_steps*dt beyond the sum-of-exponentials validity range (T <~ 3e4)");
        h = new wfp2d_plan_s();
        Plan &p = h->p;
        p.M = M;
        p.Nx = Nx;
        p.dt = dt;
        p.tol = tol;
        p.W = window_W;
        p.p = o.interp_order;
        p.lookahead = o.lookahead;
        p.precision = o.precision;
        p.Delta = o.Delta;
        p.a = o.a;
        p.Kf = o.Kf;
        p.b_Delta = o.b_Delta;
        p.nufft_tol = o.nufft_tol;
        p.device = o.device;
        p.stream = (hipStream_t)o.stream;
        p.spread_tile = o.spread_tile ? o.spread_tile : 6;
        p.opts = o;
        p.h_src_xy.assign(src_xy, src_xy + 2 * M);
        p.h_tgt_xy.assign(tgt_xy, tgt_xy + 2 * Nx);
        build(p, src_xy, tgt_xy);
        *out = h;
        return WFP2D_OK;
    } catch (const Failure &f) {
        g_init_error = f.msg;
        delete h;
        return f.code;
    } catch (const std::bad_alloc &) {
        g_init_error = "host allocation failed";
        delete h;
        return WFP2D_ERR_NOMEM;
    } catch (const std::exception &e) {
        g_init_error = e.what();
        delete h;
        return WFP2D_ERR_DEVICE;
    }
}

wfp2d_status wfp2d_step(wfp2d_plan plan, const double *sigma)
{
    if (!plan) return WFP2D_ERR_STATE;
    WFP2D_GUARD(plan, {
        if (!sigma) fail(WFP2D_ERR_ARG, "NULL sigma");
        do_step(plan->p, sigma);
    });
    return WFP2D_OK;
}

wfp2d_status wfp2d_evaluate(wfp2d_plan plan, double *u)
{
    if (!plan) return WFP2D_ERR_STATE;
    wfp2d_status st = WFP2D_OK;
    WFP2D_GUARD(plan, {
        if (!u) fail(WFP2D_ERR_ARG, "NULL u");
        Plan &p = plan->p;
        hip_check(hipSetDevice(p.device), "hipSetDevice");
        st = evaluate_into(p, u, [&](double *dst) { enqueue_evaluate(p, dst); });
        if (st == WFP2D_ERR_NONFINITE) p.err = "non-finite samples were ingested (taken as 0)";
    });
    return st;
}

wfp2d_status wfp2d_evaluate_noalloc(wfp2d_plan plan, double *u)
{
    if (!plan) return WFP2D_ERR_STATE;
    wfp2d_status st = WFP2D_OK;
    WFP2D_GUARD(plan, {
        Plan &p = plan->p;
        if (!u) fail(WFP2D_ERR_ARG, "NULL u");
        if (p.timing) fail(WFP2D_ERR_STATE, "stage timing is enabled");
        if (!p.scratch) fail(WFP2D_ERR_STATE, "no fixed workspace address for this device");
        // the evaluation's transient buffers, carved from the fixed workspace on 256-byte boundaries
        auto up = [](size_t b) { return (b + 255) / 256 * 256; };
        const size_t t2 = up((size_t)(p.g.R + 1) * p.g.Lpad * 2 * p.sizeof_real);
        const size_t cg = up((size_t)p.g.Lpad * p.g.Lpad * p.sizeof_real);
        const size_t uv = up((size_t)p.Nx * sizeof(double));
        const size_t need = 2 * t2 + cg + 2 * uv;
        if (need > kScratchBytes)
            fail(WFP2D_ERR_ARG, "evaluation workspace of " + std::to_string(need) + " bytes exceeds the fixed " +
                                    std::to_string(kScratchBytes) + "-byte workspace (use wfp2d_evaluate)");
        hip_check(hipSetDevice(p.device), "hipSetDevice");
        if (p.opts.host_pointers && !p.d_u_out) fail(WFP2D_ERR_STATE, "no field staging");
        char *base = (char *)p.scratch;
        void *own[5] = {p.d_T2, p.d_T2t, p.d_cgrid, p.d_uh, p.d_ul};
        p.d_T2 = base;
        p.d_T2t = base + t2;
        p.d_cgrid = base + 2 * t2;
        p.d_uh = (double *)(base + 2 * t2 + cg);
        p.d_ul = (double *)(base + 2 * t2 + cg + uv);
        try {
            // each buffer is written in full before it is read (u_l by a fill kernel)
            st = evaluate_into(p, u, [&](double *dst) { enqueue_evaluate(p, dst); });
        } catch (...) {
            p.d_T2 = own[0], p.d_T2t = own[1], p.d_cgrid = own[2], p.d_uh = (double *)own[3], p.d_ul = (double *)own[4];
            throw;
        }
        p.d_T2 = own[0], p.d_T2t = own[1], p.d_cgrid = own[2], p.d_uh = (double *)own[3], p.d_ul = (double *)own[4];
        if (st == WFP2D_ERR_NONFINITE) p.err = "non-finite samples were ingested (taken as 0)";
    });
    return st;
}

wfp2d_status wfp2d_evaluate_dot(wfp2d_plan plan, const double *weights, double *acc)
{
    if (!plan) return WFP2D_ERR_STATE;
    WFP2D_GUARD(plan, {
        if (!weights || !acc) fail(WFP2D_ERR_ARG, "NULL weights or acc");
        Plan &p = plan->p;
        hip_check(hipSetDevice(p.device), "hipSetDevice");
        enqueue_evaluate(p, nullptr, weights, acc);
        if (nonfinite_news(p)) {
            p.err = "non-finite samples were ingested (taken as 0)";
            return WFP2D_ERR_NONFINITE;
        }
    });
    return WFP2D_OK;
}

wfp2d_status wfp2d_adjoint_init(wfp2d_plan *out, wfp2d_plan forward)
{
    if (out) *out = nullptr;
    if (!out) return WFP2D_ERR_ARG;
    if (!forward) return WFP2D_ERR_STATE;
    const Plan &f = forward->p;
    wfp2d_opts o = f.opts;
    o.spread_tile = 0;
    o.host_pointers = 0;   // the transposed plan is driven with device buffers
    return wfp2d_init(out, f.Nx, f.h_tgt_xy.data(), f.M, f.h_src_xy.data(), f.dt, f.W, f.tol, &o);
}

// State blob: a header, then the evolving device buffers back to back, each
// starting on a 256-byte boundary.
namespace {
struct StateHeader {
    uint64_t magic, version, steps, M, Nx, n_modes, n_bufs, bytes;
};
constexpr uint64_t kStateMagic = 0x7766703264737461ull;   // "wfp2dsta"
}  // namespace

// The buffers a checkpoint holds: all of the evolving state, or (spectral) all but the sigma
// history ring, which the caller then refills with wfp2d_put_sigma.
static std::vector<std::pair<void *, size_t>> state_buffers(const Plan &p, bool spectral)
{
    std::vector<std::pair<void *, size_t>> v;
    for (const auto &b : p.state_bufs)
        if (!(spectral && b.first == (void *)p.d_sig)) v.push_back(b);
    return v;
}

static size_t state_layout(const Plan &p, std::vector<size_t> *offs, bool spectral = false)
{
    size_t off = 256;
    for (const auto &b : state_buffers(p, spectral)) {
        if (offs) offs->push_back(off);
        off += (b.second + 255) / 256 * 256;
    }
    return off;
}

static StateHeader state_header(const Plan &p, bool spectral = false)
{
    StateHeader h{};
    h.magic = kStateMagic;
    h.version = spectral ? 2 : 1;
    h.steps = (uint64_t)p.steps;
    h.M = (uint64_t)p.M;
    h.Nx = (uint64_t)p.Nx;
    h.n_modes = (uint64_t)p.n_modes;
    h.n_bufs = state_buffers(p, spectral).size();
    h.bytes = state_layout(p, nullptr, spectral);
    return h;
}

static void save_state(Plan &p, void *dst, int64_t bytes, bool spectral)
{
    std::vector<size_t> offs;
    const size_t need = state_layout(p, &offs, spectral);
    if (!dst || bytes < (int64_t)need) fail(WFP2D_ERR_ARG, "state buffer NULL or smaller than the state's size");
    hip_check(hipSetDevice(p.device), "hipSetDevice");
    const StateHeader h = state_header(p, spectral);
    hip_check(hipMemcpyAsync(dst, &h, sizeof h, hipMemcpyHostToDevice, p.stream), "state header");
    const auto bufs = state_buffers(p, spectral);
    for (size_t k = 0; k < bufs.size(); ++k)
        hip_check(hipMemcpyAsync((char *)dst + offs[k], bufs[k].first, bufs[k].second, hipMemcpyDeviceToDevice, p.stream),
                  "state copy");
    hip_check(p.stream ? hipStreamSynchronize(p.stream) : hipDeviceSynchronize(), "synchronize");
}

static void load_state(Plan &p, const void *src, int64_t bytes, bool spectral)
{
    std::vector<size_t> offs;
    const size_t need = state_layout(p, &offs, spectral);
    if (!src || bytes < (int64_t)need) fail(WFP2D_ERR_ARG, "state buffer NULL or smaller than the state's size");
    hip_check(hipSetDevice(p.device), "hipSetDevice");
    hip_check(p.stream ? hipStreamSynchronize(p.stream) : hipDeviceSynchronize(), "synchronize");
    StateHeader h{};
    hip_check(hipMemcpy(&h, src, sizeof h, hipMemcpyDeviceToHost), "state header");
    const StateHeader mine = state_header(p, spectral);
    if (h.magic != kStateMagic || h.version != mine.version || h.M != mine.M || h.Nx != mine.Nx ||
        h.n_modes != mine.n_modes || h.n_bufs != mine.n_bufs || h.bytes != mine.bytes)
        fail(WFP2D_ERR_ARG, "state blob does not belong to a plan of this geometry and kind");
    const auto bufs = state_buffers(p, spectral);
    for (size_t k = 0; k < bufs.size(); ++k)
        hip_check(hipMemcpyAsync(bufs[k].first, (const char *)src + offs[k], bufs[k].second, hipMemcpyDeviceToDevice, p.stream),
                  "state copy");
    if (spectral)   // levels at or before step 0 are zero; the caller puts back the others
        hip_check(launch_zero_f64(p, p.d_sig, p.g.sig_depth * p.M), "sigma ring reset");
    hip_check(p.stream ? hipStreamSynchronize(p.stream) : hipDeviceSynchronize(), "synchronize");
    p.steps = (int64_t)h.steps;
}

wfp2d_status wfp2d_reset(wfp2d_plan plan)
{
    if (!plan) return WFP2D_ERR_STATE;
    WFP2D_GUARD(plan, {
        Plan &p = plan->p;
        hip_check(hipSetDevice(p.device), "hipSetDevice");
        for (const auto &b : p.state_bufs)
            hip_check(launch_zero_f64(p, (double *)b.first, (int64_t)(b.second / sizeof(double))), "reset");
        hip_check(p.stream ? hipStreamSynchronize(p.stream) : hipDeviceSynchronize(), "synchronize");
        p.steps = 0;
    });
    return WFP2D_OK;
}

wfp2d_status wfp2d_state_bytes(wfp2d_plan plan, int64_t *bytes)
{
    if (!plan) return WFP2D_ERR_STATE;
    if (!bytes) return WFP2D_ERR_ARG;
    *bytes = (int64_t)state_layout(plan->p, nullptr);
    return WFP2D_OK;
}

wfp2d_status wfp2d_save_state(wfp2d_plan plan, void *dst, int64_t bytes)
{
    if (!plan) return WFP2D_ERR_STATE;
    WFP2D_GUARD(plan, { save_state(plan->p, dst, bytes, false); });
    return WFP2D_OK;
}

wfp2d_status wfp2d_load_state(wfp2d_plan plan, const void *src, int64_t bytes)
{
    if (!plan) return WFP2D_ERR_STATE;
    WFP2D_GUARD(plan, { load_state(plan->p, src, bytes, false); });
    return WFP2D_OK;
}

wfp2d_status wfp2d_spectral_state_bytes(wfp2d_plan plan, int64_t *bytes)
{
    if (!plan) return WFP2D_ERR_STATE;
    if (!bytes) return WFP2D_ERR_ARG;
    *bytes = (int64_t)state_layout(plan->p, nullptr, true);
    return WFP2D_OK;
}

wfp2d_status wfp2d_save_spectral_state(wfp2d_plan plan, void *dst, int64_t bytes)
{
    if (!plan) return WFP2D_ERR_STATE;
    WFP2D_GUARD(plan, { save_state(plan->p, dst, bytes, true); });
    return WFP2D_OK;
}

wfp2d_status wfp2d_load_spectral_state(wfp2d_plan plan, const void *src, int64_t bytes)
{
    if (!plan) return WFP2D_ERR_STATE;
    WFP2D_GUARD(plan, { load_state(plan->p, src, bytes, true); });
    return WFP2D_OK;
}

wfp2d_status wfp2d_put_sigma(wfp2d_plan plan, int64_t n, const double *sigma)
{
    if (!plan) return WFP2D_ERR_STATE;
    WFP2D_GUARD(plan, {
        Plan &p = plan->p;
        if (!sigma) fail(WFP2D_ERR_ARG, "NULL sigma");
        if (n < 1 || n > p.steps || n <= p.steps - p.g.sig_depth)
            fail(WFP2D_ERR_ARG, "step outside the sigma ring's reach (steps - depth < n <= steps, n >= 1)");
        hip_check(hipSetDevice(p.device), "hipSetDevice");
        hip_check(launch_ingest_at(p, stage_sigma(p, sigma), n), "put sigma");
    });
    return WFP2D_OK;
}

wfp2d_status wfp2d_query(wfp2d_plan plan, wfp2d_info *info)
{
    if (!plan || !info) return WFP2D_ERR_ARG;
    Plan &p = plan->p;
    bool nonfinite = false;
    if (p.d_nonfinite) {
        WFP2D_GUARD(plan, {
            hip_check(hipSetDevice(p.device), "hipSetDevice");
            hip_check(p.stream ? hipStreamSynchronize(p.stream) : hipDeviceSynchronize(), "synchronize");
            hip_check(hipMemcpy(p.h_nonfinite, p.d_nonfinite, sizeof(unsigned long long), hipMemcpyDeviceToHost),
                      "non-finite count copy");
            nonfinite = nonfinite_news(p);
        });
    }
    std::memset(info, 0, sizeof *info);
    info->dt = p.dt;
    info->delta = p.delta;
    info->b = p.b;
    info->A = p.A;
    info->Aplus = p.Aplus;
    info->a = p.a;
    info->dk = p.dk;
    info->K = p.K;
    info->Kf = p.Kf;
    info->Kmax = p.Kmax;
    info->LA = p.LA;
    info->R = p.g.R;
    info->n_modes = p.n_modes;
    info->n_near = p.n_near;
    info->n_far = p.n_far;
    info->n_far_classes = p.n_classes;
    info->nf = p.g.nf;
    info->band = p.g.Lpad;
    info->fft_q = p.g.Q;
    info->fft_p = p.g.P;
    info->nufft_w = p.g.w;
    info->W = p.W;
    info->p = p.p;
    info->lookahead = p.lookahead;
    info->n_levels = p.g.nlev;
    info->level_min = p.g.lev_min;
    info->n_subpanels = p.n_sub;
    info->cheb_degree = p.local_pairs ? p.local_terms : kChebDeg;
    info->M = p.M;
    info->Nx = p.Nx;
    info->n_local_pairs = p.n_local_pairs;
    info->sigma_depth = p.g.sig_depth;
    info->bytes_device = p.bytes_device;
    info->steps_ingested = p.steps;
    info->step_reported = p.steps - p.lookahead;
    info->precision = p.precision;
    info->spread_tile = p.spread_tile;
    info->local_path = p.local_pairs ? 2 : p.local_fast ? 1 : 0;
    info->local_pair_bytes = p.pair_bytes;
    info->local_pair_words = p.local_pairs ? p.pair_nword : 0;
    for (int k = 0; k < 7; ++k) info->init_ms[k] = p.init_ms[k];
    info->n_regular_subpanels = p.n_reg;
    if (nonfinite) {
        p.err = "non-finite samples were ingested (taken as 0)";
        return WFP2D_ERR_NONFINITE;
    }
    return WFP2D_OK;
}

wfp2d_status wfp2d_destroy(wfp2d_plan plan)
{
    if (!plan) return WFP2D_OK;
    delete plan;
    return WFP2D_OK;
}

const char *wfp2d_last_error(wfp2d_plan plan)
{
    if (!plan) return g_init_error.c_str();
    return plan->p.err.c_str();
}

wfp2d_status wfp2d_debug_copy(wfp2d_plan plan, int32_t what, void *dst, int64_t *bytes)
{
    if (!plan) return WFP2D_ERR_STATE;
    WFP2D_GUARD(plan, {
        Plan &p = plan->p;
        if (!dst || !bytes) fail(WFP2D_ERR_ARG, "NULL argument");
        hip_check(hipSetDevice(p.device), "hipSetDevice");
        hip_check(p.stream ? hipStreamSynchronize(p.stream) : hipDeviceSynchronize(), "synchronize");
        const int64_t m = p.steps - p.lookahead;
        auto md = [](int64_t a, int64_t b) { return ((a % b) + b) % b; };
        const int64_t csz = 2 * p.sizeof_real * p.n_modes;
        const void *src = nullptr;
        int64_t n = 0;
        std::vector<int32_t> modes;
        switch (what) {
        case 1: src = (const char *)p.d_ring_cur + md(m, p.W) * csz; n = csz; break;
        case 2: src = (const char *)p.d_ring_lag + md(m - p.LA, p.W) * csz; n = csz; break;
        case 3: src = p.d_atot; n = csz; break;
        case 4: case 5: {
            if (*bytes < 8 * p.Nx) fail(WFP2D_ERR_ARG, "destination too small");
            std::vector<double> tmp(p.Nx), outv(p.Nx);
            std::vector<int32_t> rank(p.Nx);
            hip_check(hipMemcpy(tmp.data(), what == 4 ? p.d_uh : p.d_ul, 8 * p.Nx, hipMemcpyDeviceToHost), "copy");
            hip_check(hipMemcpy(rank.data(), p.d_tgt_rank, 4 * p.Nx, hipMemcpyDeviceToHost), "copy");
            for (int64_t i = 0; i < p.Nx; ++i) outv[i] = tmp[rank[i]];
            std::memcpy(dst, outv.data(), 8 * p.Nx);
            *bytes = 8 * p.Nx;
            return WFP2D_OK;
        }
        case 7: {
            // per distinct |k| of the far modes: kappa, then its 640 Hankel coefficients (device table)
            const size_t row = 1 + kNsoe, need = (size_t)p.n_classes * row * sizeof(double);
            if ((size_t)*bytes < need) fail(WFP2D_ERR_ARG, "destination too small");
            std::vector<double> H((size_t)p.n_classes * kNsoe);
            hip_check(hipMemcpy(H.data(), p.d_H, H.size() * sizeof(double), hipMemcpyDeviceToHost), "copy");
            double *o = (double *)dst;
            for (int64_t c = 0; c < p.n_classes; ++c) {
                o[c * row] = p.h_class_kappa[c];
                std::memcpy(o + c * row + 1, &H[(size_t)c * kNsoe], kNsoe * sizeof(double));
            }
            *bytes = (int64_t)need;
            return WFP2D_OK;
        }
        case 6: {
            for (int64_t nx = 0; nx <= p.g.R; ++nx)
                for (int64_t i = 0; i < p.col_off[nx + 1] - p.col_off[nx]; ++i) {
                    modes.push_back((int32_t)nx);
                    modes.push_back((int32_t)(p.col_ny0[nx] + i));
                }
            n = 4 * (int64_t)modes.size();
            if (*bytes < n) fail(WFP2D_ERR_ARG, "destination too small");
            std::memcpy(dst, modes.data(), n);
            *bytes = n;
            return WFP2D_OK;
        }
        default: fail(WFP2D_ERR_ARG, "unknown stage");
        }
        if (*bytes < n) fail(WFP2D_ERR_ARG, "destination too small");
        hip_check(hipMemcpy(dst, src, n, hipMemcpyDeviceToHost), "copy");
        *bytes = n;
    });
    return WFP2D_OK;
}

wfp2d_status wfp2d_graph_capture(wfp2d_plan plan, const double *sigma, double *u)
{
    if (!plan) return WFP2D_ERR_STATE;
    WFP2D_GUARD(plan, {
        Plan &p = plan->p;
        if (!sigma || !u) fail(WFP2D_ERR_ARG, "NULL pointer");
        if (p.timing) fail(WFP2D_ERR_STATE, "stage timing is enabled");
        if (p.opts.host_pointers) fail(WFP2D_ERR_STATE, "a plan with host pointers cannot be captured");
        if (!p.stream) fail(WFP2D_ERR_STATE, "graph capture needs a non-default stream");
        hip_check(hipSetDevice(p.device), "hipSetDevice");
        capture_graph(p.stream, p.graph, p.graph_exec, [&] {
            enqueue_step(p, sigma);
            enqueue_evaluate(p, u);
        });
    });
    return WFP2D_OK;
}

wfp2d_status wfp2d_graph_launch(wfp2d_plan plan)
{
    if (!plan) return WFP2D_ERR_STATE;
    WFP2D_GUARD(plan, {
        Plan &p = plan->p;
        if (!p.graph_exec) fail(WFP2D_ERR_STATE, "no graph captured");
        hip_check(hipSetDevice(p.device), "hipSetDevice");
        hip_check(hipGraphLaunch(p.graph_exec, p.stream), "hipGraphLaunch");
        p.steps += 1;
    });
    return WFP2D_OK;
}

wfp2d_status wfp2d_batch_create(wfp2d_batch *out, int32_t n, const wfp2d_plan *plans, const double *const *sigma,
                                double *const *u, int32_t n_streams, void *stream)
{
    if (out) *out = nullptr;
    wfp2d_batch_s *b = nullptr;
    try {
        if (!out || n <= 0 || !plans || !sigma || !u) fail(WFP2D_ERR_ARG, "bad batch arguments");
        const int dev = plans[0] ? plans[0]->p.device : 0;
        for (int i = 0; i < n; ++i) {
            if (!plans[i] || !sigma[i] || !u[i]) fail(WFP2D_ERR_ARG, "NULL plan or pointer in batch");
            if (plans[i]->p.device != dev) fail(WFP2D_ERR_ARG, "batch plans must share a device");
            if (plans[i]->p.timing) fail(WFP2D_ERR_STATE, "stage timing is enabled on a batch plan");
            if (plans[i]->p.opts.host_pointers) fail(WFP2D_ERR_STATE, "a batch plan has host pointers");
        }
        if (!stream) fail(WFP2D_ERR_ARG, "a batch needs a non-default stream");
        b = new wfp2d_batch_s();
        b->plans.assign(plans, plans + n);
        b->stream = (hipStream_t)stream;
        hip_check(hipSetDevice(dev), "hipSetDevice");
        const int ns = std::max(1, std::min<int>(n_streams, n));
        std::vector<hipStream_t> cap(ns);
        for (int k = 0; k < ns; ++k) {
            hipStream_t s;
            hip_check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate");
            b->side.push_back(s);
            cap[k] = s;
        }
        for (int k = 0; k < 2 * ns + 1; ++k) {
            hipEvent_t e;
            hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
            b->events.push_back(e);
        }
        // plans are re-pointed at the capture streams while recording
        std::vector<hipStream_t> saved(n);
        for (int i = 0; i < n; ++i) saved[i] = plans[i]->p.stream;
        try {
            capture_graph(b->stream, b->graph, b->exec, [&] {
                hip_check(hipEventRecord(b->events[0], b->stream), "hipEventRecord");
                for (int k = 0; k < ns; ++k) hip_check(hipStreamWaitEvent(cap[k], b->events[0], 0), "hipStreamWaitEvent");
                for (int i = 0; i < n; ++i) {
                    Plan &p = plans[i]->p;
                    p.stream = cap[i % ns];
                    enqueue_step(p, sigma[i]);
                    enqueue_evaluate(p, u[i]);
                }
                for (int k = 0; k < ns; ++k) {
                    hip_check(hipEventRecord(b->events[1 + k], cap[k]), "hipEventRecord");
                    hip_check(hipStreamWaitEvent(b->stream, b->events[1 + k], 0), "hipStreamWaitEvent");
                }
            });
        } catch (...) {
            for (int i = 0; i < n; ++i) plans[i]->p.stream = saved[i];
            throw;
        }
        for (int i = 0; i < n; ++i) plans[i]->p.stream = saved[i];
        for (int i = 0; i < n; ++i) plans[i]->p.batch_refs += 1;
        *out = b;
        return WFP2D_OK;
    } catch (const Failure &f) {
        g_init_error = f.msg;
        delete b;
        return f.code;
    } catch (const std::exception &e) {
        g_init_error = e.what();
        delete b;
        return WFP2D_ERR_DEVICE;
    }
}

wfp2d_status wfp2d_batch_launch(wfp2d_batch b)
{
    if (!b || !b->exec) return WFP2D_ERR_STATE;
    try {
        hip_check(hipGraphLaunch(b->exec, b->stream), "hipGraphLaunch");
        for (wfp2d_plan pl : b->plans) pl->p.steps += 1;
        return WFP2D_OK;
    } catch (const Failure &f) {
        g_init_error = f.msg;
        return f.code;
    }
}

wfp2d_status wfp2d_batch_destroy(wfp2d_batch b)
{
    if (!b) return WFP2D_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (wfp2d_plan pl : b->plans) pl->p.batch_refs -= 1;
    delete b;
    return WFP2D_OK;
}

wfp2d_status wfp2d_set_spread_tile(wfp2d_plan plan, int32_t code)
{
    if (!plan) return WFP2D_ERR_STATE;
    WFP2D_GUARD(plan, {
        Plan &p = plan->p;
        if (p.graph_exec || p.batch_refs) fail(WFP2D_ERR_STATE, "a captured graph uses the current tile lists");
        hip_check(hipSetDevice(p.device), "hipSetDevice");
        hip_check(p.stream ? hipStreamSynchronize(p.stream) : hipDeviceSynchronize(), "synchronize");
        build_spread_tiles(p, code);
    });
    return WFP2D_OK;
}

wfp2d_status wfp2d_time_spread(wfp2d_plan plan, int32_t code, int32_t reps, double *ms)
{
    if (!plan) return WFP2D_ERR_STATE;
    WFP2D_GUARD(plan, {
        Plan &p = plan->p;
        if (!ms || reps < 1) fail(WFP2D_ERR_ARG, "bad reps or NULL ms");
        if (p.graph_exec || p.batch_refs) fail(WFP2D_ERR_STATE, "a captured graph uses the current tile lists");
        hip_check(hipSetDevice(p.device), "hipSetDevice");
        hip_check(p.stream ? hipStreamSynchronize(p.stream) : hipDeviceSynchronize(), "synchronize");
        if (code != p.spread_tile) build_spread_tiles(p, code);
        hipEvent_t e0, e1;
        hip_check(hipEventCreate(&e0), "hipEventCreate");
        hip_check(hipEventCreate(&e1), "hipEventCreate");
        hip_check(launch_spread(p), "spread");   // warm-up
        hip_check(hipEventRecord(e0, p.stream), "hipEventRecord");
        for (int r = 0; r < reps; ++r) hip_check(launch_spread(p), "spread");
        hip_check(hipEventRecord(e1, p.stream), "hipEventRecord");
        hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
        float t = 0.f;
        hip_check(hipEventElapsedTime(&t, e0, e1), "hipEventElapsedTime");
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        *ms = (double)t / reps;
    });
    return WFP2D_OK;
}

wfp2d_status wfp2d_set_timing(wfp2d_plan plan, int32_t enable)
{
    if (!plan) return WFP2D_ERR_ARG;
    WFP2D_GUARD(plan, {
        Plan &p = plan->p;
        drain_timing(p);
        for (int s = 0; s < Plan::kStages; ++s) {
            p.stage_ms[s] = 0.0;
            p.stage_n[s] = 0;
        }
        p.timing = enable != 0;
    });
    return WFP2D_OK;
}

wfp2d_status wfp2d_get_timing(wfp2d_plan plan, double *ms, int64_t *launches, int32_t n)
{
    if (!plan || !ms || n < 0) return WFP2D_ERR_ARG;
    WFP2D_GUARD(plan, {
        Plan &p = plan->p;
        drain_timing(p);
        for (int s = 0; s < n && s < Plan::kStages; ++s) {
            ms[s] = p.stage_ms[s];
            if (launches) launches[s] = p.stage_n[s];
        }
    });
    return WFP2D_OK;
}

wfp2d_status wfp2d_host_eval(int32_t what, const double *in, int64_t n_in, double *out, int64_t n_out,
                             int64_t *out_count)
{
    try {
        if (!in && n_in > 0) fail(WFP2D_ERR_ARG, "NULL input");
        if (!out) fail(WFP2D_ERR_ARG, "NULL output");
        int64_t cnt = 0;
        auto need = [&](int64_t n) {
            if (n_out < n) fail(WFP2D_ERR_ARG, "output too small");
            cnt = n;
        };
        switch (what) {
        case 1: {
            if (n_in < 8) fail(WFP2D_ERR_ARG, "need 8 inputs");
            Params P = derive_params(in[0], (int)in[1], in[2], in[5], in[6], in[7], (int)in[3], (int)in[4]);
            need(12);
            double v[12] = {P.delta, P.b, P.A, P.Aplus, P.a, P.dk, P.K, P.Kmax, (double)P.LA, (double)P.R,
                            (double)P.lookahead, (double)(2 * P.R + 1)};
            std::copy(v, v + 12, out);
            break;
        }
        case 2: {
            std::vector<double> lam, q;
            soe_nodes(lam, q);
            need(2 * kNsoe);
            std::copy(lam.begin(), lam.end(), out);
            std::copy(q.begin(), q.end(), out + kNsoe);
            break;
        }
        case 3: {
            if (n_in < 3) fail(WFP2D_ERR_ARG, "need A, Delta, b_Delta");
            std::vector<double> lam, q, H, kap(in + 3, in + n_in);
            soe_nodes(lam, q);
            hankel_table(kap, in[0], in[1], in[2], lam, q, H);
            need((int64_t)H.size());
            std::copy(H.begin(), H.end(), out);
            break;
        }
        case 4: case 5: {
            if (n_in < 5) fail(WFP2D_ERR_ARG, "need dt, W, p, lookahead, tol");
            const double dt = in[0], tol = in[4];
            const int W = (int)in[1], p = (int)in[2];
            int look = (int)in[3];
            if (look < 0) look = (p + 1) / 2 - 1;
            if (!(dt > 0) || W < 2 || p < 2 || !(tol > 0 && tol < 1)) fail(WFP2D_ERR_ARG, "bad local parameters");
            Blend phi(W * dt, std::log(1.0 / tol), 160);
            LocalWeights LW(dt, W, p, -look, phi);
            const int64_t k = n_in - 5;
            need(k * LW.nlev);
            if (what == 4) {
                for (int64_t i = 0; i < k; ++i) LW.eta(in[5 + i], out + i * LW.nlev);
            } else {
                LocalTable T = build_local_table(LW, 40, 1e-11);
                for (int64_t i = 0; i < k; ++i) local_table_eval(T, dt, W, in[5 + i], out + i * LW.nlev);
            }
            break;
        }
        case 8: {
            if (n_in < 5) fail(WFP2D_ERR_ARG, "need dt, W, p, lookahead, tol");
            const double dt = in[0], tol = in[4];
            const int W = (int)in[1], p = (int)in[2];
            int look = (int)in[3];
            if (look < 0) look = (p + 1) / 2 - 1;
            if (!(dt > 0) || W < 2 || p < 2 || !(tol > 0 && tol < 1)) fail(WFP2D_ERR_ARG, "bad local parameters");
            Blend phi(W * dt, std::log(1.0 / tol), 160);
            LocalWeights LW(dt, W, p, -look, phi);
            LocalTable T = build_local_table(LW, 40, 1e-11);
            double tail = 0.0, cmax = 0.0;
            const int terms = local_table_terms(T, tol, &tail, &cmax);
            const int64_t k = n_in - 5;
            need(3 + k * T.nlev);
            out[0] = terms;
            out[1] = tail;
            out[2] = cmax;
            for (int64_t i = 0; i < k; ++i) local_table_eval(T, dt, W, in[5 + i], out + 3 + i * T.nlev, terms);
            break;
        }
        case 10: {
            if (n_in < 6) fail(WFP2D_ERR_ARG, "need dt, W, p, lookahead, tol, terms");
            const double dt = in[0], tol = in[4];
            const int W = (int)in[1], p = (int)in[2], terms = (int)in[5];
            int look = (int)in[3];
            if (look < 0) look = (p + 1) / 2 - 1;
            if (!(dt > 0) || W < 2 || p < 2 || !(tol > 0 && tol < 1) || terms < 2 || terms > kChebDeg)
                fail(WFP2D_ERR_ARG, "bad local parameters");
            Blend phi(W * dt, std::log(1.0 / tol), 160);
            LocalWeights LW(dt, W, p, -look, phi);
            LocalTable T = build_local_table(LW, 40, 1e-11);
            const int64_t k = n_in - 6;
            need(k * T.nlev);
            for (int64_t i = 0; i < k; ++i) local_table_eval_power(T, dt, W, in[6 + i], out + i * T.nlev, terms);
            break;
        }
        case 7: {
            if (n_in < 5) fail(WFP2D_ERR_ARG, "need dt, W, p, lookahead, tol");
            const double dt = in[0], tol = in[4];
            const int W = (int)in[1], p = (int)in[2];
            int look = (int)in[3];
            if (look < 0) look = (p + 1) / 2 - 1;
            Blend phi(W * dt, std::log(1.0 / tol), 160);
            LocalWeights LW(dt, W, p, -look, phi);
            LocalTable T = build_local_table(LW, 40, 1e-11);
            need(4 + W);
            out[0] = (double)T.subs.size();
            out[1] = (double)T.dy_base;
            out[2] = (double)T.nlev;
            out[3] = T.max_err;
            for (int k = 0; k < W; ++k) out[4 + k] = (double)T.panel_l2n[k];
            break;
        }
        case 9: {
            if (n_in < 3) fail(WFP2D_ERR_ARG, "need w, beta, nf");
            const int w = (int)in[0];
            const double beta = in[1];
            const int64_t nf = (int64_t)in[2];
            if (w < 2 || w > 16 || !(beta > 0) || nf < 2 * w) fail(WFP2D_ERR_ARG, "bad spreading kernel parameters");
            int64_t R = 0;
            for (int64_t i = 3; i < n_in; ++i) R = std::max<int64_t>(R, std::llabs((int64_t)in[i]));
            if (R >= nf / 2) fail(WFP2D_ERR_ARG, "frequency index beyond nf/2");
            std::vector<double> ft;
            es_fourier(w, beta, nf, R, ft);
            need(n_in - 3);
            for (int64_t i = 3; i < n_in; ++i) out[i - 3] = ft[(int64_t)in[i] + R];
            break;
        }
        case 6: {
            if (n_in < 2) fail(WFP2D_ERR_ARG, "need width, b");
            Blend B(in[0], in[1], 160);
            const int64_t k = n_in - 2;
            need(2 * k);
            for (int64_t i = 0; i < k; ++i) {
                out[2 * i] = B.phi(in[2 + i]);
                out[2 * i + 1] = B.dphi(in[2 + i]);
            }
            break;
        }
        default: fail(WFP2D_ERR_ARG, "unknown what");
        }
        if (out_count) *out_count = cnt;
        return WFP2D_OK;
    } catch (const Failure &f) {
        g_init_error = f.msg;
        return f.code;
    } catch (const std::exception &e) {
        g_init_error = e.what();
        return WFP2D_ERR_ARG;
    }
}

}  // extern "C"
