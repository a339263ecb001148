// HIP kernels of the wfp2d per-step pipeline, written for gfx950 (wave64).
//
// Step (Sec. 4.2 and Sec. 5):   ingest sigma -> packed type-1 NUFFT of
//   sigma(t_m) + i sigma(t_{m-LA}) (spread, row FFTs, column FFTs, Hermitian
//   split into the near and lag rings) -> near-history recurrence per mode ->
//   far-history SOE recurrence per far mode.
// Evaluate (eqs. uhtraptrunc, ufhApprox, ul_GL): column and row inverse FFTs
//   of the combined coefficients -> interpolation at the targets -> local
//   singular quadrature -> u = u_h + u_l in caller order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <map>
#include <mutex>

#include "wfp2d_internal.h"

namespace wfp2d {

// ---------------------------------------------------------------------------
// complex helpers
// ---------------------------------------------------------------------------
template <class R> struct cplx;
template <> struct cplx<float> { using T = float2; };
template <> struct cplx<double> { using T = double2; };

template <class C> __device__ __forceinline__ C cmul(C a, C b) { return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
template <class C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <class C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <class C> __device__ __forceinline__ C cconj(C a) { return C{a.x, -a.y}; }
__device__ __forceinline__ double2 to_d(float2 a) { return make_double2(a.x, a.y); }
__device__ __forceinline__ double2 to_d(double2 a) { return a; }
template <class C> __device__ __forceinline__ C from_d(double2 a);
template <> __device__ __forceinline__ float2 from_d<float2>(double2 a) { return make_float2((float)a.x, (float)a.y); }
template <> __device__ __forceinline__ double2 from_d<double2>(double2 a) { return a; }

template <class R> constexpr int qmax() { return sizeof(R) == 4 ? 8192 : 4096; }

// ---------------------------------------------------------------------------
// The step counter lives in device memory so that one step is a fixed
// sequence of launches with fixed arguments (capturable in a graph):
// k_step_begin advances it; every later kernel derives the ingested step n,
// the reported step m = n - lookahead and its ring slots from it.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t pmod(int64_t a, int64_t b) { return ((a % b) + b) % b; }

__global__ void k_step_begin(int64_t *step) { step[0] += 1; }

// sigma ingest: ring slot of step n <- caller's samples gathered into sorted order.
// With a counter, a non-finite sample is stored as 0 and counted.
__global__ void k_ingest(const double *__restrict__ in, const int32_t *__restrict__ perm, double *__restrict__ sig, int64_t M,
                         const int64_t *__restrict__ step, int64_t depth, unsigned long long *__restrict__ nonfinite)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    double v = in[perm[j]];
    if (nonfinite && !isfinite(v)) {
        v = 0.0;
        atomicAdd(nonfinite, 1ull);
    }
    sig[pmod(step[0], depth) * M + j] = v;
}

// sigma(t_n) of a past step n into its ring slot (checkpoint restore), as k_ingest stores it
__global__ void k_ingest_slot(const double *__restrict__ in, const int32_t *__restrict__ perm, double *__restrict__ sig,
                              int64_t M, int64_t slot, unsigned long long *__restrict__ nonfinite)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    double v = in[perm[j]];
    if (nonfinite && !isfinite(v)) {
        v = 0.0;
        atomicAdd(nonfinite, 1ull);
    }
    sig[slot * M + j] = v;
}

// ---------------------------------------------------------------------------
// Type-1 spreading of c_j = sigma_cur[j] + i sigma_lag[j] onto the band grid.
// One wave owns one TX x TY tile of the grid and a precomputed list of the
// sources whose w x w kernel support meets the tile.  Each lane owns PPL =
// TX*TY/64 fixed grid points (column x = lane mod TX, rows y0 + i*(64/TX)) and
// keeps their sums in registers: the list is staged in LDS 64 sources at a
// time (one source per lane: sample pair, kernel origin, 2w weights), then
// every lane adds each staged source's contribution to its own points.  No
// two lanes write the same point, so there are no atomics and no LDS traffic
// on the accumulators; the tile is written once with coalesced stores.
// Consecutive workgroups go to different XCDs, so the tile order is remapped
// to give each XCD a contiguous band of tiles (neighbouring tiles share
// sources, which then stay in that XCD's L2).
// ---------------------------------------------------------------------------
template <class R, int TX, int TY>
__global__ __launch_bounds__(64) void k_spread(const double *__restrict__ sig, const int64_t *__restrict__ step,
                                               const int2 *__restrict__ base, const R *__restrict__ wts,
                                               const int32_t *__restrict__ tile_off, const int32_t *__restrict__ tile_src,
                                               typename cplx<R>::T *__restrict__ grid, int w, int ntx, int ntile,
                                               int Lpad, Geom g)
{
    using C = typename cplx<R>::T;
    constexpr int S = 64 / TX, PPL = TX * TY / 64;
    static_assert(TX * TY % 64 == 0 && 64 % TX == 0, "tile shape");
    extern __shared__ unsigned char spread_lds[];
    __shared__ R st_c[64][2];
    __shared__ int2 st_b[64];
    const int ws = 2 * w + 1;                      // staged weights per source (odd stride: no bank aliasing)
    R *st_w = (R *)spread_lds;                     // [64][ws]
    const int per_xcd = (ntile + 7) >> 3;
    const int tile = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
    if (tile >= ntile) return;
    const int64_t m = step[0] - g.lookahead;
    const double *__restrict__ sig_cur = sig + pmod(m, g.sig_depth) * g.M;
    const double *__restrict__ sig_lag = sig + pmod(m - g.LA, g.sig_depth) * g.M;
    const int ox = (tile % ntx) * TX, oy = (tile / ntx) * TY;
    const int lane = threadIdx.x;
    const int px = lane % TX, py0 = lane / TX;     // this lane's points: (px, py0 + i S), i < PPL
    R are[PPL], aim[PPL];
#pragma unroll
    for (int i = 0; i < PPL; ++i) are[i] = aim[i] = R(0);
    const int beg = tile_off[tile], end = tile_off[tile + 1];
    for (int r0 = beg; r0 < end; r0 += 64) {
        const int e = r0 + lane;
        if (e < end) {
            const int j = tile_src[e];
            st_c[lane][0] = (R)sig_cur[j];
            st_c[lane][1] = (R)sig_lag[j];
            const int2 b = base[j];
            st_b[lane] = make_int2(b.x - ox, b.y - oy);
            const R *wj = wts + (size_t)j * 2 * w;
            for (int a = 0; a < 2 * w; ++a) st_w[lane * ws + a] = wj[a];
        }
        __syncthreads();
        const int ns = min(64, end - r0);
        for (int k = 0; k < ns; ++k) {
            const int2 b = st_b[k];
            const int dx = px - b.x;
            if ((unsigned)dx < (unsigned)w) {
                const R *wk = st_w + k * ws;
                const R wx = wk[dx];
                const R cr = st_c[k][0] * wx, ci = st_c[k][1] * wx;
#pragma unroll
                for (int i = 0; i < PPL; ++i) {
                    const int dy = py0 + i * S - b.y;
                    if ((unsigned)dy < (unsigned)w) {
                        const R wy = wk[w + dy];
                        are[i] += cr * wy;
                        aim[i] += ci * wy;
                    }
                }
            }
        }
        __syncthreads();
    }
    const int gx = ox + px;
    if (gx < Lpad) {
#pragma unroll
        for (int i = 0; i < PPL; ++i) {
            const int gy = oy + py0 + i * S;
            if (gy < Lpad) grid[(size_t)gy * Lpad + gx] = C{are[i], aim[i]};
        }
    }
}

// ---------------------------------------------------------------------------
// The same type-1 input sums on the matrix cores.  The kernel is a tensor
// product, so on a 16 x 16 tile the sum over the tile's sources is a
// contraction over them:
//   G[y][x] = sum_k (c_k wy_k(y - by_k)) wx_k(x - bx_k) = (A B)[y][x],
// A[y][k] = c_k wy_k(y - by_k) and B[k][x] = wx_k(x - bx_k), both zero off the
// kernel's support.  Every four staged sources take one 16x16x4 MFMA per part
// (real part: c = S(t_m) samples, imaginary part: S(t_{m-LA})), in a fixed
// order, so the sums are deterministic.  Operand layout of the 16x16x4 MFMAs:
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; it receives
// D[4 (l / 16) + v][l % 16] (FP32) or D[l / 16 + 4 v][l % 16] (FP64), v < 4.
// The sources' weights are staged cooperatively with 16-byte loads (each
// source's 2w weights are one contiguous row).
// ---------------------------------------------------------------------------
typedef float mfma_f4 __attribute__((ext_vector_type(4)));
typedef double mfma_d4 __attribute__((ext_vector_type(4)));

template <class R> struct mfma_acc;
template <> struct mfma_acc<float> {
    using T = mfma_f4;
    static __device__ __forceinline__ T step(float a, float b, T c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <> struct mfma_acc<double> {
    using T = mfma_d4;
    static __device__ __forceinline__ T step(double a, double b, T c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

template <class R>
__global__ __launch_bounds__(64) void k_spread_mfma(const double *__restrict__ sig, const int64_t *__restrict__ step,
                                                    const int2 *__restrict__ base, const R *__restrict__ wts,
                                                    const int32_t *__restrict__ tile_off, const int32_t *__restrict__ tile_src,
                                                    typename cplx<R>::T *__restrict__ grid, int w, int ntx, int ntile,
                                                    int Lpad, Geom g)
{
    using C = typename cplx<R>::T;
    using M = mfma_acc<R>;
    extern __shared__ unsigned char spread_lds[];
    __shared__ R st_c[64][2];
    __shared__ int2 st_b[64];
    __shared__ int st_j[64];
    const int ws = 2 * w + 1;                      // staged weights per source (odd stride: no bank aliasing)
    R *st_w = (R *)spread_lds;                     // [64][ws]
    const int per_xcd = (ntile + 7) >> 3;
    const int tile = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
    if (tile >= ntile) return;
    const int64_t m = step[0] - g.lookahead;
    const double *__restrict__ sig_cur = sig + pmod(m, g.sig_depth) * g.M;
    const double *__restrict__ sig_lag = sig + pmod(m - g.LA, g.sig_depth) * g.M;
    const int ox = (tile % ntx) * 16, oy = (tile / ntx) * 16;
    const int lane = threadIdx.x, q = lane & 15, kq = lane >> 4;
    typename M::T are = {0, 0, 0, 0}, aim = {0, 0, 0, 0};
    constexpr int PER = 16 / (int)sizeof(R);       // weights per 16-byte load
    const bool vec = (2 * w) % PER == 0;
    const int nv = vec ? 2 * w / PER : 0;          // 16-byte loads per source
    const int beg = tile_off[tile], end = tile_off[tile + 1];
    for (int r0 = beg; r0 < end; r0 += 64) {
        const int ns = min(64, end - r0);
        if (lane < ns) {
            const int j = tile_src[r0 + lane];
            st_j[lane] = j;
            st_c[lane][0] = (R)sig_cur[j];
            st_c[lane][1] = (R)sig_lag[j];
            const int2 b = base[j];
            st_b[lane] = make_int2(b.x - ox, b.y - oy);
            if (!vec)
                for (int a = 0; a < 2 * w; ++a) st_w[lane * ws + a] = wts[(size_t)j * 2 * w + a];
        }
        if (vec) {
            __syncthreads();
            for (int i = lane; i < ns * nv; i += 64) {
                const int s = i / nv, a = i - s * nv;
                R vr[PER];                         // one 16-byte load (rows are 16-byte aligned), no type punning
                __builtin_memcpy(vr, __builtin_assume_aligned(wts + (size_t)st_j[s] * 2 * w + a * PER, 16), 16);
#pragma unroll
                for (int k = 0; k < PER; ++k) st_w[s * ws + a * PER + k] = vr[k];
            }
        }
        __syncthreads();
        for (int k0 = 0; k0 < ns; k0 += 4) {
            const int k = k0 + kq;
            R ar = R(0), ai = R(0), bx = R(0);
            if (k < ns) {
                const int2 b = st_b[k];
                const R *wk = st_w + k * ws;
                const int dy = q - b.y, dx = q - b.x;
                if ((unsigned)dy < (unsigned)w) {
                    const R wy = wk[w + dy];
                    ar = st_c[k][0] * wy;
                    ai = st_c[k][1] * wy;
                }
                if ((unsigned)dx < (unsigned)w) bx = wk[dx];
            }
            are = M::step(ar, bx, are);
            aim = M::step(ai, bx, aim);
        }
        __syncthreads();
    }
    const int gx = ox + q;
    if (gx < Lpad) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int gy = oy + M::row(lane, v);
            if (gy < Lpad) grid[(size_t)gy * Lpad + gx] = C{are[v], aim[v]};
        }
    }
}

// ---------------------------------------------------------------------------
// Line FFTs of length Q = 2^L (L >= 4) in one workgroup of T = Q/16 threads.
// Each thread holds 16 values; Stockham passes of radix 16 run in registers
// with one LDS exchange per pass, and a last pass of radix 2, 4 or 8 covers
// L mod 4.  sign = +1 computes X[k] = sum_m x[m] e^{+2 pi i k m/Q}, sign = -1
// the conjugate kernel.  Twiddles e^{2 pi i j/nf} (nf = P Q) come from the
// workgroup's two-level LDS table (tw_d) and their powers (twiddle_powers).
// The LDS index is padded by one element every 16 against bank conflicts.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }

// Twiddles e^{2 pi i j/nf}, j in [0, nf), from a two-level FP64 table in LDS (staged
// once per workgroup by tw_stage): tt[j & 63] * tt[64 + (j >> 6)], formed in FP64.
// Gathers from a global table go through L2 at random strides and cost about half of
// the transform time; one lookup per thread and pass, with the other twiddles its
// powers, leaves the LDS to the transform's own exchanges.
__device__ __forceinline__ double2 tw_d(const double2 *tt, int j)
{
    const double2 a = tt[64 + (j >> 6)], b = tt[j & 63];
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double2 cmul_d(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// v[r] *= w^r for r = 1 .. N-1, w = e^{sign 2 pi i j/nf}: one table entry, its powers by
// repeated multiplication in FP64 (relative error below N units of FP64 rounding), each
// rounded once to the working precision.  A Stockham pass's twiddles for one thread are
// exactly such powers, so this replaces N-1 table lookups by one.
template <int N, class C>
__device__ __forceinline__ void twiddle_powers(C *v, const double2 *tt, int j, int sign)
{
    double2 w = tw_d(tt, j);
    if (sign < 0) w.y = -w.y;
    double2 t = w;
#pragma unroll
    for (int r = 1; r < N; ++r) {
        v[r] = cmul(v[r], from_d<C>(t));
        if (r + 1 < N) t = cmul_d(t, w);
    }
}

// stage the two-level table of e^{2 pi i j/nf} (from the global FP64 table tw) into tt
__device__ __forceinline__ void tw_stage(double2 *tt, const double2 *__restrict__ tw, int nf)
{
    for (int i = threadIdx.x; i < 64 + nf / 64; i += blockDim.x) tt[i] = tw[i < 64 ? i : (i - 64) * 64];
    __syncthreads();
}

// multiply by sign*i
template <class C> __device__ __forceinline__ C mul_si(C a, int sign) { return sign > 0 ? C{-a.y, a.x} : C{a.y, -a.x}; }

template <class C> __device__ __forceinline__ void dft2(C &a, C &b)
{
    const C t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <class C> __device__ __forceinline__ void dft4(C &a, C &b, C &c, C &d, int sign)
{
    const C s02 = cadd(a, c), d02 = csub(a, c), s13 = cadd(b, d), d13 = mul_si(csub(b, d), sign);
    a = cadd(s02, s13);
    b = cadd(d02, d13);
    c = csub(s02, s13);
    d = csub(d02, d13);
}

// multiply by e^{sign 2 pi i m / 16}, m in [0, 16), with exact constants
template <class C> __device__ __forceinline__ C rot16(C a, int m, int sign)
{
    using R = decltype(a.x);
    const R c1 = R(0.92387953251128675613), s1 = R(0.38268343236508977173), h = R(0.70710678118654752440);
    R cr, ci;
    switch (m & 15) {
    case 0: return a;
    case 1: cr = c1; ci = s1; break;
    case 2: cr = h; ci = h; break;
    case 3: cr = s1; ci = c1; break;
    case 4: cr = 0; ci = 1; break;
    case 5: cr = -s1; ci = c1; break;
    case 6: cr = -h; ci = h; break;
    case 7: cr = -c1; ci = s1; break;
    case 8: cr = -1; ci = 0; break;
    case 9: cr = -c1; ci = -s1; break;
    default: cr = -h; ci = -h; break;   // m = 10 (largest used)
    }
    if (sign < 0) ci = -ci;
    return C{a.x * cr - a.y * ci, a.x * ci + a.y * cr};
}

template <class C> __device__ __forceinline__ void dft8(C *v, int sign)
{
    // even/odd split: X[k] = E[k] + w8^k O[k], X[k+4] = E[k] - w8^k O[k]
    C e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6], o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3, sign);
    dft4(o0, o1, o2, o3, sign);
    o1 = rot16(o1, 2, sign);
    o2 = rot16(o2, 4, sign);
    o3 = rot16(o3, 6, sign);
    v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
}

// dft4 of (a, b, c, d) whose inputs from the NB-th on are zero
template <int NB, class C> __device__ __forceinline__ void dft4_z(C &a, C &b, C &c, C &d, int sign)
{
    if constexpr (NB >= 4) {
        dft4(a, b, c, d, sign);
    } else if constexpr (NB == 3) {                 // d = 0
        const C s02 = cadd(a, c), d02 = csub(a, c), d13 = mul_si(b, sign);
        a = cadd(s02, b);
        c = csub(s02, b);
        b = cadd(d02, d13);
        d = csub(d02, d13);
    } else if constexpr (NB == 2) {                 // c = d = 0
        const C t = a, d13 = mul_si(b, sign);
        a = cadd(t, b);
        c = csub(t, b);
        b = cadd(t, d13);
        d = csub(t, d13);
    } else if constexpr (NB == 1) {                 // b = c = d = 0
        b = a;
        c = a;
        d = a;
    } else {
        a = b = c = d = C{0, 0};
    }
}

// nonzero inputs among v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12] when v[r] = 0 for r >= NZ
constexpr int dft16_nb(int nz, int n2) { return nz <= n2 ? 0 : ((nz - n2 + 3) / 4 > 4 ? 4 : (nz - n2 + 3) / 4); }

// DFT of 16 values in registers; v[r] for r >= NZ must be zero (a pruned first stage)
template <int NZ = 16, class C> __device__ __forceinline__ void dft16(C *v, int sign)
{
    // n = 4 n1 + n2, k = k1 + 4 k2
    dft4_z<dft16_nb(NZ, 0)>(v[0], v[4], v[8], v[12], sign);
    dft4_z<dft16_nb(NZ, 1)>(v[1], v[5], v[9], v[13], sign);
    dft4_z<dft16_nb(NZ, 2)>(v[2], v[6], v[10], v[14], sign);
    dft4_z<dft16_nb(NZ, 3)>(v[3], v[7], v[11], v[15], sign);
    // now v[4 k1 + n2] = Y[n2][k1]; twiddle by w16^{n2 k1}
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1)
#pragma unroll
        for (int n2 = 1; n2 < 4; ++n2) v[4 * k1 + n2] = rot16(v[4 * k1 + n2], n2 * k1, sign);
    C out[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        C a = v[4 * k1], b = v[4 * k1 + 1], c = v[4 * k1 + 2], d = v[4 * k1 + 3];
        dft4(a, b, c, d, sign);
        out[k1] = a;
        out[k1 + 4] = b;
        out[k1 + 8] = c;
        out[k1 + 12] = d;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = out[i];
}

// last Stockham pass of radix R in {2, 4, 8}: each thread does 16/R butterflies.
// Q and Ns = 2^lns are powers of two: index arithmetic by shifts and masks.
// LDS index of line element i: padded by one slot every 16 (against bank conflicts)
// when Q >= 256, unpadded below.  Every stride the passes use is then either a multiple
// of 16 (padded case) or unpadded, so the index of a + r S is idx(a) + r S' with
// S' = S + S/16 (padded) or S: a base plus uniform multiples, no per-element arithmetic.
__device__ __forceinline__ int fidx(int i, bool pad) { return pad ? lpad(i) : i; }
__device__ __forceinline__ int fstr(int s, bool pad) { return pad ? s + (s >> 4) : s; }

// last Stockham pass of radix R in {2, 4, 8}: each thread does 16/R butterflies.
// Q and Ns = 2^lns are powers of two: index arithmetic by shifts and masks.
template <int R, class C>
__device__ __forceinline__ void tail_pass(C *lds, C *v, int Q, int lns, int sign, const double2 *tw, int P, bool pad)
{
    constexpr int nb = 16 / R, lR = R == 2 ? 1 : R == 4 ? 2 : 3;
    const int tid = threadIdx.x, T = Q >> 4, QR = Q >> lR, Ns = 1 << lns;
    const int rb = fidx(tid, pad), Tp = fstr(T, pad), QRp = fstr(QR, pad), Nsp = fstr(Ns, pad);
#pragma unroll
    for (int i = 0; i < nb; ++i)
#pragma unroll
        for (int r = 0; r < R; ++r) v[i * R + r] = lds[rb + i * Tp + r * QRp];
    __syncthreads();
    const int stride = (Q >> (lR + lns)) * P;
#pragma unroll
    for (int i = 0; i < nb; ++i) {
        const int j = tid + T * i, k = j & (Ns - 1);
        twiddle_powers<R>(v + i * R, tw, k * stride, sign);
        if (R == 2) dft2(v[i * R], v[i * R + 1]);
        else if (R == 4) dft4(v[i * R], v[i * R + 1], v[i * R + 2], v[i * R + 3], sign);
        else dft8(v + i * R, sign);
        const int ob = fidx(((j >> lns) << (lns + lR)) + k, pad);
#pragma unroll
        for (int r = 0; r < R; ++r) lds[ob + r * Nsp] = v[i * R + r];
    }
    __syncthreads();
}

// One workgroup transforms one line.  v[r] (r < 16) holds x[tid + r Q/16] on
// entry, zero for r >= NZ; the result is left in lds (natural order, index fidx).
template <int NZ = 16, class C>
__device__ void fft_line(C *lds, C *v, int Q, int L, int sign, const double2 *tw, int P)
{
    const bool pad = Q >= 256;
    const int tid = threadIdx.x, T = Q >> 4, Tp = fstr(T, pad), rb = fidx(tid, pad);
    // first radix-16 pass (Ns = 1): no twiddles; idx(16 tid + r) = idx(16 tid) + r
    dft16<NZ>(v, sign);
    const int b1 = pad ? tid * 17 : tid * 16;
#pragma unroll
    for (int r = 0; r < 16; ++r) lds[b1 + r] = v[r];
    __syncthreads();
    int lns = 4, Lleft = L - 4;                     // Ns = 2^lns
    while (Lleft >= 4) {
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = lds[rb + r * Tp];
        __syncthreads();
        const int Ns = 1 << lns, k = tid & (Ns - 1), stride = (Q >> (4 + lns)) * P, Nsp = fstr(Ns, pad);
        twiddle_powers<16>(v, tw, k * stride, sign);
        dft16(v, sign);
        const int ob = fidx(((tid >> lns) << (lns + 4)) + k, pad);
#pragma unroll
        for (int r = 0; r < 16; ++r) lds[ob + r * Nsp] = v[r];
        __syncthreads();
        lns += 4;
        Lleft -= 4;
    }
    if (Lleft == 1) tail_pass<2>(lds, v, Q, lns, sign, tw, P, pad);
    else if (Lleft == 2) tail_pass<4>(lds, v, Q, lns, sign, tw, P, pad);
    else if (Lleft == 3) tail_pass<8>(lds, v, Q, lns, sign, tw, P, pad);
}

// map sub-transform output k' of branch s to a signed mode n in [-R, R]; false if unused
__device__ __forceinline__ bool out_mode(int kp, int s, const Geom &g, int &n)
{
    const int k = g.P * kp + s;
    if (k <= g.R) { n = k; return true; }
    if (k >= g.nf - g.R) { n = k - g.nf; return true; }
    return false;
}

__device__ __forceinline__ int ilog2(int q)
{
    int l = 0;
    while ((1 << l) < q) ++l;
    return l;
}

// ---------------------------------------------------------------------------
// Type-1 transform of one line (a band row, or a column after transposition):
// x[m], m < Lpad (zero beyond), -> X(n) for n in [-R, R] times corr[n+R],
// where the length-nf transform is split into P length-Q transforms of the
// twiddled line (nf = P Q).  mode 0 writes out[n + R] for every n; mode 1
// writes only the disk n_x^2 + n_y^2 <= Rd2 (n_x = line - R).
// ---------------------------------------------------------------------------
// (FP32: bounded to three waves per SIMD, two workgroups' worth of latency hiding per CU
// instead of one.)  NZ: in the FP32 form, a branch line x_s is zero from element NZ T on
// (P NZ T >= Lpad), so each thread loads NZ of its 16 values and the first radix-16 pass
// is pruned accordingly.
template <class R, int MODE, int NZ = 16>
__global__ __launch_bounds__(512, sizeof(R) == 4 ? 3 : 1) void k_fft_t1(const typename cplx<R>::T *__restrict__ in, typename cplx<R>::T *__restrict__ out,
                                                const typename cplx<R>::T *__restrict__ corr, const double2 *__restrict__ tw, Geom g)
{
    using C = typename cplx<R>::T;
    extern __shared__ char smem[];
    C *lds = reinterpret_cast<C *>(smem);
    double2 *tt = reinterpret_cast<double2 *>(smem + (size_t)lpad(g.Q) * sizeof(C));   // two-level twiddle table
    tw_stage(tt, tw, g.nf);
    const int line = blockIdx.x, tid = threadIdx.x, T = g.Q >> 4, L = ilog2(g.Q);
    const C *x = in + (size_t)line * g.Lpad;
    const int nx = line - g.R;
    C v[16];
    if constexpr (sizeof(R) == 4) {
        // Decimation in time over the P branches: x_s[m'] = x[P m' + s],
        // X(k) = sum_s e^{2 pi i k s/nf} FFT_Q(x_s)[k mod Q].  Slot k'' = k mod Q serves
        // n = k'' (if k'' <= R) and n = k'' - Q (if k'' >= Q - R); each thread accumulates
        // its slots over the branches and writes every output once, in natural order.
        // The grid keeps 2R + 1 <= P Q / 2 <= 3 Q / 2 modes (checked at plan creation), so
        // R < 12 T: slots i >= 12 (kk >= 12 T) never hold a nonnegative mode and slots i < 4
        // (kk < 4 T < Q - R) never a negative one.  acc_p[i] serves i < 12, acc_n[i - 4] i >= 4.
        C acc_p[12], acc_n[12];
#pragma unroll
        for (int i = 0; i < 12; ++i) acc_p[i] = acc_n[i] = C{0, 0};
        for (int s = 0; s < g.P; ++s) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = g.P * (tid + r * T) + s;
                v[r] = (r < NZ && m < g.Lpad) ? x[m] : C{0, 0};
            }
            fft_line<NZ>(lds, v, g.Q, L, +1, tt, g.P);
            // branch twiddles e^{2 pi i kk s/nf}, kk = tid + i T: a geometric sequence in i, formed
            // in FP64; slot kk's negative frequency kk - Q takes the extra factor e^{-2 pi i Q s/nf}
            double2 t = tw_d(tt, tid * s);
            const double2 st = tw_d(tt, T * s), cq = tw_d(tt, s == 0 ? 0 : g.nf - g.Q * s);   // 0 < s < P: nf - Q s in (0, nf)
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int kk = tid + i * T;
                const C y = lds[fidx(kk, g.Q >= 256)];
                if (i < 12 && kk <= g.R) acc_p[i] = cadd(acc_p[i], s == 0 ? y : cmul(y, from_d<C>(t)));
                if (i >= 4 && kk >= g.Q - g.R)
                    acc_n[i - 4] = cadd(acc_n[i - 4], s == 0 ? y : cmul(y, from_d<C>(cmul_d(t, cq))));
                if (i < 15) t = cmul_d(t, st);
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int kk = tid + i * T;
            if (i < 12 && kk <= g.R && !(MODE == 1 && (double)(nx * nx + kk * kk) > g.Rd2))
                out[(size_t)line * g.N + kk + g.R] = cmul(acc_p[i], corr[kk + g.R]);
            const int n2 = kk - g.Q;
            if (i >= 4 && kk >= g.Q - g.R && !(MODE == 1 && (double)(nx * nx + n2 * n2) > g.Rd2))
                out[(size_t)line * g.N + n2 + g.R] = cmul(acc_n[i - 4], corr[n2 + g.R]);
        }
    } else {
        // FP64: decimation in frequency (fewer registers), k = P k' + s per branch
        for (int s = 0; s < g.P; ++s) {
            // the line is re-read for each branch (from L2) rather than held in registers
            double2 t = tw_d(tt, tid * s);                 // e^{2 pi i s m/nf}, m = tid + r T: geometric in r
            const double2 st = tw_d(tt, T * s);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = tid + r * T;
                const C xm = m < g.Lpad ? x[m] : C{0, 0};
                v[r] = s == 0 ? xm : cmul(xm, from_d<C>(t));
                if (r < 15) t = cmul_d(t, st);
            }
            fft_line(lds, v, g.Q, L, +1, tt, g.P);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int kp = tid + i * T;
                int n;
                if (!out_mode(kp, s, g, n)) continue;
                if (MODE == 1 && (double)(nx * nx + n * n) > g.Rd2) continue;
                out[(size_t)line * g.N + n + g.R] = cmul(lds[fidx(kp, g.Q >= 256)], corr[n + g.R]);
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Type-2 transform of one line: input coefficients X(k) for k = n mod nf
// (gathered by a functor), output y[m] = sum_k X(k) e^{-2 pi i k m/nf} for
// m < Lpad, accumulated over the P branches.
//   MODE 0 (columns): X from the packed half-disk coefficients of column n_x =
//     line, times (2 or 1) conj(corr_x) conj(corr_y); output complex T2[line][m].
//   MODE 1 (rows): two rows per workgroup, lines 2b and 2b+1, with half spectra
//     H(k) = T2t[line][k], k <= R, whose real transforms are wanted: Re of the
//     transform of H is the transform of the Hermitian X(k) = (H(k) + conj H(-k))/2,
//     so one complex transform of X1 + i X2 gives row 2b in its real part and row
//     2b+1 in its imaginary part (half the transforms).
// ---------------------------------------------------------------------------
template <class R, int MODE>
__global__ __launch_bounds__(512, sizeof(R) == 4 ? 3 : 1) void k_fft_t2(const typename cplx<R>::T *__restrict__ in, void *__restrict__ outv, const int32_t *__restrict__ col_off,
                         const int32_t *__restrict__ col_ny0, const typename cplx<R>::T *__restrict__ corr,
                         const double2 *__restrict__ tw, Geom g)
{
    using C = typename cplx<R>::T;
    extern __shared__ char smem[];
    C *lds = reinterpret_cast<C *>(smem);
    double2 *tt = reinterpret_cast<double2 *>(smem + (size_t)lpad(g.Q) * sizeof(C));   // two-level twiddle table
    tw_stage(tt, tw, g.nf);
    const int line = MODE == 1 ? 2 * blockIdx.x : blockIdx.x, tid = threadIdx.x, T = g.Q >> 4, L = ilog2(g.Q);
    const bool two = MODE == 1 && line + 1 < g.Lpad;   // second row of the pair exists
    int off = 0, cnt = 0, ny0 = 0;
    C cx{1, 0};
    if (MODE == 0) {
        off = col_off[line];
        cnt = col_off[line + 1] - off;
        ny0 = col_ny0[line];
        cx = cconj(corr[line + g.R]);
    }
    C acc[16], v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = C{0, 0};
    for (int s = 0; s < g.P; ++s) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int kp = tid + r * T;
            C val{0, 0};
            if (MODE == 0) {
                int ny;
                if (out_mode(kp, s, g, ny) && ny >= ny0 && ny < ny0 + cnt) {
                    const R fac = (line > 0 || ny > 0) ? R(2) : R(1);
                    val = cmul(cmul(in[off + (ny - ny0)], cx), cconj(corr[ny + g.R]));
                    val.x *= fac;
                    val.y *= fac;
                }
            } else {
                const int k = g.P * kp + s;
                const C *h1r = in + (size_t)line * (g.R + 1), *h2r = h1r + (g.R + 1);
                if (k <= g.R) {                                   // (H1 + i H2)/2; k = 0: Re H1 + i Re H2
                    const C h1 = h1r[k], h2 = two ? h2r[k] : C{0, 0};
                    val = k == 0 ? C{h1.x, h2.x} : C{R(0.5) * (h1.x - h2.y), R(0.5) * (h1.y + h2.x)};
                } else if (k >= g.nf - g.R) {                     // (conj H1 + i conj H2)/2 at -k
                    const int kk = g.nf - k;
                    const C h1 = h1r[kk], h2 = two ? h2r[kk] : C{0, 0};
                    val = C{R(0.5) * (h1.x + h2.y), R(0.5) * (h2.x - h1.y)};
                }
            }
            v[r] = val;
        }
        fft_line(lds, v, g.Q, L, -1, tt, g.P);
        double2 t = tw_d(tt, tid * s);                     // e^{2 pi i s m/nf}, m = tid + i T: geometric in i
        const double2 st = tw_d(tt, T * s);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int m = tid + i * T;
            if (m < g.Lpad) {
                C r2 = lds[fidx(m, g.Q >= 256)];
                if (s > 0) r2 = cmul(r2, cconj(from_d<C>(t)));
                acc[i] = cadd(acc[i], r2);
            }
            if (i < 15) t = cmul_d(t, st);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int m = tid + i * T;
        if (m >= g.Lpad) continue;
        if (MODE == 0) {
            reinterpret_cast<C *>(outv)[(size_t)line * g.Lpad + m] = acc[i];
        } else {
            reinterpret_cast<R *>(outv)[(size_t)line * g.Lpad + m] = acc[i].x;
            if (two) reinterpret_cast<R *>(outv)[(size_t)(line + 1) * g.Lpad + m] = acc[i].y;
        }
    }
}

// ---------------------------------------------------------------------------
// Tiled transpose out[c][r] = in[r][c] of a rows x cols complex matrix.
// ---------------------------------------------------------------------------
template <class C>
__global__ __launch_bounds__(256) void k_transpose(const C *__restrict__ in, C *__restrict__ out, int rows, int cols)
{
    __shared__ C tile[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
    for (int j = 0; j < 32; j += 8) {
        const int r = by + ty + j, c = bx + tx;
        if (r < rows && c < cols) tile[ty + j][tx] = in[(size_t)r * cols + c];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 32; j += 8) {
        const int c = bx + ty + j, r = by + tx;
        if (r < rows && c < cols) out[(size_t)c * rows + r] = tile[tx][ty + j];
    }
}

// Hermitian split of the packed transform: F = S(t_m) + i S(t_{m-LA}).
template <class R>
__global__ __launch_bounds__(256) void k_split(const typename cplx<R>::T *__restrict__ F, const ModeChunk *__restrict__ chunks,
                                               typename cplx<R>::T *__restrict__ ring_cur, typename cplx<R>::T *__restrict__ ring_lag,
                                               int64_t H, const int64_t *__restrict__ step, Geom g)
{
    using C = typename cplx<R>::T;
    const int64_t m = step[0] - g.lookahead;
    C *__restrict__ cur = ring_cur + pmod(m, g.W) * H;
    C *__restrict__ lag = ring_lag + pmod(m - g.LA, g.W) * H;
    const ModeChunk c = chunks[blockIdx.x];
    const int t = threadIdx.x;
    if (t >= c.cnt) return;
    const int nx = c.nx, ny = c.ny0 + t;
    const C a = F[(size_t)(nx + g.R) * g.N + ny + g.R];
    const C b = F[(size_t)(-nx + g.R) * g.N + (-ny + g.R)];
    const R h = R(0.5);
    cur[c.off + t] = C{h * (a.x + b.x), h * (a.y - b.y)};
    // (a - conj b) / (2i)
    lag[c.off + t] = C{h * (a.y + b.y), -h * (a.x - b.x)};
}

// ---------------------------------------------------------------------------
// Near history (Sec. 4.2).  With the trapezoid rule on the time grid,
//   alpha(k, t_m) = dt sum_l sin(k l dt)/k w_l S(t_{m-l}),
//   w_l = phi(l dt) phi(A+ - l dt)   (eq. alphak),
// split into the blending edges (W-tap FIRs at delays 1..W-1 and
// LA+1..LA+W-1) and the interior l in [W, LA] where w_l = 1.  The interior sum
//   D_m = sum_{l=W}^{LA} sin(k l dt)/k S_{m-l},  C_m = sum cos(k l dt) S_{m-l}
// obeys the exact two-term rotation of eq. alphakEvolution, forced by the
// sample entering at delay W-1 and the one leaving at delay LA.  State and
// coefficients are FP64; ring taps are the plan's precision.
// ---------------------------------------------------------------------------
template <class R>
__global__ __launch_bounds__(256) void k_near(const ModeChunk *__restrict__ chunks, const typename cplx<R>::T *__restrict__ cur,
                                              const typename cplx<R>::T *__restrict__ lag, double2 *__restrict__ Dst,
                                              double2 *__restrict__ Cst, const double *__restrict__ phi_in,
                                              typename cplx<R>::T *__restrict__ atot, int64_t H, const int64_t *__restrict__ step, Geom g)
{
    using C = typename cplx<R>::T;
    const int64_t m = step[0] - g.lookahead;
    const ModeChunk c = chunks[blockIdx.x];
    const int t = threadIdx.x;
    if (t >= c.cnt) return;
    const int64_t pk = c.off + t;
    const int nx = c.nx, ny = c.ny0 + t;
    const double key = (double)(nx * nx + ny * ny);
    if (key * g.dk * g.dk > g.K * g.K) {  // far-only mode beyond the near cutoff
        atot[pk] = C{0, 0};
        return;
    }
    const double kap = g.dk * sqrt(key);
    const int W = g.W, LA = g.LA;
    double s1, c1;
    sincos(kap * g.dt, &s1, &c1);
    const double2 E = make_double2(c1, s1);
    const double inv = kap > 0.0 ? 1.0 / kap : 0.0;
    double sL, cL;
    sincos(kap * ((double)LA * g.dt), &sL, &cL);
    double2 D = Dst[pk], Cs = Cst[pk];
    double2 al = D;
    double2 Pw = E;                                  // e^{i kappa j dt}
    double fs = 0.0, fc = 1.0;
    double2 Sin = make_double2(0.0, 0.0);
    // ring slots of S_{m-j} (near ring) and S_{m-LA-j} (lag ring), wrapped incrementally
    const int b0 = (int)(((m % W) + W) % W), bL = (int)((((m - LA) % W) + W) % W);
    int s_cur = b0, s_lag = bL;
    // one rotation chain serves both edge FIRs:
    // sin(kappa (LA + j) dt) = sin(kappa LA dt) cos(kappa j dt) + cos(kappa LA dt) sin(kappa j dt)
    for (int j = 1; j < W; ++j) {
        s_cur = s_cur == 0 ? W - 1 : s_cur - 1;
        s_lag = s_lag == 0 ? W - 1 : s_lag - 1;
        const double2 S = to_d(cur[(int64_t)s_cur * H + pk]);
        const double2 T = to_d(lag[(int64_t)s_lag * H + pk]);
        const double sk = kap > 0.0 ? Pw.y * inv : j * g.dt;
        const double sLk = kap > 0.0 ? (sL * Pw.x + cL * Pw.y) * inv : (LA + j) * g.dt;
        const double cf = sk * phi_in[j], cg = sLk * phi_in[W - j];
        al.x += cf * S.x + cg * T.x;
        al.y += cf * S.y + cg * T.y;
        if (j == W - 1) {
            fs = sk;
            fc = Pw.x;
            Sin = S;
        }
        Pw = cmul(Pw, E);
    }
    const double2 SLA = to_d(lag[(int64_t)bL * H + pk]);
    const double scale = g.dt * (g.dk / (2.0 * M_PI)) * (g.dk / (2.0 * M_PI));
    atot[pk] = from_d<C>(make_double2(al.x * scale, al.y * scale));
    // advance the interior sums by one step
    const double gs = kap > 0.0 ? sL * inv : LA * g.dt, gc = cL;
    const double2 Dt = make_double2(D.x + fs * Sin.x - gs * SLA.x, D.y + fs * Sin.y - gs * SLA.y);
    const double2 Ct = make_double2(Cs.x + fc * Sin.x - gc * SLA.x, Cs.y + fc * Sin.y - gc * SLA.y);
    const double so = kap > 0.0 ? s1 * inv : g.dt;
    const double ks = kap * s1;
    Dst[pk] = make_double2(c1 * Dt.x + so * Ct.x, c1 * Dt.y + so * Ct.y);
    Cst[pk] = make_double2(c1 * Ct.x - ks * Dt.x, c1 * Ct.y - ks * Dt.y);
}

// ---------------------------------------------------------------------------
// Far history (Sec. 5): alpha_F = sum_l H_l(kappa) beta_l with, by the
// trapezoid rule on the time grid (scaled by e^{A lambda}, eq. beta0),
//   beta_l(t_m) = B_l(t_m) + sum_{i<W-1} (window taps),
//   B_l(t_{m+1}) = e^{-lambda_l dt} [B_l(t_m) + dt e^{-lambda_l((LA+W-1)dt - A)} S_{m-LA-W+1}],
// the one-term recurrence of eq. betaEvolution.  The window taps are folded
// with H into chi.  One wavefront per far mode; FP64.
// ---------------------------------------------------------------------------
template <class R>
__global__ __launch_bounds__(256) void k_far(const int32_t *__restrict__ far_pk, const int32_t *__restrict__ far_cls,
                                             const double *__restrict__ Htab, const double *__restrict__ chi,
                                             const double *__restrict__ dec, const double *__restrict__ inj,
                                             double2 *__restrict__ B, const typename cplx<R>::T *__restrict__ lag,
                                             typename cplx<R>::T *__restrict__ atot, int64_t n_far, int64_t H,
                                             const int64_t *__restrict__ step, Geom g)
{
    using C = typename cplx<R>::T;
    const int64_t m = step[0] - g.lookahead;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t f = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (f >= n_far) return;
    const int W = g.W, LA = g.LA;
    const int64_t pk = far_pk[f];
    const int cls = far_cls[f];
    const double2 Snew = to_d(lag[(((m - LA - W + 1) % W + W) % W) * H + pk]);
    double ax = 0.0, ay = 0.0;
    double2 *Bf = B + f * kNsoe;
    const double *Hc = Htab + (size_t)cls * kNsoe;
    for (int l = lane; l < kNsoe; l += 64) {
        const double2 b = Bf[l];
        const double h = Hc[l];
        ax += h * b.x;
        ay += h * b.y;
        const double d = dec[l], in = inj[l];
        Bf[l] = make_double2(d * (b.x + in * Snew.x), d * (b.y + in * Snew.y));
    }
    for (int i = lane; i < W - 1; i += 64) {
        const int64_t slot = ((m - (LA + 1 + i)) % W + W) % W;
        const double2 S = to_d(lag[slot * H + pk]);
        const double x = chi[(size_t)cls * (W - 1) + i];
        ax += x * S.x;
        ay += x * S.y;
    }
    for (int off = 32; off > 0; off >>= 1) {
        ax += __shfl_down(ax, off, 64);
        ay += __shfl_down(ay, off, 64);
    }
    if (lane == 0) {
        const double scale = (g.dk / (2.0 * M_PI)) * (g.dk / (2.0 * M_PI));
        const double2 a0 = to_d(atot[pk]);
        atot[pk] = from_d<C>(make_double2(a0.x + scale * ax, a0.y + scale * ay));
    }
}

// ---------------------------------------------------------------------------
// Type-2 interpolation (eq. uhtraptrunc on the fine grid): u_h(x_i) = sum over
// the w x w stencil of grid(origin_i + (a, b)) * wx_i[a] * wy_i[b].
// One workgroup per kTile x kTile tile of stencil origins: it stages the tile
// and its w - 1 halo rows and columns of the grid in LDS with coalesced row
// loads (each grid value is read from memory about (1 + (w - 1)/kTile)^2 times
// in all), then each thread evaluates whole targets of the tile from LDS.  With an
// FP32 grid every staging load of a thread is issued before its first LDS store, and
// its first target's data is loaded before the staging (one memory latency per
// workgroup instead of one per staging round).
// Tiles are remapped so that each XCD (workgroups are dealt to the 8 XCDs in
// turn) takes one contiguous band of tiles, whose halos then meet in its L2.
// Accumulation in FP64.
// ---------------------------------------------------------------------------
constexpr int kInterpThreads = 128;
template <class R, int WM>   // kernel width w <= WM: the target's weights are held in registers
__global__ __launch_bounds__(kInterpThreads) void k_interp(const R *__restrict__ cgrid, const int2 *__restrict__ base,
                                                           const R *__restrict__ wts, const int32_t *__restrict__ tlist,
                                                           const int32_t *__restrict__ toff, double *__restrict__ uh, int w,
                                                           int Lpad, int ntx)
{
    extern __shared__ unsigned char interp_lds[];
    R *const tl = reinterpret_cast<R *>(interp_lds);   // [S][S + 1], S = kTile + w - 1
    const int ntile = ntx * ntx, per_xcd = (ntile + 7) >> 3;
    const int tile = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
    if (tile >= ntile) return;
    const int e0 = toff[tile], e1 = toff[tile + 1];
    if (e0 == e1) return;
    const int ox = (tile % ntx) * kTile, oy = (tile / ntx) * kTile, S = kTile + w - 1, ld = S + 1;
    if constexpr (sizeof(R) == 8) {
        // FP64 grid: the tile staged by a plain loop, targets read after it (measured faster in
        // FP64 than the prefetching form below, whose registers lower the occupancy)
        for (int q = threadIdx.x; q < S * S; q += kInterpThreads) {
            const int yy = q / S, xx = q - yy * S, gx = ox + xx, gy = oy + yy;
            tl[yy * ld + xx] = (gx < Lpad && gy < Lpad) ? cgrid[(size_t)gy * Lpad + gx] : R(0);
        }
        __syncthreads();
        for (int e = e0 + (int)threadIdx.x; e < e1; e += kInterpThreads) {
            const int2 b = base[e];
            const R *__restrict__ wi = wts + (size_t)e * 2 * w;
            double wx[WM], wy[WM];
#pragma unroll
            for (int a = 0; a < WM; ++a) {
                wx[a] = a < w ? (double)wi[a] : 0.0;
                wy[a] = a < w ? (double)wi[w + a] : 0.0;
            }
            const R *row = tl + (b.y - oy) * ld + (b.x - ox);
            double acc = 0.0;
#pragma unroll
            for (int bb = 0; bb < WM; ++bb) {
                if (bb < w) {
                    double sx = 0.0;
#pragma unroll
                    for (int a = 0; a < WM; ++a)
                        if (a < w) sx = fma(wx[a], (double)row[bb * ld + a], sx);
                    acc = fma(sx, wy[bb], acc);
                }
            }
            uh[tlist[e]] = acc;
        }
        return;
    }
    // FP32 grid: this thread's first target (origin, weights, output slot) is loaded before the
    // tile, so that its latency overlaps the staging
    int2 b = make_int2(ox, oy);
    int dst = 0;
    R wr[2 * WM];
    auto load_target = [&](int e) {
        b = base[e];                                  // origins and weights are stored in processing order
        dst = tlist[e];
        const R *__restrict__ wi = wts + (size_t)e * 2 * w;
#pragma unroll
        for (int a = 0; a < WM; ++a) {
            wr[a] = a < w ? wi[a] : R(0);
            wr[WM + a] = a < w ? wi[w + a] : R(0);
        }
    };
    int e = e0 + (int)threadIdx.x;
    if (e < e1) load_target(e);
    // the tile and its halo: every load issued before the first LDS store (fixed count)
    constexpr int SMAX = kTile + WM - 1, NIT = (SMAX * SMAX + kInterpThreads - 1) / kInterpThreads;
    R tv[NIT];
#pragma unroll
    for (int i = 0; i < NIT; ++i) {
        const int q = (int)threadIdx.x + i * kInterpThreads;
        const int yy = q / S, xx = q - yy * S, gx = ox + xx, gy = oy + yy;
        tv[i] = (q < S * S && gx < Lpad && gy < Lpad) ? cgrid[(size_t)gy * Lpad + gx] : R(0);
    }
#pragma unroll
    for (int i = 0; i < NIT; ++i) {
        const int q = (int)threadIdx.x + i * kInterpThreads;
        const int yy = q / S, xx = q - yy * S;
        if (q < S * S) tl[yy * ld + xx] = tv[i];
    }
    __syncthreads();
    for (; e < e1; e += kInterpThreads) {
        const R *row = tl + (b.y - oy) * ld + (b.x - ox);
        double acc = 0.0;
#pragma unroll
        for (int bb = 0; bb < WM; ++bb) {
            if (bb < w) {
                double sx = 0.0;
#pragma unroll
                for (int a = 0; a < WM; ++a)
                    if (a < w) sx = fma((double)wr[a], (double)row[bb * ld + a], sx);
                acc = fma(sx, (double)wr[WM + bb], acc);
            }
        }
        uh[dst] = acc;
        if (e + kInterpThreads < e1) load_target(e + kInterpThreads);
    }
}

// ---------------------------------------------------------------------------
// Local part (Sec. 6, eq. ul_GL with eq. sigInterp):
//   u_l(x_i, t_m) = (1/2pi) sum_{j: 0 < r_ij < delta} f_j(r_ij),
//   f_j(r) = sum_d eta_d(r) sigma_j(t_{m-d}),
// where eta_d is held as Chebyshev series on sub-panels of r.  For every
// regular sub-panel P (r >= dt/2) the kernel first synthesises, per source,
// the Chebyshev coefficients of f_j on P:  psi_{j,P,c} = sum_d C_{P,c,d} sigma_{j,d}
// (a small dense contraction), then each source-target pair costs one Clenshaw
// evaluation.  One workgroup owns one source cell (side >= delta/2); its
// targets are the 5 x 5 block of target cells around it.  Pairs with
// r < dt/2 (dyadic sub-panels, about 1e-3 of all pairs) are queued and
// evaluated level by level, one wavefront per pair.  Per-target sums are
// accumulated in LDS and added to u_l with one FP64 atomic per (target, cell).
// ---------------------------------------------------------------------------
struct LocalArgs {
    const double2 *txy, *sxy;
    const int32_t *scell_start, *tcell_start;
    const SubPanel *subs;
    const double *cheb, *creg;
    const double *cpow;   // regular panels' truncated series in the power basis (pair kernel)
    const int32_t *pbase, *pl2n;
    const double *sig;
    double *ul;
    int ncell, n_reg, dy_base, n_dy, sc;
    double delta, inv_dt;
    double two_over_ua, two_over_ua0;   // 2/sqrt(dt), 2/sqrt(dt/2): Chebyshev coordinate of a panel
};

__device__ __forceinline__ double cheb_eval(const double *c, double x)
{
    double b1 = 0.0, b2 = 0.0;
    const double tx = 2.0 * x;
#pragma unroll
    for (int k = kChebDeg - 1; k >= 1; --k) {
        const double b0 = fma(tx, b1, c[k] - b2);
        b2 = b1;
        b1 = b0;
    }
    return fma(x, b1, c[0] - b2);
}

// two independent Clenshaw recurrences of NT terms interleaved (instruction-level parallelism)
template <int NT>
__device__ __forceinline__ void cheb_eval2n(const double *c0, double x0, const double *c1, double x1, double &v0, double &v1)
{
    double a1 = 0.0, a2 = 0.0, b1 = 0.0, b2 = 0.0;
    const double t0 = 2.0 * x0, t1 = 2.0 * x1;
#pragma unroll
    for (int k = NT - 1; k >= 1; --k) {
        const double a0 = fma(t0, a1, c0[k] - a2);
        const double b0 = fma(t1, b1, c1[k] - b2);
        a2 = a1;
        a1 = a0;
        b2 = b1;
        b1 = b0;
    }
    v0 = fma(x0, a1, c0[0] - a2);
    v1 = fma(x1, b1, c1[0] - b2);
}

// two power-basis polynomials of NT (even) coefficients summed by Horner's rule, interleaved;
// coefficients read two at a time (16-byte aligned rows)
template <int NT>
__device__ __forceinline__ void horner2n(const double *c0, double x0, const double *c1, double x1, double &v0, double &v1)
{
    static_assert(NT % 2 == 0, "coefficient pairs");
    const double2 *a = reinterpret_cast<const double2 *>(c0), *b = reinterpret_cast<const double2 *>(c1);
    double2 ta = a[NT / 2 - 1], tb = b[NT / 2 - 1];
    double y0 = fma(ta.y, x0, ta.x), y1 = fma(tb.y, x1, tb.x);
#pragma unroll
    for (int j = NT / 2 - 2; j >= 0; --j) {
        ta = a[j];
        tb = b[j];
        y0 = fma(fma(y0, x0, ta.y), x0, ta.x);
        y1 = fma(fma(y1, x1, tb.y), x1, tb.x);
    }
    v0 = y0;
    v1 = y1;
}

// four power-basis polynomials of NT (even) coefficients (rows of 16-byte coefficient pairs)
// summed by Horner's rule, interleaved
template <int NT>
__device__ __forceinline__ void horner4n(const double2 *const (&r)[4], const double (&x)[4], double (&y)[4])
{
    static_assert(NT % 2 == 0, "coefficient pairs");
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double2 t = r[i][NT / 2 - 1];
        y[i] = fma(t.y, x[i], t.x);
    }
#pragma unroll
    for (int j = NT / 2 - 2; j >= 0; --j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double2 t = r[i][j];
            y[i] = fma(fma(y[i], x[i], t.y), x[i], t.x);
        }
}

__device__ __forceinline__ void cheb_eval2(const double *c0, double x0, const double *c1, double x1, double &v0, double &v1)
{
    cheb_eval2n<kChebDeg>(c0, x0, c1, x1, v0, v1);
}

__device__ __forceinline__ double sub_coord(const SubPanel &sp, double r)
{
    const double v = sp.c > 0.0 ? sqrt(fmax(0.0, sp.c - r)) : r;
    return fmin(1.0, fmax(-1.0, (2.0 * v - sp.ua - sp.ub) * sp.inv));
}

__device__ __forceinline__ int regular_sub(const LocalArgs &A, double rr, int W)
{
    const int k = min((int)rr, W - 1);
    const double lo = k == 0 ? 0.5 : (double)k, sc = k == 0 ? 2.0 : 1.0;
    const int nsp = 1 << A.pl2n[k];
    return A.pbase[k] + min((int)((rr - lo) * sc * nsp), nsp - 1);
}

__device__ __forceinline__ int dyadic_sub(const LocalArgs &A, double rr)
{
    int e;
    frexp(rr, &e);
    return A.dy_base + min(-e, A.n_dy) - 1;
}

// eta-weighted sum over levels for a pair with r < dt/2 (dyadic sub-panel)
__device__ double dyadic_direct(const LocalArgs &A, const double *sg, int nlev, double r, double rr)
{
    const int sub = dyadic_sub(A, rr);
    const double xc = sub_coord(A.subs[sub], r);
    double v = 0.0;
    for (int d = 0; d < nlev; ++d) v = fma(cheb_eval(A.cheb + ((size_t)sub * nlev + d) * kChebDeg, xc), sg[d], v);
    return v;
}

__device__ __forceinline__ int64_t sig_slot(int64_t m, int d, const Geom &g)
{
    const int64_t lvl = m - (g.lev_min + d);
    return ((lvl % g.sig_depth) + g.sig_depth) % g.sig_depth;
}

__global__ __launch_bounds__(kLocalThreads) void k_local(LocalArgs A, const int64_t *__restrict__ step, Geom g)
{
    const int64_t m = step[0] - g.lookahead;
    __shared__ double psi[kLocalPsi];          // [sc][n_reg][D]
    __shared__ double sigs[kLocalSig];         // [sc][nlev]
    __shared__ double2 spos[kLocalMaxSrc];
    __shared__ int qs[kLocalQueue], qt[kLocalQueue];
    __shared__ double qr[kLocalQueue];
    __shared__ int qn;
    __shared__ int rbeg[5], rcum[6];

    const int n = A.ncell;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwave = blockDim.x >> 6;
    const int nlev = g.nlev, nreg = A.n_reg, D = kChebDeg;
    const double d2 = A.delta * A.delta;
    // grid-stride over source cells (a dispatch is limited to 2^32 work-items)
    for (int cell = blockIdx.x; cell < n * n; cell += gridDim.x) {
    const int cx = cell % n, cy = cell / n;
    const int s0 = A.scell_start[cell], s1 = A.scell_start[cell + 1];
    if (s0 == s1) continue;                     // uniform: no sources in this cell

    // the 5 x 5 block of target cells: up to 5 contiguous runs of sorted targets
    if (tid == 0) {
        int cum = 0, r = 0;
        const int xa = max(0, cx - 2), xb = min(n - 1, cx + 2);
        for (int yy = max(0, cy - 2); yy <= min(n - 1, cy + 2); ++yy, ++r) {
            const int b = A.tcell_start[yy * n + xa], e = A.tcell_start[yy * n + xb + 1];
            rbeg[r] = b;
            rcum[r] = cum;
            cum += e - b;
        }
        for (; r < 5; ++r) {
            rbeg[r] = 0;
            rcum[r] = cum;
        }
        rcum[5] = cum;
    }
    __syncthreads();
    const int NT = rcum[5];

    const int bd = blockDim.x;
    for (int tc0 = 0; tc0 < NT; tc0 += kLocalOwn * bd) {
        // each thread owns up to kLocalOwn targets of the block and accumulates in registers
        const int nown = min(kLocalOwn, (NT - tc0 + bd - 1) / bd);
        int tg[kLocalOwn];
        double2 x[kLocalOwn];
        double acc[kLocalOwn];
#pragma unroll
        for (int j = 0; j < kLocalOwn; ++j) {
            const int kk = tc0 + tid + j * bd;
            tg[j] = -1;
            x[j] = make_double2(1e30, 1e30);
            acc[j] = 0.0;
            if (j < nown && kk < NT) {
                int r = 0;
                while (r < 4 && kk >= rcum[r + 1]) ++r;
                tg[j] = rbeg[r] + (kk - rcum[r]);
                x[j] = A.txy[tg[j]];
            }
        }
        for (int sb = s0; sb < s1; sb += A.sc) {
            const int ns = min(A.sc, s1 - sb);
            for (int e = tid; e < ns * nlev; e += bd) {
                const int sidx = e / nlev, d = e - sidx * nlev;
                sigs[sidx * nlev + d] = A.sig[sig_slot(m, d, g) * g.M + sb + sidx];
            }
            if (tid < ns) spos[tid] = A.sxy[sb + tid];
            if (tid == 0) qn = 0;
            __syncthreads();
            // profile coefficients psi = C sigma on every regular sub-panel
            for (int e = tid; e < nreg * D; e += bd) {
                const double *cf = A.creg + (size_t)e * nlev;
                double pa[kLocalMaxSrc];
#pragma unroll
                for (int q = 0; q < kLocalMaxSrc; ++q) pa[q] = 0.0;
                for (int d = 0; d < nlev; ++d) {
                    const double c = cf[d];
#pragma unroll
                    for (int q = 0; q < kLocalMaxSrc; ++q)
                        if (q < ns) pa[q] = fma(c, sigs[q * nlev + d], pa[q]);
                }
                const int P = e / D, c = e - P * D;
#pragma unroll
                for (int q = 0; q < kLocalMaxSrc; ++q)
                    if (q < ns) psi[(q * nreg + P) * D + c] = pa[q];
            }
            __syncthreads();
            // pairs (owned targets) x (chunk sources), two sources at a time
#pragma unroll
            for (int j = 0; j < kLocalOwn; ++j) {
                if (j >= nown) continue;
                const double2 xj = x[j];
                for (int sidx = 0; sidx < ns; sidx += 2) {
                    const bool two = sidx + 1 < ns;
                    const int s2 = two ? sidx + 1 : sidx;
                    const double2 y0 = spos[sidx], y1 = spos[s2];
                    const double ax = xj.x - y0.x, ay = xj.y - y0.y, bx = xj.x - y1.x, by = xj.y - y1.y;
                    const double ra2 = ax * ax + ay * ay, rb2 = bx * bx + by * by;
                    bool ha = ra2 > 0.0 && ra2 < d2, hb = two && rb2 > 0.0 && rb2 < d2;
                    if (!(ha || hb)) continue;
                    const double ra = sqrt(ra2), rb = sqrt(rb2);
                    const double rra = ra * A.inv_dt, rrb = rb * A.inv_dt;
                    if ((ha && rra < 0.5) || (hb && rrb < 0.5)) {   // rare: queue, evaluated level by level
                        const bool qa = ha && rra < 0.5, qb = hb && rrb < 0.5;
                        const int q = atomicAdd(&qn, (qa ? 1 : 0) + (qb ? 1 : 0));
                        int qq = q;
                        if (qa) {
                            if (qq < kLocalQueue) { qs[qq] = sidx; qt[qq] = tg[j]; qr[qq] = ra; }
                            else acc[j] += dyadic_direct(A, sigs + sidx * nlev, nlev, ra, rra);
                            ++qq;
                            ha = false;
                        }
                        if (qb) {
                            if (qq < kLocalQueue) { qs[qq] = s2; qt[qq] = tg[j]; qr[qq] = rb; }
                            else acc[j] += dyadic_direct(A, sigs + s2 * nlev, nlev, rb, rrb);
                            hb = false;
                        }
                        if (!(ha || hb)) continue;
                    }
                    const int sa = ha ? regular_sub(A, rra, g.W) : 0;
                    const int sbb = hb ? regular_sub(A, rrb, g.W) : 0;
                    const double xa = ha ? sub_coord(A.subs[sa], ra) : 0.0;
                    const double xb = hb ? sub_coord(A.subs[sbb], rb) : 0.0;
                    double va, vb;
                    cheb_eval2(psi + (sidx * nreg + sa) * D, xa, psi + (s2 * nreg + sbb) * D, xb, va, vb);
                    acc[j] += (ha ? va : 0.0) + (hb ? vb : 0.0);
                }
            }
            __syncthreads();
            // queued pairs with r < dt/2: one wavefront per pair, lanes over levels
            const int nq = min(qn, kLocalQueue);
            for (int q = wave; q < nq; q += nwave) {
                const int sidx = qs[q];
                const double r = qr[q];
                const int sub = dyadic_sub(A, r * A.inv_dt);
                const double xc = sub_coord(A.subs[sub], r);
                double v = 0.0;
                for (int d = lane; d < nlev; d += 64)
                    v = fma(cheb_eval(A.cheb + ((size_t)sub * nlev + d) * D, xc), sigs[sidx * nlev + d], v);
                for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
                if (lane == 0) unsafeAtomicAdd(&A.ul[qt[q]], v);
            }
            __syncthreads();
        }
#pragma unroll
        for (int j = 0; j < kLocalOwn; ++j)
            if (tg[j] >= 0 && acc[j] != 0.0) unsafeAtomicAdd(&A.ul[tg[j]], acc[j]);
    }
    __syncthreads();                            // rbeg / rcum are rewritten for the next cell
    }
}

// ---------------------------------------------------------------------------
// Local part, fast form (one sub-panel per time-step panel, NL sigma levels).
// Persistent over source cells.  Thread e holds row e = (sub-panel P,
// Chebyshev index c) of the coefficient table C_{P,c,d} in registers, so the
// per-source profile coefficients psi_{j,P,c} = sum_d C_{P,c,d} sigma_{j,d} of
// a chunk of sources need only sigma from LDS.  Pairs are then found and
// evaluated in two decoupled passes per wave:
//   filter:  candidates (source, target) of the chunk x target batch, one per
//            lane, tested on r^2 alone; hits are compacted into a wave-private
//            LDS ring (ballot + prefix count);
//   evaluate: whenever 128 hits are pending, every lane takes two of them:
//            panel k = floor(r/dt), coordinate x = 2 sqrt((k+1) dt - r)/u_a - 1,
//            two interleaved Clenshaw sums of the source's profile on panel k,
//            added to per-target sums in LDS.
// So the Clenshaw work runs on full waves of true neighbours only.  Pairs with
// r < dt/2 (dyadic sub-panels) go to a workgroup queue, one wave per pair.
// Per-target sums are added to u_l with one FP64 atomic per (target, cell).
// ---------------------------------------------------------------------------
constexpr int kFastTB = 512;     // targets per batch (their positions and sums in LDS)
constexpr int kFastRing = 192;   // per-wave ring of pending hits (>= 128 + 64)

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// panel and Chebyshev coordinate of a regular pair (r >= dt/2)
__device__ __forceinline__ int fast_panel(const LocalArgs &A, double r, int W, double dt, double &x)
{
    const int k = min((int)(r * A.inv_dt), W - 1);
    x = fmin(1.0, fmax(-1.0, sqrt(fmax(0.0, (k + 1) * dt - r)) * (k ? A.two_over_ua : A.two_over_ua0) - 1.0));
    return k;
}

// psi layout in LDS: row (source q, panel k) at q * psiSrc + k * kPsiRow, with the
// row stride padded to 21 doubles and the source stride to 16 * 21 + 1, so that
// lanes reading different panels (and sources) spread over the LDS banks.
constexpr int kPsiRow = kChebDeg + 1;
constexpr int kFastRB = 4;       // 16-row blocks of the coefficient table per wave (rows <= 64 per wave)
__device__ __forceinline__ int psi_src_stride(int n_reg) { return n_reg * kPsiRow + 1; }

template <int NL>
__global__ __launch_bounds__(kFastRow) void k_local_fast(LocalArgs A, const int64_t *__restrict__ step, Geom g)
{
    const int64_t m = step[0] - g.lookahead;
    extern __shared__ double fast_lds[];              // psi [kFastSrc][psiSrc], then the hit rings
    __shared__ double sigs[kFastSrc * NL];
    __shared__ double2 spos[kFastSrc];
    __shared__ double2 tpos[kFastTB];
    __shared__ double tacc[kFastTB];
    __shared__ int tglob[kFastTB];
    __shared__ int qs[kLocalQueue], qt[kLocalQueue];
    __shared__ double qr[kLocalQueue];
    __shared__ int qn;
    __shared__ int rbeg[5], rcum[6];

    const int tid = threadIdx.x, bd = blockDim.x, lane = tid & 63, wave = tid >> 6, nwave = bd >> 6;
    const int n = A.ncell, D = kChebDeg, nrow = A.n_reg * kChebDeg, psiSrc = psi_src_stride(A.n_reg);
    const double d2 = A.delta * A.delta, dt = g.dt, q2 = 0.25 * dt * dt;
    double *psi = fast_lds;
    double *ring_r2 = fast_lds + kFastSrc * psiSrc + wave * kFastRing;
    uint32_t *ring_ts = reinterpret_cast<uint32_t *>(fast_lds + kFastSrc * psiSrc + nwave * kFastRing) + wave * kFastRing;
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;   // lanes below this one
    // psi = C sigma as FP64 MFMA 16x16x4 tiles: this wave owns row blocks rb = wave + j nwave
    // (16 table rows each); its A operands C[rb*16 + lane%16][4 ks + lane/16] are read from
    // the (L2-resident) table for each chunk, so they occupy registers only in that phase.
    constexpr int KS = (NL + 3) / 4;
    const int nblk = (nrow + 15) / 16;

    // targets kk in [tb0, tb0 + ntb) of the current 5 x 5 block -> LDS
    auto load_batch = [&](int tb0, int ntb) {
        for (int t = tid; t < ntb; t += bd) {
            const int kk = tb0 + t;
            int r = 0;
            while (r < 4 && kk >= rcum[r + 1]) ++r;
            const int tg = rbeg[r] + (kk - rcum[r]);
            tglob[t] = tg;
            tpos[t] = A.txy[tg];
            tacc[t] = 0.0;
        }
    };
    auto flush_batch = [&](int ntb) {
        for (int t = tid; t < ntb; t += bd)
            if (tacc[t] != 0.0) unsafeAtomicAdd(&A.ul[tglob[t]], tacc[t]);
    };
    // evaluate ring entries [h, h + 128) of this wave (those at or beyond `cnt` are padding)
    auto evaluate = [&](int h, int cnt) {
        const int e0 = h + lane, e1 = h + 64 + lane;
        const bool v0 = e0 < cnt, v1 = e1 < cnt;
        const int p0 = e0 % kFastRing, p1 = e1 % kFastRing;
        const uint32_t w0 = v0 ? ring_ts[p0] : 0u, w1 = v1 ? ring_ts[p1] : 0u;
        const double r0 = v0 ? sqrt(ring_r2[p0]) : dt, r1 = v1 ? sqrt(ring_r2[p1]) : dt;
        double x0, x1, u0, u1;
        const int k0 = fast_panel(A, r0, g.W, dt, x0), k1 = fast_panel(A, r1, g.W, dt, x1);
        cheb_eval2(psi + (int)(w0 >> 16) * psiSrc + k0 * kPsiRow, x0, psi + (int)(w1 >> 16) * psiSrc + k1 * kPsiRow, x1,
                   u0, u1);
        if (v0) atomicAdd(&tacc[w0 & 0xffffu], u0);
        if (v1) atomicAdd(&tacc[w1 & 0xffffu], u1);
    };

    for (int cell = blockIdx.x; cell < n * n; cell += gridDim.x) {
        const int s0 = A.scell_start[cell], s1 = A.scell_start[cell + 1];
        if (s0 == s1) continue;                     // uniform across the workgroup
        const int cx = cell % n, cy = cell / n;
        if (tid == 0) {
            int cum = 0, r = 0;
            const int xa = max(0, cx - 2), xb = min(n - 1, cx + 2);
            for (int yy = max(0, cy - 2); yy <= min(n - 1, cy + 2); ++yy, ++r) {
                const int b = A.tcell_start[yy * n + xa], e = A.tcell_start[yy * n + xb + 1];
                rbeg[r] = b;
                rcum[r] = cum;
                cum += e - b;
            }
            for (; r < 5; ++r) {
                rbeg[r] = 0;
                rcum[r] = cum;
            }
            rcum[5] = cum;
        }
        __syncthreads();
        const int NT = rcum[5];
        const bool single = NT <= kFastTB;        // all targets stay in LDS for the whole cell
        if (single) load_batch(0, NT);
        for (int sb = s0; sb < s1; sb += kFastSrc) {
            const int ns = min(kFastSrc, s1 - sb);
            for (int e = tid; e < ns * NL; e += bd) {
                const int sidx = e / NL, d = e - sidx * NL;
                sigs[e] = A.sig[sig_slot(m, d, g) * g.M + sb + sidx];
            }
            if (tid < ns) spos[tid] = A.sxy[sb + tid];
            {
                // A operands of this wave's row blocks: issued before the barrier so that their
                // latency overlaps the sigma loads
                double ca[kFastRB][KS];
#pragma unroll
                for (int j = 0; j < kFastRB; ++j) {
                    const int row = (wave + j * nwave) * 16 + (lane & 15);
                    const double *__restrict__ crow = A.creg + (size_t)min(row, nrow - 1) * NL;
#pragma unroll
                    for (int ks = 0; ks < KS; ++ks) {
                        const int d = 4 * ks + (lane >> 4);
                        ca[j][ks] = (row < nrow && d < NL) ? crow[d] : 0.0;
                    }
                }
                __syncthreads();
                mfma_d4 acc[kFastRB];
#pragma unroll
                for (int j = 0; j < kFastRB; ++j) acc[j] = mfma_d4{0.0, 0.0, 0.0, 0.0};
                const int q = lane & 15;
#pragma unroll
                for (int j = 0; j < kFastRB; ++j) {
                    const int rb = wave + j * nwave;
                    if (rb >= nblk) continue;              // uniform across the wave
#pragma unroll
                    for (int ks = 0; ks < KS; ++ks) {
                        const int d = 4 * ks + (lane >> 4);
                        const double b = (q < ns && d < NL) ? sigs[q * NL + d] : 0.0;   // B[d][q] = sigma_{q,d}
                        acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[j][ks], b, acc[j], 0, 0, 0);
                    }
                }
#pragma unroll
                for (int j = 0; j < kFastRB; ++j) {
                    const int rb = wave + j * nwave;
                    if (rb >= nblk || q >= ns) continue;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = rb * 16 + (lane >> 4) + 4 * r;   // D[lane][r] = C[lane/16 + 4 r][lane%16]
                        if (row < nrow) psi[q * psiSrc + (row / D) * kPsiRow + row % D] = acc[j][r];
                    }
                }
            }
            for (int tb0 = 0; tb0 < NT; tb0 += kFastTB) {
                const int ntb = min(kFastTB, NT - tb0);
                if (!single) load_batch(tb0, ntb);
                if (tid == 0) qn = 0;
                __syncthreads();
                // filter (source-major: lanes over targets) + compaction + evaluation, per wave
                int head = 0, cnt = 0;                  // wave-uniform ring counters
                const int ntb64 = (ntb + 63) >> 6;      // 64-target blocks per source
                for (int blk = wave; blk < ns * ntb64; blk += nwave) {   // (source, target block) round robin
                    const int sidx = blk / ntb64;
                    const double2 y = spos[sidx];
                    {
                        const int t = (blk - sidx * ntb64) * 64 + lane;
                        bool hit = false;
                        double r2 = 0.0;
                        if (t < ntb) {
                            const double2 x = tpos[t];
                            const double dx = x.x - y.x, dy = x.y - y.y;
                            r2 = dx * dx + dy * dy;
                            hit = r2 > 0.0 && r2 < d2;
                            if (hit && r2 < q2) {       // r < dt/2: dyadic sub-panels
                                hit = false;
                                const int q = atomicAdd(&qn, 1);
                                const double r = sqrt(r2);
                                if (q < kLocalQueue) {
                                    qs[q] = sidx;
                                    qt[q] = t;
                                    qr[q] = r;
                                } else {
                                    atomicAdd(&tacc[t], dyadic_direct(A, sigs + sidx * NL, NL, r, r * A.inv_dt));
                                }
                            }
                        }
                        const uint64_t mask = __ballot(hit);
                        if (hit) {
                            const int pos = (cnt + __popcll(mask & below)) % kFastRing;
                            ring_ts[pos] = (uint32_t)t | ((uint32_t)sidx << 16);
                            ring_r2[pos] = r2;
                        }
                        cnt += __popcll(mask);
                        if (cnt - head >= 128) {
                            wave_sync();
                            evaluate(head, cnt);
                            head += 128;
                            wave_sync();
                        }
                    }
                }
                wave_sync();
                for (; head < cnt; head += 128) evaluate(head, cnt);
                __syncthreads();
                // queued pairs with r < dt/2: one wavefront per pair, lanes over levels
                const int nq = min(qn, kLocalQueue);
                for (int q = wave; q < nq; q += nwave) {
                    const int sidx = qs[q];
                    const double r = qr[q];
                    const int sub = dyadic_sub(A, r * A.inv_dt);
                    const double xc = sub_coord(A.subs[sub], r);
                    double v = 0.0;
                    for (int d = lane; d < NL; d += 64)
                        v = fma(cheb_eval(A.cheb + ((size_t)sub * NL + d) * D, xc), sigs[sidx * NL + d], v);
                    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
                    if (lane == 0) atomicAdd(&tacc[qt[q]], v);
                }
                __syncthreads();
                if (!single) {
                    flush_batch(ntb);
                    __syncthreads();
                }
            }
        }
        if (single) {
            flush_batch(NT);
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Local part from pair lists made once per plan.  Sources and targets do not
// move, so the set of pairs with 0 < r < delta, each pair's time-step panel k
// and its Chebyshev coordinate x on that panel are the same at every step.
// k_pairs_build finds them per work unit (kPairUnit adjacent cells of a row,
// whose sources are contiguous in the sorted order; its targets are the union
// of their 5 x 5 cell blocks) with a count pass, then a fill pass at offsets
// scanned on the host, and stores them per segment (a chunk of kFastSrc sources
// of the unit x a batch of kPairTB of its targets): for a pair with r >= dt/2
// one 64-bit word (pair_pack:
// target in the batch, source in the chunk, panel k, Chebyshev coordinate x);
// for a pair with r < dt/2 (dyadic sub-panels) the word t | s << 16 and its
// weights eta_d(r).  Within a segment the regular pairs are ordered by source,
// then panel, then target (so the pairs of a 64-lane block mostly read one
// profile row: LDS broadcasts).
// k_local_pairs then does, per step and chunk: the profile coefficients
// psi = C sigma with FP64 MFMA, C being each regular panel's truncated series
// in the power basis, then its waves take 128-pair blocks of the segment in
// turn, two interleaved Horner sums per lane, with per-target sums in LDS;
// there is no candidate test, compaction or square root per pair, and every
// wave gets the same number of pairs.
// ---------------------------------------------------------------------------
static_assert(kFastSrc <= 16 && kPairTB <= 1024, "pair words hold the target in 10 bits and the source in 4");

// A regular pair in one 64-bit word: its target in the batch (bits 0-10; 1024 and above:
// private sums of the padding entries), the LDS offset of its profile row in 16-byte units
// (bits 11-22: s psiSrc + k D doubles for source s of the chunk and panel k), and its
// Chebyshev coordinate x in [-1, 1] as the 41-bit fraction f = (x + 1) / 2 (bits 23-63;
// resolution 9.1e-13), which under the exponent bits of 1.0 is the double 1 + f.
// Within a slot the pairs of each panel are padded to whole runs of kRunPairs with padding
// entries (target 1024 + e mod 128, the panel's profile row, x = 0), which add to private sums
// past the targets': every run of an item's list shares one profile row.  A segment's runs are
// stored interleaved by 16-byte chunks: chunk c (words 2c, 2c + 1) of run r of a segment of R
// runs at 16-byte offset c R + r, so that the lanes of a wave, one run each, read each chunk
// as one contiguous span.
constexpr int kRunPairs = 8;
constexpr int kPcFlushRounds = (kPairTB + 255) / 256;   // flush rounds of the local kernel's consumers (at least 4 waves)
constexpr int kPairTBPad = kPairTB + 128;             // per-target sums plus the padding entries' sums
__device__ __forceinline__ uint64_t pair_pack(int t, int row16, double x)
{
    const double f = 0.5 * (fmin(1.0, fmax(-1.0, x)) + 1.0);
    const uint64_t q = min((uint64_t)llrint(f * 2199023255552.0), (uint64_t)2199023255551ull);   // 2^41 f
    return (uint64_t)t | ((uint64_t)row16 << 11) | (q << 23);
}
__device__ __forceinline__ uint64_t pair_pad(int64_t e) { return (uint64_t)(1024 + (e & 127)) | ((uint64_t)1 << 63); }
// storage index of word e (in run order) of a segment of nrun runs starting at word s0
__device__ __forceinline__ int64_t pair_pos(int64_t s0, int64_t nrun, int64_t e)
{
    const int64_t rel = e - s0, r = rel / kRunPairs;
    const int j = (int)(rel - r * kRunPairs);
    return s0 + (int64_t)(j >> 1) * 2 * nrun + 2 * r + (j & 1);
}
__device__ __forceinline__ int pair_t(uint64_t w) { return (int)(w & 2047u); }
__device__ __forceinline__ int pair_row16(uint64_t w) { return (int)((w >> 11) & 4095u); }
__device__ __forceinline__ double pair_x(uint64_t w)
{
    const uint64_t one_f = ((w >> 12) & ~(uint64_t)0x7FF) | 0x3FF0000000000000ull;   // 1 + f
    return fma(2.0, __longlong_as_double((long long)one_f), -3.0);
}

// Work units (units with sources and with targets in their block), one record
// of kCellRec int32 each: the unit's sources [s0, s1) in sorted order, then the
// five runs (block rows) of its targets (rbeg[5], rcum[6]; see block_target).
constexpr int kCellRec = kPairRec;

// One item of the producer / consumer local kernel: the pair words [p0, p1) of one segment (a
// source chunk [sb, sb + ns) of work unit wk against target batch b), whole runs of kRunPairs.
// Each workgroup's items are consecutive (PairLists::ioff), the items of one (unit, batch)
// consecutive among them.
struct LpDesc {
    int64_t p0, p1;
    int32_t sb, ns, wk, b;
};

struct PairLists {
    const int32_t *wrec;          // [n_work][kCellRec]
    const int64_t *wseg;          // first segment of each work unit, [n_work + 1]
    int n_work;
    const int64_t *off, *doff;    // first pair of each (segment, source in chunk), [n_seg * kFastSrc + 1]
    const uint64_t *pw;           // regular pairs (pair_pack)
    const uint32_t *dent;         // pairs with r < dt/2: t | s << 16
    const double *dw;             //   their weights eta_d(r), [nlev][ndy] (dyadic sub-panel tables)
    const int32_t *dtg, *dsg;     //   their sorted target and source indices
    int64_t ndy;
    const LpDesc *desc;           // items of the producer / consumer kernel, by workgroup
    const int32_t *ioff;          //   first item of each workgroup, [grid + 1]
};

struct PairBuild {
    int64_t *cnt, *dcnt;          // count pass, per (segment, source in chunk): words | pairs << 32, dyadic pairs
    uint64_t *pw;                 // fill pass: the lists, at the offsets of PairLists
    uint32_t *dent;
    double *dw;                   //   weights of the pairs with r < dt/2, [nlev][ndy]
    int32_t *dtg, *dsg;           //   and their sorted target and source indices
    int64_t ndy;
    int fill, nlev;
    int psi_src, dterms;          // profile layout of the pair kernel (row offsets in the words)
};

// targets of a work unit's block: five runs of the sorted target order (rows
// cy-2..cy+2); run r starts at rbeg[r] and holds block positions [rcum[r], rcum[r+1])
__device__ __forceinline__ int block_target(const int *rbeg, const int *rcum, int kk)
{
    int r = 0;
    while (r < 4 && kk >= rcum[r + 1]) ++r;
    return rbeg[r] + (kk - rcum[r]);
}

// One wave per (chunk, batch, source): the wave walks the batch's targets 64 at a
// time and keeps the hits in target order (ballot + prefix count).
__global__ __launch_bounds__(256) void k_pairs_build(LocalArgs A, PairLists P, PairBuild B, double dt, int W)
{
    __shared__ int rec[kCellRec];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwave = blockDim.x >> 6;
    const double d2 = A.delta * A.delta, q2 = 0.25 * dt * dt;
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int *rbeg = rec + 2, *rcum = rec + 7;
    for (int wk = blockIdx.x; wk < P.n_work; wk += gridDim.x) {
        __syncthreads();                                         // the previous record is no longer read
        if (tid < kCellRec) rec[tid] = P.wrec[(int64_t)wk * kCellRec + tid];
        __syncthreads();
        const int s0 = rec[0], s1 = rec[1];
        const int64_t seg0 = P.wseg[wk];
        const int NT = rcum[5], nb = (NT + kPairTB - 1) / kPairTB;
        const int nch = (s1 - s0 + kFastSrc - 1) / kFastSrc;
        for (int task = wave; task < nch * nb * kFastSrc; task += nwave) {
            const int sl = task % kFastSrc, ib = task / kFastSrc, b = ib % nb, i = ib / nb;
            const int64_t slot = (seg0 + (int64_t)i * nb + b) * kFastSrc + sl;
            const int j = s0 + i * kFastSrc + sl;
            int64_t c_reg = 0, c_dy = 0, c_real = 0;
            if (j < s1) {
                const double2 y = A.sxy[j];
                const int tb0 = b * kPairTB, ntb = min(kPairTB, NT - tb0);
                const int64_t o_reg = B.fill ? P.off[slot] : 0, o_dy = B.fill ? P.doff[slot] : 0;
                const int64_t seg = slot / kFastSrc, sg0 = B.fill ? P.off[seg * kFastSrc] : 0;
                const int64_t nrun = B.fill ? (P.off[(seg + 1) * kFastSrc] - sg0) / kRunPairs : 0;
                // the fill pass writes the slot's regular pairs panel by panel (then in target
                // order), so that a wave's consecutive pairs mostly share one profile row
                for (int kk = 0; kk < W; ++kk) {
                const int64_t c_start = c_reg;
                for (int t0 = 0; t0 < ntb; t0 += 64) {
                    const int t = t0 + lane;
                    bool reg = false, dya = false;
                    double r2 = 0.0, x = 0.0;
                    int k = 0;
                    if (t < ntb) {
                        const double2 xt = A.txy[block_target(rbeg, rcum, tb0 + t)];
                        const double dx = xt.x - y.x, dy = xt.y - y.y;
                        r2 = dx * dx + dy * dy;
                        const bool hit = r2 > 0.0 && r2 < d2;
                        dya = hit && r2 < q2;
                        reg = hit && !dya;
                        if (reg) {
                            k = fast_panel(A, sqrt(r2), W, dt, x);
                            reg = k == kk;
                        }
                        dya = dya && kk == 0;
                    }
                    const uint64_t mr = __ballot(reg), md = __ballot(dya);
                    if (B.fill && reg) {
                        const int64_t e = o_reg + c_reg + __popcll(mr & below);
                        B.pw[pair_pos(sg0, nrun, e)] = pair_pack(t, (sl * B.psi_src + k * B.dterms) / 2, x);
                    }
                    if (B.fill && dya) {
                        const int64_t e = o_dy + c_dy + __popcll(md & below);
                        B.dent[e] = (uint32_t)t | ((uint32_t)sl << 16);
                        B.dtg[e] = block_target(rbeg, rcum, tb0 + t);
                        B.dsg[e] = j;
                        const double r = sqrt(r2);
                        const int sub = dyadic_sub(A, r * A.inv_dt);
                        const double xc = sub_coord(A.subs[sub], r);
                        for (int d = 0; d < B.nlev; ++d)
                            B.dw[d * B.ndy + e] = cheb_eval(A.cheb + ((size_t)sub * B.nlev + d) * kChebDeg, xc);
                    }
                    c_reg += __popcll(mr);
                    c_real += __popcll(mr);
                    c_dy += __popcll(md);
                }
                // the panel's group padded to whole runs of kRunPairs (padding: the group's row, x = 0)
                const int64_t padded = c_start + (c_reg - c_start + kRunPairs - 1) / kRunPairs * kRunPairs;
                if (B.fill)
                    for (int64_t e = c_reg + lane; e < padded; e += 64)
                        B.pw[pair_pos(sg0, nrun, o_reg + e)] =
                            pair_pad(o_reg + e) | ((uint64_t)((sl * B.psi_src + kk * B.dterms) / 2) << 11);
                c_reg = padded;
                }
            }
            if (!B.fill && lane == 0) {
                B.cnt[slot] = c_reg | c_real << 32;       // words (pairs and padding), pairs
                B.dcnt[slot] = c_dy;
            }
        }
    }
}

// every pair word set to the padding entry of its position (the fill pass then writes the pairs)
__global__ void k_pairs_pad(uint64_t *__restrict__ pw, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) pw[e] = pair_pad(e);
}

// a value the whole wave holds (loaded from LDS or memory), moved to a scalar register
// so that loops and branches on it are uniform
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// ---------------------------------------------------------------------------
// Local part from the pair lists, producer / consumer form.  One workgroup of
// 16 waves per CU walks its work items (work unit, target batch, source chunk:
// a segment of the lists) in order.  The first nprod waves (producers)
// synthesise the profile coefficients psi = C sigma of item t+1 with FP64 MFMA
// into one of two LDS buffers while the other waves (consumers) evaluate the
// pairs of item t from the other buffer, with the item's pair words loaded one
// item ahead; one workgroup barrier per item.  Producers hold the MFMA A
// operands and the sigma (B) operands in registers, consumers only pair words:
// each role fits its registers, and the matrix units and the vector units work
// at the same time.  Per-target sums of a (work unit, batch) collect in one of
// two LDS buffers and are flushed to u_l with device atomics one item after
// the batch ends (its buffer is then no longer written).  Pairs with
// r < dt/2 are summed by k_local_dyadic.
// ---------------------------------------------------------------------------
// A uniform record spread over the lanes of one register (lane k holds 32-bit word k),
// loaded ahead of use without tying up a register per word; fields are read with readlane.
// (src is wave-uniform; every lane loads, lanes from nwords on the last word, so no branch
// surrounds the load and no use of the value other than word32 / word64 waits for it)
__device__ __forceinline__ uint32_t lane_words(const void *src, int nwords, int lane)
{
    return reinterpret_cast<const uint32_t *>(src)[(uint32_t)min(lane, nwords - 1)];
}
__device__ __forceinline__ int word32(uint32_t v, int k) { return __builtin_amdgcn_readlane((int)v, k); }
__device__ __forceinline__ int64_t word64(uint32_t v, int k)
{
    return (int64_t)(((uint64_t)(uint32_t)word32(v, k + 1) << 32) | (uint32_t)word32(v, k));
}
// LpDesc words: p0 = 0..1, p1 = 2..3, sb = 4, ns = 5, wk = 6, b = 7
constexpr int kDescWords = 8;


// RB 16-row MFMA blocks per producer wave; the A operands (the power-basis table) in registers
// (RB == 2), in LDS (RB == 4: the table is staged once per launch), or read from cache (RB == 3).
template <int NL, int NTERM, int RB>
__global__ __launch_bounds__(1024) void k_local_pc(LocalArgs A, PairLists P, const int64_t *__restrict__ step, Geom g, int nprod)
{
    // Every global load is issued at least one item before its value is used, and the loop
    // bodies have no data-dependent branches around loads or MFMAs, so the in-order wait on
    // outstanding loads never waits for a prefetch of a later item.
    constexpr int KS = (NL + 3) / 4, D = NTERM;
    constexpr bool kRegA = RB == 2, kLdsA = RB == 4;
    if (kLdsA) nprod = 4;                             // the LDS-table form always has four producers
    const int64_t m = step[0] - g.lookahead;
    // dynamic LDS: [A table (RB == 4): rows [64 r, 64 r + 64) hold the levels from 4 kst(r) on]
    // then psi[2][kFastSrc][psiSrc] (16-byte rows; RB == 4 pads each panel's row, pc_panel_stride)
    constexpr int PS = kLdsA && D == 16 ? 18 : D;     // doubles per panel row in psi (pc_panel_stride)
    extern __shared__ __align__(16) double lp_dyn[];
    double *const ctab = lp_dyn;
    double *const lp_lds = lp_dyn + (kLdsA ? pc_ctab_doubles(D, KS) : 0);
    __shared__ double tacc[2][kPairTBPad];            // per-target sums of a (unit, batch), by parity
    // compacted table: row stride and start of region r
    auto ct_len = [](int r) { return pc_ctab_stride(r, D, KS); };
    auto ct_off = [&](int r) {
        int o = 0;
        for (int rr = 0; rr < r; ++rr) o += 64 * ct_len(rr);
        return o;
    };

    const int tid = threadIdx.x, lane = tid & 63, wave = uniform(tid >> 6);
    const int nrow = A.n_reg * D, psiSrc = A.n_reg * PS + 2;
    const int i0 = P.ioff[blockIdx.x], ni = P.ioff[blockIdx.x + 1] - i0;   // this workgroup's items
    const LpDesc *__restrict__ desc = P.desc + i0;
    auto item = [&](int t) { return lane_words(desc + min(t, ni - 1), kDescWords, lane); };   // in range when ni > 0
    for (int t = tid; t < 2 * kPairTBPad; t += 1024) (&tacc[0][0])[t] = 0.0;
    if (kLdsA)                                        // A table C[row][d], rows past the table and d >= NL zero
#pragma unroll
        for (int r = 0; r < 4; ++r)
            for (int e = tid; e < 64 * ct_len(r); e += 1024) {
                const int row = 64 * r + e / ct_len(r), j = e % ct_len(r), d = 4 * pc_kst(r, D) + j;
                ctab[ct_off(r) + e] = (j < ct_len(r) - 2 && row < nrow && d < NL)
                                          ? A.cpow[(size_t)((row / D) * kChebDeg + row % D) * NL + d] : 0.0;
            }
    __syncthreads();
    if (ni == 0) return;                              // uniform, after the only barrier so far

    if (wave < nprod) {
        // ---------------- producer ----------------
        // A operand of block r, step ks: C[row][d], row = (wave + r nprod) 16 + lane % 16, d = 4 ks + lane / 16
        // (zero for rows past the table: their MFMAs add nothing and their rows are not stored)
        auto a_op = [&](int r, int ks) {
            const int row = (wave + r * nprod) * 16 + (lane & 15), d = 4 * ks + (lane >> 4);
            if (kLdsA) return ctab[ct_off(r) + (row - 64 * r) * ct_len(r) + (d - 4 * pc_kst(r, D))];   // ks >= kst(r)
            const int rr = min(row, nrow - 1), dd = min(d, NL - 1);
            const double v = A.cpow[(size_t)((rr / D) * kChebDeg + rr % D) * NL + dd];
            return (row < nrow && d < NL) ? v : 0.0;
        };
        double ca[kRegA ? RB : 1][KS];
#pragma unroll
        for (int r = 0; r < (kRegA ? RB : 0); ++r)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) ca[r][ks] = a_op(r, ks);
        // B operands sigma[q][d] (q = lane % 16, d = 4 ks + lane / 16) of two items, loaded two
        // items ahead.  A lane past the chunk loads the chunk's first source: its column of psi is
        // never read.  A lane past the levels loads level NL - 1: its A column is zero, so it adds
        // nothing (a non-finite sample there makes the result non-finite either way).
        // The ring slot of level d is (s0 - d) mod depth with s0 the slot of level 0 (d < NL <= depth).
        const int s0 = (int)sig_slot(m, 0, g), depth = (int)g.sig_depth;
        double bva[KS], bvb[KS];
        auto load_b = [&](double (&bv)[KS], uint32_t dv) {
            const int sb = word32(dv, 4), ns = word32(dv, 5), q = lane & 15;
            const int64_t src = sb + (q < ns ? q : 0);
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int sl = s0 - min(4 * ks + (lane >> 4), NL - 1);
                bv[ks] = A.sig[(int64_t)(sl < 0 ? sl + depth : sl) * g.M + src];
            }
        };
        auto synth = [&](const double (&bv)[KS], double *dst) {
            mfma_d4 acc[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) acc[r] = mfma_d4{0.0, 0.0, 0.0, 0.0};
            if (kLdsA) {
                // A regular panel k weights only levels d >= k (its nodes lie at delays >= k dt and
                // the centred stencils reach back, never forward, from there; the plan takes this
                // form only when its table has those zeros): block r holds panels >= (64 r)/D, so
                // its k-steps below kst(r) are zero and the table does not hold them.
#pragma unroll
                for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                    for (int r = 0; r < RB; ++r)
                        if (ks >= pc_kst(r, D))
                            acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_op(r, ks), bv[ks], acc[r], 0, 0, 0);
            } else {
#pragma unroll
                for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                    for (int r = 0; r < RB; ++r)
                        acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(kRegA ? ca[kRegA ? r : 0][ks] : a_op(r, ks), bv[ks], acc[r],
                                                                      0, 0, 0);
            }
            // D[lane][e] = C[row = (wave + r nprod) 16 + lane / 16 + 4 e][q = lane % 16], stored at
            // q psiSrc + (row / D) PS + row % D; with nprod known at compile time and PS = D the
            // stores share one address register and immediate offsets
            double *const dq = dst + (lane & 15) * psiSrc;
            if constexpr (PS == D || D == 16) {
                // a 16-row block is one panel (D = 16) or rows are dense: one base, immediate offsets
                constexpr int BS = D == 16 ? PS : 16;  // psi doubles per 16-row block
                double *const db = dq + wave * BS + (lane >> 4);
#pragma unroll
                for (int r = 0; r < RB; ++r)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if ((lane >> 4) < nrow - (wave + r * nprod) * 16 - 4 * e) db[r * nprod * BS + 4 * e] = acc[r][e];
            } else {
#pragma unroll
                for (int r = 0; r < RB; ++r)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int row = (wave + r * nprod) * 16 + (lane >> 4) + 4 * e;
                        if (row < nrow) dq[row + (row / D) * (PS - D)] = acc[r][e];
                    }
            }
        };
        load_b(bva, item(0));
        synth(bva, lp_lds);                           // item 0 -> buffer 0
        load_b(bva, item(1));
        load_b(bvb, item(2));
        uint32_t d3 = item(3);                        // descriptor of the next item whose sigma is loaded
        __syncthreads();
        // item t: synthesise item t + 1 from the registers loaded two items ago (bva for even t,
        // bvb for odd t), then load item t + 3's sigma into them (clamped at the last item)
        auto iter = [&](double (&bv)[KS], int t) {
            synth(bv, lp_lds + (size_t)((t + 1) & 1) * kFastSrc * psiSrc);   // past the last item: unused
            const uint32_t dv = d3;
            d3 = item(t + 4);
            load_b(bv, dv);
            __syncthreads();
        };
        for (int t = 0; t < ni; t += 2) {
            iter(bva, t);
            if (t + 1 < ni) iter(bvb, t + 1);
        }
        return;
    }

    // ---------------- consumer ----------------
    // Lane cl of the consumers takes run cl of the item (words p0 + kRunPairs cl, ...): its pairs
    // share one profile row, loaded once into registers; the run's pairs are independent Horner
    // chains.  The next item's run is loaded during this one; runs past the consumers' lanes
    // (items of more runs) follow from memory.
    const int cw = wave - nprod, ncons = 16 - nprod, nl = ncons * 64, cl = cw * 64 + lane;
    // the (unit, batch) whose sums are in tacc[(sub - 1) & 1]; its predecessor is flushed one item later
    int sub = 0, pwk = -1, pb = 0;
    uint32_t prec = 0u;                               // record of the (unit, batch) being summed (lane words)
    // (a fixed number of predicated atomics per lane, so that the compiler's count of
    // outstanding memory operations stays exact across the loop)
    auto flush = [&](int buf, int fb, uint32_t rec) {
        int rbeg[5], rcum[6];
#pragma unroll
        for (int k = 0; k < 5; ++k) rbeg[k] = word32(rec, 2 + k);
#pragma unroll
        for (int k = 0; k < 6; ++k) rcum[k] = word32(rec, 7 + k);
        const int tb0 = fb * kPairTB, ntb = min(kPairTB, rcum[5] - tb0);
#pragma unroll
        for (int k = 0; k < kPcFlushRounds; ++k) {
            const int t = cl + k * nl;
            const double v = t < ntb ? tacc[buf][t] : 0.0;
            if (v != 0.0) {
                unsafeAtomicAdd(&A.ul[block_target(rbeg, rcum, tb0 + t)], v);
                tacc[buf][t] = 0.0;
            }
        }
    };
    // run r of the item [p0, p1) (p0, p1 uniform; an item holds fewer than 2^28 runs); a lane
    // past the item's runs loads run 0 (word 0 of the lists if the item is empty), and its sums
    // go to the padding entries.  The loads are unconditional.
    auto load_run = [&](uint64_t (&w)[kRunPairs], int64_t p0, int64_t p1, int r) {
        const ulonglong2 *base = reinterpret_cast<const ulonglong2 *>(P.pw + (p1 > p0 ? p0 : 0));
        const uint32_t nrun = (uint32_t)((p1 - p0) / kRunPairs), rr = (uint32_t)r < nrun ? (uint32_t)r : 0u;
#pragma unroll
        for (int c = 0; c < kRunPairs / 2; ++c) {
            const ulonglong2 v = base[c * nrun + rr];
            w[2 * c] = v.x;
            w[2 * c + 1] = v.y;
        }
    };
    auto run = [&](const uint64_t (&w)[kRunPairs], bool ok, const double2 *ps, double *acc) {
        const double2 *row = ps + pair_row16(w[0]);
        double2 c[D / 2];
#pragma unroll
        for (int j = 0; j < D / 2; ++j) c[j] = row[j];
        // two halves of four chains each (the scheduler barrier keeps their registers apart)
#pragma unroll
        for (int h = 0; h < kRunPairs; h += kRunPairs / 2) {
            double x[kRunPairs / 2], y[kRunPairs / 2];
#pragma unroll
            for (int i = 0; i < kRunPairs / 2; ++i) {
                x[i] = pair_x(w[h + i]);
                y[i] = fma(c[D / 2 - 1].y, x[i], c[D / 2 - 1].x);
            }
#pragma unroll
            for (int j = D / 2 - 2; j >= 0; --j)
#pragma unroll
                for (int i = 0; i < kRunPairs / 2; ++i) y[i] = fma(fma(y[i], x[i], c[j].y), x[i], c[j].x);
#pragma unroll
            for (int i = 0; i < kRunPairs / 2; ++i)
                atomicAdd(&acc[ok ? pair_t(w[h + i]) : kPairTB + h + i], y[i]);
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    // item t with its run wc, descriptor dc and unit record rc, all loaded during item t - 1; it
    // loads item t + 1's run and record into wn and rn, and item t + 2's descriptor into dc.  The
    // loop runs two items per pass with the registers' roles swapped, so that no loaded value is
    // copied (a copy would wait for every load issued before it).
    auto iter = [&](uint64_t (&wc)[kRunPairs], uint64_t (&wn)[kRunPairs], uint32_t &dc, uint32_t dn, uint32_t rc,
                    uint32_t &rn, int t) {
        const int64_t p0 = word64(dc, 0), p1 = word64(dc, 2);
        const int wk = word32(dc, 6), b = word32(dc, 7);
        const int64_t q0 = word64(dn, 0), q1 = word64(dn, 2);
        const int wkn = word32(dn, 6);
        const bool fresh = wk != pwk || b != pb;      // a new (unit, batch) starts with this item
        // the previous (unit, batch), all its items summed, is flushed after the last wait for
        // loads of the previous item and before this item's loads are issued, so that the next
        // wait (for those loads) finds the atomics long done
        if (fresh && pwk >= 0) flush((sub - 1) & 1, pb, prec);
        load_run(wn, q0, q1, cl);                     // in flight during this item
        rn = lane_words(P.wrec + (int64_t)wkn * kCellRec, 13, lane);
        dc = item(t + 2);
        if (fresh) {
            prec = rc;
            pwk = wk;
            pb = b;
            sub += 1;
        }
        double *acc = tacc[(sub - 1) & 1];
        const double2 *ps = reinterpret_cast<const double2 *>(lp_lds + (size_t)(t & 1) * kFastSrc * psiSrc);
        if (kRunPairs * (int64_t)(cw * 64) < p1 - p0)                      // waves past the item's runs idle
            run(wc, (int64_t)kRunPairs * cl < p1 - p0, ps, acc);
        for (int r = cl + nl; (int64_t)kRunPairs * r < p1 - p0; r += nl) {   // items of more runs than consumer lanes
            uint64_t w[kRunPairs];
            load_run(w, p0, p1, r);
            run(w, true, ps, acc);
        }
        __syncthreads();
    };
    uint64_t wa[kRunPairs], wb[kRunPairs];
    uint32_t da = item(0), db = item(1);
    uint32_t ra = lane_words(P.wrec + (int64_t)word32(da, 6) * kCellRec, 13, lane), rb = 0u;
    load_run(wa, word64(da, 0), word64(da, 2), cl);
    __syncthreads();                                  // psi of item 0 is ready
    for (int t = 0; t < ni; t += 2) {
        iter(wa, wb, da, db, ra, rb, t);              // da <- item t + 2
        if (t + 1 < ni) iter(wb, wa, db, da, rb, ra, t + 1);   // db <- item t + 3
    }
    if (pwk >= 0) flush((sub - 1) & 1, pb, prec);     // the last (unit, batch): all items summed
}

// Pairs with r < dt/2 (their stored weights over the sigma levels), one lane per pair.
__global__ __launch_bounds__(256) void k_local_dyadic(LocalArgs A, PairLists P, const int64_t *__restrict__ step, Geom g)
{
    __shared__ int64_t slot_base[kLocalMaxLevels];
    const int64_t m = step[0] - g.lookahead;
    if ((int)threadIdx.x < g.nlev) slot_base[threadIdx.x] = sig_slot(m, threadIdx.x, g) * g.M;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < P.ndy; q += stride) {
        const int s = P.dsg[q];
        double v = 0.0;
        for (int d = 0; d < g.nlev; ++d) v = fma(P.dw[(int64_t)d * P.ndy + q], A.sig[slot_base[d] + s], v);
        unsafeAtomicAdd(&A.ul[P.dtg[q]], v);
    }
}

// Grid-stride fill: a dispatch covers at most 2^32 work-items, and the sigma
// ring alone can exceed that (4.3e9 doubles at 10^6 sources).
// Exponential-of-semicircle weights of the NUFFT kernel (R18), psi(z) = exp(beta (sqrt(1 - (2z/w)^2)
// - 1)) for |z| <= w/2, at the w grid offsets of each point's stencil in x and in y: point e
// (coordinates xy[idx[e]], or xy[e] without idx) with origin base[e] (relative to lmin).
template <class R>
__global__ __launch_bounds__(256) void k_es_weights(const double2 *__restrict__ xy, const int32_t *__restrict__ idx,
                                                    const int2 *__restrict__ base, int64_t n, double gscale, int lmin,
                                                    int w, double beta, R *__restrict__ wts)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const double2 pt = xy[idx ? idx[e] : e];
    const double gx = pt.x * gscale, gy = pt.y * gscale;
    const int2 b = base[e];
    auto psi = [&](double z) {
        const double t = 2.0 * z / w, a = 1.0 - t * t;
        return a < 0.0 ? 0.0 : exp(beta * (sqrt(a) - 1.0));
    };
    for (int a2 = 0; a2 < w; ++a2) {
        wts[e * 2 * w + a2] = (R)psi((double)(b.x + lmin + a2) - gx);
        wts[e * 2 * w + w + a2] = (R)psi((double)(b.y + lmin + a2) - gy);
    }
}

hipError_t launch_es_weights(Plan &p, const double2 *xy, const int32_t *idx, const int2 *base, int64_t n, double gscale,
                             void *wts)
{
    if (n == 0) return hipSuccess;
    const unsigned nb = (unsigned)((n + 255) / 256);
    if (p.precision == WFP2D_PREC_MIXED)
        hipLaunchKernelGGL(k_es_weights<float>, dim3(nb), dim3(256), 0, p.stream, xy, idx, base, n, gscale, (int)p.g.lmin, p.g.w,
                           p.es_beta, (float *)wts);
    else
        hipLaunchKernelGGL(k_es_weights<double>, dim3(nb), dim3(256), 0, p.stream, xy, idx, base, n, gscale, (int)p.g.lmin,
                           p.g.w, p.es_beta, (double *)wts);
    return hipGetLastError();
}

// Hankel coefficients of eq. H on the device: H[c][l] = sum_g J0(kappa_c r_g) E[l][g], the
// quadrature nodes r and weights-with-kernel E from hankel_quadrature.  One workgroup per 16
// classes x 64 SOE terms; the nodes in chunks of 64 with J0 and E staged in LDS (E rows padded
// to 65 doubles: the 16 rows a wave reads fall in distinct banks).
constexpr int kHkC = 16, kHkL = 64, kHkG = 64;
__global__ __launch_bounds__(256) void k_hankel(const double *__restrict__ kappa, int64_t nk, const double *__restrict__ r,
                                                int nr, const double *__restrict__ E, int L, double *__restrict__ H)
{
    __shared__ double sJ[kHkC][kHkG];
    __shared__ double sE[kHkL][kHkG + 1];
    const int tid = threadIdx.x, cl = tid >> 4, lq = tid & 15;
    const int64_t c0 = (int64_t)blockIdx.x * kHkC;
    const int l0 = blockIdx.y * kHkL;
    double acc[kHkL / 16] = {0.0, 0.0, 0.0, 0.0};
    for (int g0 = 0; g0 < nr; g0 += kHkG) {
        for (int e = tid; e < kHkC * kHkG; e += 256) {
            const int ci = e / kHkG, gi = e % kHkG;
            const int64_t c = c0 + ci;
            sJ[ci][gi] = (c < nk && g0 + gi < nr) ? j0(kappa[c] * r[g0 + gi]) : 0.0;
        }
        for (int e = tid; e < kHkL * kHkG; e += 256) {
            const int li = e / kHkG, gi = e % kHkG;
            sE[li][gi] = (l0 + li < L && g0 + gi < nr) ? E[(size_t)(l0 + li) * nr + g0 + gi] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int gi = 0; gi < kHkG; ++gi) {
            const double j = sJ[cl][gi];
#pragma unroll
            for (int k = 0; k < kHkL / 16; ++k) acc[k] = fma(j, sE[lq + 16 * k][gi], acc[k]);
        }
        __syncthreads();
    }
    const int64_t c = c0 + cl;
    if (c < nk)
#pragma unroll
        for (int k = 0; k < kHkL / 16; ++k)
            if (l0 + lq + 16 * k < L) H[c * L + l0 + lq + 16 * k] = acc[k];
}

__global__ void k_zero_f64(double *__restrict__ p, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0.0;
}

// u (caller order) = u_h + u_l, or zeros before the first reported step
__global__ void k_combine(const double *__restrict__ uh, const double *__restrict__ ul, const int32_t *__restrict__ rank,
                          double *__restrict__ u, int64_t Nx, const int64_t *__restrict__ step, int lookahead)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Nx) return;
    if (step[0] - lookahead < 1) {   // u(t <= 0) = 0 (zero initial data)
        u[i] = 0.0;
        return;
    }
    const int s = rank[i];
    u[i] = uh[s] + ul[s];
}

// acc[i] += wts[i] * u(x_i, t_m): the field folded into a running weighted sum
// (used by the adjoint to reduce d(loss)/d(sigma_j(t_l)) against sigma's
// dependence on source strengths without materialising the field)
__global__ void k_combine_dot(const double *__restrict__ uh, const double *__restrict__ ul, const int32_t *__restrict__ rank,
                              const double *__restrict__ wts, double *__restrict__ acc, int64_t Nx,
                              const int64_t *__restrict__ step, int lookahead)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Nx || step[0] - lookahead < 1) return;
    const int s = rank[i];
    acc[i] += wts[i] * (uh[s] + ul[s]);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_step_begin(Plan &p)
{
    hipLaunchKernelGGL(k_step_begin, dim3(1), dim3(1), 0, p.stream, p.d_step);
    return hipGetLastError();
}

hipError_t launch_ingest_at(Plan &p, const double *sigma_in, int64_t n)
{
    const int64_t slot = ((n % p.g.sig_depth) + p.g.sig_depth) % p.g.sig_depth;
    hipLaunchKernelGGL(k_ingest_slot, dim3(nblk(p.M, 256)), dim3(256), 0, p.stream, sigma_in, p.d_src_perm, p.d_sig, p.M, slot,
                       p.d_nonfinite);
    return hipGetLastError();
}

hipError_t launch_ingest(Plan &p, const double *sigma_in)
{
    hipLaunchKernelGGL(k_ingest, dim3(nblk(p.M, 256)), dim3(256), 0, p.stream, sigma_in, p.d_src_perm, p.d_sig, p.M, p.d_step,
                       p.g.sig_depth, p.d_nonfinite);
    return hipGetLastError();
}

template <class R, int TX, int TY>
static hipError_t spread_as(Plan &p)
{
    const Geom &g = p.g;
    const size_t lds = (size_t)64 * (2 * g.w + 1) * sizeof(R);
    const int ntile = p.sp_ntx * p.sp_nty;
    const unsigned nblk = (unsigned)(((ntile + 7) >> 3) << 3);
    hipLaunchKernelGGL((k_spread<R, TX, TY>), dim3(nblk), dim3(64), lds, p.stream, p.d_sig, p.d_step, p.d_src_base,
                       (const R *)p.d_src_wts, p.d_tile_off, p.d_tile_src, (typename cplx<R>::T *)p.d_grid, g.w,
                       p.sp_ntx, ntile, g.Lpad, g);
    return hipGetLastError();
}

// the contraction form on 16 x 16 tiles (the source lists of shape 16 x 16)
template <class R>
static hipError_t spread_mfma(Plan &p)
{
    const Geom &g = p.g;
    if (p.sp_tx != 16 || p.sp_ty != 16 || g.w > 16) return hipErrorInvalidValue;
    const size_t lds = (size_t)64 * (2 * g.w + 1) * sizeof(R);
    const int ntile = p.sp_ntx * p.sp_nty;
    const unsigned nblk = (unsigned)(((ntile + 7) >> 3) << 3);
    hipLaunchKernelGGL((k_spread_mfma<R>), dim3(nblk), dim3(64), lds, p.stream, p.d_sig, p.d_step, p.d_src_base,
                       (const R *)p.d_src_wts, p.d_tile_off, p.d_tile_src, (typename cplx<R>::T *)p.d_grid, g.w,
                       p.sp_ntx, ntile, g.Lpad, g);
    return hipGetLastError();
}

template <class R>
static hipError_t spread_typed(Plan &p)
{
    switch (p.spread_tile) {
    case 1: return spread_as<R, 8, 8>(p);
    case 2: return spread_as<R, 16, 8>(p);
    case 3: return spread_as<R, 16, 16>(p);
    case 4: return spread_as<R, 32, 16>(p);
    case 5: return spread_as<R, 32, 32>(p);
    case 6: return spread_mfma<R>(p);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_spread(Plan &p)
{
    return p.precision == WFP2D_PREC_MIXED ? spread_typed<float>(p) : spread_typed<double>(p);
}

// dynamic LDS of the local kernels: the fast one's kFastRow rows x kFastSrc sources of profile
// coefficients plus one hit ring per wave; the pair-list one's two profile buffers
hipError_t kernel_setup(Plan &)
{
    const int bytes = kFastSrc * (kFastRow / kChebDeg * (kChebDeg + 1) + 1) * (int)sizeof(double) +
                      (kFastRow / 64) * kFastRing * 12;
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void *)k_local_fast<35>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes))) return e;
    if ((e = hipFuncSetAttribute((const void *)k_local_fast<43>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes))) return e;
    // producer / consumer kernel: two profile buffers and two pair-word buffers (the LDS left)
    const int pcbytes = (int)kPcDynLds;
    const void *pc[] = {(const void *)k_local_pc<35, 12, 2>, (const void *)k_local_pc<35, 14, 2>, (const void *)k_local_pc<35, 16, 2>,
                        (const void *)k_local_pc<35, 20, 2>, (const void *)k_local_pc<43, 12, 2>, (const void *)k_local_pc<43, 14, 2>,
                        (const void *)k_local_pc<43, 16, 2>, (const void *)k_local_pc<43, 20, 2>, (const void *)k_local_pc<35, 20, 3>,
                        (const void *)k_local_pc<43, 20, 3>, (const void *)k_local_pc<35, 12, 4>,
                        (const void *)k_local_pc<35, 14, 4>, (const void *)k_local_pc<35, 16, 4>};
    for (const void *k : pc)
        if ((e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, pcbytes))) return e;
    return hipSuccess;
}

static size_t fft_lds_bytes(const Plan &p)
{
    const size_t line = (size_t)(p.g.Q + p.g.Q / 16) * 2 * p.sizeof_real;   // multiple of 16 bytes
    return line + (size_t)(64 + p.g.nf / 64) * sizeof(double2);
}

template <class R>
static hipError_t fft_attrs(size_t bytes)
{
    hipError_t e;
    if ((e = hipFuncSetAttribute((const void *)k_fft_t1<R, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes))) return e;
    if ((e = hipFuncSetAttribute((const void *)k_fft_t1<R, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes))) return e;
    if constexpr (sizeof(R) == 4) {
        const void *pruned[] = {(const void *)k_fft_t1<R, 0, 5>, (const void *)k_fft_t1<R, 1, 5>, (const void *)k_fft_t1<R, 0, 6>,
                                (const void *)k_fft_t1<R, 1, 6>, (const void *)k_fft_t1<R, 0, 8>, (const void *)k_fft_t1<R, 1, 8>};
        for (const void *k : pruned)
            if ((e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes))) return e;
    }
    if ((e = hipFuncSetAttribute((const void *)k_fft_t2<R, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes))) return e;
    return hipFuncSetAttribute((const void *)k_fft_t2<R, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t fft_setup(Plan &p)
{
    const size_t bytes = fft_lds_bytes(p);
    return p.precision == WFP2D_PREC_MIXED ? fft_attrs<float>(bytes) : fft_attrs<double>(bytes);
}

template <class C>
static void transpose(const Plan &p, const void *in, void *out, int rows, int cols)
{
    dim3 grid((cols + 31) / 32, (rows + 31) / 32);
    hipLaunchKernelGGL(k_transpose<C>, grid, dim3(256), 0, p.stream, (const C *)in, (C *)out, rows, cols);
}

// FP32 type-1 line transforms with the first pass pruned to the NZ nonzero values per
// thread: NZ >= ceil(Lpad / (P T)), rounded up to an instantiated count
template <int MODE>
static void launch_t1_f32(Plan &p, const void *in, void *out, unsigned nlines)
{
    const Geom &g = p.g;
    const size_t sh = fft_lds_bytes(p);
    const int T = g.Q / 16, nz = (g.Lpad + g.P * T - 1) / (g.P * T);
    const float2 *x = (const float2 *)in, *corr = (const float2 *)p.d_corr;
    float2 *y = (float2 *)out;
    const double2 *tw = (const double2 *)p.d_tw;
    if (nz <= 5) hipLaunchKernelGGL((k_fft_t1<float, MODE, 5>), dim3(nlines), dim3(T), sh, p.stream, x, y, corr, tw, g);
    else if (nz <= 6) hipLaunchKernelGGL((k_fft_t1<float, MODE, 6>), dim3(nlines), dim3(T), sh, p.stream, x, y, corr, tw, g);
    else if (nz <= 8) hipLaunchKernelGGL((k_fft_t1<float, MODE, 8>), dim3(nlines), dim3(T), sh, p.stream, x, y, corr, tw, g);
    else hipLaunchKernelGGL((k_fft_t1<float, MODE, 16>), dim3(nlines), dim3(T), sh, p.stream, x, y, corr, tw, g);
}

hipError_t launch_fft_rows1(Plan &p)
{
    const Geom &g = p.g;
    const size_t sh = fft_lds_bytes(p);
    const unsigned T = (unsigned)(g.Q / 16);
    if (p.precision == WFP2D_PREC_MIXED)
        launch_t1_f32<0>(p, p.d_grid, p.d_T1, (unsigned)g.Lpad);
    else
        hipLaunchKernelGGL((k_fft_t1<double, 0>), dim3(g.Lpad), dim3(T), sh, p.stream, (const double2 *)p.d_grid, (double2 *)p.d_T1,
                           (const double2 *)p.d_corr, (const double2 *)p.d_tw, g);
    return hipGetLastError();
}

hipError_t launch_fft_cols1(Plan &p)
{
    const Geom &g = p.g;
    const size_t sh = fft_lds_bytes(p);
    const unsigned T = (unsigned)(g.Q / 16);
    if (p.precision == WFP2D_PREC_MIXED) {
        transpose<float2>(p, p.d_T1, p.d_T1t, g.Lpad, g.N);
        launch_t1_f32<1>(p, p.d_T1t, p.d_F, (unsigned)g.N);
    } else {
        transpose<double2>(p, p.d_T1, p.d_T1t, g.Lpad, g.N);
        hipLaunchKernelGGL((k_fft_t1<double, 1>), dim3(g.N), dim3(T), sh, p.stream, (const double2 *)p.d_T1t, (double2 *)p.d_F,
                           (const double2 *)p.d_corr, (const double2 *)p.d_tw, g);
    }
    return hipGetLastError();
}

hipError_t launch_split(Plan &p)
{
    const Geom &g = p.g;
    const int64_t H = p.n_modes;
    if (p.precision == WFP2D_PREC_MIXED)
        hipLaunchKernelGGL(k_split<float>, dim3((unsigned)p.n_chunks), dim3(kChunk), 0, p.stream, (const float2 *)p.d_F, p.d_chunks,
                           (float2 *)p.d_ring_cur, (float2 *)p.d_ring_lag, H, p.d_step, g);
    else
        hipLaunchKernelGGL(k_split<double>, dim3((unsigned)p.n_chunks), dim3(kChunk), 0, p.stream, (const double2 *)p.d_F, p.d_chunks,
                           (double2 *)p.d_ring_cur, (double2 *)p.d_ring_lag, H, p.d_step, g);
    return hipGetLastError();
}

hipError_t launch_near(Plan &p)
{
    const Geom &g = p.g;
    if (p.precision == WFP2D_PREC_MIXED)
        hipLaunchKernelGGL(k_near<float>, dim3((unsigned)p.n_chunks), dim3(kChunk), 0, p.stream, p.d_chunks, (const float2 *)p.d_ring_cur,
                           (const float2 *)p.d_ring_lag, p.d_D, p.d_C, p.d_phi_in, (float2 *)p.d_atot, p.n_modes, p.d_step, g);
    else
        hipLaunchKernelGGL(k_near<double>, dim3((unsigned)p.n_chunks), dim3(kChunk), 0, p.stream, p.d_chunks, (const double2 *)p.d_ring_cur,
                           (const double2 *)p.d_ring_lag, p.d_D, p.d_C, p.d_phi_in, (double2 *)p.d_atot, p.n_modes, p.d_step, g);
    return hipGetLastError();
}

hipError_t launch_far(Plan &p)
{
    const Geom &g = p.g;
    if (p.n_far == 0) return hipSuccess;
    const unsigned nb = nblk(p.n_far, 4);
    if (p.precision == WFP2D_PREC_MIXED)
        hipLaunchKernelGGL(k_far<float>, dim3(nb), dim3(256), 0, p.stream, p.d_far_pk, p.d_far_cls, p.d_H, p.d_chi, p.d_dec, p.d_inj,
                           p.d_B, (const float2 *)p.d_ring_lag, (float2 *)p.d_atot, p.n_far, p.n_modes, p.d_step, g);
    else
        hipLaunchKernelGGL(k_far<double>, dim3(nb), dim3(256), 0, p.stream, p.d_far_pk, p.d_far_cls, p.d_H, p.d_chi, p.d_dec, p.d_inj,
                           p.d_B, (const double2 *)p.d_ring_lag, (double2 *)p.d_atot, p.n_far, p.n_modes, p.d_step, g);
    return hipGetLastError();
}

hipError_t launch_fft_cols2(Plan &p)
{
    const Geom &g = p.g;
    const size_t sh = fft_lds_bytes(p);
    const unsigned T = (unsigned)(g.Q / 16);
    if (p.precision == WFP2D_PREC_MIXED)
        hipLaunchKernelGGL((k_fft_t2<float, 0>), dim3(g.R + 1), dim3(T), sh, p.stream, (const float2 *)p.d_atot, p.d_T2, p.d_col_off,
                           p.d_col_ny0, (const float2 *)p.d_corr, (const double2 *)p.d_tw, g);
    else
        hipLaunchKernelGGL((k_fft_t2<double, 0>), dim3(g.R + 1), dim3(T), sh, p.stream, (const double2 *)p.d_atot, p.d_T2, p.d_col_off,
                           p.d_col_ny0, (const double2 *)p.d_corr, (const double2 *)p.d_tw, g);
    return hipGetLastError();
}

hipError_t launch_fft_rows2(Plan &p)
{
    const Geom &g = p.g;
    const size_t sh = fft_lds_bytes(p);
    const unsigned T = (unsigned)(g.Q / 16);
    if (p.precision == WFP2D_PREC_MIXED) {
        transpose<float2>(p, p.d_T2, p.d_T2t, g.R + 1, g.Lpad);
        hipLaunchKernelGGL((k_fft_t2<float, 1>), dim3((g.Lpad + 1) / 2), dim3(T), sh, p.stream, (const float2 *)p.d_T2t, p.d_cgrid, nullptr,
                           nullptr, (const float2 *)p.d_corr, (const double2 *)p.d_tw, g);
    } else {
        transpose<double2>(p, p.d_T2, p.d_T2t, g.R + 1, g.Lpad);
        hipLaunchKernelGGL((k_fft_t2<double, 1>), dim3((g.Lpad + 1) / 2), dim3(T), sh, p.stream, (const double2 *)p.d_T2t, p.d_cgrid, nullptr,
                           nullptr, (const double2 *)p.d_corr, (const double2 *)p.d_tw, g);
    }
    return hipGetLastError();
}

template <class R, int WM>
static void interp_as(Plan &p)
{
    const Geom &g = p.g;
    const int ntile = g.ntx * g.ntx, S = kTile + g.w - 1;
    const unsigned nb = (unsigned)((ntile + 7) / 8 * 8);   // padded to a multiple of 8 (XCD remap)
    hipLaunchKernelGGL((k_interp<R, WM>), dim3(nb), dim3(kInterpThreads), (size_t)S * (S + 1) * sizeof(R), p.stream,
                       (const R *)p.d_cgrid, p.d_tgt_base, (const R *)p.d_tgt_wts, p.d_ttile_tgt, p.d_ttile_off, p.d_uh, g.w,
                       g.Lpad, g.ntx);
}

template <class R>
static void interp_typed(Plan &p)
{
    if (p.g.w <= 8) interp_as<R, 8>(p);
    else if (p.g.w <= 12) interp_as<R, 12>(p);
    else interp_as<R, 16>(p);
}

hipError_t launch_interp(Plan &p)
{
    if (p.precision == WFP2D_PREC_MIXED) interp_typed<float>(p);
    else interp_typed<double>(p);
    return hipGetLastError();
}

static LocalArgs local_args(const Plan &p)
{
    LocalArgs A;
    A.txy = p.d_tgt_xy;
    A.sxy = p.d_src_xy;
    A.scell_start = p.d_cell_start;
    A.tcell_start = p.d_tcell_start;
    A.subs = p.d_subs;
    A.cheb = p.d_cheb;
    A.creg = p.d_creg;
    A.cpow = p.d_cpow;
    A.pbase = p.d_panel_base;
    A.pl2n = p.d_panel_l2n;
    A.sig = p.d_sig;
    A.ul = p.d_ul;
    A.ncell = p.ncell;
    A.n_reg = p.n_reg;
    A.dy_base = p.dy_base;
    A.n_dy = p.n_dy;
    A.sc = p.local_sc;
    A.delta = p.delta;
    A.inv_dt = 1.0 / p.dt;
    A.two_over_ua = 2.0 / sqrt(p.dt);
    A.two_over_ua0 = 2.0 / sqrt(0.5 * p.dt);
    return A;
}

static PairLists pair_lists(const Plan &p)
{
    PairLists P;
    P.wrec = p.d_pair_wrec;
    P.wseg = p.d_pair_wseg;
    P.n_work = (int)p.pair_n_work;
    P.off = p.d_pair_off;
    P.doff = p.d_pair_doff;
    P.pw = p.d_pair_pw;
    P.dent = p.d_pair_dent;
    P.dw = p.d_pair_dw;
    P.dtg = p.d_pair_dtg;
    P.dsg = p.d_pair_dsg;
    P.ndy = p.pair_ndy;
    P.desc = (const LpDesc *)p.d_pc_desc;
    P.ioff = p.d_pc_ioff;
    return P;
}

hipError_t launch_pairs_build(Plan &p, bool fill, int64_t *cnt, int64_t *dcnt)
{
    const LocalArgs A = local_args(p);
    PairLists P = pair_lists(p);
    PairBuild B;
    B.cnt = cnt;
    B.dcnt = dcnt;
    B.pw = p.d_pair_pw;
    B.dent = p.d_pair_dent;
    B.dw = p.d_pair_dw;
    B.dtg = p.d_pair_dtg;
    B.dsg = p.d_pair_dsg;
    B.ndy = p.pair_ndy;
    B.psi_src = pc_psi_src(p.pc_rb, p.n_reg, p.local_terms);
    B.dterms = pc_panel_stride(p.pc_rb, p.local_terms);
    B.fill = fill ? 1 : 0;
    B.nlev = p.g.nlev;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(p.pair_n_work, 4096));
    if (fill) hipLaunchKernelGGL(k_pairs_pad, dim3(4096), dim3(256), 0, p.stream, p.d_pair_pw, p.pair_nword);
    hipLaunchKernelGGL(k_pairs_build, dim3(grid), dim3(256), 0, p.stream, A, P, B, p.dt, (int)p.W);
    return hipGetLastError();
}

static hipError_t launch_local_dyadic(Plan &p, const LocalArgs &A)
{
    if (p.pair_ndy == 0) return hipGetLastError();
    const unsigned grid = (unsigned)std::min<int64_t>((p.pair_ndy + 255) / 256, (int64_t)p.n_cu * 8);
    hipLaunchKernelGGL(k_local_dyadic, dim3(grid), dim3(256), 0, p.stream, A, pair_lists(p), p.d_step, p.g);
    return hipGetLastError();
}

hipError_t launch_local(Plan &p)
{
    const LocalArgs A = local_args(p);
    if (p.local_pairs) {
        const int rb = p.pc_rb, nprod = p.pc_nprod;
        const unsigned grid = (unsigned)p.pc_grid;
        const size_t lds = (size_t)2 * kFastSrc * pc_psi_src(rb, p.n_reg, p.local_terms) * sizeof(double) +
                           (rb == 4 ? (size_t)pc_ctab_doubles(p.local_terms, (p.g.nlev + 3) / 4) * sizeof(double) : 0);
        const PairLists P = pair_lists(p);
#define WFP2D_LAUNCH_PC(NLV, NTV, RBV) \
    hipLaunchKernelGGL((k_local_pc<NLV, NTV, RBV>), dim3(grid), dim3(1024), lds, p.stream, A, P, p.d_step, p.g, nprod)
#define WFP2D_LAUNCH_PC_NL(NTV, RBV) \
    do { if (p.g.nlev == 35) WFP2D_LAUNCH_PC(35, NTV, RBV); else WFP2D_LAUNCH_PC(43, NTV, RBV); } while (0)
        if (rb == 4 && p.local_terms == 16) WFP2D_LAUNCH_PC(35, 16, 4);
        else if (rb == 4 && p.local_terms == 14) WFP2D_LAUNCH_PC(35, 14, 4);
        else if (rb == 4) WFP2D_LAUNCH_PC(35, 12, 4);
        else switch (p.local_terms) {
        case 12: WFP2D_LAUNCH_PC_NL(12, 2); break;
        case 14: WFP2D_LAUNCH_PC_NL(14, 2); break;
        case 16: WFP2D_LAUNCH_PC_NL(16, 2); break;
        default:
            if (rb == 2) WFP2D_LAUNCH_PC_NL(20, 2);
            else WFP2D_LAUNCH_PC_NL(20, 3);
            break;
        }
#undef WFP2D_LAUNCH_PC_NL
#undef WFP2D_LAUNCH_PC
        hipError_t e = hipGetLastError();
        return e != hipSuccess ? e : launch_local_dyadic(p, A);
    }
    if (p.local_fast) {
        const int nrow = p.n_reg * kChebDeg;
        const unsigned threads = (unsigned)((nrow + 63) / 64 * 64);
        const int cells = p.ncell * p.ncell;
        const unsigned grid = (unsigned)std::min(cells, 2 * 256);
        const size_t lds = (size_t)kFastSrc * (p.n_reg * (kChebDeg + 1) + 1) * sizeof(double) +
                           (size_t)(threads / 64) * kFastRing * 12;
        if (p.g.nlev == 35)
            hipLaunchKernelGGL(k_local_fast<35>, dim3(grid), dim3(threads), lds, p.stream, A, p.d_step, p.g);
        else
            hipLaunchKernelGGL(k_local_fast<43>, dim3(grid), dim3(threads), lds, p.stream, A, p.d_step, p.g);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_local, dim3((unsigned)std::min<int64_t>((int64_t)p.ncell * p.ncell, 65536)), dim3(kLocalThreads), 0,
                       p.stream, A, p.d_step, p.g);
    return hipGetLastError();
}

hipError_t launch_hankel(Plan &p, const double *kappa, int64_t nk, const double *r, int nr, const double *E, int L, double *H)
{
    if (nk == 0) return hipSuccess;
    const dim3 grid((unsigned)((nk + kHkC - 1) / kHkC), (unsigned)((L + kHkL - 1) / kHkL));
    hipLaunchKernelGGL(k_hankel, grid, dim3(256), 0, p.stream, kappa, nk, r, nr, E, L, H);
    return hipGetLastError();
}

hipError_t launch_zero_f64(Plan &p, double *ptr, int64_t n)
{
    hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)std::min<int64_t>(std::max<int64_t>(nblk(n, 256), 1), 65536)), dim3(256), 0,
                       p.stream, ptr, n);
    return hipGetLastError();
}

hipError_t launch_combine(Plan &p, double *u_out)
{
    hipLaunchKernelGGL(k_combine, dim3(nblk(p.Nx, 256)), dim3(256), 0, p.stream, p.d_uh, p.d_ul, p.d_tgt_rank, u_out, p.Nx, p.d_step,
                       p.lookahead);
    return hipGetLastError();
}

hipError_t launch_combine_dot(Plan &p, const double *wts, double *acc)
{
    hipLaunchKernelGGL(k_combine_dot, dim3(nblk(p.Nx, 256)), dim3(256), 0, p.stream, p.d_uh, p.d_ul, p.d_tgt_rank, wts, acc,
                       p.Nx, p.d_step, p.lookahead);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed workspace for callers that cannot allocate (wfp2d_evaluate_noalloc).
// In host code the array's name is only a stand-in: kernels get the address
// returned by hipGetSymbolAddress, taken once per device with that device
// current (each device holds its own copy of the array).
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(int device, void **out)
{
    static std::mutex mu;
    static std::map<int, void *> addr;
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(device);
    if (it != addr.end()) {
        *out = it->second;
        return hipSuccess;
    }
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = ptr;
    *out = ptr;
    return hipSuccess;
}

}  // namespace wfp2d
