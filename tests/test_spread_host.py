"""The spreading kernels, compiled for the host (the matrix-core one with emulated MFMAs) (CPU).

`k_spread_mfma` sums, on each 16 x 16 tile of the fine grid, the tensor-product kernels of the
tile's sources (eq. sighat's spreading) as a contraction over them.  Here it is built from the
kernels file as plain C++ with 64 host threads as the wave's lanes; the 16x16x4 MFMA builtins are
replaced by a host function written from the documented operand layout (lane l supplies
A[l % 16][l / 16] and B[l / 16][l % 16]; it receives D[4 (l / 16) + v][l % 16] in FP32 and
D[l / 16 + 4 v][l % 16] in FP64).  The grid must equal the direct sum
    G[y][x] = sum_j (sigma_j(t_m) + i sigma_j(t_{m-LA})) wx_j[x - bx_j] wy_j[y - by_j]
over the sources whose w x w support holds (x, y), with the tile source lists built as the host
builds them, for tiles with no source, several 64-source chunks (a last chunk not a multiple of
4), supports at the band's edges, FP32 and FP64, and weight rows staged by 16-byte loads (2w a
multiple of 16 bytes) or one by one.  This checks the kernel's tiling, staging, chunk loop and
stores against the layout; that the hardware has this layout is checked by the GPU parity tests
(`test_stage_type1_against_direct_sum` on tile code 6).  The vector-unit kernel `k_spread` of tile
codes 1..5 (8x8 to 32x32 tiles, each lane accumulating its own points) is checked the same way.
Nothing here runs on a GPU or calls the oracle.
"""
import shutil
import subprocess

import pytest

from kernel_source import HOST_PRELUDE, between, definition, host_shared, internal_source, kernels_source, struct

DRIVER = r"""
using std::max;
using std::min;
struct int2 { int x, y; };
inline int2 make_int2(int x, int y) { return int2{x, y}; }
struct alignas(16) float4 { float x, y, z, w; };
typedef float mfma_f4 __attribute__((vector_size(16)));
typedef double mfma_d4 __attribute__((vector_size(32)));
alignas(64) unsigned char spread_lds[1 << 16];
template <class R> struct cplx;
template <> struct cplx<float> { using T = float2; };
template <> struct cplx<double> { using T = double2; };

// one 16x16x4 MFMA of the wave: every lane publishes its operands, then forms its outputs
template <class V, class E, bool F32>
V host_mfma(E a, E b, V c)
{
    static E sa[64], sb[64];
    const int l = threadIdx.x;
    sa[l] = a;
    sb[l] = b;
    __syncthreads();
    V d = c;
    for (int v = 0; v < 4; ++v) {
        const int row = F32 ? 4 * (l >> 4) + v : (l >> 4) + 4 * v, col = l & 15;
        E s = d[v];
        for (int k = 0; k < 4; ++k) s += sa[16 * k + row] * sb[16 * k + col];
        d[v] = s;
    }
    __syncthreads();
    return d;
}
#define __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, x, y, z) host_mfma<mfma_f4, float, true>(a, b, c)
#define __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, x, y, z) host_mfma<mfma_d4, double, false>(a, b, c)
@BLOCKS@

template <class R, int TX, int TY, bool MF>
void check(int Lpad, int w, int M, unsigned seed)
{
    using C = typename cplx<R>::T;
    Geom g{};
    g.M = M; g.LA = 3; g.lookahead = 2; g.sig_depth = 7;
    const int64_t step = 12;                                 // m = 10, lag level 7
    std::mt19937 rng(seed);
    std::normal_distribution<double> nd;
    std::vector<double> sig((size_t)g.sig_depth * M);
    for (auto &v : sig) v = nd(rng);
    std::vector<int2> base(M);
    std::vector<R> wts((size_t)M * 2 * w);
    for (auto &v : wts) v = (R)nd(rng);
    for (int j = 0; j < M; ++j) {
        // a cluster in the first tile (several chunks), the rest spread over the band, some at its edges
        const int hi = Lpad - w;
        if (j < M / 2) base[j] = make_int2((int)(rng() % 12), (int)(rng() % 12));
        else if (j % 17 == 0) base[j] = make_int2(hi, (int)(rng() % (hi + 1)));
        else base[j] = make_int2((int)(rng() % (hi / 2 + 1)), (int)(rng() % (hi / 2 + 1)));
    }
    // per-tile source lists, as the plan builds them: each tile the support meets
    const int ntx = (Lpad + TX - 1) / TX, nty = (Lpad + TY - 1) / TY, ntile = ntx * nty;
    std::vector<std::vector<int32_t>> lists(ntile);
    for (int j = 0; j < M; ++j)
        for (int y = base[j].y / TY; y <= (base[j].y + w - 1) / TY; ++y)
            for (int x = base[j].x / TX; x <= (base[j].x + w - 1) / TX; ++x) lists[y * ntx + x].push_back(j);
    std::vector<int32_t> off(ntile + 1, 0), src;
    size_t most = 0;
    for (int t = 0; t < ntile; ++t) {
        for (int j : lists[t]) src.push_back(j);
        off[t + 1] = (int32_t)src.size();
        most = std::max(most, lists[t].size());
    }
    std::vector<C> grid((size_t)Lpad * Lpad, C{(R)NAN, (R)NAN});
    const unsigned nb = (unsigned)(((ntile + 7) >> 3) << 3);
    blockDim.x = 64;
    for (unsigned blk = 0; blk < nb; ++blk) {
        blockIdx.x = blk;
        std::barrier<> bar(64);
        host_group = &bar;
        std::vector<std::thread> th;
        for (int t = 0; t < 64; ++t)
            th.emplace_back([&, t] {
                threadIdx.x = t;
                if constexpr (MF)
                    k_spread_mfma<R>(sig.data(), &step, base.data(), wts.data(), off.data(), src.data(), grid.data(), w, ntx,
                                     ntile, Lpad, g);
                else
                    k_spread<R, TX, TY>(sig.data(), &step, base.data(), wts.data(), off.data(), src.data(), grid.data(), w,
                                        ntx, ntile, Lpad, g);
            });
        for (auto &x : th) x.join();
    }
    const int64_t m = step - g.lookahead;
    const double *cur = sig.data() + (m % g.sig_depth) * M, *lag = sig.data() + ((m - g.LA) % g.sig_depth) * M;
    std::vector<long double> re((size_t)Lpad * Lpad, 0), im((size_t)Lpad * Lpad, 0);
    for (int j = 0; j < M; ++j)
        for (int b = 0; b < w; ++b)
            for (int a = 0; a < w; ++a) {
                const size_t q = (size_t)(base[j].y + b) * Lpad + base[j].x + a;
                const long double k = (long double)wts[(size_t)j * 2 * w + a] * (long double)wts[(size_t)j * 2 * w + w + b];
                re[q] += (long double)(R)cur[j] * k;
                im[q] += (long double)(R)lag[j] * k;
            }
    double err = 0, big = 0;
    long unwritten = 0;
    for (size_t q = 0; q < grid.size(); ++q) {
        if (std::isnan(grid[q].x) || std::isnan(grid[q].y)) { ++unwritten; continue; }
        err = std::fmax(err, (double)std::fabs(re[q] - grid[q].x));
        err = std::fmax(err, (double)std::fabs(im[q] - grid[q].y));
        big = std::fmax(big, (double)std::fmax(std::fabs(re[q]), std::fabs(im[q])));
    }
    printf("%s %d %zu %.3e %ld %s\n", sizeof(R) == 4 ? "f32" : "f64", w, most, err / big, unwritten, MF ? "mfma" : "vector");
}

int main()
{
    check<float, 16, 16, true>(64, 8, 400, 1);      // 16-byte staging (2w = 16 floats)
    check<float, 16, 16, true>(64, 7, 400, 2);      // one-by-one staging
    check<double, 16, 16, true>(64, 12, 300, 3);    // 16-byte staging (2w = 24 doubles)
    check<double, 16, 16, true>(48, 5, 300, 4);     // one-by-one staging, band not a multiple of 32
    // the vector-unit tiles (codes 1..5)
    check<float, 8, 8, false>(64, 8, 400, 5);
    check<float, 16, 8, false>(64, 7, 400, 6);
    check<double, 16, 16, false>(64, 12, 300, 7);
    check<float, 32, 16, false>(64, 8, 400, 8);
    check<double, 32, 32, false>(48, 5, 300, 9);
}
"""


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    src = kernels_source()
    acc = between(src, "template <class R> struct mfma_acc;", "__global__ __launch_bounds__(64) void k_spread_mfma(")
    acc = acc.rstrip()
    acc = acc[:acc.rindex("\n")] if acc.endswith("template <class R>") else acc   # the kernel's own header
    blocks = "\n".join([struct(internal_source(), "Geom"), definition(src, "pmod"), host_shared(definition(src, "k_spread")),
                        acc, host_shared(definition(src, "k_spread_mfma"))])
    d = tmp_path_factory.mktemp("spreadmfma")
    cpp, exe = d / "spread.cpp", d / "spread"
    cpp.write_text(HOST_PRELUDE + DRIVER.replace("@BLOCKS@", blocks))
    subprocess.run([gxx, "-O2", "-std=c++20", "-pthread", "-Wno-unknown-pragmas", "-Wno-psabi", "-ffp-contract=off", str(cpp),
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=240).stdout
    rows = [line.split() for line in out.strip().splitlines()]
    assert len(rows) == 9, out
    return [{"prec": f[0], "w": int(f[1]), "most": int(f[2]), "err": float(f[3]), "unwritten": int(f[4]), "form": f[5]}
            for f in rows]


def test_spread_grid_matches_the_direct_sum(results):
    for r in results:
        assert r["most"] > 64 and r["err"] < (1e-6 if r["prec"] == "f32" else 1e-14), r


def test_every_grid_point_written(results):
    for r in results:
        assert r["unwritten"] == 0, r
