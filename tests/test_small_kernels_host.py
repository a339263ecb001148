"""The step's small kernels, compiled for the host and checked against their definitions (CPU).

* `k_ingest` / `k_ingest_slot` write sigma_j(t_n), in the plan's source order (caller index perm[j]),
  into ring slot n mod depth (or the given slot) and leave every other slot alone; with the
  non-finite check on, a NaN or Inf sample is taken as 0 and counted once; with it off, it passes
  through unchanged.
* `k_combine` returns u = u_h + u_l in caller order (target i from the plan's slot rank[i]), and 0
  while the reported step is not yet positive (zero initial data).
* `k_transpose` writes out[c][r] = in[r][c] for sizes that are not multiples of its 32 x 32 tile.
* `k_local_dyadic` adds, for each pair with r < dt/2 (Sec. 6, eq. ul_GL on the dyadic panels), its
  weighted levels sum_d w_d(q) sigma_s(t_{m - lev_min - d}) to u_l at its target; checked with
  several pairs per target, a grid smaller than the pair count (the grid-stride loop) and the
  sigma ring wrapping.
Each is built from the kernels file as plain C++ (host threads as lanes, a barrier for the
transpose's __syncthreads).  Nothing here runs on a GPU or calls the oracle.
"""
import shutil
import subprocess

import pytest

from kernel_source import HOST_PRELUDE, definition, host_shared, internal_source, kernels_source, struct

DRIVER = r"""
#include <algorithm>
#include <atomic>
#include <numeric>
using std::isfinite;
inline unsigned long long atomicAdd(unsigned long long *p, unsigned long long v)
{
    return std::atomic_ref<unsigned long long>(*p).fetch_add(v);
}
inline double unsafeAtomicAdd(double *p, double v) { return std::atomic_ref<double>(*p).fetch_add(v); }
HostDim gridDim;
@BLOCKS@

template <class F> void grid1d(int64_t n, F f)
{
    blockDim.x = 256;
    for (unsigned b = 0; b < (unsigned)((n + 255) / 256); ++b) {
        blockIdx.x = b;
        for (int t = 0; t < 256; ++t) { threadIdx.x = t; f(); }
    }
}

int main()
{
    std::mt19937 rng(3);
    std::normal_distribution<double> nd;
    long bad = 0;
    // ingest
    const int64_t M = 1000, depth = 5, step = 17;
    std::vector<int32_t> perm(M);
    std::iota(perm.begin(), perm.end(), 0);
    std::shuffle(perm.begin(), perm.end(), rng);
    std::vector<double> in(M);
    for (auto &v : in) v = nd(rng);
    in[3] = NAN; in[500] = INFINITY; in[999] = -INFINITY;
    for (int check = 0; check < 2; ++check) {
        std::vector<double> sig((size_t)depth * M, -7.0);
        unsigned long long cnt = 0;
        grid1d(M, [&] { k_ingest(in.data(), perm.data(), sig.data(), M, &step, depth, check ? &cnt : nullptr); });
        for (int64_t s = 0; s < depth; ++s)
            for (int64_t j = 0; j < M; ++j) {
                const double v = sig[s * M + j], x = in[perm[j]];
                if (s != step % depth) bad += v != -7.0;
                else if (std::isfinite(x)) bad += v != x;
                else bad += check ? v != 0.0 : !(std::isnan(x) ? std::isnan(v) : v == x);
            }
        bad += check ? cnt != 3 : cnt != 0;
    }
    {
        std::vector<double> sig((size_t)depth * M, -7.0);
        unsigned long long cnt = 0;
        grid1d(M, [&] { k_ingest_slot(in.data(), perm.data(), sig.data(), M, 2, &cnt); });
        for (int64_t s = 0; s < depth; ++s)
            for (int64_t j = 0; j < M; ++j) {
                const double v = sig[s * M + j], x = in[perm[j]];
                bad += s != 2 ? v != -7.0 : v != (std::isfinite(x) ? x : 0.0);
            }
        bad += cnt != 3;
    }
    printf("ingest %ld\n", bad);
    // combine
    bad = 0;
    const int64_t Nx = 777;
    std::vector<int32_t> rank(Nx);
    std::iota(rank.begin(), rank.end(), 0);
    std::shuffle(rank.begin(), rank.end(), rng);
    std::vector<double> uh(Nx), ul(Nx), u(Nx);
    for (auto &v : uh) v = nd(rng);
    for (auto &v : ul) v = nd(rng);
    for (int64_t st : {5, 14}) {
        std::fill(u.begin(), u.end(), NAN);
        grid1d(Nx, [&] { k_combine(uh.data(), ul.data(), rank.data(), u.data(), Nx, &st, 9); });
        for (int64_t i = 0; i < Nx; ++i) bad += st - 9 < 1 ? u[i] != 0.0 : u[i] != uh[rank[i]] + ul[rank[i]];
    }
    printf("combine %ld\n", bad);
    // transpose
    bad = 0;
    for (auto rc : {std::pair<int, int>{70, 45}, std::pair<int, int>{32, 96}, std::pair<int, int>{1, 33}}) {
        const int rows = rc.first, cols = rc.second;
        std::vector<float2> a((size_t)rows * cols), o((size_t)rows * cols, float2{NAN, NAN});
        for (auto &v : a) v = float2{(float)nd(rng), (float)nd(rng)};
        blockDim.x = 256;
        for (unsigned by = 0; by < (unsigned)((rows + 31) / 32); ++by)
            for (unsigned bx = 0; bx < (unsigned)((cols + 31) / 32); ++bx) {
                blockIdx.x = bx;
                blockIdx.y = by;
                std::barrier<> bar(256);
                host_group = &bar;
                std::vector<std::thread> th;
                for (int t = 0; t < 256; ++t)
                    th.emplace_back([&, t] { threadIdx.x = t; k_transpose<float2>(a.data(), o.data(), rows, cols); });
                for (auto &x : th) x.join();
            }
        for (int r = 0; r < rows; ++r)
            for (int c = 0; c < cols; ++c) {
                const float2 x = a[(size_t)r * cols + c], y = o[(size_t)c * rows + r];
                bad += x.x != y.x || x.y != y.y;
            }
    }
    printf("transpose %ld\n", bad);
    // dyadic local pairs
    bad = 0;
    {
        Geom g{};
        g.M = 50; g.lookahead = 9; g.lev_min = 2; g.nlev = 27; g.sig_depth = 31;
        const int64_t ndy = 3000, Nt = 40, st = 100;
        std::vector<double> sig((size_t)g.sig_depth * g.M), dw((size_t)g.nlev * ndy), ul(Nt, 0.0);
        for (auto &v : sig) v = nd(rng);
        for (auto &v : dw) v = nd(rng);
        std::vector<int32_t> dtg(ndy), dsg(ndy);
        for (int64_t q = 0; q < ndy; ++q) { dtg[q] = (int32_t)(rng() % Nt); dsg[q] = (int32_t)(rng() % g.M); }
        std::sort(dtg.begin(), dtg.end());
        LocalArgs A{};
        A.sig = sig.data();
        A.ul = ul.data();
        PairLists P{};
        P.dw = dw.data(); P.dtg = dtg.data(); P.dsg = dsg.data(); P.ndy = ndy;
        gridDim.x = 4;
        blockDim.x = 256;
        for (unsigned b = 0; b < gridDim.x; ++b) {
            blockIdx.x = b;
            std::barrier<> bar(256);
            host_group = &bar;
            std::vector<std::thread> th;
            for (int t = 0; t < 256; ++t) th.emplace_back([&, t] { threadIdx.x = t; k_local_dyadic(A, P, &st, g); });
            for (auto &x : th) x.join();
        }
        std::vector<long double> ref(Nt, 0.0L);
        const int64_t m = st - g.lookahead;
        for (int64_t q = 0; q < ndy; ++q)
            for (int d = 0; d < g.nlev; ++d) {
                const int64_t lvl = m - g.lev_min - d, slot = ((lvl % g.sig_depth) + g.sig_depth) % g.sig_depth;
                ref[dtg[q]] += (long double)dw[(size_t)d * ndy + q] * sig[(size_t)slot * g.M + dsg[q]];
            }
        for (int t = 0; t < Nt; ++t) bad += std::fabs((double)ref[t] - ul[t]) > 1e-12 * (1.0 + std::fabs((double)ref[t]));
    }
    printf("dyadic %ld\n", bad);
}
"""


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    src = kernels_source()
    inl = internal_source()
    consts = "\n".join(l for l in inl.splitlines() if l.startswith("constexpr int kLocalMaxLevels"))
    blocks = "\n".join([definition(src, "pmod"), definition(src, "k_ingest"), definition(src, "k_ingest_slot"),
                        definition(src, "k_combine"), host_shared(definition(src, "k_transpose")), consts,
                        struct(inl, "Geom"), struct(inl, "SubPanel"), struct(src, "LocalArgs"), "struct LpDesc;",
                        struct(src, "PairLists"), definition(src, "sig_slot"), host_shared(definition(src, "k_local_dyadic"))])
    d = tmp_path_factory.mktemp("small")
    cpp, exe = d / "small.cpp", d / "small"
    cpp.write_text(HOST_PRELUDE + DRIVER.replace("@BLOCKS@", blocks))
    subprocess.run([gxx, "-O2", "-std=c++20", "-pthread", "-Wno-unknown-pragmas", str(cpp), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=120).stdout
    return {f[0]: int(f[1]) for f in (line.split() for line in out.strip().splitlines())}


@pytest.mark.parametrize("kernel", ["ingest", "combine", "transpose", "dyadic"])
def test_small_kernel_matches_its_definition(results, kernel):
    assert results[kernel] == 0, results
