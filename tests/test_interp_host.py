"""The interpolation kernel, compiled for the host and checked against its definition (CPU).

`k_interp` (eq. uhtraptrunc's evaluation on the fine grid: u_h(x_i) = sum over the w x w
stencil of grid(origin_i + (a, b)) wx_i[a] wy_i[b]) is built from the kernels file as plain
C++; 128 host threads stand in for a workgroup's lanes and a barrier for __syncthreads.  Tiles
hold from no target to several hundred (so the FP32 form's prefetch of a lane's next target is
taken), origins reach the band's last columns and rows (halo beyond the band read as zero), and
the FP32 (w = 8 and 16) and FP64 (w = 12) grids are used.  Every target must be written once, to
its caller-order slot, within FP64 rounding of the sum evaluated directly in long double from
the same grid values and weights.  Nothing here runs on a GPU or calls the oracle.
"""
import shutil
import subprocess

import pytest

from kernel_source import HOST_PRELUDE, definition, kernels_source

DRIVER = r"""
struct int2 { int x, y; };
inline int2 make_int2(int x, int y) { return int2{x, y}; }
constexpr int kTile = 32;
alignas(64) unsigned char interp_lds[1 << 17];
@BLOCKS@

template <class R, int WM>
void check(int Lpad, int w, unsigned seed)
{
    const int ntx = Lpad / kTile, ntile = ntx * ntx;
    std::mt19937 rng(seed);
    std::normal_distribution<double> nd;
    std::vector<R> grid((size_t)Lpad * Lpad);
    for (auto &v : grid) v = (R)nd(rng);
    // targets per tile: tile 0 crowded (300), the last tile's band edge, some tiles empty
    std::vector<std::vector<int2>> per(ntile);
    std::uniform_int_distribution<int> u32(0, kTile - 1);
    for (int t = 0; t < ntile; ++t) {
        const int n = t == 0 ? 300 : (t % 3 == 1 ? 0 : 1 + (int)(rng() % 140));
        const int ox = (t % ntx) * kTile, oy = (t / ntx) * kTile;
        for (int k = 0; k < n; ++k) per[t].push_back(make_int2(ox + u32(rng), oy + u32(rng)));
        if (t == ntile - 1) per[t].push_back(make_int2(Lpad - 1, Lpad - 1));
    }
    std::vector<int32_t> toff(ntile + 1, 0);
    std::vector<int2> base;
    for (int t = 0; t < ntile; ++t) {
        for (auto b : per[t]) base.push_back(b);
        toff[t + 1] = (int32_t)base.size();
    }
    const int nt = (int)base.size();
    std::vector<int32_t> tlist(nt);
    for (int e = 0; e < nt; ++e) tlist[e] = (int32_t)((e * 7919LL) % nt);   // a permutation: nt is not a multiple of 7919
    std::vector<R> wts((size_t)nt * 2 * w);
    for (auto &v : wts) v = (R)nd(rng);
    std::vector<double> uh(nt, NAN);
    const unsigned nb = (unsigned)((ntile + 7) / 8 * 8);
    blockDim.x = kInterpThreads;
    for (unsigned blk = 0; blk < nb; ++blk) {
        blockIdx.x = blk;
        std::barrier<> bar(kInterpThreads);
        host_group = &bar;
        std::vector<std::thread> th;
        for (int t = 0; t < kInterpThreads; ++t)
            th.emplace_back([&, t] {
                threadIdx.x = t;
                k_interp<R, WM>(grid.data(), base.data(), wts.data(), tlist.data(), toff.data(), uh.data(), w, Lpad, ntx);
            });
        for (auto &x : th) x.join();
    }
    double err = 0, big = 0;
    long unwritten = 0;
    for (int e = 0; e < nt; ++e) {
        long double s = 0;
        for (int b = 0; b < w; ++b)
            for (int a = 0; a < w; ++a) {
                const int gx = base[e].x + a, gy = base[e].y + b;
                const long double gv = (gx < Lpad && gy < Lpad) ? (long double)grid[(size_t)gy * Lpad + gx] : 0.0L;
                s += gv * (long double)wts[(size_t)e * 2 * w + a] * (long double)wts[(size_t)e * 2 * w + w + b];
            }
        const double got = uh[tlist[e]];
        if (std::isnan(got)) { ++unwritten; continue; }
        err = std::fmax(err, std::fabs((double)(s - (long double)got)));
        big = std::fmax(big, std::fabs((double)s));
    }
    printf("%s %d %d %.3e %ld\n", sizeof(R) == 4 ? "f32" : "f64", w, nt, err / big, unwritten);
}

int main()
{
    check<float, 8>(96, 8, 1);
    check<float, 16>(96, 16, 2);
    check<double, 12>(128, 12, 3);
}
"""


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    src = kernels_source()
    kthreads = next(l for l in src.splitlines() if l.startswith("constexpr int kInterpThreads"))
    blocks = kthreads + "\n" + definition(src, "k_interp")
    d = tmp_path_factory.mktemp("interp")
    cpp, exe = d / "interp.cpp", d / "interp"
    cpp.write_text(HOST_PRELUDE + DRIVER.replace("@BLOCKS@", blocks))
    subprocess.run([gxx, "-O2", "-std=c++20", "-pthread", "-Wno-unknown-pragmas", "-ffp-contract=off", str(cpp),
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=240).stdout
    rows = [line.split() for line in out.strip().splitlines()]
    assert len(rows) == 3, out
    return [{"prec": f[0], "w": int(f[1]), "n": int(f[2]), "err": float(f[3]), "unwritten": int(f[4])} for f in rows]


def test_interpolation_matches_the_stencil_sum(results):
    for r in results:
        assert r["n"] > 300 and r["err"] < 1e-14, r


def test_every_target_written(results):
    for r in results:
        assert r["unwritten"] == 0, r
