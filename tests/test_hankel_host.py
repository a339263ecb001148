"""The device-side Hankel contraction, compiled for the host and checked against its definition (CPU).

`k_hankel` forms the coefficients of eq. H for every wavenumber class from the quadrature of the
plan's set-up, H[c][l] = sum_g J0(kappa_c r_g) E[l][g], in tiles of 16 classes x 64 terms with the
nodes staged in chunks of 64.  Here it is built from the kernels file as plain C++ (256 host
threads per workgroup, a barrier for __syncthreads) and compared with that double sum evaluated
directly, over class, term and node counts that leave partial tiles in every dimension.  The
Bessel function is the host's j0 on both sides; the device's own j0 against the host evaluation
of eq. H is checked on the GPU (test_gpu_precompute.py).  Nothing here runs on a GPU or calls the
oracle.
"""
import shutil
import subprocess

import pytest

from kernel_source import HOST_PRELUDE, definition, host_shared, kernels_source

DRIVER = r"""
@BLOCKS@

void check(int nk, int nr, int L)
{
    std::mt19937 rng(nk * 7 + nr);
    std::uniform_real_distribution<double> uk(0.0, 80.0), ur(0.0, 1.0);
    std::normal_distribution<double> nd;
    std::vector<double> kappa(nk), r(nr), E((size_t)L * nr), H((size_t)nk * L, NAN);
    for (auto &v : kappa) v = uk(rng);
    for (auto &v : r) v = ur(rng);
    for (auto &v : E) v = nd(rng);
    blockDim.x = 256;
    for (unsigned by = 0; by < (unsigned)((L + kHkL - 1) / kHkL); ++by)
        for (unsigned bx = 0; bx < (unsigned)((nk + kHkC - 1) / kHkC); ++bx) {
            blockIdx.x = bx;
            blockIdx.y = by;
            std::barrier<> bar(256);
            host_group = &bar;
            std::vector<std::thread> th;
            for (int t = 0; t < 256; ++t)
                th.emplace_back([&, t] { threadIdx.x = t; k_hankel(kappa.data(), nk, r.data(), nr, E.data(), L, H.data()); });
            for (auto &x : th) x.join();
        }
    double err = 0, big = 0;
    long unwritten = 0;
    for (int c = 0; c < nk; ++c)
        for (int l = 0; l < L; ++l) {
            long double s = 0;
            for (int g = 0; g < nr; ++g) s += (long double)j0(kappa[c] * r[g]) * E[(size_t)l * nr + g];
            const double got = H[(size_t)c * L + l];
            if (std::isnan(got)) { ++unwritten; continue; }
            err = std::fmax(err, std::fabs((double)(s - got)));
            big = std::fmax(big, std::fabs((double)s));
        }
    printf("%d %d %d %.3e %ld\n", nk, nr, L, err / big, unwritten);
}

int main()
{
    check(37, 200, 640);    // partial class tile and node chunk
    check(16, 64, 100);     // one class tile, one node chunk, a partial term tile
}
"""


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    src = kernels_source()
    consts = next(l for l in src.splitlines() if l.startswith("constexpr int kHkC"))
    blocks = consts + "\n" + host_shared(definition(src, "k_hankel"))
    d = tmp_path_factory.mktemp("hankel")
    cpp, exe = d / "hankel.cpp", d / "hankel"
    cpp.write_text(HOST_PRELUDE + DRIVER.replace("@BLOCKS@", blocks))
    subprocess.run([gxx, "-O2", "-std=c++20", "-pthread", "-Wno-unknown-pragmas", "-ffp-contract=off", str(cpp), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=240).stdout
    rows = [line.split() for line in out.strip().splitlines()]
    assert len(rows) == 2, out
    return [{"nk": int(f[0]), "nr": int(f[1]), "L": int(f[2]), "err": float(f[3]), "unwritten": int(f[4])} for f in rows]


def test_hankel_tiles_match_the_double_sum(results):
    for r in results:
        assert r["err"] < 1e-14 and r["unwritten"] == 0, r
