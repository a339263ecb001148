"""The type-1 line transform kernel, compiled for the host and checked against direct sums (CPU).

`k_fft_t1` (eq. sighat on the fine grid: one workgroup per line, P branch transforms of
length Q, radix-16 passes with a radix-2, 4 or 8 tail) is built from the kernels file as plain
C++; one host thread stands in for each of a workgroup's Q/16 lanes and a barrier for
__syncthreads.  Its output for line l is compared with the definition
    out[l][n + R] = corr[n + R] sum_{m < Lpad} x_l[m] e^{+2 pi i n m/nf},  n in [-R, R],
evaluated directly, over FP32 (decimation in time over the branches, first pass pruned to
the NZ nonzero values per lane) and FP64 (decimation in frequency) lines, every tail radix,
P = 1, 2, 3, and both output modes (all modes, or the disk nx^2 + n^2 <= Rd2 only, which is
also checked to leave the rest unwritten).  Nothing here runs on a GPU or calls the oracle.
"""
import shutil
import subprocess

import pytest

from kernel_source import HOST_PRELUDE, definition, internal_source, kernels_source, struct

NAMES = ["cmul", "cadd", "csub", "cconj", "from_d", "lpad", "tw_d", "cmul_d", "twiddle_powers", "tw_stage", "mul_si",
         "dft2", "dft4", "rot16", "dft8", "dft4_z", "dft16_nb", "dft16", "fidx", "fstr", "tail_pass", "fft_line",
         "out_mode", "ilog2", "k_fft_t1"]

DRIVER = r"""
template <class R> struct cplx;
template <> struct cplx<float> { using T = float2; };
template <> struct cplx<double> { using T = double2; };
@BLOCKS@

// one workgroup per listed line, its lanes on host threads
template <class R, int MODE, int NZ>
void run_lines(const Geom &g, const typename cplx<R>::T *in, typename cplx<R>::T *out, const typename cplx<R>::T *corr,
               const double2 *tw, const std::vector<int> &lines)
{
    const int T = g.Q / 16;
    blockDim.x = T;
    for (int line : lines) {
        blockIdx.x = line;
        std::barrier<> bar(T);
        host_group = &bar;
        std::vector<std::thread> th;
        for (int t = 0; t < T; ++t)
            th.emplace_back([&, t] { threadIdx.x = t; k_fft_t1<R, MODE, NZ>(in, out, corr, tw, g); });
        for (auto &x : th) x.join();
    }
}

template <class R, int MODE, int NZ>
void check(int P, int Q, int Lpad, int R_, double Rd2)
{
    using C = typename cplx<R>::T;
    Geom g{};
    g.P = P; g.Q = Q; g.nf = P * Q; g.Lpad = Lpad; g.R = R_; g.N = 2 * R_ + 1; g.Rd2 = Rd2;
    const int nlin = MODE == 0 ? Lpad : g.N;          // rows of the band, or columns of the kept modes
    std::vector<int> lines = {0, nlin / 3, nlin / 2, nlin - 1};
    if (MODE == 1) lines = {0, R_ / 3, R_, g.N - 1 - R_ / 4};
    std::mt19937 rng(P * 1000 + Q + MODE);
    std::normal_distribution<double> nd;
    std::vector<C> in((size_t)nlin * Lpad), corr(g.N), out((size_t)nlin * g.N, C{NAN, NAN});
    for (auto &v : in) v = C{(R)nd(rng), (R)nd(rng)};
    for (auto &v : corr) v = C{(R)nd(rng), (R)nd(rng)};
    std::vector<double2> tw(g.nf);
    for (int j = 0; j < g.nf; ++j) tw[j] = double2{std::cos(2 * M_PI * j / g.nf), std::sin(2 * M_PI * j / g.nf)};
    run_lines<R, MODE, NZ>(g, in.data(), out.data(), corr.data(), tw.data(), lines);
    std::vector<std::complex<long double>> e(g.nf);
    for (int j = 0; j < g.nf; ++j) {
        const long double a = 2.0L * 3.14159265358979323846264338327950288L * j / g.nf;
        e[j] = std::complex<long double>(std::cos(a), std::sin(a));
    }
    double err = 0, big = 0;
    long bad_written = 0, bad_skipped = 0;
    for (int line : lines) {
        const int nx = line - R_;
        for (int n = -R_; n <= R_; ++n) {
            const C got = out[(size_t)line * g.N + n + R_];
            const bool want = !(MODE == 1 && (double)(nx * nx + n * n) > Rd2);
            if (!want) { bad_written += !std::isnan(got.x); continue; }
            if (std::isnan(got.x)) { ++bad_skipped; continue; }
            std::complex<long double> s = 0;
            const long nn = ((long)n % g.nf + g.nf) % g.nf;
            for (int m = 0; m < Lpad; ++m) {
                const C x = in[(size_t)line * Lpad + m];
                s += std::complex<long double>(x.x, x.y) * e[(nn * m) % g.nf];
            }
            s *= std::complex<long double>(corr[n + R_].x, corr[n + R_].y);
            err = std::fmax(err, (double)std::abs(s - std::complex<long double>(got.x, got.y)));
            big = std::fmax(big, (double)std::abs(s));
        }
    }
    printf("%s %d %d %d %d %d %.3e %ld %ld\n", sizeof(R) == 4 ? "f32" : "f64", MODE, NZ, P, Q, Lpad, err / big, bad_written,
           bad_skipped);
}

int main()
{
    // FP32: the launcher's NZ = ceil(Lpad / (P Q/16)) rounded up to 5, 6, 8 or 16
    check<float, 0, 5>(3, 256, 240, 190, 0);      // two radix-16 passes
    check<float, 0, 6>(3, 256, 256, 190, 0);
    check<float, 0, 16>(3, 256, 240, 190, 0);     // unpruned form of the same line
    check<float, 1, 5>(3, 512, 480, 380, 300.0 * 300.0);   // radix-2 tail, disk output
    check<float, 0, 8>(2, 1024, 1000, 500, 0);    // radix-4 tail
    check<float, 1, 16>(1, 2048, 2000, 500, 420.0 * 420.0);  // radix-8 tail
    // FP64: decimation in frequency
    check<double, 0, 16>(3, 256, 240, 190, 0);
    check<double, 1, 16>(2, 512, 500, 250, 200.0 * 200.0);
    check<double, 0, 16>(1, 2048, 2000, 500, 0);
}
"""


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    src = kernels_source()
    blocks = struct(internal_source(), "Geom") + "\n" + "\n".join(definition(src, n) for n in NAMES)
    d = tmp_path_factory.mktemp("fftlines")
    cpp, exe = d / "lines.cpp", d / "lines"
    cpp.write_text(HOST_PRELUDE + DRIVER.replace("@BLOCKS@", blocks))
    subprocess.run([gxx, "-O2", "-std=c++20", "-pthread", "-Wno-unknown-pragmas", "-ffp-contract=off", str(cpp),
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=240).stdout
    rows = []
    for line in out.strip().splitlines():
        f = line.split()
        rows.append({"prec": f[0], "mode": int(f[1]), "nz": int(f[2]), "P": int(f[3]), "Q": int(f[4]), "Lpad": int(f[5]),
                     "err": float(f[6]), "bad_written": int(f[7]), "bad_skipped": int(f[8])})
    assert len(rows) == 9, out
    return rows


def test_fp32_lines_match_the_direct_sum(results):
    for r in results:
        if r["prec"] == "f32":
            assert r["err"] < 5e-7, r


def test_fp64_lines_match_the_direct_sum(results):
    for r in results:
        if r["prec"] == "f64":
            assert r["err"] < 1e-14, r


def test_every_kept_mode_written_and_no_other(results):
    for r in results:
        assert r["bad_written"] == 0 and r["bad_skipped"] == 0, r
