"""The type-2 line transform kernel, compiled for the host and checked against direct sums (CPU).

`k_fft_t2` (eqs. uhtraptrunc, ufhApprox on the fine grid) is built from the kernels file as plain
C++, one host thread per lane and a barrier for __syncthreads, and compared with what it is
defined to compute:
  columns (mode 0): line n_x in [0, R] holds the packed half-disk coefficients c(n_y) for n_y in
    [ny0, ny0 + cnt); with X(n_y) = f c(n_y) conj(corr[n_x + R]) conj(corr[n_y + R]), f = 2 except
    f = 1 on n_x = 0, n_y <= 0, the output is T2[n_x][m] = sum X(n_y) e^{-2 pi i n_y m/nf}, m < Lpad;
  rows (mode 1): rows 2b and 2b + 1 of the real grid are Re sum_{k=0}^{R} H(k) e^{-2 pi i k m/nf}
    of their half spectra H (one complex transform serves both; an odd last row stands alone).
FP32 and FP64, P = 1, 2, 3, every tail radix.  Nothing here runs on a GPU or calls the oracle.
"""
import shutil
import subprocess

import pytest

from kernel_source import HOST_PRELUDE, definition, internal_source, kernels_source, struct

NAMES = ["cmul", "cadd", "csub", "cconj", "from_d", "lpad", "tw_d", "cmul_d", "twiddle_powers", "tw_stage", "mul_si",
         "dft2", "dft4", "rot16", "dft8", "dft4_z", "dft16_nb", "dft16", "fidx", "fstr", "tail_pass", "fft_line",
         "out_mode", "ilog2", "k_fft_t2"]

DRIVER = r"""
template <class R> struct cplx;
template <> struct cplx<float> { using T = float2; };
template <> struct cplx<double> { using T = double2; };
@BLOCKS@

using cld = std::complex<long double>;

template <class R, int MODE>
void check(int P, int Q, int Lpad, int R_)
{
    using C = typename cplx<R>::T;
    Geom g{};
    g.P = P; g.Q = Q; g.nf = P * Q; g.Lpad = Lpad; g.R = R_; g.N = 2 * R_ + 1;
    std::mt19937 rng(P * 100 + Q + MODE + Lpad);
    std::normal_distribution<double> nd;
    std::vector<C> corr(g.N);
    for (auto &v : corr) v = C{(R)nd(rng), (R)nd(rng)};
    std::vector<double2> tw(g.nf);
    for (int j = 0; j < g.nf; ++j) tw[j] = double2{std::cos(2 * M_PI * j / g.nf), std::sin(2 * M_PI * j / g.nf)};
    std::vector<cld> e(g.nf);
    for (int j = 0; j < g.nf; ++j) {
        const long double a = 2.0L * 3.14159265358979323846264338327950288L * j / g.nf;
        e[j] = cld(std::cos(a), -std::sin(a));         // e^{-2 pi i j/nf}
    }
    auto ex = [&](long k, int m) { return e[(((k * m) % g.nf) + g.nf) % g.nf]; };
    // the half disk: column n_x keeps |n_y| <= h(n_x), column 0 only n_y >= -h/2 (any range is allowed)
    std::vector<int32_t> off(R_ + 2, 0), ny0(R_ + 1);
    for (int nx = 0; nx <= R_; ++nx) {
        const int h = (int)std::floor(std::sqrt((double)R_ * R_ - (double)nx * nx));
        ny0[nx] = nx == 0 ? -h / 2 : -h;
        off[nx + 1] = off[nx] + (h - ny0[nx] + 1);
    }
    std::vector<int> lines;
    size_t nin, nout;
    if (MODE == 0) {
        lines = {0, 1, R_ / 2, R_};
        nin = (size_t)off[R_ + 1];
        nout = (size_t)(R_ + 1) * Lpad * 2;                 // complex T2[R + 1][Lpad] as reals
    } else {
        lines = {0, 2 * ((Lpad / 2) / 3), 2 * ((Lpad - 1) / 2)};   // block b transforms rows 2b, 2b + 1
        nin = (size_t)Lpad * (R_ + 1);
        nout = (size_t)Lpad * Lpad;
    }
    std::vector<C> in(nin);
    for (auto &v : in) v = C{(R)nd(rng), (R)nd(rng)};
    std::vector<R> out(nout, (R)NAN);
    const int T = g.Q / 16;
    blockDim.x = T;
    for (int line : lines) {
        blockIdx.x = MODE == 1 ? line / 2 : line;
        std::barrier<> bar(T);
        host_group = &bar;
        std::vector<std::thread> th;
        for (int t = 0; t < T; ++t)
            th.emplace_back([&, t] {
                threadIdx.x = t;
                k_fft_t2<R, MODE>(in.data(), out.data(), off.data(), ny0.data(), corr.data(), tw.data(), g);
            });
        for (auto &x : th) x.join();
    }
    double err = 0, big = 0;
    long unwritten = 0;
    for (int line : lines) {
        if (MODE == 0) {
            const cld cx = std::conj(cld(corr[line + R_].x, corr[line + R_].y));
            for (int m = 0; m < Lpad; ++m) {
                cld s = 0;
                for (int ny = ny0[line]; ny < ny0[line] + off[line + 1] - off[line]; ++ny) {
                    const C c = in[off[line] + ny - ny0[line]];
                    const long double f = (line > 0 || ny > 0) ? 2 : 1;
                    s += f * cld(c.x, c.y) * cx * std::conj(cld(corr[ny + R_].x, corr[ny + R_].y)) * ex(ny, m);
                }
                const R gx = out[((size_t)line * Lpad + m) * 2], gy = out[((size_t)line * Lpad + m) * 2 + 1];
                if (std::isnan(gx) || std::isnan(gy)) { ++unwritten; continue; }
                err = std::fmax(err, (double)std::abs(s - cld(gx, gy)));
                big = std::fmax(big, (double)std::abs(s));
            }
        } else {
            for (int row = line; row < std::min(line + 2, Lpad); ++row)
                for (int m = 0; m < Lpad; ++m) {
                    long double s = 0;
                    for (int k = 0; k <= R_; ++k) {
                        const C h = in[(size_t)row * (R_ + 1) + k];
                        s += (cld(h.x, h.y) * ex(k, m)).real();
                    }
                    const R got = out[(size_t)row * Lpad + m];
                    if (std::isnan(got)) { ++unwritten; continue; }
                    err = std::fmax(err, (double)std::fabs(s - (long double)got));
                    big = std::fmax(big, (double)std::fabs(s));
                }
        }
    }
    printf("%s %d %d %d %d %.3e %ld\n", sizeof(R) == 4 ? "f32" : "f64", MODE, P, Q, Lpad, err / big, unwritten);
}

int main()
{
    check<float, 0>(3, 256, 240, 190);      // two radix-16 passes
    check<float, 1>(3, 512, 480, 380);      // radix-2 tail
    check<float, 1>(3, 256, 241, 190);      // odd band: the last row transformed alone
    check<float, 0>(2, 1024, 1000, 500);    // radix-4 tail
    check<double, 0>(1, 2048, 2000, 500);   // radix-8 tail
    check<double, 1>(2, 512, 500, 250);
}
"""


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    src = kernels_source()
    blocks = struct(internal_source(), "Geom") + "\n" + "\n".join(definition(src, n) for n in NAMES)
    d = tmp_path_factory.mktemp("fft2lines")
    cpp, exe = d / "lines2.cpp", d / "lines2"
    cpp.write_text(HOST_PRELUDE + DRIVER.replace("@BLOCKS@", blocks))
    subprocess.run([gxx, "-O2", "-std=c++20", "-pthread", "-Wno-unknown-pragmas", "-ffp-contract=off", str(cpp),
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=240).stdout
    rows = [line.split() for line in out.strip().splitlines()]
    assert len(rows) == 6, out
    return [{"prec": f[0], "mode": int(f[1]), "P": int(f[2]), "Q": int(f[3]), "Lpad": int(f[4]), "err": float(f[5]),
             "unwritten": int(f[6])} for f in rows]


def test_type2_lines_match_the_direct_sum(results):
    for r in results:
        assert r["err"] < (5e-7 if r["prec"] == "f32" else 1e-14), r


def test_every_output_written(results):
    for r in results:
        assert r["unwritten"] == 0, r
