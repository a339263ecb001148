"""The FFT building blocks of the HIP kernels, compiled for the host and checked against
exact DFTs (CPU).

The kernels' line transforms are made of register DFTs (radix 4, 8 and 16, and the radix-16
DFT whose first stage is pruned for inputs known to be zero) and of twiddles formed as FP64
powers of one entry of a two-level table of e^{2 pi i j/nf}.  This test takes those device
functions' source text from the kernels file, compiles it as plain C++ with g++ and compares
them with the definition X[k] = sum_m x[m] e^{sign 2 pi i k m/n} and with e^{sign 2 pi i j r/nf}
evaluated directly.  Nothing here runs on a GPU or calls the oracle.
"""
import shutil
import subprocess

import pytest

from kernel_source import definition, kernels_source

# device functions needed, by the name in their definition line
NAMES = ["cmul", "cadd", "csub", "from_d", "mul_si", "dft2", "dft4", "rot16", "dft8", "dft4_z", "dft16_nb", "dft16",
         "tw_d", "cmul_d", "twiddle_powers"]


HARNESS = r"""
#include <cmath>
#include <complex>
#include <cstdio>
#include <random>
#include <vector>
#define __device__
#define __forceinline__ inline
struct float2 { float x, y; };
struct double2 { double x, y; };
inline float2 make_float2(float x, float y) { return float2{x, y}; }
inline double2 make_double2(double x, double y) { return double2{x, y}; }
@BLOCKS@
using cd = std::complex<double>;

template <int NZ, class C> double dft16_err(int sign) {
    std::mt19937 g(11 + NZ);
    std::normal_distribution<double> n;
    double worst = 0;
    for (int t = 0; t < 40; ++t) {
        C v[16];
        cd x[16];
        for (int r = 0; r < 16; ++r) {
            x[r] = r < NZ ? cd(n(g), n(g)) : cd(0, 0);
            v[r] = C{(decltype(C{}.x))x[r].real(), (decltype(C{}.x))x[r].imag()};
            x[r] = cd(v[r].x, v[r].y);
        }
        dft16<NZ>(v, sign);
        double nrm = 0;
        for (int m = 0; m < 16; ++m) nrm += std::abs(x[m]);
        for (int k = 0; k < 16; ++k) {
            cd s = 0;
            for (int m = 0; m < 16; ++m) s += x[m] * std::polar(1.0, sign * 2 * M_PI * k * m / 16.0);
            worst = std::fmax(worst, std::abs(s - cd(v[k].x, v[k].y)) / (nrm + 1e-300));
        }
    }
    return worst;
}

template <class C> double dft8_err(int sign) {
    std::mt19937 g(5);
    std::normal_distribution<double> n;
    double worst = 0;
    for (int t = 0; t < 40; ++t) {
        C v[8];
        cd x[8];
        for (int r = 0; r < 8; ++r) { v[r] = C{n(g), n(g)}; x[r] = cd(v[r].x, v[r].y); }
        dft8(v, sign);
        for (int k = 0; k < 8; ++k) {
            cd s = 0;
            for (int m = 0; m < 8; ++m) s += x[m] * std::polar(1.0, sign * 2 * M_PI * k * m / 8.0);
            worst = std::fmax(worst, std::abs(s - cd(v[k].x, v[k].y)));
        }
    }
    return worst;
}

// the two-level table the kernels stage: tt[i] = e(i) for i < 64, tt[64 + i] = e(64 i)
template <int N, class C> double powers_err(int nf, int sign) {
    std::vector<double2> tt(64 + nf / 64);
    for (int i = 0; i < 64 + nf / 64; ++i) {
        const int j = i < 64 ? i : (i - 64) * 64;
        tt[i] = double2{std::cos(2 * M_PI * j / nf), std::sin(2 * M_PI * j / nf)};
    }
    double worst = 0;
    for (int j = 0; j * (N - 1) < nf; ++j) {
        C v[N];
        for (int r = 0; r < N; ++r) v[r] = C{1, 0};
        twiddle_powers<N>(v, tt.data(), j, sign);
        for (int r = 1; r < N; ++r) {
            const long double a = 2.0L * 3.14159265358979323846264338327950288L * (long double)j * r / nf;
            const double ex = (double)std::cos(a), ey = sign * (double)std::sin(a);
            worst = std::fmax(worst, std::hypot(v[r].x - ex, v[r].y - ey));
        }
    }
    return worst;
}

int main() {
    for (int sign : {1, -1}) {
        printf("dft16 %d %.3e %.3e %.3e %.3e %.3e %.3e %.3e\n", sign, dft16_err<16, double2>(sign), dft16_err<8, double2>(sign),
               dft16_err<6, double2>(sign), dft16_err<5, double2>(sign), dft16_err<3, double2>(sign),
               dft16_err<1, double2>(sign), dft16_err<5, float2>(sign));
        printf("dft8 %d %.3e\n", sign, dft8_err<double2>(sign));
        printf("powers %d %.3e %.3e %.3e\n", sign, powers_err<16, double2>(12288, sign), powers_err<8, double2>(12288, sign),
               powers_err<16, float2>(12288, sign));
    }
}
"""


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    src = kernels_source()
    blocks = "\n".join(definition(src, n) for n in NAMES)
    d = tmp_path_factory.mktemp("fftblocks")
    cpp, exe = d / "blocks.cpp", d / "blocks"
    cpp.write_text(HARNESS.replace("@BLOCKS@", blocks))
    subprocess.run([gxx, "-O1", "-std=c++17", "-ffp-contract=off", str(cpp), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    res = {}
    for line in out.strip().splitlines():
        f = line.split()
        res[(f[0], int(f[1]))] = [float(x) for x in f[2:]]
    return res


@pytest.mark.parametrize("sign", [1, -1])
def test_radix16_dft_and_its_pruned_forms(results, sign):
    """dft16<NZ> with v[r] = 0 for r >= NZ (NZ = 16, 8, 6, 5, 3, 1) is the DFT of the 16 values,
    to FP64 rounding relative to sum |x|; the FP32 form (NZ = 5) to FP32 rounding."""
    e = results[("dft16", sign)]
    assert max(e[:6]) < 1e-14, e
    assert e[6] < 5e-7, e


@pytest.mark.parametrize("sign", [1, -1])
def test_radix8_dft(results, sign):
    assert results[("dft8", sign)][0] < 1e-13


@pytest.mark.parametrize("sign", [1, -1])
def test_twiddle_powers_match_the_exponentials(results, sign):
    """The powers w^r (r < 16) of one table entry, formed by repeated FP64 products, stay within
    a few units of FP64 rounding of e^{sign 2 pi i j r/nf} at nf = 12288 for every j a pass uses;
    rounded to FP32 they are within one FP32 rounding of it."""
    p16, p8, p16f = results[("powers", sign)]
    assert p16 < 5e-15 and p8 < 5e-15, (p16, p8)
    assert p16f < 1.2e-7, p16f
