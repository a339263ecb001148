"""The local part's pair-word encoding, compiled for the host and checked bit-exactly (CPU).

A regular source-target pair of the local part (Sec. 6) is one 64-bit word: its target in the
batch (11 bits), the LDS offset of its profile row (12 bits) and its coordinate x in [-1, 1] as a
41-bit fraction.  Padding words carry a private target slot (1024 + e mod 128) and x = 0.  Within a
segment of R runs of 8 words, pair_pos stores 16-byte chunk c of run r at chunk offset c R + r.
Checked from the kernels file's own helpers: target and row round-trip exactly and x to within
the encoding's resolution (half of its 2^-40 step inside, one step at x = 1); padding words
decode as described; pair_pos is a bijection of each segment onto itself that keeps each 16-byte
chunk's two words together at chunk c R + r, the layout the local kernel's consumer waves load.
Nothing here runs on a GPU.
"""
import shutil
import subprocess

import pytest

from kernel_source import HOST_PRELUDE, definition, kernels_source

DRIVER = r"""
#include <cstring>
using std::min;
inline double __longlong_as_double(long long v) { double d; std::memcpy(&d, &v, 8); return d; }
constexpr int kRunPairs = @RUN@;
@BLOCKS@

int main()
{
    std::mt19937_64 rng(9);
    long bad_t = 0, bad_row = 0, bad_pad = 0, bad_pos = 0;
    double xerr = 0, xerr_in = 0;
    for (int i = 0; i < 200000; ++i) {
        const int t = (int)(rng() % 1024), row = (int)(rng() % 4096);
        double x = std::ldexp((double)(rng() >> 11), -53) * 2.0 - 1.0;
        if (i == 0) x = -1.0;
        if (i == 1) x = 1.0;
        const uint64_t w = pair_pack(t, row, x);
        bad_t += pair_t(w) != t;
        bad_row += pair_row16(w) != row;
        xerr = std::fmax(xerr, std::fabs(pair_x(w) - x));
        if (i > 1) xerr_in = std::fmax(xerr_in, std::fabs(pair_x(w) - x));
    }
    for (int64_t e = 0; e < 5000; ++e) {
        const uint64_t w = pair_pad(e) | ((uint64_t)(e % 4096) << 11);
        bad_pad += pair_t(w) != 1024 + (int)(e & 127) || pair_x(w) != 0.0 || pair_row16(w) != (int)(e % 4096);
    }
    for (int64_t nrun : {1, 2, 7, 64, 300}) {
        const int64_t s0 = 1000, n = nrun * kRunPairs;
        std::vector<int> seen(n, 0);
        for (int64_t e = s0; e < s0 + n; ++e) {
            const int64_t p = pair_pos(s0, nrun, e);
            if (p < s0 || p >= s0 + n) { ++bad_pos; continue; }
            ++seen[p - s0];
            const int64_t r = (e - s0) / kRunPairs, j = (e - s0) % kRunPairs;
            bad_pos += p != s0 + 2 * ((j / 2) * nrun + r) + (j % 2);
        }
        for (int c : seen) bad_pos += c != 1;
    }
    printf("%ld %ld %ld %ld %.17e %.17e\n", bad_t, bad_row, bad_pad, bad_pos, xerr, xerr_in);
}
"""


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    src = kernels_source()
    run = next(l for l in src.splitlines() if l.startswith("constexpr int kRunPairs")).split("=")[1].split(";")[0].strip()
    blocks = "\n".join(definition(src, n) for n in ["pair_pack", "pair_pad", "pair_pos", "pair_t", "pair_row16", "pair_x"])
    d = tmp_path_factory.mktemp("pairwords")
    cpp, exe = d / "pw.cpp", d / "pw"
    cpp.write_text(HOST_PRELUDE + DRIVER.replace("@RUN@", run).replace("@BLOCKS@", blocks))
    subprocess.run([gxx, "-O2", "-std=c++20", "-pthread", str(cpp), "-o", str(exe)], check=True)
    f = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=60).stdout.split()
    return {"bad_t": int(f[0]), "bad_row": int(f[1]), "bad_pad": int(f[2]), "bad_pos": int(f[3]), "xerr": float(f[4]),
            "xerr_in": float(f[5])}


def test_target_and_row_round_trip_exactly(results):
    assert results["bad_t"] == 0 and results["bad_row"] == 0, results


def test_coordinate_within_the_encoding_resolution(results):
    """Rounded to the nearest point of the 2^-40 grid in x (half a step) inside; x = 1 itself is
    stored one step below (the 41-bit fraction stops at 1 - 2^-41)."""
    ulp = 2.0 ** -53                  # the difference x' - x itself is formed in FP64
    assert results["xerr_in"] <= 2.0 ** -41 + ulp and results["xerr"] <= 2.0 ** -40 + ulp, results


def test_padding_words(results):
    assert results["bad_pad"] == 0, results


def test_run_interleaving_is_a_bijection_with_chunks_together(results):
    assert results["bad_pos"] == 0, results
