"""The near-history kernel, compiled for the host and run step by step against the trapezoid sum (CPU).

`k_near` (Sec. 4.2; eqs. alphak, alphakEvolution, hggrid) advances, per Fourier mode of
wavenumber kappa, the interior pair (D, C) by the exact rotation and adds the two edge FIRs; it
reports alpha_tot = (dk/2pi)^2 alpha with
    alpha_n(kappa) = dt sum_{l=0}^{LA+W} w_l sin(kappa l dt)/kappa S_{n-l},
w_l = phi(l dt) on the opening edge l < W, 1 inside, phi((LA+W-l) dt) on the closing edge.
Here the kernel is built from the kernels file as plain C++ (its lanes are independent, so they
run one after another), fed the near and lag rings of S step by step as the step pipeline fills
them, and compared with that sum evaluated directly, for wavenumbers from 0 (the sin(x)/x -> x
limit) through the near cutoff (modes beyond it must report 0), with FP64 and FP32 rings.
Nothing here runs on a GPU or calls the oracle.
"""
import shutil
import subprocess

import numpy as np
import pytest

from kernel_source import HOST_PRELUDE, definition, internal_source, kernels_source, struct

pa = pytest.importorskip("paper_2604_07170_amd")

DRIVER = r"""
#include <cmath>
template <class R> struct cplx;
template <> struct cplx<float> { using T = float2; };
template <> struct cplx<double> { using T = double2; };
@BLOCKS@

static const double PHI[] = {@PHI@};

template <class R>
void check(int W, int LA, double dt, double dk, double K)
{
    using C = typename cplx<R>::T;
    Geom g{};
    g.W = W; g.LA = LA; g.dt = dt; g.dk = dk; g.K = K; g.lookahead = 4;
    // modes: a row through kappa = 0, a row crossing the near cutoff, a diagonal one
    std::vector<ModeChunk> chunks = {{0, 0, 0, 12}, {0, (int)(K / dk) - 5, 12, 10}, {7, -3, 22, 9}};
    const int H = 31;
    std::vector<double2> D(H, double2{0, 0}), Cs(H, double2{0, 0});
    std::vector<C> cur((size_t)W * H), lag((size_t)W * H), atot(H);
    const int nt = LA + 3 * W + 40;
    std::mt19937 rng(7 + sizeof(R));
    std::normal_distribution<double> nd;
    std::vector<std::vector<C>> S(nt + 1, std::vector<C>(H, C{0, 0}));
    for (int n = 1; n <= nt; ++n)
        for (int k = 0; k < H; ++k) S[n][k] = C{(R)nd(rng), (R)nd(rng)};
    auto at = [&](int n, int k) { return n >= 1 ? S[n][k] : C{0, 0}; };
    std::vector<double> w(LA + W + 1, 1.0);
    for (int l = 0; l < W; ++l) w[l] = PHI[l];
    for (int l = LA + 1; l <= LA + W; ++l) w[l] = PHI[LA + W - l];
    const double scale = (dk / (2 * M_PI)) * (dk / (2 * M_PI));
    double err = 0, big = 0;
    long bad_far = 0, n_far = 0;
    for (int n = 1; n <= nt; ++n) {
        // the rings as the split fills them: S_n into the near ring, S_{n-LA} into the lag ring
        for (int k = 0; k < H; ++k) {
            cur[(size_t)(n % W) * H + k] = at(n, k);
            lag[(size_t)(((n - LA) % W + W) % W) * H + k] = at(n - LA, k);
        }
        const int64_t step = n + g.lookahead;
        for (unsigned b = 0; b < chunks.size(); ++b) {
            blockIdx.x = b;
            for (int t = 0; t < 256; ++t) {
                threadIdx.x = t;
                k_near<R>(chunks.data(), cur.data(), lag.data(), D.data(), Cs.data(), PHI, atot.data(), H, &step, g);
            }
        }
        for (const auto &c : chunks)
            for (int t = 0; t < c.cnt; ++t) {
                const int k = c.off + t, ny = c.ny0 + t;
                const double key = (double)c.nx * c.nx + (double)ny * ny, kap = dk * std::sqrt(key);
                if (key * dk * dk > K * K) { ++n_far; bad_far += atot[k].x != 0 || atot[k].y != 0; continue; }
                long double sx = 0, sy = 0;
                for (int l = 1; l <= LA + W; ++l) {
                    const long double sn = kap > 0 ? std::sin((long double)kap * l * dt) / kap : (long double)l * dt;
                    const C v = at(n - l, k);
                    sx += dt * w[l] * sn * v.x;
                    sy += dt * w[l] * sn * v.y;
                }
                err = std::fmax(err, std::hypot((double)(sx * scale) - atot[k].x, (double)(sy * scale) - atot[k].y));
                big = std::fmax(big, (double)(std::hypot((double)sx, (double)sy) * scale));
            }
    }
    printf("%s %d %d %.3e %ld %ld\n", sizeof(R) == 4 ? "f32" : "f64", W, LA, err / big, bad_far, n_far);
}

int main()
{
    check<double>(@W@, @LA@, @DT@, @DK@, @K@);
    check<float>(@W@, @LA@, @DT@, @DK@, @K@);
}
"""


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    dt, W, tol, p = 0.05, 24, 1e-7, 20
    v = pa.host_eval(1, [dt, W, tol, p, -1, 1.0, 0.0, 80.0], 12)
    delta, b, LA = v[0], v[1], int(round(v[8]))
    phi = [pa.host_eval(6, [delta, b, i * dt], 2)[0] for i in range(W + 1)]
    K = np.pi / dt
    dk = 2 * np.pi / 9.2          # a wavenumber spacing of the kind the plan uses
    src = kernels_source()
    to_d = "\n".join(l for l in src.splitlines() if " to_d(" in l and l.startswith("__device__"))
    blocks = "\n".join([struct(internal_source(), "Geom"), struct(internal_source(), "ModeChunk"), definition(src, "cmul"),
                        to_d, definition(src, "from_d"), definition(src, "k_near")])
    drv = (DRIVER.replace("@BLOCKS@", blocks).replace("@PHI@", ", ".join(repr(float(x)) for x in phi))
           .replace("@W@", str(W)).replace("@LA@", str(LA)).replace("@DT@", repr(dt)).replace("@DK@", repr(dk))
           .replace("@K@", repr(float(K))))
    d = tmp_path_factory.mktemp("near")
    cpp, exe = d / "near.cpp", d / "near"
    cpp.write_text(HOST_PRELUDE + drv)
    subprocess.run([gxx, "-O2", "-std=c++20", "-pthread", "-Wno-unknown-pragmas", "-ffp-contract=off", str(cpp), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=240).stdout
    rows = [line.split() for line in out.strip().splitlines()]
    assert len(rows) == 2, out
    return [{"prec": f[0], "W": int(f[1]), "LA": int(f[2]), "err": float(f[3]), "bad_far": int(f[4]), "n_far": int(f[5])}
            for f in rows]


def test_near_kernel_reproduces_the_trapezoid_sum(results):
    for r in results:
        assert r["err"] < (1e-13 if r["prec"] == "f64" else 1e-7), r


def test_modes_beyond_the_near_cutoff_report_zero(results):
    for r in results:
        assert r["n_far"] > 0 and r["bad_far"] == 0, r
