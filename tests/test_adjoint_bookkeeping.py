"""Host logic of the adjoint (CPU): the time-reversal index mapping of
StrengthRun and the segment recomputation of the checkpointed loss, run on a
stand-in plan that applies a known causal kernel with the library's step /
evaluate / look-ahead semantics.  The expected gradients come from the
explicit matrix of the stand-in operator, so a wrong index, a dropped
boundary step or a wrong segment fails here without a GPU.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2604_07170_amd.adjoint import StrengthRun, strength_field, strength_loss_checkpointed


class KernelPlan:
    """u_i(m) = sum_j sum_{d >= -L} k[d + L][i][j] sigma_j(m - d), reported with delay L after each step.

    Same contract as the library's plan: step(sigma(t_n)); evaluate() gives u(t_{n-L})
    (zero while n - L < 1); adjoint() exchanges the roles of sources and targets."""

    def __init__(self, kern, L, transposed=False):
        self.kern, self.L, self.transposed = kern, L, transposed
        self.Nx, self.M = (kern.shape[2], kern.shape[1]) if transposed else (kern.shape[1], kern.shape[2])
        self.device = torch.device("cpu")
        self.reset()

    def info(self):
        # samples older than the kernel's span are never read again: the ring's depth
        return {"lookahead": self.L, "sigma_depth": self.kern.shape[0]}

    def reset(self):
        self.hist = []

    def step(self, sigma):
        self.hist.append(sigma.detach().double().clone())

    def _u(self):
        n = len(self.hist)
        m = n - self.L
        out = torch.zeros(self.Nx, dtype=torch.float64)
        if m < 1:
            return out
        for l in range(1, n + 1):               # sigma(t_l), l <= m + L
            d = m - l
            if d + self.L < 0 or d + self.L >= self.kern.shape[0]:
                continue
            K = self.kern[d + self.L]
            out += (K.T if self.transposed else K) @ self.hist[l - 1]
        return out

    def evaluate(self, out=None):
        u = self._u()
        if out is not None:
            out.copy_(u)
            return out
        return u

    def evaluate_dot(self, w, acc):
        acc += w * self._u()

    def adjoint(self):
        return KernelPlan(self.kern, self.L, not self.transposed)

    def save_state(self):
        return [h.clone() for h in self.hist]

    def load_state(self, st):
        self.hist = [h.clone() for h in st]

    # spectral checkpoint: everything but the sample history, here just the step count; the
    # samples come back through put_sigma, and any the caller does not put back stay zero
    def save_spectral_state(self):
        return len(self.hist)

    def load_spectral_state(self, n):
        self.hist = [torch.zeros(self.M, dtype=torch.float64) for _ in range(n)]

    def put_sigma(self, l, sigma):
        n = len(self.hist)
        assert 1 <= l <= n and l > n - self.info()["sigma_depth"]
        self.hist[l - 1] = sigma.detach().double().clone()

    def close(self):
        pass


def _setup(seed=0, M=5, Nx=4, L=2, span=9, nt=12, m0=4):
    rng = np.random.default_rng(seed)
    kern = torch.as_tensor(rng.standard_normal((span, Nx, M)))
    S = torch.as_tensor(rng.standard_normal((nt + L, M)))     # unit signatures s_j(t_l)
    plan = KernelPlan(kern, L)
    run = StrengthRun(plan, lambda l: S[l - 1], nt=nt, m0=m0)
    A = torch.as_tensor(rng.standard_normal(M))
    return kern, S, plan, run, A, L, nt, m0


def _dense_operator(kern, L, nt, M, Nx):
    """Matrix G with u(m)_i = sum G[(m, i), (l, j)] sigma_j(t_l), m = 1..nt, l = 1..nt + L."""
    G = np.zeros((nt, Nx, nt + L, M))
    for m in range(1, nt + 1):
        for l in range(1, nt + L + 1):
            d = m - l
            if 0 <= d + L < kern.shape[0]:
                G[m - 1, :, l - 1, :] = kern[d + L].numpy()
    return G


def test_forward_window_matches_dense_operator():
    kern, S, plan, run, A, L, nt, m0 = _setup()
    u = run.forward_field(A)
    G = _dense_operator(kern, L, nt, run.M, run.Nx)
    sigma = (A.numpy()[None, :] * S.numpy())                  # (nt + L, M)
    ref = np.einsum("minj,nj->mi", G, sigma)[m0 - 1:]
    assert np.allclose(u.numpy(), ref, rtol=1e-12, atol=1e-12)


def test_strength_gradient_is_the_transpose():
    kern, S, plan, run, A, L, nt, m0 = _setup(seed=1)
    Gw = torch.as_tensor(np.random.default_rng(5).standard_normal((nt - m0 + 1, run.Nx)))
    Ar = A.clone().requires_grad_(True)
    (Gw * strength_field(Ar, run)).sum().backward()
    G = _dense_operator(kern, L, nt, run.M, run.Nx)
    g = np.zeros((nt, run.Nx))
    g[m0 - 1:] = Gw.numpy()
    sigma_bar = np.einsum("minj,mi->nj", G, g)                 # K^T g, (nt + L, M)
    ref = (S.numpy() * sigma_bar).sum(axis=0)
    assert np.allclose(Ar.grad.numpy(), ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("spectral", [False, True])
@pytest.mark.parametrize("every", [1, 3, 5, 100])
def test_checkpointed_loss_equals_stored(every, spectral):
    """Also with spectral checkpoints, whose restore puts back exactly the samples the
    history still reads (the stand-in zeroes the rest, so a short refill shows)."""
    kern, S, plan, run, A, L, nt, m0 = _setup(seed=2, nt=13, m0=3)
    Y = torch.as_tensor(np.random.default_rng(6).standard_normal((nt - m0 + 1, run.Nx)))

    def loss_fn(m, um):
        return 0.5 * ((um - Y[m - m0]) ** 2).sum() * (1.0 + 0.1 * m)

    A1 = A.clone().requires_grad_(True)
    u = strength_field(A1, run)
    w = torch.as_tensor([1.0 + 0.1 * m for m in range(m0, nt + 1)], dtype=torch.float64)
    L1 = (0.5 * w[:, None] * (u - Y) ** 2).sum()
    L1.backward()
    A2 = A.clone().requires_grad_(True)
    L2 = strength_loss_checkpointed(A2, run, loss_fn, every=every, spectral=spectral)
    L2.backward()
    l1, l2 = float(L1.detach()), float(L2.detach())
    assert abs(l1 - l2) <= 1e-12 * abs(l1)
    assert np.allclose(A1.grad.numpy(), A2.grad.numpy(), rtol=1e-12, atol=1e-12)
