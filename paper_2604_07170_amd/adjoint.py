"""Gradients of losses of the wave field with respect to source strengths.

Sources carry sigma_j(t) = A_j s_j(t) with fixed unit signatures s_j and
strengths A_j.  The plan's discrete operator u(t_m) = sum_l K(m - l) sigma(t_l)
is linear, so for any loss L(u):

    dL/dA_j = sum_l s_j(t_l) (K^T g)_j(t_l),   g(t_m) = dL/du(t_m),

and K^T is the method run on the transposed plan (sources and targets
exchanged) with g fed in reverse time (see wfp2d_adjoint_init).  Each adjoint
step ends with wfp2d_evaluate_dot, which folds s_j(t_l) into the gradient on
the device, so neither sigma-bar nor the forward state is stored.

Two entry points (both torch.autograd.Function):

* ``strength_field(A, run)`` returns u on the loss window [m0, T] as a tensor
  (memory: window x Nx), for any loss built on it with torch.
* ``strength_loss_checkpointed(A, run, loss_fn, every)`` returns the scalar
  sum_m loss_fn(m, u(t_m)) over the window without keeping u: the forward
  saves the plan state every `every` reported steps ("checkpointed Fourier
  history"), and the backward recomputes one segment of u at a time, last
  segment first, to form g for the adjoint (memory: checkpoints x state +
  every x Nx).  By default the checkpoints are spectral: the Fourier history
  without the sigma history ring (4.5 GB instead of 39 GB at 10^6 sources),
  whose samples are put back from the signatures on restore.
"""
from __future__ import annotations

import torch


class StrengthRun:
    """A forward plan, its transpose, the unit signatures and the loss window.

    signature(l) must return s(t_l) for l >= 1 as a float64 CUDA tensor of M
    elements (caller source order).  Reported steps m = 1..nt; the loss
    window is m0..nt."""

    def __init__(self, plan, signature, nt: int, m0: int = 1):
        if not (1 <= m0 <= nt):
            raise ValueError("need 1 <= m0 <= nt")
        self.plan, self.signature, self.nt, self.m0 = plan, signature, int(nt), int(m0)
        self.la = plan.info()["lookahead"]
        self.M, self.Nx = plan.M, plan.Nx
        self.device = plan.device
        self._adj = None

    @property
    def adj(self):
        if self._adj is None:
            self._adj = self.plan.adjoint()
        return self._adj

    @property
    def window(self) -> int:
        return self.nt - self.m0 + 1

    # ---- forward: u(t_m) for m in the window ----
    def _forward_steps(self, A, on_report, start_step: int = 1, stop_step: int | None = None):
        """Ingest steps start_step..stop_step of sigma = A * s; call on_report(m) after each
        step whose reported m lies in the window (the plan's u is ready for evaluate)."""
        stop = self.nt + self.la if stop_step is None else stop_step
        for n in range(start_step, stop + 1):
            self.plan.step((A * self.signature(n)).contiguous())
            m = n - self.la
            if self.m0 <= m <= self.nt:
                on_report(m)

    def forward_field(self, A) -> torch.Tensor:
        u = torch.empty((self.window, self.Nx), dtype=torch.float64, device=self.device)
        self.plan.reset()
        self._forward_steps(A, lambda m: self.plan.evaluate(u[m - self.m0]))
        return u

    # ---- backward: dL/dA from g = dL/du on the window ----
    def backward_strengths(self, g_at) -> torch.Tensor:
        """g_at(m) -> dL/du(t_m) (float64 CUDA [Nx]) for m in the window, requested in
        decreasing m.  Returns dL/dA (float64 CUDA [M])."""
        adj, nt, la = self.adj, self.nt, self.la
        zero = torch.zeros(self.Nx, dtype=torch.float64, device=self.device)
        acc = torch.zeros(self.M, dtype=torch.float64, device=self.device)
        adj.reset()
        for n in range(1, nt + 2 * la + 1):
            m = nt + la + 1 - n                   # forward report time fed at this adjoint step
            x = g_at(m) if self.m0 <= m <= nt else zero
            adj.step(x.contiguous())
            if n > la:
                l = nt + 2 * la + 1 - n           # forward input time whose sigma-bar is reported
                adj.evaluate_dot(self.signature(l).contiguous(), acc)
        return acc

    def close(self):
        if self._adj is not None:
            self._adj.close()
            self._adj = None


class _Field(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, run):
        ctx.run = run
        return run.forward_field(A.detach())

    @staticmethod
    def backward(ctx, gu):
        run = ctx.run
        gu = gu.contiguous()
        return run.backward_strengths(lambda m: gu[m - run.m0]), None


def strength_field(A: torch.Tensor, run: StrengthRun) -> torch.Tensor:
    """u(x_i, t_m) for m = run.m0..run.nt as a [window, Nx] tensor, differentiable in A."""
    return _Field.apply(A, run)


class _CheckpointedLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, run, loss_fn, every, spectral):
        A = A.detach()
        plan, la = run.plan, run.la
        u = torch.empty(run.Nx, dtype=torch.float64, device=run.device)
        total = torch.zeros((), dtype=torch.float64, device=run.device)
        ckpts = []                                 # (first m of the segment, saved state)
        plan.reset()
        # steps before the window
        first_n = run.m0 + la
        run._forward_steps(A, lambda m: None, 1, first_n - 1)
        n = first_n
        while n <= run.nt + la:
            m_seg = n - la
            ckpts.append((m_seg, plan.save_spectral_state() if spectral else plan.save_state()))
            stop = min(n + every - 1, run.nt + la)

            def report(m):
                plan.evaluate(u)
                nonlocal total
                total = total + loss_fn(m, u).detach()
            run._forward_steps(A, report, n, stop)
            n = stop + 1
        ctx.run, ctx.loss_fn, ctx.every, ctx.A, ctx.ckpts, ctx.spectral = run, loss_fn, every, A, ckpts, spectral
        return total

    @staticmethod
    def backward(ctx, gL):
        run, loss_fn, A, ckpts = ctx.run, ctx.loss_fn, ctx.A, ctx.ckpts
        plan, la = run.plan, run.la
        seg_g = {}

        def g_at(m):
            if m not in seg_g:
                # recompute the segment holding m from its checkpoint (segments are requested last first)
                seg_g.clear()
                k = max(i for i, (ms, _) in enumerate(ckpts) if ms <= m)
                ms, state = ckpts[k]
                me = ckpts[k + 1][0] - 1 if k + 1 < len(ckpts) else run.nt
                if ctx.spectral:
                    plan.load_spectral_state(state)
                    n0 = ms + la - 1                          # steps ingested when the checkpoint was taken
                    depth = plan.info()["sigma_depth"]
                    for l in range(max(1, n0 - depth + 1), n0 + 1):
                        plan.put_sigma(l, (A * run.signature(l)).contiguous())
                else:
                    plan.load_state(state)
                u = torch.empty(run.Nx, dtype=torch.float64, device=run.device)

                def report(mm):
                    plan.evaluate(u)
                    uu = u.clone().requires_grad_(True)
                    with torch.enable_grad():
                        (g,) = torch.autograd.grad(loss_fn(mm, uu), uu)
                    seg_g[mm] = (gL * g).detach()
                run._forward_steps(A, report, ms + la, me + la)
            return seg_g[m]

        grad = run.backward_strengths(g_at)
        return grad, None, None, None, None


def strength_loss_checkpointed(A: torch.Tensor, run: StrengthRun, loss_fn, every: int,
                               spectral: bool = True) -> torch.Tensor:
    """sum_m loss_fn(m, u(t_m)) over the window, differentiable in A, with u recomputed
    from plan checkpoints taken every `every` reported steps (spectral: without the
    sigma history ring, refilled from run.signature on restore)."""
    if every < 1:
        raise ValueError("every must be >= 1")
    return _CheckpointedLoss.apply(A, run, loss_fn, int(every), bool(spectral))
