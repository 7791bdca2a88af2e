"""Reverse mode through N PCEXP steps with checkpointing.

Objective (a pressure-fluctuation functional along a trajectory with a fixed
time step): J(u_0) = sum_{n=1}^{N} dt int_Omega (p_h(t_n) - p_ref)^2 dx.
Its gradient is accumulated backwards: ubar_N = s dt dP/du(u_N), then for
n = N-1 .. 0, ubar_n = (du_{n+1}/du_n)^T ubar_{n+1} (+ s dt dP/du(u_n) for
n >= 1), with s the incoming cotangent.  Every step of both sweeps runs in
the library (pcexp_step, pcexp_step_vjp, and pcexp_pressure_functional_acc,
which adds s dt P and s dt dP/du into device accumulators); this module
only schedules the calls and owns the buffers.  The forward sweep keeps the
state every `every` steps; the reverse sweep recomputes each segment forward
from its checkpoint before sweeping it backwards, so at most
ceil(N / every) + every states are held at once.
"""

import math


class Trajectory:
    def __init__(self, ctx, dt, nsteps, m=30, every=8, p_ref=1.0, scheme="pcexp"):
        if not (dt > 0.0):
            raise ValueError("the reverse sweep needs a fixed dt > 0")
        if nsteps < 1 or every < 1:
            raise ValueError("nsteps and every must be >= 1")
        self.ctx, self.dt, self.n, self.m, self.every = ctx, float(dt), int(nsteps), int(m), int(every)
        self.p_ref, self.scheme = float(p_ref), scheme

    def _step(self, u):
        self.ctx.step(u, dt=self.dt, m=self.m, scheme=self.scheme)

    def forward(self, u0):
        """Forward sweep only: returns (J as a 0-dim device tensor, checkpoints),
        checkpoints being {n: u_n} for n = 0, every, 2 every, ... < N."""
        torch = self.ctx.torch
        acc = torch.zeros((), dtype=torch.float64, device=u0.device)
        ckpt = {0: u0.detach().clone().contiguous()}
        u = ckpt[0].clone()
        for n in range(1, self.n + 1):
            self._step(u)
            self.ctx.pressure_functional_acc(u, self.dt, self.p_ref, value_acc=acc)
            if n % self.every == 0 and n < self.n:
                ckpt[n] = u.clone()
        return acc, ckpt

    def backward(self, ckpt, scale=1.0):
        """Reverse sweep from the checkpoints of forward(): returns scale dJ/du_0."""
        ctx = self.ctx
        torch = ctx.torch
        s = float(scale) * self.dt
        # u_N: recompute the last segment's end from its checkpoint
        last = max(ckpt)
        u = ckpt[last].clone()
        for _ in range(last, self.n):
            self._step(u)
        ubar = torch.zeros_like(u)
        other = torch.empty_like(u)
        ctx.pressure_functional_acc(u, s, self.p_ref, grad_acc=ubar)
        del u
        for start in sorted(ckpt, reverse=True):
            end = min(start + self.every, self.n)
            states = [ckpt[start]]
            w = ckpt[start].clone()
            for _ in range(start + 1, end):
                self._step(w)
                states.append(w.clone())
            for k in range(end - 1, start - 1, -1):
                ctx.step_vjp(states[k - start], ubar, self.dt, m=self.m, scheme=self.scheme, out=other)
                ubar, other = other, ubar
                if k >= 1:
                    ctx.pressure_functional_acc(states[k - start], s, self.p_ref, grad_acc=ubar)
        return ubar

    def value(self, u0):
        acc, _ = self.forward(u0)
        return float(acc)

    def value_and_grad(self, u0):
        acc, ckpt = self.forward(u0)
        return float(acc), self.backward(ckpt)

    def peak_states(self):
        """States held at once by the reverse sweep (checkpoints + one segment)."""
        return math.ceil(self.n / self.every) + self.every


def objective(traj):
    """torch.autograd.Function applying J(u_0) of the trajectory: forward()
    runs the checkpointed forward sweep only; backward() runs the reverse
    sweep with the incoming cotangent passed to the library as a scale."""
    import torch

    class _Objective(torch.autograd.Function):
        @staticmethod
        def forward(fctx, u0):
            val, ckpt = traj.forward(u0.detach().contiguous())
            fctx.ckpt = ckpt
            return val

        @staticmethod
        def backward(fctx, gout):
            g = traj.backward(fctx.ckpt, scale=float(gout))
            fctx.ckpt = None
            return g

    return _Objective.apply
