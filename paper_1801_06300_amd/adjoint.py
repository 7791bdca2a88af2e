"""Reverse mode through N PCEXP steps with checkpointing.

Objective (a pressure-fluctuation functional along a trajectory with a fixed
time step): J(u_0) = sum_{n=1}^{N} dt int_Omega (p_h(t_n) - p_ref)^2 dx.
Its gradient is accumulated backwards: ubar_N = dt dP/du(u_N), then for
n = N-1 .. 0, ubar_n = (du_{n+1}/du_n)^T ubar_{n+1} (+ dt dP/du(u_n) for
n >= 1).  Every step of the sweep runs in the library (pcexp_step,
pcexp_step_vjp, pcexp_pressure_functional); this module only schedules
them.  States are kept every `every` steps; a segment is recomputed forward
before it is swept backwards, so at most N/every + every states are held.
"""

import math


class Trajectory:
    def __init__(self, ctx, dt, nsteps, m=30, every=8, p_ref=1.0, scheme="pcexp"):
        if not (dt > 0.0):
            raise ValueError("the reverse sweep needs a fixed dt > 0")
        self.ctx, self.dt, self.n, self.m, self.every = ctx, float(dt), int(nsteps), int(m), int(every)
        self.p_ref, self.scheme = float(p_ref), scheme

    def _step(self, u):
        self.ctx.step(u, dt=self.dt, m=self.m, scheme=self.scheme)

    def value(self, u0):
        u = u0.clone()
        total = 0.0
        for _ in range(self.n):
            self._step(u)
            total += self.dt * self.ctx.pressure_functional(u, self.p_ref)
        return total

    def value_and_grad(self, u0):
        ctx = self.ctx
        ckpt = {0: u0.clone()}
        u = u0.clone()
        total = 0.0
        for n in range(1, self.n + 1):
            self._step(u)
            total += self.dt * ctx.pressure_functional(u, self.p_ref)
            if n % self.every == 0 and n < self.n:
                ckpt[n] = u.clone()
        _, g = ctx.pressure_functional(u, self.p_ref, grad=True)
        ubar = self.dt * g
        starts = sorted(ckpt)
        for s in reversed(starts):
            e = min(s + self.every, self.n)
            states = [ckpt[s]]
            w = ckpt[s].clone()
            for _ in range(s + 1, e):
                self._step(w)
                states.append(w.clone())
            for k in range(e - 1, s - 1, -1):
                ubar = ctx.step_vjp(states[k - s], ubar, self.dt, m=self.m, scheme=self.scheme)
                if k >= 1:
                    _, g = ctx.pressure_functional(states[k - s], self.p_ref, grad=True)
                    ubar = ubar + self.dt * g
        return total, ubar

    def peak_states(self):
        """States held at once by value_and_grad (checkpoints + one segment)."""
        return math.ceil(self.n / self.every) + self.every


def objective(traj):
    """torch.autograd.Function applying J(u_0) of the trajectory."""
    import torch

    class _Objective(torch.autograd.Function):
        @staticmethod
        def forward(fctx, u0):
            val, g = traj.value_and_grad(u0.detach().contiguous())
            fctx.save_for_backward(g)
            return u0.new_tensor(val)

        @staticmethod
        def backward(fctx, gout):
            (g,) = fctx.saved_tensors
            return gout * g

    return _Objective.apply
