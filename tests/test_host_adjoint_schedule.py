"""Host logic of the checkpointed reverse sweep (paper_1801_06300_amd.adjoint),
on the CPU with a recording stand-in for the library context.

The stand-in implements the same calls on a scalar-affine model
u_{n+1} = a u_n + b with P(u) = sum u^2, so the schedule's result has a
closed form: J = dt sum_n P(u_n), dJ/du_0 = dt sum_n 2 u_n a^n.  The tests
check that forward() runs only forward steps and value accumulations,
that backward() reproduces the closed-form gradient with the cotangent as
scale, and the number of states held.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1801_06300_amd.adjoint import Trajectory, objective  # noqa: E402


class FakeCtx:
    torch = torch

    def __init__(self, a=0.9, b=0.05):
        self.a, self.b = a, b
        self.calls = []

    def step(self, u, dt, m, scheme):
        self.calls.append("step")
        u.mul_(self.a).add_(self.b)

    def pressure_functional_acc(self, u, scale, p_ref=1.0, value_acc=None, grad_acc=None):
        self.calls.append("acc_value" if value_acc is not None else "acc_grad")
        if value_acc is not None:
            value_acc.add_(scale * torch.sum(u * u))
        if grad_acc is not None:
            grad_acc.add_(scale * 2.0 * u)

    def step_vjp(self, u, ubar, dt, m=30, scheme="pcexp", out=None):
        self.calls.append("step_vjp")
        out.copy_(self.a * ubar)
        return out


def _closed_form(u0, a, b, dt, n):
    u = u0.copy()
    val, grad = 0.0, np.zeros_like(u0)
    for k in range(1, n + 1):
        u = a * u + b
        val += dt * np.sum(u * u)
        grad += dt * 2.0 * u * a ** k
    return val, grad


@pytest.mark.parametrize("n,every", [(1, 1), (5, 2), (40, 8), (7, 3), (8, 8)])
def test_schedule_gradient_and_calls(n, every):
    ctx = FakeCtx()
    dt = 0.3
    u0 = torch.linspace(-1.0, 2.0, 12, dtype=torch.float64)
    traj = Trajectory(ctx, dt, nsteps=n, m=4, every=every)
    acc, ckpt = traj.forward(u0)
    assert ctx.calls == ["step", "acc_value"] * n          # forward sweep only
    assert sorted(ckpt) == list(range(0, n, every))
    ctx.calls.clear()
    g = traj.backward(ckpt, scale=2.5)
    assert ctx.calls.count("step_vjp") == n
    assert ctx.calls.count("acc_grad") == n                # u_N and u_1 .. u_{N-1}
    assert "acc_value" not in ctx.calls
    want_val, want_grad = _closed_form(u0.numpy(), ctx.a, ctx.b, dt, n)
    assert abs(float(acc) - want_val) < 1e-12 * abs(want_val)
    assert np.allclose(g.numpy(), 2.5 * want_grad, rtol=1e-13, atol=0.0)
    assert traj.peak_states() == -(-n // every) + every


def test_autograd_forward_runs_no_reverse_work():
    ctx = FakeCtx()
    traj = Trajectory(ctx, 0.2, nsteps=6, m=4, every=2)
    x = torch.linspace(0.0, 1.0, 5, dtype=torch.float64).requires_grad_(True)
    J = objective(traj)(x)
    assert "step_vjp" not in ctx.calls and "acc_grad" not in ctx.calls
    (3.0 * J).backward()
    _, want = _closed_form(x.detach().numpy(), ctx.a, ctx.b, 0.2, 6)
    assert np.allclose(x.grad.numpy(), 3.0 * want, rtol=1e-13, atol=0.0)


def test_rejects_bad_arguments():
    with pytest.raises(ValueError):
        Trajectory(FakeCtx(), 0.0, nsteps=3)
    with pytest.raises(ValueError):
        Trajectory(FakeCtx(), 0.1, nsteps=0)
