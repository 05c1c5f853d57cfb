"""Pins for the oracle's adjoint of the relaxed end-energy."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest
import torch

import oracle
from paper_2305_07187_amd import instances

from closed_forms import scalar_loss_derivative

F32_SQRT2 = float(np.float32(math.sqrt(2.0)))


def _torch_replay(J, Q0, dt, zeta, k=0.5, m=1.0, qmax=F32_SQRT2, pmax=2.0):
    """Independent forward written with torch ops; autograd gives the gradient."""
    Jt = torch.tensor(J, dtype=torch.float64)
    q = torch.tensor(Q0, dtype=torch.float64)
    p = torch.zeros_like(q)
    d = torch.tensor(np.asarray(dt, dtype=np.float64), requires_grad=True)
    z = torch.tensor(np.asarray(zeta, dtype=np.float64), requires_grad=True)
    for n in range(len(dt)):
        u = q + d[n] / m * p
        v = p + d[n] * (-k * q + z[n] * (Jt @ q))
        q = torch.clamp(u, -qmax, qmax)
        p = torch.clamp(v, -pmax, pmax)
    loss = (-0.5 * (q * (Jt @ q)).sum(0)).mean()
    loss.backward()
    return loss.item(), d.grad.numpy(), z.grad.numpy()


@pytest.mark.parametrize("n,r,S,m", [(10, 3, 40, 1.0), (24, 5, 120, 1.0), (16, 4, 80, 2.0)])
def test_adjoint_matches_autograd_replay(n, r, S, m):
    J = instances.make_pm1(n, 5).astype(np.float64)
    Q0 = instances.make_x0(n, r, 2).T.astype(np.float64)
    dt = oracle.dt_schedule(S).astype(np.float64)
    zeta = oracle.zeta_schedule(S).astype(np.float64)
    L, gd, gz = oracle.relaxed_energy_grad(J, Q0, None, dt, zeta, m=m, qmax=F32_SQRT2)
    Lt, gdt, gzt = _torch_replay(J, Q0, dt, zeta, m=m)
    assert L == pytest.approx(Lt, rel=1e-12)
    np.testing.assert_allclose(gd, gdt, rtol=1e-9, atol=1e-9 * np.abs(gdt).max())
    np.testing.assert_allclose(gz, gzt, rtol=1e-9, atol=1e-9 * np.abs(gzt).max())
    assert L == pytest.approx(oracle.relaxed_energy(J, oracle.run(J, Q0, None, dt, zeta, m=m,
                                                                   qmax=F32_SQRT2)["Q"]), rel=1e-12)


def test_adjoint_along_a_given_trajectory():
    # The gradient along an externally supplied trajectory (here the
    # states of the independent torch forward) equals torch autograd's
    # gradient of that same forward.
    n, r, S = 20, 4, 90
    J = instances.make_pm1(n, 6).astype(np.float64)
    Q0 = instances.make_x0(n, r, 3).T.astype(np.float64)
    dt = oracle.dt_schedule(S).astype(np.float64)
    zeta = oracle.zeta_schedule(S).astype(np.float64)
    Jt = torch.tensor(J, dtype=torch.float64)
    q = torch.tensor(Q0, dtype=torch.float64)
    p = torch.zeros_like(q)
    Qs, Ps = [q.numpy().copy()], [p.numpy().copy()]
    for k in range(S):
        u = q + float(dt[k]) * p
        v = p + float(dt[k]) * (-0.5 * q + float(zeta[k]) * (Jt @ q))
        q, p = torch.clamp(u, -F32_SQRT2, F32_SQRT2), torch.clamp(v, -2.0, 2.0)
        Qs.append(q.numpy().copy())
        Ps.append(p.numpy().copy())
    L, gd, gz = oracle.relaxed_energy_grad_along(J, Qs, Ps, dt, zeta, qmax=F32_SQRT2)
    Lt, gdt, gzt = _torch_replay(J, Q0, dt, zeta)
    assert L == pytest.approx(Lt, rel=1e-12)
    np.testing.assert_allclose(gd, gdt, rtol=1e-9, atol=1e-9 * np.abs(gdt).max())
    np.testing.assert_allclose(gz, gzt, rtol=1e-9, atol=1e-9 * np.abs(gzt).max())
    with pytest.raises(ValueError):
        oracle.relaxed_energy_grad_along(J, Qs[:-1], Ps[:-1], dt, zeta)


def test_adjoint_central_differences():
    # Smooth regime (walls not reached): central FD along random directions.
    n, r, S = 12, 4, 30
    J = instances.make_gauss(n, 1).astype(np.float64)
    Q0 = instances.make_x0(n, r, 1).T.astype(np.float64)
    dt = np.full(S, 0.1)
    zeta = np.linspace(0.01, 0.05, S)
    L, gd, gz = oracle.relaxed_energy_grad(J, Q0, None, dt, zeta)
    rng = np.random.default_rng(0)
    fq = lambda d, z: oracle.relaxed_energy(J, oracle.run(J, Q0, None, d, z)["Q"])
    out = oracle.run(J, Q0, None, dt, zeta)
    assert np.abs(out["Q"]).max() < 1.0 and np.abs(out["P"]).max() < 1.5
    for _ in range(4):
        u = rng.standard_normal(S)
        v = rng.standard_normal(S)
        want = gd @ u + gz @ v
        ests = []
        for h in (1e-4, 1e-5, 1e-6):
            ests.append((fq(dt + h * u, zeta + h * v) - fq(dt - h * u, zeta - h * v)) / (2 * h))
        assert min(abs(e - want) for e in ests) <= 1e-7 * max(1.0, abs(want))


@pytest.mark.parametrize("which", ["dt", "zeta"])
def test_adjoint_exact_dual_numbers(which):
    # Uniform coupling, all spins equal: the gradient of the relaxed energy is
    # N times the exact dual-number derivative of the scalar recurrence.
    n, S, a = 8, 56, 1.0
    J = a * (np.ones((n, n)) - np.eye(n))
    lam = a * (n - 1)
    dt = [0.125] * S
    zeta = [0.05 + 0.00390625 * i for i in range(S)]
    c = 0.25
    Q0 = np.full((n, 1), c)
    L, gd, gz = oracle.relaxed_energy_grad(J, Q0, None, dt, zeta, qmax=F32_SQRT2)
    g = gd if which == "dt" else gz
    walls = False
    for nv in (0, 5, S // 2, S - 1):
        val, der = scalar_loss_derivative(Fr(c), Fr(lam), dt, zeta, Fr(1, 2), Fr(1),
                                          Fr(F32_SQRT2), Fr(2), nv, which)
        assert L == pytest.approx(float(val) * n, rel=1e-12)
        assert g[nv] == pytest.approx(float(der) * n, rel=1e-10, abs=1e-12)
    out = oracle.run(J, Q0, None, dt, zeta, qmax=F32_SQRT2, record=range(S + 1))
    walls = [abs(out["traj"][s][0][0, 0]) == F32_SQRT2 for s in range(S + 1)]
    assert any(walls) and not all(walls)  # the gradient crosses clamp kinks


def test_adjoint_zero_when_loss_independent():
    # J = 0: the loss is identically 0, so is its gradient.
    n, S = 6, 10
    L, gd, gz = oracle.relaxed_energy_grad(np.zeros((n, n)), np.full((n, 2), 0.1), None,
                                           np.full(S, 0.2), np.full(S, 0.1))
    assert L == 0 and np.all(gd == 0) and np.all(gz == 0)
