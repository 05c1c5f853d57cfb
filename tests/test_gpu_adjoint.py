"""Adjoint (gradient of the relaxed end-energy w.r.t. the Delta and zeta
schedules) through the C ABI, against the FP64 oracle adjoint, exact dual
numbers and invariants."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from paper_2305_07187_amd import instances

from closed_forms import scalar_loss_derivative
from gpu_common import DT, QMAX, ZE, ZS, F32, announce, ensure_built, to_dev

pytestmark = pytest.mark.gpu


def _grad(J, x0, dt, zeta, ckpt=100, **kw):
    import torch
    si = ensure_built()
    m = si.SpringIsing(to_dev(J), to_dev(x0), total_steps=len(dt), **kw)
    m.set_schedule(to_dev(np.asarray(dt, np.float32)), to_dev(np.asarray(zeta, np.float32)))
    loss, gd, gz = m.relaxed_energy_grad(ckpt)
    torch.cuda.synchronize()
    t = m.info()["t"]
    m.close()
    assert t == len(dt)
    return float(loss.cpu()[0]), gd.cpu().numpy(), gz.cpu().numpy()


def _sched(S_total, S):
    return (oracle.dt_schedule(S_total, DT)[:S], oracle.zeta_schedule(S_total, ZS, ZE)[:S])


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def test_adjoint_vs_oracle_small():
    n, r, S = 100, 8, 100
    announce(f"adjoint vs oracle N={n} R={r} S={S}")
    J = instances.make_pm1(n, 0)
    x0 = instances.make_x0(n, r, 0)
    dt, zeta = _sched(1000, S)
    L, gd, gz = _grad(J, x0, dt, zeta, ckpt=30)
    Lo, gdo, gzo = oracle.relaxed_energy_grad(J.astype(np.float64), x0.T.astype(np.float64), None,
                                              dt.astype(np.float64), zeta.astype(np.float64),
                                              qmax=QMAX)
    announce(f"  loss {L:.8e} vs {Lo:.8e}; grad rel err dt {_rel(gd, gdo):.2e} "
             f"zeta {_rel(gz, gzo):.2e}")
    assert abs(L - Lo) <= 1e-5 * abs(Lo)
    assert _rel(gd, gdo) <= 1e-4 and _rel(gz, gzo) <= 1e-4
    # element by element: every entry at least 1e-3 of the largest within 1e-4
    # of its own value (entries far below the largest are otherwise unchecked)
    for name, g, go in (("dt", gd, gdo), ("zeta", gz, gzo)):
        big = np.abs(go) >= 1e-3 * np.abs(go).max()
        rel = np.abs(g[big] - go[big]) / np.abs(go[big])
        announce(f"  {name}: {int(big.sum())} of {len(go)} entries checked, worst element-wise "
                 f"rel err {rel.max():.2e}")
        assert big.sum() >= len(go) // 2
        assert rel.max() <= 1e-4, (name, int(np.argmax(rel)))


@pytest.mark.parametrize("which", ["dt", "zeta"])
def test_adjoint_exact_dual_numbers(which):
    # uniform coupling a = 1, every spin at c: N times the exact derivative of
    # the scalar recurrence (walls reached during the run)
    n, S = 8, 56
    announce(f"adjoint exact dual numbers ({which})")
    J = (np.ones((n, n)) - np.eye(n)).astype(np.float32)
    c = 0.25
    x0 = np.full((1, n), c, np.float32)
    dt = [0.125] * S
    zeta = [0.05 + 0.00390625 * i for i in range(S)]
    L, gd, gz = _grad(J, x0, dt, zeta, ckpt=9)
    g = gd if which == "dt" else gz
    for nv in (0, 7, S // 2, S - 1):
        val, der = scalar_loss_derivative(Fr(c), Fr(n - 1), dt, zeta, Fr(1, 2), Fr(1), Fr(QMAX),
                                          Fr(2), nv, which)
        assert L == pytest.approx(float(val) * n, rel=1e-5)
        assert g[nv] == pytest.approx(float(der) * n, rel=2e-4, abs=1e-4 * abs(float(der) * n) + 1e-6)


def test_adjoint_invariants():
    n, r, S = 300, 32, 120
    announce("adjoint determinism, checkpoint interval, gauge")
    J = instances.make_pm1(n, 3)
    x0 = instances.make_x0(n, r, 3)
    dt, zeta = _sched(1000, S)
    a = _grad(J, x0, dt, zeta, ckpt=100)
    b = _grad(J, x0, dt, zeta, ckpt=100)
    c = _grad(J, x0, dt, zeta, ckpt=7)
    d1 = _grad(J, x0, dt, zeta, ckpt=1)
    for other in (b, c, d1):
        assert other[0] == a[0]
        assert np.array_equal(other[1], a[1]) and np.array_equal(other[2], a[2])
    d = np.where(np.random.default_rng(0).random(n) < 0.5, -1.0, 1.0).astype(np.float32)
    g = _grad((d[:, None] * J * d[None, :]).astype(np.float32), x0 * d[None, :], dt, zeta, ckpt=13)
    assert g[0] == a[0] and np.array_equal(g[1], a[1]) and np.array_equal(g[2], a[2])


def test_adjoint_full_size_first_steps():
    # N=2000, R=64 (the differentiation workload's shape), first 40 steps of
    # its 2000-step schedule, against the FP64 oracle adjoint.
    n, r, S = 2000, 64, 40
    announce(f"adjoint full size N={n} R={r} first {S} steps")
    J = instances.make_pm1(n, 0)
    x0 = instances.make_x0(n, r, 0)
    dt, zeta = _sched(2000, S)
    L, gd, gz = _grad(J, x0, dt, zeta, ckpt=10)
    Lo, gdo, gzo = oracle.relaxed_energy_grad(J.astype(np.float64), x0.T.astype(np.float64), None,
                                              dt.astype(np.float64), zeta.astype(np.float64),
                                              qmax=QMAX)
    announce(f"  loss {L:.8e} vs {Lo:.8e}; grad rel err dt {_rel(gd, gdo):.2e} "
             f"zeta {_rel(gz, gzo):.2e}")
    assert abs(L - Lo) <= 1e-5 * abs(Lo)
    assert _rel(gd, gdo) <= 1e-3 and _rel(gz, gzo) <= 1e-3


def test_adjoint_full_configuration_along_gpu_trajectory():
    # The whole differentiation workload (N=2000, R=64, 2000 steps,
    # checkpoints every 100).  Over 2000 steps the FP32 and FP64 forward
    # trajectories part ways, so the oracle's reverse sweep runs along the
    # GPU's own forward states (recorded step by step; the GPU's adjoint
    # recomputes exactly these from its checkpoints): what remains to
    # compare is the backward arithmetic and the wall masks.
    import torch
    n, r, S = 2000, 64, 2000
    announce(f"adjoint full configuration N={n} R={r} S={S} along the GPU trajectory")
    si = ensure_built()
    J = instances.make_pm1(n, 0)
    x0 = instances.make_x0(n, r, 0)
    dt, zeta = _sched(S, S)
    m = si.SpringIsing(to_dev(J), to_dev(x0), total_steps=S)
    Qs, Ps = [x0.T], [np.zeros((n, r), np.float32)]
    for _ in range(S):
        m.step()
        x, p, _ = m.state()
        torch.cuda.synchronize()
        Qs.append(x.cpu().numpy().T)
        Ps.append(p.cpu().numpy().T)
    m.set_state(to_dev(x0), None, 0)
    loss, gd, gz = m.relaxed_energy_grad(100)
    torch.cuda.synchronize()
    L, gd, gz = float(loss.cpu()[0]), gd.cpu().numpy(), gz.cpu().numpy()
    m.close()
    Lo, gdo, gzo = oracle.relaxed_energy_grad_along(J.astype(np.float64), Qs, Ps,
                                                    dt.astype(np.float64),
                                                    zeta.astype(np.float64), qmax=QMAX)
    announce(f"  loss {L:.8e} vs {Lo:.8e}; grad rel err dt {_rel(gd, gdo):.2e} "
             f"zeta {_rel(gz, gzo):.2e}")
    assert abs(L - Lo) <= 1e-5 * abs(Lo)
    assert _rel(gd, gdo) <= 1e-3 and _rel(gz, gzo) <= 1e-3


def test_adjoint_vs_device_finite_differences():
    # At the differentiation workload's shape (N=2000, R=64), in the smooth
    # regime (zeta * lambda_max < k, walls never reached): the adjoint's
    # directional derivatives against central differences of the device's
    # own forward map, with the loss evaluated in FP64 from the final
    # positions.  The perturbations are the exact FP32 schedule changes.
    import torch
    si = ensure_built()
    n, r, S = 2000, 64, 100
    announce(f"adjoint vs device central differences N={n} R={r} S={S}")
    J = instances.make_pm1(n, 0)
    J64 = J.astype(np.float64)
    x0 = instances.make_x0(n, r, 0)
    dt = np.full(S, 0.1, np.float32)
    zeta = np.linspace(0.002, 0.005, S).astype(np.float32)
    L, gd, gz = _grad(J, x0, dt, zeta, ckpt=25)
    m = si.SpringIsing(to_dev(J), to_dev(x0), total_steps=S)

    def loss(d, z):
        m.set_state(to_dev(x0), None, 0)
        m.set_schedule(to_dev(d), to_dev(z))
        m.run(S)
        x, p, _ = m.state()
        torch.cuda.synchronize()
        q = x.cpu().numpy().T.astype(np.float64)
        assert np.abs(q).max() < QMAX and np.abs(p.cpu().numpy()).max() < 2.0
        return oracle.relaxed_energy(J64, q)

    assert loss(dt, zeta) == pytest.approx(L, rel=1e-6)
    rng = np.random.default_rng(5)
    h = 1e-2
    for _ in range(3):
        u, v = rng.standard_normal(S), rng.standard_normal(S)
        dp, dm = (dt * (1 + h * u)).astype(np.float32), (dt * (1 - h * u)).astype(np.float32)
        zp, zm = (zeta * (1 + h * v)).astype(np.float32), (zeta * (1 - h * v)).astype(np.float32)
        diff = loss(dp, zp) - loss(dm, zm)
        want = gd @ (dp.astype(np.float64) - dm) + gz @ (zp.astype(np.float64) - zm)
        announce(f"  central difference {diff:.6e} vs adjoint {want:.6e}")
        assert abs(diff - want) <= 2e-3 * abs(want) + 1e-6 * abs(L)
    m.close()


def test_adjoint_full_workload_runs():
    # the full differentiation workload: N=2000, R=64, 2000 steps, checkpoints
    # every 100; deterministic and invariant to the checkpoint interval
    import time
    n, r, S = 2000, 64, 2000
    announce(f"adjoint full workload N={n} R={r} S={S}")
    J = instances.make_pm1(n, 0)
    x0 = instances.make_x0(n, r, 0)
    dt, zeta = _sched(S, S)
    t0 = time.perf_counter()
    a = _grad(J, x0, dt, zeta, ckpt=100)
    el = time.perf_counter() - t0
    b = _grad(J, x0, dt, zeta, ckpt=250)
    assert np.all(np.isfinite(a[1])) and np.all(np.isfinite(a[2]))
    assert a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    announce(f"  loss {a[0]:.6e}, |g_dt|max {np.abs(a[1]).max():.3e}, wall {el:.2f} s")


def test_autograd_function():
    import torch
    from paper_2305_07187_amd.autograd import SpringIsingRelaxedEnergy
    announce("autograd Function")
    n, r, S = 100, 8, 60
    J = instances.make_pm1(n, 1)
    x0 = instances.make_x0(n, r, 1)
    dt_np, z_np = _sched(1000, S)
    dt = to_dev(dt_np).requires_grad_(True)
    z = to_dev(z_np).requires_grad_(True)
    loss = SpringIsingRelaxedEnergy.apply(to_dev(J), to_dev(x0), None, dt, z, 20)
    (2.0 * loss).backward()
    L, gd, gz = _grad(J, x0, dt_np, z_np, ckpt=20)
    assert float(loss) == L
    np.testing.assert_allclose(dt.grad.cpu().numpy(), (2.0 * gd).astype(np.float32), rtol=1e-6)
    np.testing.assert_allclose(z.grad.cpu().numpy(), (2.0 * gz).astype(np.float32), rtol=1e-6)


def test_adjoint_unsupported_configurations():
    si = ensure_built()
    n, r = 64, 4
    J = to_dev(instances.make_pm1(n, 0))
    x0 = to_dev(instances.make_x0(n, r, 0))
    for kw in ({"order": "symplectic"}, {"wall": "inelastic"}, {"precision": "bf16x_bf16j"}):
        m = si.SpringIsing(J, x0, total_steps=10, **kw)
        with pytest.raises(si.SpringIsingError) as e:
            m.relaxed_energy_grad(5)
        assert e.value.status == si.SI_ERR_UNSUPPORTED
        m.close()


def test_forward_backward_halves_equal_combined():
    import torch
    si = ensure_built()
    announce("relaxed energy forward/backward halves vs combined call")
    n, r, S = 200, 16, 90
    J = instances.make_pm1(n, 2)
    x0 = instances.make_x0(n, r, 2)
    dt, zeta = _sched(1000, S)
    L, gd, gz = _grad(J, x0, dt, zeta, ckpt=25)
    m = si.SpringIsing(to_dev(J), to_dev(x0), total_steps=S)
    m.set_schedule(to_dev(np.asarray(dt, np.float32)), to_dev(np.asarray(zeta, np.float32)))
    loss = m.relaxed_energy_forward(25)
    torch.cuda.synchronize()
    assert m.info()["t"] == S
    # state reads do not touch the tape
    m.state()
    m.energy()
    m.spins()
    g_dt, g_z = m.relaxed_energy_backward()
    torch.cuda.synchronize()
    assert float(loss.cpu()[0]) == L
    assert np.array_equal(g_dt.cpu().numpy(), gd) and np.array_equal(g_z.cpu().numpy(), gz)
    # the tape is consumed by the sweep
    with pytest.raises(si.SpringIsingError) as e:
        m.relaxed_energy_backward()
    assert e.value.status == si.SI_ERR_STATE
    m.close()


def test_backward_rejects_a_changed_trajectory():
    import torch
    si = ensure_built()
    announce("relaxed energy backward after a change of the trajectory")
    n, r, S = 64, 4, 30
    J = to_dev(instances.make_pm1(n, 3))
    x0 = to_dev(instances.make_x0(n, r, 3))
    dt, zeta = _sched(1000, S)
    dt_d, z_d = to_dev(np.asarray(dt, np.float32)), to_dev(np.asarray(zeta, np.float32))
    # every change starts from a fresh forward half over steps 10..S
    changes = {
        "set_schedule": lambda m: m.set_schedule(dt_d, z_d),
        "set_state": lambda m: m.set_state(x0, None, 10),
        "step": lambda m: (m.set_state(x0, None, 10), m.relaxed_energy_forward(10),
                           m.set_state(x0, None, S - 1), m.step()),
        "run": lambda m: (m.set_state(x0, None, 10), m.relaxed_energy_forward(10),
                          m.set_state(x0, None, S - 3), m.run(3)),
        "set_ksplit": lambda m: m.set_ksplit(1),
    }
    for name, change in changes.items():
        m = si.SpringIsing(J, x0, total_steps=S)
        m.set_schedule(dt_d, z_d)
        m.set_state(x0, None, 10)
        m.relaxed_energy_forward(10)
        change(m)
        torch.cuda.synchronize()
        with pytest.raises(si.SpringIsingError) as e:
            m.relaxed_energy_backward()
        assert e.value.status == si.SI_ERR_STATE, name
        # a fresh forward half makes backward available again
        m.set_state(x0, None, 10)
        m.relaxed_energy_forward(10)
        g_dt, g_z = m.relaxed_energy_backward()
        torch.cuda.synchronize()
        g = g_dt.cpu().numpy()
        assert np.all(np.isfinite(g)) and np.all(g[:10] == 0.0), name
        m.close()
    # a call that fails its argument checks leaves the tape alone
    m = si.SpringIsing(J, x0, total_steps=S)
    m.set_schedule(dt_d, z_d)
    m.relaxed_energy_forward(10)
    with pytest.raises(si.SpringIsingError):
        m.step()  # t == total_steps
    g_dt, _ = m.relaxed_energy_backward()
    torch.cuda.synchronize()
    assert np.all(np.isfinite(g_dt.cpu().numpy()))
    m.close()
    # backward before any forward half
    m = si.SpringIsing(J, x0, total_steps=S)
    with pytest.raises(si.SpringIsingError) as e:
        m.relaxed_energy_backward()
    assert e.value.status == si.SI_ERR_STATE
    m.close()


def test_autograd_defers_the_sweep():
    import torch
    from paper_2305_07187_amd.autograd import SpringIsingRelaxedEnergy
    announce("autograd Function keeps the tape until backward")
    n, r, S = 100, 8, 40
    J = instances.make_pm1(n, 4)
    x0 = instances.make_x0(n, r, 4)
    dt_np, z_np = _sched(1000, S)
    dt = to_dev(dt_np).requires_grad_(True)
    z = to_dev(z_np)
    loss = SpringIsingRelaxedEnergy.apply(to_dev(J), to_dev(x0), None, dt, z, 10)
    node = loss.grad_fn
    assert node.model is not None and node.model.ctx is not None
    loss.backward()
    assert node.model is None
    L, gd, gz = _grad(J, x0, dt_np, z_np, ckpt=10)
    assert float(loss) == L
    np.testing.assert_allclose(dt.grad.cpu().numpy(), gd.astype(np.float32), rtol=1e-6)
    # no schedule requires a gradient: the context is released in forward
    loss2 = SpringIsingRelaxedEnergy.apply(to_dev(J), to_dev(x0), None, dt.detach(), z, 10)
    assert float(loss2) == L


def test_checkpoint_interval_beyond_the_schedule():
    # an interval longer than the remaining steps is one segment (the
    # workspace is sized by the segment, not by the requested interval)
    announce("adjoint with a checkpoint interval past the schedule")
    n, r, S = 100, 8, 40
    J = instances.make_pm1(n, 5)
    x0 = instances.make_x0(n, r, 5)
    dt, zeta = _sched(1000, S)
    a = _grad(J, x0, dt, zeta, ckpt=S)
    b = _grad(J, x0, dt, zeta, ckpt=2 ** 30)
    assert a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_forward_half_at_the_end_of_the_schedule():
    # with no steps left the loss is the relaxed energy of the current state
    # and every gradient entry is zero
    import torch
    si = ensure_built()
    announce("relaxed energy forward/backward with no steps left")
    n, r, S = 100, 8, 20
    J = instances.make_pm1(n, 6)
    x0 = instances.make_x0(n, r, 6)
    dt, zeta = _sched(1000, S)
    m = si.SpringIsing(to_dev(J), to_dev(x0), total_steps=S)
    m.set_schedule(to_dev(np.asarray(dt, np.float32)), to_dev(np.asarray(zeta, np.float32)))
    m.run(S)
    q, _, _ = m.state()
    loss = m.relaxed_energy_forward(10)
    g_dt, g_z = m.relaxed_energy_backward()
    torch.cuda.synchronize()
    want = oracle.relaxed_energy(J.astype(np.float64), q.cpu().numpy().T.astype(np.float64))
    assert float(loss.cpu()[0]) == pytest.approx(want, rel=1e-5)  # J q in FP32
    assert not g_dt.cpu().numpy().any() and not g_z.cpu().numpy().any()
    m.close()
