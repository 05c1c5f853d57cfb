"""Split contraction: the coupling product of problems with fewer output
tiles than CUs cut into k ranges, partial products summed in a fixed order
by the update launch.  Checked against the FP64 oracle (trajectories, the
adjoint), for determinism, and for its selection rules."""
import numpy as np
import pytest

import oracle
from paper_2305_07187_amd import instances

from gpu_common import QMAX, announce, ensure_built, oracle_schedules, rel_err, to_dev

pytestmark = pytest.mark.gpu


def _model(J, x0, S, ksplit=None, **kw):
    si = ensure_built()
    m = si.SpringIsing(to_dev(J), to_dev(x0), total_steps=S, **kw)
    if ksplit is not None:
        m.set_ksplit(ksplit)
    return m


@pytest.mark.parametrize("tile,ksplit", [(3, 2), (3, 8), (14, 3), (2, 5), (26, 4), (6, 7)])
def test_split_trajectory_vs_oracle(tile, ksplit):
    import torch
    n, r, S = 300, 64, 200
    announce(f"split contraction tile {tile} ksplit {ksplit} N={n} R={r}")
    J = instances.make_pm1(n, 7)
    x0 = instances.make_x0(n, r, 7)
    m = _model(J, x0, S, ksplit, tile=tile)
    name = m.info()["kernel_name"]
    assert name.endswith(f"_ks{ksplit}"), name
    dt, zeta = oracle_schedules(S)
    ref = oracle.run(J.astype(np.float64), x0.T.astype(np.float64), None, dt, zeta, qmax=QMAX,
                     n_steps=40, record=[10, 20, 40])
    done = 0
    for k in (10, 20, 40):
        m.run(k - done)
        done = k
        x, p, _ = m.state()
        torch.cuda.synchronize()
        eq, ep = rel_err(x.cpu().numpy(), ref["traj"][k][0]), rel_err(p.cpu().numpy(), ref["traj"][k][1])
        assert eq <= 1e-5 and ep <= 1e-5, (k, eq, ep)
    e = m.energy().cpu().numpy()
    np.testing.assert_array_equal(e, oracle.ising_energy(J, oracle.spins(x.cpu().numpy().T)))
    m.close()


def test_split_variants_with_field():
    import torch
    n, r, S = 257, 40, 100
    announce("split contraction, symplectic order, inelastic wall, field")
    J = instances.make_gauss(n, 3)
    x0 = instances.make_x0(n, r, 3)
    h = instances.make_x0(n, 1, 5, scale=2.0)[0]
    m = _model(J, x0, S, 4, tile=3, order="symplectic", wall="inelastic")
    m.set_field(to_dev(h))
    m.run(30)
    x, p, _ = m.state()
    torch.cuda.synchronize()
    dt, zeta = oracle_schedules(S)
    ref = oracle.run(J.astype(np.float64), x0.T.astype(np.float64), None, dt, zeta, qmax=QMAX,
                     order="symplectic", wall="inelastic", h=h.astype(np.float64), n_steps=30)
    assert rel_err(x.cpu().numpy(), ref["Q"]) <= 1e-5 and rel_err(p.cpu().numpy(), ref["P"]) <= 1e-5
    m.close()


def test_split_automatic_choice_and_determinism():
    import torch
    n, r, S = 2000, 64, 100
    announce("automatic split at N=2000 R=64: choice, determinism, sampled parity")
    J = instances.make_pm1(n, 0)
    x0 = instances.make_x0(n, r, 0)
    outs = []
    for _ in range(2):
        m = _model(J, x0, S)
        name = m.info()["kernel_name"]
        m.run(10)
        x, p, _ = m.state()
        torch.cuda.synchronize()
        outs.append((x.cpu().numpy(), p.cpu().numpy()))
        assert m.info()["resident_groups"] == 0  # no resident form with a split
        m.close()
    announce(f"  automatic kernel {name}")
    assert "_ks" in name
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    cols = [0, 17, 63]
    dt, zeta = oracle_schedules(S)
    ref = oracle.run(J.astype(np.float64), x0[cols].T.astype(np.float64), None, dt, zeta,
                     qmax=QMAX, n_steps=10)
    assert rel_err(outs[0][0][cols], ref["Q"]) <= 1e-5 and rel_err(outs[0][1][cols], ref["P"]) <= 1e-5
    # explicitly unsplit: a different summation order, same trajectory to rounding
    m = _model(J, x0, S, 1)
    assert "_ks" not in m.info()["kernel_name"]
    m.run(10)
    x1, _, _ = m.state()
    torch.cuda.synchronize()
    assert rel_err(x1.cpu().numpy(), outs[0][0].T) <= 1e-5
    m.close()


@pytest.mark.parametrize("ksplit", [1, 4])
def test_split_adjoint_vs_oracle(ksplit):
    import torch
    n, r, S = 300, 32, 60
    announce(f"adjoint with ksplit {ksplit} vs FP64 oracle N={n} R={r} S={S}")
    J = instances.make_pm1(n, 9)
    x0 = instances.make_x0(n, r, 9)
    m = _model(J, x0, S, ksplit)
    loss, gd, gz = m.relaxed_energy_grad(20)
    torch.cuda.synchronize()
    dt, zeta = oracle_schedules(S)
    Lo, gdo, gzo = oracle.relaxed_energy_grad(J.astype(np.float64), x0.T.astype(np.float64), None,
                                              dt.astype(np.float64), zeta.astype(np.float64),
                                              qmax=QMAX)
    rel = lambda a, b: float(np.abs(a - b).max() / np.abs(b).max())
    L = float(loss.cpu()[0])
    announce(f"  loss {L:.8e} vs {Lo:.8e}; grad rel err dt {rel(gd.cpu().numpy(), gdo):.2e} "
             f"zeta {rel(gz.cpu().numpy(), gzo):.2e}")
    assert abs(L - Lo) <= 1e-5 * abs(Lo)
    assert rel(gd.cpu().numpy(), gdo) <= 1e-4 and rel(gz.cpu().numpy(), gzo) <= 1e-4
    m.close()


def test_split_argument_rules():
    si = ensure_built()
    J = instances.make_pm1(200, 1)
    x0 = instances.make_x0(200, 16, 1)
    m = _model(J, x0, 10)
    with pytest.raises(si.SpringIsingError) as e:
        m.set_ksplit(17)
    assert e.value.status == si.SI_ERR_INVALID
    m.close()
    m = _model(J, x0, 10, tile=5)  # 128x128: no split form
    with pytest.raises(si.SpringIsingError) as e:
        m.set_ksplit(2)
    assert e.value.status == si.SI_ERR_UNSUPPORTED
    m.close()
    m = _model(J, x0, 10, precision="bf16x_bf16j")
    with pytest.raises(si.SpringIsingError) as e:
        m.set_ksplit(2)
    assert e.value.status == si.SI_ERR_UNSUPPORTED
    m.set_ksplit(1)
    m.run(10)
    m.close()
