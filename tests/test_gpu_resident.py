"""Resident launches of run(): every step of the call inside one cooperative
launch, with the tile's q and p held in registers and a grid-wide barrier
between steps.  The arithmetic of each step is the per-step kernel's, so
the trajectories must agree bit for bit with per-step launches, for every
tile that has a resident form and for the order and wall variants."""
import numpy as np
import pytest

import oracle
from paper_2305_07187_amd import instances

from gpu_common import QMAX, announce, ensure_built, oracle_schedules, rel_err, to_dev

pytestmark = pytest.mark.gpu


def _pair(J, x0, S, steps, resident, **kw):
    import torch
    si = ensure_built()
    m = si.SpringIsing(to_dev(J), to_dev(x0), total_steps=S, **kw)
    m.set_resident(resident)
    info = m.info()
    for n in steps:
        m.run(n)
    x, p, t = m.state()
    torch.cuda.synchronize()
    e = m.energy().cpu().numpy()
    m.close()
    return x.cpu().numpy(), p.cpu().numpy(), t, e, info


@pytest.mark.parametrize("tile", [27, 26, 2, 1, 3])
def test_resident_equals_per_step(tile):
    n, r, S = 500, 256, 300
    announce(f"resident vs per-step tile {tile} N={n} R={r}")
    J = instances.make_pm1(n, 3)
    x0 = instances.make_x0(n, r, 3)
    # odd and even lengths, so that both buffer parities end a call
    steps = [37, 100, 1, 162]
    a = _pair(J, x0, S, steps, 0, tile=tile)
    b = _pair(J, x0, S, steps, 2, tile=tile)
    assert a[4]["resident_steps"] == 0 and b[4]["resident_steps"] == 2, b[4]
    assert b[4]["resident_groups"] > 0
    announce(f"  {b[4]['kernel_name']}: {b[4]['resident_groups']} resident groups")
    assert a[2] == b[2] == S
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[3], b[3])


@pytest.mark.parametrize("order,wall", [("symplectic", "clamp"), ("paper", "inelastic")])
def test_resident_variants_and_field(order, wall):
    import torch
    n, r, S = 300, 64, 120
    announce(f"resident {order}/{wall} with a field")
    J = instances.make_pm1(n, 4)
    x0 = instances.make_x0(n, r, 4)
    h = to_dev(instances.make_x0(n, 1, 9, scale=2.0)[0])
    res = []
    for resident in (0, 2):
        si = ensure_built()
        m = si.SpringIsing(to_dev(J), to_dev(x0), total_steps=S, order=order, wall=wall, tile=3)
        m.set_field(h)
        m.set_resident(resident)
        m.run(S)
        x, p, _ = m.state()
        torch.cuda.synchronize()
        res.append((x.cpu().numpy(), p.cpu().numpy(), m.info()["resident_steps"]))
        m.close()
    assert res[1][2] > 0
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])


def test_resident_vs_oracle():
    import torch
    n, r, S = 100, 8, 1000
    announce("resident run vs FP64 oracle, N=100 R=8, first 100 steps")
    si = ensure_built()
    J = instances.make_pm1(n, 0)
    x0 = instances.make_x0(n, r, 0)
    m = si.SpringIsing(to_dev(J), to_dev(x0), total_steps=S)
    m.set_resident(2)
    assert m.info()["resident_steps"] == 2
    dt, zeta = oracle_schedules(S)
    ref = oracle.run(J.astype(np.float64), x0.T.astype(np.float64), None, dt, zeta, qmax=QMAX,
                     n_steps=100, record=[25, 50, 100])
    done = 0
    for k in (25, 50, 100):
        m.run(k - done)
        done = k
        x, p, _ = m.state()
        torch.cuda.synchronize()
        eq = rel_err(x.cpu().numpy(), ref["traj"][k][0])
        ep = rel_err(p.cpu().numpy(), ref["traj"][k][1])
        assert eq <= 1e-5 and ep <= 1e-5, (k, eq, ep)


def test_resident_full_workload_matches_per_step():
    import torch
    n, r, S = 2000, 1024, 10000
    announce("resident vs per-step at N=2000 R=1024 (200 steps)")
    si = ensure_built()
    Jd = to_dev(instances.make_pm1(n, 0))
    x0 = to_dev(instances.make_x0(n, r, 0))
    out = []
    for resident in (0, 2):
        m = si.SpringIsing(Jd, x0, total_steps=S)
        m.set_resident(resident)
        m.run(200)
        x, p, _ = m.state()
        torch.cuda.synchronize()
        out.append((x, p, m.info()))
        m.close()
    assert out[1][2]["resident_groups"] == 256 and out[1][2]["resident_steps"] == 2, out[1][2]
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])


def test_resident_not_used_when_groups_exceed_device():
    n, r, S = 4000, 2048, 10
    si = ensure_built()
    m = si.SpringIsing(to_dev(instances.make_pm1(n, 1)), to_dev(instances.make_x0(n, r, 1)),
                       total_steps=S, tile=27)
    m.set_resident(2)
    assert m.info()["resident_groups"] == 0 and m.info()["resident_steps"] == 0  # 32 x 16 tiles
    m.run(S)
    m.close()
    with pytest.raises(si.SpringIsingError):
        si.SpringIsing(to_dev(instances.make_pm1(64, 1)), to_dev(instances.make_x0(64, 4, 1)),
                       total_steps=4).set_resident(-1)
