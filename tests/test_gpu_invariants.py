"""Bit-exact invariants of the HIP path that need no oracle, plus the error
paths of the C ABI on a real device."""
import ctypes

import numpy as np
import pytest

from paper_2305_07187_amd import instances

from gpu_common import announce, ensure_built, to_dev

pytestmark = pytest.mark.gpu


def _run(J, x0, steps, S=1000, **kw):
    import torch
    si = ensure_built()
    m = si.SpringIsing(to_dev(J), to_dev(x0), total_steps=S, **kw)
    m.run(steps)
    x, p, t = m.state()
    e = m.energy()
    torch.cuda.synchronize()
    out = (x.cpu().numpy(), p.cpu().numpy(), e.cpu().numpy(), m.info())
    m.close()
    return out


@pytest.mark.parametrize("n,r", [(100, 8), (2000, 256)])
def test_gauge_z2_determinism(n, r):
    announce(f"gauge/Z2/determinism N={n} R={r}")
    J = instances.make_pm1(n, 0)
    x0 = instances.make_x0(n, r, 0)
    d = np.where(np.random.default_rng(1).random(n) < 0.5, -1.0, 1.0).astype(np.float32)
    steps = 300
    x, p, e, info = _run(J, x0, steps)
    # determinism
    x2, p2, e2, _ = _run(J, x0, steps)
    assert np.array_equal(x, x2) and np.array_equal(p, p2) and np.array_equal(e, e2)
    # gauge: J' = D J D, x0' = x0 D  ->  x' = x D exactly, same energies
    xg, pg, eg, _ = _run((d[:, None] * J * d[None, :]).astype(np.float32), x0 * d[None, :], steps)
    assert np.array_equal(xg, x * d[None, :]) and np.array_equal(pg, p * d[None, :])
    assert np.array_equal(eg, e)
    # Z2: -x0 -> -x
    xz, pz, ez, _ = _run(J, -x0, steps)
    assert np.array_equal(xz, -x) and np.array_equal(pz, -p) and np.array_equal(ez, e)


def test_replica_independence():
    announce("replica independence")
    n, r = 200, 8
    J = instances.make_pm1(n, 2)
    x0 = instances.make_x0(n, r, 5)
    x, p, e, info = _run(J, x0, 200, tile=3)
    for c in (0, 5, 7):
        x1, p1, e1, _ = _run(J, x0[c:c + 1], 200, tile=3)
        assert np.array_equal(x1[0], x[c]) and np.array_equal(p1[0], p[c]) and e1[0] == e[c]


def test_resume_is_bit_identical():
    import torch
    announce("resume from saved state")
    si = ensure_built()
    n, r, S = 300, 16, 200
    J = to_dev(instances.make_pm1(n, 4))
    x0 = to_dev(instances.make_x0(n, r, 4))
    a = si.SpringIsing(J, x0, total_steps=S)
    a.run(77)
    xm, pm, tm = a.state()
    a.run(S - 77)
    xa, pa, ta = a.state()
    b = si.SpringIsing(J, x0, total_steps=S)
    b.set_state(xm, pm, tm)
    b.run(S - 77)
    xb, pb, tb = b.state()
    torch.cuda.synchronize()
    assert ta == tb == S
    assert torch.equal(xa, xb) and torch.equal(pa, pb)


@pytest.mark.parametrize("group", [(1, 2, 4, 5, 7, 8, 9, 11, 13, 14, 15, 16, 17, 18, 25, 26, 27, 28, 29, 30, 32, 33, 34),
                                   (3, 6, 10, 12)])
def test_tiles_agree(group):
    # Tile shapes that use the same MFMA instruction add the contraction in
    # the same order (slab depth and workgroup shape only regroup the
    # work), so their trajectories are identical bit for bit.
    announce(f"tile shapes agree {group}")
    n, r = 256, 128
    J = instances.make_pm1(n, 6)
    x0 = instances.make_x0(n, r, 6)
    ref = None
    for tile in group:
        x, p, e, info = _run(J, x0, 50, tile=tile)
        assert info["tile"] == tile
        if ref is None:
            ref = (x, p)
        else:
            assert np.array_equal(x, ref[0]) and np.array_equal(p, ref[1]), info["kernel_name"]


def test_error_paths():
    import torch
    announce("error paths")
    si = ensure_built()
    n, r = 64, 4
    x0 = to_dev(instances.make_x0(n, r, 0))
    J = instances.make_pm1(n, 0)
    bad = J.copy()
    bad[3, 5] = -bad[3, 5]
    with pytest.raises(si.SpringIsingError) as e:
        si.SpringIsing(to_dev(bad), x0, total_steps=10)
    assert e.value.status == si.SI_ERR_INVALID and "symmetric" in e.value.message
    bad = J.copy()
    bad[2, 2] = 1
    with pytest.raises(si.SpringIsingError) as e:
        si.SpringIsing(to_dev(bad), x0, total_steps=10)
    assert e.value.status == si.SI_ERR_INVALID
    bad = J.copy()
    bad[1, 2] = bad[2, 1] = np.nan
    with pytest.raises(si.SpringIsingError) as e:
        si.SpringIsing(to_dev(bad), x0, total_steps=10)
    assert e.value.status == si.SI_ERR_INVALID
    m = si.SpringIsing(to_dev(J), x0, total_steps=10)
    m.run(8)
    with pytest.raises(si.SpringIsingError) as e:
        m.run(3)
    assert e.value.status == si.SI_ERR_RANGE
    assert m.info()["t"] == 8  # nothing ran
    m.run(2)
    with pytest.raises(si.SpringIsingError) as e:
        m.step()
    assert e.value.status == si.SI_ERR_RANGE
    with pytest.raises(si.SpringIsingError) as e:
        m.set_state(x0, None, 11)
    assert e.value.status == si.SI_ERR_RANGE
    # host memory through the raw ABI
    lib = si.load_library()
    host = (ctypes.c_int32 * r)()
    assert lib.spring_ising_energy(m.ctx, ctypes.cast(host, ctypes.c_void_p), None) == si.SI_ERR_INVALID
    m.set_state(x0, None, 0)
    m.run(10)
    torch.cuda.synchronize()
    m.close()
