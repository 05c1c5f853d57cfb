"""Batched form: uneven-N instances stepped together in one grouped launch."""
import numpy as np
import pytest

import oracle
from paper_2305_07187_amd import instances

from gpu_common import QMAX, announce, ensure_built, oracle_schedules, rel_err, to_dev

pytestmark = pytest.mark.gpu

SIZES = [(64, "pm1"), (100, "gauss"), (257, "pm1"), (512, "gauss"), (1000, "pm1"), (130, "pm1")]
R = 64
BATCH_TILE = 14  # the single-instance tile with the batched kernel's configuration


def _batch(specs, S, r=R):
    si = ensure_built()
    Js = [instances.make_J(n, kind, 10 + i) for i, (n, kind) in enumerate(specs)]
    xs = [instances.make_x0(n, r, 20 + i) for i, (n, kind) in enumerate(specs)]
    b = si.SpringIsingBatch([to_dev(J) for J in Js], [to_dev(x) for x in xs], total_steps=S)
    return b, Js, xs


def test_batch_equals_standalone_runs():
    import torch
    si = ensure_built()
    announce("batch vs standalone, bit for bit")
    S = 300
    b, Js, xs = _batch(SIZES, S)
    b.run(200)
    xb, pb, t = b.state()
    eb = b.energy()
    torch.cuda.synchronize()
    assert t == 200
    for i, (n, kind) in enumerate(SIZES):
        m = si.SpringIsing(to_dev(Js[i]), to_dev(xs[i]), total_steps=S, tile=BATCH_TILE)
        m.run(200)
        x, p, _ = m.state()
        e = m.energy(exact=False)
        torch.cuda.synchronize()
        assert np.array_equal(x.cpu().numpy(), xb[i].cpu().numpy()), (i, n, kind)
        assert np.array_equal(p.cpu().numpy(), pb[i].cpu().numpy()), (i, n, kind)
        assert np.array_equal(e.cpu().numpy(), eb[i].cpu().numpy()), (i, n, kind)
        m.close()
    b.close()


def test_batch_vs_oracle():
    # Larger and Gaussian instances amplify rounding differences faster
    # (their largest coupling eigenvalue grows like 2 sqrt(N)), so the
    # 1e-5 window is 30 steps here.
    import torch
    announce("batch vs oracle, 30 steps")
    S = 1000
    b, Js, xs = _batch(SIZES[:4], S)
    b.run(30)
    xb, pb, _ = b.state()
    torch.cuda.synchronize()
    dt, zeta = oracle_schedules(S)
    for i, (n, kind) in enumerate(SIZES[:4]):
        ref = oracle.run(Js[i].astype(np.float64), xs[i].T.astype(np.float64), None, dt, zeta,
                         qmax=QMAX, n_steps=30)
        eq = rel_err(xb[i].cpu().numpy(), ref["Q"])
        ep = rel_err(pb[i].cpu().numpy(), ref["P"])
        announce(f"  instance {i} N={n} {kind}: rel err q {eq:.2e} p {ep:.2e}")
        assert eq <= 1e-5 and ep <= 1e-5


def test_batch_energies_and_layout():
    import torch
    si = ensure_built()
    announce("batch energies, spins, state layout")
    specs = [(64, "pm1"), (300, "pm1"), (129, "pm1")]
    b, Js, xs = _batch(specs, 50, r=8)
    states = [instances.random_state(n, 8, 40 + i) for i, (n, _) in enumerate(specs)]
    b.set_state([to_dev(s) for s in states])
    e = b.energy(exact=True)
    s = b.spins()
    xb, _, _ = b.state()
    torch.cuda.synchronize()
    for i, (n, _) in enumerate(specs):
        sp = oracle.spins(states[i].T)
        np.testing.assert_array_equal(s[i].cpu().numpy().T, sp)
        np.testing.assert_array_equal(e[i].cpu().numpy(), oracle.ising_energy(Js[i], sp))
        np.testing.assert_array_equal(xb[i].cpu().numpy(), states[i])
    b.close()
    # mixed batch: the exact energy is refused, the real one works
    b, Js, xs = _batch(SIZES[:2], 10)
    with pytest.raises(si.SpringIsingError) as err:
        b.energy(exact=True)
    assert err.value.status == si.SI_ERR_UNSUPPORTED
    er = b.energy(exact=False)
    torch.cuda.synchronize()
    for i, (n, kind) in enumerate(SIZES[:2]):
        ref = oracle.ising_energy(Js[i].astype(np.float64), oracle.spins(xs[i].T))
        bound = n * 2.0 ** -24 * np.abs(Js[i]).astype(np.float64).sum() + 1e-6
        assert np.all(np.abs(er[i].cpu().numpy() - ref) <= bound)
    b.close()


def test_batch_full_workload_generated_on_device():
    # 256 instances, N uniform in [64, 4096], half +-1, half Gaussian, R=64
    import time

    import torch
    si = ensure_built()
    announce("batch of 256 uneven instances (generated on the device)")
    recipe = instances.make_batch(256, 0)
    dev = torch.device("cuda:0")
    Js = [instances.make_J_torch(n, kind, seed, dev) for n, kind, seed in recipe]
    xs = [instances.make_x0_torch(n, R, seed, device=dev) for n, kind, seed in recipe]
    torch.cuda.synchronize()
    b = si.SpringIsingBatch(Js, xs, total_steps=3000)
    del Js
    b.run(5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(20)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / 20
    e = b.energy()
    torch.cuda.synchronize()
    assert all(bool(torch.isfinite(v).all()) for v in e)
    info = b.info()
    announce(f"  {info['kernel_name']}: {el * 1e3:.3f} ms/step, total spins {info['n']}")
    b.close()
