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


def _batch(specs, S, r=R, **kw):
    si = ensure_built()
    Js = [instances.make_J(n, kind, 10 + i) for i, (n, kind) in enumerate(specs)]
    xs = [instances.make_x0(n, r, 20 + i) for i, (n, kind) in enumerate(specs)]
    b = si.SpringIsingBatch([to_dev(J) for J in Js], [to_dev(x) for x in xs], total_steps=S, **kw)
    return b, Js, xs


@pytest.mark.parametrize("btile", [1, 2])
def test_batch_equals_standalone_runs(btile):
    import torch
    si = ensure_built()
    announce(f"batch (tile {btile}) vs standalone, bit for bit")
    S = 300
    b, Js, xs = _batch(SIZES, S, tile=btile)
    info = b.info()
    assert info["tile"] == btile and si.TILE_SOURCES[info["tile_source"]] == "caller"
    assert info["kernel_name"].startswith(f"step_batch_f32_{128 if btile == 1 else 64}x64")
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


def test_batch_vs_oracle_large_instances():
    # A +-1 and a Gaussian instance of at least 2048 spins inside one batch
    # with smaller ones, in the FP32 batch, against the oracle on sampled
    # replicas for the first 10 steps (the window in which FP32 arithmetic
    # stays within 1e-5 of FP64 at this size).
    import torch
    specs = [(2048, "pm1"), (2100, "gauss"), (300, "pm1"), (777, "gauss")]
    announce(f"batch with N >= 2048 instances vs oracle, 10 steps {specs}")
    S, r, steps = 1000, 64, 10
    b, Js, xs = _batch(specs, S, r=r)
    b.run(steps)
    xb, pb, _ = b.state()
    torch.cuda.synchronize()
    dt, zeta = oracle_schedules(S)
    cols = [0, 1, 31, 32, 62, 63]
    for i, (n, kind) in enumerate(specs):
        ref = oracle.run(Js[i].astype(np.float64), xs[i][cols].T.astype(np.float64), None, dt,
                         zeta, qmax=QMAX, n_steps=steps)
        eq = rel_err(xb[i].cpu().numpy()[cols], ref["Q"])
        ep = rel_err(pb[i].cpu().numpy()[cols], ref["P"])
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


def test_batch_energy_paths():
    # The grouped energy of a batch mixing the three cases: +-1 couplings
    # (int8 matrix cores, exact), integer couplings whose sum could pass
    # 2^31 (N^2 max|J| >= 2^31: FP32 path although J is integer) and
    # Gaussian couplings (FP32 path).  Two calls in a row must agree (the
    # integer accumulators are reset by each call).
    import torch
    si = ensure_built()
    announce("batch energy paths: +-1, integer 127 at N=4200, Gaussian")
    r = 8
    Js = [instances.make_pm1(300, 31), 127.0 * instances.make_pm1(4200, 32),
          instances.make_gauss(200, 33)]
    Js = [J.astype(np.float32) for J in Js]
    states = [instances.random_state(J.shape[0], r, 50 + i) for i, J in enumerate(Js)]
    b = si.SpringIsingBatch([to_dev(J) for J in Js], [to_dev(x) for x in states], total_steps=4)
    with pytest.raises(si.SpringIsingError) as err:
        b.energy(exact=True)
    assert err.value.status == si.SI_ERR_UNSUPPORTED
    e1 = [e.cpu().numpy() for e in b.energy(exact=False)]
    e2 = [e.cpu().numpy() for e in b.energy(exact=False)]
    torch.cuda.synchronize()
    for i, J in enumerate(Js):
        n = J.shape[0]
        np.testing.assert_array_equal(e1[i], e2[i])
        ref = oracle.ising_energy(J.astype(np.float64), oracle.spins(states[i].T))
        if i == 0:
            np.testing.assert_array_equal(e1[i], ref)
        else:
            bound = n * 2.0 ** -24 * np.abs(J).astype(np.float64).sum() + 1e-6
            assert np.all(np.abs(e1[i] - ref) <= bound), (i, np.abs(e1[i] - ref).max(), bound)
    b.close()
    # the +-1 instance alone in a batch: exact energies, twice
    b = si.SpringIsingBatch([to_dev(Js[0])], [to_dev(states[0])], total_steps=4)
    ea = b.energy(exact=True)[0].cpu().numpy()
    eb = b.energy(exact=True)[0].cpu().numpy()
    ref = oracle.ising_energy(Js[0].astype(np.float64), oracle.spins(states[0].T))
    np.testing.assert_array_equal(ea, ref)
    np.testing.assert_array_equal(eb, ref)
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


# ---------------------------------------------------------------------------
# Batched precision form: FP8 J for the +-1 instances, hi + lo BF16 J for
# the Gaussian ones, in one grouped launch per step.
# ---------------------------------------------------------------------------
FORM_TILE = {"pm1": ("bf16x_fp8j", 9), "gauss": ("bf16x_hiloj", 7)}


@pytest.mark.parametrize("btile", [1, 2])
def test_bf16_batch_equals_standalone_runs(btile):
    import torch
    si = ensure_built()
    announce(f"BF16 batch (tile {btile}; FP8 / hi+lo per instance) vs standalone runs, bit for bit")
    S = 300
    b, Js, xs = _batch(SIZES, S, precision="bf16x_mixedj", tile=btile)
    assert b.info()["kernel_name"].startswith(f"step_batch_bf16_{128 if btile == 1 else 64}x64")
    b.run(150)
    xb, pb, t = b.state()
    eb = b.energy(exact=False)
    torch.cuda.synchronize()
    assert t == 150
    for i, (n, kind) in enumerate(SIZES):
        form, tile = FORM_TILE[kind]
        m = si.SpringIsing(to_dev(Js[i]), to_dev(xs[i]), total_steps=S, precision=form, tile=tile)
        m.run(150)
        x, p, _ = m.state()
        e = m.energy(exact=False)
        torch.cuda.synchronize()
        assert np.array_equal(x.cpu().numpy(), xb[i].cpu().numpy()), (i, n, kind)
        assert np.array_equal(p.cpu().numpy(), pb[i].cpu().numpy()), (i, n, kind)
        assert np.array_equal(e.cpu().numpy(), eb[i].cpu().numpy()), (i, n, kind)
        m.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16x_mixedj"])
def test_batch_tiny_and_ragged_instances(precision):
    # Degenerate and ragged members: N = 1 (no couplings: q moves with p
    # only), N = 2, N one past a tile edge, and three replicas (R padded to
    # 64).  Each equals its standalone run bit for bit, and the FP32 batch
    # follows the oracle.  An odd step count leaves the state in the second
    # ping-pong buffer, where the spins and energies are then read.
    import torch
    si = ensure_built()
    announce(f"batch of tiny and ragged instances ({precision})")
    specs = [(1, "pm1"), (2, "gauss"), (65, "pm1"), (129, "gauss"), (3, "pm1")]
    r, S, steps = 3, 60, 41
    b, Js, xs = _batch(specs, S, r=r, precision=precision)
    b.run(steps)
    xb, pb, t = b.state()
    eb = b.energy(exact=False)
    sb = b.spins()
    torch.cuda.synchronize()
    assert t == steps
    dt, zeta = oracle_schedules(S)
    for i, (n, kind) in enumerate(specs):
        np.testing.assert_array_equal(sb[i].cpu().numpy().T, oracle.spins(xb[i].cpu().numpy().T))
        form, tile = ("fp32", BATCH_TILE) if precision == "fp32" else FORM_TILE[kind]
        m = si.SpringIsing(to_dev(Js[i]), to_dev(xs[i]), total_steps=S, precision=form, tile=tile)
        m.run(steps)
        x, p, _ = m.state()
        e = m.energy(exact=False)
        torch.cuda.synchronize()
        assert np.array_equal(x.cpu().numpy(), xb[i].cpu().numpy()), (i, n, kind)
        assert np.array_equal(p.cpu().numpy(), pb[i].cpu().numpy()), (i, n, kind)
        assert np.array_equal(e.cpu().numpy(), eb[i].cpu().numpy()), (i, n, kind)
        m.close()
        if precision == "fp32":
            ref = oracle.run(Js[i].astype(np.float64), xs[i].T.astype(np.float64), None, dt, zeta,
                             qmax=QMAX, n_steps=steps)
            assert rel_err(xb[i].cpu().numpy(), ref["Q"]) <= 1e-5, (i, n, kind)
            assert rel_err(pb[i].cpu().numpy(), ref["P"]) <= 1e-5, (i, n, kind)
    b.close()


def test_bf16_batch_one_step_bound():
    # One step from a random state: every instance within the element-wise
    # bound that BF16 positions (and the hi + lo residual of J) allow.
    import torch
    announce("BF16 batch one-step bound vs FP64 oracle")
    S = 100
    specs = SIZES[:4]
    b, Js, _ = _batch(specs, S, precision="bf16x_mixedj")
    xs = [instances.random_state(n, R, 60 + i, scale=1.4) for i, (n, _) in enumerate(specs)]
    ps = [instances.random_state(n, R, 70 + i, scale=1.9) for i, (n, _) in enumerate(specs)]
    b.set_state([to_dev(x) for x in xs], [to_dev(p) for p in ps], 37)
    b.step()
    xb, pb, _ = b.state()
    torch.cuda.synchronize()
    dt, zeta = oracle_schedules(S)
    d, z = float(dt[37]), float(zeta[37])
    for i, (n, kind) in enumerate(specs):
        J64 = Js[i].astype(np.float64)
        Q, P = oracle.step(J64, xs[i].T.astype(np.float64), ps[i].T.astype(np.float64), d, z,
                           qmax=QMAX)
        mag = np.abs(J64) @ np.abs(xs[i].T.astype(np.float64))
        jrel = 2.0 ** -16 if kind == "gauss" else 0.0
        bound = d * z * mag * (2.0 ** -8 + jrel) * 1.01 + 4 * 2.0 ** -24 * (np.abs(P) + 2.0) \
            + d * z * mag * n * 2.0 ** -24
        err = np.abs(pb[i].cpu().numpy().T - P)
        assert np.all(err <= bound), (i, err.max())
        assert np.abs(xb[i].cpu().numpy().T - Q).max() <= 4e-7
        announce(f"  instance {i} N={n} {kind}: max one-step momentum error {err.max():.2e}")
    b.close()


def test_bf16_batch_format_rules():
    si = ensure_built()
    with pytest.raises(si.SpringIsingError) as err:   # Gaussian J is not exact in FP8
        _batch(SIZES[:2], 10, precision="bf16x_fp8j")
    assert err.value.status == si.SI_ERR_UNSUPPORTED
    with pytest.raises(si.SpringIsingError) as err:   # no batched form
        _batch(SIZES[:2], 10, precision="bf16x3_exactj")
    assert err.value.status == si.SI_ERR_UNSUPPORTED
    b, _, _ = _batch(SIZES[:2], 10, precision="bf16x_hiloj")  # hi + lo for every instance
    b.run(10)
    b.close()


def test_bf16_batch_full_workload_vs_fp32():
    # The 256-instance workload in both forms for 3000 steps: per-instance
    # final energies agree in distribution (z-scores of the mean difference
    # over 64 replicas behave like a standard normal sample), and the BF16
    # batch is faster per step.
    import time

    import torch
    si = ensure_built()
    announce("256-instance batch, FP32 vs BF16 (FP8 / hi+lo), 3000 steps")
    S = 3000
    recipe = instances.make_batch(256, 0)
    dev = torch.device("cuda:0")
    Js = [instances.make_J_torch(n, kind, seed, dev) for n, kind, seed in recipe]
    xs = [instances.make_x0_torch(n, R, seed, device=dev) for n, kind, seed in recipe]
    torch.cuda.synchronize()
    res = {}
    for form in ("fp32", "bf16x_mixedj"):
        b = si.SpringIsingBatch(Js, xs, total_steps=S, precision=form)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.run(S)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        e = [v.cpu().numpy().astype(np.float64) for v in b.energy(exact=False)]
        res[form] = (e, el / S)
        announce(f"  {form} ({b.info()['kernel_name']}): {1e3 * el / S:.3f} ms/step")
        b.close()
    del Js, xs
    z = []
    for e32, elp in zip(res["fp32"][0], res["bf16x_mixedj"][0]):
        se = np.sqrt(e32.var() / R + elp.var() / R)
        z.append((elp.mean() - e32.mean()) / se if se > 0 else 0.0)
    z = np.array(z)
    announce(f"  per-instance z of mean final energy: mean {z.mean():+.3f}, sd {z.std():.3f}, "
             f"max |z| {np.abs(z).max():.2f}")
    assert abs(z.mean()) < 0.35 and z.std() < 1.4 and (np.abs(z) > 4).mean() < 0.02
    assert res["bf16x_mixedj"][1] < res["fp32"][1]


@pytest.mark.parametrize("precision", ["fp32", "bf16x_mixedj"])
def test_batch_autotune_fills_the_tile_cache(precision, tmp_path):
    import torch
    si = ensure_built()
    announce(f"batch autotune and tile cache ({precision})")
    si.spring_ising_tile_cache_clear()
    S = 60
    specs = SIZES[:4]
    b, Js, xs = _batch(specs, S, precision=precision)
    assert si.TILE_SOURCES[b.info()["tile_source"]] == "table" and b.info()["tile"] == 1
    b.run(10)
    tile, us = b.autotune(4)
    assert tile in (1, 2) and us > 0
    info = b.info()
    assert info["tile"] == tile and si.TILE_SOURCES[info["tile_source"]] == "autotune"
    assert info["t"] == 10
    b.run(20)
    xb, pb, t = b.state()
    torch.cuda.synchronize()
    # the state was restored after every candidate: same as an untuned run
    ref, _, _ = _batch(specs, S, precision=precision, tile=1)
    ref.run(30)
    xr, pr, _ = ref.state()
    torch.cuda.synchronize()
    for i in range(len(specs)):
        assert np.array_equal(xb[i].cpu().numpy(), xr[i].cpu().numpy()), i
        assert np.array_equal(pb[i].cpu().numpy(), pr[i].cpu().numpy()), i
    ref.close()
    # a new batch of the same key starts on the cached tile
    b2, _, _ = _batch(specs, S, precision=precision)
    assert b2.info()["tile"] == tile and si.TILE_SOURCES[b2.info()["tile_source"]] == "cache"
    b2.close()
    # the cache survives a save / clear / load round trip
    path = tmp_path / "tiles.txt"
    si.spring_ising_tile_cache_save(str(path))
    si.spring_ising_tile_cache_clear()
    b3, _, _ = _batch(specs, S, precision=precision)
    assert si.TILE_SOURCES[b3.info()["tile_source"]] == "table"
    b3.close()
    assert si.spring_ising_tile_cache_load(str(path)) == 1
    b4, _, _ = _batch(specs, S, precision=precision)
    assert b4.info()["tile"] == tile and si.TILE_SOURCES[b4.info()["tile_source"]] == "cache"
    b4.close()
    b.close()
    si.spring_ising_tile_cache_clear()


@pytest.mark.parametrize("precision,btile", [("fp32", 1), ("bf16x_mixedj", 2)])
def test_batch_timeline(precision, btile):
    import torch
    si = ensure_built()
    announce(f"batch timeline ({precision}, tile {btile})")
    S = 40
    b, Js, xs = _batch(SIZES, S, precision=precision, tile=btile)
    b.run(5)
    rec, mhz = b.timeline(3)
    xb, pb, t = b.state()
    torch.cuda.synchronize()
    assert t == 8 and mhz > 0
    rows = 128 if btile == 1 else 64
    n_items = sum(((n + 127) // 128 * 128) // rows for n, _ in SIZES)
    assert rec.shape == (3 * n_items, 4)
    steps = (rec[:, 3] >> np.uint64(32)).astype(np.int64)
    items = (rec[:, 3] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    ends = []
    for s in range(3):
        m = steps == s
        assert np.array_equal(np.sort(items[m]), np.arange(n_items)), s
        assert np.all(rec[m, 1] >= rec[m, 0])
        if ends:
            assert rec[m, 0].min() >= ends[-1]  # stream order: steps do not overlap
        ends.append(rec[m, 1].max())
    assert len(np.unique(rec[:, 2])) <= 256
    stats = si.batch_timeline_stats(rec, mhz)
    assert len(stats) == 3 and all(0 < st["cu_busy_mean"] <= 1 for st in stats)
    # traced steps are ordinary steps
    ref, _, _ = _batch(SIZES, S, precision=precision, tile=btile)
    ref.run(8)
    xr, pr, _ = ref.state()
    torch.cuda.synchronize()
    for i in range(len(SIZES)):
        assert np.array_equal(xb[i].cpu().numpy(), xr[i].cpu().numpy()), i
        assert np.array_equal(pb[i].cpu().numpy(), pr[i].cpu().numpy()), i
    # argument rules
    with pytest.raises(si.SpringIsingError) as e:
        b.timeline(17)
    assert e.value.status == si.SI_ERR_INVALID
    b.run(S - 8)
    with pytest.raises(si.SpringIsingError) as e:
        b.timeline(1)
    assert e.value.status == si.SI_ERR_RANGE
    m = si.SpringIsing(to_dev(Js[0]), to_dev(xs[0]), total_steps=S)
    with pytest.raises(si.SpringIsingError) as e:
        si.spring_ising_batch_timeline(m.ctx, 1)
    assert e.value.status == si.SI_ERR_UNSUPPORTED
    m.close()
    ref.close()
    b.close()


@pytest.mark.parametrize("precision,btile", [("fp32", 1), ("fp32", 2), ("bf16x_mixedj", 1)])
def test_batch_with_several_replica_tiles(precision, btile):
    # R = 130 pads to three 64-replica column tiles: every instance has items
    # in several columns, dealt to its XCD queue together
    import torch
    si = ensure_built()
    announce(f"batch with R = 130 ({precision}, tile {btile}) vs standalone runs")
    specs = [(300, "pm1"), (129, "gauss"), (64, "pm1"), (1000, "gauss"), (520, "pm1")]
    r, S = 130, 40
    b, Js, xs = _batch(specs, S, r=r, precision=precision, tile=btile)
    b.run(S)
    xb, pb, t = b.state()
    torch.cuda.synchronize()
    assert t == S
    for i, (n, kind) in enumerate(specs):
        if precision == "fp32":
            m = si.SpringIsing(to_dev(Js[i]), to_dev(xs[i]), total_steps=S, tile=BATCH_TILE)
        else:
            form, tile = FORM_TILE[kind]
            m = si.SpringIsing(to_dev(Js[i]), to_dev(xs[i]), total_steps=S, precision=form,
                               tile=tile)
        m.run(S)
        x, p, _ = m.state()
        torch.cuda.synchronize()
        assert np.array_equal(x.cpu().numpy(), xb[i].cpu().numpy()), (i, n, kind)
        assert np.array_equal(p.cpu().numpy(), pb[i].cpu().numpy()), (i, n, kind)
        m.close()
    b.close()
