"""Runtime features: HIP-graph replay of run(), the autotuner, kernel naming."""
import numpy as np
import pytest

import oracle
from paper_2305_07187_amd import instances

from gpu_common import QMAX, announce, ensure_built, oracle_schedules, rel_err, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp32", "bf16x_fp8j", "bf16x3_exactj"])
def test_graph_replays_match_direct_launches(precision):
    import torch
    si = ensure_built()
    announce(f"graph replay vs direct launches ({precision})")
    n, r, S = 500, 128, 400
    J = to_dev(instances.make_pm1(n, 2))
    x0 = to_dev(instances.make_x0(n, r, 2))
    direct = si.SpringIsing(J, x0, total_steps=S, precision=precision)
    direct.run(S)
    xd, pd, _ = direct.state()
    ed = direct.energy()
    torch.cuda.synchronize()
    g = si.SpringIsing(J, x0, total_steps=S, precision=precision)
    g.set_graph(50)
    assert g.info()["graph_steps"] == 50
    for rep in range(3):
        g.set_state(x0, None, 0)
        g.run(S)
        xg, pg, t = g.state()
        eg = g.energy()           # eager work between replays
        torch.cuda.synchronize()
        assert t == S
        assert torch.equal(xg, xd) and torch.equal(pg, pd) and torch.equal(eg, ed), rep
    # a different start and length is captured separately
    g.set_state(x0, None, 0)
    g.run(150)
    g.run(S - 150)
    xg, _, _ = g.state()
    torch.cuda.synchronize()
    assert torch.equal(xg, xd)
    direct.close()
    g.close()


def test_graph_on_batch():
    import torch
    si = ensure_built()
    announce("graph replay on a batch")
    specs = [(64, "pm1"), (300, "gauss"), (129, "pm1")]
    Js = [to_dev(instances.make_J(n, k, i)) for i, (n, k) in enumerate(specs)]
    xs = [to_dev(instances.make_x0(n, 64, i)) for i, (n, k) in enumerate(specs)]
    a = si.SpringIsingBatch(Js, xs, total_steps=100)
    a.run(100)
    xa, pa, _ = a.state()
    ea = a.energy()
    b = si.SpringIsingBatch(Js, xs, total_steps=100)
    b.set_graph(10)
    for rep in range(3):
        # restarts of the schedule replay the graph captured by the first run
        b.set_state(xs, None, 0)
        b.run(100)
        xb, pb, t = b.state()
        eb = b.energy()  # eager work between replays
        torch.cuda.synchronize()
        assert t == 100
        for u, v in zip(xa + pa + ea, xb + pb + eb):
            assert torch.equal(u, v), rep
    a.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16x_bf16j"])
def test_autotune_keeps_state_and_parity(precision):
    import torch
    si = ensure_built()
    announce(f"autotune ({precision})")
    n, r, S = 100, 8, 1000
    Jn = instances.make_pm1(n, 0)
    x0n = instances.make_x0(n, r, 0)
    m = si.SpringIsing(to_dev(Jn), to_dev(x0n), total_steps=S, precision=precision)
    m.run(3)
    x_before, p_before, t_before = m.state()
    tile, us = m.autotune(5)
    x_after, p_after, t_after = m.state()
    torch.cuda.synchronize()
    info = m.info()
    announce(f"  chose tile {tile} ({info['kernel_name']}) at {us:.2f} us/step")
    assert info["tile"] == tile and us > 0
    assert t_after == t_before == 3
    assert torch.equal(x_before, x_after) and torch.equal(p_before, p_after)
    assert si.TILE_SOURCES[info["tile_source"]] == "autotune"
    # later contexts of the same key (precision, N-bucket, R) start on the
    # tuned tile; N = 120 shares N = 100's bucket (64, 128]
    for nn in (100, 120):
        m2 = si.SpringIsing(to_dev(instances.make_pm1(nn, 1)), to_dev(instances.make_x0(nn, r, 1)),
                            total_steps=S, precision=precision)
        assert m2.info()["tile"] == tile, nn
        assert si.TILE_SOURCES[m2.info()["tile_source"]] == "cache", nn
        m2.close()
    m3 = si.SpringIsing(to_dev(instances.make_pm1(200, 1)), to_dev(instances.make_x0(200, r, 1)),
                        total_steps=S, precision=precision)
    assert si.TILE_SOURCES[m3.info()["tile_source"]] == "table"  # another bucket
    m3.close()
    if precision == "fp32":
        m.run(47)
        x, _, _ = m.state()
        torch.cuda.synchronize()
        dt, zeta = oracle_schedules(S)
        ref = oracle.run(Jn.astype(np.float64), x0n.T.astype(np.float64), None, dt, zeta,
                         qmax=QMAX, n_steps=50)
        assert rel_err(x.cpu().numpy(), ref["Q"]) <= 1e-5
    m.close()


def test_library_loaded_before_torch():
    # A fresh process that loads the library before it imports torch itself
    # (torch ships its own HIP runtime; the binding loads it first so that
    # torch's device pointers are recognised).
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_2305_07187_amd import spring_ising as si\n"
        "si.load_library()\n"
        "import numpy as np, torch\n"
        "from paper_2305_07187_amd import instances\n"
        "J = torch.from_numpy(instances.make_pm1(64, 0)).cuda()\n"
        "x = torch.from_numpy(instances.make_x0(64, 4, 0)).cuda()\n"
        "m = si.SpringIsing(J, x, total_steps=10)\n"
        "m.run(10); print('ok', m.energy().cpu().numpy().tolist())\n" % root)
    announce("library loaded before torch, fresh process")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=180)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout[-500:] + r.stderr[-2000:]


def test_c_program_runs(tmp_path):
    # The C ABI without Python or torch: tests/c_abi_demo.c allocates with
    # the HIP runtime, steps a +-1 instance and checks the exact energies of
    # the spins it reads back against Eq. (1) on the host.
    import subprocess
    from c_demo import build_c_demo
    exe = tmp_path / "c_abi_demo"
    ok, msg = build_c_demo(exe)
    assert ok, msg
    announce("C program through the C ABI")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    announce("  " + r.stdout.strip())
    assert r.returncode == 0 and "match" in r.stdout, r.stdout + r.stderr



def test_kernel_names_match_tile_tables_and_traffic_keys():
    # Every tile id the library accepts reports the kernel name that its
    # tile table spells out, and every counter-measured traffic entry of the
    # benchmark names a kernel the library runs for that form.
    import importlib.util
    import os
    import re

    si = ensure_built()
    announce("kernel names of every tile id, against the tile tables and the traffic keys")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_names", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    n, r = 256, 128
    J = to_dev(instances.make_pm1(n, 5))
    x0 = to_dev(instances.make_x0(n, r, 5))
    seen = {}
    for prec in ("fp32", "bf16x_fp8j", "bf16x_bf16j", "bf16x_hiloj", "bf16x3_exactj"):
        names = set()
        for tile in range(1, 64):
            try:
                m = si.SpringIsing(J, x0, total_steps=2, precision=prec, tile=tile)
            except si.SpringIsingError as e:
                assert e.status == si.SI_ERR_INVALID, (prec, tile, e)
                continue
            name = m.info()["kernel_name"]
            assert m.info()["tile"] == tile
            m.close()
            pat = r"step_f32_\d+x\d+_w\dx\d_mfma\d+_k\d+_s\d_a\d" if prec == "fp32" else \
                r"step_bf16_\d+x\d+_w\dx\d_k\d+_s\d(_p[12])?"
            assert re.fullmatch(pat, name), (prec, tile, name)
            names.add(name)
        assert names, prec
        seen[prec] = names
    for (kernel, form, _, _), _ in bench.MEASURED_TRAFFIC_BYTES.items():
        assert kernel in seen[form], (kernel, form)


def test_set_field_invalidates_captured_graphs():
    # A captured run(n) holds the field pointer in its kernel arguments:
    # changing the field must drop the graphs, so that a replay after a
    # rewind uses the new field exactly like direct launches do.
    import torch
    si = ensure_built()
    announce("set_field after a graph capture: graphs dropped")
    n, r, S = 200, 64, 120
    J = to_dev(instances.make_pm1(n, 7))
    x0 = to_dev(instances.make_x0(n, r, 7))
    h = to_dev(np.linspace(-1.0, 1.0, n).astype(np.float32))

    def sequence(graph):
        m = si.SpringIsing(J, x0, total_steps=S)
        if graph:
            m.set_graph(10)
        m.run(60)                     # captured (graph on) with no field
        m.set_field(h)
        m.set_state(x0, None, 0)
        m.run(60)                     # same key (t0 = 0, 60 steps): must see the field
        x1, p1, _ = m.state()
        m.set_field(None)
        m.set_state(x0, None, 0)
        m.run(60)                     # and again without it
        x2, p2, _ = m.state()
        torch.cuda.synchronize()
        m.close()
        return x1, p1, x2, p2

    direct = sequence(False)
    graphed = sequence(True)
    for a, b in zip(direct, graphed):
        assert torch.equal(a, b)
    # the field made a difference (the test would be void otherwise)
    assert not torch.equal(direct[0], direct[2])


@pytest.mark.parametrize("after", [1, 3])
def test_injected_hip_failure_poisons_context(after):
    # The test hook makes the n-th checked HIP call report a failure
    # although the call succeeded: that call returns SI_ERR_HIP, every later
    # call other than destroy SI_ERR_STATE.  No device operation is altered.
    import torch
    si = ensure_built()
    announce(f"injected HIP failure after {after} checked calls")
    n, r = 64, 8
    m = si.SpringIsing(to_dev(instances.make_pm1(n, 1)), to_dev(instances.make_x0(n, r, 1)),
                       total_steps=100)
    with pytest.raises(si.SpringIsingError) as e:
        si.spring_ising_debug_inject_hip_error(m.ctx, -1)
    assert e.value.status == si.SI_ERR_INVALID
    si.spring_ising_debug_inject_hip_error(m.ctx, 0)   # cancel: nothing pending
    m.run(5)
    si.spring_ising_debug_inject_hip_error(m.ctx, after)
    with pytest.raises(si.SpringIsingError) as e:
        m.run(10)                     # ten step launches: the after-th reports failure
    assert e.value.status == si.SI_ERR_HIP, e.value
    for call in (lambda: m.run(1), lambda: m.energy(), lambda: m.state(),
                 lambda: m.autotune(2), lambda: m.set_graph(5)):
        with pytest.raises(si.SpringIsingError) as e:
            call()
        assert e.value.status == si.SI_ERR_STATE
    torch.cuda.synchronize()
    m.close()                         # destroy still works
    # other contexts are unaffected
    m2 = si.SpringIsing(to_dev(instances.make_pm1(n, 1)), to_dev(instances.make_x0(n, r, 1)),
                        total_steps=10)
    m2.run(10)
    m2.energy()
    torch.cuda.synchronize()
    m2.close()


def test_autotune_failure_after_launch_poisons_context():
    # A failure after a candidate has been launched is not skipped: the
    # autotuner returns SI_ERR_HIP and the context stays poisoned.
    si = ensure_built()
    announce("autotune: a failure after launch poisons the context")
    n, r = 256, 128
    m = si.SpringIsing(to_dev(instances.make_pm1(n, 3)), to_dev(instances.make_x0(n, r, 3)),
                       total_steps=100)
    si.spring_ising_debug_inject_hip_error(m.ctx, 12)
    with pytest.raises(si.SpringIsingError) as e:
        m.autotune(3)
    assert e.value.status == si.SI_ERR_HIP
    with pytest.raises(si.SpringIsingError) as e:
        m.run(1)
    assert e.value.status == si.SI_ERR_STATE
    m.close()


def test_batch_initial_momenta():
    # init_batch takes per-instance initial momenta (NULL entries are zero):
    # every instance equals its single-instance run from the same (x0, p0)
    # on the tile whose contraction order the batch uses (FP32: tile 14).
    import torch
    si = ensure_built()
    announce("batch with initial momenta vs single-instance runs")
    specs = [(96, "pm1"), (200, "gauss"), (130, "pm1")]
    r, S = 64, 40
    Js = [to_dev(instances.make_J(n, k, 20 + i)) for i, (n, k) in enumerate(specs)]
    xs = [to_dev(instances.make_x0(n, r, 20 + i)) for i, (n, k) in enumerate(specs)]
    ps = [to_dev(0.5 * instances.make_x0(specs[0][0], r, 40)), None,
          to_dev(-0.3 * instances.make_x0(specs[2][0], r, 60))]
    b = si.SpringIsingBatch(Js, xs, total_steps=S, p0s=ps)
    b.run(S)
    xb, pb, _ = b.state()
    for i in range(len(specs)):
        m = si.SpringIsing(Js[i], xs[i], ps[i], total_steps=S, tile=14)
        m.run(S)
        x, p, _ = m.state()
        torch.cuda.synchronize()
        assert torch.equal(x, xb[i]) and torch.equal(p, pb[i]), i
        m.close()
    b.close()
