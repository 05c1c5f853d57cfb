"""In-run best-state tracking and the Eq. (7) Hamiltonian diagnostic."""
import numpy as np
import pytest

import oracle
from paper_2305_07187_amd import instances

from gpu_common import QMAX, announce, ensure_built, oracle_schedules, to_dev

pytestmark = pytest.mark.gpu


def test_hamiltonian_matches_oracle():
    import torch
    si = ensure_built()
    announce("Eq. (7) Hamiltonian vs oracle")
    n, r, S = 300, 40, 100
    J = instances.make_pm1(n, 4)
    x = instances.random_state(n, r, 5, scale=1.4)
    p = instances.random_state(n, r, 6, scale=1.9)
    h = np.random.default_rng(0).integers(-2, 3, n).astype(np.float32)
    m = si.SpringIsing(to_dev(J), to_dev(instances.make_x0(n, r, 0)), total_steps=S)
    m.set_state(to_dev(x), to_dev(p), 17)
    m.set_field(to_dev(h))
    H = m.hamiltonian().cpu().numpy()
    torch.cuda.synchronize()
    _, zeta = oracle_schedules(S)
    Ho = oracle.hamiltonian(J.astype(np.float64), x.T.astype(np.float64), p.T.astype(np.float64),
                            float(zeta[17]), h=h.astype(np.float64))
    # FP32 row products of +-1 couplings and FP32 per-tile sums
    bound = 1e-5 * (np.abs(Ho) + n * 3.0)
    assert np.all(np.abs(H - Ho) <= bound), np.abs(H - Ho).max()
    m.close()


def test_best_state_tracking():
    import torch
    si = ensure_built()
    announce("best-state tracking")
    n, r, S, every = 200, 16, 1000, 25
    J = instances.make_pm1(n, 8)
    m = si.SpringIsing(to_dev(J), to_dev(instances.make_x0(n, r, 8)), total_steps=S)
    with pytest.raises(si.SpringIsingError):
        m.best()
    running = np.full(r, np.inf)
    for _ in range(S // every):
        m.run(every)
        m.update_best()
        running = np.minimum(running, m.energy().cpu().numpy().astype(np.float64))
    be, bs = m.best()
    torch.cuda.synchronize()
    be = be.cpu().numpy()
    np.testing.assert_array_equal(be, running)
    # the stored spins have the stored energy (Eq. (1) on the generator's J)
    np.testing.assert_array_equal(oracle.ising_energy(J, bs.cpu().numpy().T.astype(np.int64)), be)
    e_final = m.energy().cpu().numpy()
    assert np.all(be <= e_final)
    announce(f"  best-along-run mean {be.mean():.1f} vs final mean {e_final.mean():.1f}")
    m.close()


def _chunked_energies(si, make, S, every, exact):
    """Reference for the in-run checks: the same run in chunks of `every`
    steps with an explicit energy call after each chunk (no in-run checks)."""
    import torch
    m = make(0)
    rows = []
    for _ in range(S // every):
        m.run(every)
        rows.append(m.energy(exact=exact).double())
    torch.cuda.synchronize()
    m.close()
    return torch.stack(rows)


@pytest.mark.parametrize("precision,kind", [("fp32", "pm1"), ("bf16x_fp8j", "pm1"),
                                            ("fp32", "gauss"), ("bf16x_hiloj", "gauss")])
def test_in_run_energy_checks_match_explicit_energies(precision, kind):
    # With energy_every = E the library records, after every E-th step and on
    # the stream, the energies of all replicas and updates the best state.
    # The trace equals explicit energy calls at the same steps, bit for bit
    # (same kernels), and the best record equals the running minimum.
    import torch
    si = ensure_built()
    announce(f"in-run energy checks ({precision}, {kind} couplings)")
    n, r, S, every = 300, 64, 400, 25
    Jn = instances.make_J(n, kind, 11)
    J, x0 = to_dev(Jn), to_dev(instances.make_x0(n, r, 11))
    make = lambda e: si.SpringIsing(J, x0, total_steps=S, precision=precision, energy_every=e)
    exact = kind == "pm1"
    ref = _chunked_energies(si, make, S, every, exact)
    m = make(every)
    assert m.energy_trace().shape == (0, r)
    m.run(130)
    m.run(S - 130)                     # checks do not depend on run() boundaries
    tr = m.energy_trace()
    be, bs = m.best()
    torch.cuda.synchronize()
    assert tr.shape == (S // every, r)
    assert torch.equal(tr, ref)
    assert torch.equal(be, tr.min(dim=0).values)
    if exact:   # the recorded spins carry the recorded energies (Eq. (1) on the host)
        np.testing.assert_array_equal(
            oracle.ising_energy(Jn, bs.cpu().numpy().T.astype(np.int64)), be.cpu().numpy())
    # a rewind resets the record and the row count
    m.set_state(x0, None, 0)
    with pytest.raises(si.SpringIsingError) as e:
        m.best()
    assert e.value.status == si.SI_ERR_STATE
    m.run(60)
    tr2 = m.energy_trace()
    be2, _ = m.best()
    torch.cuda.synchronize()
    assert tr2.shape == (2, r) and torch.equal(tr2, ref[:2])
    assert torch.equal(be2, ref[:2].min(dim=0).values)
    m.close()


def test_in_run_checks_inside_captured_graphs():
    # The checks are launched with the steps, so captured launch sequences
    # contain them; the best record's reset is a device flag, so a replay
    # after a rewind starts a fresh record exactly as direct launches do.
    import torch
    si = ensure_built()
    announce("in-run checks inside captured graphs")
    n, r, S, every = 256, 64, 200, 20
    J, x0 = to_dev(instances.make_pm1(n, 12)), to_dev(instances.make_x0(n, r, 12))
    d = si.SpringIsing(J, x0, total_steps=S, energy_every=every)
    d.run(S)
    trd, (bed, bsd) = d.energy_trace(), d.best()
    g = si.SpringIsing(J, x0, total_steps=S, energy_every=every)
    g.set_graph(50)
    for rep in range(3):
        g.set_state(x0, None, 0)
        g.run(100)
        g.run(100)
        g.energy()                   # eager work between replays
        tr, (be, bs) = g.energy_trace(), g.best()
        torch.cuda.synchronize()
        assert torch.equal(tr, trd) and torch.equal(be, bed) and torch.equal(bs, bsd), rep
    d.close()
    g.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16x_mixedj"])
def test_in_run_checks_on_a_batch(precision):
    import torch
    si = ensure_built()
    announce(f"in-run checks on a batch ({precision})")
    specs = [(100, "pm1"), (260, "gauss"), (64, "pm1"), (130, "gauss")]
    r, S, every = 64, 120, 30
    Jn = [instances.make_J(n, k, 30 + i) for i, (n, k) in enumerate(specs)]
    Js = [to_dev(a) for a in Jn]
    xs = [to_dev(instances.make_x0(n, r, 30 + i)) for i, (n, k) in enumerate(specs)]
    ref = si.SpringIsingBatch(Js, xs, total_steps=S, precision=precision)
    rows = []
    for _ in range(S // every):
        ref.run(every)
        rows.append(torch.stack(ref.energy(exact=False)))
    ref.close()
    b = si.SpringIsingBatch(Js, xs, total_steps=S, precision=precision, energy_every=every)
    b.set_graph(S)
    b.run(S)
    tr = b.energy_trace()
    be, bs = b.best()
    torch.cuda.synchronize()
    assert torch.equal(tr, torch.stack(rows))
    for i, (n, kind) in enumerate(specs):
        assert torch.equal(be[i], tr[:, i, :].min(dim=0).values), i
        if kind == "pm1":
            np.testing.assert_array_equal(
                oracle.ising_energy(Jn[i], bs[i].cpu().numpy().T.astype(np.int64)),
                be[i].cpu().numpy())
    b.close()


def test_in_run_checks_with_a_partial_last_interval():
    # S not a multiple of E: checks at E, 2E, ... <= S only; E > S: no check
    import torch
    si = ensure_built()
    announce("in-run energy checks with S % E != 0 and E > S")
    n, r = 200, 8
    J, x0 = to_dev(instances.make_pm1(n, 12)), to_dev(instances.make_x0(n, r, 12))
    S, every = 107, 25
    m = si.SpringIsing(J, x0, total_steps=S, energy_every=every)
    m.run(S)
    tr = m.energy_trace()
    ref = si.SpringIsing(J, x0, total_steps=S)
    rows = []
    for k in range(S // every):
        ref.run(every)
        rows.append(ref.energy(exact=True).double())
    torch.cuda.synchronize()
    assert tr.shape == (S // every, r)
    assert torch.equal(tr, torch.stack(rows))
    ref.close()
    m.close()
    m = si.SpringIsing(J, x0, total_steps=S, energy_every=S + 1)
    m.run(S)
    assert m.energy_trace().shape == (0, r)
    with pytest.raises(si.SpringIsingError) as e:
        m.best()
    assert e.value.status == si.SI_ERR_STATE
    m.close()
