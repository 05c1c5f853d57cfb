"""The allocation-free energy entry point against the context-based one.

spring_ising_energy_noalloc takes caller-owned J and positions and keeps its
scratch in a static device array; its energies must equal, bit for bit,
those of spring_ising_energy on a context holding the same couplings and
positions, on two calls in a row (the second smaller, so that what the
first left in the shared scratch must not leak into it)."""
import numpy as np
import pytest

from paper_2305_07187_amd import instances

from gpu_common import announce, ensure_built, to_dev

pytestmark = pytest.mark.gpu


def _reference(si, J, x):
    """Energies of sign(x) from the context-based entry point."""
    import torch
    m = si.SpringIsing(J, x, total_steps=1)
    e = m.energy(exact=True)
    torch.cuda.synchronize()
    m.close()
    return e


def test_noalloc_energy_matches_context_energy_twice():
    import torch
    si = ensure_built()
    cases = [(300, 100, 0, 40), (70, 9, 1, 25)]   # second call smaller in n and r
    for n, r, seed, steps in cases:
        announce(f"energy_noalloc vs energy: N={n} R={r} seed={seed}")
        J = to_dev(instances.make_pm1(n, seed))
        x0 = to_dev(instances.make_x0(n, r, seed))
        m = si.SpringIsing(J, x0, total_steps=steps)
        m.run(steps)                       # positions of a real trajectory
        x, _, _ = m.state()
        e_ctx = m.energy(exact=True)
        m.close()
        e = torch.full((r,), 12345, dtype=torch.int32, device="cuda:0")
        si.spring_ising_energy_noalloc(J, x, e)
        torch.cuda.synchronize()
        assert torch.equal(e, e_ctx), (n, r)
        assert torch.equal(_reference(si, J, x), e)


def test_noalloc_energy_integer_couplings_and_ragged_shapes():
    import torch
    si = ensure_built()
    rng = np.random.default_rng(5)
    for n, r in [(1, 1), (65, 3), (129, 130), (64, 64)]:
        announce(f"energy_noalloc, integer couplings in [-127, 127]: N={n} R={r}")
        A = rng.integers(-127, 128, size=(n, n)).astype(np.float32)
        Jn = np.triu(A, 1)
        Jn = Jn + Jn.T
        J = to_dev(Jn)
        x = to_dev(rng.uniform(-1, 1, size=(r, n)).astype(np.float32))
        e = torch.empty(r, dtype=torch.int32, device="cuda:0")
        si.spring_ising_energy_noalloc(J, x, e)
        torch.cuda.synchronize()
        assert torch.equal(e, _reference(si, J, x)), (n, r)


def test_noalloc_energy_rejects_and_flags():
    import torch
    si = ensure_built()
    announce("energy_noalloc: size limits, host pointers, non-integer couplings")
    n, r = 40, 5
    J = to_dev(instances.make_pm1(n, 2))
    x = to_dev(instances.make_x0(n, r, 2))
    e = torch.empty(r, dtype=torch.int32, device="cuda:0")
    lib = si.load_library()
    import ctypes
    # more replicas than the static scratch holds
    big = torch.empty(70000, dtype=torch.int32, device="cuda:0")
    st = lib.spring_ising_energy_noalloc(n, 70000, ctypes.c_void_p(J.data_ptr()),
                                         ctypes.c_void_p(x.data_ptr()),
                                         ctypes.c_void_p(big.data_ptr()), None)
    assert st == si.SI_ERR_INVALID and "65536" in si.last_error()
    st = lib.spring_ising_energy_noalloc(70000, r, ctypes.c_void_p(J.data_ptr()),
                                         ctypes.c_void_p(x.data_ptr()),
                                         ctypes.c_void_p(e.data_ptr()), None)
    assert st == si.SI_ERR_INVALID
    host = np.zeros(r, dtype=np.int32)
    st = lib.spring_ising_energy_noalloc(n, r, ctypes.c_void_p(J.data_ptr()),
                                         ctypes.c_void_p(x.data_ptr()),
                                         host.ctypes.data_as(ctypes.c_void_p), None)
    assert st == si.SI_ERR_INVALID
    # a coupling that is not an integer: every entry is the sentinel
    Jh = J.clone()
    Jh[3, 7] = Jh[7, 3] = 0.5
    si.spring_ising_energy_noalloc(Jh, x, e)
    torch.cuda.synchronize()
    assert bool((e == torch.iinfo(torch.int32).min).all())
    # and the next valid call is clean again
    si.spring_ising_energy_noalloc(J, x, e)
    torch.cuda.synchronize()
    assert torch.equal(e, _reference(si, J, x))
