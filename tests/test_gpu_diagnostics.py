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
