"""FP64 CPU oracle for the Spring-Ising hot path -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, obviously correct restatement of the paper's
method (arXiv 2305.07187) in float64 NumPy, used to check the HIP path.  Only
the test suite, the smoke check and the benchmark's CPU-baseline leg may
import it; the product path never does, and it shares no code with the HIP
library (inputs come from the separate seeded generator module).

Contents
  spring_ising  Eq. (1) energy, MAX-CUT readout, the zeta(t) schedule, the
                Eq. (8) iteration with the walls of Eq. (6), and variants.
  bruteforce    exhaustive 2^N ground-state search for small N.
  adjoint       reverse-mode gradient of the relaxed end-energy with respect
                to the per-step time-step and zeta schedules.

Every function is pinned by CPU tests against brute force, closed forms,
exact rational replays and finite differences, never against itself.
"""
from .spring_ising import (  # noqa: F401
    PAPER,
    cut_value,
    hamiltonian,
    ising_energy,
    ising_energy_pairs,
    relaxed_energy,
    run,
    spins,
    step,
    zeta_schedule,
    dt_schedule,
)
from .bruteforce import ground_state_bruteforce  # noqa: F401
from .adjoint import relaxed_energy_grad, relaxed_energy_grad_along  # noqa: F401
