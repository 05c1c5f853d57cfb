"""Exhaustive ground-state search -- test infrastructure (oracle).

Enumerates all 2^N spin vectors of Eq. (1) (N <= 22) and returns the lowest
energy.  The energy of every state is the plain pair sum over i < j, so this
pins both the ground state and the energy definition on small instances.
"""
from __future__ import annotations

import numpy as np


def all_states(n: int, start: int, stop: int) -> np.ndarray:
    """Spin vectors for integers start..stop-1: bit i set -> s_i = -1."""
    idx = np.arange(start, stop, dtype=np.int64)[:, None]
    bits = (idx >> np.arange(n, dtype=np.int64)[None, :]) & 1
    return (1 - 2 * bits).astype(np.int64)


def ground_state_bruteforce(J, h=None, chunk: int = 1 << 16):
    """Return (E_min, s_min, energies) over all 2^N states.

    ``energies`` holds the energy of state index x (bit i -> s_i = -1) for
    every x, so callers can check degeneracies and identities.  Integer J
    gives exact int64 energies.
    """
    J = np.asarray(J, dtype=np.float64)
    n = J.shape[0]
    if n > 22:
        raise ValueError("brute force is limited to N <= 22")
    integer = bool(np.all(J == np.round(J))) and (h is None or np.all(np.asarray(h) == np.round(h)))
    dt = np.int64 if integer else np.float64
    U = np.triu(J, 1).astype(dt)
    hv = None if h is None else np.asarray(h, dtype=np.float64).astype(dt)
    total = 1 << n
    energies = np.empty(total, dtype=dt)
    for a in range(0, total, chunk):
        b = min(total, a + chunk)
        S = all_states(n, a, b).astype(dt)  # [B, N]
        e = -np.einsum("bi,ij,bj->b", S, U, S)
        if hv is not None:
            e = e - S @ hv
        energies[a:b] = e
    x = int(np.argmin(energies))
    s = all_states(n, x, x + 1)[0].astype(np.int8)
    return energies[x], s, energies
