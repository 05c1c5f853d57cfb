"""Spring-Ising iteration in float64 -- test infrastructure (oracle).

Plain restatement of the paper (arXiv 2305.07187):
  * Ising energy, Eq. (1) of "Spring vibration model":
        H = - sum_{i<j} J_ij s_i s_j - sum_i h_i s_i
  * equations of motion, Eq. (4) with origin q0 = 0, discretised as the
    "iterative formula", Eq. (5), restated with the dynamic-equilibrium weight
    in Methods, Eq. (8):
        q(t_{n+1}) = q(t_n) + (Delta/m) p(t_n)
        p(t_{n+1}) = p(t_n) - Delta k q(t_n) + zeta(t_n) Delta sum_j J_ij q_j(t_n)
    Both right-hand sides read step-n values ("paper order").
  * walls: q limited to [-sqrt2, sqrt2] (Eq. 6) and p to [-2, 2] (Methods,
    constraints of Eq. 8), both by clamping.
  * zeta(t): grows linearly with the iteration count from 0.8*zeta0 to
    10*zeta0 (zeta0 = 0.05), held piecewise constant (Fig. 4 and 5 captions,
    Methods).
  * readout: after the last step the positions are sampled and their signs
    are the spin state (Methods, "Hardware implementation").

Orientation: Q and P are [N, R] float64 arrays; column r is one independent
replica (one pixel of the paper's point-convolution feature map, Fig. 3).

Readings where the paper is silent or inconsistent (all listed in the design
notes): paper order is Eq. (8) as printed; m is kept from Eq. (5) (m = 1 in
every experiment); the field h is zero unless given; sign(+-0) = +1; the cut
of a MAX-CUT instance uses graph weights w = -J; the variant ``order=
"symplectic"`` updates p first and moves q with the new p; ``wall=
"inelastic"`` also zeroes p where q ran past the wall.
"""
from __future__ import annotations

import math

import numpy as np

# Paper constants: Fig. 4 caption (k, zeta range, Delta, m), Fig. 5 caption
# (zeta0 and staircase lengths), Eq. (6) and Methods (wall positions).
PAPER = dict(
    k=0.5,
    m=1.0,
    dt=0.2,
    zeta0=0.05,
    zeta_start=0.8 * 0.05,
    zeta_end=10.0 * 0.05,
    qmax=math.sqrt(2.0),
    pmax=2.0,
)


# --------------------------------------------------------------------------
# Eq. (1): energy, readout and the MAX-CUT view
# --------------------------------------------------------------------------
def spins(Q: np.ndarray) -> np.ndarray:
    """Sample positions into spins: +1 where q >= 0 (including -0.0), else -1."""
    Q = np.asarray(Q)
    return np.where(Q < 0, -1, 1).astype(np.int8)


def _is_integer_matrix(J: np.ndarray) -> bool:
    J = np.asarray(J, dtype=np.float64)
    return bool(np.all(np.isfinite(J)) and np.all(J == np.round(J)))


def ising_energy(J, S, h=None):
    """Eq. (1) for each replica column of S (+-1 values, [N, R] or [N]).

    H_r = - sum_{i<j} J_ij s_ir s_jr - sum_i h_i s_ir.  Exact int64 when J
    (and h) hold integers, float64 otherwise.
    """
    J = np.asarray(J, dtype=np.float64)
    S = np.asarray(S)
    vec = S.ndim == 1
    if vec:
        S = S[:, None]
    exact = _is_integer_matrix(J) and (h is None or _is_integer_matrix(np.asarray(h)[None]))
    if exact:
        U = np.triu(J, 1).astype(np.int64)
        Si = S.astype(np.int64)
        e = -np.einsum("ir,ij,jr->r", Si, U, Si)
        if h is not None:
            e = e - np.asarray(h, dtype=np.int64) @ Si
    else:
        U = np.triu(J, 1)
        Sf = S.astype(np.float64)
        e = -np.einsum("ir,ij,jr->r", Sf, U, Sf)
        if h is not None:
            e = e - np.asarray(h, dtype=np.float64) @ Sf
    return e[0] if vec else e


def ising_energy_pairs(J, s, h=None):
    """Eq. (1) for one spin vector, as the literal double loop over i < j.

    Pure Python; meant for small N only.
    """
    n = len(s)
    e = 0
    for i in range(n):
        for j in range(i + 1, n):
            e -= J[i][j] * s[i] * s[j]
    if h is not None:
        for i in range(n):
            e -= h[i] * s[i]
    return e


def cut_value(J, S):
    """MAX-CUT value of the partition given by the spins, with graph weights
    w_ij = -J_ij:  C = sum_{i<j} w_ij [s_i != s_j]  (direct edge count)."""
    J = np.asarray(J, dtype=np.float64)
    S = np.asarray(S)
    vec = S.ndim == 1
    if vec:
        S = S[:, None]
    W = -np.triu(J, 1)
    exact = _is_integer_matrix(J)
    out = []
    for r in range(S.shape[1]):
        s = S[:, r]
        differ = (s[:, None] != s[None, :])
        c = W[differ].sum()
        out.append(int(round(c)) if exact else float(c))
    out = np.array(out, dtype=np.int64 if exact else np.float64)
    return out[0] if vec else out


def relaxed_energy(J, Q):
    """Mean over replicas of the continuous Ising energy -1/2 q^T J q (h = 0)."""
    J = np.asarray(J, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    per = -0.5 * np.einsum("ir,ij,jr->r", Q, J, Q)
    return float(per.mean())


def hamiltonian(J, Q, P, zeta, k=PAPER["k"], m=PAPER["m"], h=None):
    """Eq. (7) per replica with q0 = 0 and qdot = p/m:
    H = sum_i p_i^2/(2m) + sum_i k q_i^2/2 + zeta * H_Ising(q), where
    H_Ising(q) = -1/2 q^T J q - h.q is Eq. (1) with the spins relaxed to q."""
    J = np.asarray(J, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    ising = -0.5 * np.einsum("ir,ij,jr->r", Q, J, Q)
    if h is not None:
        ising = ising - np.asarray(h, dtype=np.float64) @ Q
    return (P * P).sum(axis=0) / (2.0 * m) + 0.5 * k * (Q * Q).sum(axis=0) + zeta * ising


# --------------------------------------------------------------------------
# zeta(t) and Delta schedules
# --------------------------------------------------------------------------
def zeta_schedule(S: int, zeta_start=PAPER["zeta_start"], zeta_end=PAPER["zeta_end"],
                  stair_len: int = 1) -> np.ndarray:
    """Piecewise-constant zeta(t_step), linear in the iteration count.

    Reading (the paper gives only the end points and, for Fig. 5, the stair
    length): with K = ceil(S / L) stairs, step n uses stair s = floor(n / L)
    and zeta_n = zeta_start + (zeta_end - zeta_start) * s / (K - 1); a single
    stair holds zeta_start.  L = 1 is the exactly linear schedule, both end
    points included.  Values are formed in float64, then rounded to float32,
    and both implementations consume the float32 array.
    """
    if S < 1 or stair_len < 1:
        raise ValueError("S and stair_len must be >= 1")
    K = -(-S // stair_len)
    out = np.empty(S, dtype=np.float64)
    for n in range(S):
        s = n // stair_len
        if K == 1:
            out[n] = zeta_start
        else:
            out[n] = zeta_start + (zeta_end - zeta_start) * (s / (K - 1))
    return out.astype(np.float32)


def dt_schedule(S: int, dt=PAPER["dt"]) -> np.ndarray:
    """Constant time step Delta (Fig. 4 caption), as a float32 array."""
    return np.full(S, dt, dtype=np.float32)


# --------------------------------------------------------------------------
# Eq. (8) with the walls
# --------------------------------------------------------------------------
def step(J, Q, P, dt, zeta, k=PAPER["k"], m=PAPER["m"], qmax=PAPER["qmax"],
         pmax=PAPER["pmax"], order="paper", wall="clamp", h=None):
    """One iteration of Eq. (8) (Eq. (5) with m kept), then the walls.

    order="paper": both updates read (q_n, p_n), as printed.
    order="symplectic": p is updated first, q moves with the clamped new p.
    wall="clamp": q and p clamped to their boxes independently.
    wall="inelastic": additionally p <- 0 wherever q ran past its wall.
    """
    F = J @ Q  # sum_j J_ij q_j, the coupling (point-convolution) term
    if h is not None:
        F = F + np.asarray(h, dtype=np.float64)[:, None]
    if order == "paper":
        U = Q + (dt / m) * P
        V = P + dt * (-k * Q + zeta * F)
        Pn = np.clip(V, -pmax, pmax)
    elif order == "symplectic":
        V = P + dt * (-k * Q + zeta * F)
        Pn = np.clip(V, -pmax, pmax)
        U = Q + (dt / m) * Pn
    else:
        raise ValueError(order)
    Qn = np.clip(U, -qmax, qmax)
    if wall == "inelastic":
        Pn = np.where(np.abs(U) > qmax, 0.0, Pn)
    elif wall != "clamp":
        raise ValueError(wall)
    return Qn, Pn


def run(J, Q0, P0, dt, zeta, k=PAPER["k"], m=PAPER["m"], qmax=PAPER["qmax"],
        pmax=PAPER["pmax"], order="paper", wall="clamp", h=None, n_steps=None,
        record=()):
    """Iterate Eq. (8) over the schedules dt[n], zeta[n], n = 0 .. n_steps-1.

    J: [N, N]; Q0, P0: [N, R] (P0 None means zero momenta).  Returns a dict
    with the final "Q", "P" and, for every step index in ``record``, the
    state after that many steps under "traj" (record may include 0).
    """
    J = np.asarray(J, dtype=np.float64)
    Q = np.array(Q0, dtype=np.float64, copy=True)
    P = np.zeros_like(Q) if P0 is None else np.array(P0, dtype=np.float64, copy=True)
    dt = np.asarray(dt, dtype=np.float64)
    zeta = np.asarray(zeta, dtype=np.float64)
    if n_steps is None:
        n_steps = len(dt)
    want = set(int(x) for x in record)
    traj = {}
    if 0 in want:
        traj[0] = (Q.copy(), P.copy())
    for n in range(n_steps):
        Q, P = step(J, Q, P, dt[n], zeta[n], k=k, m=m, qmax=qmax, pmax=pmax,
                    order=order, wall=wall, h=h)
        if n + 1 in want:
            traj[n + 1] = (Q.copy(), P.copy())
    return {"Q": Q, "P": P, "traj": traj}
