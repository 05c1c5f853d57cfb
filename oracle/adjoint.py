"""Adjoint of the relaxed end-energy -- test infrastructure (oracle).

The forward map is the paper-order Eq. (8) iteration with clamping walls
(Eq. 6 and the momentum box of Methods).  The loss is the mean over
replicas of the continuous Ising energy of the final positions,
    L = (1/R) sum_r -1/2 q_{S,r}^T J q_{S,r}.
Its gradient with respect to every entry of the per-step schedules Delta_n
and zeta_n follows by reverse-mode differentiation of each step:

    u_n = q_n + (Delta_n/m) p_n,        q_{n+1} = clamp(u_n, +-qmax)
    v_n = p_n + Delta_n(-k q_n + zeta_n J q_n),  p_{n+1} = clamp(v_n, +-pmax)

    lam_q(S) = -(1/R) J q_S,  lam_p(S) = 0
    ubar = lam_q(n+1) * [|u_n| <= qmax],  vbar = lam_p(n+1) * [|v_n| <= pmax]
    lam_q(n) = ubar - Delta_n k vbar + Delta_n zeta_n J vbar
    lam_p(n) = (Delta_n/m) ubar + vbar
    dL/dDelta_n = <ubar, p_n>/m - k <vbar, q_n> + zeta_n <J vbar, q_n>
    dL/dzeta_n  = Delta_n <J vbar, q_n>

J is symmetric, which is used for J^T = J.  The clamp derivative is 1 on
the closed interval (inclusive bounds).  All arithmetic is float64; the
forward states are stored, not recomputed.
"""
from __future__ import annotations

import numpy as np

from .spring_ising import PAPER


def relaxed_energy_grad(J, Q0, P0, dt, zeta, k=PAPER["k"], m=PAPER["m"],
                        qmax=PAPER["qmax"], pmax=PAPER["pmax"]):
    """Return (L, dL/ddt [S], dL/dzeta [S]) for the paper-order iteration."""
    J = np.asarray(J, dtype=np.float64)
    Q = np.array(Q0, dtype=np.float64, copy=True)
    P = np.zeros_like(Q) if P0 is None else np.array(P0, dtype=np.float64, copy=True)
    dt = np.asarray(dt, dtype=np.float64)
    zeta = np.asarray(zeta, dtype=np.float64)
    S = len(dt)
    qs, ps, umask, vmask = [], [], [], []
    for n in range(S):
        U = Q + (dt[n] / m) * P
        V = P + dt[n] * (-k * Q + zeta[n] * (J @ Q))
        qs.append(Q)
        ps.append(P)
        umask.append(np.abs(U) <= qmax)
        vmask.append(np.abs(V) <= pmax)
        Q = np.clip(U, -qmax, qmax)
        P = np.clip(V, -pmax, pmax)
    return _reverse_sweep(J, qs, ps, umask, vmask, Q, dt, zeta, k, m)


def relaxed_energy_grad_along(J, Qs, Ps, dt, zeta, k=PAPER["k"], m=PAPER["m"],
                              qmax=PAPER["qmax"], pmax=PAPER["pmax"]):
    """The same gradient along a given trajectory: Qs[n], Ps[n] are the
    states after n steps (n = 0 .. S, [N, R] each), for instance those of
    another implementation of the forward map.  The wall masks of every
    step are evaluated from those states; the reverse sweep is the one of
    relaxed_energy_grad.  Returns (L, dL/ddt [S], dL/dzeta [S])."""
    J = np.asarray(J, dtype=np.float64)
    dt = np.asarray(dt, dtype=np.float64)
    zeta = np.asarray(zeta, dtype=np.float64)
    S = len(dt)
    if len(Qs) != S + 1 or len(Ps) != S + 1:
        raise ValueError("need the S + 1 states q_0 .. q_S and p_0 .. p_S")
    qs, ps, umask, vmask = [], [], [], []
    for n in range(S):
        Q = np.asarray(Qs[n], dtype=np.float64)
        P = np.asarray(Ps[n], dtype=np.float64)
        U = Q + (dt[n] / m) * P
        V = P + dt[n] * (-k * Q + zeta[n] * (J @ Q))
        qs.append(Q)
        ps.append(P)
        umask.append(np.abs(U) <= qmax)
        vmask.append(np.abs(V) <= pmax)
    return _reverse_sweep(J, qs, ps, umask, vmask, np.asarray(Qs[S], dtype=np.float64), dt,
                          zeta, k, m)


def _reverse_sweep(J, qs, ps, umask, vmask, Q, dt, zeta, k, m):
    """Loss at the final positions Q and the reverse sweep over the stored
    states and wall masks (the recurrences in the module docstring)."""
    S = len(dt)
    R = Q.shape[1]
    JQ = J @ Q
    loss = float((-0.5 * np.einsum("ir,ir->r", Q, JQ)).mean())
    lam_q = -(1.0 / R) * JQ
    lam_p = np.zeros_like(lam_q)
    g_dt = np.zeros(S)
    g_zeta = np.zeros(S)
    for n in range(S - 1, -1, -1):
        ubar = np.where(umask[n], lam_q, 0.0)
        vbar = np.where(vmask[n], lam_p, 0.0)
        Jv = J @ vbar
        qn, pn = qs[n], ps[n]
        g_dt[n] = (ubar * pn).sum() / m - k * (vbar * qn).sum() + zeta[n] * (Jv * qn).sum()
        g_zeta[n] = dt[n] * (Jv * qn).sum()
        lam_q = ubar - dt[n] * k * vbar + dt[n] * zeta[n] * Jv
        lam_p = (dt[n] / m) * ubar + vbar
    return loss, g_dt, g_zeta
