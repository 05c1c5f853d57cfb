"""Pins for the oracle's Eq. (8) iteration, walls and zeta(t) schedule."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from oracle import PAPER
from paper_2305_07187_amd import instances

from closed_forms import scalar_replay

F32_SQRT2 = float(np.float32(math.sqrt(2.0)))


# ---------------------------------------------------------------- P2: J = 0
@pytest.mark.parametrize("m", [1.0, 2.0])
def test_free_spring_growth_paper_order(m):
    # J = 0, walls never touched: G = k q^2 + p^2/m grows by exactly
    # (1 + Delta^2 k / m) per step in the explicit (paper) order.
    n, r, S = 7, 3, 25
    k, dt = 0.5, 0.1
    rng = np.random.default_rng(0)
    Q0 = rng.uniform(-0.05, 0.05, (n, r))
    P0 = rng.uniform(-0.05, 0.05, (n, r))
    out = oracle.run(np.zeros((n, n)), Q0, P0, np.full(S, dt), np.zeros(S), k=k, m=m,
                     record=range(S + 1))
    G = [k * out["traj"][s][0] ** 2 + out["traj"][s][1] ** 2 / m for s in range(S + 1)]
    for s in range(S):
        np.testing.assert_allclose(G[s + 1], (1 + dt * dt * k / m) * G[s], rtol=1e-13)
    assert np.abs(out["Q"]).max() < 0.5


@pytest.mark.parametrize("m", [1.0, 2.0])
def test_free_spring_invariant_symplectic_order(m):
    # p first, then q with the new p: k q^2 + p^2/m - (Delta k/m) q p is
    # conserved exactly (discrete invariant of symplectic Euler).
    n, r, S = 5, 4, 200
    k, dt = 0.5, 0.2
    rng = np.random.default_rng(1)
    Q0 = rng.uniform(-0.5, 0.5, (n, r))
    P0 = rng.uniform(-0.5, 0.5, (n, r))
    out = oracle.run(np.zeros((n, n)), Q0, P0, np.full(S, dt), np.zeros(S), k=k, m=m,
                     order="symplectic", record=range(S + 1))
    inv = [k * q * q + p * p / m - dt * k / m * q * p for q, p in
           (out["traj"][s] for s in range(S + 1))]
    for s in range(S + 1):
        np.testing.assert_allclose(inv[s], inv[0], rtol=1e-12, atol=1e-15)
    # and the paper order does NOT conserve it: the two orders differ
    outp = oracle.run(np.zeros((n, n)), Q0, P0, np.full(S, dt), np.zeros(S), k=k, m=m)
    assert np.abs(outp["Q"] - out["Q"]).max() > 1e-3


# --------------------------------------- P3: uniform coupling, exact replay
def _uniform_case(n, a, q0_pattern, S, stair, order, zeta_scale=1.0):
    J = a * (np.ones((n, n)) - np.eye(n))
    dt = oracle.dt_schedule(S, 0.25)
    zeta = oracle.zeta_schedule(S, 0.04 * zeta_scale, 0.5 * zeta_scale, stair)
    c = 0.0625
    if q0_pattern == "const":
        q0 = np.full(n, c)
        lam = a * (n - 1)
    else:
        q0 = c * np.array([1.0 if i % 2 == 0 else -1.0 for i in range(n)])
        lam = -a
    R = 2
    Q0 = np.stack([q0, -q0], axis=1)
    out = oracle.run(J, Q0, None, dt, zeta, k=0.5, m=1.0, qmax=F32_SQRT2, pmax=2.0,
                     order=order, record=range(S + 1))
    exact = scalar_replay(Fr(c), Fr(0), Fr(lam), [float(x) for x in dt],
                          [float(x) for x in zeta], Fr(1, 2), Fr(1), Fr(F32_SQRT2), Fr(2),
                          order=order)
    return out, exact, q0, R


@pytest.mark.parametrize("order", ["paper", "symplectic"])
@pytest.mark.parametrize("pattern,a,zs", [("const", 1.0, 1.0), ("const", -1.0, 1.0),
                                          ("alt", 1.0, 1.0), ("const", 1.0, 0.05)])
def test_uniform_coupling_exact_replay(order, pattern, a, zs):
    n, S = 16, 120
    out, exact, q0, R = _uniform_case(n, a, pattern, S, 7, order, zs)
    shape = np.sign(q0)
    walls_hit = False
    for s in range(S + 1):
        qe, pe = exact[s]
        Q, P = out["traj"][s]
        np.testing.assert_allclose(Q[:, 0], float(qe) * shape, rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(P[:, 0], float(pe) * shape, rtol=1e-12, atol=1e-13)
        # Z2 column
        np.testing.assert_array_equal(Q[:, 1], -Q[:, 0])
        walls_hit |= abs(qe) == Fr(F32_SQRT2) or abs(pe) == 2
    if zs == 1.0 and pattern == "const" and a > 0:
        assert walls_hit  # the case exercises the walls


# ------------------------------------------------------------ invariants
def _cfg0(n=60, r=6, S=150, seed=0):
    J = instances.make_pm1(n, seed).astype(np.float64)
    Q0 = instances.make_x0(n, r, seed).T.astype(np.float64)
    dt = oracle.dt_schedule(S)
    zeta = oracle.zeta_schedule(S)
    return J, Q0, dt, zeta


def test_gauge_and_z2_invariance():
    J, Q0, dt, zeta = _cfg0()
    d = np.where(np.random.default_rng(3).random(J.shape[0]) < 0.5, -1.0, 1.0)
    D = np.diag(d)
    base = oracle.run(J, Q0, None, dt, zeta, qmax=F32_SQRT2)
    gauge = oracle.run(D @ J @ D, D @ Q0, None, dt, zeta, qmax=F32_SQRT2)
    np.testing.assert_allclose(gauge["Q"], D @ base["Q"], rtol=0, atol=1e-12)
    z2 = oracle.run(J, -Q0, None, dt, zeta, qmax=F32_SQRT2)
    np.testing.assert_allclose(z2["Q"], -base["Q"], rtol=0, atol=1e-12)


def test_replica_independence():
    J, Q0, dt, zeta = _cfg0(S=60)
    full = oracle.run(J, Q0, None, dt, zeta, record=range(61))
    for r in (0, 3):
        one = oracle.run(J, Q0[:, r:r + 1], None, dt, zeta, record=range(61))
        for s in range(61):
            np.testing.assert_allclose(one["traj"][s][0][:, 0], full["traj"][s][0][:, r],
                                       rtol=1e-9, atol=1e-12)


def test_walls_hold_and_inelastic_variant():
    n, r = 20, 4
    J = instances.make_pm1(n, 1).astype(np.float64)
    rng = np.random.default_rng(2)
    Q = rng.uniform(-3, 3, (n, r))
    P = rng.uniform(-5, 5, (n, r))
    Qn, Pn = oracle.step(J, Q, P, 0.2, 0.3, qmax=F32_SQRT2, pmax=2.0)
    assert np.abs(Qn).max() <= F32_SQRT2 and np.abs(Pn).max() <= 2.0
    U = Q + 0.2 * P
    np.testing.assert_array_equal(Qn[np.abs(U) > F32_SQRT2],
                                  np.sign(U[np.abs(U) > F32_SQRT2]) * F32_SQRT2)
    Qi, Pi = oracle.step(J, Q, P, 0.2, 0.3, qmax=F32_SQRT2, pmax=2.0, wall="inelastic")
    np.testing.assert_array_equal(Qi, Qn)
    hit = np.abs(U) > F32_SQRT2
    assert hit.any() and (~hit).any()
    assert np.all(Pi[hit] == 0) and np.array_equal(Pi[~hit], Pn[~hit])


def test_field_shifts_force():
    # h adds zeta*Delta*h to the momentum update and nothing else.
    n, r = 12, 3
    J = instances.make_pm1(n, 4).astype(np.float64)
    rng = np.random.default_rng(7)
    Q = rng.uniform(-0.1, 0.1, (n, r))
    P = rng.uniform(-0.1, 0.1, (n, r))
    h = rng.uniform(-1, 1, n)
    Q1, P1 = oracle.step(J, Q, P, 0.2, 0.3, h=h)
    Q0_, P0_ = oracle.step(J, Q, P, 0.2, 0.3)
    np.testing.assert_array_equal(Q1, Q0_)
    np.testing.assert_allclose(P1 - P0_, 0.2 * 0.3 * h[:, None] * np.ones((1, r)), atol=1e-15)


# --------------------------------------------------------------- schedule
@pytest.mark.parametrize("S,L", [(1000, 1), (10000, 200), (10000, 1000), (999, 7), (5, 10), (1, 1)])
def test_zeta_schedule_shape(S, L):
    z = oracle.zeta_schedule(S, stair_len=L)
    assert z.dtype == np.float32 and len(z) == S
    assert z[0] == np.float32(0.04)
    K = -(-S // L)
    if K > 1:
        assert z[-1] == np.float32(0.5)
    assert np.all(np.diff(z.astype(np.float64)) >= 0)
    # constant inside a stair, changes only at multiples of L
    change = np.nonzero(np.diff(z))[0] + 1
    assert np.all(change % L == 0)
    assert len(np.unique(z)) == K
    if K > 2:
        steps = np.diff(np.unique(z).astype(np.float64))
        np.testing.assert_allclose(steps, (0.5 - 0.04) / (K - 1), rtol=0, atol=2 ** -23)


def test_paper_constants():
    assert PAPER["zeta_start"] == pytest.approx(0.04)
    assert PAPER["zeta_end"] == pytest.approx(0.5)
    assert PAPER["qmax"] == pytest.approx(math.sqrt(2))
    assert (PAPER["k"], PAPER["dt"], PAPER["m"], PAPER["pmax"]) == (0.5, 0.2, 1.0, 2.0)


# -------------------------------------------------- method-level behaviour
def test_finds_ground_state_on_small_instances():
    # The heuristic reaches the brute-force ground state on tiny instances
    # for some replica (a property of the method, not a parity check).
    hits = 0
    for seed in range(4):
        n = 14
        J = instances.make_pm1(n, seed).astype(np.float64)
        e_min, _, _ = oracle.ground_state_bruteforce(J)
        Q0 = instances.make_x0(n, 32, seed).T.astype(np.float64)
        S = 400
        out = oracle.run(J, Q0, None, oracle.dt_schedule(S), oracle.zeta_schedule(S))
        e = oracle.ising_energy(J, oracle.spins(out["Q"]))
        assert e.min() >= e_min
        hits += int(e.min() == e_min)
    assert hits >= 3


def test_qualitative_descent():
    # Energy starts near 0 from the small disturbance and falls; most
    # positions end at the walls (Fig. 4 narrative).
    n, r, S = 200, 8, 1000
    J = instances.make_pm1(n, 0).astype(np.float64)
    Q0 = instances.make_x0(n, r, 0).T.astype(np.float64)
    out = oracle.run(J, Q0, None, oracle.dt_schedule(S), oracle.zeta_schedule(S),
                     record=[0, S])
    e0 = oracle.ising_energy(J, oracle.spins(out["traj"][0][0]))
    e1 = oracle.ising_energy(J, oracle.spins(out["Q"]))
    assert np.all(e1 < e0)
    assert np.mean(np.isclose(np.abs(out["Q"]), PAPER["qmax"])) > 0.5


# ------------------------------------------------------- Eq. (7) Hamiltonian
def test_hamiltonian_free_spring_growth():
    # J = 0: H = (k q^2 + p^2/m)/2, which the paper-order step multiplies by
    # exactly (1 + Delta^2 k/m) (same identity as the free-spring pin).
    n, r, S, k, m, dt = 6, 3, 15, 0.5, 2.0, 0.1
    rng = np.random.default_rng(3)
    Q0 = rng.uniform(-0.05, 0.05, (n, r))
    P0 = rng.uniform(-0.05, 0.05, (n, r))
    out = oracle.run(np.zeros((n, n)), Q0, P0, np.full(S, dt), np.zeros(S), k=k, m=m,
                     record=range(S + 1))
    H = [oracle.hamiltonian(np.zeros((n, n)), *out["traj"][s], 0.3, k=k, m=m) for s in range(S + 1)]
    for s in range(S):
        np.testing.assert_allclose(H[s + 1], (1 + dt * dt * k / m) * H[s], rtol=1e-13)


def test_hamiltonian_at_spin_vertices():
    # q = s (+-1), p = 0: H = k N/2 + zeta E(s), with E the Eq. (1) energy.
    n = 40
    J = instances.make_pm1(n, 6).astype(np.float64)
    h = np.random.default_rng(2).integers(-2, 3, n).astype(np.float64)
    S = np.random.default_rng(1).choice([-1.0, 1.0], size=(n, 5))
    H = oracle.hamiltonian(J, S, np.zeros_like(S), 0.37, k=0.5, h=h)
    E = oracle.ising_energy(J, S.astype(np.int64), h)
    np.testing.assert_allclose(H, 0.25 * n + 0.37 * E, rtol=1e-13)
