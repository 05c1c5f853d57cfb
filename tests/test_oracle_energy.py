"""Pins for the oracle's Eq. (1) energy, readout and MAX-CUT view.

Nothing here compares the oracle with itself: every check is a closed form,
an identity with a different formula, brute force, or an invariant.
"""
import numpy as np
import pytest

import oracle
from oracle.bruteforce import all_states
from paper_2305_07187_amd import instances


def _rand_spins(n, r, seed):
    rng = np.random.default_rng(seed)
    return rng.choice(np.array([-1, 1], dtype=np.int8), size=(n, r))


@pytest.mark.parametrize("n", [2, 5, 17, 64])
def test_ferromagnet_closed_form(n):
    # J = 11^T - I:  E = -sum_{i<j} s_i s_j = -1/2 (M^2 - N), M = sum s
    J = np.ones((n, n)) - np.eye(n)
    S = _rand_spins(n, 12, n)
    M = S.astype(np.int64).sum(axis=0)
    np.testing.assert_array_equal(oracle.ising_energy(J, S), -(M * M - n) // 2)


@pytest.mark.parametrize("n", [3, 8, 31])
def test_antiferromagnet_closed_form(n):
    J = -(np.ones((n, n)) - np.eye(n))
    S = _rand_spins(n, 12, 100 + n)
    M = S.astype(np.int64).sum(axis=0)
    np.testing.assert_array_equal(oracle.ising_energy(J, S), (M * M - n) // 2)


@pytest.mark.parametrize("n", [4, 7, 10])
def test_unit_complete_graph_maxcut(n):
    # w = -J = 11^T - I is the unit complete graph; its max cut is floor(N^2/4).
    J = -(np.ones((n, n)) - np.eye(n))
    e_min, s, energies = oracle.ground_state_bruteforce(J)
    W = n * (n - 1) // 2
    assert (W - e_min) // 2 == n * n // 4
    assert oracle.cut_value(J, s) == n * n // 4


@pytest.mark.parametrize("n", [6, 11, 14])
def test_mattis_ground_state(n):
    # J_ij = xi_i xi_j (i != j): ground states are +-xi with E = -N(N-1)/2.
    rng = np.random.default_rng(n)
    xi = rng.choice([-1, 1], size=n)
    J = np.outer(xi, xi).astype(np.float64)
    np.fill_diagonal(J, 0.0)
    e_min, s, energies = oracle.ground_state_bruteforce(J)
    assert e_min == -n * (n - 1) // 2
    assert np.array_equal(s, xi) or np.array_equal(s, -xi)
    assert int((energies == e_min).sum()) == 2
    # E(s) for any s: -1/2 ((xi.s)^2 - N)
    S = _rand_spins(n, 9, 7 * n)
    ov = xi @ S.astype(np.int64)
    np.testing.assert_array_equal(oracle.ising_energy(J, S), -(ov * ov - n) // 2)


@pytest.mark.parametrize("kind", ["pm1", "gauss"])
def test_full_matrix_identity_and_z2(kind):
    # E = -sum_{i<j} J s s  ==  -1/2 sum_{ij} J_ij s_i s_j  (J symmetric, zero diag)
    n = 40
    J = instances.make_J(n, kind, 3).astype(np.float64)
    S = _rand_spins(n, 16, 5)
    e = oracle.ising_energy(J, S)
    full = -0.5 * np.einsum("ir,ij,jr->r", S.astype(np.float64), J, S.astype(np.float64))
    np.testing.assert_allclose(e, full, rtol=1e-12, atol=1e-9)
    np.testing.assert_array_equal(oracle.ising_energy(J, -S), e)
    if kind == "pm1":
        assert e.dtype == np.int64
        # sum_{ij} J s s is even for integer symmetric zero-diagonal J
        assert np.all(np.round(full * 2) % 2 == 0)


def test_bruteforce_enumerates_every_state_once():
    n = 9
    J = instances.make_pm1(n, 11).astype(np.float64)
    _, _, energies = oracle.ground_state_bruteforce(J)
    S = all_states(n, 0, 1 << n)
    assert len({tuple(s) for s in S}) == 1 << n
    # E(x) == E(complement(x)): the Z2 pairing of the full table
    comp = (1 << n) - 1 - np.arange(1 << n)
    np.testing.assert_array_equal(energies, energies[comp])


def test_bruteforce_index_convention():
    # State index x has spin i down exactly when bit i of x is set: the
    # table entry 2^i is the state with only spin i flipped.
    n = 7
    J = instances.make_gauss(n, 13).astype(np.float64)
    _, _, energies = oracle.ground_state_bruteforce(J)
    for i in range(n):
        s = np.ones(n, dtype=np.int64)
        s[i] = -1
        np.testing.assert_array_equal(all_states(n, 1 << i, (1 << i) + 1)[0], s)
        assert abs(energies[1 << i] - oracle.ising_energy_pairs(J.tolist(), s.tolist())) < 1e-12
    x = 0b1010011
    s = np.array([-1 if (x >> i) & 1 else 1 for i in range(n)])
    assert abs(energies[x] - oracle.ising_energy_pairs(J.tolist(), s.tolist())) < 1e-12


@pytest.mark.parametrize("kind", ["pm1", "gauss"])
def test_diagonal_never_enters_energy(kind):
    # Eq. (1) sums over pairs i < j only, so J_ii cannot change H.
    n = 12
    J = instances.make_J(n, kind, 21).astype(np.float64)
    D = J + np.diag(np.arange(1, n + 1, dtype=np.float64) * (3 if kind == "pm1" else 0.37))
    S = _rand_spins(n, 6, 9)
    e0 = oracle.ising_energy(J, S)
    e1 = oracle.ising_energy(D, S)
    np.testing.assert_allclose(e1, e0, rtol=0, atol=1e-12)
    for r in range(3):
        assert abs(oracle.ising_energy_pairs(D.tolist(), S[:, r].tolist()) - e0[r]) < 1e-12


def test_single_flip_local_field():
    # Flipping spin t changes E by 2 s_t (sum_j J_tj s_j + h_t).
    n = 25
    J = instances.make_pm1(n, 2).astype(np.float64)
    rng = np.random.default_rng(4)
    h = rng.integers(-3, 4, size=n).astype(np.float64)
    s = rng.choice([-1, 1], size=n)
    e0 = oracle.ising_energy(J, s, h)
    for t in range(n):
        s2 = s.copy()
        s2[t] = -s2[t]
        assert oracle.ising_energy(J, s2, h) - e0 == 2 * s[t] * (J[t] @ s + h[t])


def test_field_as_extra_pinned_spin():
    # A field h is the coupling to one extra spin held at +1:
    # E_h(s) on N spins == E(s, +1) on N+1 spins with J_{i,N} = h_i.
    n = 10
    J = instances.make_pm1(n, 8).astype(np.float64)
    h = np.random.default_rng(1).integers(-2, 3, size=n).astype(np.float64)
    Ja = np.zeros((n + 1, n + 1))
    Ja[:n, :n] = J
    Ja[:n, n] = h
    Ja[n, :n] = h
    S = _rand_spins(n, 20, 6)
    Sa = np.vstack([S, np.ones((1, S.shape[1]), dtype=np.int8)])
    np.testing.assert_array_equal(oracle.ising_energy(J, S, h), oracle.ising_energy(Ja, Sa))
    e_h, _, _ = oracle.ground_state_bruteforce(J, h)
    _, _, ea = oracle.ground_state_bruteforce(Ja)
    # states of the augmented system with the last spin +1 are x < 2^N
    assert e_h == ea[: 1 << n].min()


def test_pair_loop_agrees_on_small_case():
    n = 6
    J = instances.make_gauss(n, 1).astype(np.float64)
    S = _rand_spins(n, 5, 3)
    for r in range(5):
        assert abs(oracle.ising_energy_pairs(J.tolist(), S[:, r].tolist())
                   - oracle.ising_energy(J, S[:, r])) < 1e-12


@pytest.mark.parametrize("kind", ["pm1", "gauss"])
def test_cut_identity(kind):
    # C = (W - E)/2 with W = sum_{i<j} w_ij, w = -J  (derived from Eq. (1))
    n = 30
    J = instances.make_J(n, kind, 9).astype(np.float64)
    S = _rand_spins(n, 8, 2)
    W = -np.triu(J, 1).sum()
    np.testing.assert_allclose(oracle.cut_value(J, S), (W - oracle.ising_energy(J, S)) / 2,
                               rtol=1e-12, atol=1e-9)


def test_readout_sign_convention():
    q = np.array([[0.0, -0.0, 1e-30, -1e-30, 1.4, -1.4]]).T
    np.testing.assert_array_equal(oracle.spins(q)[:, 0], [1, 1, 1, -1, 1, -1])


def test_instances_are_symmetric_zero_diagonal():
    for kind in ("pm1", "gauss"):
        J = instances.make_J(33, kind, 0)
        assert np.array_equal(J, J.T)
        assert np.all(np.diag(J) == 0)
    J = instances.make_pm1(33, 0)
    assert set(np.unique(J[~np.eye(33, dtype=bool)])) == {-1.0, 1.0}
    x0 = instances.make_x0(33, 5, 0)
    assert x0.shape == (5, 33) and np.all(np.abs(x0) <= 0.1)
    # drawing more replicas keeps the earlier ones
    np.testing.assert_array_equal(instances.make_x0(33, 9, 0)[:5], x0)


def test_splitmix64_published_values():
    # First outputs of splitmix64 seeded with 0 (values from the generator's
    # published reference implementation).
    z = instances.splitmix64(0, 3)
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
