"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Trajectory bar (plain method, FP32 on the GPU vs the FP64 oracle): max-norm
relative error of q and of p at most 1e-5 at every one of the first 100
steps.  Energies of the same spin vectors are bit-exact.
"""
import numpy as np
import pytest

import oracle
from paper_2305_07187_amd import instances

from gpu_common import (DT, QMAX, ZE, ZS, F32, announce, ensure_built, oracle_schedules,
                        rel_err, to_dev)

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _model(J, x0, S, p0=None, **kw):
    si = ensure_built()
    return si.SpringIsing(to_dev(J), to_dev(x0), None if p0 is None else to_dev(p0),
                          total_steps=S, **kw)


def _trajectory_check(J, x0, S_check, S_total, qmax=QMAX, order="paper", wall="clamp",
                      h=None, tol=TOL, label="", **kw):
    import torch
    announce(f"trajectory {label} N={J.shape[0]} R={x0.shape[0]} steps={S_check}")
    m = _model(J, x0, S_total, order=order, wall=wall, qmax=qmax, **kw)
    if h is not None:
        m.set_field(to_dev(np.asarray(h, dtype=np.float32)))
        h = np.asarray(h, dtype=np.float32).astype(np.float64)
    dt, zeta = oracle_schedules(S_total)
    ref = oracle.run(J.astype(np.float64), x0.T.astype(np.float64), None, dt, zeta, qmax=qmax,
                     order=order, wall=wall, h=h, n_steps=S_check, record=range(S_check + 1))
    worst_q = worst_p = 0.0
    for n in range(1, S_check + 1):
        m.step()
        x, p, t = m.state()
        torch.cuda.synchronize()
        assert t == n
        eq = rel_err(x.cpu().numpy(), ref["traj"][n][0])
        ep = rel_err(p.cpu().numpy(), ref["traj"][n][1])
        worst_q, worst_p = max(worst_q, eq), max(worst_p, ep)
        assert eq <= tol and ep <= tol, f"step {n}: rel err q {eq:.3e} p {ep:.3e}"
    announce(f"  max rel err over {S_check} steps: q {worst_q:.3e} p {worst_p:.3e}")
    return m


@pytest.mark.parametrize("qmax", [QMAX, 1.0])
def test_plain_trajectory_small(qmax):
    # N=100 +-1 complete graph, R=8, x0 ~ U(-0.1, 0.1), p0 = 0, paper schedule
    n, r, S = 100, 8, 1000
    J = instances.make_pm1(n, 0)
    x0 = instances.make_x0(n, r, 0)
    m = _trajectory_check(J, x0, 100, S, qmax=qmax, label=f"qmax={qmax:.4f}")
    # run the rest of the schedule; compare the final spin states and energies
    import torch
    m.run(S - 100)
    x, _, t = m.state()
    e = m.energy().cpu().numpy()
    torch.cuda.synchronize()
    assert t == S
    dt, zeta = oracle_schedules(S)
    ref = oracle.run(J.astype(np.float64), x0.T.astype(np.float64), None, dt, zeta, qmax=qmax)
    s_ref = oracle.spins(ref["Q"])
    e_ref = oracle.ising_energy(J, s_ref)
    s_gpu = oracle.spins(x.cpu().numpy().T)
    same = [bool(np.array_equal(s_gpu[:, c], s_ref[:, c])) for c in range(r)]
    announce(f"  final: GPU energies {e.tolist()} oracle {e_ref.tolist()} same spins {same}")
    for c in range(r):
        if same[c]:
            assert e[c] == e_ref[c]


@pytest.mark.parametrize("precision,tile", [("fp32", 27), ("fp32", 26), ("bf16x3_exactj", 26)])
def test_production_tiles_hold_the_100_step_bar(precision, tile):
    # The 1e-5 bar over the first 100 steps on the kernels that produce the
    # benchmark's numbers, forced onto the N=100, R=8 instance (padded to the
    # tile): the automatic FP32 tiles of the N=2000, R=1024 workload (eight
    # waves, 64x128 and 128x64, direct-to-LDS rings) and the exact
    # three-plane BF16 tile of that workload.
    n, r, S = 100, 8, 1000
    J = instances.make_pm1(n, 0)
    x0 = instances.make_x0(n, r, 0)
    m = _trajectory_check(J, x0, 100, S, label=f"{precision} tile {tile}", tile=tile,
                          precision=precision)
    info = m.info()
    announce(f"  kernel {info['kernel_name']}")
    assert info["tile"] == tile
    m.close()


def test_full_size_sampled_replicas():
    # N=2000, R=1024 in the launch configuration of the benchmark; the oracle
    # follows 12 sampled replicas for the first 10 steps.
    import torch
    n, r, S = 2000, 1024, 10000
    announce(f"full-size sampled parity N={n} R={r}")
    J = instances.make_pm1(n, 0)
    x0 = instances.make_x0(n, r, 0)
    m = _model(J, x0, S)
    cols = [0, 1, 63, 64, 127, 128, 500, 511, 512, 777, 1022, 1023]
    dt, zeta = oracle_schedules(S)
    steps = 10
    ref = oracle.run(J.astype(np.float64), x0[cols].T.astype(np.float64), None, dt, zeta,
                     qmax=QMAX, n_steps=steps, record=range(steps + 1))
    for k in range(1, steps + 1):
        m.step()
        x, p, t = m.state()
        torch.cuda.synchronize()
        xs = x.cpu().numpy()[cols]
        ps = p.cpu().numpy()[cols]
        eq, ep = rel_err(xs, ref["traj"][k][0]), rel_err(ps, ref["traj"][k][1])
        assert eq <= TOL and ep <= TOL, f"step {k}: {eq:.3e} {ep:.3e}"
    announce(f"  step {steps}: rel err q {eq:.3e} p {ep:.3e} kernel {m.info()['kernel_name']}")


def _fp32_emulation(J, Q, P, dt, zeta, steps, qmax, pmax=2.0, k=0.5):
    """A second FP32 implementation of the paper-order step (NumPy float32
    products, sums and updates, no fused operations), used only to size
    the divergence from FP64 that FP32 arithmetic alone produces."""
    f = np.float32
    J32, Q32, P32 = J.astype(f), Q.astype(f), P.astype(f)
    out = {}
    for n in range(steps):
        F = J32 @ Q32
        d, z = f(dt[n]), f(zeta[n])
        U = Q32 + d * P32
        V = P32 + d * (z * F - f(k) * Q32)
        Q32, P32 = np.clip(U, -f(qmax), f(qmax)), np.clip(V, -f(pmax), f(pmax))
        out[n + 1] = (Q32.astype(np.float64), P32.astype(np.float64))
    return out


def test_full_size_fp32_envelope():
    # At N = 2000 the dynamics amplify rounding so fast that no FP32
    # implementation stays within 1e-5 of FP64 for 100 steps.  The bar there
    # is the envelope of FP32 arithmetic itself: at every checkpoint the
    # GPU's distance from the FP64 oracle must be of the same order (at most
    # 10x, or 1e-5) as that of an independent FP32 implementation; after
    # step 100 the spins are compared where the oracle's |q| > 1e-3.
    import torch
    n, r, S, steps = 2000, 1024, 10000, 100
    announce(f"full-size FP32 envelope N={n} R={r} {steps} steps")
    J = instances.make_pm1(n, 0)
    x0 = instances.make_x0(n, r, 0)
    cols = [0, 255, 511, 640, 900, 1023]
    dt, zeta = oracle_schedules(S)
    marks = [10, 25, 50, 75, 100]
    J64 = J.astype(np.float64)
    Q0 = x0[cols].T.astype(np.float64)
    ref = oracle.run(J64, Q0, None, dt, zeta, qmax=QMAX, n_steps=steps, record=marks)
    emu = _fp32_emulation(J64, Q0, np.zeros_like(Q0), dt, zeta, steps, QMAX)
    m = _model(J, x0, S)
    done = 0
    for mark in marks:
        m.run(mark - done)
        done = mark
        x, p, t = m.state()
        torch.cuda.synchronize()
        assert t == mark
        xs, ps = x.cpu().numpy()[cols].T, p.cpu().numpy()[cols].T
        Qr, Pr = ref["traj"][mark]
        gq, gp = rel_err(xs.T, Qr), rel_err(ps.T, Pr)
        eq, ep = rel_err(emu[mark][0].T, Qr), rel_err(emu[mark][1].T, Pr)
        announce(f"  step {mark}: GPU vs FP64 q {gq:.2e} p {gp:.2e}; "
                 f"FP32 emulation vs FP64 q {eq:.2e} p {ep:.2e}")
        assert gq <= max(TOL, 10 * eq) and gp <= max(TOL, 10 * ep), mark
    Qr = ref["traj"][steps][0]
    firm = np.abs(Qr) > 1e-3
    gpu_mis = int(((xs < 0) != (Qr < 0))[firm].sum())
    emu_mis = int(((emu[steps][0] < 0) != (Qr < 0))[firm].sum())
    announce(f"  step {steps}: spin mismatches where |q| > 1e-3: GPU {gpu_mis}, "
             f"FP32 emulation {emu_mis} of {int(firm.sum())}")
    assert gpu_mis <= max(10 * emu_mis, int(0.01 * firm.sum()))


def test_qualitative_shape_n2000():
    # The run of Fig. 4 on the +-1 stand-in (not a parity check): the energy
    # starts near zero, most of the descent happens in the first hundred
    # steps while the mass points pile up at the walls, and the mean keeps
    # falling more slowly afterwards.  (The FP64 oracle on 8 replicas gives
    # -120, -60050 at step 100 with 97 % of positions at a wall, -63364 at
    # step 1000 and -63598 at step 10000.)
    import torch
    n, r, S = 2000, 64, 10000
    announce(f"qualitative shape N={n} R={r} {S} steps")
    J = instances.make_pm1(n, 0)
    m = _model(J, instances.make_x0(n, r, 0), S)
    means, done = {}, 0
    for mark in [0, 100, 1000, S]:
        m.run(mark - done)
        done = mark
        means[mark] = float(m.energy().cpu().numpy().astype(np.float64).mean())
        if mark == 100:
            x, _, _ = m.state()
            torch.cuda.synchronize()
            wall = float(np.mean(np.abs(x.cpu().numpy()) == np.float32(QMAX)))
    announce(f"  mean energy {means}; fraction at the walls after 100 steps {wall:.3f}")
    assert abs(means[0]) <= 0.05 * abs(means[S])
    assert means[100] <= 0.9 * means[S]
    assert wall >= 0.95
    assert means[S] <= means[1000] <= means[100]


@pytest.mark.parametrize("n,r", [(100, 8), (2000, 1024), (130, 67), (1, 1), (2000, 3), (257, 200)])
def test_energy_bit_exact(n, r):
    import torch
    announce(f"energy bit-exact N={n} R={r}")
    J = instances.make_pm1(n, 7) if n > 1 else np.zeros((1, 1), np.float32)
    x = instances.random_state(n, r, 3)
    m = _model(J, instances.make_x0(n, r, 1), 10)
    m.set_state(to_dev(x), None, 0)
    e = m.energy()
    s = m.spins()
    torch.cuda.synchronize()
    s_ref = oracle.spins(x.T)
    np.testing.assert_array_equal(s.cpu().numpy().T, s_ref)
    np.testing.assert_array_equal(e.cpu().numpy(), oracle.ising_energy(J, s_ref))
    e_real = m.energy(exact=False)
    np.testing.assert_array_equal(e_real.cpu().numpy(), oracle.ising_energy(J, s_ref))


def test_energy_integer_weights_and_field():
    import torch
    n, r = 300, 40
    announce(f"energy integer J in [-5,5] with field N={n} R={r}")
    rng = np.random.default_rng(0)
    U = np.triu(rng.integers(-5, 6, size=(n, n)), 1).astype(np.float32)
    J = U + U.T
    h = rng.integers(-3, 4, size=n).astype(np.float32)
    x = instances.random_state(n, r, 9)
    m = _model(J, instances.make_x0(n, r, 1), 10)
    m.set_state(to_dev(x))
    m.set_field(to_dev(h))
    e = m.energy()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(e.cpu().numpy(), oracle.ising_energy(J, oracle.spins(x.T), h))


def test_energy_real_couplings():
    import torch
    n, r = 500, 64
    announce(f"real-J energy N={n} R={r}")
    J = instances.make_gauss(n, 2)
    x = instances.random_state(n, r, 4)
    m = _model(J, instances.make_x0(n, r, 1), 10)
    m.set_state(to_dev(x))
    e = m.energy(exact=False).cpu().numpy()
    ref = oracle.ising_energy(J.astype(np.float64), oracle.spins(x.T))
    # FP32 products of +-J_ij are exact; the error is the FP32 row sums
    # (<= N eps sum_j |J_ij| per row) summed over rows.
    bound = n * 2.0 ** -24 * np.abs(J).astype(np.float64).sum() + 1e-6
    assert np.all(np.abs(e - ref) <= bound), (np.abs(e - ref).max(), bound)
    with pytest.raises(Exception) as err:
        m.energy(exact=True)
    assert "UNSUPPORTED" in str(err.value)


@pytest.mark.parametrize("order,wall", [("symplectic", "clamp"), ("paper", "inelastic"),
                                        ("symplectic", "inelastic")])
def test_variant_trajectories(order, wall):
    n, r = 100, 8
    J = instances.make_pm1(n, 0)
    x0 = instances.make_x0(n, r, 0)
    _trajectory_check(J, x0, 60, 1000, order=order, wall=wall, label=f"{order}/{wall}")


def test_field_trajectory():
    n, r = 100, 8
    J = instances.make_pm1(n, 1)
    h = np.random.default_rng(5).uniform(-1, 1, n).astype(np.float32)
    x0 = instances.make_x0(n, r, 2)
    _trajectory_check(J, x0, 60, 1000, h=h, label="field")


@pytest.mark.parametrize("n,r", [(1, 1), (65, 3), (127, 129), (300, 1)])
def test_ragged_shapes(n, r):
    J = instances.make_pm1(n, 3) if n > 1 else np.zeros((1, 1), np.float32)
    x0 = instances.make_x0(n, r, 4)
    _trajectory_check(J, x0, 40, 100, label="ragged")


def test_schedule_matches_oracle():
    import torch
    si = ensure_built()
    for S, L in [(1000, 1), (10000, 200), (10000, 1000), (999, 7), (3, 5)]:
        announce(f"schedule S={S} L={L}")
        m = _model(instances.make_pm1(16, 0), instances.make_x0(16, 2, 0), S, stair_len=L)
        dt, zeta = m.schedule()
        torch.cuda.synchronize()
        dt_ref, z_ref = oracle_schedules(S, L)
        np.testing.assert_array_equal(dt.cpu().numpy(), dt_ref)
        np.testing.assert_array_equal(zeta.cpu().numpy(), z_ref)
        m.close()


def test_explicit_schedule():
    # A Fig. 5 style fixed-zeta schedule passed in as arrays.  At zeta = 0.5
    # from the first step the dynamics separate nearby trajectories much
    # faster than on the linear schedule, so parity is checked over 20 steps.
    n, r, S = 100, 8, 20
    import torch
    announce("explicit fixed zeta schedule")
    J = instances.make_pm1(n, 0)
    x0 = instances.make_x0(n, r, 0)
    m = _model(J, x0, S)
    dt = np.full(S, DT, np.float32)
    zeta = np.full(S, F32(0.5), np.float32)
    m.set_schedule(to_dev(dt), to_dev(zeta))
    ref = oracle.run(J.astype(np.float64), x0.T.astype(np.float64), None, dt, zeta, qmax=QMAX,
                     record=range(S + 1))
    worst = 0.0
    for k in range(1, S + 1):
        m.step()
        x, p, _ = m.state()
        torch.cuda.synchronize()
        eq = rel_err(x.cpu().numpy(), ref["traj"][k][0])
        ep = rel_err(p.cpu().numpy(), ref["traj"][k][1])
        worst = max(worst, eq, ep)
        assert eq <= TOL and ep <= TOL, f"step {k}: {eq:.3e} {ep:.3e}"
    announce(f"  max rel err over {S} steps: {worst:.3e}")
