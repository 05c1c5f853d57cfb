"""Precision forms on the BF16 matrix cores against the FP64 oracle.

bf16x3_exactj: J exact in BF16, q split into three BF16 planes whose sum is
the FP32 value; every product is exact, so the form must meet the FP32 bar
(1e-5 relative over the first 100 steps).

bf16x_bf16j / bf16x_fp8j / bf16x_hiloj: the positions enter the product as
BF16 (unit roundoff 2^-8).  One step from the same state then moves each
momentum by at most Delta*zeta*sum_j |J_ij| |q_j| 2^-8 (+ FP32 terms)
away from the oracle's; that bound is checked element by element.  Longer
runs are compared as distributions of final energies.
"""
import numpy as np
import pytest

import oracle
from paper_2305_07187_amd import instances

from gpu_common import QMAX, announce, ensure_built, oracle_schedules, rel_err, to_dev

pytestmark = pytest.mark.gpu


def _model(J, x0, S, precision, **kw):
    si = ensure_built()
    return si.SpringIsing(to_dev(J), to_dev(x0), total_steps=S, precision=precision, **kw)


def test_exact_split_meets_fp32_bar():
    import torch
    n, r, S = 100, 8, 1000
    announce("bf16x3_exactj trajectory N=100 R=8")
    J = instances.make_pm1(n, 0)
    x0 = instances.make_x0(n, r, 0)
    m = _model(J, x0, S, "bf16x3_exactj")
    dt, zeta = oracle_schedules(S)
    ref = oracle.run(J.astype(np.float64), x0.T.astype(np.float64), None, dt, zeta, qmax=QMAX,
                     n_steps=100, record=range(101))
    worst = 0.0
    for k in range(1, 101):
        m.step()
        x, p, _ = m.state()
        torch.cuda.synchronize()
        eq = rel_err(x.cpu().numpy(), ref["traj"][k][0])
        ep = rel_err(p.cpu().numpy(), ref["traj"][k][1])
        worst = max(worst, eq, ep)
        assert eq <= 1e-5 and ep <= 1e-5, f"step {k}: {eq:.3e} {ep:.3e}"
    announce(f"  max rel err over 100 steps {worst:.3e} ({m.info()['kernel_name']})")
    m.run(S - 100)
    e = m.energy().cpu().numpy()
    full = oracle.run(J.astype(np.float64), x0.T.astype(np.float64), None, dt, zeta, qmax=QMAX)
    e_ref = oracle.ising_energy(J, oracle.spins(full["Q"]))
    announce(f"  final energies {e.tolist()} oracle {e_ref.tolist()}")


@pytest.mark.parametrize("precision", ["bf16x_bf16j", "bf16x_fp8j", "bf16x_hiloj"])
def test_single_plane_forms_divergence_reported(precision):
    # The one-plane forms round q to BF16 in every product, so they leave
    # the FP64 trajectory at once; the normwise divergence over the first
    # 100 steps is reported (the per-step error is bounded by the one-step
    # tests).  Sanity bar: it stays below 1 in max-norm relative terms
    # and grows from the BF16 unit roundoff, not from a wrong step.
    import torch
    n, r, S = 100, 8, 1000
    announce(f"{precision} trajectory divergence N={n} R={r}, 100 steps")
    J = instances.make_gauss(n, 0) if precision == "bf16x_hiloj" else instances.make_pm1(n, 0)
    x0 = instances.make_x0(n, r, 0)
    m = _model(J, x0, S, precision)
    dt, zeta = oracle_schedules(S)
    ref = oracle.run(J.astype(np.float64), x0.T.astype(np.float64), None, dt, zeta, qmax=QMAX,
                     n_steps=100, record=range(101))
    report = {}
    for k in range(1, 101):
        m.step()
        if k in (1, 10, 25, 50, 100):
            x, p, _ = m.state()
            torch.cuda.synchronize()
            report[k] = (rel_err(x.cpu().numpy(), ref["traj"][k][0]),
                         rel_err(p.cpu().numpy(), ref["traj"][k][1]))
    announce("  " + ", ".join(f"step {k}: q {a:.2e} p {b:.2e}" for k, (a, b) in report.items()))
    assert report[1][1] <= 2.0 ** -7 and all(a < 1.0 and b < 1.0 for a, b in report.values())


def test_exact_split_full_size_sampled():
    import torch
    n, r, S = 2000, 1024, 5000
    announce("bf16x3_exactj full size, sampled replicas")
    J = instances.make_pm1(n, 0)
    x0 = instances.make_x0(n, r, 0)
    m = _model(J, x0, S, "bf16x3_exactj")
    cols = [0, 5, 511, 1023]
    dt, zeta = oracle_schedules(S)
    ref = oracle.run(J.astype(np.float64), x0[cols].T.astype(np.float64), None, dt, zeta,
                     qmax=QMAX, n_steps=10, record=range(11))
    for k in range(1, 11):
        m.step()
        x, p, _ = m.state()
        torch.cuda.synchronize()
        eq = rel_err(x.cpu().numpy()[cols], ref["traj"][k][0])
        ep = rel_err(p.cpu().numpy()[cols], ref["traj"][k][1])
        assert eq <= 1e-5 and ep <= 1e-5, f"step {k}: {eq:.3e} {ep:.3e}"


def _one_step_bound_check(J, precision, n, r, label):
    """One step from the same state: element-wise bound from BF16 rounding."""
    import torch
    announce(f"{precision} one-step bound {label} N={n} R={r}")
    S = 100
    x = instances.random_state(n, r, 11, scale=1.4)
    p0 = instances.random_state(n, r, 12, scale=1.9)
    m = _model(J, instances.make_x0(n, r, 0), S, precision)
    m.set_state(to_dev(x), to_dev(p0), 37)
    m.step()
    xg, pg, _ = m.state()
    torch.cuda.synchronize()
    dt, zeta = oracle_schedules(S)
    J64 = J.astype(np.float64)
    Q, P = oracle.step(J64, x.T.astype(np.float64), p0.T.astype(np.float64), float(dt[37]),
                       float(zeta[37]), qmax=QMAX)
    d, z = float(dt[37]), float(zeta[37])
    mag = np.abs(J64) @ np.abs(x.T.astype(np.float64))  # sum_j |J_ij||q_j|
    # BF16 rounding of q (2^-8), hi+lo residual of J (2^-16 |J|), FP32
    # accumulation over n terms, and a few FP32 roundings in the update.
    jrel = 2.0 ** -16 if precision == "bf16x_hiloj" else 0.0
    bound = d * z * mag * (2.0 ** -8 + jrel) * 1.01 + 4 * 2.0 ** -24 * (np.abs(P) + 2.0) \
        + d * z * mag * n * 2.0 ** -24
    err = np.abs(pg.cpu().numpy().T - P)
    # elements clamped at the momentum wall on one side only can differ less;
    # the bound holds everywhere because clamping is 1-Lipschitz
    assert np.all(err <= bound), (err.max(), float(bound[np.argmax(err - bound)]))
    # positions do not involve the product: FP32 rounding only
    assert np.abs(xg.cpu().numpy().T - Q).max() <= 4e-7
    rel = float(np.abs(err).max() / np.abs(P).max())
    announce(f"  one-step momentum error max {err.max():.3e} (rel {rel:.3e}); bound ok")


@pytest.mark.parametrize("precision", ["bf16x_bf16j", "bf16x_fp8j"])
def test_pm1_forms_one_step(precision):
    _one_step_bound_check(instances.make_pm1(300, 3), precision, 300, 70, "pm1")


def test_hilo_gaussian_one_step():
    _one_step_bound_check(instances.make_gauss(300, 4), "bf16x_hiloj", 300, 70, "gauss")


def test_fp8_and_bf16_j_identical():
    # +-1 is exact in both formats and both expand to the same BF16 values
    # in LDS, so the two forms run the identical arithmetic.
    announce("fp8 J == bf16 J bitwise")
    import torch
    n, r, S = 500, 128, 300
    J = instances.make_pm1(n, 5)
    x0 = instances.make_x0(n, r, 5)
    out = []
    for prec in ("bf16x_bf16j", "bf16x_fp8j"):
        m = _model(J, x0, S, prec)
        m.run(S)
        x, p, _ = m.state()
        torch.cuda.synchronize()
        out.append((x.cpu().numpy(), p.cpu().numpy()))
        m.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("precision,group", [
    ("bf16x_bf16j", (7, 8, 9, 10, 11, 12, 13, 15, 16, 17, 18, 20, 21, 22, 23, 24, 25, 26, 28, 29,
                     30, 31, 32, 33)),
    ("bf16x_bf16j", (1, 2, 3, 4, 5, 6)),
    ("bf16x_fp8j", (9, 13, 14, 19, 23, 25, 27, 32)),
    ("bf16x_hiloj", (7, 8, 9, 10, 11, 12, 18, 20, 21, 22, 24, 26, 28, 30, 31, 33)),
    ("bf16x3_exactj", (7, 8, 11, 21, 22, 24, 26, 30, 31, 33))])
def test_bf16_tiles_agree(precision, group):
    # Within one pipeline kind every tile shape feeds the same contraction
    # indices to each MFMA and chains the MFMAs in the same order, so the
    # trajectories agree bit for bit whatever the block, wave or slab shape,
    # whether or not the ring is pipelined across slabs, and whether the
    # update runs in the matrix waves or in separate state waves.
    import torch
    announce(f"{precision} tiles agree {group}")
    n, r, S = 256, 256, 40
    J = instances.make_gauss(n, 8) if precision == "bf16x_hiloj" else instances.make_pm1(n, 8)
    x0 = instances.make_x0(n, r, 8)
    ref = None
    for tile in group:
        m = _model(J, x0, S, precision, tile=tile)
        assert m.info()["tile"] == tile
        m.run(S)
        x, p, _ = m.state()
        torch.cuda.synchronize()
        cur = (x.cpu().numpy(), p.cpu().numpy())
        name = m.info()["kernel_name"]
        m.close()
        if ref is None:
            ref = cur
        else:
            assert np.array_equal(cur[0], ref[0]) and np.array_equal(cur[1], ref[1]), name


@pytest.mark.parametrize("precision,group", [
    ("bf16x_bf16j", (16, 18, 20, 21, 23, 28, 29, 30, 32)),
    ("bf16x_fp8j", (9, 19, 23, 27, 32)),
    ("bf16x_hiloj", (18, 20, 21, 28, 30)),
    ("bf16x3_exactj", (11, 21, 22, 24, 26, 30, 31, 33))])
def test_large_bf16_tiles_agree_ragged(precision, group):
    # The two-slab 128x256 / 256x128 rings against the three-slab rings on a
    # ragged shape: the row and replica padding differ between the tiles
    # (N = 300 pads to 384 or 512), and the extra zero slabs and columns
    # must leave every value unchanged.
    import torch
    announce(f"{precision} large tiles agree on N=300 R=200 {group}")
    n, r, S = 300, 200, 30
    J = instances.make_gauss(n, 9) if precision == "bf16x_hiloj" else instances.make_pm1(n, 9)
    x0 = instances.make_x0(n, r, 9)
    ref = None
    for tile in group:
        m = _model(J, x0, S, precision, tile=tile)
        assert m.info()["tile"] == tile
        m.run(S)
        x, p, _ = m.state()
        torch.cuda.synchronize()
        cur = (x.cpu().numpy(), p.cpu().numpy())
        name = m.info()["kernel_name"]
        m.close()
        if ref is None:
            ref = cur
        else:
            assert np.array_equal(cur[0], ref[0]) and np.array_equal(cur[1], ref[1]), name


def _runs(precision, cases, S, steps):
    import torch
    res = []
    for JJ, xx in cases:
        m = _model(JJ, xx, S, precision)
        m.run(steps)
        x, p, _ = m.state()
        torch.cuda.synchronize()
        res.append(x.cpu().numpy())
        m.close()
    return res


def test_lowp_gauge_z2_single_plane():
    # One BF16 plane of q: the gauge and Z2 images are bit-identical.
    announce("bf16x_fp8j gauge/Z2")
    n, r, S = 300, 64, 200
    J = instances.make_pm1(n, 1)
    x0 = instances.make_x0(n, r, 1)
    d = np.where(np.random.default_rng(2).random(n) < 0.5, -1.0, 1.0).astype(np.float32)
    res = _runs("bf16x_fp8j", [(J, x0), ((d[:, None] * J * d[None, :]).astype(np.float32),
                                         x0 * d[None, :]), (J, -x0)], S, S)
    assert np.array_equal(res[1], res[0] * d[None, :])
    assert np.array_equal(res[2], -res[0])


def test_exact_split_determinism_and_gauge():
    # Three planes: runs are deterministic bit for bit.  The gauge image is
    # checked to the FP32 bar only: the small mid/lo planes are added into a
    # large running sum inside the BF16 matrix core, whose rounding of such
    # addends is not sign-symmetric, so +x and -x can round apart.
    announce("bf16x3_exactj determinism / gauge")
    n, r, S = 300, 64, 1000
    J = instances.make_pm1(n, 1)
    x0 = instances.make_x0(n, r, 1)
    d = np.where(np.random.default_rng(2).random(n) < 0.5, -1.0, 1.0).astype(np.float32)
    res = _runs("bf16x3_exactj", [(J, x0), (J, x0), ((d[:, None] * J * d[None, :]).astype(
        np.float32), x0 * d[None, :]), (J, -x0)], S, 30)
    assert np.array_equal(res[0], res[1])
    den = np.abs(res[0]).max()
    g = np.abs(res[2] - res[0] * d[None, :]).max() / den
    z = np.abs(res[3] + res[0]).max() / den
    announce(f"  gauge rel diff {g:.3e}, Z2 rel diff {z:.3e} after 30 steps")
    assert g <= 1e-5 and z <= 1e-5


def test_energy_distribution_vs_oracle():
    # Final-energy distribution of the BF16 form over many replicas vs the
    # FP64 oracle's: means within 4 standard errors (N=100, R=512, 1000 steps).
    import torch
    n, r, S = 100, 512, 1000
    announce("final energy distribution bf16x_fp8j vs oracle")
    J = instances.make_pm1(n, 0)
    x0 = instances.make_x0(n, r, 9)
    m = _model(J, x0, S, "bf16x_fp8j")
    m.run(S)
    e = m.energy().cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    dt, zeta = oracle_schedules(S)
    ref = oracle.run(J.astype(np.float64), x0.T.astype(np.float64), None, dt, zeta, qmax=QMAX)
    e_ref = oracle.ising_energy(J, oracle.spins(ref["Q"])).astype(np.float64)
    se = np.sqrt(e.var() / r + e_ref.var() / r)
    announce(f"  mean {e.mean():.2f} vs oracle {e_ref.mean():.2f} (se {se:.2f}); "
             f"min {e.min():.0f} vs {e_ref.min():.0f}")
    assert abs(e.mean() - e_ref.mean()) <= 4 * se + 1e-9


def test_format_requirements():
    si = ensure_built()
    announce("precision format requirements")
    n, r = 64, 4
    x0 = instances.make_x0(n, r, 0)
    G = instances.make_gauss(n, 0)
    for prec in ("bf16x_bf16j", "bf16x_fp8j", "bf16x3_exactj"):
        with pytest.raises(si.SpringIsingError) as e:
            _model(G, x0, 10, prec)
        assert e.value.status == si.SI_ERR_UNSUPPORTED
    # 3.5 and -0.25 are exact in FP8 e4m3; hi/lo accepts anything
    J = np.zeros((n, n), np.float32)
    J[0, 1] = J[1, 0] = 3.5
    J[2, 3] = J[3, 2] = -0.25
    m = _model(J, x0, 10, "bf16x_fp8j")
    assert m.info()["j_fp8_exact"] == 1
    m.close()
    _model(G, x0, 10, "bf16x_hiloj").close()
