"""Precision forms at their full configurations, against the FP64 oracle.

* +-1 couplings in FP8 e4m3 (exact), N = 2000, R = 2048, 5000 steps.
* Gaussian couplings split into hi + lo BF16, N = 8000, R = 2048, 5000 steps.

Both run in the launch configuration the library picks for that shape.  The
oracle cannot follow 2048 replicas at these sizes, so it is used on sampled
replicas: one step from the same state must stay inside the element-wise
bound that BF16 rounding of the positions (and the hi + lo residual of J)
allows, and the energies of the GPU's final spins are recomputed exactly.
The full runs are compared with the plain FP32 method at the same
configuration as distributions of final energies.
"""
import time

import numpy as np
import pytest

import oracle
from paper_2305_07187_amd import instances

from gpu_common import QMAX, announce, ensure_built, oracle_schedules, to_dev

pytestmark = pytest.mark.gpu

R, S = 2048, 5000
COLS = [0, 1, 777, 1500, 2047]


def _one_step_sampled(si, Jd, J64, precision, seed, r=R, cols=COLS):
    """One step at t = 37 from a random state; check sampled replicas."""
    import torch
    n = J64.shape[0]
    x = instances.random_state(n, r, seed, scale=1.4)
    p0 = instances.random_state(n, r, seed + 1, scale=1.9)
    m = si.SpringIsing(Jd, to_dev(instances.make_x0(n, r, 0)), total_steps=S,
                       precision=precision)
    m.set_state(to_dev(x), to_dev(p0), 37)
    m.step()
    xg, pg, _ = m.state()
    torch.cuda.synchronize()
    name = m.info()["kernel_name"]
    m.close()
    dt, zeta = oracle_schedules(S)
    d, z = float(dt[37]), float(zeta[37])
    xs = x[cols].T.astype(np.float64)
    Q, P = oracle.step(J64, xs, p0[cols].T.astype(np.float64), d, z, qmax=QMAX)
    mag = np.abs(J64) @ np.abs(xs)
    jrel = 2.0 ** -16 if precision == "bf16x_hiloj" else 0.0
    qrel = 0.0 if precision == "bf16x3_exactj" else 2.0 ** -8  # BF16 positions
    bound = d * z * mag * (qrel + jrel) * 1.01 + 4 * 2.0 ** -24 * (np.abs(P) + 2.0) \
        + d * z * mag * n * 2.0 ** -24
    err = np.abs(pg.cpu().numpy()[cols].T - P)
    assert np.all(err <= bound), (err.max(), float(bound[np.argmax(err - bound)]))
    assert np.abs(xg.cpu().numpy()[cols].T - Q).max() <= 4e-7
    announce(f"  {precision} ({name}) one-step momentum error vs FP64 oracle: max {err.max():.3e}, "
             f"relative {err.max() / np.abs(P).max():.3e}, worst fraction of bound "
             f"{float((err / bound).max()):.3f}")


def _full_run(si, Jd, x0, precision):
    """5000 steps from x0; returns (spins [R, N] int8, energies, ms per step)."""
    import torch
    m = si.SpringIsing(Jd, x0, total_steps=S, precision=precision)
    m.run(20)
    m.set_state(x0, None, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.run(S)
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - t0) / S
    s = m.spins().cpu().numpy()
    integer = m.info()["j_integer"]
    e = m.energy(exact=bool(integer)).cpu().numpy()
    name = m.info()["kernel_name"]
    m.close()
    announce(f"  {precision} ({name}): {S} steps at {ms:.3f} ms/step")
    return s, e.astype(np.float64), ms


def _compare_distributions(e_lp, e_32, label):
    from scipy.stats import ks_2samp
    se = np.sqrt(e_lp.var() / len(e_lp) + e_32.var() / len(e_32))
    diff = (e_lp.mean() - e_32.mean()) / se
    ks = ks_2samp(e_lp, e_32).pvalue
    announce(f"  {label}: mean energy {e_lp.mean():.2f} vs FP32 {e_32.mean():.2f} "
             f"({diff:+.2f} s.e.), best {e_lp.min():.2f} vs {e_32.min():.2f}, KS p = {ks:.3f}")
    assert abs(diff) < 4.0
    assert ks > 1e-3


@pytest.mark.parametrize("precision", ["bf16x_fp8j", "bf16x_bf16j", "bf16x3_exactj"])
def test_forms_one_step_at_benchmark_shape(precision):
    # The time-to-target workload (N = 2000, R = 1024) in the launch
    # configuration the library picks for it: one step on sampled replicas
    # against the oracle (the three-plane split: FP32 accumulation only).
    si = ensure_built()
    n, r = 2000, 1024
    announce(f"{precision} one step at N={n} R={r}, sampled replicas")
    J = instances.make_pm1(n, 0)
    _one_step_sampled(si, to_dev(J), J.astype(np.float64), precision, 41, r=r,
                      cols=[0, 3, 511, 512, 1000, 1023])


def test_fp8_pm1_full_configuration():
    import torch
    si = ensure_built()
    n = 2000
    announce(f"bf16x_fp8j full configuration N={n} R={R} S={S}")
    J = instances.make_pm1(n, 0)
    J64 = J.astype(np.float64)
    Jd = to_dev(J)
    _one_step_sampled(si, Jd, J64, "bf16x_fp8j", 21)
    x0 = to_dev(instances.make_x0(n, R, 0))
    s8, e8, ms8 = _full_run(si, Jd, x0, "bf16x_fp8j")
    s32, e32, ms32 = _full_run(si, Jd, x0, "fp32")
    # energies of the GPU's own spins, recomputed exactly by the oracle
    for s, e in ((s8, e8), (s32, e32)):
        ref = oracle.ising_energy(J, s[COLS].T)
        np.testing.assert_array_equal(e[COLS].astype(np.int64), ref)
    _compare_distributions(e8, e32, "fp8 J vs FP32")
    announce(f"  step time FP8-J {ms8:.3f} ms vs FP32 {ms32:.3f} ms ({ms32 / ms8:.2f}x)")
    del torch


def test_hilo_gauss_full_configuration():
    import torch
    si = ensure_built()
    n = 8000
    announce(f"bf16x_hiloj full configuration N={n} R={R} S={S}")
    Jd = instances.make_gauss_torch(n, 0, device="cuda:0")
    J = Jd.cpu().numpy()
    J64 = J.astype(np.float64)
    _one_step_sampled(si, Jd, J64, "bf16x_hiloj", 31)
    x0 = to_dev(instances.make_x0(n, R, 0))
    sh, eh, msh = _full_run(si, Jd, x0, "bf16x_hiloj")
    s32, e32, ms32 = _full_run(si, Jd, x0, "fp32")
    # real couplings: the FP32 readout of the GPU's spins within its
    # accumulation bound of the exact FP64 energy
    bound = n * 2.0 ** -24 * np.abs(J64).sum() + 1e-6
    for s, e in ((sh, eh), (s32, e32)):
        ref = oracle.ising_energy(J64, s[COLS].T)
        assert np.all(np.abs(e[COLS] - ref) <= bound), (np.abs(e[COLS] - ref).max(), bound)
    _compare_distributions(eh, e32, "hi+lo J vs FP32")
    announce(f"  step time hi+lo {msh:.3f} ms vs FP32 {ms32:.3f} ms ({ms32 / msh:.2f}x)")
    del torch
