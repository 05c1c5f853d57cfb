"""The largest supported sizes, with closed-form expected values.

J is the complete ferromagnet (J_ij = 1 for i != j) and the positions are
+-0.25 (seeded signs): every product is exact and every partial sum is a
multiple of 0.25 below 2^14 in magnitude, so the FP32 coupling sums are
exact at any N, and the step and the energy have closed forms:
    F_i = S - q_i (S = sum_j q_j),  E = -((sum_i s_i)^2 - N) / 2.
N = 65536 is the largest N the library accepts; N = 46340 is the largest
at which the exact int32 energy is available (N^2 max|J| < 2^31).
"""
import numpy as np
import pytest

from paper_2305_07187_amd import instances

from gpu_common import DT, QMAX, ZS, announce, ensure_built

pytestmark = pytest.mark.gpu


def _ferromagnet(n):
    import torch
    J = torch.ones(n, n, dtype=torch.float32, device="cuda:0")
    J.fill_diagonal_(0.0)
    return J


def _signs(n, r, seed):
    return np.where(instances.make_x0(n, r, seed) < 0, -0.25, 0.25).astype(np.float32)


def _closed_form_step(q):
    """One paper-order step from (q, p = 0) at the first schedule entry,
    F = S - q, evaluated in float64."""
    q64 = q.astype(np.float64)
    F = q64.sum(axis=1, keepdims=True) - q64
    dt, zeta, k = float(DT), float(ZS), 0.5
    P = np.clip(dt * (-k * q64 + zeta * F), -2.0, 2.0)
    Q = np.clip(q64, -QMAX, QMAX)  # p = 0, so q does not move
    return Q, P


def test_largest_n_one_step_and_energy():
    import torch
    si = ensure_built()
    n, r = 65536, 3
    announce(f"largest N: complete ferromagnet N={n} R={r}, one step and the energy")
    J = _ferromagnet(n)
    x = _signs(n, r, 3)
    m = si.SpringIsing(J, torch.from_numpy(x).cuda(), total_steps=4)
    del J
    torch.cuda.empty_cache()
    info = m.info()
    assert info["n_pad"] == 65536 and info["j_integer"] == 1
    m.step()
    q, p, t = m.state()
    torch.cuda.synchronize()
    Q, P = _closed_form_step(x)
    qg, pg = q.cpu().numpy().astype(np.float64), p.cpu().numpy().astype(np.float64)
    assert t == 1 and np.array_equal(qg, Q)
    # F is exact; the update rounds twice in FP32 (the force, then dt * force)
    F = x.astype(np.float64).sum(axis=1, keepdims=True) - x
    bound = 2.0 ** -22 * float(DT) * (float(ZS) * np.abs(F) + 0.5 * np.abs(x)) + 2.0 ** -23 * np.abs(P)
    err = np.abs(pg - P)
    assert np.all(err <= bound), float((err / bound).max())
    # exact int32 energy is out of range here (N^2 > 2^31): the real energy
    # is exact as well for +-1 sums (integers below 2^24 per row tile)
    with pytest.raises(si.SpringIsingError) as e:
        m.energy(exact=True)
    assert e.value.status == si.SI_ERR_UNSUPPORTED
    er = m.energy(exact=False).cpu().numpy()
    s = np.where(qg < 0, -1, 1).sum(axis=1).astype(np.float64)
    np.testing.assert_array_equal(er, -(s * s - n) / 2)
    announce(f"  {info['kernel_name']}: max momentum error {err.max():.2e}; energies {er.tolist()}")
    m.close()


def test_largest_exact_energy():
    import torch
    si = ensure_built()
    n, r = 46340, 2
    announce(f"largest exact int32 energy: complete ferromagnet N={n}")
    J = _ferromagnet(n)
    x = _signs(n, r, 4)
    x[1] = 0.25  # all spins up: the extreme energy -N(N-1)/2
    m = si.SpringIsing(J, torch.from_numpy(x).cuda(), total_steps=2)
    del J
    torch.cuda.empty_cache()
    e = m.energy(exact=True).cpu().numpy().astype(np.int64)
    s = np.where(x < 0, -1, 1).sum(axis=1).astype(np.int64)
    np.testing.assert_array_equal(e, -(s * s - n) // 2)
    assert e[1] == -n * (n - 1) // 2
    announce(f"  energies {e.tolist()}")
    m.close()


def test_sizes_beyond_the_limit_are_refused():
    import torch
    si = ensure_built()
    J = torch.zeros(1, 1, device="cuda:0")
    x = torch.zeros(1, 1, device="cuda:0")
    lib = si.load_library()
    prm = si.spring_ising_default_params(4)
    import ctypes
    ctx = ctypes.c_void_p()
    rc = lib.spring_ising_init(ctypes.byref(ctx), 65537, 1, ctypes.c_void_p(J.data_ptr()),
                               ctypes.c_void_p(x.data_ptr()), None, ctypes.byref(prm), None)
    assert rc == si.SI_ERR_INVALID and not ctx.value


@pytest.mark.parametrize("precision", ["bf16x_fp8j", "bf16x_bf16j", "bf16x_hiloj", "bf16x3_exactj"])
def test_largest_n_precision_forms(precision):
    # The same closed form through the BF16 matrix cores: +-1 couplings are
    # exact in FP8 and BF16 (hi + lo: lo = 0), +-0.25 positions are exact in
    # BF16 (three-plane split: lower planes 0), every product is exact and
    # every FP32 partial sum is a multiple of 0.25 below 2^14, so one step
    # has the FP32 form's closed-form values; 64-bit offsets throughout.
    import torch
    si = ensure_built()
    n, r = 65536, 3
    announce(f"largest N in {precision}: complete ferromagnet N={n} R={r}, one step")
    J = _ferromagnet(n)
    x = _signs(n, r, 5)
    m = si.SpringIsing(J, torch.from_numpy(x).cuda(), total_steps=4, precision=precision)
    del J
    torch.cuda.empty_cache()
    assert m.info()["n_pad"] >= n
    m.step()
    q, p, t = m.state()
    torch.cuda.synchronize()
    Q, P = _closed_form_step(x)
    qg, pg = q.cpu().numpy().astype(np.float64), p.cpu().numpy().astype(np.float64)
    assert t == 1 and np.array_equal(qg, Q)
    F = x.astype(np.float64).sum(axis=1, keepdims=True) - x
    bound = 2.0 ** -22 * float(DT) * (float(ZS) * np.abs(F) + 0.5 * np.abs(x)) + 2.0 ** -23 * np.abs(P)
    err = np.abs(pg - P)
    assert np.all(err <= bound), float((err / bound).max())
    er = m.energy(exact=False).cpu().numpy()
    s = np.where(qg < 0, -1, 1).sum(axis=1).astype(np.float64)
    np.testing.assert_array_equal(er, -(s * s - n) / 2)
    announce(f"  {m.info()['kernel_name']}: max momentum error {err.max():.2e}")
    m.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16x_mixedj"])
def test_largest_n_in_a_batch(precision):
    # a batch holding the largest instance beside a small one: the large
    # member follows the closed form, the small one its standalone run
    import torch
    si = ensure_built()
    n, r = 65536, 3
    announce(f"largest N inside a batch ({precision})")
    J = _ferromagnet(n)
    x = _signs(n, r, 7)
    Js = instances.make_pm1(100, 3)
    xs = instances.make_x0(100, r, 3)
    b = si.SpringIsingBatch([J, torch.from_numpy(Js).cuda()],
                            [torch.from_numpy(x).cuda(), torch.from_numpy(xs).cuda()],
                            total_steps=4, precision=precision)
    del J
    torch.cuda.empty_cache()
    b.step()
    qb, pb, t = b.state()
    torch.cuda.synchronize()
    Q, P = _closed_form_step(x)
    qg, pg = qb[0].cpu().numpy().astype(np.float64), pb[0].cpu().numpy().astype(np.float64)
    assert t == 1 and np.array_equal(qg, Q)
    F = x.astype(np.float64).sum(axis=1, keepdims=True) - x
    bound = 2.0 ** -22 * float(DT) * (float(ZS) * np.abs(F) + 0.5 * np.abs(x)) + 2.0 ** -23 * np.abs(P)
    assert np.all(np.abs(pg - P) <= bound)
    form, tile = ("fp32", 14) if precision == "fp32" else ("bf16x_fp8j", 9)
    m = si.SpringIsing(torch.from_numpy(Js).cuda(), torch.from_numpy(xs).cuda(), total_steps=4,
                       precision=form, tile=tile)
    m.step()
    q1, p1, _ = m.state()
    torch.cuda.synchronize()
    assert np.array_equal(q1.cpu().numpy(), qb[1].cpu().numpy())
    assert np.array_equal(p1.cpu().numpy(), pb[1].cpu().numpy())
    e = b.energy(exact=False)
    s = np.where(qg < 0, -1, 1).sum(axis=1).astype(np.float64)
    np.testing.assert_array_equal(e[0].cpu().numpy(), -(s * s - n) / 2)
    m.close()
    b.close()
