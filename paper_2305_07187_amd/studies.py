"""Dynamic-equilibrium (zeta) strategy study of Fig. 5 on the synthetic
K2000-shaped instance, run entirely on the HIP hot path.

Fig. 5 compares a fixed zeta of 0.8 zeta0 or 10 zeta0 with schedules that
rise from 0.8 zeta0 to 10 zeta0 in stairs of 200 or 1000 steps (zeta0 = 0.05).
This study runs those four strategies, the exactly linear schedule, and the
linear schedule with zeta scaled down (the paper prints no normalisation of
J, so the scale of zeta against the spectrum of J is a free choice).  For each
it reports the final and the best-along-the-run cut (energy checked every 50
steps on the device) over all replicas.

    python -m paper_2305_07187_amd.studies [--replicas R] [--steps S]
"""
from __future__ import annotations

import argparse
import json
import time


def zeta_strategies(n=2000, replicas=1024, steps=10000, seed=0, check_every=50):
    import numpy as np
    import torch

    from . import instances
    from . import spring_ising as si

    dev = torch.device("cuda:0")
    Jn = instances.make_pm1(n, seed)
    J = torch.from_numpy(Jn).to(dev)
    x0 = torch.from_numpy(instances.make_x0(n, replicas, seed)).to(dev)
    W = float(-np.triu(Jn.astype(np.float64), 1).sum())
    z0 = 0.05
    f32 = lambda v: float(np.float32(v))
    strategies = {
        "fixed_0.8zeta0": dict(zeta_start=f32(0.8 * z0), zeta_end=f32(0.8 * z0)),
        "fixed_10zeta0": dict(zeta_start=f32(10 * z0), zeta_end=f32(10 * z0)),
        "stairs_1000": dict(stair_len=1000),
        "stairs_200": dict(stair_len=200),
        "linear": dict(stair_len=1),
        "linear_x0.25": dict(zeta_start=f32(0.25 * 0.8 * z0), zeta_end=f32(0.25 * 10 * z0)),
        "linear_x0.1": dict(zeta_start=f32(0.1 * 0.8 * z0), zeta_end=f32(0.1 * 10 * z0)),
    }
    out = {"workload": f"K2000-shaped +-1 complete graph N={n}, R={replicas}, {steps} steps",
           "strategies": {}}
    for name, kw in strategies.items():
        m = si.SpringIsing(J, x0, total_steps=steps, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps // check_every):
            m.run(check_every)
            m.update_best()
        e_final = m.energy().cpu().numpy().astype(np.float64)
        best_e, _ = m.best()
        best_e = best_e.cpu().numpy()
        el = time.perf_counter() - t0
        cut_f = (W - e_final) / 2
        cut_b = (W - best_e) / 2
        out["strategies"][name] = {
            "final_cut_mean": float(cut_f.mean()), "final_cut_best": float(cut_f.max()),
            "run_best_cut_mean": float(cut_b.mean()), "run_best_cut_best": float(cut_b.max()),
            "seconds": el}
        m.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--replicas", type=int, default=1024)
    ap.add_argument("--steps", type=int, default=10000)
    args = ap.parse_args()
    print(json.dumps(zeta_strategies(replicas=args.replicas, steps=args.steps), indent=1))


if __name__ == "__main__":
    main()
