"""Shared helpers for the GPU tests (inputs from the seeded generator only)."""
import math
import os
import sys

import numpy as np

F32 = lambda x: float(np.float32(x))
QMAX = F32(math.sqrt(2.0))
ZS, ZE, DT = F32(0.04), F32(0.5), F32(0.2)


def announce(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def ensure_built():
    from paper_2305_07187_amd import spring_ising as si
    if not os.path.exists(si.LIB_PATH):
        from paper_2305_07187_amd import build
        build.build(verbose=False)
    si.load_library()
    return si


def oracle_schedules(S, stair=1, zs=ZS, ze=ZE, dt=DT):
    import oracle
    return oracle.dt_schedule(S, dt), oracle.zeta_schedule(S, zs, ze, stair)


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def rel_err(gpu_rn, ref_nr):
    """max-norm relative error; gpu state is [R, N], oracle state is [N, R]."""
    g = np.asarray(gpu_rn, dtype=np.float64).T
    den = max(np.abs(ref_nr).max(), 1e-30)
    return float(np.abs(g - ref_nr).max() / den)
