"""Python binding of the Spring-Ising C ABI (include/spring_ising.h).

Argument marshalling only: every function below forwards to the entry point
of the same name in libspring_ising.so, passing device pointers of torch
tensors and the current HIP stream.  No step of the method runs in Python;
if the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libspring_ising.so")

SI_OK = 0
SI_ERR_INVALID = -1
SI_ERR_OOM = -2
SI_ERR_HIP = -3
SI_ERR_STATE = -4
SI_ERR_UNSUPPORTED = -5
SI_ERR_RANGE = -6
STATUS_NAMES = {0: "SI_OK", -1: "SI_ERR_INVALID", -2: "SI_ERR_OOM", -3: "SI_ERR_HIP",
                -4: "SI_ERR_STATE", -5: "SI_ERR_UNSUPPORTED", -6: "SI_ERR_RANGE"}

SI_ORDER_PAPER, SI_ORDER_SYMPLECTIC = 0, 1
SI_WALL_CLAMP, SI_WALL_INELASTIC = 0, 1
SI_PREC_FP32 = 0
SI_PREC_BF16X_FP8J = 1
SI_PREC_BF16X_BF16J = 2
SI_PREC_BF16X_HILOJ = 3
SI_PREC_BF16X3_EXACTJ = 4
SI_PREC_BF16X_MIXEDJ = 5
PRECISIONS = {"fp32": 0, "bf16x_fp8j": 1, "bf16x_bf16j": 2, "bf16x_hiloj": 3, "bf16x3_exactj": 4,
              "bf16x_mixedj": 5}


class si_params(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_float), ("m", ctypes.c_float), ("dt", ctypes.c_float),
        ("zeta_start", ctypes.c_float), ("zeta_end", ctypes.c_float),
        ("total_steps", ctypes.c_int32), ("stair_len", ctypes.c_int32),
        ("qmax", ctypes.c_float), ("pmax", ctypes.c_float),
        ("order", ctypes.c_int32), ("wall", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("tile", ctypes.c_int32),
        ("energy_every", ctypes.c_int32),
    ]


class si_info(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("r", ctypes.c_int32),
        ("n_pad", ctypes.c_int32), ("r_pad", ctypes.c_int32),
        ("t", ctypes.c_int32), ("total_steps", ctypes.c_int32),
        ("j_integer", ctypes.c_int32), ("j_fp8_exact", ctypes.c_int32),
        ("j_bf16_exact", ctypes.c_int32), ("tile", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("graph_steps", ctypes.c_int32),
        ("device_bytes", ctypes.c_int64), ("kernel_name", ctypes.c_char * 64),
        ("resident_steps", ctypes.c_int32), ("resident_groups", ctypes.c_int32),
        ("tile_source", ctypes.c_int32), ("n_inst", ctypes.c_int32),
    ]

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["kernel_name"] = self.kernel_name.decode()
        return d


class SpringIsingError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


_lib = None
_P = ctypes.c_void_p
_I = ctypes.c_int32

_SIGNATURES = {
    "spring_ising_default_params": [ctypes.POINTER(si_params), _I],
    "spring_ising_init": [ctypes.POINTER(_P), _I, _I, _P, _P, _P, ctypes.POINTER(si_params), _P],
    "spring_ising_set_schedule": [_P, _P, _P],
    "spring_ising_get_schedule": [_P, _P, _P],
    "spring_ising_set_field": [_P, _P],
    "spring_ising_step": [_P],
    "spring_ising_run": [_P, _I],
    "spring_ising_spins": [_P, _P],
    "spring_ising_energy": [_P, _P, _P],
    "spring_ising_get_state": [_P, _P, _P, ctypes.POINTER(_I)],
    "spring_ising_set_state": [_P, _P, _P, _I],
    "spring_ising_info": [_P, ctypes.POINTER(si_info)],
    "spring_ising_relaxed_energy_grad": [_P, _I, _P, _P, _P],
    "spring_ising_relaxed_energy_forward": [_P, _I, _P],
    "spring_ising_tile_cache_save": [ctypes.c_char_p],
    "spring_ising_tile_cache_load": [ctypes.c_char_p, ctypes.POINTER(_I)],
    "spring_ising_tile_cache_clear": [],
    "spring_ising_batch_timeline": [_P, _I, _P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(ctypes.c_double)],
    "spring_ising_relaxed_energy_backward": [_P, _P, _P],
    "spring_ising_set_graph": [_P, _I],
    "spring_ising_set_resident": [_P, _I],
    "spring_ising_set_ksplit": [_P, _I],
    "spring_ising_update_best": [_P],
    "spring_ising_get_best": [_P, _P, _P],
    "spring_ising_hamiltonian": [_P, _P],
    "spring_ising_autotune": [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_float)],
    "spring_ising_init_batch": [ctypes.POINTER(_P), _I, _P, _I, _P, _P, _P,
                                ctypes.POINTER(si_params), _P],
    "spring_ising_debug_inject_hip_error": [_P, _I],
    "spring_ising_energy_noalloc": [_I, _I, _P, _P, _P, _P],
    "spring_ising_get_energy_trace": [_P, _P, ctypes.POINTER(_I)],
    "spring_ising_destroy": [_P],
}


def load_library(path: str = LIB_PATH):
    """Load libspring_ising.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with "
                           "`python -m paper_2305_07187_amd.build` (no fallback exists)")
    # refuse a library built from other sources than those in the tree
    from . import build as _build
    expected = _build.check_fresh(path)
    # torch carries its own copy of the HIP runtime; load it first so that
    # the library binds to that copy and recognises torch's device pointers
    # (a second runtime in the process would not know them)
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, args in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.spring_ising_last_error.argtypes = []
    lib.spring_ising_last_error.restype = ctypes.c_char_p
    lib.spring_ising_build_id.argtypes = []
    lib.spring_ising_build_id.restype = ctypes.c_char_p
    loaded = lib.spring_ising_build_id().decode()
    if loaded != expected:
        raise _build.StaleLibraryError(f"loaded library reports build id {loaded}, "
                                       f"file and tree {expected}")
    _lib = lib
    return lib


def last_error() -> str:
    return load_library().spring_ising_last_error().decode()


def spring_ising_build_id() -> str:
    return load_library().spring_ising_build_id().decode()


def spring_ising_energy_noalloc(J, x, e_int, stream=None):
    """J: [N, N] float32, x: [R, N] float32, e_int: [R] int32 CUDA tensors."""
    import torch
    n, r = int(J.shape[0]), int(x.shape[0])
    _check(load_library().spring_ising_energy_noalloc(
        n, r, _ptr(J, torch.float32, n * n, "J"), _ptr(x, torch.float32, n * r, "x"),
        _ptr(e_int, torch.int32, r, "e_int"), stream if stream is not None else _stream()))


def spring_ising_get_energy_trace(ctx, e=None):
    """Copy the recorded in-run energy checks into e (float64 CUDA tensor, or
    None to query); returns the number of rows recorded."""
    import torch
    k = ctypes.c_int32()
    _check(load_library().spring_ising_get_energy_trace(ctx, _ptr(e, torch.float64, name="e"),
                                                       ctypes.byref(k)))
    return k.value


def spring_ising_debug_inject_hip_error(ctx, n):
    _check(load_library().spring_ising_debug_inject_hip_error(ctx, int(n)))


def _check(status: int):
    if status != SI_OK:
        raise SpringIsingError(status, last_error())


def _ptr(t, dtype=None, numel=None, name="tensor"):
    """Device pointer of a contiguous CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must live on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# ---------------------------------------------------------------- C-ABI mirrors
def spring_ising_default_params(total_steps: int) -> si_params:
    p = si_params()
    _check(load_library().spring_ising_default_params(ctypes.byref(p), int(total_steps)))
    return p


def spring_ising_init(n, r, J, x0, p0=None, params=None, stream=None):
    import torch
    lib = load_library()
    if params is None:
        raise ValueError("params required (spring_ising_default_params)")
    ctx = ctypes.c_void_p()
    st = lib.spring_ising_init(ctypes.byref(ctx), int(n), int(r),
                               _ptr(J, torch.float32, n * n, "J"),
                               _ptr(x0, torch.float32, n * r, "x0"),
                               _ptr(p0, torch.float32, n * r, "p0"),
                               ctypes.byref(params), stream if stream is not None else _stream())
    _check(st)
    return ctx


def spring_ising_init_batch(ns, r, Js, x0s, params, stream=None, p0s=None):
    """Js, x0s: lists of CUDA float32 tensors (n_i*n_i and r*n_i elements);
    p0s: None (zero momenta) or a list of such tensors or None per instance."""
    import torch
    lib = load_library()
    k = len(ns)
    if not (len(Js) == len(x0s) == k) or (p0s is not None and len(p0s) != k):
        raise ValueError("one J, one x0 (and one p0 entry if given) per instance")
    p_arr = None
    if p0s is not None:
        p_arr = (ctypes.c_void_p * k)(*[None if p0s[i] is None else
                                        _ptr(p0s[i], torch.float32, ns[i] * r, "p0").value
                                        for i in range(k)])
    n_arr = (ctypes.c_int32 * k)(*[int(v) for v in ns])
    j_arr = (ctypes.c_void_p * k)(*[_ptr(Js[i], torch.float32, ns[i] * ns[i], "J").value
                                    for i in range(k)])
    x_arr = (ctypes.c_void_p * k)(*[_ptr(x0s[i], torch.float32, ns[i] * r, "x0").value
                                    for i in range(k)])
    ctx = ctypes.c_void_p()
    st = lib.spring_ising_init_batch(ctypes.byref(ctx), k, ctypes.cast(n_arr, ctypes.c_void_p),
                                     int(r), ctypes.cast(j_arr, ctypes.c_void_p),
                                     ctypes.cast(x_arr, ctypes.c_void_p),
                                     None if p_arr is None else ctypes.cast(p_arr, ctypes.c_void_p),
                                     ctypes.byref(params),
                                     stream if stream is not None else _stream())
    _check(st)
    return ctx


def spring_ising_set_schedule(ctx, dt, zeta):
    import torch
    _check(load_library().spring_ising_set_schedule(ctx, _ptr(dt, torch.float32, name="dt"),
                                                    _ptr(zeta, torch.float32, name="zeta")))


def spring_ising_get_schedule(ctx, dt, zeta):
    import torch
    _check(load_library().spring_ising_get_schedule(ctx, _ptr(dt, torch.float32, name="dt"),
                                                    _ptr(zeta, torch.float32, name="zeta")))


def spring_ising_set_field(ctx, h):
    import torch
    _check(load_library().spring_ising_set_field(ctx, _ptr(h, torch.float32, name="h")))


def spring_ising_step(ctx):
    _check(load_library().spring_ising_step(ctx))


def spring_ising_run(ctx, n_steps):
    _check(load_library().spring_ising_run(ctx, int(n_steps)))


def spring_ising_spins(ctx, s):
    import torch
    _check(load_library().spring_ising_spins(ctx, _ptr(s, torch.int8, name="s")))


def spring_ising_energy(ctx, e_int=None, e_real=None):
    import torch
    _check(load_library().spring_ising_energy(ctx, _ptr(e_int, torch.int32, name="e_int"),
                                              _ptr(e_real, torch.float64, name="e_real")))


def spring_ising_get_state(ctx, x=None, p=None):
    import torch
    t = ctypes.c_int32()
    _check(load_library().spring_ising_get_state(ctx, _ptr(x, torch.float32, name="x"),
                                                 _ptr(p, torch.float32, name="p"),
                                                 ctypes.byref(t)))
    return t.value


def spring_ising_set_state(ctx, x, p=None, t=0):
    import torch
    _check(load_library().spring_ising_set_state(ctx, _ptr(x, torch.float32, name="x"),
                                                 _ptr(p, torch.float32, name="p"), int(t)))


def spring_ising_relaxed_energy_grad(ctx, ckpt_every, loss, dl_ddt, dl_dzeta):
    import torch
    _check(load_library().spring_ising_relaxed_energy_grad(
        ctx, int(ckpt_every), _ptr(loss, torch.float64, 1, "loss"),
        _ptr(dl_ddt, torch.float64, name="dL_ddt"), _ptr(dl_dzeta, torch.float64, name="dL_dzeta")))


def spring_ising_relaxed_energy_forward(ctx, ckpt_every, loss):
    import torch
    _check(load_library().spring_ising_relaxed_energy_forward(
        ctx, int(ckpt_every), _ptr(loss, torch.float64, 1, "loss")))


def spring_ising_relaxed_energy_backward(ctx, dl_ddt, dl_dzeta):
    import torch
    _check(load_library().spring_ising_relaxed_energy_backward(
        ctx, _ptr(dl_ddt, torch.float64, name="dL_ddt"),
        _ptr(dl_dzeta, torch.float64, name="dL_dzeta")))


def spring_ising_update_best(ctx):
    _check(load_library().spring_ising_update_best(ctx))


def spring_ising_get_best(ctx, best_e=None, best_s=None):
    import torch
    _check(load_library().spring_ising_get_best(ctx, _ptr(best_e, torch.float64, name="best_e"),
                                                _ptr(best_s, torch.int8, name="best_s")))


def spring_ising_hamiltonian(ctx, H):
    import torch
    _check(load_library().spring_ising_hamiltonian(ctx, _ptr(H, torch.float64, name="H")))


def spring_ising_set_graph(ctx, min_steps):
    _check(load_library().spring_ising_set_graph(ctx, int(min_steps)))


def spring_ising_set_resident(ctx, min_steps):
    _check(load_library().spring_ising_set_resident(ctx, int(min_steps)))


def spring_ising_set_ksplit(ctx, ksplit):
    _check(load_library().spring_ising_set_ksplit(ctx, int(ksplit)))


def spring_ising_autotune(ctx, steps):
    tile = ctypes.c_int32()
    us = ctypes.c_float()
    _check(load_library().spring_ising_autotune(ctx, int(steps), ctypes.byref(tile),
                                                ctypes.byref(us)))
    return tile.value, us.value


TILE_SOURCES = {0: "table", 1: "cache", 2: "caller", 3: "autotune"}


def spring_ising_batch_timeline(ctx, n_steps):
    """Run n_steps traced steps of a batch; returns (records uint64 [k, 4]:
    start, end, CU, step << 32 | item; clock rate in MHz)."""
    import numpy as np
    lib = load_library()
    need = ctypes.c_int64()
    mhz = ctypes.c_double()
    st = lib.spring_ising_batch_timeline(ctx, int(n_steps), None, 0, ctypes.byref(need), None)
    if need.value == 0:
        _check(st)
    out = np.zeros((need.value, 4), dtype=np.uint64)
    _check(lib.spring_ising_batch_timeline(ctx, int(n_steps), out.ctypes.data, need.value,
                                           ctypes.byref(need), ctypes.byref(mhz)))
    return out, mhz.value


def batch_timeline_stats(records, clock_mhz):
    """Per-step figures of a batch timeline: span (first start to last end),
    the CUs' mean and least busy share of the span (a CU counts as busy while
    any of its workgroups runs), the time from the first CU running out of
    work to the end, and the gap to the next step's first start (us)."""
    import numpy as np
    steps = (records[:, 3] >> np.uint64(32)).astype(np.int64)
    out = []
    for s in np.unique(steps):
        r = records[steps == s]
        t0 = r[:, 0].astype(np.int64)
        t1 = r[:, 1].astype(np.int64)
        base = t0.min()
        span = t1.max() - base
        busy, ends = [], []
        for cu in np.unique(r[:, 2]):
            m = r[:, 2] == cu
            iv = sorted(zip(t0[m], t1[m]))
            tot, cs, ce = 0, iv[0][0], iv[0][1]
            for a, b in iv[1:]:
                if a > ce:
                    tot += ce - cs
                    cs, ce = a, b
                else:
                    ce = max(ce, b)
            busy.append(tot + ce - cs)
            ends.append(ce)
        busy = np.array(busy, dtype=np.float64)
        us = 1.0 / clock_mhz
        out.append({"step": int(s), "span_us": span * us, "cus": len(busy),
                    "cu_busy_mean": float(busy.mean() / span),
                    "cu_busy_min": float(busy.min() / span),
                    "tail_us": float((t1.max() - min(ends)) * us),
                    "start": int(base), "end": int(t1.max())})
    for a, b in zip(out, out[1:]):
        a["gap_to_next_us"] = (b["start"] - a["end"]) / clock_mhz
    return out


def spring_ising_tile_cache_save(path):
    _check(load_library().spring_ising_tile_cache_save(os.fsencode(path)))


def spring_ising_tile_cache_load(path):
    n = ctypes.c_int32()
    _check(load_library().spring_ising_tile_cache_load(os.fsencode(path), ctypes.byref(n)))
    return n.value


def spring_ising_tile_cache_clear():
    _check(load_library().spring_ising_tile_cache_clear())


def spring_ising_info(ctx) -> dict:
    info = si_info()
    _check(load_library().spring_ising_info(ctx, ctypes.byref(info)))
    return info.as_dict()


def spring_ising_destroy(ctx):
    _check(load_library().spring_ising_destroy(ctx))


# ------------------------------------------------------------ convenience
class SpringIsingBatch:
    """Owns one batched context: instances of uneven size stepped together.

    Js: list of [N_i, N_i] float32 CUDA tensors; x0s: list of [R, N_i];
    p0s: None (zero momenta) or a list of [R, N_i] tensors or None.
    Outputs are lists per instance.
    """

    def __init__(self, Js, x0s, total_steps=1000, p0s=None, **overrides):
        import torch
        self.ns = [int(J.shape[0]) for J in Js]
        self.r = int(x0s[0].shape[0])
        prm = spring_ising_default_params(total_steps)
        for key, val in overrides.items():
            if key == "precision" and isinstance(val, str):
                val = PRECISIONS[val]
            setattr(prm, key, val)
        self.total_steps = int(prm.total_steps)
        self.device = Js[0].device
        keep = ([J.contiguous() for J in Js], [x.contiguous() for x in x0s],
                None if p0s is None else [None if p is None else p.contiguous() for p in p0s])
        self.ctx = spring_ising_init_batch(self.ns, self.r, keep[0], keep[1], prm, p0s=keep[2])
        torch.cuda.current_stream().synchronize()
        self.offsets = [0]
        for n in self.ns:
            self.offsets.append(self.offsets[-1] + self.r * n)

    def close(self):
        if self.ctx is not None:
            spring_ising_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, n_steps):
        spring_ising_run(self.ctx, n_steps)

    def step(self):
        spring_ising_step(self.ctx)

    def set_graph(self, min_steps):
        spring_ising_set_graph(self.ctx, min_steps)

    def autotune(self, steps=5):
        """Time both batch tiles from the current state; keep and cache the
        faster.  Returns (tile, us per step)."""
        return spring_ising_autotune(self.ctx, steps)

    def timeline(self, n_steps=2):
        """n_steps traced steps: (records, clock MHz); see
        spring_ising_batch_timeline."""
        return spring_ising_batch_timeline(self.ctx, n_steps)

    def _split(self, flat):
        return [flat[self.offsets[i]:self.offsets[i + 1]].view(self.r, n)
                for i, n in enumerate(self.ns)]

    def state(self):
        import torch
        x = torch.empty(self.offsets[-1], dtype=torch.float32, device=self.device)
        p = torch.empty_like(x)
        t = spring_ising_get_state(self.ctx, x, p)
        return self._split(x), self._split(p), t

    def set_state(self, xs, ps=None, t=0):
        import torch
        x = torch.cat([v.reshape(-1) for v in xs]).contiguous()
        p = None if ps is None else torch.cat([v.reshape(-1) for v in ps]).contiguous()
        spring_ising_set_state(self.ctx, x, p, t)
        torch.cuda.current_stream().synchronize()

    def spins(self):
        import torch
        s = torch.empty(self.offsets[-1], dtype=torch.int8, device=self.device)
        spring_ising_spins(self.ctx, s)
        return self._split(s)

    def energy(self, exact=False):
        import torch
        k = len(self.ns)
        e_real = torch.empty(k * self.r, dtype=torch.float64, device=self.device)
        e_int = torch.empty(k * self.r, dtype=torch.int32, device=self.device) if exact else None
        spring_ising_energy(self.ctx, e_int, e_real)
        e = e_int if exact else e_real
        return [e[i * self.r:(i + 1) * self.r] for i in range(k)]

    def info(self):
        return spring_ising_info(self.ctx)

    def update_best(self):
        spring_ising_update_best(self.ctx)

    def best(self):
        """(best energies as a list per instance, best spins per instance)."""
        import torch
        k = len(self.ns)
        e = torch.empty(k * self.r, dtype=torch.float64, device=self.device)
        s = torch.empty(self.offsets[-1], dtype=torch.int8, device=self.device)
        spring_ising_get_best(self.ctx, e, s)
        return [e[i * self.r:(i + 1) * self.r] for i in range(k)], self._split(s)

    def energy_trace(self):
        """In-run checks so far: float64 tensor [checks, n_inst, R]."""
        import torch
        rows = spring_ising_get_energy_trace(self.ctx, None)
        e = torch.empty(max(rows, 1) * len(self.ns) * self.r, dtype=torch.float64,
                        device=self.device)
        spring_ising_get_energy_trace(self.ctx, e)
        return e[:rows * len(self.ns) * self.r].view(rows, len(self.ns), self.r)


class SpringIsing:
    """Owns one context; torch tensors carry inputs and outputs.

    J: [N, N] float32 CUDA tensor; x0: [R, N]; p0: [R, N] or None.
    """

    def __init__(self, J, x0, p0=None, total_steps=1000, *, precision="fp32", order="paper",
                 wall="clamp", tile=0, **overrides):
        import torch
        self.n = int(J.shape[0])
        self.r = int(x0.shape[0])
        prm = spring_ising_default_params(total_steps)
        prm.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        prm.order = {"paper": 0, "symplectic": 1}[order] if isinstance(order, str) else int(order)
        prm.wall = {"clamp": 0, "inelastic": 1}[wall] if isinstance(wall, str) else int(wall)
        prm.tile = int(tile)
        for key, val in overrides.items():
            if not hasattr(prm, key):
                raise KeyError(key)
            setattr(prm, key, val)
        self.params = prm
        self.total_steps = int(prm.total_steps)
        self.device = J.device
        self._keep = (J.contiguous(), x0.contiguous(), None if p0 is None else p0.contiguous())
        self.ctx = spring_ising_init(self.n, self.r, self._keep[0], self._keep[1], self._keep[2],
                                     prm)
        torch.cuda.current_stream().synchronize()
        self._keep = None

    def close(self):
        if self.ctx is not None:
            spring_ising_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self):
        spring_ising_step(self.ctx)

    def run(self, n_steps):
        spring_ising_run(self.ctx, n_steps)

    def state(self):
        import torch
        x = torch.empty(self.r, self.n, dtype=torch.float32, device=self.device)
        p = torch.empty_like(x)
        t = spring_ising_get_state(self.ctx, x, p)
        return x, p, t

    def set_state(self, x, p=None, t=0):
        spring_ising_set_state(self.ctx, x.contiguous(), None if p is None else p.contiguous(), t)

    def spins(self):
        import torch
        s = torch.empty(self.r, self.n, dtype=torch.int8, device=self.device)
        spring_ising_spins(self.ctx, s)
        return s

    def energy(self, exact=True):
        import torch
        e_real = torch.empty(self.r, dtype=torch.float64, device=self.device)
        if exact:
            e_int = torch.empty(self.r, dtype=torch.int32, device=self.device)
            spring_ising_energy(self.ctx, e_int, e_real)
            return e_int
        spring_ising_energy(self.ctx, None, e_real)
        return e_real

    def schedule(self):
        import torch
        dt = torch.empty(self.total_steps, dtype=torch.float32, device=self.device)
        zeta = torch.empty_like(dt)
        spring_ising_get_schedule(self.ctx, dt, zeta)
        return dt, zeta

    def set_schedule(self, dt, zeta):
        spring_ising_set_schedule(self.ctx, dt.contiguous(), zeta.contiguous())

    def set_field(self, h):
        spring_ising_set_field(self.ctx, None if h is None else h.contiguous())

    def info(self):
        return spring_ising_info(self.ctx)

    def update_best(self):
        spring_ising_update_best(self.ctx)

    def energy_trace(self):
        """In-run checks so far: float64 tensor [checks, R]."""
        import torch
        rows = spring_ising_get_energy_trace(self.ctx, None)
        e = torch.empty(max(rows, 1) * self.r, dtype=torch.float64, device=self.device)
        spring_ising_get_energy_trace(self.ctx, e)
        return e[:rows * self.r].view(rows, self.r)

    def best(self):
        import torch
        e = torch.empty(self.r, dtype=torch.float64, device=self.device)
        s = torch.empty(self.r, self.n, dtype=torch.int8, device=self.device)
        spring_ising_get_best(self.ctx, e, s)
        return e, s

    def hamiltonian(self):
        import torch
        H = torch.empty(self.r, dtype=torch.float64, device=self.device)
        spring_ising_hamiltonian(self.ctx, H)
        return H

    def set_graph(self, min_steps):
        spring_ising_set_graph(self.ctx, min_steps)

    def set_resident(self, min_steps):
        spring_ising_set_resident(self.ctx, min_steps)

    def set_ksplit(self, ksplit):
        spring_ising_set_ksplit(self.ctx, ksplit)

    def autotune(self, steps=20):
        return spring_ising_autotune(self.ctx, steps)

    def relaxed_energy_grad(self, ckpt_every=100):
        """Run the remaining steps; return (loss, dL/ddt, dL/dzeta) as float64
        CUDA tensors (see spring_ising_relaxed_energy_grad)."""
        import torch
        loss = torch.empty(1, dtype=torch.float64, device=self.device)
        g_dt = torch.empty(self.total_steps, dtype=torch.float64, device=self.device)
        g_z = torch.empty_like(g_dt)
        spring_ising_relaxed_energy_grad(self.ctx, ckpt_every, loss, g_dt, g_z)
        return loss, g_dt, g_z

    def relaxed_energy_forward(self, ckpt_every=100):
        """Forward half of relaxed_energy_grad: run the remaining steps with
        checkpoints and return the loss (float64 CUDA tensor [1]); the tape
        stays in the context for relaxed_energy_backward."""
        import torch
        loss = torch.empty(1, dtype=torch.float64, device=self.device)
        spring_ising_relaxed_energy_forward(self.ctx, ckpt_every, loss)
        return loss

    def relaxed_energy_backward(self):
        """Reverse sweep over the tape of the last relaxed_energy_forward:
        (dL/ddt, dL/dzeta) as float64 CUDA tensors.  Raises SpringIsingError
        (SI_ERR_STATE) when the trajectory changed since that forward half, or
        when its tape was already used."""
        import torch
        g_dt = torch.empty(self.total_steps, dtype=torch.float64, device=self.device)
        g_z = torch.empty_like(g_dt)
        spring_ising_relaxed_energy_backward(self.ctx, g_dt, g_z)
        return g_dt, g_z
