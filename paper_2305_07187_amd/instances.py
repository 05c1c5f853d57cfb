"""Seeded synthetic inputs for the Spring-Ising hot path.

This module only draws random numbers; it holds none of the method's
arithmetic.  Both the GPU path and the FP64 oracle consume what it returns,
so neither depends on the other for its inputs.

Generator: splitmix64 (S. Vigna's published 64-bit mixer).  The k-th output
(k = 0, 1, ...) of a stream seeded with ``seed`` is ``mix(seed + (k+1)*G)``
mod 2**64 with G = 0x9E3779B97F4A7C15, which lets a whole stream be drawn as
one vectorised NumPy expression.

Instances follow the paper's benchmark shape (Discussion: K2000 is a complete
undirected graph on 2000 vertices).  The K2000 file itself is not available,
so a complete graph with iid +-1 couplings of the same size stands in for it.
Gaussian N(0,1) couplings give the real-valued instances of the batched and
precision workloads.

Layouts (all NumPy, C order):
  J   float32 [N, N], symmetric, zero diagonal.
  x0  float32 [R, N]: replica-major, so replica r's spins are contiguous and
      drawing more replicas never changes earlier ones.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
# Stream salts: J, x0 and the batch recipe draw from unrelated streams.
_SALT_J = 0x4A5F_1D0C_0000_0001
_SALT_X0 = 0x58_30_5F_30_0000_0002
_SALT_BATCH = 0x42_41_54_43_48_000003
_SALT_GAUSS = 0x47_41_55_53_53_000004


def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Outputs ``start .. start+count-1`` of a splitmix64 stream (uint64)."""
    k = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, count: int) -> np.ndarray:
    """float64 in [0, 1): top 53 bits of each draw times 2**-53."""
    return (splitmix64(seed, count) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def _mirror_upper(n: int, upper: np.ndarray, dtype) -> np.ndarray:
    J = np.zeros((n, n), dtype=dtype)
    iu = np.triu_indices(n, 1)  # row-major order of the strict upper triangle
    J[iu] = upper
    J.T[iu] = upper
    return J


def make_pm1(n: int, seed: int = 0) -> np.ndarray:
    """Complete graph, J_ij = +-1 iid for i<j (bit 63 of each draw), mirrored."""
    m = n * (n - 1) // 2
    bits = splitmix64(seed ^ _SALT_J, m) >> np.uint64(63)
    upper = np.where(bits == 1, 1.0, -1.0).astype(np.float32)
    return _mirror_upper(n, upper, np.float32)


def make_gauss(n: int, seed: int = 0) -> np.ndarray:
    """Complete graph, J_ij ~ N(0,1) iid for i<j (Box-Muller, cosine branch)."""
    m = n * (n - 1) // 2
    raw = splitmix64(seed ^ _SALT_GAUSS, 2 * m) >> np.uint64(11)
    u1 = (raw[0::2].astype(np.float64) + 1.0) * 2.0 ** -53  # (0, 1]
    u2 = raw[1::2].astype(np.float64) * 2.0 ** -53
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return _mirror_upper(n, z.astype(np.float32), np.float32)


def make_x0(n: int, r: int, seed: int = 0, scale: float = 0.1) -> np.ndarray:
    """Initial positions near the origin: x0 ~ U(-scale, scale) iid, [R, N]."""
    u = uniform01(seed ^ _SALT_X0, n * r)
    return (-scale + 2.0 * scale * u).astype(np.float32).reshape(r, n)


def make_batch(n_inst: int, seed: int = 0, n_min: int = 64, n_max: int = 4096):
    """Uneven-N batch recipe: N_i uniform in [n_min, n_max]; even i -> +-1,
    odd i -> Gaussian.  Returns a list of (N_i, kind, J_seed)."""
    draws = splitmix64(seed ^ _SALT_BATCH, n_inst)
    span = n_max - n_min + 1
    out = []
    for i in range(n_inst):
        n_i = n_min + int(draws[i] % np.uint64(span))
        kind = "pm1" if i % 2 == 0 else "gauss"
        j_seed = (seed * 1_000_003 + i) & 0xFFFFFFFF
        out.append((n_i, kind, j_seed))
    return out


def make_J(n: int, kind: str, seed: int) -> np.ndarray:
    if kind == "pm1":
        return make_pm1(n, seed)
    if kind == "gauss":
        return make_gauss(n, seed)
    raise ValueError(f"unknown instance kind {kind!r}")


def random_state(n: int, r: int, seed: int, scale: float = 1.5) -> np.ndarray:
    """Arbitrary positions in [-scale, scale) for readout/energy tests, with
    exact zeros, negative zeros and wall values planted at fixed spots."""
    u = uniform01(seed ^ 0x5EED_0005, n * r)
    x = (-scale + 2.0 * scale * u).astype(np.float32).reshape(r, n)
    if n >= 4:
        x[:, 0] = 0.0
        x[:, 1] = -0.0
        x[:, 2] = np.float32(np.sqrt(2.0))
        x[:, 3] = -np.float32(np.sqrt(2.0))
    return x


# ---------------------------------------------------------------------------
# The same streams drawn with torch int64 arithmetic (two's-complement
# wrap-around equals arithmetic mod 2**64; logical shifts are emulated by
# masking), so large instances can be generated directly in device memory.
# Bit-identical to the NumPy functions above.
# ---------------------------------------------------------------------------
def _s64(v: int) -> int:
    v &= 0xFFFFFFFFFFFFFFFF
    return v - (1 << 64) if v >= (1 << 63) else v


def _lsr(z, s: int):
    import torch
    return (z >> s) & torch.tensor((1 << (64 - s)) - 1, dtype=torch.int64, device=z.device)


def splitmix64_torch(seed: int, count: int, device, start: int = 0):
    import torch
    k = torch.arange(start + 1, start + count + 1, dtype=torch.int64, device=device)
    z = k * _s64(0x9E3779B97F4A7C15) + _s64(seed)
    z = (z ^ _lsr(z, 30)) * _s64(0xBF58476D1CE4E5B9)
    z = (z ^ _lsr(z, 27)) * _s64(0x94D049BB133111EB)
    return z ^ _lsr(z, 31)


def _mirror_upper_torch(n, upper, device):
    import torch
    J = torch.zeros((n, n), dtype=torch.float32, device=device)
    iu = torch.triu_indices(n, n, 1, device=device)
    J[iu[0], iu[1]] = upper
    J[iu[1], iu[0]] = upper
    return J


def make_pm1_torch(n: int, seed: int = 0, device="cpu"):
    import torch
    m = n * (n - 1) // 2
    z = splitmix64_torch(seed ^ _SALT_J, m, device)
    upper = torch.where(z < 0, 1.0, -1.0).to(torch.float32)  # bit 63 set <=> negative
    return _mirror_upper_torch(n, upper, device)


def make_gauss_torch(n: int, seed: int = 0, device="cpu"):
    import math

    import torch
    m = n * (n - 1) // 2
    raw = _lsr(splitmix64_torch(seed ^ _SALT_GAUSS, 2 * m, device), 11)
    u1 = (raw[0::2].to(torch.float64) + 1.0) * 2.0 ** -53
    u2 = raw[1::2].to(torch.float64) * 2.0 ** -53
    z = torch.sqrt(-2.0 * torch.log(u1)) * torch.cos(2.0 * math.pi * u2)
    return _mirror_upper_torch(n, z.to(torch.float32), device)


def make_x0_torch(n: int, r: int, seed: int = 0, scale: float = 0.1, device="cpu"):
    import torch
    raw = _lsr(splitmix64_torch(seed ^ _SALT_X0, n * r, device), 11)
    u = raw.to(torch.float64) * 2.0 ** -53
    return (-scale + 2.0 * scale * u).to(torch.float32).reshape(r, n)


def make_J_torch(n: int, kind: str, seed: int, device="cpu"):
    if kind == "pm1":
        return make_pm1_torch(n, seed, device)
    if kind == "gauss":
        return make_gauss_torch(n, seed, device)
    raise ValueError(f"unknown instance kind {kind!r}")
