"""Seeded synthetic inputs with the distribution of the paper's experiments.

Section 3.2 draws every entry as (rand - 0.5) * exp(phi * randn), with rand
uniform on [0, 1) and randn standard normal; phi sets the spread of the entry
magnitudes.  This module reproduces that distribution with a counter-based
stream so that any entry can be regenerated from (seed, stream, index):

    x_i   = mix64(key + (i + 1) * 0x9E3779B97F4A7C15)
    key   = mix64(seed XOR mix64(stream))
    rand  = (x_i >> 11) * 2**-53

``mix64`` is the finaliser of Vigna's public-domain SplitMix64 generator.
randn uses the Box-Muller transform on two further streams.  Matrix A uses
streams 0, 1, 2 and matrix B streams 3, 4, 5 (rand, Box-Muller u1, u2); the
imaginary parts of complex A and B use streams 6-8 and 9-11; the entry (r, c)
of an R x C matrix has index r * C + c.

``ozaki_matrix_torch`` evaluates the same streams with torch integer ops on
any device (integer arithmetic wraps modulo 2**64 exactly as in numpy, so the
uniforms are bit-identical; the log/cos/exp of the Box-Muller and exp(phi z)
steps use the device's math library and may differ from numpy's in the last
bit).  Whichever generator produced a matrix, the oracle is given that same
matrix.

This module holds no part of the emulation method; both the HIP path and the
CPU oracle consume the arrays it returns.
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix64(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _key(seed: int, stream: int) -> np.uint64:
    s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
    return _mix64(s ^ _mix64(np.uint64(stream)))


def uniform(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    """rand in [0, 1) for indices start .. start+count-1 of a stream."""
    key = _key(seed, stream)
    idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        x = _mix64(key + idx * _GAMMA)
    return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def ozaki_matrix(rows: int, cols: int, phi: float, seed: int = 0, which: int = 0,
                 chunk: int = 1 << 22) -> np.ndarray:
    """rows x cols binary64 matrix, entries (rand - 0.5) * exp(phi * randn).

    ``which`` = 0 for A and 1 for B selects the streams.  Row-major.
    """
    total = rows * cols
    out = np.empty(total, dtype=np.float64)
    base = 3 * which
    for s in range(0, total, chunk):
        c = min(chunk, total - s)
        r = uniform(seed, base + 0, s, c)
        u1 = uniform(seed, base + 1, s, c)
        u2 = uniform(seed, base + 2, s, c)
        z = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)
        out[s:s + c] = (r - 0.5) * np.exp(phi * z)
    return out.reshape(rows, cols)


def problem(m: int, n: int, k: int, phi: float, seed: int = 0):
    """(A, B) for C = A B with A m x k and B k x n (row-major binary64)."""
    return ozaki_matrix(m, k, phi, seed, 0), ozaki_matrix(k, n, phi, seed, 1)


def complex_problem(m: int, n: int, k: int, phi: float, seed: int = 0):
    """(A, B) complex128 for C = A B: real and imaginary parts drawn
    independently from the distribution above (A: streams 0-2 real, 6-8
    imaginary; B: streams 3-5 real, 9-11 imaginary)."""
    A = ozaki_matrix(m, k, phi, seed, 0) + 1j * ozaki_matrix(m, k, phi, seed, 2)
    B = ozaki_matrix(k, n, phi, seed, 1) + 1j * ozaki_matrix(k, n, phi, seed, 3)
    return A, B


def ones_problem(m: int, n: int, k: int, s: int):
    """A = 2**s J (m x k) and B = 2**s J (k x n), the all-ones case of
    Section 3.1."""
    a = np.full((m, k), 2.0 ** s)
    b = np.full((k, n), 2.0 ** s)
    return a, b


# --- the same streams with torch (any device) -------------------------------

def _i64(u: int) -> int:
    """An unsigned 64-bit constant as the int64 with the same bits."""
    return u - (1 << 64) if u >= (1 << 63) else u


def _t_shr(z, s: int):
    """Logical right shift of int64 bit patterns."""
    return (z >> s) & ((1 << (64 - s)) - 1)


def _t_mix64(z):
    z = (z ^ _t_shr(z, 30)) * _i64(0xBF58476D1CE4E5B9)
    z = (z ^ _t_shr(z, 27)) * _i64(0x94D049BB133111EB)
    return z ^ _t_shr(z, 31)


def uniform_torch(seed: int, stream: int, start: int, count: int, device):
    import torch
    key = int(_key(seed, stream))
    idx = torch.arange(start + 1, start + count + 1, dtype=torch.int64, device=device)
    x = _t_mix64(_i64(key) + idx * _i64(int(_GAMMA)))
    return _t_shr(x, 11).to(torch.float64) * (2.0 ** -53)


def ozaki_matrix_torch(rows: int, cols: int, phi: float, seed: int = 0, which: int = 0,
                       device="cuda", chunk: int = 1 << 24):
    """Same distribution and streams as ``ozaki_matrix``, as a row-major
    float64 torch tensor on ``device``."""
    import torch
    total = rows * cols
    out = torch.empty(total, dtype=torch.float64, device=device)
    base = 3 * which
    for s in range(0, total, chunk):
        c = min(chunk, total - s)
        r = uniform_torch(seed, base + 0, s, c, device)
        u1 = uniform_torch(seed, base + 1, s, c, device)
        u2 = uniform_torch(seed, base + 2, s, c, device)
        z = torch.sqrt(-2.0 * torch.log1p(-u1)) * torch.cos(2.0 * torch.pi * u2)
        out[s:s + c] = (r - 0.5) * torch.exp(phi * z)
    return out.view(rows, cols)


def complex_matrix_torch(rows: int, cols: int, phi: float, seed: int = 0, which: int = 0,
                         device="cuda"):
    """Complex counterpart of ``ozaki_matrix_torch`` (``complex_problem``'s
    streams: which = 0 for A, 1 for B) as a row-major complex128 tensor."""
    import torch
    re = ozaki_matrix_torch(rows, cols, phi, seed, which, device)
    im = ozaki_matrix_torch(rows, cols, phi, seed, which + 2, device)
    return torch.complex(re, im)
