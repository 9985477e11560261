"""Autotuner: the number of moduli N per accuracy target.

The error of the emulated product is set by how many bits of each entry the
scaled integers keep (Section 2.2: more moduli, larger P, wider integers) and
by the spread of the entry magnitudes, which for the distribution of the
paper's experiments, (rand - 0.5) exp(phi randn), is controlled by phi
(Section 3.2).  The autotuner therefore

* calibrates, on the GPU, the maximum relative error of ``ozaki2_dgemm``
  against the exact product of sampled entries for a grid of (k, phi, N)
  (``calibrate``, stored in ``autotune_table.json``), and
* picks, for a problem, the smallest N whose calibrated error at the next
  larger grid point in k and phi is below the target (``pick_N``), with phi
  estimated from the data: for this distribution log|a| has variance
  1 + phi^2 (``estimate_phi``).

The exact reference is computed here with Python integers (every binary64
value is an integer times a power of two).
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "autotune_table.json")

K_GRID = (64, 256, 1024, 2048)
PHI_GRID = (0.5, 1.0, 1.5, 2.0, 2.5, 3.0)
N_GRID = tuple(range(10, 21))


def exact_dot(a, b):
    """sum_h a_h b_h exactly, as (integer, exponent) with value int * 2**exp."""
    terms = []
    for x, y in zip(np.asarray(a, np.float64).tolist(), np.asarray(b, np.float64).tolist()):
        if x == 0.0 or y == 0.0:
            continue
        nx, dx = x.as_integer_ratio()
        ny, dy = y.as_integer_ratio()
        terms.append((nx * ny, -((dx * dy).bit_length() - 1)))
    if not terms:
        return 0, 0
    emin = min(e for _, e in terms)
    return sum(n << (e - emin) for n, e in terms), emin


def rel_err(c: float, ref) -> float:
    n, e = ref
    if n == 0:
        return 0.0 if c == 0.0 else math.inf
    cn, cd = float(c).as_integer_ratio()
    ce = -(cd.bit_length() - 1)
    lo = min(e, ce)
    diff = (cn << (ce - lo)) - (n << (e - lo))
    return abs(diff) / abs(n << (e - lo))


def estimate_phi(A) -> float:
    """phi of (rand-0.5) exp(phi randn) from a tensor or array of samples."""
    try:
        import torch
        if isinstance(A, torch.Tensor):
            x = A.reshape(-1)[: 1 << 20]
            x = x[x != 0].abs().log()
            v = float(x.var()) if x.numel() > 1 else 1.0
            return math.sqrt(max(v - 1.0, 0.0))
    except ImportError:
        pass
    x = np.asarray(A, np.float64).ravel()[: 1 << 20]
    x = np.log(np.abs(x[x != 0]))
    v = float(x.var()) if x.size > 1 else 1.0
    return math.sqrt(max(v - 1.0, 0.0))


_table_cache = None


def load_table(path: str = TABLE):
    global _table_cache
    if _table_cache is None:
        with open(path) as f:
            _table_cache = json.load(f)
    return _table_cache


def pick_N(k: int, phi: float, target: float, table=None, margin: float = 4.0) -> int:
    """Smallest N whose calibrated max relative error (at the next grid point
    at or above k and phi) is below target / margin; 20 if none is."""
    t = table or load_table()
    ks = sorted(int(x) for x in t["errors"].keys())
    kk = next((x for x in ks if x >= k), ks[-1])
    phis = sorted(float(x) for x in t["errors"][str(kk)].keys())
    pp = next((x for x in phis if x >= phi - 1e-12), phis[-1])
    row = t["errors"][str(kk)][str(pp)]
    for N in sorted(int(x) for x in row.keys()):
        if row[str(N)] * margin <= target:
            return N
    return 20


def calibrate(m: int = 256, block: int = 32, seed: int = 7, path: str = TABLE, log=print):
    """Measure max relative errors on the GPU for the (k, phi, N) grid and
    write the table.  Needs a GPU."""
    import torch
    from . import inputs
    from . import ozaki2 as oz

    dev = torch.device("cuda:0")
    rng = np.random.default_rng(seed)
    table = {"m": m, "block": block, "seed": seed, "errors": {}}
    for k in K_GRID:
        table["errors"][str(k)] = {}
        for phi in PHI_GRID:
            A = inputs.ozaki_matrix_torch(m, k, phi, seed, 0, dev)
            B = inputs.ozaki_matrix_torch(k, m, phi, seed, 1, dev)
            rows = rng.choice(m, block, replace=False)
            cols = rng.choice(m, block, replace=False)
            Ah = A[rows].cpu().numpy()
            Bh = B[:, cols].cpu().numpy()
            refs = [[exact_dot(Ah[i], Bh[:, j]) for j in range(block)] for i in range(block)]
            errs = {}
            for N in N_GRID:
                C = oz.dgemm(A, B, N=N)[rows][:, cols].cpu().numpy()
                errs[str(N)] = max(rel_err(C[i, j], refs[i][j])
                                   for i in range(block) for j in range(block))
            table["errors"][str(k)][str(phi)] = errs
            log(f"k={k} phi={phi}: " + " ".join(f"N{N}={errs[str(N)]:.1e}" for N in N_GRID))
    with open(path, "w") as f:
        json.dump(table, f, indent=1)
    return table


if __name__ == "__main__":
    calibrate(log=lambda s: print(s, flush=True))
