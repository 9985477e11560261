"""Autotuner: the number of moduli N per accuracy target, and the GEMM tile.

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
  1 + phi^2 (``estimate_phi``: pooled within the rows of A and the columns of B).

The exact reference is computed here with Python integers (every binary64
value is an integer times a power of two).

Tiles: the library chooses among three GEMM tiles (256x256, 128x128,
256x64; ``ozaki2_set_tile``) with a cost model of padded work and workgroup
rounds whose constants (a relative rate and a fixed per-round cost in k
slabs for each tile) come from ``measure_tiles`` (times of ``ozaki2_dgemm``
with each tile forced, over a grid of shapes and N, stored in
``autotune_tiles.json``) and ``fit_tile_model`` (the constants that minimise
the summed slowdown of the model's pick against the best measured tile).
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "autotune_table.json")
TILE_TABLE = os.path.join(HERE, "autotune_tiles.json")
TILES = {1: (256, 256), 2: (128, 128), 3: (256, 64)}     # OZ2_TILE_* -> (rows, cols)
TILE_SHAPES = ((1024, 1024, 1024), (2048, 2048, 2048), (4096, 4096, 4096), (8192, 8192, 8192),
               (8192, 8192, 1024), (4096, 4096, 512), (2048, 2048, 8192), (65536, 64, 4096),
               (32768, 128, 4096), (16384, 256, 2048), (512, 512, 4096), (3000, 3000, 3000),
               (16384, 16384, 16384))

K_GRID = (64, 256, 1024, 2048, 8192, 16384)
PHI_GRID = (0.5, 1.0, 1.5, 2.0, 2.5, 3.0, 4.0)
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


def estimate_phi(X, vectors: str = "rows") -> float:
    """phi of (rand-0.5) exp(phi randn) from a matrix (numpy array or torch
    tensor, the logical rows x cols matrix): sqrt(max(var - 1, 0)) with var
    the variance of log|x| within the vectors the scaling treats -- its rows
    (``vectors="rows"``, as for A) or its columns (``"cols"``, as for B) --
    pooled over the vectors, on the sample ozaki2_estimate_phi uses (every
    vector with its first max(2, 2^20 / (number of vectors)) entries); zeros
    and non-finite entries skipped, vectors with fewer than two entries left
    out (0 when none has two).  Rows or columns scaled by different powers
    of two leave it unchanged, as they leave the revised scaling's bits."""
    if vectors not in ("rows", "cols"):
        raise ValueError(vectors)
    rows, cols = X.shape
    nvec, full = (rows, cols) if vectors == "rows" else (cols, rows)
    L = min(full, max(2, (1 << 20) // max(nvec, 1)))
    S = X[:, :L] if vectors == "rows" else X[:L, :]
    try:
        import torch
        if isinstance(S, torch.Tensor):
            S = S.detach().cpu().numpy()
    except ImportError:
        pass
    S = np.asarray(S, np.float64)
    if vectors == "cols":
        S = S.T
    ok = (S != 0) & np.isfinite(S)
    lg = np.where(ok, np.log(np.where(ok, np.abs(S), 1.0)), 0.0)
    n = ok.sum(axis=1)
    mean = lg.sum(axis=1) / np.maximum(n, 1)
    dev = np.where(ok, lg - mean[:, None], 0.0)
    use = n >= 2
    D = float((n[use] - 1).sum())
    if D <= 0:
        return 0.0
    var = float((dev[use] ** 2).sum()) / D
    return math.sqrt(max(var - 1.0, 0.0))


_table_cache = None


def load_table(path: str = TABLE):
    global _table_cache
    if _table_cache is None:
        with open(path) as f:
            _table_cache = json.load(f)
    return _table_cache


def _envelope(t, ks, phis, kg, pg, N):
    """Largest tabulated error at or below grid point (kg, pg), for N or any
    larger N."""
    e = 0.0
    for k2 in ks:
        if k2 > kg:
            break
        for p2 in phis:
            if p2 > pg:
                break
            row = t["errors"][str(k2)][str(p2)]
            e = max([e] + [row[str(Nx)] for Nx in (int(x) for x in row.keys()) if Nx >= N])
    return e


def error_estimate(k: int, phi: float, N: int, table=None):
    """Upper envelope of the calibrated maxima for (k, phi, N): at each grid
    point the largest tabulated error at or below it, for N or any larger N;
    between grid points the envelope's log interpolated bilinearly in
    (log2 k, phi) (end points below the grid); beyond the largest calibrated
    k scaled by sqrt(k / k_max); None beyond the largest calibrated phi."""
    t = table or load_table()
    ks = sorted(int(x) for x in t["errors"].keys())
    phis = sorted(float(x) for x in t["errors"][str(ks[0])].keys())
    if phi > phis[-1] + 1e-12:
        return None
    kc = max(k, ks[0])
    i1 = next((i for i, x in enumerate(ks) if x >= kc), len(ks) - 1)
    i0 = max(i1 - 1, 0)
    wk = 0.0
    if i1 > i0:
        wk = math.log2(kc / ks[i0]) / math.log2(ks[i1] / ks[i0]) if kc < ks[i1] else 1.0
    pc = max(phi, phis[0])
    j1 = next((j for j, x in enumerate(phis) if x >= pc - 1e-12), len(phis) - 1)
    j0 = max(j1 - 1, 0)
    wp = min((pc - phis[j0]) / (phis[j1] - phis[j0]), 1.0) if j1 > j0 else 0.0
    if wk in (0.0, 1.0) and wp in (0.0, 1.0):        # on a grid point
        e = _envelope(t, ks, phis, ks[i0 if wk == 0.0 else i1], phis[j0 if wp == 0.0 else j1], N)
    else:
        L = {(a, b): math.log2(_envelope(t, ks, phis, ks[a], phis[b], N))
             for a in (i0, i1) for b in (j0, j1)}
        e = 2.0 ** ((1 - wk) * ((1 - wp) * L[i0, j0] + wp * L[i0, j1])
                    + wk * ((1 - wp) * L[i1, j0] + wp * L[i1, j1]))
    if k > ks[-1]:
        e *= math.sqrt(k / ks[-1])
    return e


def pick_N(k: int, phi: float, target: float, table=None, margin: float = 4.0) -> int:
    """Smallest N whose error estimate (``error_estimate``) is at most
    target / margin; 20 if none is or phi lies beyond the calibration."""
    t = table or load_table()
    ks = sorted(int(x) for x in t["errors"].keys())
    phis = sorted(float(x) for x in t["errors"][str(ks[0])].keys())
    Ns = sorted(int(x) for x in t["errors"][str(ks[0])][str(phis[0])].keys())
    for N in Ns:
        e = error_estimate(k, phi, N, t)
        if e is None:
            break
        if e * margin <= target:
            return N
    return 20


HEADER = os.path.join(HERE, "csrc", "oz2_autotune_table.hpp")


def header_text(table=None) -> str:
    """The calibrated table as a C++ header for the library's own N choice
    (``ozaki2_autotune_N``, and N = 0 in ``ozaki2_dgemm_batched``): the k and
    phi grid points, the N range and the max relative errors, each printed
    with repr (the shortest string that reads back to the same binary64)."""
    t = table or load_table()
    ks = sorted(int(x) for x in t["errors"].keys())
    phis = sorted(float(x) for x in t["errors"][str(ks[0])].keys())
    Ns = sorted(int(x) for x in t["errors"][str(ks[0])][str(phis[0])].keys())
    assert Ns == list(range(Ns[0], Ns[-1] + 1))
    lines = [
        "// oz2_autotune_table.hpp -- generated by paper_2606_29129_amd/autotune.py",
        "// (header_text) from autotune_table.json: the maximum relative error of",
        "// ozaki2_dgemm measured against exact products of sampled entries, per",
        "// grid point (k, phi) of the input distribution (rand - 0.5) exp(phi randn)",
        f"// and number of moduli N (m = {t.get('m')}, {t.get('block')}x{t.get('block')} sampled"
        f" blocks, seed {t.get('seed')}).",
        "#pragma once",
        "",
        "namespace oz2 {",
        "",
        f"constexpr int kTuneNK = {len(ks)}, kTuneNPhi = {len(phis)}, kTuneN0 = {Ns[0]}, "
        f"kTuneNN = {len(Ns)};",
        "constexpr long long kTuneK[kTuneNK] = {" + ", ".join(str(k) for k in ks) + "};",
        "constexpr double kTunePhi[kTuneNPhi] = {" + ", ".join(repr(p) for p in phis) + "};",
        "constexpr double kTuneErr[kTuneNK][kTuneNPhi][kTuneNN] = {",
    ]
    for k in ks:
        lines.append("  {")
        for p in phis:
            row = t["errors"][str(k)][str(p)]
            lines.append("    {" + ", ".join(repr(float(row[str(N)])) for N in Ns) + "},")
        lines.append("  },")
    lines += ["};", "", "}  // namespace oz2", ""]
    return "\n".join(lines)


def write_header(path: str = HEADER, table=None) -> bool:
    """Write the header if its content changed; True if written."""
    text = header_text(table)
    if os.path.exists(path) and open(path).read() == text:
        return False
    with open(path, "w") as f:
        f.write(text)
    return True


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


def measure_tiles(shapes=TILE_SHAPES, Ns=(14, 20), phi=1.0, path: str = TILE_TABLE, log=print):
    """Time ozaki2_dgemm with each tile forced (median-free mean of a few
    calls after two warmups) and store the table.  Needs a GPU."""
    import torch
    from . import inputs
    from . import ozaki2 as oz

    dev = torch.device("cuda:0")
    rows = []
    for (m, n, k) in shapes:
        A = inputs.ozaki_matrix_torch(m, k, phi, 0, 0, dev)
        B = inputs.ozaki_matrix_torch(k, n, phi, 0, 1, dev)
        Acm, Bcm = A.t().contiguous(), B.t().contiguous()
        C = torch.empty((n, m), dtype=torch.float64, device=dev)
        oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
        oz.ensure_workspace(oz.ozaki2_workspace_size(m, n, k, max(Ns), 0))
        rec = dict(m=m, n=n, k=k, ms={})
        for N in Ns:
            for tile in TILES:
                oz._check("ozaki2_set_tile", oz.ozaki2_set_tile(tile))
                f = lambda: oz._check("ozaki2_dgemm", oz.ozaki2_dgemm(
                    m, n, k, Acm, m, Bcm, k, C, m, N, 0))
                f()
                f()
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                reps = 5 if m * n * k < 2 ** 36 else 2
                e0.record()
                for _ in range(reps):
                    f()
                e1.record()
                torch.cuda.synchronize()
                rec["ms"][f"{N}/{tile}"] = round(e0.elapsed_time(e1) / reps, 4)
        oz.ozaki2_set_tile(0)
        rows.append(rec)
        log(json.dumps(rec))
        del A, B, Acm, Bcm, C
        torch.cuda.empty_cache()
    table = dict(phi=phi, Ns=list(Ns), tiles={str(t): list(v) for t, v in TILES.items()},
                 shapes=rows)
    with open(path, "w") as f:
        json.dump(table, f, indent=1)
    return table


def tile_model_time(m, n, k, N, tile, rate, fixed, per_cu=(0, 1, 2, 2)):
    """The library's cost model (relative units) for one tile."""
    bm, bn = TILES[tile]
    tiles = math.ceil(m / bm) * math.ceil(n / bn) * N
    rounds = math.ceil(tiles / (256 * per_cu[tile]))
    return rounds * bm * bn * per_cu[tile] * (math.ceil(k / 128) + fixed[tile]) / rate[tile]


def tile_regret(table, rate, fixed):
    """(summed, worst) relative slowdown of the model's pick vs the best
    measured tile over the table."""
    total = worst = 0.0
    for rec in table["shapes"]:
        for N in table["Ns"]:
            ms = {t: rec["ms"][f"{N}/{t}"] for t in TILES}
            pick = min(TILES, key=lambda t: tile_model_time(rec["m"], rec["n"], rec["k"], N, t,
                                                            rate, fixed))
            r = ms[pick] / min(ms.values()) - 1.0
            total += r
            worst = max(worst, r)
    return total, worst


def fit_tile_model(table=None, path: str = TILE_TABLE):
    """Grid search of the rates of the two smaller tiles and the fixed
    per-round costs; among the fits within 0.3% of the least summed slowdown,
    the one whose rates are closest to the large-problem rates measured in
    the table (16384^3) is returned as (rate, fixed, summed, worst)."""
    if table is None:
        with open(path) as f:
            table = json.load(f)
    big = [r for r in table["shapes"] if r["m"] == r["n"] == r["k"] == 16384]
    ref = {2: 0.8, 3: 0.45}
    if big:
        N = table["Ns"][0]
        for t in (2, 3):
            ref[t] = big[0]["ms"][f"{N}/1"] / big[0]["ms"][f"{N}/{t}"]
    fits = []
    for r2 in [x / 100 for x in range(45, 90, 5)]:
        for r3 in [x / 100 for x in range(25, 70, 5)]:
            for f1 in (0, 2, 4, 6, 8, 12, 16):
                for f2 in (0, 1, 2, 4):
                    for f3 in (0, 1, 2, 4):
                        rate = {1: 1.0, 2: r2, 3: r3}
                        fixed = {1: f1, 2: f2, 3: f3}
                        tot, worst = tile_regret(table, rate, fixed)
                        fits.append((tot, worst, rate, fixed))
    best = min(f[0] for f in fits)
    near = [f for f in fits if f[0] <= best + 0.003]
    near.sort(key=lambda f: abs(f[2][2] - ref[2]) + abs(f[2][3] - ref[3]) + 0.001 * f[3][1])
    tot, worst, rate, fixed = near[0]
    return rate, fixed, tot, worst


if __name__ == "__main__":
    import sys
    if len(sys.argv) > 1 and sys.argv[1] == "tiles":
        measure_tiles(log=lambda s: print(s, flush=True))
        print(fit_tile_model())
    else:
        calibrate(log=lambda s: print(s, flush=True))
