#!/usr/bin/env python3
"""Emulated DGEMM throughput (2mnk/t) at a fixed maximum relative error, of
Ozaki scheme II in fast mode with the revised scale-invariant scaling, on
one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--size S] [--N N]
                    [--target 1e-15] [--phi PHI] [--mode revised|original|...]

A step is one ozaki2_dgemm call (norms and exponents, convert and split, N
INT8 GEMMs, CRT and unscale) on a fixed synthetic problem already resident in
HBM.  Default workload: m = n = k = 16384, entries (rand - 0.5) exp(phi randn)
with phi = 0.5 and seed 0 (the distribution of the paper's experiments), N
picked by the library's autotuner for a maximum relative error of 1e-15
(--N forces a count instead).  ``value`` is 2mnk over the median of the K
timed steps (each step between two HIP events on the library's stream).

The same JSON line carries:
  roofline        the dominant kernel (the INT8 GEMM) against the INT8 MFMA
                  peak, its average launch time from HIP events on the
                  library's stream during the timed steps;
  error           max relative and componentwise error of the timed result
                  on a 512-entry block (32 rows x 16 columns by seeded
                  permutation) against a double-double reference, beside
                  native FP64 on the same block;
  paper_protocol  the same step under the paper's timing protocol (warm up
                  at least 3 calls and until 3 s or 100 calls, time at least
                  5 calls and until 12 s or 100 calls, median);
  fixed_N14       the same product with N = 14 (K steps, median, same block);
  cpu_baseline    the CPU oracle on sampled entries of this workload (each
                  entry from scratch; checked bit for bit against the GPU),
                  plus the whole oracle on 256^3, N = 14 against the GPU;
  batched         256 uneven problems (N per problem for the target) in one
                  graph launch against one call per problem, per-stage times
                  of the same kernels launched directly, the INT8 rate of
                  the persistent GEMM and native FP64 on the same problems;
  complex         ZGEMM at 8192^3 beside native complex128 matmul;
  fp8_engine      the FP8 (E4M3) engine variant at 8192^3 beside the INT8
                  engine (bit-identical C, engine rate vs the FP8 peak).
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

INT8_PEAK_TOPS = 5000.0      # MI355X dense INT8 MFMA, 5.0 POP/s
FP8_PEAK_TFLOPS = 5000.0     # MI355X dense FP8 MFMA, 5.0 PFLOP/s
FP8_FLAG = 16                # OZ2_ENGINE_FP8
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k3_gemm_i8_traffic.txt")
K3_SOURCE = os.path.join(ROOT, "paper_2606_29129_amd", "csrc", "oz2_k3_gemm.hpp")
MODES = {"revised": 0, "original": 1, "accurate": 2, "exact": 3}


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cpu():
    """CPU model, logical CPUs and the CPUs this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = os.cpu_count()
    return dict(cpu_model=model, os_cpu_count=os.cpu_count(), cpus_allowed=allowed)


def load_traffic(m, n, k, N):
    """HBM bytes per K3 launch from the committed rocprofv3 counter summary,
    or None if it is missing, for another workload, or for older K3 code."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line:
            key, val = line.split(":", 1)
            kv[key.strip()] = val.strip()
    try:
        from paper_2606_29129_amd.profiling import source_sha
        if kv.get("kernel_code_sha256") != source_sha(K3_SOURCE):
            return None
        if kv.get("workload") != f"m={m} n={n} k={k} N={N}":
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def timed_steps(torch, step, stream, steps, warmup):
    """W untimed steps, then K steps each between two events on `stream`.
    Returns (per-step ms list, total ms of the K steps)."""
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    evs[0].record(stream)
    for s in range(steps):
        step()
        evs[s + 1].record(stream)
    torch.cuda.synchronize()
    per = [evs[s].elapsed_time(evs[s + 1]) for s in range(steps)]
    return per, evs[0].elapsed_time(evs[-1])


def paper_protocol(torch, step, stream):
    """Warm up at least 3 calls and until 3 s or 100 calls; then time at least
    5 calls and until 12 s or 100 calls, each between two events; median."""
    t0, warm = time.time(), 0
    while warm < 3 or (time.time() - t0 < 3.0 and warm < 100):
        step()
        torch.cuda.synchronize()
        warm += 1
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    per, t0 = [], time.time()
    while len(per) < 5 or (time.time() - t0 < 12.0 and len(per) < 100):
        e0.record(stream)
        step()
        e1.record(stream)
        torch.cuda.synchronize()
        per.append(e0.elapsed_time(e1))
    return dict(warmup_calls=warm, timed_calls=len(per), median_ms=round(statistics.median(per), 4),
                min_ms=round(min(per), 4), max_ms=round(max(per), 4))


def error_block(A_rm, B_rm, seed, rows=32, cols=16):
    """Rows and columns of the error block (seeded permutations), the
    double-double reference there and sum |a||b| for the componentwise error."""
    import numpy as np
    from paper_2606_29129_amd import sweep
    m, n = A_rm.shape[0], B_rm.shape[1]
    r = np.sort(np.random.default_rng(seed + 11).permutation(m)[:rows])
    c = np.sort(np.random.default_rng(seed + 12).permutation(n)[:cols])
    Ah = A_rm[r].cpu().numpy()
    Bh = B_rm[:, c].cpu().numpy()
    ref = sweep.dd_block(Ah, Bh)
    absAB = np.abs(Ah) @ np.abs(Bh)
    return r, c, ref, absAB


def block_errors(C_cm, blk):
    """Errors of the column-major C (n x m storage) on the block."""
    from paper_2606_29129_amd import sweep
    r, c, ref, absAB = blk
    Cb = C_cm[c][:, r].t().cpu().numpy()
    e = sweep.errors(Cb, ref, absAB)
    return dict(max_rel_err=e["max_rel"], max_cw_err=e["max_cw"], zero_ref_nonzero=e["zero_ref_nonzero"])


def _oracle_entries(rows_path, cols_path, pairs, N, mode, budget_s):
    """Worker of cpu_baseline (a process of its own): the oracle's entries
    for the (row, column) index pairs in order until the time budget is
    spent.  Returns [(pair index, C_ij)] and the seconds spent computing."""
    import numpy as np
    from oracle import constants, ozaki2 as ref, scaling
    R = np.load(rows_path, mmap_mode="r")
    Q = np.load(cols_path, mmap_mode="r")
    pp = constants.p_prime_prop(N)
    pf, d = constants.p_prime_fast(N), constants.delta()
    out, spent = [], 0.0
    for idx, (r, c) in pairs:
        if spent >= budget_s and out:
            break
        row, col = np.array(R[r]), np.array(Q[c])
        t0 = time.perf_counter()
        Si, Sj = scaling.norm_sq_ru(row), scaling.norm_sq_ru(col)
        if mode == 0:
            ei, fj = scaling.alg2_log2_mu(Si, pp), scaling.alg2_log2_mu(Sj, pp)
        elif mode == 3:
            _, P, _, _ = constants.step1(N)
            ei = scaling.exact_mode_log2_mu(row, P)[0]
            fj = scaling.exact_mode_log2_mu(col, P)[0]
        else:
            ei = scaling.alg1_log2_mu(Si, float(np.max(np.abs(row))), pf, d)
            fj = scaling.alg1_log2_mu(Sj, float(np.max(np.abs(col))), pf, d)
        c_ij, _, _ = ref.entry(row, col, ei, fj, N)
        spent += time.perf_counter() - t0
        out.append((idx, c_ij))
    return out, spent


def cpu_baseline(A_rm, B_rm, C_cm, N, mode, budget_s, seed=0, vectors=48):
    """Time the CPU oracle computing sampled entries of the same product from
    scratch (row and column norms, exponents, residues, N dot products, CRT,
    unscaling) on the host's cores: one process per CPU this process may run
    on (at most 16), each working through its own share of (row, column)
    pairs of `vectors` seeded rows of A and columns of B for `budget_s`
    seconds; every entry is checked bit for bit against the GPU."""
    import multiprocessing as mp
    import tempfile
    import numpy as np
    import torch

    m, k = A_rm.shape
    n = B_rm.shape[1]
    rng = np.random.default_rng(seed)
    ri = rng.choice(m, min(vectors, m), replace=False)
    ci = rng.choice(n, min(vectors, n), replace=False)
    cpu = host_cpu()
    workers = max(1, min(16, cpu["cpus_allowed"] or 1))
    pairs = [(len(ci) * a + b, (a, b)) for a in range(len(ri)) for b in range(len(ci))]
    order = rng.permutation(len(pairs))
    shares = [[pairs[int(x)] for x in order[w::workers]] for w in range(workers)]
    with tempfile.TemporaryDirectory() as tmp:
        rows_path, cols_path = os.path.join(tmp, "rows.npy"), os.path.join(tmp, "cols.npy")
        rix = torch.as_tensor(ri, dtype=torch.long, device=A_rm.device)
        cix = torch.as_tensor(ci, dtype=torch.long, device=B_rm.device)
        np.save(rows_path, A_rm[rix].cpu().numpy())
        np.save(cols_path, B_rm[:, cix].t().contiguous().cpu().numpy())
        # fresh interpreters (spawn): the workers import numpy and the oracle only
        ctx = mp.get_context("spawn")
        t0 = time.perf_counter()
        pool = ctx.Pool(workers)
        try:
            res = pool.starmap_async(_oracle_entries, [
                (rows_path, cols_path, sh, N, mode, budget_s) for sh in shares
            ]).get(timeout=4 * budget_s + 120)
        finally:
            pool.terminate()
            pool.join()
        wall = time.perf_counter() - t0
    done = exact_ok = 0
    busy = 0.0
    for out, spent in res:
        busy += spent
        for idx, c in out:
            a, b = divmod(idx, len(ci))
            g = float(C_cm[int(ci[b]), int(ri[a])])
            exact_ok += int(np.float64(g).view(np.uint64) == np.float64(c).view(np.uint64))
            done += 1
    per_worker = busy / workers
    return dict(value=2.0 * k * done / per_worker / 1e12, unit="TFLOPS", cores=workers,
                kind="oracle",
                sample=f"{done} entries C_ij of this workload, pairs of {len(ri)} seeded rows of A "
                       f"and {len(ci)} seeded columns of B, each computed from scratch from its "
                       f"full row and column (k={k}, N={N}) by {workers} worker processes: 2k "
                       f"flops credited per entry, over the mean compute seconds per worker",
                seconds=round(per_worker, 2), wall_seconds=round(wall, 2),
                threads=f"{workers} processes x 1 thread (pure Python integers)",
                **cpu), done, exact_ok


def accurate_sample_check(A_rm, B_rm, C_cm, N, samples=8, seed=0):
    """Accurate mode on sampled entries: the oracle's bar matrices in array
    form over all of A and B, the needed rows and columns of their product
    (binary64, exact: integers below 2^53), the oracle's final exponent step
    and entry."""
    import numpy as np
    from oracle import constants, ozaki2 as ref, scaling
    Ah = A_rm.cpu().numpy()
    Bh = B_rm.cpu().numpy()
    k = Ah.shape[1]
    if 4096.0 * k >= 2.0 ** 53:
        raise ValueError("bar products would not be exact in binary64")
    e1A, nzA, barA = scaling.accurate_bars(Ah)
    e1B, nzB, barBt = scaling.accurate_bars(Bh.T)
    Af = barA.astype(np.float64)
    Bf = np.ascontiguousarray(barBt.T.astype(np.float64))
    del barA, barBt
    pa, d = constants.p_prime_accu(N), constants.delta()
    rng = np.random.default_rng(seed + 5)
    ok = 0
    t0 = time.perf_counter()
    for _ in range(samples):
        i, j = int(rng.integers(Ah.shape[0])), int(rng.integers(Bh.shape[1]))
        ei = scaling.accurate_final_exponent(int(e1A[i]) if nzA[i] else None,
                                             int((Af[i] @ Bf).max()), pa, d)
        fj = scaling.accurate_final_exponent(int(e1B[j]) if nzB[j] else None,
                                             int((Af @ Bf[:, j]).max()), pa, d)
        c, _, _ = ref.entry(Ah[i], Bh[:, j], ei, fj, N)
        ok += int(np.float64(float(C_cm[j, i])).view(np.uint64) == np.float64(c).view(np.uint64))
    return dict(entries=samples, bit_exact=ok, seconds=round(time.perf_counter() - t0, 2),
                how="bar matrices of all of A and B, the sampled rows and columns of their "
                    "product, then each entry from scratch")


def full_oracle_config1(torch, oz, seed=0, N=14, phi=0.5, size=256):
    """The whole oracle on the small configuration (m = n = k = 256, N = 14)
    against the GPU's result of the same problem, bit for bit."""
    import numpy as np
    from oracle import ozaki2 as ref
    from paper_2606_29129_amd import inputs
    A, B = inputs.problem(size, size, size, phi, seed=seed)
    dev = torch.device("cuda:0")
    C = oz.dgemm(torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev), N=N)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    want = ref.dgemm(A, B, N, ref.REVISED)
    secs = time.perf_counter() - t0
    got = C.cpu().numpy()
    same = int(np.sum(got.view(np.uint64) == want.view(np.uint64)))
    return dict(workload=f"m=n=k={size}, (rand-0.5)*exp({phi}*randn) seed {seed}, N={N}",
                seconds=round(secs, 3), tflops=2.0 * size ** 3 / secs / 1e12,
                threads="1 (Python integers, numpy int64 products)",
                entries_bit_exact=same, entries=size * size)


def batched_leg(steps, warmup, target=1e-15, count=256, seed=0, check=4):
    """256 independent DGEMMs, m, n, k log-uniform in [64, 2048], phi uniform
    in [0.5, 3], N per problem from the library's autotuner for the target max
    relative error (one call with N = 0; the timed calls replay the graph with
    the N it chose, and calls that re-run the autotuner every time are timed
    separately); one graph launch per batch versus one ozaki2_dgemm call per
    problem; per-stage times of the same kernels launched directly; native
    FP64 torch.matmul on the same problems."""
    import numpy as np
    import torch
    from paper_2606_29129_amd import autotune, inputs
    from paper_2606_29129_amd import ozaki2 as oz

    dev = torch.device("cuda:0")
    rng = np.random.default_rng(seed)
    shapes = np.exp(rng.uniform(np.log(64), np.log(2048), (count, 3))).round().astype(int)
    phis = rng.uniform(0.5, 3.0, count)
    pairs, flops = [], 0.0
    for i in range(count):
        m, n, k = (int(x) for x in shapes[i])
        A = inputs.ozaki_matrix_torch(m, k, float(phis[i]), seed + i, 0, dev)
        B = inputs.ozaki_matrix_torch(k, n, float(phis[i]), seed + i, 1, dev)
        pairs.append((A, B))
        flops += 2.0 * m * n * k
    stream = torch.cuda.current_stream()
    _, Ns = oz.dgemm_batched(pairs, 0, target=target, return_N=True)
    torch.cuda.synchronize()
    py_Ns = [autotune.pick_N(A.shape[1], max(autotune.estimate_phi(A, "rows"),
                                             autotune.estimate_phi(B, "cols")), target)
             for A, B in pairs]
    # fixed outputs: every replay writes the same matrices (no pointer refresh)
    outs = [torch.empty((A.shape[0], B.shape[1]), dtype=torch.float64, device=dev)
            for A, B in pairs]
    probs = [(B.shape[1], A.shape[0], A.shape[1], B, max(1, B.shape[1]), A, max(1, A.shape[1]),
              C, max(1, B.shape[1]), N) for (A, B), C, N in zip(pairs, outs, Ns)]
    ws = oz.ozaki2_dgemm_batched_workspace_size(probs)
    oz.ensure_workspace(ws)
    oz.ozaki2_set_stream(stream.cuda_stream)

    def run_batched():
        rc, bad, _ = oz.ozaki2_dgemm_batched(probs, 0)
        if rc:
            raise oz.Ozaki2Error(f"ozaki2_dgemm_batched (problem {bad})", rc)

    def run_autotuned():
        return oz.dgemm_batched(pairs, 0, target=target)

    def run_plain():
        return [oz.dgemm(A, B, N=N) for (A, B), N in zip(pairs, Ns)]

    def run_native():
        return [torch.matmul(A, B) for A, B in pairs]

    per_b, tot_b = timed_steps(torch, run_batched, stream, steps, warmup)
    ms_b = statistics.median(per_b)
    # the same kernels launched directly, with stage events
    oz._check("ozaki2_set_timing", oz.ozaki2_set_timing(1))
    for _ in range(steps):
        run_batched()
    stage_ms, calls = oz.ozaki2_get_stage_times()
    oz.ozaki2_set_timing(0)
    st = {name: round(v / max(calls, 1), 4) for name, v in zip(oz.STAGE_NAMES, stage_ms)}
    gemm_ms = stage_ms[2] / max(calls, 1)
    int8_ops = sum(2.0 * N * A.shape[0] * B.shape[1] * A.shape[1] for (A, B), N in zip(pairs, Ns))
    padded_ops = sum(2.0 * N * ((A.shape[0] + 127) // 128 * 128) * ((B.shape[1] + 127) // 128 * 128)
                     * ((A.shape[1] + 127) // 128 * 128) for (A, B), N in zip(pairs, Ns))
    ms_auto = statistics.median(timed_steps(torch, run_autotuned, stream, steps, warmup)[0])
    ms_p = statistics.median(timed_steps(torch, run_plain, stream, steps, warmup)[0])
    ms_n = statistics.median(timed_steps(torch, run_native, stream, steps, warmup)[0])
    outs_p = run_plain()
    torch.cuda.synchronize()
    same = all(torch.equal(a.view(torch.int64), b.view(torch.int64)) for a, b in zip(outs, outs_p))
    max_rel = 0.0
    crng = np.random.default_rng(seed + 1)
    for i in crng.choice(count, check, replace=False):
        A, B = pairs[i]
        C = outs[i]
        for _ in range(16):
            r = int(crng.integers(A.shape[0]))
            c = int(crng.integers(B.shape[1]))
            ref = autotune.exact_dot(A[r].cpu().numpy(), B[:, c].cpu().numpy())
            max_rel = max(max_rel, autotune.rel_err(float(C[r, c]), ref))
    hist = {str(N): Ns.count(N) for N in sorted(set(Ns))}
    return dict(problems=count, target_max_rel_err=target, total_flops=flops,
                ms_batched=round(ms_b, 4), tflops_batched=round(flops / ms_b / 1e9, 2),
                ms_plain=round(ms_p, 4), tflops_plain=round(flops / ms_p / 1e9, 2),
                speedup=round(ms_p / ms_b, 2), bit_identical_to_plain=bool(same),
                native_fp64_ms=round(ms_n, 4), native_fp64_tflops=round(flops / ms_n / 1e9, 2),
                stage_ms_direct_launch=st,
                int8_ops=int8_ops, int8_ops_padded=padded_ops,
                int8_gemm_top_s=round(int8_ops / (gemm_ms * 1e-3) / 1e12, 1),
                int8_gemm_frac=round(int8_ops / (gemm_ms * 1e-3) / 1e12 / INT8_PEAK_TOPS, 4),
                int8_gemm_frac_padded=round(padded_ops / (gemm_ms * 1e-3) / 1e12 / INT8_PEAK_TOPS, 4),
                workspace_bytes=ws, N_histogram=hist, max_rel_err_sampled=max_rel,
                N_source="library autotuner (ozaki2_dgemm_batched with N = 0 and the target)",
                N_agrees_with_python_autotuner=int(sum(a == b for a, b in zip(Ns, py_Ns))),
                ms_batched_autotune_every_call=round(ms_auto, 4),
                timing="median of K graph replays between events; stage times from K direct "
                       "launches of the same kernels",
                sampled="16 entries of each of %d problems vs the exact product" % check)


def complex_leg(size, N, phi, seed, steps, warmup, samples=8):
    """ZGEMM m = n = k = size on complex128 inputs whose real and imaginary
    parts follow the same distribution: 8mnk/t, per-stage times, the INT8
    rate of its 3N GEMMs, native complex128 torch.matmul of the same GPU, and
    the normwise error |c - r| / |r| of sampled entries against their exact
    values."""
    import math
    from fractions import Fraction
    import numpy as np
    import torch
    from paper_2606_29129_amd import autotune, inputs
    from paper_2606_29129_amd import ozaki2 as oz

    dev = torch.device("cuda:0")
    A = inputs.complex_matrix_torch(size, size, phi, seed, 0, dev)
    B = inputs.complex_matrix_torch(size, size, phi, seed, 1, dev)
    A_cm, B_cm = A.t().contiguous(), B.t().contiguous()
    C_cm = torch.empty((size, size), dtype=torch.complex128, device=dev)
    stream = torch.cuda.current_stream()
    oz.ensure_workspace(oz.ozaki2_zgemm_workspace_size(size, size, size, N, 0))

    def step():
        rc = oz.ozaki2_zgemm(size, size, size, A_cm, size, B_cm, size, C_cm, size, N, 0)
        if rc:
            raise oz.Ozaki2Error("ozaki2_zgemm", rc)

    oz._check("ozaki2_set_timing", oz.ozaki2_set_timing(1))
    per, _ = timed_steps(torch, step, stream, steps, warmup)
    stage_ms, calls = oz.ozaki2_get_stage_times()
    oz.ozaki2_set_timing(0)
    ms = statistics.median(per)
    st = {name: round(v / max(calls, 1), 4) for name, v in zip(oz.STAGE_NAMES, stage_ms)}
    k3_ms = stage_ms[2] / max(calls, 1)
    k3_ops = 6.0 * N * size ** 3
    flops = 8.0 * size ** 3
    Cn = torch.empty_like(C_cm)
    nat = statistics.median(timed_steps(torch, lambda: torch.matmul(A, B, out=Cn), stream, 3, 1)[0])
    native = flops / (nat * 1e-3) / 1e12
    del Cn

    def frac(v):
        n, e = v
        return Fraction(n) * Fraction(2) ** e

    rng = np.random.default_rng(seed + 7)
    worst = 0.0
    for _ in range(samples):
        i, j = int(rng.integers(size)), int(rng.integers(size))
        a, b = A[i].cpu().numpy(), B[:, j].cpu().numpy()
        Rr = frac(autotune.exact_dot(np.concatenate([a.real, -a.imag]),
                                     np.concatenate([b.real, b.imag])))
        Ri = frac(autotune.exact_dot(np.concatenate([a.real, a.imag]),
                                     np.concatenate([b.imag, b.real])))
        c = complex(C_cm[j, i].item())
        dr, di = Fraction(c.real) - Rr, Fraction(c.imag) - Ri
        den = Rr * Rr + Ri * Ri
        if den:
            worst = max(worst, math.sqrt(float((dr * dr + di * di) / den)))
    del A, B, A_cm, B_cm, C_cm
    torch.cuda.empty_cache()
    return dict(workload=f"square ZGEMM m=n=k={size}, real and imaginary parts "
                         f"(rand-0.5)*exp({phi}*randn) seed {seed}, revised scaling, N={N}",
                N=N, ms_per_step=round(ms, 4), tflops=round(flops / (ms * 1e-3) / 1e12, 2),
                flops_per_step="8mnk", stage_ms_per_step=st,
                int8_gemm_top_s=round(k3_ops / (k3_ms * 1e-3) / 1e12, 1),
                int8_gemm_frac=round(k3_ops / (k3_ms * 1e-3) / 1e12 / INT8_PEAK_TOPS, 4),
                native_zgemm_tflops=round(native, 2), sampled_entries=samples,
                max_rel_err_sampled=worst)


def fp8_leg(size, N, phi, seed, steps, warmup):
    """The FP8 (E4M3) engine variant (mode | OZ2_ENGINE_FP8) at m = n = k =
    size beside the INT8 engine on the same operands: ms per call, 2mnk/t,
    the engine rate of the residue products (four E4M3 products of 2mnk
    flops per modulus) against the FP8 MFMA peak, and whether C is
    bit-identical to the INT8 engine's."""
    import torch
    from paper_2606_29129_amd import inputs
    from paper_2606_29129_amd import ozaki2 as oz

    dev = torch.device("cuda:0")
    A = inputs.ozaki_matrix_torch(size, size, phi, seed, 0, dev)
    B = inputs.ozaki_matrix_torch(size, size, phi, seed, 1, dev)
    A_cm, B_cm = A.t().contiguous(), B.t().contiguous()
    del A, B
    stream = torch.cuda.current_stream()
    oz.ensure_workspace(oz.ozaki2_workspace_size(size, size, size, N, FP8_FLAG))
    out = {}
    Cs = {}
    for name, mode in (("int8", 0), ("fp8", FP8_FLAG)):
        C = torch.empty((size, size), dtype=torch.float64, device=dev)

        def step():
            rc = oz.ozaki2_dgemm(size, size, size, A_cm, size, B_cm, size, C, size, N, mode)
            if rc:
                raise oz.Ozaki2Error("ozaki2_dgemm", rc)

        oz._check("ozaki2_set_timing", oz.ozaki2_set_timing(1))
        per, _ = timed_steps(torch, step, stream, steps, warmup)
        stage_ms, calls = oz.ozaki2_get_stage_times()
        oz.ozaki2_set_timing(0)
        ms = statistics.median(per)
        k3 = stage_ms[2] / max(calls, 1)
        engine_ops = (4.0 if mode else 1.0) * 2.0 * N * size ** 3
        rate = engine_ops / (k3 * 1e-3) / 1e12
        out[name] = dict(ms_per_call=round(ms, 4), tflops=round(2.0 * size ** 3 / (ms * 1e-3) / 1e12, 2),
                         stage_ms={n: round(v / max(calls, 1), 4) for n, v in zip(oz.STAGE_NAMES, stage_ms)},
                         products_rate=round(rate, 1),
                         products_unit="TFLOP/s (E4M3)" if mode else "TOP/s (INT8)",
                         products_frac=round(rate / (FP8_PEAK_TFLOPS if mode else INT8_PEAK_TOPS), 4))
        Cs[name] = C
    torch.cuda.synchronize()
    same = torch.equal(Cs["int8"].view(torch.int64), Cs["fp8"].view(torch.int64))
    del Cs, A_cm, B_cm
    torch.cuda.empty_cache()
    return dict(workload=f"square DGEMM m=n=k={size}, (rand-0.5)*exp({phi}*randn) seed {seed}, "
                         f"revised scaling, N={N}", N=N, bit_identical_to_int8=bool(same), **out)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=16384, help="m = n = k")
    ap.add_argument("--m", type=int)
    ap.add_argument("--n", type=int)
    ap.add_argument("--k", type=int)
    ap.add_argument("--N", type=int, default=0,
                    help="moduli; 0 (default) lets the autotuner pick N for --target")
    ap.add_argument("--target", type=float, default=1e-15,
                    help="max relative error target (headline N and the batched leg)")
    ap.add_argument("--phi", type=float, default=0.5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--mode", default="revised", choices=list(MODES))
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-native", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-protocol", action="store_true", help="skip the paper-protocol leg")
    ap.add_argument("--no-n14", action="store_true", help="skip the N = 14 leg")
    ap.add_argument("--no-error", action="store_true", help="skip the 512-entry error block")
    ap.add_argument("--no-complex", action="store_true", help="skip the ZGEMM leg")
    ap.add_argument("--complex-size", type=int, default=8192)
    ap.add_argument("--no-fp8", action="store_true", help="skip the FP8 engine leg")
    ap.add_argument("--fp8-size", type=int, default=8192)
    ap.add_argument("--traffic-calibration", type=int, default=0, metavar="BYTES",
                    help="before the steps, run one torch.abs over a float64 tensor of "
                         "BYTES bytes (the known-size kernel that scales rocprofv3 "
                         "FETCH_SIZE/WRITE_SIZE)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: the benchmark runs on one GPU only (the emulated DGEMM is a "
              "single-GPU kernel pipeline); --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2606_29129_amd import inputs
    from paper_2606_29129_amd import ozaki2 as oz

    m = args.m or args.size
    n = args.n or args.size
    k = args.k or args.size
    mode = MODES[args.mode]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    oz.ozaki2_set_stream(stream.cuda_stream)

    t0 = time.time()
    A_rm = inputs.ozaki_matrix_torch(m, k, args.phi, args.seed, 0, dev)
    B_rm = inputs.ozaki_matrix_torch(k, n, args.phi, args.seed, 1, dev)
    A_cm = A_rm.t().contiguous()          # column-major A, lda = m
    B_cm = B_rm.t().contiguous()          # column-major B, ldb = k
    C_cm = torch.empty((n, m), dtype=torch.float64, device=dev)   # ldc = m

    # N for the error target: the library's autotuner on phi estimated from
    # the operands (the larger of the two estimates)
    oz.ensure_workspace(1024)
    phi_hat = max(oz.ozaki2_estimate_phi(m, k, A_cm, m, 0),    # the rows of A
                  oz.ozaki2_estimate_phi(k, n, B_cm, k, 1))    # the columns of B
    N_tuned = oz.ozaki2_autotune_N(k, phi_hat, args.target)
    N = args.N or N_tuned
    Ns_used = {N} | (set() if args.no_n14 else {14})
    ws_bytes = max(oz.ozaki2_workspace_size(m, n, k, Nx, mode) for Nx in Ns_used)
    oz.ensure_workspace(ws_bytes)
    torch.cuda.synchronize()
    _log(f"inputs {m}x{k} and {k}x{n} generated in {time.time() - t0:.1f}s; phi estimate "
         f"{phi_hat:.3f} -> N={N_tuned} for {args.target:g} (using N={N}); workspace "
         f"{ws_bytes / 2**30:.2f} GiB")

    if args.traffic_calibration:
        src = torch.ones(args.traffic_calibration // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.abs(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    def make_step(Nx, out):
        def step():
            rc = oz.ozaki2_dgemm(m, n, k, A_cm, m, B_cm, k, out, m, Nx, mode)
            if rc:
                raise oz.Ozaki2Error("ozaki2_dgemm", rc)
        return step

    step = make_step(N, C_cm)
    oz._check("ozaki2_set_timing", oz.ozaki2_set_timing(1))
    per, total_ms = timed_steps(torch, step, stream, args.steps, args.warmup)
    stage_ms, calls = oz.ozaki2_get_stage_times()     # warmup and timed calls
    oz.ozaki2_set_timing(0)
    ms_median = statistics.median(per)
    ms_mean = total_ms / args.steps
    flops = 2.0 * m * n * k
    value = flops / (ms_median * 1e-3) / 1e12
    _log(f"timed {args.steps} steps at N={N}: median {ms_median:.3f} ms (mean {ms_mean:.3f}) "
         f"-> {value:.1f} TFLOPS emulated")

    st = {name: round(v / max(calls, 1), 4) for name, v in zip(oz.STAGE_NAMES, stage_ms)}
    k3_ms = stage_ms[2] / max(calls, 1)
    k3_ops = 2.0 * m * n * k * N
    achieved = k3_ops / (k3_ms * 1e-3) / 1e12
    roofline = dict(kernel="k3_gemm_i8 (N INT8 GEMMs, one launch)", bound="mfma",
                    achieved=round(achieved, 1), peak=INT8_PEAK_TOPS, unit="TOP/s",
                    frac=round(achieved / INT8_PEAK_TOPS, 4), traffic=load_traffic(m, n, k, N),
                    avg_launch_ms=round(k3_ms, 4), ops_per_launch=k3_ops,
                    launches_averaged=calls)
    _log(f"stages ms/call: {st}; K3 {achieved:.0f} TOP/s = "
         f"{100 * achieved / INT8_PEAK_TOPS:.1f}% of INT8 peak")

    blk = None
    error = None
    if not args.no_error:
        t1 = time.time()
        blk = error_block(A_rm, B_rm, args.seed)
        error = dict(block="32 rows x 16 columns by seeded permutation (512 entries)",
                     reference="double-double dot products over the full k", N=N,
                     **block_errors(C_cm, blk), seconds=round(time.time() - t1, 1))
        _log(f"error on the 512-entry block: max rel {error['max_rel_err']:.3e}, "
             f"max cw {error['max_cw_err']:.3e}")

    protocol = None
    if not args.no_protocol:
        protocol = paper_protocol(torch, step, stream)
        protocol["tflops"] = round(flops / (protocol["median_ms"] * 1e-3) / 1e12, 2)
        _log(f"paper protocol: {protocol}")

    sample_check = None
    cpu = None
    if mode == 2:
        if not args.no_cpu_baseline:
            sample_check = accurate_sample_check(A_rm, B_rm, C_cm, N, seed=args.seed)
            _log(f"accurate-mode sampled entries bit-exact: {sample_check['bit_exact']}/"
                 f"{sample_check['entries']}")
    elif not args.no_cpu_baseline:
        cpu, done, ok = cpu_baseline(A_rm, B_rm, C_cm, N, mode, args.cpu_seconds, args.seed)
        sample_check = dict(entries=done, bit_exact=ok)
        _log(f"cpu oracle: {cpu['value']:.3e} TFLOPS on {done} entries; GPU entries "
             f"bit-exact: {ok}/{done}")
        cpu["full_problem"] = full_oracle_config1(torch, oz, seed=args.seed)
        _log(f"whole oracle at 256^3: {cpu['full_problem']}")
        oz.ensure_workspace(ws_bytes)

    n14 = None
    if not args.no_n14 and N != 14:
        C14 = torch.empty_like(C_cm)
        per14, _ = timed_steps(torch, make_step(14, C14), stream, args.steps, args.warmup)
        ms14 = statistics.median(per14)
        n14 = dict(N=14, ms_median=round(ms14, 4), tflops=round(flops / (ms14 * 1e-3) / 1e12, 2))
        if blk is not None:
            n14.update(block_errors(C14, blk))
        del C14
        _log(f"N=14: {n14}")

    native = None
    native_err = None
    if not args.no_native:
        Cn = torch.empty((m, n), dtype=torch.float64, device=dev)
        pn = timed_steps(torch, lambda: torch.matmul(A_rm, B_rm, out=Cn), stream, 3, 1)[0]
        native = flops / (statistics.median(pn) * 1e-3) / 1e12
        if blk is not None:
            native_err = block_errors(Cn.t(), blk)
        del Cn
        _log(f"native FP64 torch.matmul: {native:.1f} TFLOPS; block errors {native_err}")

    batched = None
    if not args.no_batched:
        batched = batched_leg(args.steps, args.warmup, target=args.target)
        _log(f"batched: {batched['tflops_batched']} TFLOPS in one graph launch vs "
             f"{batched['tflops_plain']} plain, {batched['native_fp64_tflops']} native; "
             f"GEMM {batched['int8_gemm_top_s']} TOP/s; stages {batched['stage_ms_direct_launch']}")

    cplx = None
    if not args.no_complex:
        cplx = complex_leg(args.complex_size, 14, args.phi, args.seed, args.steps, args.warmup)
        _log(f"zgemm {args.complex_size}^3 N=14: {cplx['tflops']} TFLOPS (8mnk/t) vs native "
             f"{cplx['native_zgemm_tflops']}; INT8 GEMMs at {cplx['int8_gemm_top_s']} TOP/s")

    fp8 = None
    if not args.no_fp8:
        fp8 = fp8_leg(args.fp8_size, 14, args.phi, args.seed, max(3, args.steps // 2), 2)
        _log(f"fp8 engine {args.fp8_size}^3 N=14: {fp8['fp8']['tflops']} TFLOPS vs int8 "
             f"{fp8['int8']['tflops']}; products {fp8['fp8']['products_rate']} TFLOP/s; "
             f"bit-identical {fp8['bit_identical_to_int8']}")

    shape = f"m=n=k={m}" if m == n == k else f"m={m} n={n} k={k}"
    how_N = (f"N={N} from the autotuner for max rel. error {args.target:g}" if not args.N
             else f"N={N} (fixed)")
    out = {
        "metric": "Emulated DGEMM TFLOPS (2mnk/t) at fixed max rel. error; batched vs plain",
        "value": round(value, 2),
        "unit": "TFLOPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_median, 4),
        "ms_mean": round(ms_mean, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8",
        "io_dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"square DGEMM {shape}, entries (rand-0.5)*exp({args.phi}*randn) seed "
                        f"{args.seed}, Ozaki-II {args.mode} scaling, {how_N}, plain call",
            "m": m, "n": n, "k": k, "phi": args.phi, "phi_estimated": round(phi_hat, 4),
            "N": N, "N_autotuned": N_tuned, "target_max_rel_err": args.target,
            "mode": args.mode, "seed": args.seed, "parallelism": "single GPU",
        },
        "timing": "value = 2mnk / median of the K timed steps (HIP events on the library stream)",
        "roofline": roofline,
        "cpu_baseline": cpu,
        "stage_ms_per_step": st,
        "error": error,
        "native_fp64_tflops": None if native is None else round(native, 2),
        "native_fp64_error": native_err,
        "paper_protocol": protocol,
        "sample_check": sample_check,
        "fixed_N14": n14,
        "batched": batched,
        "complex": cplx,
        "fp8_engine": fp8,
        "context": {"paper_gh200_cublas_dgemm_tflops": 60.9,
                    "paper_gh200_ozaki2_dgemm_tflops_up_to": 80.2},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
