#!/usr/bin/env python3
"""Emulated DGEMM throughput (2mnk/t) of Ozaki scheme II, fast mode with the
revised scale-invariant scaling, on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--size S] [--N N]
                    [--phi PHI] [--mode revised|original]

A step is one ozaki2_dgemm call (norms and exponents, convert and split, N
INT8 GEMMs, CRT and unscale) on a fixed synthetic problem already resident in
HBM.  Default workload: m = n = k = 16384, entries (rand - 0.5) exp(phi randn)
with phi = 0.5 and seed 0 (the distribution of the paper's experiments), N =
14 moduli.  Prints one JSON line with the throughput, the roofline position of
the dominant kernel (the INT8 GEMM, timed with HIP events on the library's
stream during the timed steps), the CPU oracle timed on a bounded sample of
the same problem, and the native FP64 DGEMM of the same GPU for context.
Two more legs fill fields of the same line: ``fixed_error`` times the same
product with N picked by the autotuner for a max relative error target
(default 1e-15, measured on sampled entries against exact values), and
``batched`` times 256 uneven problems (N per problem for the same target) in
one graph launch against one call per problem; ``complex`` times ZGEMM at
8192^3 (three INT8 GEMMs per modulus) beside native complex128 matmul.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

INT8_PEAK_TOPS = 5000.0      # MI355X dense INT8 MFMA, 5.0 POP/s
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k3_gemm_i8_traffic.txt")
K3_SOURCE = os.path.join(ROOT, "paper_2606_29129_amd", "csrc", "oz2_k3_gemm.hpp")


def _log(*a):
    print(*a, file=sys.stderr, flush=True)




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


def cpu_baseline(A_rm, B_rm, C_cm, N, mode, budget_s, seed=0):
    """Time the CPU oracle computing sampled entries of the same product from
    scratch (row and column norms, exponents, residues, N dot products, CRT,
    unscaling), and check the GPU's entries against it bit for bit."""
    import numpy as np
    from oracle import constants, ozaki2 as ref, reference, scaling

    m, k = A_rm.shape
    n = B_rm.shape[1]
    rng = np.random.default_rng(seed)
    pp = constants.p_prime_prop(N)
    pf, d = constants.p_prime_fast(N), constants.delta()
    done = exact_ok = 0
    elapsed = 0.0
    max_rel = 0.0
    while elapsed < budget_s or done < 2:
        i, j = int(rng.integers(m)), int(rng.integers(n))
        row = A_rm[i].double().cpu().numpy()
        col = B_rm[:, j].double().cpu().numpy()
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
        c, _, _ = ref.entry(row, col, ei, fj, N)
        elapsed += time.perf_counter() - t0
        g = float(C_cm[j, i])
        exact_ok += int(np.float64(g).view(np.uint64) == np.float64(c).view(np.uint64))
        R = reference.exact_dot(row, col)
        if R != 0:
            max_rel = max(max_rel, float(abs((type(R)(g) - R) / R)))
        done += 1
    return dict(value=2.0 * k * done / elapsed / 1e12, unit="TFLOPS", cores=1,
                kind="oracle",
                sample=f"{done} entries C_ij at seeded random (i, j), each computed from "
                       f"its full row of A and column of B (k={k}), single Python thread",
                seconds=round(elapsed, 2)), done, exact_ok, max_rel


def fixed_error_leg(A_rm, B_rm, A_cm, B_cm, m, n, k, mode, target, stream, seed,
                    steps=3, samples=16):
    """The same product with N picked by the autotuner for the max relative
    error target (phi estimated from the data); its error is measured on
    sampled entries against their exact values."""
    import numpy as np
    import torch
    from paper_2606_29129_amd import autotune
    from paper_2606_29129_amd import ozaki2 as oz

    phi_hat = max(autotune.estimate_phi(A_rm), autotune.estimate_phi(B_rm))
    Nt = autotune.pick_N(k, phi_hat, target)
    C_cm = torch.empty((n, m), dtype=torch.float64, device=A_cm.device)  # its own output

    def step():
        rc = oz.ozaki2_dgemm(m, n, k, A_cm, m, B_cm, k, C_cm, m, Nt, mode)
        if rc:
            raise oz.Ozaki2Error("ozaki2_dgemm", rc)

    step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    rng = np.random.default_rng(seed + 99)
    worst = 0.0
    for _ in range(samples):
        i, j = int(rng.integers(m)), int(rng.integers(n))
        ref = autotune.exact_dot(A_rm[i].cpu().numpy(), B_rm[:, j].cpu().numpy())
        worst = max(worst, autotune.rel_err(float(C_cm[j, i]), ref))
    del C_cm
    torch.cuda.empty_cache()
    return dict(target_max_rel_err=target, phi_estimated=round(phi_hat, 3), N=Nt,
                ms_per_step=round(ms, 4), tflops=round(2.0 * m * n * k / (ms * 1e-3) / 1e12, 2),
                sampled_entries=samples, max_rel_err_sampled=worst,
                note="N from the autotuner's calibrated table for the target")


def batched_leg(steps, warmup, target=1e-15, count=256, seed=0, check=4):
    """256 independent DGEMMs, m, n, k log-uniform in [64, 2048], phi uniform
    in [0.5, 3], N per problem from the library's autotuner for the target max
    relative error (one call with N = 0; the timed calls replay the graph with
    the N it chose, and calls that re-run the autotuner every time are timed
    separately); one graph launch per batch versus one ozaki2_dgemm call per
    problem."""
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
    # N per problem from the library's autotuner (N = 0 with the target),
    # compared with the Python autotuner's pick for the same data
    _, Ns = oz.dgemm_batched(pairs, 0, target=target, return_N=True)
    torch.cuda.synchronize()
    py_Ns = [autotune.pick_N(A.shape[1], max(autotune.estimate_phi(A), autotune.estimate_phi(B)),
                             target) for A, B in pairs]

    def run_batched():
        return oz.dgemm_batched(pairs, Ns)

    def run_autotuned():
        return oz.dgemm_batched(pairs, 0, target=target)

    def run_plain():
        return [oz.dgemm(A, B, N=N) for (A, B), N in zip(pairs, Ns)]

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            out = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps, out

    ms_b, outs = timed(run_batched)
    ms_auto, _ = timed(run_autotuned)
    ms_p, outs_p = timed(run_plain)
    same = all(torch.equal(a.view(torch.int64), b.view(torch.int64)) for a, b in zip(outs, outs_p))
    # accuracy on sampled entries of a few problems, against the exact product
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
                N_histogram=hist, max_rel_err_sampled=max_rel,
                N_source="library autotuner (ozaki2_dgemm_batched with N = 0 and the target)",
                N_agrees_with_python_autotuner=int(sum(a == b for a, b in zip(Ns, py_Ns))),
                ms_batched_autotune_every_call=round(ms_auto, 4),
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

    def step():
        rc = oz.ozaki2_zgemm(size, size, size, A_cm, size, B_cm, size, C_cm, size, N, 0)
        if rc:
            raise oz.Ozaki2Error("ozaki2_zgemm", rc)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    oz._check("ozaki2_set_timing", oz.ozaki2_set_timing(1))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    stage_ms, calls = oz.ozaki2_get_stage_times()
    oz.ozaki2_set_timing(0)
    ms = e0.elapsed_time(e1) / steps
    st = {name: round(v / max(calls, 1), 4) for name, v in zip(oz.STAGE_NAMES, stage_ms)}
    k3_ms = stage_ms[2] / max(calls, 1)
    k3_ops = 6.0 * N * size ** 3
    flops = 8.0 * size ** 3

    Cn = torch.matmul(A, B)
    torch.cuda.synchronize()
    reps = 2
    e0.record(stream)
    for _ in range(reps):
        torch.matmul(A, B, out=Cn)
    e1.record(stream)
    torch.cuda.synchronize()
    native = flops / (e0.elapsed_time(e1) / reps * 1e-3) / 1e12
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


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=16384, help="m = n = k")
    ap.add_argument("--m", type=int)
    ap.add_argument("--n", type=int)
    ap.add_argument("--k", type=int)
    ap.add_argument("--N", type=int, default=14)
    ap.add_argument("--phi", type=float, default=0.5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--mode", default="revised",
                    choices=["revised", "original", "accurate", "exact"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-native", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-fixed-error", action="store_true",
                    help="skip the leg with N picked by the autotuner for --target")
    ap.add_argument("--no-complex", action="store_true", help="skip the ZGEMM leg")
    ap.add_argument("--complex-size", type=int, default=8192)
    ap.add_argument("--target", type=float, default=1e-15,
                    help="max relative error target of the fixed-error and batched legs")
    ap.add_argument("--traffic-calibration", type=int, default=0, metavar="BYTES",
                    help="before the steps, run one torch.abs over a float64 tensor of "
                         "BYTES bytes (the known-size kernel that scales rocprofv3 "
                         "FETCH_SIZE/WRITE_SIZE)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the emulated DGEMM is a "
              "single-GPU kernel pipeline); --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2606_29129_amd import inputs
    from paper_2606_29129_amd import ozaki2 as oz

    m = args.m or args.size
    n = args.n or args.size
    k = args.k or args.size
    N, mode = args.N, {"revised": 0, "original": 1, "accurate": 2, "exact": 3}[args.mode]
    if mode == 2 and not args.no_cpu_baseline:
        # the oracle's accurate-mode exponents need the whole bar product
        _log("accurate mode: no sampled CPU oracle leg")
        args.no_cpu_baseline = True
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    t0 = time.time()
    A_rm = inputs.ozaki_matrix_torch(m, k, args.phi, args.seed, 0, dev)
    B_rm = inputs.ozaki_matrix_torch(k, n, args.phi, args.seed, 1, dev)
    A_cm = A_rm.t().contiguous()          # column-major A, lda = m
    B_cm = B_rm.t().contiguous()          # column-major B, ldb = k
    C_cm = torch.empty((n, m), dtype=torch.float64, device=dev)   # ldc = m
    ws_bytes = oz.ozaki2_workspace_size(m, n, k, N, mode)
    ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=dev)
    ws_ptr = (ws.data_ptr() + 255) // 256 * 256
    oz._check("ozaki2_set_workspace", oz.ozaki2_set_workspace(ws_ptr, ws_bytes))
    stream = torch.cuda.current_stream()
    oz.ozaki2_set_stream(stream.cuda_stream)
    torch.cuda.synchronize()
    _log(f"inputs {m}x{k} and {k}x{n} generated in {time.time() - t0:.1f}s; "
         f"workspace {ws_bytes / 2**30:.2f} GiB")

    if args.traffic_calibration:
        src = torch.ones(args.traffic_calibration // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.abs(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    def step():
        rc = oz.ozaki2_dgemm(m, n, k, A_cm, m, B_cm, k, C_cm, m, N, mode)
        if rc:
            raise oz.Ozaki2Error("ozaki2_dgemm", rc)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    _log(f"warmup done ({args.warmup} steps)")

    oz._check("ozaki2_set_timing", oz.ozaki2_set_timing(1))
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    evs[0].record(stream)
    for s in range(args.steps):
        step()
        evs[s + 1].record(stream)
    torch.cuda.synchronize()
    stage_ms, calls = oz.ozaki2_get_stage_times()
    oz.ozaki2_set_timing(0)
    total_ms = evs[0].elapsed_time(evs[-1])
    per_step = sorted(evs[s].elapsed_time(evs[s + 1]) for s in range(args.steps))
    ms_per_step = total_ms / args.steps
    ms_median = per_step[len(per_step) // 2]
    flops = 2.0 * m * n * k
    value = flops / (ms_per_step * 1e-3) / 1e12
    _log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step "
         f"(median {ms_median:.3f}) -> {value:.1f} TFLOPS emulated")

    st = {name: round(v / max(calls, 1), 4) for name, v in zip(oz.STAGE_NAMES, stage_ms)}
    k3_ms = stage_ms[2] / max(calls, 1)
    k3_ops = 2.0 * m * n * k * N
    achieved = k3_ops / (k3_ms * 1e-3) / 1e12
    traffic = load_traffic(m, n, k, N)
    roofline = dict(kernel="k3_gemm_i8 (N INT8 GEMMs, one launch)", bound="mfma",
                    achieved=round(achieved, 1), peak=INT8_PEAK_TOPS, unit="TOP/s",
                    frac=round(achieved / INT8_PEAK_TOPS, 4), traffic=traffic,
                    avg_launch_ms=round(k3_ms, 4), ops_per_launch=k3_ops)
    _log(f"stages ms/call: {st}; K3 {achieved:.0f} TOP/s = "
         f"{100 * achieved / INT8_PEAK_TOPS:.1f}% of INT8 peak")

    fixed = None
    if not args.no_fixed_error and mode != 2:
        fixed = fixed_error_leg(A_rm, B_rm, A_cm, B_cm, m, n, k, mode, args.target,
                                stream, args.seed)
        _log(f"fixed error {args.target:g}: N={fixed['N']} -> {fixed['tflops']} TFLOPS, "
             f"max rel err on {fixed['sampled_entries']} entries {fixed['max_rel_err_sampled']:.2e}")

    native = None
    if not args.no_native:
        Cn = torch.matmul(A_rm, B_rm)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 3
        e0.record(stream)
        for _ in range(reps):
            torch.matmul(A_rm, B_rm, out=Cn)
        e1.record(stream)
        torch.cuda.synchronize()
        native = flops / (e0.elapsed_time(e1) / reps * 1e-3) / 1e12
        del Cn
        _log(f"native FP64 torch.matmul: {native:.1f} TFLOPS")

    cpu = None
    sample_check = None
    if not args.no_cpu_baseline:
        cpu, done, ok, max_rel = cpu_baseline(A_rm, B_rm, C_cm, N, mode, args.cpu_seconds,
                                              args.seed)
        sample_check = dict(entries=done, bit_exact=ok, max_rel_err_vs_exact=max_rel)
        _log(f"cpu oracle: {cpu['value']:.3e} TFLOPS on {done} entries; "
             f"GPU entries bit-exact: {ok}/{done}; max rel err vs exact {max_rel:.3e}")

    batched = None
    if not args.no_batched:
        batched = batched_leg(args.steps, args.warmup, target=args.target)
        _log(f"batched: {batched['tflops_batched']} TFLOPS in one graph launch vs "
             f"{batched['tflops_plain']} TFLOPS plain ({batched['speedup']}x), "
             f"N {batched['N_histogram']}, max rel err {batched['max_rel_err_sampled']:.2e}")

    cplx = None
    if not args.no_complex:
        cplx = complex_leg(args.complex_size, N, args.phi, args.seed, args.steps, args.warmup)
        _log(f"zgemm {args.complex_size}^3 N={N}: {cplx['tflops']} TFLOPS (8mnk/t) vs native "
             f"{cplx['native_zgemm_tflops']}; INT8 GEMMs at {cplx['int8_gemm_top_s']} TOP/s; "
             f"max rel err {cplx['max_rel_err_sampled']:.2e}")

    out = {
        "metric": "Emulated DGEMM TFLOPS (2mnk/t) at fixed max rel. error; batched vs plain",
        "value": round(value, 2),
        "unit": "TFLOPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "ms_median": round(ms_median, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8",
        "io_dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"square DGEMM m=n=k={m if m == n == k else (m, n, k)}, "
                        f"entries (rand-0.5)*exp({args.phi}*randn) seed {args.seed}, "
                        f"Ozaki-II {args.mode} fast-mode scaling, N={N} INT8 moduli, plain",
            "m": m, "n": n, "k": k, "phi": args.phi, "N": N, "mode": args.mode,
            "seed": args.seed, "parallelism": "single GPU",
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "stage_ms_per_step": st,
        "native_fp64_tflops": None if native is None else round(native, 2),
        "sample_check": sample_check,
        "fixed_error": fixed,
        "batched": batched,
        "complex": cplx,
        "context": {"paper_gh200_cublas_dgemm_tflops": 60.9,
                    "paper_gh200_ozaki2_dgemm_tflops_up_to": 80.2},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
