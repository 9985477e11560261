"""Summaries of rocprofv3 output for the committed profiles (host only).

    python -m paper_2606_29129_amd.profiling stats DIR TITLE COMMAND > summary.md
    python -m paper_2606_29129_amd.profiling traffic FETCH_DIR WRITE_DIR COMMAND \
        --workload "m=16384 n=16384 k=16384 N=14" --copy-bytes B > traffic.txt
    python -m paper_2606_29129_amd.profiling counters COMMAND DIR... --ms T --ops X
    python -m paper_2606_29129_amd.profiling batch [--replays R] [--timing]
    python -m paper_2606_29129_amd.profiling zeros [--size S] [--N N] [--phi P] [--modes 0,1]
    python -m paper_2606_29129_amd.profiling shape --m M --n N --k K [--N NM] [--calls C]
    python -m paper_2606_29129_amd.profiling clock DIR COMMAND --labels a,b,...
    python -m paper_2606_29129_amd.profiling issue COMMAND DIR... [--units NAME=COUNT ...]

``stats`` reads the ``*kernel_stats.csv`` that ``rocprofv3 --kernel-trace
--stats --output-format csv`` writes and prints a short markdown table of the
library's kernels.  ``traffic`` reads the ``*counter_collection.csv`` of two
``rocprofv3 --pmc`` runs (FETCH_SIZE, then WRITE_SIZE; both in KiB per
dispatch), averages each counter over the dispatches of the INT8 GEMM kernel,
and scales it by what the same counter reads for a plain streaming kernel of
known size in the same run (``bench.py --traffic-calibration``: one
``torch.abs`` over a float64 tensor of ``--copy-bytes`` bytes, which reads and
writes that many bytes once).  The result is the file that ``bench.py`` reads
to fill ``roofline.traffic``.  ``zeros`` runs emulated DGEMMs of one
workload in several scaling modes (operands generated on the device, a few
calls per mode, twice over) and prints the fraction of zero entries of the
scaled integers A'; ``clock`` reads a ``rocprofv3 --kernel-trace --pmc
GRBM_GUI_ACTIVE SQ_BUSY_CU_CYCLES SQ_VALU_MFMA_BUSY_CYCLES`` run of it and
prints, per INT8 GEMM dispatch, its duration, the shader clock it ran at and
the MFMA pipes' busy fraction.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
K3_SOURCE = os.path.join(HERE, "csrc", "oz2_k3_gemm.hpp")
K3_NAME = "k3_gemm_i8"
COPY_NAME = "AbsFunctor"


def source_sha(path: str = K3_SOURCE) -> str:
    """sha256 (16 hex digits) of a C++ source with its comments, leading and
    trailing blanks and empty lines removed: a profile stays matched to the
    code it measured when only comments change."""
    with open(path) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    lines = [ln.strip() for ln in text.splitlines()]
    code = "\n".join(ln for ln in lines if ln)
    return hashlib.sha256(code.encode()).hexdigest()[:16]


def _find(d: str, suffix: str) -> list[str]:
    files = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return files


def _short(name: str) -> str:
    return name.split("(")[0].replace("void ", "").strip()


def kernel_stats(d: str):
    rows = []
    for path in _find(d, "kernel_stats.csv"):
        with open(path, newline="") as f:
            for r in csv.DictReader(f):
                rows.append(dict(name=r["Name"], calls=int(r["Calls"]),
                                 total_ns=float(r["TotalDurationNs"]),
                                 avg_ns=float(r["AverageNs"]),
                                 pct=float(r["Percentage"]),
                                 min_ns=float(r.get("MinNs", "nan") or "nan"),
                                 max_ns=float(r.get("MaxNs", "nan") or "nan")))
    return rows


def stats_markdown(d: str, title: str, cmd: str) -> str:
    rows = kernel_stats(d)
    out = [f"# {title}", "", "Command (run from the repository root on one MI355X):", "",
           "```", cmd, "```", "",
           "rocprofv3 kernel statistics (`*kernel_stats.csv`; durations in microseconds):", "",
           "| kernel | calls | total us | average us | min us | max us | % of GPU time |",
           "|---|---|---|---|---|---|---|"]
    other = [0, 0.0, 0.0, 0]
    for r in sorted(rows, key=lambda r: -r["total_ns"]):
        s = _short(r["name"])
        if s.startswith("oz2::"):
            out.append(f"| `{s}` | {r['calls']} | {r['total_ns'] / 1e3:.1f} | "
                       f"{r['avg_ns'] / 1e3:.1f} | {r['min_ns'] / 1e3:.1f} | "
                       f"{r['max_ns'] / 1e3:.1f} | {r['pct']:.2f} |")
        else:
            other[0] += r["calls"]
            other[1] += r["total_ns"]
            other[2] += r["pct"]
            other[3] += 1
    out.append(f"| (other kernels: input generation, copies; {other[3]} kinds) | {other[0]} | "
               f"{other[1] / 1e3:.1f} | - | - | - | {other[2]:.2f} |")
    return "\n".join(out) + "\n"


def counter_means(d: str, counter: str):
    """{short kernel name: mean over dispatches of the counter's per-dispatch
    total} and the dispatch counts."""
    per = defaultdict(float)
    names = {}
    for path in _find(d, "counter_collection.csv"):
        with open(path, newline="") as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                key = (path, r["Dispatch_Id"])
                per[key] += float(r["Counter_Value"])
                names[key] = _short(r["Kernel_Name"])
    sums, counts = defaultdict(float), defaultdict(int)
    for key, v in per.items():
        sums[names[key]] += v
        counts[names[key]] += 1
    return {k: sums[k] / counts[k] for k in sums}, dict(counts)


def _pick(means: dict, needle: str) -> str:
    hits = [k for k in means if needle in k]
    if len(hits) != 1:
        raise ValueError(f"expected one kernel matching {needle!r}, found {hits}")
    return hits[0]


def traffic_text(fetch_dir: str, write_dir: str, cmd: str, workload: str, copy_bytes: int) -> str:
    fm, fc = counter_means(fetch_dir, "FETCH_SIZE")
    wm, wc = counter_means(write_dir, "WRITE_SIZE")
    k3f, k3w = _pick(fm, K3_NAME), _pick(wm, K3_NAME)
    cpf, cpw = _pick(fm, COPY_NAME), _pick(wm, COPY_NAME)
    f_scale = copy_bytes / (fm[cpf] * 1024.0)
    w_scale = copy_bytes / (wm[cpw] * 1024.0)
    fetch_b = fm[k3f] * 1024.0 * f_scale
    write_b = wm[k3w] * 1024.0 * w_scale
    lines = [
        "# HBM traffic of the INT8 GEMM kernel (rocprofv3 --pmc, two passes)",
        f"command: {cmd}",
        f"kernel: {k3f}",
        f"kernel_code_sha256: {source_sha()}",
        f"workload: {workload}",
        f"k3_dispatches_fetch_pass: {fc[k3f]}",
        f"k3_dispatches_write_pass: {wc[k3w]}",
        f"k3_fetch_size_kib_per_dispatch: {fm[k3f]:.1f}",
        f"k3_write_size_kib_per_dispatch: {wm[k3w]:.1f}",
        f"copy_kernel: {cpf}",
        f"copy_bytes_read_and_written: {copy_bytes}",
        f"copy_fetch_size_kib: {fm[cpf]:.1f}",
        f"copy_write_size_kib: {wm[cpw]:.1f}",
        f"fetch_scale: {f_scale:.4f}",
        f"write_scale: {w_scale:.4f}",
        f"hbm_fetch_bytes_per_launch: {fetch_b:.6e}",
        f"hbm_write_bytes_per_launch: {write_b:.6e}",
        f"hbm_bytes_per_launch: {fetch_b + write_b:.6e}",
    ]
    return "\n".join(lines) + "\n"


def counters_markdown(dirs, cmd: str, kernel: str, ms_per_launch: float, ops_per_launch: float,
                      cus: int = 256, xcds: int = 8, peak_tops: float = 5000.0) -> str:
    """Per-dispatch means of every counter collected for the kernel over the
    given ``--pmc`` runs, plus derived figures: the shader clock
    (GRBM_GUI_ACTIVE, summed over the XCDs, over the launch time), the MFMA
    busy fraction (SQ_VALU_MFMA_BUSY_CYCLES over SQ_BUSY_CU_CYCLES x 4 SIMDs),
    the fraction of wave cycles spent in s_waitcnt and the achieved fraction
    of the INT8 MFMA peak."""
    vals = {}
    for d in dirs:
        for path in _find(d, "counter_collection.csv"):
            per = defaultdict(float)
            names = {}
            with open(path, newline="") as f:
                for r in csv.DictReader(f):
                    if kernel not in r["Kernel_Name"]:
                        continue
                    key = (r["Counter_Name"], r["Dispatch_Id"])
                    per[key] += float(r["Counter_Value"])
            sums, counts = defaultdict(float), defaultdict(int)
            for (cname, _), v in per.items():
                sums[cname] += v
                counts[cname] += 1
            for cname in sums:
                vals[cname] = (sums[cname] / counts[cname], counts[cname])
    out = [f"# Counters of `{kernel}` (rocprofv3 --pmc)", "", "Command (run from the repository "
           "root on one MI355X; one run per counter group):", "", "```", cmd, "```", "",
           "| counter | mean per dispatch | dispatches |", "|---|---|---|"]
    for cname in sorted(vals):
        v, c = vals[cname]
        out.append(f"| {cname} | {v:.6g} | {c} |")
    out.append("")
    gui = vals.get("GRBM_GUI_ACTIVE", (None, 0))[0]
    cu_cycles = vals.get("SQ_BUSY_CU_CYCLES", (None, 0))[0]
    if gui:
        out.append(f"* shader clock: GRBM_GUI_ACTIVE / ({xcds} XCDs x launch time) = "
                   f"{gui / xcds / (ms_per_launch * 1e-3) / 1e9:.3f} GHz (the counter is "
                   f"summed over the XCDs; launch time {ms_per_launch} ms from the kernel trace)")
    if cu_cycles:
        out.append(f"* busy cycles per CU: SQ_BUSY_CU_CYCLES / {cus} = {cu_cycles / cus:.4g} "
                   f"({cu_cycles / cus / (ms_per_launch * 1e-3) / 1e9:.3f} GHz over the launch)")
        busy = vals.get("SQ_VALU_MFMA_BUSY_CYCLES", (None, 0))[0]
        if busy:
            out.append(f"* MFMA busy: SQ_VALU_MFMA_BUSY_CYCLES / (SQ_BUSY_CU_CYCLES x 4 SIMDs) = "
                       f"{busy / (cu_cycles * 4):.4f}")
        wait = vals.get("SQ_WAIT_ANY", (None, 0))[0]
        wave = vals.get("SQ_WAVE_CYCLES", (None, 0))[0]
        if wait and wave:
            out.append(f"* waves waiting (s_waitcnt): SQ_WAIT_ANY / SQ_WAVE_CYCLES = {wait / wave:.4f}")
    out.append(f"* achieved INT8 rate: {ops_per_launch:.4g} ops / {ms_per_launch} ms = "
               f"{ops_per_launch / (ms_per_launch * 1e-3) / 1e12:.1f} TOP/s = "
               f"{ops_per_launch / (ms_per_launch * 1e-3) / 1e12 / peak_tops:.4f} of "
               f"{peak_tops:.0f} TOP/s")
    return "\n".join(out) + "\n"


def batch_problems(count=256, seed=0):
    """The batch of the benchmark's batched leg: m, n, k each
    round(exp(U(ln 64, ln 2048))), phi ~ U(0.5, 3), problem i from seed + i.
    Returns [(m, n, k, phi, seed_i)]."""
    import numpy as np
    rng = np.random.default_rng(seed)
    shapes = np.exp(rng.uniform(np.log(64), np.log(2048), (count, 3))).round().astype(int)
    phis = rng.uniform(0.5, 3.0, count)
    return [(int(m), int(n), int(k), float(phis[i]), seed + i)
            for i, (m, n, k) in enumerate(shapes)]


def run_batch(replays=3, count=256, seed=0, target=1e-15, timing=False):
    """Driver for profiling the batched path: the benchmark's batch with its
    operands generated on the host (numpy) and copied to the GPU, so that the
    only kernels of the process are the library's own (profilers then see no
    framework kernels); one call with N = 0 (the library's autotuner for the
    target), then `replays` graph replays with the chosen N.  Prints the
    median replay time."""
    import statistics
    import time
    import torch
    from paper_2606_29129_amd import inputs
    from paper_2606_29129_amd import ozaki2 as oz
    dev = torch.device("cuda:0")
    pairs = []
    for m, n, k, phi, s in batch_problems(count, seed):
        A = torch.from_numpy(inputs.ozaki_matrix(m, k, phi, s, 0)).to(dev)
        B = torch.from_numpy(inputs.ozaki_matrix(k, n, phi, s, 1)).to(dev)
        pairs.append((A, B))
    outs, Ns = oz.dgemm_batched(pairs, 0, target=target, return_N=True)
    probs = [(B.shape[1], A.shape[0], A.shape[1], B, max(1, B.shape[1]), A, max(1, A.shape[1]),
              C, max(1, B.shape[1]), N) for (A, B), C, N in zip(pairs, outs, Ns)]
    oz.ensure_workspace(oz.ozaki2_dgemm_batched_workspace_size(probs))
    oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
    if timing:
        oz.ozaki2_set_timing(1)
    per = []
    for _ in range(replays):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, bad, _ = oz.ozaki2_dgemm_batched(probs, 0)
        torch.cuda.synchronize()
        per.append((time.perf_counter() - t0) * 1e3)
        if rc:
            raise oz.Ozaki2Error(f"ozaki2_dgemm_batched (problem {bad})", rc)
    print(f"batch of {count}: N {min(Ns)}..{max(Ns)}, median replay {statistics.median(per):.3f} ms "
          f"(host clock)", flush=True)
    if timing:
        st, calls = oz.ozaki2_get_stage_times()
        oz.ozaki2_set_timing(0)
        print("stages ms/call:", {n: round(v / max(calls, 1), 4)
                                  for n, v in zip(oz.STAGE_NAMES, st)}, flush=True)


def run_zeros(size=16384, N=9, phi=4.0, modes=(0, 1), reps=3):
    """Driver for the clock-by-data measurement: `reps` calls per mode, the
    mode sequence run twice, then the zero fraction of A' per mode."""
    import torch
    from paper_2606_29129_amd import inputs
    from paper_2606_29129_amd.sweep import Problem, zero_fraction
    dev = torch.device("cuda:0")
    A = inputs.ozaki_matrix_torch(size, size, phi, 0, 0, dev)
    B = inputs.ozaki_matrix_torch(size, size, phi, 0, 1, dev)
    P = Problem(torch, A, B, N)
    for mode in list(modes) * 2:
        for _ in range(reps):
            P.run(N, mode)
        torch.cuda.synchronize()
        eA, _ = P.exponents(N, mode)
        print(f"m=n=k={size} phi={phi} N={N} mode {mode}: {reps} calls; zero fraction of A' "
              f"{zero_fraction(torch, A, eA, 0):.4f}", flush=True)
    P.release()


def run_shape(m, n, k, N=14, phi=1.0, calls=5):
    """Driver for counter runs of one DGEMM shape: operands generated on the
    host and copied to the GPU (the process's only kernels are the library's
    and copies), `calls` calls in the revised mode."""
    import torch
    from paper_2606_29129_amd import inputs
    from paper_2606_29129_amd import ozaki2 as oz
    dev = torch.device("cuda:0")
    A, B = inputs.problem(m, n, k, phi, seed=0)
    A_cm = torch.from_numpy(A.T.copy()).to(dev)
    B_cm = torch.from_numpy(B.T.copy()).to(dev)
    C_cm = torch.empty((n, m), dtype=torch.float64, device=dev)
    oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
    oz.ensure_workspace(oz.ozaki2_workspace_size(m, n, k, N, 0))
    for _ in range(calls):
        oz._check("ozaki2_dgemm", oz.ozaki2_dgemm(m, n, k, A_cm, m, B_cm, k, C_cm, m, N, 0))
    torch.cuda.synchronize()
    print(f"{calls} calls of {m}x{n}x{k}, N={N}, phi={phi}", flush=True)


def clock_markdown(d: str, cmd: str, labels, kernel: str = K3_NAME) -> str:
    """Per dispatch of `kernel` in a --kernel-trace --pmc run: duration (from
    the counter file's timestamps), shader clock GRBM_GUI_ACTIVE / (8 XCDs x
    duration), MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / (4 SIMDs x
    SQ_BUSY_CU_CYCLES); labels name the dispatches in order."""
    per = {}
    for f in _find(d, "counter_collection.csv"):
        for r in csv.DictReader(open(f)):
            if kernel not in r["Kernel_Name"]:
                continue
            k = int(r["Dispatch_Id"])
            e = per.setdefault(k, {"dur": (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9})
            e[r["Counter_Name"]] = float(r["Counter_Value"])
    out = [f"# Shader clock of `{kernel}` by operand data (rocprofv3 --kernel-trace --pmc)", "",
           "Command (run from the repository root on one MI355X):", "", "```", cmd, "```", "",
           "| dispatch | label | ms | clock GHz | MFMA busy |", "|---|---|---|---|---|"]
    for i, k in enumerate(sorted(per)):
        e = per[k]
        clk = e["GRBM_GUI_ACTIVE"] / 8 / e["dur"] / 1e9
        busy = e["SQ_VALU_MFMA_BUSY_CYCLES"] / (4 * e["SQ_BUSY_CU_CYCLES"])
        lab = labels[i] if i < len(labels) else "?"
        out.append(f"| {k} | {lab} | {e['dur'] * 1e3:.2f} | {clk:.3f} | {busy:.3f} |")
    return "\n".join(out) + "\n"


def issue_markdown(dirs, cmd: str, units=None) -> str:
    """Per kernel of ``--kernel-trace --pmc`` runs (counter files with
    timestamps): mean duration, shader clock, VALU wave instructions, the
    VALU issue fraction (4 cycles per wave instruction over 1024 SIMDs'
    cycles at that clock), and the s_waitcnt fraction of wave cycles when
    those counters were collected.  `units` maps a kernel-name fragment to a
    unit count (entries, outputs) for lane-operations per unit."""
    per = defaultdict(dict)
    for d in dirs:
        for f in _find(d, "counter_collection.csv"):
            for r in csv.DictReader(open(f)):
                key = (d, int(r["Dispatch_Id"]))
                e = per[key]
                e["name"] = _short(r["Kernel_Name"])
                e["dur"] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
                e[r["Counter_Name"]] = float(r["Counter_Value"])
    agg = defaultdict(lambda: defaultdict(list))
    for e in per.values():
        for c, v in e.items():
            if c != "name":
                agg[e["name"]][c].append(v)
    out = ["# VALU issue and waits of the element-wise kernels (rocprofv3 --pmc)", "",
           "Command (run from the repository root on one MI355X; one run per counter group):",
           "", "```", cmd, "```", "",
           "| kernel | ms | clock GHz | VALU wave instructions | lane-ops per unit | VALU issue | "
           "waves in s_waitcnt |", "|---|---|---|---|---|---|---|"]
    for name in sorted(agg):
        m = {c: sum(v) / len(v) for c, v in agg[name].items()}
        clk = m["GRBM_GUI_ACTIVE"] / 8 / m["dur"] if "GRBM_GUI_ACTIVE" in m else float("nan")
        valu = m.get("SQ_INSTS_VALU", float("nan"))
        issue = valu * 4 / 1024 / (clk * m["dur"])
        wait = (m["SQ_WAIT_ANY"] / m["SQ_WAVE_CYCLES"]) if "SQ_WAIT_ANY" in m else float("nan")
        per_unit = "-"
        for frag, cnt in (units or {}).items():
            if frag in name:
                per_unit = f"{valu * 64 / cnt:.0f}"
        out.append(f"| `{name}` | {m['dur'] * 1e3:.3f} | {clk / 1e9:.2f} | {valu:.3e} | {per_unit} | "
                   f"{issue:.2f} | {wait:.2f} |")
    return "\n".join(out) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("title")
    s.add_argument("command")
    t = sub.add_parser("traffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    t.add_argument("command")
    t.add_argument("--workload", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    c = sub.add_parser("counters")
    c.add_argument("command")
    c.add_argument("dirs", nargs="+")
    c.add_argument("--kernel", default=K3_NAME)
    c.add_argument("--ms", type=float, required=True, help="average launch time, ms")
    c.add_argument("--ops", type=float, required=True, help="algorithmic ops per launch")
    b = sub.add_parser("batch", help="run the benchmark's batch (host-generated operands)")
    b.add_argument("--replays", type=int, default=3)
    b.add_argument("--count", type=int, default=256)
    b.add_argument("--timing", action="store_true", help="stage events instead of the graph")
    z = sub.add_parser("zeros", help="DGEMMs of one workload in several modes; zero fractions")
    z.add_argument("--size", type=int, default=16384)
    z.add_argument("--N", type=int, default=9)
    z.add_argument("--phi", type=float, default=4.0)
    z.add_argument("--modes", default="0,1")
    z.add_argument("--reps", type=int, default=3)
    h = sub.add_parser("shape", help="DGEMMs of one shape, host-generated operands")
    h.add_argument("--m", type=int, required=True)
    h.add_argument("--n", type=int, required=True)
    h.add_argument("--k", type=int, required=True)
    h.add_argument("--N", type=int, default=14)
    h.add_argument("--phi", type=float, default=1.0)
    h.add_argument("--calls", type=int, default=5)
    k = sub.add_parser("clock")
    k.add_argument("dir")
    k.add_argument("command")
    k.add_argument("--labels", default="")
    i = sub.add_parser("issue")
    i.add_argument("command")
    i.add_argument("dirs", nargs="+")
    i.add_argument("--units", nargs="*", default=[], help="kernel fragment=count")
    a = ap.parse_args(argv)
    if a.what == "issue":
        units = {u.split("=")[0]: float(u.split("=")[1]) for u in a.units}
        sys.stdout.write(issue_markdown(a.dirs, a.command, units))
    elif a.what == "shape":
        run_shape(a.m, a.n, a.k, a.N, a.phi, a.calls)
    elif a.what == "zeros":
        run_zeros(a.size, a.N, a.phi, tuple(int(x) for x in a.modes.split(",")), a.reps)
    elif a.what == "clock":
        sys.stdout.write(clock_markdown(a.dir, a.command, a.labels.split(",") if a.labels else []))
    elif a.what == "batch":
        run_batch(a.replays, a.count, timing=a.timing)
    elif a.what == "counters":
        sys.stdout.write(counters_markdown(a.dirs, a.command, a.kernel, a.ms, a.ops))
    elif a.what == "stats":
        sys.stdout.write(stats_markdown(a.dir, a.title, a.command))
    else:
        sys.stdout.write(traffic_text(a.fetch_dir, a.write_dir, a.command, a.workload,
                                      a.copy_bytes))


if __name__ == "__main__":
    main()
