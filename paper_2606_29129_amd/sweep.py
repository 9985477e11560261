"""Measurement sweeps over the benchmark configurations, on one GPU.

    python -m paper_2606_29129_amd.sweep throughput [--sizes 1024,4096,...]
    python -m paper_2606_29129_amd.sweep shapes
    python -m paper_2606_29129_amd.sweep scale
    python -m paper_2606_29129_amd.sweep accuracy [--block 512]
    python -m paper_2606_29129_amd.sweep sgemm [--sizes 4096,8192,16384]
    python -m paper_2606_29129_amd.sweep complex [--sizes 4096,8192] [--zNs ...] [--cNs ...]
    python -m paper_2606_29129_amd.sweep alpha [--alpha-sizes 1024,16384] [--alpha-cases ...]
    python -m paper_2606_29129_amd.sweep modes [--alpha-sizes 1024,16384]

Every result is one JSON line on stdout.

* ``throughput``: square m = n = k, entries (rand - 0.5) exp(phi randn)
  (Section 3.2), over sizes, phi and N (revised fast mode): emulated TFLOPS
  2mnk/t (median of timed steps), per-stage milliseconds, INT8 MFMA
  utilisation of the GEMM stage, native FP64 ``torch.matmul`` of the same
  GPU, and the error on a sampled block.
* ``shapes``: rectangular and skinny shapes (m = n = 8192 with k = 1024,
  8192, 65536; m = 65536, n = 64, k = 4096; phi = 1, N = 14), the revised
  fast mode beside the original fast mode (Algorithm 1) and accurate mode.
* ``scale``: A multiplied by 2^300, 2^-300 (C must be the unscaled result
  times the same power, bit for bit, in every row whose Algorithm 2 exponent
  shifted exactly; rows where the binary32 rounding of w lowered it by one
  are counted; the exact mode must shift every row and scale all of C) and
  by 3.7e100, 3.7e-100 (error).
* ``accuracy``: m = n = k = 8192, phi = 2; DGEMM for N = 8..20 and SGEMM on
  the binary32-rounded inputs for N = 5..9: maximum relative and
  componentwise error on a block of rows and columns picked by a seeded
  permutation, against a double-double product over the full k; the
  fraction of zero entries of A' and B' (a' = trunc(a 2^e)).

* ``sgemm``: binary32 emulation (Section 5) over sizes for N = 5..9 beside
  native binary32 ``torch.matmul``.
* ``alpha``: the scale experiment of Sections 3.2 and 4: fixed matrices
  Ahat, Bhat (random with phi in the list, or all ones) and the inputs
  A = 2^s Ahat, B = 2^s Bhat for s = -10..10; the maximum relative and
  componentwise error of the revised fast mode, the original fast mode
  (Algorithm 1) and accurate mode at one N, and of native FP64, on a
  sampled block (the reference is the block's double-double product times
  4^s, exact); over the whole matrix, the original and accurate modes'
  largest relative and componentwise distance from the revised result and
  the number of entries more than 0.1% away from it (failed CRT recoveries
  show up there).
* ``modes``: the accuracy comparison of Section 5.1: DGEMM for N = 9..20
  at phi = 0.5, 1, 2, 3, 4 and SGEMM (binary32-rounded inputs) for N = 3..12
  at phi = 0, 0.5, 1, 1.5, each in the revised fast mode, the original fast
  mode and accurate mode, beside native ``torch.matmul``: the error of a
  sampled block against its double-double product, and over the whole
  matrix the maximum relative distance from the revised binary64 emulation
  at N = 20 of the same inputs (whose sampled error is at the binary64
  floor; for SGEMM far below binary32's); and each run's throughput 2mnk/t
  (median of timed calls) beside native ``torch.matmul``'s, for the
  accuracy-throughput trade-off of Section 5.3.
* ``complex``: ZGEMM and CGEMM emulation (8mnk/t) over sizes and N beside
  native complex ``torch.matmul``; errors per part against a double-double
  reference (Re = [Re A, -Im A][Re B; Im B], Im = [Re A, Im A][Im B; Re B]).

Errors: ``max_rel`` = max |C - R| / |R| over R != 0 (``zero_ref_nonzero``
counts R = 0 with C != 0), ``max_cw`` = max |C - R| / (|A||B|)_ij.  The
reference R is a double-double dot product (TwoProduct by Veltkamp
splitting, TwoSum accumulation in the order of h), written here in plain
numpy; its own error is near 2^-100 relative, far below what is measured.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import inputs
from . import ozaki2 as oz

INT8_PEAK_TOPS = 5000.0


def _emit(d):
    print(json.dumps(d), flush=True)


# --- double-double reference --------------------------------------------------

def _split(x):
    c = x * 134217729.0          # 2^27 + 1
    hi = c - (c - x)
    return hi, x - hi


def dd_block(Ar, Bc):
    """Ar (r x k) times Bc (k x c) in double-double; returns (hi, lo)."""
    Ar = np.ascontiguousarray(Ar, np.float64)
    Bc = np.ascontiguousarray(Bc, np.float64)
    r, k = Ar.shape
    c = Bc.shape[1]
    ah, al = _split(Ar)
    bh, bl = _split(Bc)
    s = np.zeros((r, c))
    e = np.zeros((r, c))
    for h in range(k):
        a, b = Ar[:, h:h + 1], Bc[h:h + 1, :]
        p = a * b
        ahh, alh, bhh, blh = ah[:, h:h + 1], al[:, h:h + 1], bh[h:h + 1, :], bl[h:h + 1, :]
        perr = ((ahh * bhh - p) + ahh * blh + alh * bhh) + alh * blh
        t = s + p
        z = t - s
        e += ((s - (t - z)) + (p - z)) + perr
        s = t
    hi = s + e
    lo = e - (hi - s)
    return hi, lo


def errors(C, ref, absAB):
    hi, lo = ref
    d = np.abs((C - hi) - lo)
    nz = hi != 0
    max_rel = float(np.max(d[nz] / np.abs(hi[nz]))) if nz.any() else 0.0
    zero_bad = int(np.count_nonzero((~nz) & (C != 0)))
    pos = absAB > 0
    max_cw = float(np.max(d[pos] / absAB[pos])) if pos.any() else 0.0
    return dict(max_rel=max_rel, max_cw=max_cw, zero_ref_nonzero=zero_bad)


# --- timing -----------------------------------------------------------------

def _timed(torch, fn, steps, warmup):
    """Median time of `steps` calls, each between two events on the current
    stream (no stage events inside them), then the mean per-stage times of
    `steps` further calls made with stage timing on."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    evs[0].record(stream)
    for s in range(steps):
        fn()
        evs[s + 1].record(stream)
    torch.cuda.synchronize()
    per = sorted(evs[s].elapsed_time(evs[s + 1]) for s in range(steps))
    oz._check("ozaki2_set_timing", oz.ozaki2_set_timing(1))
    for _ in range(steps):
        fn()
    stage_ms, calls = oz.ozaki2_get_stage_times()
    oz.ozaki2_set_timing(0)
    st = {name: round(v / max(calls, 1), 4) for name, v in zip(oz.STAGE_NAMES, stage_ms)}
    return per[len(per) // 2], st


def _native_ms(torch, A, B, steps=10):
    """Median time of `steps` torch.matmul calls (each between two events),
    after one warm-up call; also returns the product."""
    C = torch.matmul(A, B)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    evs[0].record(stream)
    for s in range(steps):
        torch.matmul(A, B, out=C)
        evs[s + 1].record(stream)
    torch.cuda.synchronize()
    per = sorted(evs[s].elapsed_time(evs[s + 1]) for s in range(steps))
    return per[len(per) // 2], C


class Problem:
    """Column-major device operands of C = A B (A m x k, B k x n) plus the
    output and a caller workspace sized for the largest N used."""

    def __init__(self, torch, A_rm, B_rm, Nmax, mode=0, single=False):
        self.torch = torch
        self.m, self.k = A_rm.shape
        self.n = B_rm.shape[1]
        dt = torch.float32 if single else torch.float64
        self.A_cm = A_rm.to(dt).t().contiguous()
        self.B_cm = B_rm.to(dt).t().contiguous()
        self.C_cm = torch.empty((self.n, self.m), dtype=dt, device=A_rm.device)
        nb = max(oz.ozaki2_workspace_size(self.m, self.n, self.k, Nmax, md) for md in (0, 1, 2))
        self.ws = torch.empty(nb + 256, dtype=torch.uint8, device=A_rm.device)
        ptr = (self.ws.data_ptr() + 255) // 256 * 256
        oz._check("ozaki2_set_workspace", oz.ozaki2_set_workspace(ptr, nb))
        oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
        self.fn = oz.ozaki2_sgemm if single else oz.ozaki2_dgemm

    def run(self, N, mode=0):
        rc = self.fn(self.m, self.n, self.k, self.A_cm, self.m, self.B_cm, self.k, self.C_cm,
                     self.m, N, mode)
        if rc:
            raise oz.Ozaki2Error(self.fn.__name__, rc)

    def C_block(self, rows, cols):
        """C[rows][:, cols] on the host as float64."""
        t = self.torch
        r = t.as_tensor(rows, device=self.C_cm.device)
        c = t.as_tensor(cols, device=self.C_cm.device)
        return self.C_cm.index_select(0, c).index_select(1, r).t().double().cpu().numpy()

    def exponents(self, N, mode=0):
        t = self.torch
        eA = t.zeros(self.m, dtype=t.int32, device=self.C_cm.device)
        eB = t.zeros(self.n, dtype=t.int32, device=self.C_cm.device)
        # the binary32 path scales by the same exponents as its binary64 image
        A64, B64 = self.A_cm.double(), self.B_cm.double()
        rc = oz.ozaki2_debug_stages(self.m, self.n, self.k, A64, self.m, B64, self.k,
                                    N, mode, 0, eA, eB)
        if rc:
            raise oz.Ozaki2Error("ozaki2_debug_stages", rc)
        t.cuda.synchronize()
        return eA, eB

    def release(self):
        oz.ozaki2_set_workspace(None, 0)
        del self.ws, self.A_cm, self.B_cm, self.C_cm
        self.torch.cuda.empty_cache()


def zero_fraction(torch, X_rm, e, axis):
    """Fraction of entries x with trunc(x 2^e) == 0 (e per row if axis = 0,
    per column if axis = 1), computed exactly with ldexp and trunc."""
    zeros = 0
    total = 0
    rows = X_rm.shape[0]
    for r0 in range(0, rows, 2048):
        blk = X_rm[r0:r0 + 2048]
        ee = e[r0:r0 + 2048].view(-1, 1) if axis == 0 else e.view(1, -1)
        a = torch.ldexp(blk, ee.to(torch.float64)).trunc()
        zeros += int((a == 0).sum())
        total += a.numel()
    return zeros / total


def _block(Ar_host, Bc_host, A_rows, B_cols):
    ref = dd_block(Ar_host, Bc_host)
    absAB = np.abs(Ar_host) @ np.abs(Bc_host)
    return ref, absAB


def sweep_throughput(args):
    import torch
    dev = torch.device("cuda:0")
    sizes = [int(s) for s in args.sizes.split(",")]
    phis = [float(p) for p in args.phis.split(",")]
    Ns = [int(x) for x in args.Ns.split(",")]
    rng = np.random.default_rng(0)
    for S in sizes:
        native = None
        for phi in phis:
            A = inputs.ozaki_matrix_torch(S, S, phi, 0, 0, dev)
            B = inputs.ozaki_matrix_torch(S, S, phi, 0, 1, dev)
            if native is None:
                native, _ = _native_ms(torch, A, B)
            rows = np.sort(rng.choice(S, args.sample, replace=False))
            cols = np.sort(rng.choice(S, args.sample, replace=False))
            Ah = A[torch.as_tensor(rows, device=dev)].cpu().numpy()
            Bh = B[:, torch.as_tensor(cols, device=dev)].cpu().numpy()
            ref, absAB = _block(Ah, Bh, rows, cols)
            P = Problem(torch, A, B, max(Ns))
            for N in Ns:
                ms, st = _timed(torch, lambda: P.run(N), args.steps, args.warmup)
                flops = 2.0 * S ** 3
                k3 = st["int8_gemm"]
                _emit(dict(leg="throughput", m=S, n=S, k=S, phi=phi, N=N, mode="revised",
                           ms=round(ms, 4), tflops=round(flops / ms / 1e9, 2),
                           stage_ms=st,
                           int8_mfma_util=round(2.0 * N * S ** 3 / (k3 * 1e-3) / 1e12
                                                / INT8_PEAK_TOPS, 4) if k3 > 0 else None,
                           native_fp64_tflops=round(flops / native / 1e9, 2),
                           sample=f"{args.sample}x{args.sample} block",
                           **errors(P.C_block(rows, cols), ref, absAB)))
            P.release()
            del A, B
            torch.cuda.empty_cache()


def sweep_sgemm(args):
    """SGEMM emulation (binary32 in and out, Section 5): throughput for
    N = 5..9 beside native binary32 torch.matmul, error on a sampled block
    against a double-double product of the binary32 inputs."""
    import torch
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(3)
    for S in [int(x) for x in args.sizes.split(",")]:
        A = inputs.ozaki_matrix_torch(S, S, 1.0, 0, 0, dev).float()
        B = inputs.ozaki_matrix_torch(S, S, 1.0, 0, 1, dev).float()
        native, _ = _native_ms(torch, A, B)
        rows = np.sort(rng.choice(S, args.sample, replace=False))
        cols = np.sort(rng.choice(S, args.sample, replace=False))
        Ah = A[torch.as_tensor(rows, device=dev)].double().cpu().numpy()
        Bh = B[:, torch.as_tensor(cols, device=dev)].double().cpu().numpy()
        ref, absAB = _block(Ah, Bh, rows, cols)
        P = Problem(torch, A, B, 9, single=True)
        for N in range(5, 10):
            ms, st = _timed(torch, lambda: P.run(N), args.steps, args.warmup)
            flops = 2.0 * S ** 3
            _emit(dict(leg="sgemm", m=S, n=S, k=S, phi=1.0, N=N, ms=round(ms, 4),
                       tflops=round(flops / ms / 1e9, 2), stage_ms=st,
                       native_fp32_tflops=round(flops / native / 1e9, 2),
                       sample=f"{args.sample}x{args.sample} block",
                       **errors(P.C_block(rows, cols), ref, absAB)))
        P.release()
        del A, B
        torch.cuda.empty_cache()


def sweep_shapes(args):
    import torch
    dev = torch.device("cuda:0")
    shapes = [(8192, 8192, 1024), (8192, 8192, 8192), (8192, 8192, 65536), (65536, 64, 4096)]
    rng = np.random.default_rng(1)
    phi, N = 1.0, 14
    for (m, n, k) in shapes:
        A = inputs.ozaki_matrix_torch(m, k, phi, 0, 0, dev)
        B = inputs.ozaki_matrix_torch(k, n, phi, 0, 1, dev)
        native, _ = _native_ms(torch, A, B)
        rows = np.sort(rng.choice(m, min(args.sample, m), replace=False))
        cols = np.sort(rng.choice(n, min(args.sample, n), replace=False))
        Ah = A[torch.as_tensor(rows, device=dev)].cpu().numpy()
        Bh = B[:, torch.as_tensor(cols, device=dev)].cpu().numpy()
        ref, absAB = _block(Ah, Bh, rows, cols)
        P = Problem(torch, A, B, N)
        for mode, name in ((0, "revised"), (1, "original"), (2, "accurate")):
            ms, st = _timed(torch, lambda: P.run(N, mode), args.steps, args.warmup)
            flops = 2.0 * m * n * k
            _emit(dict(leg="shapes", m=m, n=n, k=k, phi=phi, N=N, mode=name, ms=round(ms, 4),
                       tflops=round(flops / ms / 1e9, 2), stage_ms=st,
                       native_fp64_tflops=round(flops / native / 1e9, 2),
                       sample=f"{len(rows)}x{len(cols)} block",
                       **errors(P.C_block(rows, cols), ref, absAB)))
        P.release()
        del A, B
        torch.cuda.empty_cache()


def sweep_scale(args):
    import torch
    dev = torch.device("cuda:0")
    S, phi, N = args.scale_size, 0.5, 14
    A = inputs.ozaki_matrix_torch(S, S, phi, 0, 0, dev)
    B = inputs.ozaki_matrix_torch(S, S, phi, 0, 1, dev)
    P = Problem(torch, A, B, N)
    P.run(N)
    C0 = P.C_cm.clone()
    e0, _ = P.exponents(N)
    P.release()
    rng = np.random.default_rng(2)
    rows = np.sort(rng.choice(S, args.sample, replace=False))
    cols = np.sort(rng.choice(S, args.sample, replace=False))
    for c, label in ((2.0 ** 300, "2^300"), (2.0 ** -300, "2^-300"),
                     (3.7e100, "3.7e100"), (3.7e-100, "3.7e-100")):
        Ac = A * c
        P = Problem(torch, Ac, B, N)
        P.run(N)
        torch.cuda.synchronize()
        out = dict(leg="scale", m=S, n=S, k=S, phi=phi, N=N, factor=label)
        if label.startswith("2^"):
            # Section 4: exponents shift by -+300 and C scales exactly, except
            # where Algorithm 2's binary32 rounding of w lowers an exponent by
            # one; those rows are counted and the rest compared bit for bit
            sh = -300 if label == "2^300" else 300
            e1, _ = P.exponents(N)
            lower = (e1 != e0 + sh)
            out["rows_exponent_shifted_exactly"] = int((~lower).sum())
            out["rows_exponent_one_lower"] = int((e1 == e0 + sh - 1).sum())
            keep = (~lower).nonzero().flatten()
            same = torch.equal(P.C_cm.index_select(1, keep), C0.index_select(1, keep) * c)
            out["bit_identical_to_scaled_in_exact_rows"] = bool(same)
        Ah = Ac[torch.as_tensor(rows, device=dev)].cpu().numpy()
        Bh = B[:, torch.as_tensor(cols, device=dev)].cpu().numpy()
        ref, absAB = _block(Ah, Bh, rows, cols)
        out.update(sample=f"{args.sample}x{args.sample} block",
                   **errors(P.C_block(rows, cols), ref, absAB))
        _emit(out)
        if label.startswith("2^"):
            # exact mode: the exact maximal exponent shifts by exactly -+300
            # in every row, so C scales exactly everywhere
            P.run(N, 3)
            torch.cuda.synchronize()
            Cx = P.C_cm.clone()
            e1, _ = P.exponents(N, 3)
            P.release()
            P = Problem(torch, A, B, N, mode=3)
            P.run(N, 3)
            torch.cuda.synchronize()
            e0x, _ = P.exponents(N, 3)
            _emit(dict(leg="scale", m=S, n=S, k=S, phi=phi, N=N, factor=label, mode="exact",
                       rows_exponent_shifted_exactly=int((e1 == e0x + sh).sum()),
                       bit_identical_to_scaled=bool(torch.equal(Cx, P.C_cm * c))))
        P.release()
        del Ac


def sweep_accuracy(args):
    import torch
    dev = torch.device("cuda:0")
    S, phi = args.acc_size, 2.0
    A = inputs.ozaki_matrix_torch(S, S, phi, 0, 0, dev)
    B = inputs.ozaki_matrix_torch(S, S, phi, 0, 1, dev)
    perm = np.random.default_rng(0).permutation(S)
    rows = np.sort(perm[:args.block])
    cols = np.sort(np.random.default_rng(1).permutation(S)[:args.block])
    rt = torch.as_tensor(rows, device=dev)
    ct = torch.as_tensor(cols, device=dev)
    for single in (False, True):
        Au = A.float().double() if single else A
        Bu = B.float().double() if single else B
        Ah = Au[rt].cpu().numpy()
        Bh = Bu[:, ct].cpu().numpy()
        t0 = time.time()
        ref, absAB = _block(Ah, Bh, rows, cols)
        ref_s = time.time() - t0
        # native product of the same GPU, same block
        if single:
            Cn = torch.matmul(A.float(), B.float()).double()
        else:
            Cn = torch.matmul(A, B)
        nat = errors(Cn[rt][:, ct].cpu().numpy(), ref, absAB)
        del Cn
        _emit(dict(leg="accuracy", m=S, n=S, k=S, phi=phi, precision="fp32" if single else "fp64",
                   method="native torch.matmul", sample=f"{args.block}x{args.block} block",
                   reference_seconds=round(ref_s, 1), **nat))
        Ns = range(5, 10) if single else range(8, 21)
        P = Problem(torch, A, B, max(Ns), single=single)
        for N in Ns:
            P.run(N)
            eA, eB = P.exponents(N)
            Xa = A.float().double() if single else A
            Xb = B.float().double() if single else B
            zA = zero_fraction(torch, Xa, eA, 0)
            zB = zero_fraction(torch, Xb.t().contiguous(), eB, 0)
            _emit(dict(leg="accuracy", m=S, n=S, k=S, phi=phi,
                       precision="fp32" if single else "fp64", method="ozaki2 revised", N=N,
                       sample=f"{args.block}x{args.block} block", zero_frac_A=round(zA, 6),
                       zero_frac_B=round(zB, 6), **errors(P.C_block(rows, cols), ref, absAB)))
        P.release()


def _complex_block(Ah, Bh):
    """Double-double reference of both parts of a complex block product, with
    the componentwise scales (|Re A||Re B| + |Im A||Im B| for the real part,
    |Re A||Im B| + |Im A||Re B| for the imaginary part)."""
    xr, xi, ur, ui = Ah.real, Ah.imag, Bh.real, Bh.imag
    re = dd_block(np.hstack([xr, -xi]), np.vstack([ur, ui]))
    im = dd_block(np.hstack([xr, xi]), np.vstack([ui, ur]))
    are = np.abs(xr) @ np.abs(ur) + np.abs(xi) @ np.abs(ui)
    aim = np.abs(xr) @ np.abs(ui) + np.abs(xi) @ np.abs(ur)
    return (re, are), (im, aim)


def _complex_errors(C, blocks):
    (re, are), (im, aim) = blocks
    er, ei = errors(C.real, re, are), errors(C.imag, im, aim)
    return dict(max_rel=max(er["max_rel"], ei["max_rel"]),
                max_cw=max(er["max_cw"], ei["max_cw"]),
                zero_ref_nonzero=er["zero_ref_nonzero"] + ei["zero_ref_nonzero"])


def sweep_complex(args):
    """ZGEMM (complex128) and CGEMM (complex64) emulation: 8mnk/t over sizes
    and N beside native complex torch.matmul of the same GPU, per-stage
    times, the INT8 rate of the 3N GEMMs, and errors per part on a sampled
    block against a double-double reference."""
    import torch
    dev = torch.device("cuda:0")
    sizes = [int(x) for x in args.sizes.split(",")]
    phi = float(args.phis.split(",")[0])
    rng = np.random.default_rng(0)
    for S in sizes:
        A = inputs.complex_matrix_torch(S, S, phi, 0, 0, dev)
        B = inputs.complex_matrix_torch(S, S, phi, 0, 1, dev)
        rows = np.sort(rng.choice(S, args.sample, replace=False))
        cols = np.sort(rng.choice(S, args.sample, replace=False))
        rt, ctt = torch.as_tensor(rows, device=dev), torch.as_tensor(cols, device=dev)
        for single in (False, True):
            dt = torch.complex64 if single else torch.complex128
            Au, Bu = A.to(dt), B.to(dt)
            Ah = Au[rt].to(torch.complex128).cpu().numpy()
            Bh = Bu[:, ctt].to(torch.complex128).cpu().numpy()
            blocks = _complex_block(Ah, Bh)
            nat_ms, Cn = _native_ms(torch, Au, Bu)
            nat_err = _complex_errors(Cn[rt][:, ctt].to(torch.complex128).cpu().numpy(), blocks)
            del Cn
            flops = 8.0 * S ** 3
            name = "cgemm" if single else "zgemm"
            _emit(dict(leg="complex", op=name, m=S, n=S, k=S, phi=phi,
                       method="native torch.matmul", tflops=round(flops / nat_ms / 1e9, 2),
                       sample=f"{args.sample}x{args.sample} block", **nat_err))
            A_cm, B_cm = Au.t().contiguous(), Bu.t().contiguous()
            C_cm = torch.empty((S, S), dtype=dt, device=dev)
            oz.ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)
            fn = oz.ozaki2_cgemm if single else oz.ozaki2_zgemm
            Ns = [int(x) for x in (args.cNs if single else args.zNs).split(",")]
            oz.ensure_workspace(max(oz.ozaki2_zgemm_workspace_size(S, S, S, N, 0) for N in Ns))
            for N in Ns:
                def run():
                    rc = fn(S, S, S, A_cm, S, B_cm, S, C_cm, S, N, 0)
                    if rc:
                        raise oz.Ozaki2Error(fn.__name__, rc)
                ms, st = _timed(torch, run, args.steps, args.warmup)
                k3 = st["int8_gemm"]
                C = C_cm.index_select(0, ctt).index_select(1, rt).t()
                _emit(dict(leg="complex", op=name, m=S, n=S, k=S, phi=phi,
                           method="ozaki2 revised", N=N, ms=round(ms, 4),
                           tflops=round(flops / ms / 1e9, 2), stage_ms=st,
                           int8_mfma_util=round(6.0 * N * S ** 3 / (k3 * 1e-3) / 1e12
                                                / INT8_PEAK_TOPS, 4) if k3 > 0 else None,
                           native_tflops=round(flops / nat_ms / 1e9, 2),
                           sample=f"{args.sample}x{args.sample} block",
                           **_complex_errors(C.to(torch.complex128).cpu().numpy(), blocks)))
            del A_cm, B_cm, C_cm, Au, Bu
            torch.cuda.empty_cache()
        del A, B
        torch.cuda.empty_cache()


def sweep_alpha(args):
    import torch
    dev = torch.device("cuda:0")
    sizes = [int(x) for x in args.alpha_sizes.split(",")]
    cases = args.alpha_cases.split(",")
    N = args.alpha_N
    rng = np.random.default_rng(4)
    modes = ((0, "revised"), (1, "original"), (2, "accurate"))
    for S in sizes:
        for case in cases:
            if case == "ones":
                Ah = torch.ones((S, S), dtype=torch.float64, device=dev)
                Bh = torch.ones((S, S), dtype=torch.float64, device=dev)
            else:
                phi = float(case)
                Ah = inputs.ozaki_matrix_torch(S, S, phi, 0, 0, dev)
                Bh = inputs.ozaki_matrix_torch(S, S, phi, 0, 1, dev)
            rows = np.sort(rng.choice(S, args.sample, replace=False))
            cols = np.sort(rng.choice(S, args.sample, replace=False))
            rt, ct = torch.as_tensor(rows, device=dev), torch.as_tensor(cols, device=dev)
            ref, absAB = _block(Ah[rt].cpu().numpy(), Bh[:, ct].cpu().numpy(), rows, cols)
            P = Problem(torch, Ah, Bh, N)
            A0, B0 = P.A_cm.clone(), P.B_cm.clone()
            # (|A||B|)^T over the whole matrix, in the layout of C^T = B^T A^T
            absT = torch.matmul(B0.abs(), A0.abs())
            for s in range(-10, 11):
                a = 2.0 ** s          # exact scalings: no entry leaves the normal range
                torch.mul(A0, a, out=P.A_cm)
                torch.mul(B0, a, out=P.B_cm)
                sc = a * a
                rs = ((ref[0] * sc, ref[1] * sc), absAB * sc)
                out = dict(leg="alpha", m=S, n=S, k=S, case=case, s=s, N=N,
                           sample=f"{args.sample}x{args.sample} block")
                Crev = None
                for md, name in modes:
                    P.run(N, md)
                    torch.cuda.synchronize()
                    out[name] = errors(P.C_block(rows, cols), *rs)
                    if Crev is None:
                        Crev = P.C_cm.clone()
                    else:
                        # over every entry, against the revised result (its
                        # sampled errors are at the binary64 floor): the
                        # largest relative and componentwise distances, and
                        # the entries more than 0.1% away from it
                        d = (P.C_cm - Crev).abs()
                        pos = absT > 0
                        nz = Crev != 0
                        rel = d[nz] / Crev[nz].abs()
                        out[name]["full_max_rel_vs_revised"] = float(rel.max())
                        out[name]["full_max_cw_vs_revised"] = float((d[pos] / (absT[pos] * sc)).max())
                        out[name]["full_entries_off_1e-3"] = int((rel > 1e-3).sum())
                        del d, pos, nz, rel
                del Crev
                Cn = torch.matmul(Ah * a, Bh * a)
                out["native"] = errors(Cn.index_select(0, rt).index_select(1, ct).cpu().numpy(),
                                       *rs)
                del Cn
                _emit(out)
            P.release()
            del A0, B0, Ah, Bh, absT
            torch.cuda.empty_cache()


def sweep_modes(args):
    import torch
    dev = torch.device("cuda:0")
    sizes = [int(x) for x in args.alpha_sizes.split(",")]
    rng = np.random.default_rng(5)
    legs = ((False, (0.5, 1.0, 2.0, 3.0, 4.0), range(9, 21)),
            (True, (0.0, 0.5, 1.0, 1.5), range(3, 13)))
    modes = ((0, "revised"), (1, "original"), (2, "accurate"))
    for S in sizes:
        for single, phis, Ns in legs:
            for phi in phis:
                A = inputs.ozaki_matrix_torch(S, S, phi, 0, 0, dev)
                B = inputs.ozaki_matrix_torch(S, S, phi, 0, 1, dev)
                if single:      # the binary32 inputs, held exactly in binary64
                    A, B = A.float().double(), B.float().double()
                rows = np.sort(rng.choice(S, args.sample, replace=False))
                cols = np.sort(rng.choice(S, args.sample, replace=False))
                rt, ct = torch.as_tensor(rows, device=dev), torch.as_tensor(cols, device=dev)
                ref, absAB = _block(A[rt].cpu().numpy(), B[:, ct].cpu().numpy(), rows, cols)
                P = Problem(torch, A, B, 20)
                P.run(20)
                Cref = P.C_cm.clone()               # C^T, revised binary64 emulation, N = 20
                P.release()
                nz = Cref != 0
                absref = Cref[nz].abs()

                def full_rel(CT):
                    return float(((CT.double() - Cref).abs()[nz] / absref).max())

                base = dict(leg="modes", m=S, n=S, k=S, phi=phi,
                            precision="fp32" if single else "fp64",
                            sample=f"{args.sample}x{args.sample} block")
                flops = 2.0 * S ** 3
                Ax, Bx = (A.float(), B.float()) if single else (A, B)
                nat_ms, Cn = _native_ms(torch, Ax, Bx)
                _emit(dict(base, method="native torch.matmul", ms=round(nat_ms, 4),
                           tflops=round(flops / nat_ms / 1e9, 2),
                           full_max_rel_vs_N20=full_rel(Cn.t()),
                           **errors(Cn.index_select(0, rt).index_select(1, ct).double()
                                    .cpu().numpy(), ref, absAB)))
                del Cn, Ax, Bx
                P = Problem(torch, A, B, max(Ns), single=single)
                for N in Ns:
                    for md, name in modes:
                        ms, st = _timed(torch, lambda: P.run(N, md), args.steps, args.warmup)
                        torch.cuda.synchronize()
                        _emit(dict(base, method=name, N=N, ms=round(ms, 4),
                                   tflops=round(flops / ms / 1e9, 2), stage_ms=st,
                                   full_max_rel_vs_N20=full_rel(P.C_cm),
                                   **errors(P.C_block(rows, cols), ref, absAB)))
                P.release()
                del A, B, Cref, nz, absref
                torch.cuda.empty_cache()


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("leg", choices=["throughput", "shapes", "scale", "accuracy", "sgemm",
                                    "complex", "alpha", "modes"])
    ap.add_argument("--sizes", default="1024,4096,8192,16384")
    ap.add_argument("--phis", default="0.5,1,2,4")
    ap.add_argument("--Ns", default="12,14,16,18,20")
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sample", type=int, default=32, help="sampled block edge (throughput legs)")
    ap.add_argument("--block", type=int, default=512, help="sampled block edge (accuracy leg)")
    ap.add_argument("--acc-size", type=int, default=8192)
    ap.add_argument("--scale-size", type=int, default=4096)
    ap.add_argument("--zNs", default="12,14,16,18", help="N list of the ZGEMM runs")
    ap.add_argument("--cNs", default="5,6,7,8", help="N list of the CGEMM runs")
    ap.add_argument("--alpha-sizes", default="1024,16384")
    ap.add_argument("--alpha-cases", default="0.5,1,2,3,4,ones",
                    help="phi values of Ahat, Bhat, or 'ones' (all-ones matrices)")
    ap.add_argument("--alpha-N", type=int, default=20)
    a = ap.parse_args(argv)
    {"throughput": sweep_throughput, "shapes": sweep_shapes, "scale": sweep_scale,
     "accuracy": sweep_accuracy, "sgemm": sweep_sgemm, "complex": sweep_complex,
     "alpha": sweep_alpha, "modes": sweep_modes}[a.leg](a)


if __name__ == "__main__":
    main()
