"""Python binding of libozaki2 (include/ozaki2.h): argument marshalling only.

Every function named ``ozaki2_*`` calls the C entry point of the same name;
pointer arguments accept a torch tensor (its ``data_ptr()``) or an int.  All
computation happens in the HIP library; if it is not built or cannot be
loaded, the first call raises.

``dgemm``/``sgemm``/``zgemm``/``cgemm`` are conveniences for row-major torch
tensors on the GPU: a row-major m x k tensor is the column-major k x m
matrix, so C = A B is computed as the column-major C^T = B^T A^T by swapping
the operands (a plain transpose, also for complex tensors).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libozaki2.so")

MODE_REVISED, MODE_ORIGINAL, MODE_ACCURATE, MODE_EXACT = 0, 1, 2, 3
_MODES = {"revised": 0, "original": 1, "fast": 1, "accurate": 2, "exact": 3}
NUM_STAGES = 5
STAGE_NAMES = ("norms_exponents", "convert_split", "int8_gemm", "crt_unscale", "other")

_lib = None

_c_i64, _c_int, _vp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p


class Oz2Problem(ctypes.Structure):
    """struct oz2_problem of include/ozaki2.h."""
    _fields_ = [("m", _c_i64), ("n", _c_i64), ("k", _c_i64), ("A", _vp), ("lda", _c_i64),
                ("B", _vp), ("ldb", _c_i64), ("C", _vp), ("ldc", _c_i64), ("N", _c_int),
                ("N_used", _c_int)]

_SIGS = {
    "ozaki2_dgemm": ([_c_i64] * 3 + [_vp, _c_i64, _vp, _c_i64, _vp, _c_i64, _c_int, _c_int], _c_int),
    "ozaki2_dgemm_noalloc": ([_c_i64] * 3 + [_vp, _c_i64, _vp, _c_i64, _vp, _c_i64, _c_int, _c_int],
                             _c_int),
    "ozaki2_sgemm": ([_c_i64] * 3 + [_vp, _c_i64, _vp, _c_i64, _vp, _c_i64, _c_int, _c_int], _c_int),
    "ozaki2_zgemm": ([_c_i64] * 3 + [_vp, _c_i64, _vp, _c_i64, _vp, _c_i64, _c_int, _c_int], _c_int),
    "ozaki2_cgemm": ([_c_i64] * 3 + [_vp, _c_i64, _vp, _c_i64, _vp, _c_i64, _c_int, _c_int], _c_int),
    "ozaki2_zgemm_workspace_size": ([_c_i64] * 3 + [_c_int, _c_int, ctypes.POINTER(ctypes.c_size_t)],
                                    _c_int),
    "ozaki2_set_stream": ([_vp], _c_int),
    "ozaki2_workspace_size": ([_c_i64] * 3 + [_c_int, _c_int, ctypes.POINTER(ctypes.c_size_t)], _c_int),
    "ozaki2_set_workspace": ([_vp, ctypes.c_size_t], _c_int),
    "ozaki2_set_workspace_policy": ([_c_int], _c_int),
    "ozaki2_get_device_status": ([ctypes.POINTER(_c_int)], _c_int),
    "ozaki2_status_string": ([_c_int], ctypes.c_char_p),
    "ozaki2_version": ([], ctypes.c_char_p),
    "ozaki2_finalize": ([], _c_int),
    "ozaki2_query_constants": ([_c_int, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_float),
                                ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                ctypes.POINTER(ctypes.c_double)], _c_int),
    "ozaki2_set_timing": ([_c_int], _c_int),
    "ozaki2_set_tile": ([_c_int], _c_int),
    "ozaki2_get_tile": ([_c_i64] * 3 + [_c_int, ctypes.POINTER(_c_int)], _c_int),
    "ozaki2_get_stage_times": ([ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_c_int)], _c_int),
    "ozaki2_debug_stages": ([_c_i64] * 3 + [_vp, _c_i64, _vp, _c_i64, _c_int, _c_int, _c_int]
                            + [_vp] * 7, _c_int),
    "ozaki2_debug_log2f": ([_vp, _vp, _c_i64], _c_int),
    "ozaki2_dgemm_batched": ([_c_int, ctypes.POINTER(Oz2Problem), _c_int, ctypes.c_double,
                              ctypes.POINTER(_c_int)], _c_int),
    "ozaki2_dgemm_batched_workspace_size": ([_c_int, ctypes.POINTER(Oz2Problem), _c_int,
                                             ctypes.POINTER(ctypes.c_size_t)], _c_int),
    "ozaki2_autotune_N": ([_c_i64, ctypes.c_double, ctypes.c_double, ctypes.POINTER(_c_int)], _c_int),
    "ozaki2_estimate_phi": ([_c_i64, _c_i64, _vp, _c_i64, _c_int, ctypes.POINTER(ctypes.c_double)],
                            _c_int),
}


class Ozaki2Error(RuntimeError):
    def __init__(self, fn, code):
        self.code = code
        msg = lib().ozaki2_status_string(code).decode()
        super().__init__(f"{fn} returned {code}: {msg}")


def lib():
    """The loaded libozaki2 (raises if the HIP library is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libozaki2.so is not built ({LIB_PATH}); run "
                               "python -m paper_2606_29129_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _check(fn, rc):
    if rc != 0:
        raise Ozaki2Error(fn, rc)
    return rc


# --- C entry points (same names) -------------------------------------------

def ozaki2_dgemm(m, n, k, A, lda, B, ldb, C, ldc, N, mode=MODE_REVISED):
    return lib().ozaki2_dgemm(m, n, k, _ptr(A), lda, _ptr(B), ldb, _ptr(C), ldc, N, mode)


def ozaki2_dgemm_noalloc(m, n, k, A, lda, B, ldb, C, ldc, N, mode=MODE_REVISED):
    return lib().ozaki2_dgemm_noalloc(m, n, k, _ptr(A), lda, _ptr(B), ldb, _ptr(C), ldc, N, mode)


def ozaki2_sgemm(m, n, k, A, lda, B, ldb, C, ldc, N, mode=MODE_REVISED):
    return lib().ozaki2_sgemm(m, n, k, _ptr(A), lda, _ptr(B), ldb, _ptr(C), ldc, N, mode)


def ozaki2_zgemm(m, n, k, A, lda, B, ldb, C, ldc, N, mode=MODE_REVISED):
    return lib().ozaki2_zgemm(m, n, k, _ptr(A), lda, _ptr(B), ldb, _ptr(C), ldc, N, mode)


def ozaki2_cgemm(m, n, k, A, lda, B, ldb, C, ldc, N, mode=MODE_REVISED):
    return lib().ozaki2_cgemm(m, n, k, _ptr(A), lda, _ptr(B), ldb, _ptr(C), ldc, N, mode)


def ozaki2_zgemm_workspace_size(m, n, k, N, mode=MODE_REVISED):
    b = ctypes.c_size_t(0)
    _check("ozaki2_zgemm_workspace_size",
           lib().ozaki2_zgemm_workspace_size(m, n, k, N, mode, ctypes.byref(b)))
    return b.value


def ozaki2_set_stream(stream):
    """stream: a torch.cuda.Stream, a raw hipStream_t as int, or None."""
    if stream is not None and not isinstance(stream, int):
        stream = stream.cuda_stream
    return lib().ozaki2_set_stream(stream)


def ozaki2_workspace_size(m, n, k, N, mode=MODE_REVISED):
    b = ctypes.c_size_t(0)
    _check("ozaki2_workspace_size", lib().ozaki2_workspace_size(m, n, k, N, mode, ctypes.byref(b)))
    return b.value


def ozaki2_set_workspace(ptr, nbytes):
    return lib().ozaki2_set_workspace(_ptr(ptr), nbytes)


WORKSPACE_CALLER, WORKSPACE_LIBRARY = 0, 1


def ozaki2_set_workspace_policy(policy):
    return lib().ozaki2_set_workspace_policy(policy)


def ozaki2_get_device_status():
    s = ctypes.c_int(0)
    _check("ozaki2_get_device_status", lib().ozaki2_get_device_status(ctypes.byref(s)))
    return s.value


def ozaki2_status_string(code):
    return lib().ozaki2_status_string(code).decode()


def ozaki2_version():
    return lib().ozaki2_version().decode()


def ozaki2_finalize():
    return lib().ozaki2_finalize()


def ozaki2_query_constants(N):
    """dict(moduli, p_prime_prop, p_prime_fast, delta, log2_P) as the library
    computes them (host only)."""
    mod = (ctypes.c_int32 * 20)()
    pp, pf, d = ctypes.c_float(), ctypes.c_float(), ctypes.c_float()
    lp = ctypes.c_double()
    _check("ozaki2_query_constants", lib().ozaki2_query_constants(
        N, mod, ctypes.byref(pp), ctypes.byref(pf), ctypes.byref(d), ctypes.byref(lp)))
    return dict(moduli=list(mod[:N]), p_prime_prop=pp.value, p_prime_fast=pf.value,
                delta=d.value, log2_P=lp.value)


TILE_AUTO, TILE_256x256, TILE_128x128, TILE_256x64 = 0, 1, 2, 3


def ozaki2_set_tile(tile):
    return lib().ozaki2_set_tile(tile)


def ozaki2_get_tile(m, n, k, N):
    t = ctypes.c_int(0)
    _check("ozaki2_get_tile", lib().ozaki2_get_tile(m, n, k, N, ctypes.byref(t)))
    return t.value


def ozaki2_set_timing(enable):
    return lib().ozaki2_set_timing(int(bool(enable)))


def ozaki2_get_stage_times():
    ms = (ctypes.c_double * NUM_STAGES)()
    calls = ctypes.c_int(0)
    _check("ozaki2_get_stage_times", lib().ozaki2_get_stage_times(ms, ctypes.byref(calls)))
    return list(ms), calls.value


def ozaki2_debug_stages(m, n, k, A, lda, B, ldb, N, mode, t,
                        eA=None, eB=None, SA=None, SB=None, RA=None, RB=None, Ct=None):
    return lib().ozaki2_debug_stages(m, n, k, _ptr(A), lda, _ptr(B), ldb, N, mode, t,
                                     _ptr(eA), _ptr(eB), _ptr(SA), _ptr(SB), _ptr(RA),
                                     _ptr(RB), _ptr(Ct))


def _problem_array(problems):
    arr = (Oz2Problem * max(1, len(problems)))()
    for i, q in enumerate(problems):
        if isinstance(q, Oz2Problem):
            arr[i] = q
        else:
            m, n, k, A, lda, B, ldb, C, ldc, N = q
            arr[i] = Oz2Problem(m, n, k, _ptr(A), lda, _ptr(B), ldb, _ptr(C), ldc, N, 0)
    return arr


def ozaki2_dgemm_batched_workspace_size(problems, mode=MODE_REVISED):
    """Workspace bytes of a batch (problems as for ozaki2_dgemm_batched)."""
    arr = _problem_array(problems)
    b = ctypes.c_size_t(0)
    _check("ozaki2_dgemm_batched_workspace_size",
           lib().ozaki2_dgemm_batched_workspace_size(len(problems), arr, mode, ctypes.byref(b)))
    return b.value


def ozaki2_dgemm_batched(problems, mode=MODE_REVISED, target=0.0):
    """problems: a sequence of Oz2Problem (or of tuples with its fields up to
    N, pointers as tensors or ints; N = 0 lets the library pick N for the
    target).  Returns (rc, bad_index, [N_used per problem])."""
    arr = _problem_array(problems)
    bad = ctypes.c_int(-1)
    rc = lib().ozaki2_dgemm_batched(len(problems), arr, mode, float(target), ctypes.byref(bad))
    return rc, bad.value, [arr[i].N_used for i in range(len(problems))]


def ozaki2_autotune_N(k, phi, target):
    N = ctypes.c_int(0)
    _check("ozaki2_autotune_N", lib().ozaki2_autotune_N(k, float(phi), float(target),
                                                          ctypes.byref(N)))
    return N.value


def ozaki2_estimate_phi(rows, cols, X, ld, vectors):
    phi = ctypes.c_double(0.0)
    _check("ozaki2_estimate_phi", lib().ozaki2_estimate_phi(rows, cols, _ptr(X), ld, vectors,
                                                              ctypes.byref(phi)))
    return phi.value


def ozaki2_debug_log2f(x, y, n):
    return lib().ozaki2_debug_log2f(_ptr(x), _ptr(y), n)


# --- torch conveniences ------------------------------------------------------

_workspaces = {}   # device index -> (uint8 tensor, 256-aligned address, usable bytes)


def ensure_workspace(nbytes, device=None):
    """Point the library at a workspace of at least ``nbytes`` on ``device``
    (default: the current one): a uint8 torch tensor cached per device and
    replaced by a larger one when a call needs more.  The library itself
    never allocates device memory (its default workspace policy); this is
    where the conveniences below get theirs.  Returns the address."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    cur = _workspaces.get(idx)
    if cur is None or cur[2] < nbytes:
        t = torch.empty(max(int(nbytes), 1) + 256, dtype=torch.uint8, device=dev)
        cur = (t, (t.data_ptr() + 255) // 256 * 256, max(int(nbytes), 1))
        _workspaces[idx] = cur
    # the tensor is used on the current stream from here on
    cur[0].record_stream(torch.cuda.current_stream(dev))
    _check("ozaki2_set_workspace", ozaki2_set_workspace(cur[1], cur[2]))
    return cur[1]


def release_workspaces():
    """Unset the library's workspace and drop the cached tensors."""
    ozaki2_set_workspace(None, 0)
    _workspaces.clear()

def _mode(mode):
    return _MODES[mode] if isinstance(mode, str) else int(mode)


def _bind_current_stream(torch):
    ozaki2_set_stream(torch.cuda.current_stream().cuda_stream)


def dgemm(A, B, N=14, mode="revised", out=None):
    """C = A @ B for row-major float64 CUDA tensors A (m x k), B (k x n)."""
    import torch
    if A.dtype != torch.float64 or B.dtype != torch.float64:
        raise TypeError("dgemm needs float64 tensors")
    return _gemm(A, B, N, mode, out, ozaki2_dgemm)


def sgemm(A, B, N=7, mode="revised", out=None):
    """C = A @ B for row-major float32 CUDA tensors A (m x k), B (k x n)."""
    import torch
    if A.dtype != torch.float32 or B.dtype != torch.float32:
        raise TypeError("sgemm needs float32 tensors")
    return _gemm(A, B, N, mode, out, ozaki2_sgemm)


def zgemm(A, B, N=14, mode="revised", out=None):
    """C = A @ B for row-major complex128 CUDA tensors A (m x k), B (k x n)."""
    import torch
    if A.dtype != torch.complex128 or B.dtype != torch.complex128:
        raise TypeError("zgemm needs complex128 tensors")
    return _gemm(A, B, N, mode, out, ozaki2_zgemm)


def cgemm(A, B, N=7, mode="revised", out=None):
    """C = A @ B for row-major complex64 CUDA tensors A (m x k), B (k x n)."""
    import torch
    if A.dtype != torch.complex64 or B.dtype != torch.complex64:
        raise TypeError("cgemm needs complex64 tensors")
    return _gemm(A, B, N, mode, out, ozaki2_cgemm)


def _gemm(A, B, N, mode, out, fn):
    import torch
    if A.dim() != 2 or B.dim() != 2 or A.shape[1] != B.shape[0]:
        raise ValueError("shapes do not compose")
    if not (A.is_cuda and B.is_cuda):
        raise ValueError("tensors must be on the GPU")
    A = A.contiguous()
    B = B.contiguous()
    m, k = A.shape
    n = B.shape[1]
    C = out if out is not None else torch.empty((m, n), dtype=A.dtype, device=A.device)
    if not C.is_contiguous() or C.shape != (m, n):
        raise ValueError("out must be a contiguous m x n tensor")
    _bind_current_stream(torch)
    size_fn = ozaki2_zgemm_workspace_size if fn in (ozaki2_zgemm, ozaki2_cgemm) else \
        ozaki2_workspace_size
    ensure_workspace(size_fn(n, m, k, N, _mode(mode)), A.device)
    # Column-major view: C^T (n x m, ld n) = B^T (n x k, ld n) * A^T (k x m, ld k).
    rc = fn(n, m, k, B, max(1, n), A, max(1, k), C, max(1, n), N, _mode(mode))
    _check(fn.__name__, rc)
    return C


def dgemm_batched(pairs, N=0, mode="revised", target=None, return_N=False):
    """C_i = A_i @ B_i for a list of row-major float64 CUDA tensor pairs, in one
    batched call.  N is an int or a list with one moduli count per problem;
    0 lets the library pick N for the max relative error ``target``.  With
    ``return_N`` also returns the N used per problem."""
    import torch
    Ns = [N] * len(pairs) if isinstance(N, int) else list(N)
    outs, probs = [], []
    for (A, B), Ni in zip(pairs, Ns):
        A = A.contiguous()
        B = B.contiguous()
        m, k = A.shape
        n = B.shape[1]
        C = torch.empty((m, n), dtype=torch.float64, device=A.device)
        outs.append((A, B, C))
        # row-major C = A B is column-major C^T = B^T A^T
        probs.append((n, m, k, B, max(1, n), A, max(1, k), C, max(1, n), Ni))
    _bind_current_stream(torch)
    if outs:
        ensure_workspace(ozaki2_dgemm_batched_workspace_size(probs, _mode(mode)),
                         outs[0][0].device)
    rc, bad, used = ozaki2_dgemm_batched(probs, _mode(mode), 0.0 if target is None else target)
    if rc:
        raise Ozaki2Error(f"ozaki2_dgemm_batched (problem {bad})", rc)
    Cs = [c for _, _, c in outs]
    return (Cs, used) if return_N else Cs
