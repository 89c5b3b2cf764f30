"""ctypes binding of libstark.so (include/stark.h).

Argument marshalling only: every step of the multiply runs in the library's
HIP kernels.  The functions below carry the C names; tensors are passed as
device pointers (torch is used for device memory and streams only).  If the
library is missing this module raises at import time -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
# STARK_LIBRARY selects another build of the same library (e.g. a different
# leaf-GEMM configuration); by default the in-tree libstark.so.  The tests
# refuse to run with it set, and the benchmark reports the path it loaded.
DEFAULT_LIB_PATH = os.path.join(_HERE, "libstark.so")
LIB_PATH = os.environ.get("STARK_LIBRARY") or DEFAULT_LIB_PATH
HEADER = os.path.join(os.path.dirname(_HERE), "include", "stark.h")

STARK_OK = 0
STARK_PENDING = 1
STARK_EINVAL = -1
STARK_ENOMEM = -2
STARK_EDEVICE = -3
STARK_EBUSY = -4
STARK_ENOTFOUND = -5
STARK_EUNSUPPORTED = -6

STARK_FP32 = 0
STARK_BF16X3 = 1
STARK_BF16X6 = 2
STARK_FP16X3 = 3
STARK_WINOGRAD = 16      # flag: Winograd's variant of the recursion (OR into any precision)
STARK_FUSED = 32         # flag: binary32 leaf operands formed inside the leaf GEMM (where the plan allows it)
STARK_PEEL = 64          # flag: peel every residue n mod (64 * 2^depth) up to 64 (default: up to 16)
STARK_PAD = 128          # flag: never peel; zero-pad to the next multiple of 64 * 2^depth
PRECISIONS = {"fp32": STARK_FP32, "bf16x3": STARK_BF16X3, "bf16x6": STARK_BF16X6, "fp16x3": STARK_FP16X3}
PRECISIONS.update({k + "_winograd": v | STARK_WINOGRAD for k, v in list(PRECISIONS.items())})

STARK_DEPTH_AUTO = -1
STARK_MAX_DEPTH = 8
STARK_PHASE_DIVIDE = 1
STARK_PHASE_LEAF = 2
STARK_PHASE_COMBINE = 4
STARK_PHASE_ALL = 7


class StarkError(RuntimeError):
    def __init__(self, call: str, status: int, message: str):
        super().__init__(f"{call} failed with status {status}: {message}")
        self.status = status


class stark_config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t), ("hbm_budget_bytes", ctypes.c_size_t),
                ("max_slots", ctypes.c_int), ("tuner_cache", ctypes.c_char_p)]


class stark_request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("precision", ctypes.c_int), ("depth", ctypes.c_int),
                ("A", ctypes.c_void_p), ("B", ctypes.c_void_p), ("C", ctypes.c_void_p),
                ("seed", ctypes.c_uint64), ("tag", ctypes.c_uint64)]


class stark_result(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("depth", ctypes.c_int), ("status", ctypes.c_int),
                ("t_submit_us", ctypes.c_double), ("t_admit_us", ctypes.c_double),
                ("t_done_us", ctypes.c_double), ("gpu_ms", ctypes.c_double),
                ("checksum", ctypes.c_double)]


class stark_stats_t(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("throughput_tflops", ctypes.c_double), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("max_inflight_bytes", ctypes.c_double),
                ("max_concurrent", ctypes.c_int)]


class stark_tune_point(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int), ("ms", ctypes.c_double), ("err", ctypes.c_double), ("tile", ctypes.c_int)]


class stark_plan_desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_pad", ctypes.c_int64), ("leaf", ctypes.c_int64),
                ("depth", ctypes.c_int), ("precision", ctypes.c_int), ("planes", ctypes.c_int),
                ("div_a", ctypes.c_int64 * STARK_MAX_DEPTH), ("div_b", ctypes.c_int64 * STARK_MAX_DEPTH),
                ("div_slots", ctypes.c_int * STARK_MAX_DEPTH),
                ("leaf_a", ctypes.c_int64), ("leaf_b", ctypes.c_int64), ("leaf_m", ctypes.c_int64),
                ("comb", ctypes.c_int64 * STARK_MAX_DEPTH),
                ("pad_a", ctypes.c_int64), ("pad_b", ctypes.c_int64), ("bytes", ctypes.c_size_t),
                ("gemm_tile", ctypes.c_int), ("scale", ctypes.c_int64),
                ("divide_bytes", ctypes.c_double), ("split_bytes", ctypes.c_double),
                ("combine_bytes", ctypes.c_double), ("leaf_flops", ctypes.c_double),
                ("mfma_flops", ctypes.c_double), ("variant", ctypes.c_int), ("fused", ctypes.c_int),
                ("peel", ctypes.c_int), ("peel_flops", ctypes.c_double)]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_1811_07325_amd/build.py (or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P, I64, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    sig = {
        "stark_create": ([ctypes.POINTER(P), ctypes.POINTER(stark_config)], I),
        "stark_destroy": ([P], I),
        "stark_workspace_size": ([I64, I, I, ctypes.POINTER(ctypes.c_size_t)], I),
        "stark_max_depth": ([I64], I),
        "stark_model_depth": ([I64, I], I),
        "stark_gemm": ([P, P, P, P, I64, I, I, P], I),
        "stark_gemm_batched": ([P, I, P, P, P, P, I, I, P], I),
        "stark_submit": ([P, ctypes.POINTER(stark_request), ctypes.POINTER(ctypes.c_uint64)], I),
        "stark_poll": ([P, ctypes.c_uint64, ctypes.POINTER(stark_result)], I),
        "stark_stats": ([P, ctypes.POINTER(stark_stats_t)], I),
        "stark_stats_reset": ([P], I),
        "stark_last_error": ([], ctypes.c_char_p),
        "stark_matvec_f64": ([P, P, P, I64, P], I),
        "stark_row_errors": ([P, I64, P, I64, P, P, P], I),
        "stark_generate_normal": ([P, I64, ctypes.c_uint64, P], I),
        "stark_plan_info": ([I64, I, I, ctypes.POINTER(stark_plan_desc)], I),
        "stark_plan_batched": ([P, I, ctypes.POINTER(I64), I, I, ctypes.POINTER(stark_plan_desc)], I),
        "stark_gemm_phases": ([P, P, P, P, I64, I, I, ctypes.c_uint, P], I),
        "stark_workspace": ([P, ctypes.POINTER(P), ctypes.POINTER(ctypes.c_size_t)], I),
        "stark_tune": ([P, P, P, P, I64, I, I, I, ctypes.c_double, ctypes.POINTER(stark_tune_point), I,
                        ctypes.POINTER(I), P], I),
        "stark_gemm_rect": ([P, P, P, P, I64, I64, I64, I, I, P], I),
        "stark_rect_block_edge": ([I64, I64, I64, I], I64),
        "stark_gemm_noalloc": ([P, P, P, I64, I, I, P], I),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = _load()


def header_symbols() -> list[str]:
    """Every function the public header declares."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:stark_status|int|int64_t|const char\*)\s+(stark_\w+)\s*\(", text, re.M)))


def _check(call: str, rc: int, ok=(STARK_OK,)) -> int:
    if rc not in ok:
        raise StarkError(call, rc, stark_last_error())
    return rc


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        return ctypes.c_void_p(0)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    if t is None:
        return ctypes.c_void_p(0)
    if isinstance(t, int):
        return ctypes.c_void_p(t)
    return ctypes.c_void_p(t.data_ptr())


# -- the C calls, same names ---------------------------------------------------

def stark_last_error() -> str:
    return (_lib.stark_last_error() or b"").decode()


def stark_create(device: int = 0, workspace=None, workspace_bytes: int = 0, hbm_budget_bytes: int = 0,
                 max_slots: int = 0, tuner_cache: str | None = None) -> ctypes.c_void_p:
    cfg = stark_config(device, _ptr(workspace).value, workspace_bytes, hbm_budget_bytes, max_slots,
                       tuner_cache.encode() if tuner_cache else None)
    ctx = ctypes.c_void_p()
    _check("stark_create", _lib.stark_create(ctypes.byref(ctx), ctypes.byref(cfg)))
    return ctx


def stark_destroy(ctx) -> None:
    _check("stark_destroy", _lib.stark_destroy(ctx))


def stark_workspace_size(n: int, depth: int, precision: int) -> int:
    b = ctypes.c_size_t()
    _check("stark_workspace_size", _lib.stark_workspace_size(n, depth, precision, ctypes.byref(b)))
    return b.value


def stark_max_depth(n: int) -> int:
    return _lib.stark_max_depth(n)


def stark_model_depth(n: int, precision: int) -> int:
    """Depth used for STARK_DEPTH_AUTO requests without an autotuner record."""
    return _lib.stark_model_depth(n, precision)


def stark_gemm(ctx, A, B, C, n: int, depth: int, precision: int, stream=None) -> None:
    _check("stark_gemm", _lib.stark_gemm(ctx, _ptr(A), _ptr(B), _ptr(C), n, depth, precision, _stream(stream)))


def stark_gemm_batched(ctx, As, Bs, Cs, ns, depth: int, precision: int, stream=None) -> None:
    count = len(ns)
    arrP = ctypes.c_void_p * count
    a = arrP(*[_ptr(x).value for x in As])
    b = arrP(*[_ptr(x).value for x in Bs])
    c = arrP(*[_ptr(x).value for x in Cs])
    nn = (ctypes.c_int64 * count)(*ns)
    _check("stark_gemm_batched", _lib.stark_gemm_batched(ctx, count, a, b, c, nn, depth, precision, _stream(stream)))


def stark_gemm_rect(ctx, A, B, C, m: int, k: int, n: int, depth: int, precision: int, stream=None) -> None:
    """C (m x n) = A (m x k) B (k x n) by square-block partition."""
    _check("stark_gemm_rect", _lib.stark_gemm_rect(ctx, _ptr(A), _ptr(B), _ptr(C), m, k, n, depth, precision,
                                                   _stream(stream)))


def stark_rect_block_edge(m: int, k: int, n: int, depth: int) -> int:
    return int(_lib.stark_rect_block_edge(m, k, n, depth))


def stark_submit(ctx, n: int, precision: int, depth: int = STARK_DEPTH_AUTO, A=None, B=None, C=None,
                 seed: int = 0, tag: int = 0) -> int:
    r = stark_request(n, precision, depth, _ptr(A).value, _ptr(B).value, _ptr(C).value, seed, tag)
    t = ctypes.c_uint64()
    _check("stark_submit", _lib.stark_submit(ctx, ctypes.byref(r), ctypes.byref(t)))
    return t.value


STARK_NOALLOC_SCRATCH_BYTES = 64 << 20


def stark_gemm_noalloc(A, B, C, n: int, depth: int, precision: int, stream=None) -> None:
    _check("stark_gemm_noalloc", _lib.stark_gemm_noalloc(_ptr(A), _ptr(B), _ptr(C), n, depth, precision,
                                                         _stream(stream)))


def stark_gemm_noalloc_status(A, B, C, n: int, depth: int, precision: int, stream=None) -> int:
    """Status of stark_gemm_noalloc without raising."""
    return _lib.stark_gemm_noalloc(_ptr(A), _ptr(B), _ptr(C), n, depth, precision, _stream(stream))


def stark_poll(ctx, ticket: int):
    """None while pending, else the stark_result (raises on a failed request)."""
    out = stark_result()
    rc = _lib.stark_poll(ctx, ticket, ctypes.byref(out))
    if rc == STARK_PENDING:
        return None
    _check("stark_poll", rc)
    return out


def stark_poll_status(ctx, ticket: int):
    """(status, result) without raising."""
    out = stark_result()
    rc = _lib.stark_poll(ctx, ticket, ctypes.byref(out))
    return rc, out


def stark_stats_reset(ctx) -> None:
    _check("stark_stats_reset", _lib.stark_stats_reset(ctx))


def stark_stats(ctx) -> stark_stats_t:
    s = stark_stats_t()
    _check("stark_stats", _lib.stark_stats(ctx, ctypes.byref(s)))
    return s


def stark_matvec_f64(M, x, y, n: int, stream=None) -> None:
    _check("stark_matvec_f64", _lib.stark_matvec_f64(_ptr(M), _ptr(x), _ptr(y), n, _stream(stream)))


def stark_row_errors(C, n: int, rows, nrows: int, ref, out, stream=None) -> None:
    _check("stark_row_errors", _lib.stark_row_errors(_ptr(C), n, _ptr(rows), nrows, _ptr(ref), _ptr(out),
                                                     _stream(stream)))


def stark_generate_normal(X, n: int, seed: int, stream=None) -> None:
    _check("stark_generate_normal", _lib.stark_generate_normal(_ptr(X), n, seed, _stream(stream)))


def stark_plan_info(n: int, depth: int, precision: int) -> stark_plan_desc:
    d = stark_plan_desc()
    _check("stark_plan_info", _lib.stark_plan_info(n, depth, precision, ctypes.byref(d)))
    return d


def stark_plan_batched(ctx, ns, depth: int, precision: int) -> list:
    """Plans stark_gemm_batched gives the problems of edges `ns` (ctx may be
    None: no autotuner records)."""
    count = len(ns)
    out = (stark_plan_desc * count)()
    nn = (ctypes.c_int64 * count)(*ns)
    _check("stark_plan_batched", _lib.stark_plan_batched(ctx, count, nn, depth, precision, out))
    return list(out)


def stark_gemm_phases(ctx, A, B, C, n: int, depth: int, precision: int, mask: int, stream=None) -> None:
    _check("stark_gemm_phases", _lib.stark_gemm_phases(ctx, _ptr(A), _ptr(B), _ptr(C), n, depth, precision,
                                                       mask, _stream(stream)))


def stark_workspace(ctx):
    p = ctypes.c_void_p()
    b = ctypes.c_size_t()
    _check("stark_workspace", _lib.stark_workspace(ctx, ctypes.byref(p), ctypes.byref(b)))
    return p.value, b.value


def stark_tune(ctx, A, B, C, n: int, precision: int, min_depth: int, max_depth: int, tol: float = 0.0,
               stream=None):
    """Autotune; returns the list of (depth, ms, err, tile) points measured."""
    cap = 64
    pts = (stark_tune_point * cap)()
    cnt = ctypes.c_int()
    _check("stark_tune", _lib.stark_tune(ctx, _ptr(A), _ptr(B), _ptr(C), n, precision, min_depth, max_depth, tol,
                                         pts, cap, ctypes.byref(cnt), _stream(stream)))
    return [(pts[i].depth, pts[i].ms, pts[i].err, pts[i].tile) for i in range(min(cnt.value, cap))]


def raw_call(name: str, *args) -> int:
    """Call an exported function and return its raw status (error-path tests)."""
    return getattr(_lib, name)(*args)
