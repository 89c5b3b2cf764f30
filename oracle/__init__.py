"""Stark CPU oracle -- test infrastructure only.

Plain FP64 CPU statements of what the Strassen hot path computes (Algorithm 1,
Section III-A; divide / leaf / combine phases of Section III-C).  The C code in
``oracle.c`` does the arithmetic; this module only builds it with gcc and
marshals numpy arrays.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The GPU library (``paper_1811_07325_amd``) never imports it, and
this package never imports that one.

Pins (tests/test_oracle.py): brute force on small integers for every n <= 16
and every depth, the 2x2 worked example of Algorithm 1, exact identities
(A*I, I*B, 0*B, sign and power-of-two scaling), the structural counts of
Section III-C-1 (7^k leaves, 18 additions per node, 4/2/2/4 quadrant uses) and
the double-precision classical loop against numpy's BLAS matmul.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain IEEE, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Counts(ctypes.Structure):
    """Structural counters of one Strassen run (see oracle.c)."""
    _fields_ = [
        ("leaf_products", ctypes.c_int64),
        ("internal_nodes", ctypes.c_int64),
        ("block_additions", ctypes.c_int64),
        ("uses_a", ctypes.c_int64 * 4),
        ("uses_b", ctypes.c_int64 * 4),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    lib.oracle_gemm_f64.argtypes = [P, P, P, I64]
    lib.oracle_gemm_i64.argtypes = [P, P, P, I64]
    lib.oracle_gemm_rect_f64.argtypes = [P, P, P, I64, I64, I64]
    lib.oracle_rows_f64.argtypes = [P, P, I64, P, I64, P]
    lib.oracle_gemv_f64.argtypes = [P, P, P, I64]
    lib.oracle_strassen_f64.argtypes = [P, P, P, I64, ctypes.c_int, I64, ctypes.POINTER(Counts)]
    lib.oracle_strassen_f64.restype = ctypes.c_int
    lib.oracle_divide_f32.argtypes = [P, I64, P, I64, I64, P, P]
    lib.oracle_combine_f32.argtypes = [P, I64, P, I64]
    lib.oracle_split_bf16.argtypes = [P, I64, ctypes.c_int, P]
    lib.oracle_set_mutation.argtypes = [ctypes.c_int]
    lib.oracle_strassen_model_f32.argtypes = [P, P, P, I64, ctypes.c_int, I64, ctypes.c_int]
    lib.oracle_strassen_model_f32.restype = ctypes.c_int
    lib.oracle_model_f32.argtypes = [P, P, P, I64, ctypes.c_int, I64, ctypes.c_int, ctypes.c_int]
    lib.oracle_model_f32.restype = ctypes.c_int
    lib.oracle_peel_model_f32.argtypes = [P, P, P, I64, I64, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.oracle_peel_model_f32.restype = ctypes.c_int
    lib.oracle_winograd_f64.argtypes = [P, P, P, I64, ctypes.c_int, I64, ctypes.POINTER(Counts)]
    lib.oracle_winograd_f64.restype = ctypes.c_int
    lib.oracle_divide_f32_w.argtypes = [P, I64, P, I64, I64, P, P]
    lib.oracle_combine_f32_w.argtypes = [P, I64, P, I64]
    lib.oracle_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_f16_scale_exp.argtypes = [P, I64, ctypes.c_int]
    lib.oracle_f16_scale_exp.restype = ctypes.c_int
    lib.oracle_split_f16.argtypes = [P, I64, ctypes.c_int, P]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _f64(a) -> np.ndarray:
    """Exact widening of a float32 (or any real) array to contiguous float64."""
    return np.ascontiguousarray(np.asarray(a), dtype=np.float64)


def gemm_f64(A, B) -> np.ndarray:
    """Classical product in FP64: C[i][j] = sum_t A[i][t] B[t][j]."""
    A, B = _f64(A), _f64(B)
    n = A.shape[0]
    assert A.shape == (n, n) and B.shape == (n, n)
    C = np.empty((n, n), dtype=np.float64)
    _load().oracle_gemm_f64(_ptr(A), _ptr(B), _ptr(C), n)
    return C


def gemm_i64(A, B) -> np.ndarray:
    """Classical product in exact 64-bit integer arithmetic (brute force)."""
    A = np.ascontiguousarray(A, dtype=np.int64)
    B = np.ascontiguousarray(B, dtype=np.int64)
    n = A.shape[0]
    C = np.empty((n, n), dtype=np.int64)
    _load().oracle_gemm_i64(_ptr(A), _ptr(B), _ptr(C), n)
    return C


def rows_f64(A, B, rows) -> np.ndarray:
    """Rows `rows` of the classical FP64 product (same loop order as gemm_f64)."""
    A, B = _f64(A), _f64(B)
    n = A.shape[0]
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    assert rows.min() >= 0 and rows.max() < n
    out = np.empty((rows.size, n), dtype=np.float64)
    _load().oracle_rows_f64(_ptr(A), _ptr(B), n, _ptr(rows), rows.size, _ptr(out))
    return out


def gemv_f64(M, x) -> np.ndarray:
    """y = M x in FP64."""
    M, x = _f64(M), _f64(x)
    n = M.shape[0]
    y = np.empty(n, dtype=np.float64)
    _load().oracle_gemv_f64(_ptr(M), _ptr(x), _ptr(y), n)
    return y


def padded_size(n: int, depth: int, granule: int = 1) -> int:
    """Smallest multiple of 2^depth * granule that is >= n."""
    q = (1 << depth) * granule
    return -(-n // q) * q


def strassen_f64(A, B, depth: int, n_pad: int | None = None, with_counts: bool = False):
    """C = A B by `depth` levels of Algorithm 1 on zero-padded operands, FP64."""
    A, B = _f64(A), _f64(B)
    n = A.shape[0]
    assert A.shape == (n, n) and B.shape == (n, n)
    if n_pad is None:
        n_pad = padded_size(n, depth)
    C = np.empty((n, n), dtype=np.float64)
    cnt = Counts()
    rc = _load().oracle_strassen_f64(_ptr(A), _ptr(B), _ptr(C), n, depth, n_pad, ctypes.byref(cnt))
    if rc != 0:
        raise ValueError(f"oracle_strassen_f64: bad arguments n={n} depth={depth} n_pad={n_pad}")
    if with_counts:
        return C, cnt
    return C


VARIANTS = ("strassen", "winograd")


def winograd_f64(A, B, depth: int, n_pad: int | None = None, with_counts: bool = False):
    """C = A B by `depth` levels of Winograd's variant (15 additions per
    node) on zero-padded operands, FP64."""
    A, B = _f64(A), _f64(B)
    n = A.shape[0]
    assert A.shape == (n, n) and B.shape == (n, n)
    if n_pad is None:
        n_pad = padded_size(n, depth)
    C = np.empty((n, n), dtype=np.float64)
    cnt = Counts()
    rc = _load().oracle_winograd_f64(_ptr(A), _ptr(B), _ptr(C), n, depth, n_pad, ctypes.byref(cnt))
    if rc != 0:
        raise ValueError(f"oracle_winograd_f64: bad arguments n={n} depth={depth} n_pad={n_pad}")
    if with_counts:
        return C, cnt
    return C


def divide_f32(X, Y, variant: str = "strassen"):
    """Operand pairs (S_i, T_i), i = 1..7, of one node in binary32 -> (7,h,h) x2."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    Y = np.ascontiguousarray(Y, dtype=np.float32)
    m = X.shape[0]
    assert X.shape == (m, m) and Y.shape == (m, m) and m % 2 == 0
    h = m // 2
    S = np.empty((7, h, h), dtype=np.float32)
    T = np.empty((7, h, h), dtype=np.float32)
    fn = _load().oracle_divide_f32_w if variant == "winograd" else _load().oracle_divide_f32
    assert variant in VARIANTS
    fn(_ptr(X), m, _ptr(Y), m, m, _ptr(S), _ptr(T))
    return S, T


def combine_f32(M, variant: str = "strassen") -> np.ndarray:
    """C (2h x 2h) from the seven products M (7,h,h) in binary32."""
    M = np.ascontiguousarray(M, dtype=np.float32)
    assert M.ndim == 3 and M.shape[0] == 7 and M.shape[1] == M.shape[2]
    assert variant in VARIANTS
    h = M.shape[1]
    C = np.empty((2 * h, 2 * h), dtype=np.float32)
    fn = _load().oracle_combine_f32_w if variant == "winograd" else _load().oracle_combine_f32
    fn(_ptr(M), h, _ptr(C), 2 * h)
    return C


def split_bf16(x, terms: int = 2) -> np.ndarray:
    """bfloat16 split planes (terms, *x.shape) as uint16 bit patterns (RNE)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    assert terms in (2, 3)
    out = np.empty((terms,) + x.shape, dtype=np.uint16)
    _load().oracle_split_bf16(_ptr(x), x.size, terms, _ptr(out))
    return out


def bf16_bits_to_f32(b) -> np.ndarray:
    """Exact value of bfloat16 bit patterns as float32."""
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


MODEL_MODES = {"fp32": 0, "bf16x3": 2, "bf16x6": 3, "fp16x3": 4}


def f16_scale_exp(X, depth: int) -> int:
    """Power-of-two exponent that scales the FP16X3 leaf operands of X below 2^14."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    return int(_load().oracle_f16_scale_exp(_ptr(X), X.size, depth))


def split_f16(x, e: int) -> np.ndarray:
    """binary16 split of x * 2^e: planes (2, *x.shape) as binary32 values."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty((2,) + x.shape, dtype=np.float32)
    _load().oracle_split_f16(_ptr(x), x.size, e, _ptr(out))
    return out


def strassen_model_f32(A, B, depth: int, mode: str, n_pad: int | None = None,
                       variant: str = "strassen") -> np.ndarray:
    """Arithmetic model of the GPU path: binary32 divide/combine (Algorithm 1
    or Winograd's variant), leaf products exact in binary64 from the leaf
    operands as seen by `mode` ("fp32", "bf16x3", "bf16x6", "fp16x3"),
    rounded to binary32.  Returns float32 n x n."""
    A = np.ascontiguousarray(A, dtype=np.float32)
    B = np.ascontiguousarray(B, dtype=np.float32)
    n = A.shape[0]
    if n_pad is None:
        n_pad = padded_size(n, depth)
    C = np.empty((n, n), dtype=np.float32)
    rc = _load().oracle_model_f32(_ptr(A), _ptr(B), _ptr(C), n, depth, n_pad, MODEL_MODES[mode],
                                  VARIANTS.index(variant))
    if rc != 0:
        raise ValueError("oracle_strassen_model_f32: bad arguments")
    return C


def peel_model_f32(A, B, depth: int, mode: str, r: int, variant: str = "strassen") -> np.ndarray:
    """Arithmetic model of a peeled multiply: the recursion on the leading
    (n - r) x (n - r) blocks of A and B by the model of the square path
    (unpadded), every core output plus the r products through A's last r
    columns and B's last r rows, and the border rows and columns as whole
    inner products, each of these sums exact in binary64 and rounded once.
    Returns float32 n x n."""
    A = np.ascontiguousarray(A, dtype=np.float32)
    B = np.ascontiguousarray(B, dtype=np.float32)
    n = A.shape[0]
    C = np.empty((n, n), dtype=np.float32)
    rc = _load().oracle_peel_model_f32(_ptr(A), _ptr(B), _ptr(C), n, n - r, depth, MODEL_MODES[mode],
                                       VARIANTS.index(variant))
    if rc != 0:
        raise ValueError("oracle_peel_model_f32: bad arguments")
    return C


def gemm_rect_f64(A, B) -> np.ndarray:
    """Rectangular classical product in FP64: C (m x n) = A (m x k) B (k x n)."""
    A, B = _f64(A), _f64(B)
    m, k = A.shape
    k2, n = B.shape
    assert k == k2
    C = np.empty((m, n), dtype=np.float64)
    _load().oracle_gemm_rect_f64(_ptr(A), _ptr(B), _ptr(C), m, k, n)
    return C


def rect_blocks(m: int, k: int, n: int, s: int):
    """Block counts of the square partition of C (m x n) = A (m x k) B (k x n)
    into s x s blocks: (row blocks, inner blocks, column blocks)."""
    return -(-m // s), -(-k // s), -(-n // s)


def rect_model_f32(A, B, s: int, depth: int, mode: str, variant: str = "strassen",
                   n_pad: int | None = None) -> np.ndarray:
    """Rectangular product by partitioning into square problems (the paper
    defers sizes other than 2^p to partitioning, Section III-A): A and B are
    zero-padded to whole s x s blocks, C_ij = sum over p of A_ip B_pj, every
    block product by the arithmetic model of the square path (padded to
    n_pad), the sum over p in binary32 in ascending p, then cropped."""
    A = np.ascontiguousarray(A, dtype=np.float32)
    B = np.ascontiguousarray(B, dtype=np.float32)
    m, k = A.shape
    _, n = B.shape
    MB, KB, NB = rect_blocks(m, k, n, s)
    Ap = np.zeros((MB * s, KB * s), np.float32); Ap[:m, :k] = A
    Bp = np.zeros((KB * s, NB * s), np.float32); Bp[:k, :n] = B
    C = np.empty((MB * s, NB * s), np.float32)
    for i in range(MB):
        for j in range(NB):
            acc = None
            for p in range(KB):
                blk = strassen_model_f32(Ap[i * s:(i + 1) * s, p * s:(p + 1) * s],
                                         Bp[p * s:(p + 1) * s, j * s:(j + 1) * s], depth, mode, n_pad, variant)
                acc = blk if acc is None else (acc + blk).astype(np.float32)
            C[i * s:(i + 1) * s, j * s:(j + 1) * s] = acc
    return C[:m, :n]


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_load().oracle_threads())


def set_threads(count: int) -> None:
    """Threads of the oracle's parallel loops from here on (count >= 1)."""
    _load().oracle_set_threads(int(count))


def set_mutation(m: int) -> None:
    """Test hook: plant a known mistake in the oracle (0 = none)."""
    _load().oracle_set_mutation(int(m))


def rel_frobenius(C, ref) -> float:
    """||C - ref||_F / ||ref||_F in FP64."""
    C, ref = _f64(C), _f64(ref)
    d = C - ref
    return float(np.sqrt(np.sum(d * d)) / np.sqrt(np.sum(ref * ref)))


def max_abs(C, ref) -> float:
    return float(np.max(np.abs(_f64(C) - _f64(ref))))


def freivalds_rel(A, B, C, x) -> float:
    """||C x - A (B x)|| / ||A (B x)|| in FP64 (Freivalds 1977, Gaussian x).

    For Gaussian x, E||E x||^2 = ||E||_F^2, so this estimates the relative
    Frobenius error of C."""
    Bx = gemv_f64(B, x)
    ABx = gemv_f64(A, Bx)
    Cx = gemv_f64(C, x)
    return float(np.linalg.norm(Cx - ABx) / np.linalg.norm(ABx))
