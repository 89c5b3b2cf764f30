"""Accuracy of the FP16X3 leaf precision away from well-scaled inputs,
through the C ABI.

FP16X3 scales each whole matrix by one power of two (from its largest
magnitude) before splitting leaf operands into two binary16 terms, so an
entry 2^-k below the largest magnitude of its matrix keeps about
min(22, 38 - depth - k) significant bits (binary16 subnormals below that).

* rows of A and columns of B scaled by 2^0 .. 2^-20: at depth 0 every row and
  every column keeps the binary32-level accuracy the header states; at
  depth 2 Strassen's recursion adds rows (and columns) of different scales,
  so a small row loses accuracy in any leaf precision -- FP16X3 is then held
  next to FP32 at the same depth;
* a matrix whose largest magnitude is near 2^-113: the scale exponent is
  capped so that it stays a finite binary32, and the product is finite and
  accurate.
"""
import numpy as np
import pytest

import oracle
from paper_1811_07325_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def S():
    from paper_1811_07325_amd import stark
    return stark


@pytest.fixture(scope="module")
def ctx(S):
    c = S.stark_create(0)
    yield c
    S.stark_destroy(c)


def gemm(S, ctx, A, B, depth, prec):
    n = A.shape[0]
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dC = torch.full((n, n), float("nan"), dtype=torch.float32, device="cuda")
    S.stark_gemm(ctx, dA, dB, dC, n, depth, prec, None)
    torch.cuda.synchronize()
    return dC.cpu().numpy()


def scaled_inputs(n):
    """A with row r scaled by 2^-(r mod 21), B with column c by 2^-(c mod 21)."""
    k = np.arange(n) % 21
    A = (inputs.uniform(n, 40) * (2.0 ** -k)[:, None]).astype(np.float32)
    B = (inputs.uniform(n, 41) * (2.0 ** -k)[None, :]).astype(np.float32)
    return A, B, k


def per_scale_errors(C, exact, k):
    """Largest relative Frobenius error over the rows, and over the columns,
    of each scale class 2^-s, s = 0..20."""
    d = C.astype(np.float64) - exact
    er = np.sqrt((d * d).sum(1) / (exact * exact).sum(1))
    ec = np.sqrt((d * d).sum(0) / (exact * exact).sum(0))
    return np.array([max(er[k == s].max(), ec[k == s].max()) for s in range(21)])


def test_fp16x3_rows_and_columns_of_many_scales_classical(S, ctx):
    n = 1000
    A, B, k = scaled_inputs(n)
    exact = oracle.gemm_f64(A, B)
    C = gemm(S, ctx, A, B, 0, S.STARK_FP16X3)
    e = per_scale_errors(C, exact, k)
    print("fp16x3 depth 0, worst row/column error per scale 2^-s:", " ".join(f"{x:.1e}" for x in e))
    # s <= 20: at least 18 significant bits per operand (38 - 0 - 20)
    assert np.all(e <= 1e-5)
    # same arithmetic as the oracle's model (exact leaf sums, binary32 result)
    model = oracle.strassen_model_f32(A, B, 0, "fp16x3", S.stark_plan_info(n, 0, S.STARK_FP16X3).n_pad)
    assert oracle.rel_frobenius(C, model) <= 4 * 2.0 ** -24 * np.sqrt(1024)


def test_fp16x3_rows_and_columns_of_many_scales_strassen(S, ctx):
    n, depth = 1000, 2
    A, B, k = scaled_inputs(n)
    exact = oracle.gemm_f64(A, B)
    e16 = per_scale_errors(gemm(S, ctx, A, B, depth, S.STARK_FP16X3), exact, k)
    e32 = per_scale_errors(gemm(S, ctx, A, B, depth, S.STARK_FP32), exact, k)
    print("depth 2 worst row/column error per scale, fp16x3:", " ".join(f"{x:.1e}" for x in e16))
    print("depth 2 worst row/column error per scale, fp32:  ", " ".join(f"{x:.1e}" for x in e32))
    # the rows of the largest scales keep the binary32 level in both precisions
    assert np.all(e16[:4] <= 1e-5) and np.all(e32[:4] <= 1e-5)
    # smaller rows mix (through the operand sums) with rows up to 2^8 larger
    # (row r and r + 512 of the padded 1024-row matrix): Strassen's own
    # cancellation dominates and FP16X3 stays within a small factor of FP32
    assert np.all(e16 <= 4 * e32 + 5e-6)


@pytest.mark.parametrize("prec", ["fp16x3", "fp16x3_winograd"])
def test_fp16x3_tiny_matrix_scale_exponent_capped(S, ctx, prec):
    """max|A| about 2^-120: the exponent 14 - depth - E would exceed 127;
    capped at 127 the operands stay finite, padding zeros stay zeros and the
    product keeps its accuracy (n = 1000 is padded to 1024)."""
    n, depth = 1000, 2
    A = (inputs.uniform(n, 42) * 2.0 ** -120).astype(np.float32)
    B = inputs.uniform(n, 43)
    assert np.all(np.abs(A[A != 0]) >= 2.0 ** -149)
    C = gemm(S, ctx, A, B, depth, S.PRECISIONS[prec])
    assert np.all(np.isfinite(C))
    variant = "winograd" if prec.endswith("_winograd") else "strassen"
    err = oracle.rel_frobenius(C, oracle.gemm_f64(A, B))
    model = oracle.strassen_model_f32(A, B, depth, "fp16x3", S.stark_plan_info(n, depth, S.PRECISIONS[prec]).n_pad,
                                      variant)
    print(f"{prec} tiny A: rel_frob={err:.3e} vs model {oracle.rel_frobenius(C, model):.3e}")
    assert err <= 1e-5
    assert oracle.rel_frobenius(C, model) <= 4 * 2.0 ** -24 * np.sqrt(256) * 2 ** depth
