"""Pins for the oracle's arithmetic model of the GPU path (CPU only)."""
import os

import numpy as np
import pytest

import oracle
from paper_1811_07325_amd import inputs


@pytest.mark.parametrize("mode", ["fp32", "bf16x3", "bf16x6", "fp16x3"])
@pytest.mark.parametrize("n,depth", [(16, 0), (16, 2), (13, 1), (40, 3)])
def test_model_exact_on_small_integers(mode, n, depth):
    A = inputs.integers(n, 1)
    B = inputs.integers(n, 2)
    C = oracle.strassen_model_f32(A, B, depth, mode)
    assert np.array_equal(C.astype(np.int64), A.astype(np.int64) @ B.astype(np.int64))


@pytest.mark.parametrize("mode", ["fp32", "bf16x3", "bf16x6", "fp16x3"])
@pytest.mark.parametrize("n,depth,r", [(17, 2, 1), (23, 1, 7), (71, 3, 7), (127, 2, 63), (9, 0, 1), (50, 1, 2)])
def test_peel_model_exact_on_small_integers(mode, n, depth, r):
    """Core by the recursion, border and fix-up classical: on integers the
    peeled model is the exact product (a dropped fix-up term, a border
    computed over the core only or a wrong core offset would not be)."""
    A = inputs.integers(n, 3)
    B = inputs.integers(n, 4)
    C = oracle.peel_model_f32(A, B, depth, mode, r)
    assert np.array_equal(C.astype(np.int64), A.astype(np.int64) @ B.astype(np.int64))


def test_peel_model_without_residue_is_the_square_model():
    A = inputs.uniform(64, 5)
    B = inputs.uniform(64, 6)
    for mode in ("fp32", "bf16x3", "fp16x3"):
        assert np.array_equal(oracle.peel_model_f32(A, B, 2, mode, 0), oracle.strassen_model_f32(A, B, 2, mode, 64))


def test_peel_model_float_error_is_the_cores():
    """On floats the peeled model sits within binary32 rounding of the exact
    product: its border is exact rounded once, its core the square model's."""
    A = inputs.uniform(131, 7)
    B = inputs.uniform(131, 8)
    exact = oracle.gemm_f64(A, B)
    C = oracle.peel_model_f32(A, B, 2, "fp32", 3)
    assert oracle.rel_frobenius(C, exact) < 1e-6
    # border entries: each the rounded exact inner product
    assert np.array_equal(C[128:, :], exact[128:, :].astype(np.float32))
    assert np.array_equal(C[:128, 128:], exact[:128, 128:].astype(np.float32))


def test_model_fp32_depth0_is_rounded_classical():
    A = inputs.uniform(48, 3)
    B = inputs.uniform(48, 4)
    C = oracle.strassen_model_f32(A, B, 0, "fp32")
    assert np.array_equal(C, oracle.gemm_f64(A, B).astype(np.float32))


def test_model_bf16x3_depth0_matches_library_split():
    torch = pytest.importorskip("torch")
    A = inputs.normal(64, 5)
    B = inputs.normal(64, 6)

    def planes(x):
        hi = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
        lo = torch.from_numpy(x - hi).to(torch.bfloat16).to(torch.float32).numpy()
        return hi.astype(np.float64), lo.astype(np.float64)

    ah, al = planes(A)
    bh, bl = planes(B)
    ref = (ah @ bh + ah @ bl + al @ bh).astype(np.float32)
    C = oracle.strassen_model_f32(A, B, 0, "bf16x3")
    assert np.max(np.abs(C - ref) / (np.abs(ref) + 1e-30)) <= 2.0 ** -22


def test_model_split_error_sizes():
    """bf16x6 keeps binary32 accuracy; bf16x3 loses about 8 bits (2^-17 per operand)."""
    A = inputs.normal(64, 7)
    B = inputs.normal(64, 8)
    exact = oracle.gemm_f64(A, B)
    e32 = oracle.rel_frobenius(oracle.strassen_model_f32(A, B, 0, "fp32"), exact)
    e6 = oracle.rel_frobenius(oracle.strassen_model_f32(A, B, 0, "bf16x6"), exact)
    e3 = oracle.rel_frobenius(oracle.strassen_model_f32(A, B, 0, "bf16x3"), exact)
    assert e32 < 1e-7 and e6 < 1e-7
    assert 5e-7 < e3 < 2e-5


def test_philox_known_answers():
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    with open(path) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    for r in rows:
        v = [np.uint64(int(x, 16)) for x in r]
        out = inputs.philox4x32_10(*v[:6])
        assert [int(x) for x in out] == [int(x) for x in v[6:]]


def test_philox_normal_moments():
    """The serving generator's host twin draws normal(0, 1): moments up to
    the fourth (a sum of twelve uniforms would show kurtosis 2.9), the tail
    mass beyond 3 and 4 standard deviations, and Kolmogorov-Smirnov against
    the normal CDF over 2^18 values."""
    from scipy import stats
    x = inputs.philox_normal(512, 11).astype(np.float64).ravel()
    assert abs(x.mean()) < 0.01 and abs(x.var() - 1.0) < 0.01
    assert abs(stats.skew(x)) < 0.03 and abs(stats.kurtosis(x, fisher=False) - 3.0) < 0.05
    for t in (3.0, 4.0):
        expect = 2 * stats.norm.sf(t) * x.size
        assert abs(np.sum(np.abs(x) > t) - expect) < 5 * np.sqrt(expect)
    assert stats.kstest(x, "norm").pvalue > 1e-3
    assert np.all(np.abs(x) <= 6.7)
    # other seeds give other values; the same seed the same ones
    assert not np.array_equal(inputs.philox_normal(64, 11), inputs.philox_normal(64, 12))
    assert np.array_equal(inputs.philox_normal(64, 11), inputs.philox_normal(512, 11).ravel()[:4096].reshape(64, 64))


def test_f16_rounding_matches_library():
    """binary16 rounding of the oracle against numpy's float16 conversion."""
    x = inputs.normal(300, 19).ravel() * np.float32(40)
    x = np.concatenate([x, np.float32([0.0, 65504.0, 65519.0, 1e-7, 6e-8, 2.0 ** -25, 1 + 2.0 ** -11,
                                       1 + 3 * 2.0 ** -11, 1.5 * 2.0 ** -24, 2.5 * 2.0 ** -24, -3.0e-5])])
    planes = oracle.split_f16(x, 0)
    assert np.array_equal(planes[0], x.astype(np.float16).astype(np.float32))
    assert np.array_equal(planes[1], (x - planes[0]).astype(np.float16).astype(np.float32))


def test_f16_scale_exponent():
    A = inputs.normal(64, 20)
    m = float(np.max(np.abs(A)))
    E = int(np.frexp(m)[1])
    for depth in range(4):
        e = oracle.f16_scale_exp(A, depth)
        assert e == 14 - depth - E
        assert m * 2.0 ** e * 2 ** depth < 2 ** 14
    assert oracle.f16_scale_exp(np.zeros((4, 4), np.float32), 2) == 0


def test_f16_scale_exponent_capped_for_tiny_matrices():
    """The exponent is capped at 127 so that 2^e is a finite binary32; a
    matrix near 2^-120 is then scaled by 2^127 only, its operands stay well
    inside binary16's range and the model's product keeps its accuracy."""
    A = (inputs.uniform(64, 23) * 2.0 ** -120).astype(np.float32)
    B = inputs.uniform(64, 24)
    E = int(np.frexp(float(np.max(np.abs(A))))[1])
    assert 14 - 2 - E > 127
    assert oracle.f16_scale_exp(A, 2) == 127
    assert np.isfinite(np.float32(2.0) ** 127)
    M = oracle.strassen_model_f32(A, B, 2, "fp16x3")
    assert np.all(np.isfinite(M))
    assert oracle.rel_frobenius(M, oracle.gemm_f64(A, B)) < 1e-6


def test_fp16x3_keeps_binary32_accuracy():
    A = inputs.normal(64, 21)
    B = inputs.normal(64, 22)
    exact = oracle.gemm_f64(A, B)
    e16 = oracle.rel_frobenius(oracle.strassen_model_f32(A, B, 0, "fp16x3"), exact)
    e3 = oracle.rel_frobenius(oracle.strassen_model_f32(A, B, 0, "bf16x3"), exact)
    assert e16 < 1e-6 < e3


def test_model_error_growth_with_depth():
    """Error of the split precisions against recursion depth (n = 512,
    normal(0, 1)): a two-term bf16 split keeps 16 significant bits (about
    4.4e-6 at depth 0) and each Strassen level doubles the error (operand
    sums before and quadrant sums after each leaf), so BF16X3 stays within
    1e-5 at depth 1 and not at depth 2; FP16X3 (22 bits) and BF16X6 (24 bits)
    stay at the binary32 level at every depth."""
    n = 512
    A = inputs.normal(n, 31)
    B = inputs.normal(n, 32)
    exact = oracle.gemm_f64(A, B)
    err = {m: [oracle.rel_frobenius(oracle.strassen_model_f32(A, B, d, m), exact) for d in range(4)]
           for m in ("bf16x3", "bf16x6", "fp16x3")}
    e3 = err["bf16x3"]
    assert 3e-6 < e3[0] < 6e-6
    for k in range(3):
        assert 1.6 < e3[k + 1] / e3[k] < 2.4
    assert e3[1] < 1e-5 < e3[2]
    assert max(err["bf16x6"]) < 1e-6 and max(err["fp16x3"]) < 1e-6
