"""Pins for the oracle's rectangular product (runs without a GPU).

The paper treats n = 2^p and defers other shapes to partitioning (Section
III-A).  The rectangular path partitions C (m x n) = A (m x k) B (k x n) into
square s x s block products and sums the inner blocks; its oracle is the
plain rectangular definition, pinned to brute force and to numpy/BLAS, and a
block-partition model pinned to the square model and to exact integers.
"""
import numpy as np
import pytest

import oracle
from paper_1811_07325_amd import inputs


def _rect(m, k, seed, lo=-8, hi=8):
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=(m, k)).astype(np.float32)


@pytest.mark.parametrize("m,k,n", [(1, 1, 1), (3, 5, 2), (7, 16, 9), (16, 3, 11), (12, 12, 12)])
def test_rect_classical_brute_force(m, k, n):
    A, B = _rect(m, k, 1), _rect(k, n, 2)
    exact = A.astype(np.int64) @ B.astype(np.int64)
    assert np.array_equal(oracle.gemm_rect_f64(A, B), exact.astype(np.float64))


def test_rect_classical_matches_blas_and_square():
    rng = np.random.default_rng(3)
    A = rng.uniform(-1, 1, (40, 72))
    B = rng.uniform(-1, 1, (72, 24))
    ref = A @ B
    C = oracle.gemm_rect_f64(A, B)
    assert np.max(np.abs(C - ref)) <= 1e-13 * np.max(np.abs(ref))
    S = inputs.uniform(32, 4)
    T = inputs.uniform(32, 5)
    assert np.array_equal(oracle.gemm_rect_f64(S, T), oracle.gemm_f64(S, T))


def test_rect_blocks():
    assert oracle.rect_blocks(1000, 4000, 2000, 1024) == (1, 4, 2)
    assert oracle.rect_blocks(1024, 1024, 1024, 1024) == (1, 1, 1)
    assert oracle.rect_blocks(1, 1, 1, 64) == (1, 1, 1)


@pytest.mark.parametrize("mode", ["fp32", "bf16x3"])
@pytest.mark.parametrize("variant", ["strassen", "winograd"])
def test_rect_model_integer_exact(mode, variant):
    A, B = _rect(70, 150, 6), _rect(150, 40, 7)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float32)
    C = oracle.rect_model_f32(A, B, 64, 1, mode, variant)
    assert C.shape == (70, 40) and np.array_equal(C, exact)


def test_rect_model_one_block_is_the_square_model():
    A, B = inputs.uniform(64, 8), inputs.uniform(64, 9)
    for mode in ("fp32", "bf16x3", "fp16x3"):
        assert np.array_equal(oracle.rect_model_f32(A, B, 64, 1, mode), oracle.strassen_model_f32(A, B, 1, mode))


def test_rect_model_float_close_to_exact():
    rng = np.random.default_rng(10)
    A = rng.uniform(-1, 1, (100, 300)).astype(np.float32)
    B = rng.uniform(-1, 1, (300, 70)).astype(np.float32)
    ref = oracle.gemm_rect_f64(A, B)
    C = oracle.rect_model_f32(A, B, 128, 1, "fp32")
    assert oracle.rel_frobenius(C, ref) < 1e-6
