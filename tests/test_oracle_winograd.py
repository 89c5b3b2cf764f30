"""Pins for the oracle's Winograd variant (runs without a GPU).

Winograd's form of Strassen's algorithm reaches the same product with 15
block additions per node instead of 18.  Its oracle routines are pinned to a
hand-computed 2x2 example, exact brute force on small integers, the
structural counts, the classical product, and planted mistakes that must
fail those pins.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1811_07325_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "winograd_2x2.txt")


def _golden():
    vals = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *nums = line.split()
            vals[key] = np.array([float(x) for x in nums])
    return vals


@pytest.fixture(autouse=True)
def _no_mutation():
    oracle.set_mutation(0)
    yield
    oracle.set_mutation(0)


def test_worked_example_2x2():
    g = _golden()
    A, B, C = g["A"].reshape(2, 2), g["B"].reshape(2, 2), g["C"].reshape(2, 2)
    assert np.array_equal(oracle.winograd_f64(A, B, 1), C)
    S, T = oracle.divide_f32(A, B, "winograd")
    assert np.array_equal(S[:, 0, 0], g["S"]) and np.array_equal(T[:, 0, 0], g["T"])
    M = S[:, 0, 0].astype(np.float64) * T[:, 0, 0].astype(np.float64)
    assert np.array_equal(M, g["M"])
    assert np.array_equal(oracle.combine_f32(g["M"].reshape(7, 1, 1), "winograd"), C)
    # the Strassen combine applied to Winograd's products is not the product
    assert not np.array_equal(oracle.combine_f32(g["M"].reshape(7, 1, 1)), C)


@pytest.mark.parametrize("n", list(range(1, 17)))
def test_brute_force_small_integers(n):
    A = inputs.integers(n, 300 + n)
    B = inputs.integers(n, 301 + n)
    exact = oracle.gemm_i64(A.astype(np.int64), B.astype(np.int64)).astype(np.float64)
    for depth in range(0, 5):
        assert np.array_equal(oracle.winograd_f64(A, B, depth), exact), (n, depth)


@pytest.mark.parametrize("mutation", [5, 6])
def test_planted_mistakes_fail_brute_force(mutation):
    """S4 formed from S1 instead of S2; the sign of M4 in C21 flipped."""
    A, B = inputs.integers(8, 7), inputs.integers(8, 8)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    oracle.set_mutation(mutation)
    assert not np.array_equal(oracle.winograd_f64(A, B, 2), exact)


def test_structure_counts():
    A, B = inputs.integers(16, 1), inputs.integers(16, 2)
    for depth in range(0, 4):
        _, c = oracle.winograd_f64(A, B, depth, with_counts=True)
        internal = sum(7 ** l for l in range(depth))
        assert c.leaf_products == 7 ** depth
        assert c.internal_nodes == internal
        assert c.block_additions == 15 * internal
        # A11, A12, A22 and B11, B21, B22 each feed one product directly
        assert list(c.uses_a) == [internal, internal, 0, internal]
        assert list(c.uses_b) == [internal, 0, internal, internal]


@pytest.mark.parametrize("depth", [1, 2, 3])
def test_double_close_to_classical(depth):
    A, B = inputs.uniform(64, 10), inputs.uniform(64, 11)
    assert oracle.rel_frobenius(oracle.winograd_f64(A, B, depth), oracle.gemm_f64(A, B)) < 1e-14


def test_padding_is_exact_and_cropped():
    A, B = inputs.integers(13, 3), inputs.integers(13, 4)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    for depth, n_pad in [(1, 14), (2, 16), (3, 24)]:
        assert np.array_equal(oracle.winograd_f64(A, B, depth, n_pad=n_pad), exact)


def test_binary32_steps_with_exact_leaves_are_brute_force():
    """Divide step, exact leaf products, combine step, on integers: every
    intermediate is an integer below 2^24, so the binary32 steps are exact."""
    A, B = inputs.integers(32, 5), inputs.integers(32, 6)
    S, T = oracle.divide_f32(A, B, "winograd")
    M = np.stack([oracle.gemm_f64(S[i], T[i]) for i in range(7)]).astype(np.float32)
    C = oracle.combine_f32(M, "winograd")
    assert np.array_equal(C.astype(np.int64), A.astype(np.int64) @ B.astype(np.int64))


def test_binary32_divide_rounds_each_chained_sum_once():
    """S2 = S1 - A11 uses the rounded S1 (and T2 = B22 - T1 the rounded T1):
    recomputing the chain in numpy binary32 reproduces the step bit for bit,
    and differs from the unchained form for some inputs."""
    X, Y = inputs.normal(64, 7), inputs.normal(64, 8)
    S, T = oracle.divide_f32(X, Y, "winograd")
    h = 32
    a11, a12, a21, a22 = X[:h, :h], X[:h, h:], X[h:, :h], X[h:, h:]
    b11, b12, b21, b22 = Y[:h, :h], Y[:h, h:], Y[h:, :h], Y[h:, h:]
    s1 = a21 + a22
    s2 = s1 - a11
    t1 = b12 - b11
    t2 = b22 - t1
    assert np.array_equal(S[4], s1) and np.array_equal(S[5], s2) and np.array_equal(S[2], a12 - s2)
    assert np.array_equal(T[4], t1) and np.array_equal(T[5], t2) and np.array_equal(T[3], t2 - b21)
    assert np.array_equal(S[6], a11 - a21) and np.array_equal(T[6], b22 - b12)
    unchained = (a21.astype(np.float64) + a22 - a11).astype(np.float32)
    assert not np.array_equal(S[5], unchained)


@pytest.mark.parametrize("mode", ["fp32", "bf16x3", "fp16x3"])
def test_model_integer_exact_and_float_close(mode):
    A, B = inputs.integers(64, 9), inputs.integers(64, 10)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float32)
    for depth in (1, 2):
        assert np.array_equal(oracle.strassen_model_f32(A, B, depth, mode, variant="winograd"), exact)
    Af, Bf = inputs.uniform(64, 11), inputs.uniform(64, 12)
    ref = oracle.gemm_f64(Af, Bf)
    C = oracle.strassen_model_f32(Af, Bf, 2, mode, variant="winograd")
    bound = {"fp32": 1e-6, "bf16x3": 3e-5, "fp16x3": 1e-5}[mode]
    assert oracle.rel_frobenius(C, ref) < bound
