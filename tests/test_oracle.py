"""Pins for the CPU oracle (runs without a GPU).

Each test fixes the oracle to something other than itself: hand-computed values
of the 2x2 worked example (Algorithm 1), exact brute force on small integers,
algebraic identities that hold bit for bit, the structural counts of the
divide/replicate step (Section III-C-1), and library routines (numpy matmul,
torch's bfloat16 rounding).  Planted mistakes in the oracle must fail them.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1811_07325_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "strassen_2x2.txt")


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
    A = g["A"].reshape(2, 2)
    B = g["B"].reshape(2, 2)
    C = g["C"].reshape(2, 2)
    for depth in (0, 1):
        assert np.array_equal(oracle.strassen_f64(A, B, depth), C)
    # divide step: the seven operand pairs multiply to the hand-computed M1..M7
    S, T = oracle.divide_f32(A, B)
    M = (S[:, 0, 0].astype(np.float64) * T[:, 0, 0].astype(np.float64))
    assert np.array_equal(M, g["M"])
    # combine step: M1..M7 fold back into the product
    Cc = oracle.combine_f32(g["M"].reshape(7, 1, 1))
    assert np.array_equal(Cc, C)


def test_printed_c22_sign_fails_the_worked_example():
    """The C22 of Algorithm 1 as printed (-M3) gives 54, not the product's 50."""
    g = _golden()
    oracle.set_mutation(1)
    C = oracle.strassen_f64(g["A"].reshape(2, 2), g["B"].reshape(2, 2), 1)
    assert C[1, 1] == g["C22_printed"][0]
    assert C[1, 1] != g["C"][3]


def _int_pair(n, seed):
    A = inputs.integers(n, seed)
    B = inputs.integers(n, seed + 1)
    return A, B


@pytest.mark.parametrize("n", list(range(1, 17)))
def test_brute_force_small_integers(n):
    A, B = _int_pair(n, 100 + n)
    exact = oracle.gemm_i64(A.astype(np.int64), B.astype(np.int64))
    assert np.array_equal(exact, A.astype(np.int64) @ B.astype(np.int64))
    assert np.array_equal(oracle.gemm_f64(A, B), exact.astype(np.float64))
    for depth in range(0, 5):
        C = oracle.strassen_f64(A, B, depth)
        assert np.array_equal(C, exact.astype(np.float64)), (n, depth)


@pytest.mark.parametrize("mutation", [1, 2, 3, 4])
def test_planted_mistakes_fail_brute_force(mutation):
    """Wrong sign, exchanged operands, a wrong quadrant, a dropped term."""
    A, B = _int_pair(8, 7)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    oracle.set_mutation(mutation)
    C = oracle.strassen_f64(A, B, 2)
    assert not np.array_equal(C, exact)


def test_padding_is_exact_and_cropped():
    A, B = _int_pair(13, 3)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    for depth, n_pad in [(1, 14), (2, 16), (2, 32), (3, 24)]:
        C = oracle.strassen_f64(A, B, depth, n_pad=n_pad)
        assert C.shape == (13, 13)
        assert np.array_equal(C, exact)
    with pytest.raises(ValueError):
        oracle.strassen_f64(A, B, 2, n_pad=14)  # not a multiple of 4


def test_classical_matches_blas_double():
    A = inputs.uniform(96, 0).astype(np.float64)
    B = inputs.uniform(96, 1).astype(np.float64)
    ref = A @ B
    C = oracle.gemm_f64(A, B)
    assert np.max(np.abs(C - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("depth", [1, 2, 3])
def test_strassen_double_close_to_classical(depth):
    A = inputs.uniform(64, 10)
    B = inputs.uniform(64, 11)
    ref = oracle.gemm_f64(A, B)
    C = oracle.strassen_f64(A, B, depth)
    assert oracle.rel_frobenius(C, ref) < 1e-14


def test_identities_exact():
    n = 16
    A = inputs.integers(n, 21)
    B = inputs.integers(n, 22)
    I = np.eye(n, dtype=np.float32)
    Z = np.zeros((n, n), dtype=np.float32)
    Af = inputs.uniform(n, 23)
    Bf = inputs.uniform(n, 24)
    for depth in range(0, 4):
        assert np.array_equal(oracle.strassen_f64(A, I, depth), A.astype(np.float64))
        assert np.array_equal(oracle.strassen_f64(I, B, depth), B.astype(np.float64))
        assert np.array_equal(oracle.strassen_f64(Z, Bf, depth), np.zeros((n, n)))
        C = oracle.strassen_f64(Af, Bf, depth)
        # negation commutes with round-to-nearest: bit-identical
        assert np.array_equal(oracle.strassen_f64(-Af, Bf, depth), -C)
        # power-of-two scaling is exact absent over/underflow
        assert np.array_equal(oracle.strassen_f64(Af * 8.0, Bf * 0.25, depth), C * 2.0)


@pytest.mark.parametrize("depth", [0, 1, 2, 3])
def test_structure_counts(depth):
    """7^k leaf products; 18 additions and 4/2/2/4 quadrant uses per node."""
    A, B = _int_pair(16, 5)
    _, cnt = oracle.strassen_f64(A, B, depth, with_counts=True)
    nodes = (7 ** depth - 1) // 6
    assert cnt.leaf_products == 7 ** depth
    assert cnt.internal_nodes == nodes
    assert cnt.block_additions == 18 * nodes
    # A11 and A22 four times, A12 and A21 twice (same for B): Section III-C-1
    assert list(cnt.uses_a) == [4 * nodes, 2 * nodes, 2 * nodes, 4 * nodes]
    assert list(cnt.uses_b) == [4 * nodes, 2 * nodes, 2 * nodes, 4 * nodes]


def test_sampled_rows_match_full_product():
    n = 80
    A = inputs.normal(n, 1)
    B = inputs.normal(n, 2)
    full = oracle.gemm_f64(A, B)
    rows = inputs.sample_rows(n, 17, 3)
    R = oracle.rows_f64(A, B, rows)
    assert np.array_equal(R, full[rows])


def test_freivalds_detects_a_planted_error_and_estimates_frobenius():
    n = 64
    A = inputs.normal(n, 1)
    B = inputs.normal(n, 2)
    C = oracle.gemm_f64(A, B)
    x = inputs.gaussian_vector(n, 3)
    assert oracle.freivalds_rel(A, B, C, x) < 1e-14
    bad = C.copy()
    bad[17, 40] += 1.0
    assert oracle.freivalds_rel(A, B, bad, x) > 1e-4
    # Gaussian probes: mean of ||E x||^2 approaches ||E||_F^2
    rng = np.random.default_rng(9)
    E = rng.standard_normal((n, n)) * 1e-6
    est = np.mean([np.sum((E @ rng.standard_normal(n)) ** 2) for _ in range(400)])
    assert abs(est / np.sum(E * E) - 1.0) < 0.15


def test_divide_combine_compose_to_exact_product():
    """One divide + exact leaf products + one combine == brute force (binary32)."""
    for m in (2, 8, 32):
        X, Y = _int_pair(m, 40 + m)
        S, T = oracle.divide_f32(X, Y)
        M = np.stack([oracle.gemm_i64(S[i].astype(np.int64), T[i].astype(np.int64))
                      for i in range(7)]).astype(np.float32)
        C = oracle.combine_f32(M)
        exact = X.astype(np.int64) @ Y.astype(np.int64)
        assert np.array_equal(C.astype(np.int64), exact)


def test_divide_operand_pairs_two_levels():
    """Two nested divide/combine levels reproduce the product exactly."""
    m = 16
    X, Y = _int_pair(m, 77)
    S, T = oracle.divide_f32(X, Y)
    Ms = []
    for i in range(7):
        S2, T2 = oracle.divide_f32(S[i], T[i])
        M2 = np.stack([oracle.gemm_i64(S2[j].astype(np.int64), T2[j].astype(np.int64))
                       for j in range(7)]).astype(np.float32)
        Ms.append(oracle.combine_f32(M2))
    C = oracle.combine_f32(np.stack(Ms))
    assert np.array_equal(C.astype(np.int64), X.astype(np.int64) @ Y.astype(np.int64))


def test_bf16_split_matches_library_rounding():
    torch = pytest.importorskip("torch")
    x = inputs.normal(64, 5).ravel()
    x = np.concatenate([x, np.float32([1.0, -2.5, 3.0e-30, 1.00390625, 1.01171875, 65504.0])])
    planes = oracle.split_bf16(x, terms=3)
    hi_lib = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(planes[0], hi_lib)
    hi = oracle.bf16_bits_to_f32(planes[0])
    mid = oracle.bf16_bits_to_f32(planes[1])
    lo = oracle.bf16_bits_to_f32(planes[2])
    r1 = (x - hi).astype(np.float32)
    mid_lib = torch.from_numpy(r1).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(planes[1], mid_lib)
    # two terms keep 16 significant bits, three keep 24 (all of binary32)
    xd = x.astype(np.float64)
    two = hi.astype(np.float64) + mid.astype(np.float64)
    three = two + lo.astype(np.float64)
    nz = xd != 0
    assert np.max(np.abs(two - xd)[nz] / np.abs(xd[nz])) <= 2.0 ** -16
    assert np.max(np.abs(three - xd)[nz] / np.abs(xd[nz])) <= 2.0 ** -24
    # ties round to even: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7
    t = oracle.split_bf16(np.float32([1.00390625, 1.01171875]), terms=2)
    assert oracle.bf16_bits_to_f32(t[0]).tolist() == [1.0, 1.015625]
