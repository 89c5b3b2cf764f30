"""The workload configurations at their full sizes, through the C ABI.

* n = 512, binary32, uniform[-1, 1], two levels to 128 x 128 leaves: against
  the whole FP64 product, plus an integer copy that must be bit-exact;
* n = 4096, binary32, uniform[-1, 1], three levels to 512 x 512 leaves, next
  to the classical product (depth 0) on the same GPU: sampled rows against
  the FP64 oracle, integer copy bit-exact on sampled rows;
* n = 16384, normal(0, 1), split-precision leaves, depth chosen by the
  autotuner among 2..4, run as the benchmark runs it (one stream, eager call
  then graph replay): 256 sampled rows against the FP64 oracle and Freivalds'
  check, within 1e-5 for the benchmark's headline path; BF16X3's error growth
  with depth;
* n = 49152 and 49120 (n^2 > 2^31), integer inputs: exact on rows whose
  element offsets cross 2^31.
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


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def multiply(S, ctx, dA, dB, n, depth, prec, stream=None):
    C = torch.full((n, n), float("nan"), dtype=torch.float32, device="cuda")
    S.stark_gemm(ctx, dA, dB, C, n, depth, prec, stream)
    torch.cuda.synchronize()
    return C


def rel_rows(C, ref, rows):
    got = C[torch.from_numpy(rows).cuda()].cpu().numpy().astype(np.float64)
    d = got - ref
    return float(np.sqrt(np.sum(d * d) / np.sum(ref * ref))), float(np.max(np.abs(d)))


# Relative Frobenius error allowed against the FP64 oracle for the binary32
# and 22-bit split paths (measured errors are about 1e-6 at these sizes).
TOL = 1e-5


def test_n512_two_levels_fp32_and_integer_copy(S, ctx):
    n, depth = 512, 2
    A, B = inputs.uniform(n, 0), inputs.uniform(n, 1)
    C = multiply(S, ctx, dev(A), dev(B), n, depth, S.STARK_FP32).cpu().numpy()
    ref = oracle.gemm_f64(A, B)
    err = oracle.rel_frobenius(C, ref)
    print(f"n=512 depth 2 fp32: rel_frob={err:.3e} max_abs={oracle.max_abs(C, ref):.3e}")
    assert err <= TOL
    Ai, Bi = inputs.integers(n, 0), inputs.integers(n, 1)
    Ci = multiply(S, ctx, dev(Ai), dev(Bi), n, depth, S.STARK_FP32).cpu().numpy()
    assert np.array_equal(Ci.astype(np.int64), oracle.gemm_i64(Ai, Bi))


def test_n4096_three_levels_fp32_next_to_classical(S, ctx):
    n, depth = 4096, 3
    A, B = inputs.uniform(n, 0), inputs.uniform(n, 1)
    dA, dB = dev(A), dev(B)
    rows = inputs.sample_rows(n, 256, 2)
    ref = oracle.rows_f64(A, B, rows)
    Cs = multiply(S, ctx, dA, dB, n, depth, S.STARK_FP32)
    Cc = multiply(S, ctx, dA, dB, n, 0, S.STARK_FP32)
    es, ms = rel_rows(Cs, ref, rows)
    ec, mc = rel_rows(Cc, ref, rows)
    print(f"n=4096 fp32: depth 3 rel_frob={es:.3e} max_abs={ms:.3e}; classical rel_frob={ec:.3e} max_abs={mc:.3e}")
    assert es <= TOL
    assert ec <= TOL
    # both results estimate the same product: their difference is bounded by
    # the sum of their errors
    d = (Cs - Cc).double()
    assert float(torch.linalg.norm(d) / torch.linalg.norm(Cc.double())) <= 2 * TOL
    # element by element against the oracle's arithmetic model of depth 3
    # (binary32 divide / combine, exact leaf sums): what remains is the
    # binary32 accumulation inside the 512-long leaf sums, amplified by at
    # most 2 per level
    model = oracle.strassen_model_f32(A, B, depth, "fp32", n)
    got = Cs.cpu().numpy()
    dm = oracle.rel_frobenius(got, model)
    ulp_bound = 4 * 2.0 ** -24 * np.sqrt(n >> depth) * 2 ** depth
    print(f"  depth 3 vs model: rel_frob={dm:.3e} (bound {ulp_bound:.3e})")
    assert dm <= ulp_bound
    # elementwise: every entry within that many units of the entry's scale
    scale = np.sqrt(np.mean(model.astype(np.float64) ** 2))
    assert np.max(np.abs(got.astype(np.float64) - model)) <= 8 * ulp_bound * scale
    # integer copy: exact on sampled rows (every intermediate is an integer
    # below 2^24 at this size)
    Ai, Bi = inputs.integers(n, 0), inputs.integers(n, 1)
    Ci = multiply(S, ctx, dev(Ai), dev(Bi), n, depth, S.STARK_FP32)
    got = Ci[torch.from_numpy(rows).cuda()].cpu().numpy().astype(np.int64)
    exact = oracle.rows_f64(Ai, Bi, rows)    # integer sums below 2^53: exact in FP64
    assert np.array_equal(got, exact.astype(np.int64))


# Split-precision paths at n = 16384, normal(0, 1) inputs, relative Frobenius
# error against the FP64 oracle on 256 sampled rows.
HEADLINE_TOL = 1e-5


def row_and_freivalds_errors(S, st, dA, dB, C, A, B, n):
    rows = inputs.sample_rows(n, 256, 2)
    ref = oracle.rows_f64(A, B, rows)
    err, mabs = rel_rows(C, ref, rows)
    x = dev(inputs.gaussian_vector(n, 3))
    y = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(3)]
    S.stark_matvec_f64(dB, x, y[0], n, st)
    S.stark_matvec_f64(dA, y[0], y[1], n, st)
    S.stark_matvec_f64(C, x, y[2], n, st)
    st.synchronize()
    freiv = float(torch.linalg.norm(y[2] - y[1]) / torch.linalg.norm(y[1]))
    return err, mabs, freiv


@pytest.fixture(scope="module")
def big_inputs():
    n = 16384
    A, B = inputs.normal(n, 0), inputs.normal(n, 1)
    return n, A, B, dev(A), dev(B)


def test_n16384_headline_path_within_tolerance(S, ctx, big_inputs):
    """The benchmark's headline: among the three-product split paths on the
    16-bit matrix cores (FP16X3, BF16X3), depths 2..4 autotuned, the fastest
    whose Freivalds error is within 1e-5; its result must then be within 1e-5
    on 256 sampled rows, eager, captured and replayed alike."""
    n, A, B, dA, dB = big_inputs
    C = torch.empty((n, n), dtype=torch.float32, device="cuda")
    st = torch.cuda.Stream()
    best = None
    for name in ("fp16x3", "bf16x3"):
        prec = S.PRECISIONS[name]
        pts = S.stark_tune(ctx, dA, dB, C, n, prec, 2, 4, HEADLINE_TOL, st)
        assert sorted(set(p[0] for p in pts)) == [2, 3, 4]
        for d in (2, 3, 4):      # the planner's tile class is always measured; every class divides the leaf
            assert S.stark_plan_info(n, d, prec).gemm_tile in [p[3] for p in pts if p[0] == d]
        assert all((n >> p[0]) % p[3] == 0 for p in pts)
        print(f"n=16384 {name}: tune {[(d, t, round(m, 3), f'{e:.2e}') for d, m, e, t in pts]}", flush=True)
        for p in pts:
            if p[2] <= HEADLINE_TOL and (best is None or p[1] < best[2][1]):
                best = (name, prec, p)
    assert best is not None, "no split path within the tolerance at depths 2..4"
    name, prec, tuned = best
    outs = []
    for _ in range(3):                 # eager, capture, replay of what the autotuner recorded
        C.fill_(float("nan"))
        torch.cuda.synchronize()
        S.stark_gemm(ctx, dA, dB, C, n, S.STARK_DEPTH_AUTO, prec, st)
        st.synchronize()
        outs.append(C.clone())
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])
    err, mabs, freiv = row_and_freivalds_errors(S, st, dA, dB, C, A, B, n)
    print(f"headline {name} depth {tuned[0]} tile {tuned[3]}: "
          f"rel_frob(256 rows)={err:.3e} max_abs={mabs:.3e} freivalds={freiv:.3e}")
    assert err <= HEADLINE_TOL
    assert freiv <= HEADLINE_TOL
    # Freivalds' estimate and the sampled rows measure the same error: same order
    assert 0.25 * err <= freiv <= 4 * err
    # the tuner's own Freivalds figure agrees with this one
    assert 0.25 * freiv <= tuned[2] <= 4 * freiv


@pytest.mark.parametrize("name,depth", [("fp32", 3), ("bf16x6", 2), ("fp16x3_winograd", 2)])
def test_n16384_other_paths_within_tolerance(S, ctx, big_inputs, name, depth):
    """The comparison paths the benchmark reports at n = 16384 (binary32
    leaves at depth 3, the six-product bf16 split, Winograd's variant with
    binary16 leaves): 256 sampled rows and Freivalds' check within 1e-5 of
    the FP64 product."""
    n, A, B, dA, dB = big_inputs
    prec = S.PRECISIONS[name]
    C = torch.full((n, n), float("nan"), dtype=torch.float32, device="cuda")
    st = torch.cuda.Stream()
    torch.cuda.synchronize()
    S.stark_gemm(ctx, dA, dB, C, n, depth, prec, st)
    st.synchronize()
    err, mabs, freiv = row_and_freivalds_errors(S, st, dA, dB, C, A, B, n)
    print(f"n=16384 {name} depth {depth}: rel_frob(256 rows)={err:.3e} max_abs={mabs:.3e} freivalds={freiv:.3e}",
          flush=True)
    assert bool(torch.isfinite(C).all())
    assert err <= HEADLINE_TOL and freiv <= HEADLINE_TOL
    assert 0.25 * err <= freiv <= 4 * err


def test_n16384_bf16x3_error_grows_with_depth(S, ctx, big_inputs):
    """Documents why BF16X3 is not the headline: a two-term bf16 split keeps
    16 significant bits (about 4.4e-6 at depth 0) and every Strassen level
    roughly doubles the error, so at depths 2..4 it misses 1e-5; each depth
    stays within twice that growth, and the autotuner records nothing for a
    depth range with no point within the tolerance."""
    n, A, B, dA, dB = big_inputs
    C = torch.empty((n, n), dtype=torch.float32, device="cuda")
    st = torch.cuda.Stream()
    errs = []
    for depth in (2, 3, 4):
        C.fill_(float("nan"))
        torch.cuda.synchronize()
        S.stark_gemm(ctx, dA, dB, C, n, depth, S.STARK_BF16X3, st)
        st.synchronize()
        err, mabs, freiv = row_and_freivalds_errors(S, st, dA, dB, C, A, B, n)
        print(f"n=16384 bf16x3 depth {depth}: rel_frob(256 rows)={err:.3e} freivalds={freiv:.3e}", flush=True)
        assert err <= 2 * 4.4e-6 * 2 ** depth
        assert err > HEADLINE_TOL
        errs.append(err)
    assert all(1.5 < errs[i + 1] / errs[i] < 2.6 for i in range(2))


# n^2 > 2^31: every element offset of A, B, C and the workspace needs 64 bits.
# Integers in [-2, 2] keep every intermediate exact (|C| <= 4n < 2^24, leaf
# operands at most 8, exact in bf16), so sampled rows must equal the exact
# product bit for bit -- rows whose offsets cross 2^31 and the last row
# included.  49120 is not a multiple of 64: padding and crop at those offsets.
@pytest.mark.parametrize("n,prec,depth", [(49152, "fp32", 0), (49152, "fp32", 1), (49120, "bf16x3", 2)])
def test_beyond_32bit_offsets_integer_exact(S, ctx, n, prec, depth):
    print(f"case n={n} depth={depth} prec={prec} (n^2 = {n * n} > 2^31)", flush=True)
    g = torch.Generator(device="cuda")
    g.manual_seed(n + depth)
    A = torch.randint(-2, 3, (n, n), generator=g, device="cuda", dtype=torch.float32)
    B = torch.randint(-2, 3, (n, n), generator=g, device="cuda", dtype=torch.float32)
    C = torch.full((n, n), float("nan"), dtype=torch.float32, device="cuda")
    S.stark_gemm(ctx, A, B, C, n, depth, S.PRECISIONS[prec], None)
    torch.cuda.synchronize()
    cross = (1 << 31) // n
    rows = torch.tensor([0, 1, cross - 1, cross, cross + 1, n // 2, n - 2, n - 1], device="cuda")
    Ar = A[rows].double()
    ref = torch.empty((rows.numel(), n), dtype=torch.float64, device="cuda")
    for c0 in range(0, n, 8192):                 # exact in binary64, column chunks of B
        ref[:, c0:c0 + 8192] = Ar @ B[:, c0:c0 + 8192].double()
    got = C[rows].double()
    assert torch.equal(got, ref), (got - ref).abs().max().item()
    del A, B, C, Ar, ref, got
    torch.cuda.empty_cache()
