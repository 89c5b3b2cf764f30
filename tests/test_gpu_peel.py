"""Peeled sizes through the C ABI: n = 64 * 2^depth * m + r with the residue
r peeled off (the recursion runs on the leading (n - r)^2 core in place, the
border rows and columns are classical inner products, every core output
takes the r-term fix-up when the last combine level writes it).

* integer inputs: exact, bit for bit, for r = 1, 7, 63 and, with rows that
  stay 16-byte aligned, 4, 12 and 64 (STARK_PEEL, so
  the case does not depend on the planner's choice), every leaf precision,
  depths 1-3, Algorithm 1 and Winograd's variant, 64-, 128- and 256-wide
  leaf tiles;
* float inputs: against the oracle's model of the peeled scheme on every
  element and within the fixed bounds against the FP64 product;
* C starts as NaN, so an element the border or the combine misses fails;
* batched: peeled, padded and exact-multiple problems in one grouped launch
  sequence, each equal to its single multiply bit for bit, eager and graph.
"""
import numpy as np
import pytest

import oracle
from paper_1811_07325_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

PREC = {"fp32": 0, "bf16x3": 1, "bf16x6": 2, "fp16x3": 3}
PREC.update({k + "_winograd": v | 16 for k, v in list(PREC.items())})


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


def multiply(S, ctx, A, B, depth, prec):
    n = A.shape[0]
    C = torch.full((n, n), float("nan"), dtype=torch.float32, device="cuda")
    S.stark_gemm(ctx, dev(A), dev(B), C, n, depth, prec, None)
    torch.cuda.synchronize()
    return C.cpu().numpy()


def base(prec):
    return (prec[:-9], "winograd") if prec.endswith("_winograd") else (prec, "strassen")


PEEL = 64   # STARK_PEEL
# (n, depth, precision name, flags): r = 1, 7 and 63
INT_CASES = [(1025, 1, "fp32", PEEL), (1031, 1, "bf16x3", PEEL), (1087, 1, "fp32", PEEL), (2049, 2, "fp32", PEEL),
             (2055, 2, "fp16x3", PEEL), (2111, 2, "bf16x6", PEEL), (2111, 2, "bf16x3", PEEL), (4097, 3, "fp32", PEEL),
             (4103, 3, "fp16x3", PEEL), (4159, 3, "bf16x3", PEEL), (2049, 2, "fp32_winograd", PEEL),
             (1031, 1, "bf16x3_winograd", PEEL), (2111, 2, "fp16x3_winograd", PEEL), (8199, 1, "fp32", PEEL),
             (8199, 1, "bf16x3", PEEL), (2055, 1, "fp16x3", PEEL)]
# residues that keep the rows 16-byte aligned (n % 4 == 0): the core is read
# and written with vector accesses, level-0 views of A and B included
INT_CASES += [(1028, 1, "fp32", PEEL), (2112, 2, "bf16x3", PEEL), (4160, 3, "fp16x3", PEEL),
              (2060, 2, "fp32_winograd", PEEL), (8204, 1, "bf16x6", PEEL), (2112, 2, "fp32", PEEL)]


@pytest.mark.parametrize("n,depth,prec,flags", INT_CASES)
def test_peeled_integer_inputs_exact(S, ctx, n, depth, prec, flags):
    p = PREC[prec] | flags
    d = S.stark_plan_info(n, depth, p)
    print(f"case n={n} depth={depth} prec={prec} peel={d.peel} tile={d.gemm_tile}", flush=True)
    assert d.peel == n % (64 << depth) and d.n_pad == n - d.peel
    # Winograd's chains grow 4x per level: keep depth-3 intermediates below 2^24
    lim = 2 if (prec.endswith("_winograd") and depth >= 3) else 8
    A = inputs.integers(n, 0, -lim, lim)
    B = inputs.integers(n, 1, -lim, lim)
    exact = (A.astype(np.float64) @ B.astype(np.float64)).astype(np.float32)
    C = multiply(S, ctx, A, B, depth, p)
    assert np.array_equal(C, exact)


def test_peeled_tiles_cover_every_class(S):
    tiles = {S.stark_plan_info(n, d, PREC[p] | f).gemm_tile for n, d, p, f in INT_CASES}
    assert tiles == {64, 128, 256}


def fixed_bound(prec, depth):
    mode, variant = base(prec)
    if mode == "bf16x3":
        return 1.5 * 4.4e-6 * 2 ** depth * (2 if variant == "winograd" else 1)
    return 1e-5


FLOAT_CASES = [(1025, 1, "fp32", PEEL), (2055, 2, "bf16x3", PEEL), (2111, 2, "fp16x3", PEEL),
               (1087, 1, "bf16x6", PEEL), (4097, 3, "fp32", PEEL), (2049, 2, "fp32_winograd", PEEL),
               (8199, 1, "bf16x3", PEEL), (1028, 1, "fp32", PEEL), (2112, 2, "fp16x3", PEEL)]


@pytest.mark.parametrize("n,depth,prec,flags", FLOAT_CASES)
def test_peeled_float_inputs_match_model(S, ctx, n, depth, prec, flags):
    p = PREC[prec] | flags
    d = S.stark_plan_info(n, depth, p)
    print(f"case n={n} depth={depth} prec={prec} peel={d.peel}", flush=True)
    A = inputs.uniform(n, 2)
    B = inputs.uniform(n, 3)
    C = multiply(S, ctx, A, B, depth, p)
    mode, variant = base(prec)
    model = oracle.peel_model_f32(A, B, depth, mode, d.peel, variant)
    rows = inputs.sample_rows(n, 96, 4)
    rows[-1] = n - 1                     # a border row
    ref = oracle.rows_f64(A, B, rows)
    e_gpu, e_model = oracle.rel_frobenius(C[rows], ref), oracle.rel_frobenius(model[rows], ref)
    diff = oracle.rel_frobenius(C, model)
    L = d.leaf
    bound = 4 * 2.0 ** -24 * np.sqrt(L) * 2 ** depth
    print(f"  rel_frob(rows) gpu={e_gpu:.3e} model={e_model:.3e} gpu-vs-model={diff:.3e}", flush=True)
    assert diff <= bound
    assert e_gpu <= 1.5 * e_model + bound
    assert e_gpu <= fixed_bound(prec, depth)
    # the border alone (classical binary32 inner products of length n)
    border = np.concatenate([C[n - d.peel:, :].ravel(), C[:n - d.peel, n - d.peel:].ravel()])
    mborder = np.concatenate([model[n - d.peel:, :].ravel(), model[:n - d.peel, n - d.peel:].ravel()])
    assert oracle.rel_frobenius(border, mborder) <= 4 * 2.0 ** -24 * np.sqrt(n)


@pytest.mark.parametrize("n,depth,prec", [(16385, 2, "fp16x3"), (16448, 3, "fp32")])
def test_peeled_full_size_sampled_rows(S, ctx, n, depth, prec):
    """Full size, the planner's own choice (peeling: padding would either
    run 64-wide tiles on leaves of 4096 + 64 or pad to 17408): 64 sampled
    rows and the last (border) row within 1e-5 of the FP64 product, and
    Freivalds' check over the whole result."""
    d = S.stark_plan_info(n, depth, PREC[prec])
    print(f"case n={n} depth={depth} prec={prec} peel={d.peel}", flush=True)
    assert d.peel == n % (64 << depth) and d.gemm_tile == 256
    A = inputs.normal(n, 0)
    B = inputs.normal(n, 1)
    dA, dB = dev(A), dev(B)
    C = torch.full((n, n), float("nan"), dtype=torch.float32, device="cuda")
    S.stark_gemm(ctx, dA, dB, C, n, depth, PREC[prec], None)
    torch.cuda.synchronize()
    rows = inputs.sample_rows(n, 64, 2)
    rows[-1] = n - 1
    ref = oracle.rows_f64(A, B, rows)
    got = C[torch.from_numpy(rows).cuda()].cpu().numpy()
    assert oracle.rel_frobenius(got, ref) <= 1e-5
    x = np.random.default_rng(3).standard_normal(n)
    assert oracle.freivalds_rel(A, B, C.cpu().numpy(), x) <= 1e-5


def test_peeled_and_padded_agree(S, ctx):
    """The same product peeled and padded: both within the bound of the
    FP64 product, and equal on integers."""
    n, depth = 2049, 2
    A, B = inputs.uniform(n, 5), inputs.uniform(n, 6)
    Cp = multiply(S, ctx, A, B, depth, PREC["fp32"] | PEEL)
    Cz = multiply(S, ctx, A, B, depth, PREC["fp32"] | S.STARK_PAD)
    assert S.stark_plan_info(n, depth, PREC["fp32"] | PEEL).peel == 1
    padded = S.stark_plan_info(n, depth, PREC["fp32"] | S.STARK_PAD)
    assert padded.peel == 0 and padded.n_pad > n and padded.n_pad % 256 == 0
    exact = oracle.gemm_f64(A, B)
    assert oracle.rel_frobenius(Cp, exact) <= 1e-5 and oracle.rel_frobenius(Cz, exact) <= 1e-5
    with pytest.raises(S.StarkError):
        S.stark_gemm(ctx, dev(A), dev(B), dev(np.empty_like(A)), n, depth, S.STARK_PEEL | S.STARK_PAD, None)


def test_peeled_graph_replays(S, ctx):
    n, depth = 4103, 2
    dA, dB = dev(inputs.uniform(n, 7)), dev(inputs.uniform(n, 8))
    outs = []
    for _ in range(3):     # eager, then the captured graph twice
        C = torch.full((n, n), float("nan"), dtype=torch.float32, device="cuda")
        S.stark_gemm(ctx, dA, dB, C, n, depth, PREC["fp16x3"] | PEEL, None)
        torch.cuda.synchronize()
        outs.append(C)
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])
    assert bool(torch.isfinite(outs[0]).all())


def test_batched_mixes_peeled_padded_and_exact_problems(S, ctx):
    """One batch at depth 1 (binary32, STARK_PEEL): 1025, 1087 and 1031
    peeled (r = 1, 63, 7), 1024 an exact multiple, 200 padded (r = 72 is
    beyond the peelable residues); each equals its single multiply bit for
    bit."""
    ns = [1025, 1087, 1024, 1031, 200]
    depth = 1
    peels = [S.stark_plan_info(n, depth, PEEL).peel for n in ns]
    assert peels == [1, 63, 0, 7, 0]
    As = [dev(inputs.uniform(n, 30 + i)) for i, n in enumerate(ns)]
    Bs = [dev(inputs.uniform(n, 40 + i)) for i, n in enumerate(ns)]
    singles = []
    for a, b, n in zip(As, Bs, ns):
        C = torch.full((n, n), float("nan"), dtype=torch.float32, device="cuda")
        S.stark_gemm(ctx, a, b, C, n, depth, PEEL, None)
        singles.append(C)
    torch.cuda.synchronize()
    for _ in range(2):     # eager, then the captured graph
        Cs = [torch.full((n, n), float("nan"), dtype=torch.float32, device="cuda") for n in ns]
        S.stark_gemm_batched(ctx, As, Bs, Cs, ns, depth, PEEL, None)
        torch.cuda.synchronize()
        for C, ref in zip(Cs, singles):
            assert torch.equal(C, ref)
