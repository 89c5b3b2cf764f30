"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

* integer inputs (uniform in [-8, 8]): every result is an exact integer below
  2^24, so every precision must match brute force bit for bit;
* per-phase checks: the divide, split and combine kernels against the
  oracle's binary32 step routines, bit for bit;
* float inputs: against the oracle's arithmetic model of the same depth and
  leaf precision (binary32 divide/combine, exact leaf sums); the only
  difference left is the binary32 accumulation order inside the leaf GEMM;
* full-size configurations on sampled rows and Freivalds' check.
"""
import numpy as np
import pytest

import oracle
from paper_1811_07325_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PREC = {"fp32": 0, "bf16x3": 1, "bf16x6": 2, "fp16x3": 3}
PREC.update({k + "_winograd": v | 16 for k, v in list(PREC.items())})   # Winograd's variant flag


def base(prec):
    """(leaf precision name, recursion variant) of a test precision name."""
    return (prec[:-9], "winograd") if prec.endswith("_winograd") else (prec, "strassen")


@pytest.fixture(scope="module")
def S():
    from paper_1811_07325_amd import stark
    return stark


WS_BYTES = 512 << 20


@pytest.fixture(scope="module")
def ws():
    # torch-allocated workspace lent to the context, so tests can read it
    return torch.empty(WS_BYTES, dtype=torch.uint8, device="cuda")


@pytest.fixture(scope="module")
def ctx(S, ws):
    c = S.stark_create(0, ws, WS_BYTES)
    yield c
    S.stark_destroy(c)


@pytest.fixture(scope="module")
def ctx_big(S):
    c = S.stark_create(0)     # library-owned workspace
    yield c
    S.stark_destroy(c)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def run(S, ctx, A, B, depth, prec, C=None):
    n = A.shape[0]
    dA, dB = dev(A), dev(B)
    dC = torch.full((n, n), float("nan"), dtype=torch.float32, device="cuda") if C is None else C
    S.stark_gemm(ctx, dA, dB, dC, n, depth, PREC[prec], None)
    torch.cuda.synchronize()
    return dC.cpu().numpy()


def rel_f(C, ref):
    return oracle.rel_frobenius(C, ref)


def plan_model(S, A, B, depth, prec):
    """The oracle's arithmetic model of the plan the library takes for this
    size (padded to its n_pad, or peeled), and that plan."""
    mode, variant = base(prec)
    d = S.stark_plan_info(A.shape[0], depth, PREC[prec])
    if d.peel:
        return oracle.peel_model_f32(A, B, depth, mode, d.peel, variant), d
    return oracle.strassen_model_f32(A, B, depth, mode, d.n_pad, variant), d


# ---------------------------------------------------------------------------
# Bit-exact integer products (all precisions, padded and ragged sizes).
# ---------------------------------------------------------------------------
INT_CASES = [(512, 2, "fp32"), (512, 2, "bf16x3"), (512, 2, "bf16x6"),
             (512, 0, "fp32"), (512, 1, "fp32"), (512, 3, "fp32"), (512, 0, "bf16x3"), (512, 3, "bf16x3"),
             (1000, 2, "fp32"), (1000, 2, "bf16x3"), (300, 1, "fp32"), (300, 1, "bf16x3"),
             (65, 0, "fp32"), (65, 0, "bf16x3"), (200, 2, "fp32"), (200, 2, "bf16x6"), (384, 1, "bf16x3"),
             (129, 0, "fp32"), (250, 1, "bf16x6"), (1, 0, "fp32"), (2, 0, "bf16x3"), (63, 0, "bf16x6"),
             (512, 2, "fp16x3"), (1000, 2, "fp16x3"), (65, 0, "fp16x3"), (300, 1, "fp16x3"), (512, 3, "fp16x3")]


# Winograd's operand chains grow by up to 4x per level (S4, T4 sum four
# blocks): integers in [-8, 8] keep every intermediate below 2^24 to depth 2,
# integers in [-2, 2] to depth 3.
INT_CASES += [(512, 2, "fp32_winograd"), (512, 2, "bf16x3_winograd"), (1000, 2, "bf16x6_winograd"),
              (300, 1, "fp16x3_winograd"), (65, 0, "fp32_winograd"), (200, 2, "fp32_winograd"),
              (512, 3, "fp32_winograd"), (512, 3, "bf16x3_winograd"), (500, 3, "fp16x3_winograd")]


@pytest.mark.parametrize("n,depth,prec", INT_CASES)
def test_integer_inputs_bit_exact(S, ctx, n, depth, prec):
    print(f"case n={n} depth={depth} prec={prec}", flush=True)
    r = 2 if (prec.endswith("_winograd") and depth >= 3) else 8
    A = inputs.integers(n, 0, -r, r)
    B = inputs.integers(n, 1, -r, r)
    # binary64 BLAS is exact on these integers (every partial sum is an
    # integer below 2^53) and far faster than numpy's int64 product
    exact = (A.astype(np.float64) @ B.astype(np.float64)).astype(np.int64)
    C = run(S, ctx, A, B, depth, prec)
    assert np.all(np.isfinite(C))
    assert np.array_equal(C.astype(np.int64), exact)
    assert np.array_equal(C, exact.astype(np.float32))


@pytest.mark.parametrize("n,depth,prec", [(4096, 1, "bf16x3"), (4096, 0, "bf16x6"), (4096, 1, "bf16x6"),
                                          (4032, 1, "bf16x3"), (4096, 1, "fp16x3"), (4096, 0, "fp32"),
                                          (4096, 1, "fp32"), (4032, 1, "fp32"), (4096, 1, "bf16x3_winograd"),
                                          (4032, 1, "fp32_winograd"), (2048, 3, "fp32"), (2048, 2, "fp32")])
def test_integer_inputs_bit_exact_large_tiles(S, ctx_big, n, depth, prec):
    """Leaves wide enough for the 256-wide tile class (n = 2048 at depth 3:
    leaves of 256, the shortest K loop of the binary32 kernel, whose steps
    go two to a barrier)."""
    print(f"case n={n} depth={depth} prec={prec}", flush=True)
    assert S.stark_plan_info(n, depth, PREC[prec]).gemm_tile == 256
    A = inputs.integers(n, 0)
    B = inputs.integers(n, 1)
    # every partial sum is an integer below 2^53: BLAS double products are exact
    exact = (A.astype(np.float64) @ B.astype(np.float64)).astype(np.float32)
    C = run(S, ctx_big, A, B, depth, prec)
    assert np.array_equal(C, exact)


# ---------------------------------------------------------------------------
# Floating-point inputs against the arithmetic model of the same method.
# ---------------------------------------------------------------------------
FLOAT_CASES = [(512, 2, "fp32"), (512, 2, "bf16x3"), (512, 2, "bf16x6"), (256, 1, "fp32"),
               (384, 1, "bf16x3"), (1000, 2, "fp32"), (1000, 2, "bf16x3"), (512, 0, "fp32"),
               (512, 0, "bf16x3"), (512, 3, "bf16x6"), (512, 2, "fp16x3"), (1000, 2, "fp16x3"),
               (512, 0, "fp16x3"), (384, 1, "fp16x3")]


FLOAT_CASES += [(512, 2, "fp32_winograd"), (1000, 2, "bf16x3_winograd"), (512, 3, "bf16x6_winograd"),
                (384, 1, "fp16x3_winograd"), (512, 0, "bf16x3_winograd")]


# Fixed error bounds against the FP64 product (relative Frobenius).  FP32,
# FP16X3 and BF16X6 keep 22 or more significant bits per leaf operand and sit
# at the binary32 level: 1e-5.  BF16X3 keeps 16 and its error doubles per
# Strassen level from about 4.4e-6 at depth 0 (the oracle's model gives the
# same growth); it is held to 1.5 times that growth.
def fixed_bound(prec, depth):
    mode, variant = base(prec)
    if mode == "bf16x3":
        return 1.5 * 4.4e-6 * 2 ** depth * (2 if variant == "winograd" else 1)
    return 1e-5


@pytest.mark.parametrize("n,depth,prec", FLOAT_CASES)
def test_float_inputs_match_model(S, ctx, n, depth, prec):
    print(f"case n={n} depth={depth} prec={prec}", flush=True)
    A = inputs.uniform(n, 0)
    B = inputs.uniform(n, 1)
    C = run(S, ctx, A, B, depth, prec)
    # the same padding (or peeling) as the library's plan
    model, plan = plan_model(S, A, B, depth, prec)
    exact = oracle.gemm_f64(A, B)
    e_gpu, e_model = rel_f(C, exact), rel_f(model, exact)
    d = rel_f(C, model)
    print(f"  rel_frob gpu={e_gpu:.3e} model={e_model:.3e} gpu-vs-model={d:.3e}", flush=True)
    # binary32 accumulation over a leaf of edge L: a few units of 2^-24 sqrt(L)
    L = plan.leaf
    assert d <= 4 * 2.0 ** -24 * np.sqrt(L) * 2 ** depth
    assert e_gpu <= 1.5 * e_model + 1e-6
    assert e_gpu <= fixed_bound(prec, depth)


@pytest.mark.parametrize("n,depth,prec", [(4096, 1, "fp32"), (4096, 1, "bf16x3"), (4096, 1, "fp32_winograd"),
                                          (2048, 3, "fp32")])
def test_float_large_tiles_match_model(S, ctx_big, n, depth, prec):
    """The 256-wide tile kernels on float inputs: against the arithmetic
    model on every element, against the FP64 product on sampled rows."""
    print(f"case n={n} depth={depth} prec={prec}", flush=True)
    assert S.stark_plan_info(n, depth, PREC[prec]).gemm_tile == 256
    A = inputs.uniform(n, 0)
    B = inputs.uniform(n, 1)
    C = run(S, ctx_big, A, B, depth, prec)
    model, plan = plan_model(S, A, B, depth, prec)
    rows = inputs.sample_rows(n, 64, 2)
    ref = oracle.rows_f64(A, B, rows)
    e_gpu, e_model = rel_f(C[rows], ref), rel_f(model[rows], ref)
    d = rel_f(C, model)
    print(f"  rel_frob(rows) gpu={e_gpu:.3e} model={e_model:.3e} gpu-vs-model={d:.3e}", flush=True)
    # the model's leaves are exact: the GPU adds binary32 accumulation over L
    L = plan.leaf
    bound = 4 * 2.0 ** -24 * np.sqrt(L) * 2 ** depth
    assert d <= bound
    assert e_gpu <= 1.5 * e_model + bound
    assert e_gpu <= fixed_bound(prec, depth)


# ---------------------------------------------------------------------------
# Per-phase kernels, bit for bit.
# ---------------------------------------------------------------------------
def ws_view(ws, offset, count, dtype):
    itemsize = np.dtype(dtype).itemsize
    assert 0 <= offset and offset + count * itemsize <= ws.numel()
    return ws[offset:offset + count * itemsize].cpu().numpy().view(dtype)


@pytest.mark.parametrize("variant", ["strassen", "winograd"])
@pytest.mark.parametrize("n,depth", [(256, 2), (250, 2), (512, 3), (500, 3)])
def test_divide_levels_bit_exact(S, ctx, ws, n, depth, variant):
    """Every stored binary32 divide level against the oracle's divide steps.
    From depth 2 on the level above the last is formed on the fly and not
    stored, and the last level stores all seven operands."""
    A = inputs.uniform(n, 3)
    B = inputs.uniform(n, 4)
    dA, dB = dev(A), dev(B)
    dC = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    prec = 16 if variant == "winograd" else 0
    S.stark_gemm_phases(ctx, dA, dB, dC, n, depth, prec, S.STARK_PHASE_DIVIDE, None)
    torch.cuda.synchronize()
    d = S.stark_plan_info(n, depth, prec)
    np_ = d.n_pad
    Ap = np.zeros((np_, np_), np.float32); Ap[:n, :n] = A
    Bp = np.zeros((np_, np_), np.float32); Bp[:n, :n] = B
    # stored operand blocks, as indices of the products they feed
    sA5, sB5 = ([4, 5, 6, 2], [4, 5, 6, 3]) if variant == "winograd" else ([0, 1, 4, 5, 6], [0, 2, 3, 5, 6])
    assert d.div_slots[depth - 2] == 0 and d.div_slots[depth - 1] == 7
    Xs, Ys = [Ap], [Bp]           # operands of the nodes of level l, in node order
    for lvl in range(depth):
        nx, ny = [], []
        slots = d.div_slots[lvl]
        h = (np_ >> lvl) // 2
        if slots:
            ga = ws_view(ws, d.div_a[lvl], 7 ** lvl * slots * h * h, np.float32).reshape(-1, slots, h, h)
            gb = ws_view(ws, d.div_b[lvl], 7 ** lvl * slots * h * h, np.float32).reshape(-1, slots, h, h)
        ia, ib = (list(range(7)), list(range(7))) if slots == 7 else (sA5, sB5)
        for node, (X, Y) in enumerate(zip(Xs, Ys)):
            Sx, Ty = oracle.divide_f32(X, Y, variant)
            if slots:
                assert np.array_equal(ga[node], Sx[ia]), (lvl, node)
                assert np.array_equal(gb[node], Ty[ib]), (lvl, node)
            nx.extend(Sx)
            ny.extend(Ty)
        Xs, Ys = nx, ny


def unblock(x, L, BR=16):
    """Blocked bf16 plane layout of the library (1 KB blocks of BR rows x
    512/BR k, block-row-major; chunk c of row r stored at c ^ swz(r)) ->
    row-major."""
    BK = 512 // BR
    CR = BK // 8
    r = np.arange(L)[:, None]
    k = np.arange(L)[None, :]
    rr = r % BR
    swz = (((rr >> 1) & 3) ^ ((rr >> 3) & 1)) if BR == 16 else (((rr >> 2) ^ (rr >> 3)) & 1)
    off = ((r // BR) * (L // BK) + k // BK) * 512 + ((rr * CR + (((k >> 3) % CR) ^ swz)) << 3) + (k & 7)
    return x[..., off]


@pytest.mark.parametrize("prec,depth,n", [("bf16x3", 1, 256), ("bf16x6", 2, 256), ("bf16x3", 0, 128),
                                          ("bf16x3", 1, 200), ("bf16x3", 2, 250), ("bf16x3", 3, 512),
                                          ("bf16x6", 3, 500), ("bf16x3_winograd", 1, 200),
                                          ("bf16x3_winograd", 2, 250), ("bf16x6_winograd", 3, 512)])
def test_split_leaf_operands_bit_exact(S, ctx, ws, prec, depth, n):
    P = {"bf16x3": 2, "bf16x6": 3}[base(prec)[0]]
    variant = base(prec)[1]
    A = inputs.normal(n, 5)
    B = inputs.normal(n, 6)
    dA, dB = dev(A), dev(B)
    dC = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    S.stark_gemm_phases(ctx, dA, dB, dC, n, depth, PREC[prec], S.STARK_PHASE_DIVIDE, None)
    torch.cuda.synchronize()
    d = S.stark_plan_info(n, depth, PREC[prec])
    np_, L = d.n_pad, d.leaf
    Ap = np.zeros((np_, np_), np.float32); Ap[:n, :n] = A
    Bp = np.zeros((np_, np_), np.float32); Bp[:n, :n] = B
    # leaf operands by the oracle's divide, in leaf order (base-7 digits)
    Xs, Ys = [Ap], [Bp]
    for _ in range(depth):
        nx, ny = [], []
        for X, Y in zip(Xs, Ys):
            Sx, Ty = oracle.divide_f32(X, Y, variant)
            nx.extend(Sx)
            ny.extend(Ty)
        Xs, Ys = nx, ny
    nleaf = 7 ** depth
    ga = unblock(ws_view(ws, d.leaf_a, nleaf * P * L * L, np.uint16).reshape(nleaf, P, L * L), L)
    gb = unblock(ws_view(ws, d.leaf_b, nleaf * P * L * L, np.uint16).reshape(nleaf, P, L * L), L)
    for i in range(nleaf):
        assert np.array_equal(ga[i], oracle.split_bf16(Xs[i], P)), i
        # B side is stored transposed: plane[j][k] = split(T)[k][j]
        assert np.array_equal(gb[i], oracle.split_bf16(Ys[i], P).transpose(0, 2, 1)), i


@pytest.mark.parametrize("depth,n,scale_a,variant", [(1, 256, 1.0, "strassen"), (2, 256, 1e-3, "strassen"),
                                                    (0, 128, 300.0, "strassen"), (1, 200, 1.0, "strassen"),
                                                    (2, 256, 1e-3, "winograd"), (3, 512, 7.0, "winograd")])
def test_fp16_split_and_scale_bit_exact(S, ctx, ws, depth, n, scale_a, variant):
    """FP16X3: the per-matrix exponents and the binary16 planes of every leaf
    (Winograd's operands grow by up to 4 per level, its exponent uses 2 depth)."""
    A = (inputs.normal(n, 15) * np.float32(scale_a)).astype(np.float32)
    B = inputs.normal(n, 16)
    dA, dB = dev(A), dev(B)
    dC = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    prec = 3 | (16 if variant == "winograd" else 0)
    S.stark_gemm_phases(ctx, dA, dB, dC, n, depth, prec, S.STARK_PHASE_DIVIDE, None)
    torch.cuda.synchronize()
    d = S.stark_plan_info(n, depth, prec)
    np_, L = d.n_pad, d.leaf
    ex = ws_view(ws, d.scale + 4 * 512, 2, np.int32)
    growth = 2 * depth if variant == "winograd" else depth
    ea, eb = oracle.f16_scale_exp(A, growth), oracle.f16_scale_exp(B, growth)
    assert (int(ex[0]), int(ex[1])) == (ea, eb)
    Ap = np.zeros((np_, np_), np.float32); Ap[:n, :n] = A
    Bp = np.zeros((np_, np_), np.float32); Bp[:n, :n] = B
    Xs, Ys = [Ap], [Bp]
    for _ in range(depth):
        nx, ny = [], []
        for X, Y in zip(Xs, Ys):
            Sx, Ty = oracle.divide_f32(X, Y, variant)
            nx.extend(Sx)
            ny.extend(Ty)
        Xs, Ys = nx, ny
    nleaf = 7 ** depth
    f16 = lambda b: b.view(np.float16).astype(np.float32)
    ga = f16(unblock(ws_view(ws, d.leaf_a, nleaf * 2 * L * L, np.uint16).reshape(nleaf, 2, L * L), L))
    gb = f16(unblock(ws_view(ws, d.leaf_b, nleaf * 2 * L * L, np.uint16).reshape(nleaf, 2, L * L), L))
    for i in range(nleaf):
        assert np.array_equal(ga[i], oracle.split_f16(Xs[i], ea)), i
        assert np.array_equal(gb[i], oracle.split_f16(Ys[i], eb).transpose(0, 2, 1)), i


def test_fp16x3_wide_range_inputs_match_model(S, ctx):
    """Operands far from unit scale: the power-of-two scaling keeps FP16X3 on the model."""
    n, depth = 512, 2
    A = (inputs.normal(n, 17) * np.float32(3e4)).astype(np.float32)
    B = (inputs.normal(n, 18) * np.float32(2e-6)).astype(np.float32)
    C = run(S, ctx, A, B, depth, "fp16x3")
    model, _ = plan_model(S, A, B, depth, "fp16x3")
    exact = oracle.gemm_f64(A, B)
    assert rel_f(C, model) <= 4 * 2.0 ** -24 * np.sqrt(128) * 4
    assert rel_f(C, exact) < 5e-6


@pytest.mark.parametrize("variant", ["strassen", "winograd"])
@pytest.mark.parametrize("n,depth", [(256, 2), (512, 3), (256, 1)])
def test_combine_levels_bit_exact(S, ctx, ws, n, depth, variant):
    """The two deepest combine levels run as one pass (no level-(k-1)
    outputs in memory), the others one level at a time: every level written
    equals the oracle's binary32 combine steps bit for bit."""
    A = inputs.uniform(n, 7)
    B = inputs.uniform(n, 8)
    dA, dB = dev(A), dev(B)
    dC = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    prec = 16 if variant == "winograd" else 0
    S.stark_gemm_phases(ctx, dA, dB, dC, n, depth, prec, S.STARK_PHASE_ALL, None)
    torch.cuda.synchronize()
    d = S.stark_plan_info(n, depth, prec)
    L = d.leaf
    nleaf = 7 ** depth
    M = ws_view(ws, d.leaf_m, nleaf * L * L, np.float32).reshape(nleaf, L, L)
    # oracle: one level at a time from the leaf products up
    levels = {depth: M}
    for lvl in range(depth - 1, -1, -1):
        ch = levels[lvl + 1]
        levels[lvl] = np.stack([oracle.combine_f32(ch[7 * i:7 * i + 7], variant) for i in range(7 ** lvl)])
    if depth == 3:   # level 1 is written by the fused pass over levels 2 and 1
        m1 = n >> 1
        C1 = ws_view(ws, d.comb[1], 7 * m1 * m1, np.float32).reshape(7, m1, m1)
        assert np.array_equal(C1, levels[1])
    assert np.array_equal(dC.cpu().numpy(), levels[0][0])


def test_leaf_products_close_to_exact(S, ctx, ws):
    """Each leaf product (FP32 path) against the FP64 product of its operands."""
    n, depth = 256, 1
    A = inputs.uniform(n, 9)
    B = inputs.uniform(n, 10)
    dA, dB = dev(A), dev(B)
    dC = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    S.stark_gemm_phases(ctx, dA, dB, dC, n, depth, 0, S.STARK_PHASE_DIVIDE | S.STARK_PHASE_LEAF, None)
    torch.cuda.synchronize()
    d = S.stark_plan_info(n, depth, 0)
    L = d.leaf
    M = ws_view(ws, d.leaf_m, 7 * L * L, np.float32).reshape(7, L, L)
    Sx, Ty = oracle.divide_f32(A, B)
    for i in range(7):
        ref = oracle.gemm_f64(Sx[i], Ty[i])
        assert rel_f(M[i], ref) < 4 * 2.0 ** -24 * np.sqrt(L)


# ---------------------------------------------------------------------------
# Graph replay, generator, measurement helpers.
# ---------------------------------------------------------------------------
def test_graph_replays_are_identical(S, ctx):
    n = 512
    A = inputs.uniform(n, 11)
    B = inputs.uniform(n, 12)
    dA, dB = dev(A), dev(B)
    s = torch.cuda.Stream()
    outs = []
    C = torch.empty((n, n), dtype=torch.float32, device="cuda")
    for i in range(5):   # eager, capture, replays
        C.fill_(float("nan"))
        torch.cuda.synchronize()
        S.stark_gemm(ctx, dA, dB, C, n, 2, 0, s)
        s.synchronize()
        outs.append(C.cpu().numpy().copy())
        # unrelated eager work between replays
        _ = (dA * 2.0).sum().item()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    assert np.array_equal(outs[0], run(S, ctx, A, B, 2, "fp32"))


def test_graph_cache_eviction_keeps_results(S, ctx):
    """More (plan, pointer) keys than the graph cache holds (64): every call
    still gives the same result, including replays of evicted and re-captured
    graphs."""
    n = 256
    A = inputs.uniform(n, 21)
    B = inputs.uniform(n, 22)
    dA, dB = dev(A), dev(B)
    ref = run(S, ctx, A, B, 1, "bf16x3")
    Cs = [torch.empty((n, n), dtype=torch.float32, device="cuda") for _ in range(80)]
    s = torch.cuda.Stream()
    for rep in range(3):                     # eager, capture (evicting), capture again
        for C in Cs:
            C.fill_(float("nan"))
        torch.cuda.synchronize()
        for C in Cs:
            S.stark_gemm(ctx, dA, dB, C, n, 1, PREC["bf16x3"], s)
        s.synchronize()
        for i, C in enumerate(Cs):
            assert np.array_equal(C.cpu().numpy(), ref), (rep, i)


def test_batched_cache_eviction_keeps_results(S, ctx):
    """More distinct batches than the batched-call cache keeps per context
    (64): every call still gives the single-call result, including replays of
    evicted and re-captured batches."""
    n = 256
    A = inputs.uniform(n, 23)
    B = inputs.uniform(n, 24)
    dA, dB = dev(A), dev(B)
    ref = run(S, ctx, A, B, 1, "bf16x3")
    Cs = [torch.empty((n, n), dtype=torch.float32, device="cuda") for _ in range(80)]
    s = torch.cuda.Stream()
    for rep in range(3):                     # eager, capture (evicting), capture again
        for C in Cs:
            C.fill_(float("nan"))
        torch.cuda.synchronize()
        for C in Cs:
            S.stark_gemm_batched(ctx, [dA], [dB], [C], [n], 1, PREC["bf16x3"], s)
        s.synchronize()
        for i, C in enumerate(Cs):
            assert np.array_equal(C.cpu().numpy(), ref), (rep, i)


def test_calls_on_two_streams_run_in_order(S, ctx):
    """One context, calls on two streams issued back to back: the calls share
    the context's workspace, so each must wait for the previous one's work.
    Every result equals its single-call result bit for bit (eager, captured
    and replayed), also with a batched and a rectangular call in the mix."""
    n, depth, p = 2048, 2, PREC["bf16x3"]
    print(f"case n={n} depth={depth} prec=bf16x3 two streams", flush=True)
    probs = [(inputs.uniform(n, 31 + 2 * i), inputs.uniform(n, 32 + 2 * i)) for i in range(3)]
    refs = [run(S, ctx, A, B, depth, "bf16x3") for A, B in probs]
    dA = [dev(A) for A, _ in probs]
    dB = [dev(B) for _, B in probs]
    Cs = [torch.empty((n, n), dtype=torch.float32, device="cuda") for _ in range(3)]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for rep in range(3):                     # eager, capture, replay
        for C in Cs:
            C.fill_(float("nan"))
        torch.cuda.synchronize()
        S.stark_gemm(ctx, dA[0], dB[0], Cs[0], n, depth, p, s1)
        S.stark_gemm(ctx, dA[1], dB[1], Cs[1], n, depth, p, s2)
        S.stark_gemm_batched(ctx, [dA[2]], [dB[2]], [Cs[2]], [n], depth, p, s1)
        s1.synchronize()
        s2.synchronize()
        for i, C in enumerate(Cs):
            assert np.array_equal(C.cpu().numpy(), refs[i]), (rep, i)
    # a rectangular call on one stream right after a square call on the other
    m, k = 1024, 2048
    A = np.random.default_rng(41).integers(-8, 9, (m, k)).astype(np.float32)
    B = np.random.default_rng(42).integers(-8, 9, (k, n)).astype(np.float32)
    dRa, dRb = dev(A), dev(B)
    Cr = torch.full((m, n), float("nan"), dtype=torch.float32, device="cuda")
    Cs[0].fill_(float("nan"))
    torch.cuda.synchronize()
    S.stark_gemm(ctx, dA[0], dB[0], Cs[0], n, depth, p, s1)
    S.stark_gemm_rect(ctx, dRa, dRb, Cr, m, k, n, 1, p, s2)
    s1.synchronize()
    s2.synchronize()
    assert np.array_equal(Cs[0].cpu().numpy(), refs[0])
    assert np.array_equal(Cr.cpu().numpy(), oracle.gemm_rect_f64(A, B).astype(np.float32))


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp16x3", "bf16x6"])
def test_tuner_record_selects_tile(S, tmp_path, prec):
    """A record (n, precision, depth, tile) in the autotuner's cache file makes
    STARK_DEPTH_AUTO run that depth with that leaf-GEMM tile class: every
    class dividing the leaf gives the exact integer product, and the same
    float result bit for bit (same accumulation order), on the oracle's
    model."""
    n, depth = 1024, 1       # leaf 512: tile classes 64, 128 and 256 all divide it
    print(f"case n={n} depth={depth} prec={prec} tiles 64/128/256", flush=True)
    A = inputs.integers(n, 51)
    B = inputs.integers(n, 52)
    exact = oracle.gemm_i64(A.astype(np.int64), B.astype(np.int64))
    dA, dB = dev(A), dev(B)
    Af, Bf = inputs.uniform(n, 53), inputs.uniform(n, 54)
    dAf, dBf = dev(Af), dev(Bf)
    floats = []
    for tile in (64, 128, 256):
        path = tmp_path / f"tune_{prec}_{tile}.txt"
        path.write_text(f"# n precision depth ms freivalds_error tile\n{n} {PREC[prec]} {depth} 1.0 0.0 {tile}\n")
        c = S.stark_create(0, tuner_cache=str(path))
        try:
            C = torch.full((n, n), float("nan"), dtype=torch.float32, device="cuda")
            S.stark_gemm(c, dA, dB, C, n, S.STARK_DEPTH_AUTO, PREC[prec], None)
            torch.cuda.synchronize()
            assert np.array_equal(C.cpu().numpy().astype(np.int64), exact), tile
            C.fill_(float("nan"))
            S.stark_gemm(c, dAf, dBf, C, n, S.STARK_DEPTH_AUTO, PREC[prec], None)
            torch.cuda.synchronize()
            floats.append(C.cpu().numpy())
        finally:
            S.stark_destroy(c)
    # every tile class accumulates each output in the same order
    assert np.array_equal(floats[0], floats[1]) and np.array_equal(floats[0], floats[2])
    model = oracle.strassen_model_f32(Af, Bf, depth, base(prec)[0], n, "strassen")
    assert rel_f(floats[0], model) < 4 * 2.0 ** -24 * (n >> depth) ** 0.5 * 2 ** depth


def test_concurrent_threads_one_context(S, ctx):
    """Four host threads call stark_gemm on one context, each on its own
    stream, at the same time (the binding releases the interpreter lock):
    the context serialises the calls and orders their device work, so every
    result equals its single-call result bit for bit."""
    import threading
    n, depth, p = 1024, 2, PREC["bf16x3"]
    probs = [(inputs.uniform(n, 61 + 2 * i), inputs.uniform(n, 62 + 2 * i)) for i in range(4)]
    refs = [run(S, ctx, A, B, depth, "bf16x3") for A, B in probs]
    dA = [dev(A) for A, _ in probs]
    dB = [dev(B) for _, B in probs]
    Cs = [torch.full((n, n), float("nan"), dtype=torch.float32, device="cuda") for _ in range(4)]
    streams = [torch.cuda.Stream() for _ in range(4)]
    errors = []

    def work(i):
        try:
            for _ in range(6):
                S.stark_gemm(ctx, dA[i], dB[i], Cs[i], n, depth, p, streams[i])
            streams[i].synchronize()
        except Exception as e:          # noqa: BLE001 -- reported below
            errors.append(e)

    threads = [threading.Thread(target=work, args=(i,)) for i in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    for i in range(4):
        assert np.array_equal(Cs[i].cpu().numpy(), refs[i]), i


@pytest.mark.parametrize("n", [300, 301])
def test_generator_matches_host_twin(S, n):
    """Even and odd element counts (the last pair half written)."""
    X = torch.full((n + 1, n), float("nan"), dtype=torch.float32, device="cuda")
    S.stark_generate_normal(X, n, 12345, None)
    torch.cuda.synchronize()
    out = X.cpu().numpy().ravel()
    assert np.all(np.isnan(out[n * n:]))          # nothing written past n^2
    # the same Philox words and uniforms; the device's binary32 log, sincos
    # and sqrt stay within a few ulps of the radius (at most 6.7: 2^-21)
    got, twin = out[:n * n], inputs.philox_normal(n, 12345).ravel()
    assert np.max(np.abs(got.astype(np.float64) - twin)) <= 4 * 2.0 ** -21


def test_matvec_and_row_errors(S):
    n = 333
    M = inputs.normal(n, 1)
    x = inputs.gaussian_vector(n, 2)
    dM = dev(M)
    dx = torch.from_numpy(x).cuda()
    dy = torch.empty(n, dtype=torch.float64, device="cuda")
    S.stark_matvec_f64(dM, dx, dy, n, None)
    rows = inputs.sample_rows(n, 17, 3)
    ref = M.astype(np.float64)[rows] + 1e-3
    out = torch.empty(3, dtype=torch.float64, device="cuda")
    S.stark_row_errors(dM, n, torch.from_numpy(rows).cuda(), rows.size, torch.from_numpy(ref).cuda(), out, None)
    torch.cuda.synchronize()
    assert np.allclose(dy.cpu().numpy(), oracle.gemv_f64(M, x), rtol=1e-12, atol=1e-12)
    o = out.cpu().numpy()
    dref = M.astype(np.float64)[rows] - ref
    assert np.isclose(o[0], np.max(np.abs(dref)), rtol=1e-12)
    assert np.isclose(o[1], np.sum(dref ** 2), rtol=1e-10)
    assert np.isclose(o[2], np.sum(ref ** 2), rtol=1e-10)


def test_argument_errors(S, ctx):
    n = 128
    A = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    B = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    with pytest.raises(S.StarkError) as e:
        S.stark_gemm(ctx, A, B, A, n, 0, 0, None)      # C overlaps A
    assert e.value.status == S.STARK_EINVAL
    with pytest.raises(S.StarkError):
        S.stark_gemm(ctx, A, B, None, n, 0, 0, None)
    with pytest.raises(S.StarkError):
        S.stark_gemm(ctx, A, B, torch.empty_like(A), n, 5, 0, None)   # depth too deep
    with pytest.raises(S.StarkError) as e:
        S.stark_gemm(ctx, A, B, torch.empty_like(A), n, 0, 9, None)
    assert e.value.status == S.STARK_EUNSUPPORTED
    # a view 4 bytes into an allocation is rejected before any launch
    shifted = torch.zeros(n * n + 1, dtype=torch.float32, device="cuda")[1:].view(n, n)
    with pytest.raises(S.StarkError) as e:
        S.stark_gemm(ctx, shifted, B, torch.empty_like(A), n, 0, 0, None)
    assert e.value.status == S.STARK_EINVAL and "aligned" in str(e.value)


def test_caller_workspace_too_small(S):
    n = 256
    ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    c = S.stark_create(0, ws, ws.numel())
    try:
        A = torch.zeros((n, n), dtype=torch.float32, device="cuda")
        with pytest.raises(S.StarkError) as e:
            S.stark_gemm(c, A, A, torch.empty_like(A), n, 1, 0, None)
        assert e.value.status == S.STARK_ENOMEM
    finally:
        S.stark_destroy(c)
