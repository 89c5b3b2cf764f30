"""Rectangular products (square-block partition) on the GPU, through the C ABI.

Integer inputs: every block product and every inner sum is an exact integer
below 2^24, so the result must equal brute force bit for bit.  Float inputs:
against the oracle's partition model (block products by the square model,
inner sum in binary32 in ascending order) within the binary32 accumulation
bound of the leaves, and against the FP64 rectangular product.
"""
import numpy as np
import pytest

import oracle

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


def mat(r, c, seed, kind):
    rng = np.random.default_rng(seed)
    if kind == "int":
        return rng.integers(-8, 9, size=(r, c)).astype(np.float32)
    return rng.uniform(-1, 1, size=(r, c)).astype(np.float32)


def exact(A, B):
    """The integer product of integer-valued A, B: binary64 BLAS is exact here
    (entries at most 8 in magnitude, k <= 6000: every partial sum is an
    integer below 2^53), and far faster than numpy's int64 product."""
    return (A.astype(np.float64) @ B.astype(np.float64)).astype(np.int64)


def run(S, ctx, A, B, depth, prec):
    m, k = A.shape
    n = B.shape[1]
    dA = torch.from_numpy(A).cuda()
    dB = torch.from_numpy(B).cuda()
    dC = torch.full((m, n), float("nan"), dtype=torch.float32, device="cuda")
    S.stark_gemm_rect(ctx, dA, dB, dC, m, k, n, depth, PREC[prec], None)
    torch.cuda.synchronize()
    return dC.cpu().numpy()


INT_CASES = [(300, 1000, 500, 1, "fp32"), (256, 512, 128, 0, "bf16x3"), (1000, 300, 700, 2, "bf16x3"),
             (130, 70, 200, 0, "fp16x3"), (1, 5, 3, 0, "fp32"), (777, 777, 777, 2, "fp32"),
             (700, 300, 1000, 1, "bf16x3_winograd"), (2048, 4096, 1024, 1, "bf16x6"), (5, 3000, 7, 0, "bf16x3")]


@pytest.mark.parametrize("m,k,n,depth,prec", INT_CASES)
def test_rect_integer_exact(S, ctx, m, k, n, depth, prec):
    print(f"case m={m} k={k} n={n} depth={depth} prec={prec} s={S.stark_rect_block_edge(m, k, n, depth)}",
          flush=True)
    A, B = mat(m, k, 1, "int"), mat(k, n, 2, "int")
    C = run(S, ctx, A, B, depth, prec)
    assert np.array_equal(C.astype(np.int64), exact(A, B))


@pytest.mark.parametrize("m,k,n,depth,prec", [(300, 1000, 500, 1, "fp32"), (300, 1000, 500, 1, "bf16x3"),
                                              (200, 130, 400, 0, "fp16x3"), (600, 250, 520, 1, "fp32_winograd")])
def test_rect_float_matches_partition_model(S, ctx, m, k, n, depth, prec):
    s = S.stark_rect_block_edge(m, k, n, depth)
    print(f"case m={m} k={k} n={n} depth={depth} prec={prec} s={s}", flush=True)
    A, B = mat(m, k, 3, "float"), mat(k, n, 4, "float")
    C = run(S, ctx, A, B, depth, prec)
    mode, variant = (prec[:-9], "winograd") if prec.endswith("_winograd") else (prec, "strassen")
    model = oracle.rect_model_f32(A, B, s, depth, mode, variant)
    exact = oracle.gemm_rect_f64(A, B)
    d = oracle.rel_frobenius(C, model)
    e_gpu, e_model = oracle.rel_frobenius(C, exact), oracle.rel_frobenius(model, exact)
    print(f"  rel_frob gpu={e_gpu:.3e} model={e_model:.3e} gpu-vs-model={d:.3e}", flush=True)
    L = s >> depth
    bound = 4 * 2.0 ** -24 * np.sqrt(L) * 2 ** depth * np.sqrt(-(-k // s))
    assert d <= bound
    assert e_gpu <= 1.5 * e_model + bound
    # fixed bound against the FP64 product: binary32 level (1e-5), or for
    # BF16X3 1.5 x its 4.4e-6 2^depth error growth
    assert e_gpu <= (1.5 * 4.4e-6 * 2 ** depth if mode == "bf16x3" else 1e-5)


def test_rect_square_equals_square_path(S, ctx):
    """m = k = n, a multiple of the block granule: one block, and the result
    equals stark_gemm bit for bit (same kernels, same plan)."""
    n, depth = 512, 2
    A, B = mat(n, n, 5, "float"), mat(n, n, 6, "float")
    C = run(S, ctx, A, B, depth, "bf16x3")
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dC = torch.empty((n, n), dtype=torch.float32, device="cuda")
    S.stark_gemm(ctx, dA, dB, dC, n, depth, PREC["bf16x3"], None)
    torch.cuda.synchronize()
    assert np.array_equal(C, dC.cpu().numpy())


def test_rect_repeat_and_stream(S, ctx):
    """The second call with the same pointers replays a captured graph; results
    are identical, on a caller stream too."""
    m, k, n, depth = 384, 1200, 640, 1
    A, B = mat(m, k, 7, "float"), mat(k, n, 8, "float")
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dC = torch.empty((m, n), dtype=torch.float32, device="cuda")
    st = torch.cuda.Stream()
    outs = []
    for _ in range(3):
        dC.fill_(float("nan"))
        torch.cuda.synchronize()
        S.stark_gemm_rect(ctx, dA, dB, dC, m, k, n, depth, PREC["bf16x3"], st)
        st.synchronize()
        outs.append(dC.cpu().numpy().copy())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


def test_rect_argument_errors(S, ctx):
    dA = torch.zeros((64, 96), dtype=torch.float32, device="cuda")
    dB = torch.zeros((96, 32), dtype=torch.float32, device="cuda")
    dC = torch.zeros((64, 32), dtype=torch.float32, device="cuda")
    with pytest.raises(S.StarkError) as e:
        S.stark_gemm_rect(ctx, dA, dB, dC, 64, 0, 32, 0, 0, None)
    assert e.value.status == S.STARK_EINVAL
    with pytest.raises(S.StarkError) as e:
        S.stark_gemm_rect(ctx, dA, dB, dA, 64, 96, 32, 0, 0, None)     # C overlaps A
    assert e.value.status == S.STARK_EINVAL
    shifted = torch.zeros(64 * 96 + 1, dtype=torch.float32, device="cuda")[1:]
    with pytest.raises(S.StarkError) as e:
        S.stark_gemm_rect(ctx, shifted, dB, dC, 64, 96, 32, 0, 0, None)
    assert e.value.status == S.STARK_EINVAL
    with pytest.raises(S.StarkError) as e:
        S.stark_gemm_rect(ctx, dA, dB, dC, 64, 96, 32, 0, 999, None)
    assert e.value.status == S.STARK_EUNSUPPORTED


@pytest.mark.parametrize("m,k,n,prec", [(3000, 4096, 3000, "fp32"), (2048, 6000, 4096, "bf16x3")])
def test_rect_auto_depth(S, ctx, m, k, n, prec):
    """STARK_DEPTH_AUTO takes the model's depth for min(m, k, n): the same
    result as that depth given explicitly, bit for bit, and exact on
    integers."""
    d = S.stark_model_depth(min(m, k, n), PREC[prec])
    print(f"case m={m} k={k} n={n} prec={prec} auto depth {d}", flush=True)
    A, B = mat(m, k, 5, "int"), mat(k, n, 6, "int")
    C = run(S, ctx, A, B, S.STARK_DEPTH_AUTO, prec)
    assert np.array_equal(C.astype(np.int64), exact(A, B))
    A, B = mat(m, k, 7, "float"), mat(k, n, 8, "float")
    assert np.array_equal(run(S, ctx, A, B, S.STARK_DEPTH_AUTO, prec), run(S, ctx, A, B, d, prec))
