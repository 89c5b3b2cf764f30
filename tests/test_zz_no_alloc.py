"""stark_gemm_noalloc, the allocation-free entry point, through the C ABI:
its results equal stark_gemm's at the same depth (same kernels and plan, its
intermediates in the library's fixed device scratch instead of a context
workspace), on two calls in a row with the second smaller (peeled sizes
included), and a plan that does not fit the scratch is refused before
anything runs."""
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


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


# (n, depth, precision, flags): the last pair peels (STARK_PEEL: residues 7, 1)
@pytest.mark.parametrize("first,second", [((1024, 2, "fp16x3", 0), (640, 1, "bf16x3", 0)),
                                          ((1000, 2, "fp32", 0), (300, 1, "fp32_winograd", 0)),
                                          ((1031, 1, "fp16x3", 64), (1025, 1, "fp32", 64))])
def test_noalloc_equals_gemm_on_two_calls(S, first, second):
    ctx = S.stark_create(0)
    try:
        for n, depth, prec, flags in (first, second):
            print(f"case n={n} depth={depth} prec={prec} flags={flags}", flush=True)
            p = S.PRECISIONS[prec] | flags
            assert S.stark_plan_info(n, depth, p).peel == (n % (64 << depth) if flags else 0)
            assert S.stark_workspace_size(n, depth, p) <= S.STARK_NOALLOC_SCRATCH_BYTES
            A, B = inputs.normal(n, 60 + n), inputs.normal(n, 61 + n)
            dA, dB = dev(A), dev(B)
            C0 = torch.full((n, n), float("nan"), dtype=torch.float32, device="cuda")
            C1 = torch.full((n, n), float("nan"), dtype=torch.float32, device="cuda")
            st = torch.cuda.Stream()
            torch.cuda.synchronize()
            S.stark_gemm_noalloc(dA, dB, C1, n, depth, p, st)
            st.synchronize()
            S.stark_gemm(ctx, dA, dB, C0, n, depth, p, st)
            st.synchronize()
            got, ref = C1.cpu().numpy(), C0.cpu().numpy()
            assert np.all(np.isfinite(got))
            assert np.array_equal(got, ref)
            err = oracle.rel_frobenius(got, oracle.gemm_f64(A, B))
            print(f"  rel_frob vs FP64 = {err:.3e}", flush=True)
            assert err <= (1.5 * 4.4e-6 * 2 ** depth if prec.startswith("bf16x3") else 1e-5) * \
                (2 if prec.endswith("_winograd") else 1)
    finally:
        S.stark_destroy(ctx)


def test_noalloc_integer_exact_and_auto_depth(S):
    n = 777
    A, B = inputs.integers(n, 70), inputs.integers(n, 71)
    dA, dB = dev(A), dev(B)
    C = torch.full((n, n), float("nan"), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    S.stark_gemm_noalloc(dA, dB, C, n, S.STARK_DEPTH_AUTO, S.STARK_BF16X3, None)
    torch.cuda.synchronize()
    exact = (A.astype(np.float64) @ B.astype(np.float64)).astype(np.float32)
    assert np.array_equal(C.cpu().numpy(), exact)


def test_noalloc_refuses_plans_beyond_the_scratch(S):
    n, depth = 2048, 2
    assert S.stark_workspace_size(n, depth, S.STARK_FP32) > S.STARK_NOALLOC_SCRATCH_BYTES
    dA = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    dB = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    C = torch.full((n, n), 7.0, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    rc = S.stark_gemm_noalloc_status(dA, dB, C, n, depth, S.STARK_FP32, None)
    assert rc == S.STARK_ENOMEM
    assert "allocation-free" in S.stark_last_error()
    torch.cuda.synchronize()
    assert bool(torch.all(C == 7.0))     # nothing ran
