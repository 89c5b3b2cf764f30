"""Batched launches and the serving engine on the GPU, through the C ABI.

Both paths run the same kernels as a single multiply, with the same plan per
problem, so their results must equal the single-call results bit for bit;
integer inputs must equal brute force; float inputs are checked against the
FP64 oracle on sampled rows.
"""
import os

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


def single(S, ctx, dA, dB, n, depth, prec):
    C = torch.full((n, n), float("nan"), dtype=torch.float32, device="cuda")
    S.stark_gemm(ctx, dA, dB, C, n, min(depth, S.stark_max_depth(n)), prec, None)
    torch.cuda.synchronize()
    return C.cpu().numpy()


# ---------------------------------------------------------------------------
# Batched
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec", [0, 1, 2, 16, 17])   # 16: Winograd's variant flag
def test_batched_integer_exact_and_equal_to_single(S, ctx, prec):
    sizes = [256, 384, 1000, 65, 300, 1024, 448, 128, 129, 512]
    depth = 2
    As = [inputs.integers(n, 100 + i) for i, n in enumerate(sizes)]
    Bs = [inputs.integers(n, 200 + i) for i, n in enumerate(sizes)]
    dA = [dev(a) for a in As]
    dB = [dev(b) for b in Bs]
    dC = [torch.full((n, n), float("nan"), dtype=torch.float32, device="cuda") for n in sizes]
    S.stark_gemm_batched(ctx, dA, dB, dC, sizes, depth, prec, None)
    torch.cuda.synchronize()
    for i, n in enumerate(sizes):
        C = dC[i].cpu().numpy()
        exact = (As[i].astype(np.float64) @ Bs[i].astype(np.float64)).astype(np.int64)   # exact: sums < 2^53
        assert np.array_equal(C.astype(np.int64), exact), (i, n)
        assert np.array_equal(C, single(S, ctx, dA[i], dB[i], n, depth, prec)), (i, n)


def test_batched_float_equal_to_single_and_replays(S, ctx):
    sizes = [1000, 256, 2048, 384, 777]
    depth = 2
    As = [inputs.uniform(n, 300 + i) for i, n in enumerate(sizes)]
    Bs = [inputs.uniform(n, 400 + i) for i, n in enumerate(sizes)]
    dA = [dev(a) for a in As]
    dB = [dev(b) for b in Bs]
    dC = [torch.empty((n, n), dtype=torch.float32, device="cuda") for n in sizes]
    st = torch.cuda.Stream()
    outs = []
    for rep in range(4):           # eager, capture, two replays
        for c in dC:
            c.fill_(float("nan"))
        torch.cuda.synchronize()
        S.stark_gemm_batched(ctx, dA, dB, dC, sizes, depth, 1, st)
        st.synchronize()
        outs.append([c.cpu().numpy().copy() for c in dC])
    for rep in outs[1:]:
        for a, b in zip(outs[0], rep):
            assert np.array_equal(a, b)
    for i, n in enumerate(sizes):
        assert np.array_equal(outs[0][i], single(S, ctx, dA[i], dB[i], n, depth, 1)), i


@pytest.mark.parametrize("prec", [0, 1, 3])
def test_batched_auto_depth_per_problem(S, tmp_path, prec):
    """STARK_DEPTH_AUTO in a batch: a problem with an autotuner record runs
    at it (here n = 2048, from the cache file: depth 1, 128-wide tiles), the
    others at the batch planner's plans (stark_plan_batched: one tile class
    for all of them here); each result equals the single call with the same
    depth and tile class (given to a second context as records) bit for
    bit."""
    sizes = [256, 1000, 2048, 3000, 4096, 700]
    path = tmp_path / f"tune_{prec}.txt"
    path.write_text(f"# n precision depth ms freivalds_error tile\n2048 {prec} 1 1.0 0.0 128\n")
    c = S.stark_create(0, tuner_cache=str(path))
    plans = S.stark_plan_batched(c, sizes, S.STARK_DEPTH_AUTO, prec)
    assert (plans[2].depth, plans[2].gemm_tile) == (1, 128)
    assert len({p.gemm_tile for i, p in enumerate(plans) if i != 2}) == 1
    assert len({p.depth for p in plans}) > 1                  # the batch mixes depths
    ref_path = tmp_path / f"ref_{prec}.txt"
    ref_path.write_text("# n precision depth ms freivalds_error tile\n" + "".join(
        f"{n} {prec} {p.depth} 1.0 0.0 {p.gemm_tile}\n" for n, p in zip(sizes, plans)))
    cref = S.stark_create(0, tuner_cache=str(ref_path))
    try:
        As = [inputs.uniform(n, 500 + i) for i, n in enumerate(sizes)]
        Bs = [inputs.uniform(n, 600 + i) for i, n in enumerate(sizes)]
        dA = [dev(a) for a in As]
        dB = [dev(b) for b in Bs]
        dC = [torch.full((n, n), float("nan"), dtype=torch.float32, device="cuda") for n in sizes]
        refs = []
        for i, n in enumerate(sizes):
            ref = torch.full((n, n), float("nan"), dtype=torch.float32, device="cuda")
            S.stark_gemm(cref, dA[i], dB[i], ref, n, S.STARK_DEPTH_AUTO, prec, None)
            refs.append(ref)
        torch.cuda.synchronize()
        for rep in range(3):                     # eager, capture, replay
            for x in dC:
                x.fill_(float("nan"))
            torch.cuda.synchronize()
            S.stark_gemm_batched(c, dA, dB, dC, sizes, S.STARK_DEPTH_AUTO, prec, None)
            torch.cuda.synchronize()
            for i, n in enumerate(sizes):
                assert torch.equal(dC[i], refs[i]), (rep, n)
        rows = inputs.sample_rows(3000, 16, 9)
        err = oracle.rel_frobenius(dC[3].cpu().numpy()[rows], oracle.rows_f64(As[3], Bs[3], rows))
        assert err < (2e-5 if prec == 1 else 2e-6)
    finally:
        S.stark_destroy(c)
        S.stark_destroy(cref)


def test_batched_auto_mixed_tile_classes(S):
    """A batch the planner splits over two tile classes (BF16X3: one 4096
    problem on 256-wide tiles, 100 problems of 64 on 64-wide ones, where
    padding them to 256 would cost 64 times their work): integer inputs,
    every result exact, eager, captured and replayed."""
    sizes = [4096] + [64] * 100
    plans = S.stark_plan_batched(None, sizes, S.STARK_DEPTH_AUTO, 1)
    assert plans[0].gemm_tile == 256 and {p.gemm_tile for p in plans[1:]} == {64}
    c = S.stark_create(0)
    try:
        As = [inputs.integers(n, 700 + i, -8, 8) for i, n in enumerate(sizes)]
        Bs = [inputs.integers(n, 900 + i, -8, 8) for i, n in enumerate(sizes)]
        exact = [(a.astype(np.float64) @ b.astype(np.float64)).astype(np.float32) for a, b in zip(As, Bs)]
        dA = [dev(a) for a in As]
        dB = [dev(b) for b in Bs]
        for rep in range(3):
            dC = [torch.full((n, n), float("nan"), dtype=torch.float32, device="cuda") for n in sizes]
            torch.cuda.synchronize()
            S.stark_gemm_batched(c, dA, dB, dC, sizes, S.STARK_DEPTH_AUTO, 1, None)
            torch.cuda.synchronize()
            for i in range(len(sizes)):
                assert np.array_equal(dC[i].cpu().numpy(), exact[i]), (rep, i)
    finally:
        S.stark_destroy(c)


def test_batched_64_uneven_problems(S):
    """64 problems, n drawn from {256, 384, 1000, 1024, 2048, 3000, 4096}, FP32,
    uniform[-1, 1]; every problem against the FP64 oracle on sampled rows."""
    rng = np.random.default_rng(4)
    sizes = [int(x) for x in rng.choice([256, 384, 1000, 1024, 2048, 3000, 4096], size=64)]
    depth = 2
    c = S.stark_create(0)
    try:
        As = [inputs.uniform(n, 1000 + i) for i, n in enumerate(sizes)]
        Bs = [inputs.uniform(n, 2000 + i) for i, n in enumerate(sizes)]
        dA = [dev(a) for a in As]
        dB = [dev(b) for b in Bs]
        dC = [torch.empty((n, n), dtype=torch.float32, device="cuda") for n in sizes]
        S.stark_gemm_batched(c, dA, dB, dC, sizes, depth, 0, None)
        torch.cuda.synchronize()
        worst = 0.0
        for i, n in enumerate(sizes):
            rows = inputs.sample_rows(n, 4, 3000 + i)
            ref = oracle.rows_f64(As[i], Bs[i], rows)
            got = dC[i][torch.from_numpy(rows).cuda()].cpu().numpy().astype(np.float64)
            err = np.sqrt(np.sum((got - ref) ** 2) / np.sum(ref ** 2))
            worst = max(worst, err)
            assert err < 1e-5, (i, n, err)
        print(f"worst sampled-row rel error over 64 problems: {worst:.2e}")
        # spot-check bitwise equality with single calls
        for i in (0, 17, 63):
            assert np.array_equal(dC[i].cpu().numpy(), single(S, c, dA[i], dB[i], sizes[i], depth, 0))
    finally:
        S.stark_destroy(c)


# ---------------------------------------------------------------------------
# Serving
# ---------------------------------------------------------------------------
def wait(S, c, tickets):
    res = {}
    pending = list(tickets)
    while pending:
        nxt = []
        for t in pending:
            r = S.stark_poll(c, t)
            if r is None:
                nxt.append(t)
            else:
                res[t] = r
        pending = nxt
    return res


def test_serving_alone_vs_mix_bitwise(S):
    c = S.stark_create(0, hbm_budget_bytes=8 << 30, max_slots=6)
    try:
        rng = np.random.default_rng(7)
        reqs = []
        for i in range(18):
            n = int(rng.choice([128, 200, 512, 777, 1024, 2048]))
            prec = int(rng.choice([0, 1, 17]))     # 17: BF16X3, Winograd's variant
            A, B = inputs.normal(n, 50 + i), inputs.normal(n, 90 + i)
            reqs.append((n, prec, dev(A), dev(B), A, B))
        alone = []
        torch.cuda.synchronize()       # caller-owned operands must be complete before stark_submit
        for n, prec, dA, dB, _, _ in reqs:
            C = torch.empty((n, n), dtype=torch.float32, device="cuda")
            t = S.stark_submit(c, n, prec, S.STARK_DEPTH_AUTO, dA, dB, C, tag=n)
            wait(S, c, [t])
            alone.append(C.cpu().numpy())
        mixC = [torch.full((n, n), float("nan"), dtype=torch.float32, device="cuda") for n, *_ in reqs]
        # the NaN fills run on torch's stream; the engine's slot streams do not
        # wait for it, so the fills must be complete before the requests go in
        torch.cuda.synchronize()
        tickets = [S.stark_submit(c, n, prec, S.STARK_DEPTH_AUTO, dA, dB, C, tag=i)
                   for i, ((n, prec, dA, dB, _, _), C) in enumerate(zip(reqs, mixC))]
        res = wait(S, c, tickets)
        st = S.stark_stats(c)
        assert st.completed == 2 * len(reqs) and st.failed == 0
        assert st.max_concurrent > 1, "requests never overlapped"
        for i, (C, a) in enumerate(zip(mixC, alone)):
            assert np.array_equal(C.cpu().numpy(), a), i
        # and equal to the single-call path at the depth the engine used
        for i in (0, 5, 11):
            n, prec, dA, dB, A, B = reqs[i]
            d = res[tickets[i]].depth
            C = torch.empty((n, n), dtype=torch.float32, device="cuda")
            S.stark_gemm(c, dA, dB, C, n, d, prec, None)
            torch.cuda.synchronize()
            assert np.array_equal(C.cpu().numpy(), alone[i])
        assert st.p99_ms >= st.p50_ms > 0
    finally:
        S.stark_destroy(c)


def test_serving_peeled_sizes_equal_single_calls(S):
    """Served requests of sizes off the grid run the plan the planner gives
    them (peeled here: residues 1, 7 and 63 with STARK_PEEL), alone and
    together, and equal stark_gemm with that plan bit for bit."""
    c = S.stark_create(0, hbm_budget_bytes=8 << 30, max_slots=4)
    try:
        cases = [(2049, 2, 0 | 64), (1031, 1, 1 | 64), (1087, 1, 3 | 64), (4097, 2, 0)]
        assert [S.stark_plan_info(n, d, p).peel for n, d, p in cases] == [1, 7, 63, 1]
        ops = [(dev(inputs.normal(n, 300 + i)), dev(inputs.normal(n, 400 + i))) for i, (n, _, _) in enumerate(cases)]
        outs = [torch.full((n, n), float("nan"), dtype=torch.float32, device="cuda") for n, _, _ in cases]
        torch.cuda.synchronize()
        tickets = [S.stark_submit(c, n, p, d, dA, dB, C, tag=i)
                   for i, ((n, d, p), (dA, dB), C) in enumerate(zip(cases, ops, outs))]
        res = wait(S, c, tickets)
        assert all(r.status == S.STARK_OK for r in res.values())
        for (n, d, p), (dA, dB), C in zip(cases, ops, outs):
            assert np.array_equal(C.cpu().numpy(), single(S, c, dA, dB, n, d, p))
    finally:
        S.stark_destroy(c)


def test_serving_generated_operands_and_checksums(S):
    c = S.stark_create(0, hbm_budget_bytes=8 << 30, max_slots=4)
    try:
        spec = [(300, 1, 11), (640, 0, 12), (1024, 1, 13), (2000, 0, 14), (256, 2, 15)]
        alone = {}
        for n, p, seed in spec:
            t = S.stark_submit(c, n, p, S.STARK_DEPTH_AUTO, seed=seed, tag=seed)
            alone[seed] = wait(S, c, [t])[t].checksum
        tickets = [S.stark_submit(c, n, p, S.STARK_DEPTH_AUTO, seed=seed, tag=seed) for n, p, seed in spec * 3]
        res = wait(S, c, tickets)
        for t, r in res.items():
            assert r.checksum == alone[r.tag]
        # the checksum is the sum of C = (1^T A)(B 1); A, B from the host twin
        for n, p, seed in spec[:3]:
            A = inputs.philox_normal(n, 2 * seed).astype(np.float64)
            B = inputs.philox_normal(n, 2 * seed + 1).astype(np.float64)
            ref = A.sum(axis=0) @ B.sum(axis=1)
            bound = 1e-4 * n * np.sqrt(n) * n   # n * ||E||_F with ||E||_F <= 1e-4 ||C||_F
            assert abs(alone[seed] - ref) <= bound, (n, alone[seed], ref)
    finally:
        S.stark_destroy(c)


@pytest.mark.parametrize("n,prec,seed", [(300, 1, 21), (1024, 0, 22), (2000, 3, 23), (777, 17, 24)])
def test_serving_generated_operands_match_oracle_rows(S, n, prec, seed):
    """Operands generated on the device from a seed, result into a
    caller-owned C: sampled rows against the FP64 oracle on the host twin of
    the generator (Philox4x32-10, bit-identical operands), element by element
    through the relative Frobenius error of the rows."""
    c = S.stark_create(0, hbm_budget_bytes=8 << 30, max_slots=2)
    try:
        C = torch.full((n, n), float("nan"), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        t = S.stark_submit(c, n, prec, S.STARK_DEPTH_AUTO, C=C, seed=seed, tag=seed)
        r = wait(S, c, [t])[t]
        A = inputs.philox_normal(n, 2 * seed)
        B = inputs.philox_normal(n, 2 * seed + 1)
        rows = inputs.sample_rows(n, 64, seed)
        ref = oracle.rows_f64(A, B, rows)
        got = C.cpu().numpy()[rows].astype(np.float64)
        d = got - ref
        err = float(np.sqrt(np.sum(d * d) / np.sum(ref * ref)))
        print(f"served n={n} prec={prec} depth {r.depth}: rel_frob(64 rows)={err:.3e}")
        bound = 1.5 * 4.4e-6 * 2 ** r.depth * (2 if prec & 16 else 1) if (prec & 15) == 1 else 1e-5
        assert np.all(np.isfinite(got)) and err <= bound
    finally:
        S.stark_destroy(c)


def test_serving_stats_reset(S):
    """stark_stats_reset starts a new window: only requests finished after it
    count, and the latency percentiles come from them alone."""
    c = S.stark_create(0, hbm_budget_bytes=4 << 30, max_slots=2)
    try:
        S.stark_stats_reset(c)                    # no engine yet: accepted, no effect
        wait(S, c, [S.stark_submit(c, 1024, 0, 0, seed=s, tag=s) for s in range(6)])
        st = S.stark_stats(c)
        assert st.completed == 6 and st.p50_ms > 0
        S.stark_stats_reset(c)
        st = S.stark_stats(c)
        assert st.completed == 0 and st.failed == 0 and st.p50_ms == 0 and st.throughput_tflops == 0
        wait(S, c, [S.stark_submit(c, 256, 1, 0, seed=s, tag=s) for s in range(3)])
        st = S.stark_stats(c)
        assert st.completed == 3 and st.p99_ms > 0 and st.throughput_tflops > 0
    finally:
        S.stark_destroy(c)


def test_serving_concurrent_submitters(S):
    """Four host threads submit and poll at once: every request completes and
    its checksum equals the one it gets alone."""
    import threading
    c = S.stark_create(0, hbm_budget_bytes=4 << 30, max_slots=4)
    try:
        spec = [(256 + 64 * (i % 5), i % 2, 500 + i) for i in range(24)]
        alone = {}
        for n, p, seed in spec:
            t = S.stark_submit(c, n, p, S.STARK_DEPTH_AUTO, seed=seed, tag=seed)
            alone[seed] = wait(S, c, [t])[t].checksum
        got, errors = {}, []

        def worker(part):
            try:
                ts = [S.stark_submit(c, n, p, S.STARK_DEPTH_AUTO, seed=seed, tag=seed) for n, p, seed in part]
                for t, r in wait(S, c, ts).items():
                    got[r.tag] = r.checksum
            except Exception as e:      # surfaced below
                errors.append(e)

        threads = [threading.Thread(target=worker, args=(spec[k::4],)) for k in range(4)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        assert not errors, errors
        assert got == alone
    finally:
        S.stark_destroy(c)


def test_serving_admission_respects_budget(S):
    budget = 64 << 20
    c = S.stark_create(0, hbm_budget_bytes=budget, max_slots=8)
    try:
        tickets = [S.stark_submit(c, 1024, 1, 1, seed=i, tag=i) for i in range(10)]
        wait(S, c, tickets)
        st = S.stark_stats(c)
        assert st.completed == 10
        assert st.max_inflight_bytes <= budget
        with pytest.raises(S.StarkError) as e:
            S.stark_submit(c, 4096, 0, 2, seed=1)
        assert e.value.status == S.STARK_ENOMEM
        rc, _ = S.stark_poll_status(c, 123456789)
        assert rc == S.STARK_ENOTFOUND
    finally:
        S.stark_destroy(c)


def test_serving_arena_grows_and_is_replaced_when_idle(S):
    """The engine takes device memory in segments as admissions need it (4 GiB
    each, within the budget).  A request larger than a segment gets one of its
    own; when the budget is taken by segments too small for it, it waits until
    nothing is in flight and the empty segments are replaced."""
    budget = 6 << 30
    c = S.stark_create(0, hbm_budget_bytes=budget, max_slots=4)
    try:
        small = [S.stark_submit(c, 1024, 0, 0, seed=i, tag=i) for i in range(4)]
        big = S.stark_submit(c, 19200, 0, 0, seed=99, tag=99)      # 3 x 1.47 GB > 4 GiB
        more = [S.stark_submit(c, 512, 1, 0, seed=10 + i, tag=10 + i) for i in range(4)]
        res = wait(S, c, small + [big] + more)
        assert all(r.status == S.STARK_OK for r in res.values())
        st = S.stark_stats(c)
        assert st.completed == 9 and st.failed == 0
        assert st.max_inflight_bytes <= budget
        big_sum = res[big].checksum
    finally:
        S.stark_destroy(c)
    # the same request alone in an engine with room to spare: the same result
    c = S.stark_create(0, hbm_budget_bytes=16 << 30, max_slots=1)
    try:
        t = S.stark_submit(c, 19200, 0, 0, seed=99, tag=99)
        assert wait(S, c, [t])[t].checksum == big_sum
    finally:
        S.stark_destroy(c)


def test_serving_injected_failure_is_isolated(S, monkeypatch):
    monkeypatch.setenv("STARK_FAULT_INJECT", "3")
    c = S.stark_create(0, hbm_budget_bytes=2 << 30, max_slots=4)
    try:
        tickets = [S.stark_submit(c, 512, 1, 1, seed=i, tag=i) for i in range(6)]
        out = {}
        pending = list(tickets)
        while pending:
            nxt = []
            for t in pending:
                rc, r = S.stark_poll_status(c, t)
                if rc == S.STARK_PENDING:
                    nxt.append(t)
                else:
                    out[r.tag] = rc
            pending = nxt
        assert out[3] == S.STARK_EDEVICE
        assert all(out[i] == S.STARK_OK for i in range(6) if i != 3)
        st = S.stark_stats(c)
        assert st.failed == 1 and st.completed == 5
    finally:
        S.stark_destroy(c)
