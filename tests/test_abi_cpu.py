"""The C-ABI library without a GPU: it loads, exports every symbol the header
declares, and its pure host functions (planner, argument checks) behave."""
import ctypes
import subprocess

import numpy as np
import pytest

from paper_1811_07325_amd import build as _build  # noqa: F401  (import check)


@pytest.fixture(scope="module")
def S():
    import os
    from paper_1811_07325_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    from paper_1811_07325_amd import stark
    return stark


def test_exports_every_header_symbol(S):
    declared = S.header_symbols()
    assert len(declared) >= 16
    out = subprocess.run(["nm", "-D", "--defined-only", S.LIB_PATH], capture_output=True, text=True, check=True)
    exported = {l.split()[-1] for l in out.stdout.splitlines() if " T " in l}
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    lib = ctypes.CDLL(S.LIB_PATH)
    for s in declared:
        assert getattr(lib, s) is not None


def test_max_depth(S):
    assert S.stark_max_depth(512) == 3
    assert S.stark_max_depth(16384) == 7
    assert S.stark_max_depth(384) == 1
    assert S.stark_max_depth(1000) == 4
    assert S.stark_max_depth(64) == 0
    assert S.stark_max_depth(0) == 0


def _regions(d, depth):
    regs = []
    for l in range(depth):
        if d.div_a[l] >= 0:
            regs.append(("div_a%d" % l, d.div_a[l]))
            regs.append(("div_b%d" % l, d.div_b[l]))
    for name in ("leaf_a", "leaf_b", "leaf_m", "pad_a", "pad_b", "scale"):
        if getattr(d, name) >= 0:
            regs.append((name, getattr(d, name)))
    return sorted(regs, key=lambda r: r[1])


@pytest.mark.parametrize("prec", [0, 1, 2, 3, 16, 17, 19, 32, 33, 48, 64, 65, 83, 128])
@pytest.mark.parametrize("n,depth", [(512, 2), (4096, 3), (1000, 2), (384, 1), (16384, 4), (65, 0), (3000, 3),
                                     (4096, 1), (4032, 1), (4032, 2), (8192, 2), (16385, 2), (1031, 2),
                                     (4097, 1), (4160, 2), (8255, 3)])
def test_plan_layout(S, n, depth, prec):
    d = S.stark_plan_info(n, depth, prec)
    np_ = d.n_pad
    # a peeled plan runs the recursion on the core n - peel, a padded one on
    # the next multiple of 64 * 2^depth
    assert np_ == n - d.peel if d.peel else np_ >= n
    assert np_ % (64 << depth) == 0 and d.leaf == np_ >> depth
    winograd = bool(prec & S.STARK_WINOGRAD)
    assert d.variant == int(winograd)
    fused_flag = bool(prec & S.STARK_FUSED)
    g, r = 64 << depth, n % (64 << depth)
    can_peel = depth >= 1 and 1 <= r <= 64 and n - r >= g
    if can_peel and prec & S.STARK_PEEL:
        assert d.peel == r
    elif not can_peel or prec & S.STARK_PAD:
        assert d.peel == 0
    else:                      # the planner's time model chooses
        assert d.peel in (0, r)
    if d.peel:
        assert d.peel_flops == 2 * n * r * (n + np_) + 2 * r * np_ * np_
    else:
        assert d.peel_flops == 0
    prec &= 15
    planes = {0: 0, 1: 2, 2: 3, 3: 2}[prec]
    assert d.planes == planes
    # STARK_FUSED with binary32 Algorithm 1 on 256-wide tiles: the leaf GEMM
    # forms the last level's operands (not at depth 1 of a padded size), so
    # the divide stores one level fewer; elsewhere the flag is ignored
    # level 0 read element by element: padded sizes, and peeled ones whose
    # rows are not 16-byte aligned
    bounded = np_ != n and not (d.peel and n % 4 == 0)
    fused = (planes == 0 and not winograd and fused_flag and d.gemm_tile == 256 and depth >= 1
             and not (depth == 1 and bounded))
    assert d.fused == int(fused)
    stored = depth - 1 if fused else depth
    L, h = d.leaf, None
    # sizes of every region, from the layout rules
    size = {}
    # 16-bit paths: the split forms the last level (the last two from depth 2)
    fp32_levels = stored if planes == 0 else max(depth - 2, 0)
    # binary32 from two stored levels on: level stored-2 is formed on the fly
    # by the divide of level stored-1, which stores all seven operands
    unstored = stored - 2 if (planes == 0 and stored >= 2) else None
    for l in range(depth):
        if l < fp32_levels and l != unstored:
            h = (np_ >> l) // 2
            slots = 7 if (l == 0 and bounded) or (unstored is not None and l == stored - 1) else 4 if winograd else 5
            assert d.div_slots[l] == slots
            size["div_a%d" % l] = size["div_b%d" % l] = slots * 7 ** l * h * h * 4
        else:
            assert d.div_a[l] == -1 and d.div_slots[l] == 0
    if planes:
        nodes_out = 7 ** depth
        size["leaf_a"] = size["leaf_b"] = nodes_out * planes * L * L * 2
    if depth > 0:
        size["leaf_m"] = 7 ** depth * L * L * 4
    else:
        assert d.leaf_m == -1
    if d.pad_a >= 0:
        assert depth == 0 and planes == 0 and np_ != n
        size["pad_a"] = size["pad_b"] = np_ * np_ * 4
    if prec == 3:
        size["scale"] = (2 * 256 + 2) * 4
    else:
        assert d.scale == -1
    regs = _regions(d, depth)
    assert {r[0] for r in regs} == set(size)
    # live regions are disjoint and inside the workspace
    for (a, oa), (b, ob) in zip(regs, regs[1:]):
        assert oa + size[a] <= ob, (a, b)
    last = regs[-1] if regs else None
    if last:
        assert last[1] + size[last[0]] <= d.bytes
    # combine outputs: disjoint from each other and from the leaf products
    comb = [(l, d.comb[l]) for l in range(1, depth - 1)]
    if depth >= 2:
        assert d.comb[depth - 1] == -1      # combined together with level depth-2
    ends = []
    for l, off in comb:
        m = np_ >> l
        ends.append((off, off + 7 ** l * m * m * 4))
    ends.sort()
    for (a0, a1), (b0, b1) in zip(ends, ends[1:]):
        assert a1 <= b0
    for a0, a1 in ends:
        assert a1 <= d.leaf_m
        if d.scale >= 0:       # the combine outputs never overwrite the scale region
            assert a0 >= d.scale + size["scale"]


def test_peel_rule(S):
    """Residues r = n mod (64 * 2^depth) up to 64 can be peeled: always with
    STARK_PEEL, never with STARK_PAD, and by default when the planner's time
    model finds it faster than every padded plan (padding to a multiple of
    64, 128 or 256 times 2^depth); at n = 16384 + r the padded plans do more
    work or run narrower tiles, so every r <= 64 peels; at n = 257, depth 1,
    the border's extra launch costs more than the padded edge; depth 0 and
    sizes below one granule always pad; the peeled core needs the workspace
    of its own size (level 0 read element by element, so all seven operands
    stored)."""
    P = lambda n, depth, flags=0: S.stark_plan_info(n, depth, flags)
    assert (P(16385, 2).peel, P(16385, 2).n_pad) == (1, 16384)
    assert (P(16391, 2).peel, P(16391, 2).n_pad) == (7, 16384)
    assert (P(16448, 2).peel, P(16448, 2).n_pad) == (64, 16384)
    # padded, the planner avoids the multiple of 64 * 2^depth (16640: leaves
    # of 4160 for the 64-wide tiles) and takes the multiple of 256 * 2^depth
    # (17408, 256-wide tiles) over that of 128 * 2^depth (16896, 128-wide
    # tiles, 9 % fewer flops at a fifth less rate), both leaf types
    FP16X3 = S.STARK_FP16X3
    assert (P(16448, 2, FP16X3 | S.STARK_PAD).peel, P(16448, 2, FP16X3 | S.STARK_PAD).n_pad) == (0, 17408)
    assert P(16448, 2, FP16X3 | S.STARK_PAD).gemm_tile == 256 and P(16448, 2).gemm_tile == 256
    assert (P(16448, 2, S.STARK_PAD).n_pad, P(16448, 2, S.STARK_PAD).gemm_tile) == (17408, 256)
    assert (P(16000, 2, S.STARK_PAD).n_pad, P(16000, 2, S.STARK_PAD).gemm_tile) == (16384, 256)
    assert (P(16500, 2, FP16X3).peel, P(16500, 2, FP16X3).n_pad, P(16500, 2, FP16X3).gemm_tile) == (0, 17408, 256)
    assert (P(4032, 0).n_pad, P(4032, 0).gemm_tile) == (4096, 256)
    assert (P(257, 1).peel, P(257, 1).n_pad) == (0, 384)
    assert (P(1087, 1, S.STARK_PEEL).peel, P(1087, 1, S.STARK_PEEL).n_pad) == (63, 1024)
    assert P(16447, 2, S.STARK_PEEL).peel == 63
    assert P(16449, 2, S.STARK_PEEL).peel == 0          # residue 65: padded
    assert P(16385, 2, FP16X3 | S.STARK_PAD).peel == 0 and P(16385, 2, FP16X3 | S.STARK_PAD).n_pad == 17408
    assert P(16385, 0).peel == 0 and P(16385, 0).n_pad in (16448, 16512, 16640)
    assert P(257, 1, S.STARK_PEEL).peel == 1 and P(257, 1, S.STARK_PEEL).n_pad == 256
    assert P(100, 1, S.STARK_PEEL).peel == 0 and P(100, 1).n_pad == 128     # no core of 128 to recurse on
    with pytest.raises(S.StarkError):
        S.stark_plan_info(16385, 2, S.STARK_PEEL | S.STARK_PAD)
    for n, depth, prec in [(16385, 2, 0), (4103, 1, 1), (8199, 3, 3)]:
        d = P(n, depth, prec)
        assert d.peel > 0
        core = P(n - d.peel, depth, prec)
        assert d.bytes >= core.bytes and d.div_slots[0] in ((0, 7) if n % 4 else (0, 4, 5))


def test_workspace_formula_fp32(S):
    """Unpadded binary32 with stored leaf operands, depth k >= 2: levels
    0..k-3 store 5 blocks per node and side, (5/4)(7/4)^l N floats each;
    level k-2 is not stored; level k-1 stores 7, (7/4)^k N; plus the
    (7/4)^k N leaf products."""
    for n, k in [(4096, 3), (16384, 2), (8192, 4), (512, 3)]:
        N = n * n
        expect = (2 * sum(1.25 * (7 / 4) ** l for l in range(k - 2)) + 2 * (7 / 4) ** k + (7 / 4) ** k) * N * 4
        got = S.stark_workspace_size(n, k, 0)
        assert abs(got - expect) <= 256 * (4 * k + 2)
        if S.stark_plan_info(n, k, S.STARK_FUSED).gemm_tile != 256:      # the flag does not apply: the same plan
            assert S.stark_workspace_size(n, k, S.STARK_FUSED) == got


def test_workspace_formula_fp32_fused(S):
    """Unpadded binary32 with fused leaf operands (256-wide tiles), depth k:
    the divide stores the levels of depth k - 1 -- k = 1: nothing; k = 2:
    level 0 with 5 blocks per node and side; k >= 3: levels 0..k-4 with 5,
    level k-3 not stored, level k-2 with all 7, (7/4)^(k-1) N -- plus the
    (7/4)^k N leaf products."""
    for n, k in [(4096, 1), (16384, 2), (4096, 3), (16384, 3), (8192, 4)]:
        assert S.stark_plan_info(n, k, S.STARK_FUSED).fused == 1
        assert S.stark_plan_info(n, k, 0).fused == 0
        N = n * n
        j = k - 1
        if j == 0:
            div = 0.0
        elif j == 1:
            div = 2 * 1.25
        else:
            div = 2 * sum(1.25 * (7 / 4) ** l for l in range(j - 2)) + 2 * (7 / 4) ** j
        expect = (div + (7 / 4) ** k) * N * 4
        got = S.stark_workspace_size(n, k, S.STARK_FUSED)
        assert abs(got - expect) <= 256 * (4 * k + 2)
        assert got < S.stark_workspace_size(n, k, 0)


def test_winograd_flag_and_unknown_bits(S):
    """The Winograd flag combines with every precision; other bits are
    rejected.  Winograd stores 4 operand blocks per node and side, not 5."""
    for prec in (0, 1, 2, 3):
        d = S.stark_plan_info(4096, 3, prec | S.STARK_WINOGRAD)
        assert d.variant == 1 and d.precision == prec | S.STARK_WINOGRAD
    d5, d4 = S.stark_plan_info(4096, 3, 1), S.stark_plan_info(4096, 3, 1 | S.STARK_WINOGRAD)
    assert d5.div_slots[0] == 5 and d4.div_slots[0] == 4
    assert d4.divide_bytes < d5.divide_bytes and d4.split_bytes == d5.split_bytes
    for bad in (256, 4, 15, 256 | 1):
        with pytest.raises(S.StarkError):
            S.stark_workspace_size(512, 1, bad)


def test_invalid_arguments_are_rejected(S):
    with pytest.raises(S.StarkError) as e:
        S.stark_workspace_size(0, 0, 0)
    assert e.value.status == S.STARK_EINVAL
    with pytest.raises(S.StarkError):
        S.stark_workspace_size(512, 9, 0)
    with pytest.raises(S.StarkError):
        S.stark_workspace_size(512, 1, 7)
    assert "precision" in S.stark_last_error()


def test_create_without_gpu_reports_device_error(S):
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(S.StarkError) as e:
        S.stark_create(0)
    assert e.value.status == S.STARK_EDEVICE


def test_tile_class_choice(S):
    # 256-wide tiles for leaves that fill the chip with them
    assert S.stark_plan_info(16384, 2, 1).gemm_tile == 256
    assert S.stark_plan_info(16384, 4, 2).gemm_tile == 256
    assert S.stark_plan_info(16384, 2, 0).gemm_tile == 256
    assert S.stark_plan_info(16384, 3, 0).gemm_tile == 256
    assert S.stark_plan_info(4096, 3, 0).gemm_tile == 256   # 343 leaves of 512
    assert S.stark_plan_info(4096, 0, 0).gemm_tile == 256
    assert S.stark_plan_info(4096, 1, 1).gemm_tile == 256
    assert S.stark_plan_info(2048, 1, 1).gemm_tile == 128
    assert S.stark_plan_info(512, 2, 1).gemm_tile == 64    # 49 leaves of 128: more, smaller tiles
    assert S.stark_plan_info(2048, 1, 0).gemm_tile == 128
    assert S.stark_plan_info(384, 1, 1).gemm_tile == 64
    # 256-wide tiles down to about 3/4 of a wave (196 and 252 tiles), 64-wide
    # below about 3/4 of two waves of 128-wide tiles (256 tiles)
    assert S.stark_plan_info(2048, 2, 0).gemm_tile == 256   # 49 leaves of 512: 196 tiles
    assert S.stark_plan_info(3000, 1, 1).gemm_tile == 256   # 7 leaves of 1536: 252 tiles
    assert S.stark_plan_info(2048, 0, 1).gemm_tile == 64    # 256 tiles of 128
    for n in (256, 1000, 2048, 3000, 4096, 8192, 16384):
        for d in range(S.stark_max_depth(n) + 1):
            pl = S.stark_plan_info(n, d, 1)
            assert pl.leaf % pl.gemm_tile == 0


def test_model_depth(S):
    """The depth used for served requests without an autotuner record."""
    for n in (64, 128, 700, 1000, 2048, 2500, 3000, 4096, 6000, 8192, 16384, 20000):
        for p in (0, 1, 2, 3, 16, 17):
            d = S.stark_model_depth(n, p)
            assert 0 <= d <= min(3, S.stark_max_depth(n))
            if p & 15 == 1:
                assert d <= 1           # BF16X3's error roughly doubles per level
    for n in (128, 512, 1000, 1024):
        assert S.stark_model_depth(n, 0) == 0 and S.stark_model_depth(n, 1) == 0   # launches dominate
    # measured best depths (one MI355X): binary32 0 at 4096, 2 at 8192 (depth 1
    # within 2 %: 7.33 against 7.21 ms), 3 at 16384; BF16X3 1 at 3000 (7
    # leaves of 1536 on 256-wide tiles beat one 3072 leaf on 128-wide ones)
    assert S.stark_model_depth(4096, 0) == 0
    assert S.stark_model_depth(8192, 0) in (1, 2)
    assert S.stark_model_depth(16384, 0) == 3
    assert S.stark_model_depth(3000, 1) == 1
    assert S.stark_model_depth(0, 0) == -1 and S.stark_model_depth(100, 999) == -1


def test_generator_argument_errors(S):
    """The device generator refuses NULL, n <= 0 and misaligned X before
    touching the device."""
    for ptr, n in ((None, 4), (64, 0), (68, 4), (72, 4)):
        with pytest.raises(S.StarkError):
            S.stark_generate_normal(ptr, n, 1, None)


def test_plan_batched(S):
    """Plans of grouped multiplies at the automatic depth (no autotuner
    records): in a batch the other problems fill the waves, so each problem
    takes the depth and padding of least GEMM plus streaming time on a tile
    class, and the 64-problem workload of sizes {256, ..., 4096} runs on one
    class -- a single leaf-GEMM launch -- n = 384 padded to 512 for it (beyond
    the quarter a single multiply allows), 4096 recursing (binary32); a fixed
    depth plans every problem as stark_plan_info does; a batch whose small
    problems would pad 64 -> 256 keeps them on the 64-wide class."""
    rng = np.random.default_rng(7)
    sizes = [int(x) for x in rng.choice([256, 384, 1000, 1024, 2048, 3000, 4096], 64)]
    for prec in (0, 1, 3):
        plans = S.stark_plan_batched(None, sizes, S.STARK_DEPTH_AUTO, prec)
        assert {p.gemm_tile for p in plans} == {256}
        for n, p in zip(sizes, plans):
            assert p.n == n and p.n_pad >= n and p.n_pad % (256 << p.depth) == 0
            assert p.depth <= (1 if prec == 1 else 3)
        by = {n: p for n, p in zip(sizes, plans)}
        assert by[384].n_pad == 512 and S.stark_plan_info(384, 0, prec).n_pad == 384
    fp32 = {n: p for n, p in zip(sizes, S.stark_plan_batched(None, sizes, S.STARK_DEPTH_AUTO, 0))}
    assert fp32[4096].depth >= 1 and fp32[256].depth == 0
    fixed = S.stark_plan_batched(None, sizes, 1, 0)
    for n, p in zip(sizes, fixed):
        q = S.stark_plan_info(n, min(1, S.stark_max_depth(n)), 0)
        assert (p.depth, p.gemm_tile, p.n_pad, p.peel) == (q.depth, q.gemm_tile, q.n_pad, q.peel)
    mixed = S.stark_plan_batched(None, [4096] + [64] * 300, S.STARK_DEPTH_AUTO, S.STARK_BF16X3)
    assert mixed[0].gemm_tile == 256 and {p.gemm_tile for p in mixed[1:]} == {64}
    assert all(p.n_pad == 64 for p in mixed[1:])
    with pytest.raises(S.StarkError):
        S.stark_plan_batched(None, [], S.STARK_DEPTH_AUTO, 0)
    with pytest.raises(S.StarkError):
        S.stark_plan_batched(None, [256, 0], S.STARK_DEPTH_AUTO, 0)
    with pytest.raises(S.StarkError):
        S.stark_plan_batched(None, [256], S.STARK_DEPTH_AUTO, 999)


def test_plan_work_figures(S):
    """Algorithmic work reported by the planner against the formulas written
    out: BF16X3 depth 2 at n = 16384 (no binary32 level; the split reads A and
    B once and writes 49 leaf operands as two planes; one two-level combine
    pass) and FP32 depth 3 (divide level 0, then levels 1 and 2 in one pass;
    combine levels 2 and 1 in one pass, then level 0)."""
    E, n = 4.0, 16384
    d = S.stark_plan_info(n, 2, 1)
    L = n // 4
    assert d.divide_bytes == 0
    assert d.split_bytes == 2 * (n * n * E + 49 * 2 * L * L * 2)
    assert d.combine_bytes == (49 + 16) * L * L * E
    assert d.leaf_flops == 49 * 2.0 * L ** 3 and d.mfma_flops == 3 * d.leaf_flops
    d = S.stark_plan_info(n, 3, 0)
    L = n // 8
    # level 0 as usual; level 2 formed from the level-1 operands read once
    # (7 of edge n/2), all seven of its operands stored
    div = 2 * (4 + 5) * (n // 2) ** 2 * E + 2 * (7 * (n // 2) ** 2 + 49 * 7 * (n // 8) ** 2) * E
    assert d.divide_bytes == div                       # 20.1 GB
    assert d.split_bytes == 0
    assert d.combine_bytes == 7 * (49 + 16) * L * L * E + 11 * (n // 2) ** 2 * E
    assert d.mfma_flops == d.leaf_flops == 343 * 2.0 * L ** 3
