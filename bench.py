"""Benchmark of the Strassen hot path on one MI355X.

Default workload (one "step" = one full multiply: divide levels, split,
grouped leaf GEMM, combine levels): C = A B at n = 16384, A and B i.i.d.
normal(0, 1) in binary32, leaf products as three split products on the
16-bit matrix cores (FP16X3 or BF16X3, binary32 accumulation), recursion depth
autotuned among 2..4: the headline is the fastest (precision, depth, tile)
whose error against the product stays within 1e-5 (Freivalds' check in the
autotuner, then 256 sampled rows against the FP64 oracle).  BF16X3 keeps 16
significant bits and misses 1e-5 at every depth 2..4; it is reported beside
the headline with its errors.  Inputs are resident in HBM before the timed
region; the timed region is K back-to-back multiplies on one stream,
bracketed by device synchronisation.

Reported beside it, on the same GPU and inputs: the plain binary32 Strassen
path (autotuned depth), the classical product (depth 0, binary32 leaves),
BF16x3 at depths 1..4, BF16x6, classical split products, Winograd's variant,
a rectangular product and torch.matmul (external context), each with
Freivalds' check; the per-phase times with algorithmic bytes and flops at
every depth 1..4 (divide + split, leaf products, combine); the leaf GEMM's
roofline; the oracle's own speed on the host (sampled rows of this product,
plus full FP64 classical and Strassen products at n = 512 and 4096 on all
threads and at n = 512 and 1024 on one thread); a batched run (64
independent binary32 products of sizes drawn from {256, 384, 1000, 1024,
2048, 3000, 4096}, one grouped graph-captured launch sequence per depth);
and a serving run (Poisson stream of requests of mixed sizes and precisions)
with p50/p99 latency.

Prints ONE JSON line.  --gpus N > 1 is refused: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"bf16": 2.5e15, "fp32": 157.3e12, "hbm": 8.0e12}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--n", type=int, default=16384)
    p.add_argument("--precision", default="split3",
                   choices=["split3", "fp32", "bf16x3", "bf16x6", "fp16x3", "fp32_winograd", "bf16x3_winograd",
                            "bf16x6_winograd", "fp16x3_winograd"],
                   help="split3: the fastest of FP16X3 / BF16X3 within the error target")
    p.add_argument("--tol", type=float, default=1e-5, help="relative error target of the headline")
    p.add_argument("--min-depth", type=int, default=2)
    p.add_argument("--max-depth", type=int, default=4)
    p.add_argument("--depth", type=int, default=None, help="fixed depth (skips the autotuner)")
    p.add_argument("--no-compare", action="store_true", help="skip the FP32 / classical / BF16x6 legs")
    p.add_argument("--no-phase-table", action="store_true", help="skip the per-depth phase breakdown")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-serving", action="store_true")
    p.add_argument("--no-batched", action="store_true")
    p.add_argument("--no-peeling", action="store_true", help="skip the peeled-against-padded leg")
    p.add_argument("--batched-only", action="store_true",
                   help="only run the batched workload, print its JSON object and exit")
    p.add_argument("--serving-only", action="store_true",
                   help="only run the serving workload, print its JSON object and exit")
    p.add_argument("--serving-requests", type=int, default=2000)
    p.add_argument("--rows", type=int, default=256, help="sampled rows for the error check")
    p.add_argument("--cpu-rows", type=int, default=1024,
                   help="extra sampled rows the oracle computes for the CPU baseline timing")
    p.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "leaf_gemm_traffic.txt"),
                   help="HBM traffic of the leaf GEMM measured by rocprofv3 counters, if present")
    p.add_argument("--phase-reps", type=int, default=5, help="repetitions of each phase for the live roofline")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain 1 GiB device-to-device elementwise copy (counter calibration) and exit")
    return p.parse_args()


def run_serving(S, count: int, seed: int = 5, budget: int = 96 << 30, slots: int = 8) -> dict:
    """Poisson stream of `count` requests, n log-uniform in [128, 8192], 70 %
    BF16x3 / 30 % FP32, operands normal(0,1) generated on the device from
    per-request seeds.  The same request sequence is first run as a closed
    burst (all submitted at once) to measure the saturation rate; the stream
    then offers it at 0.7 x that rate."""
    rng = np.random.default_rng(seed)
    ns = np.exp(rng.uniform(math.log(128), math.log(8192), count)).astype(np.int64)
    ps = np.where(rng.uniform(size=count) < 0.7, S.STARK_BF16X3, S.STARK_FP32)
    work = float(np.sum(2.0 * ns.astype(np.float64) ** 3))

    def drain(ctx, tickets):
        pending = list(tickets)
        while pending:
            pending = [t for t in pending if S.stark_poll(ctx, t) is None]
            if pending:
                time.sleep(0.0005)

    def submit(ctx, i):
        return S.stark_submit(ctx, int(ns[i]), int(ps[i]), S.STARK_DEPTH_AUTO, seed=10000 + i, tag=i)

    # saturation: the whole sequence as a closed burst (after a short warm-up)
    ctx = S.stark_create(0, hbm_budget_bytes=budget, max_slots=slots)
    drain(ctx, [submit(ctx, i) for i in range(min(32, count))])
    t0 = time.perf_counter()
    drain(ctx, [submit(ctx, i) for i in range(count)])
    burst_s = time.perf_counter() - t0
    S.stark_destroy(ctx)
    sat = count / burst_s
    log(f"serving: saturation {sat:.0f} req/s ({work / burst_s * 1e-12:.1f} TF/s) for the closed burst")

    lam = 0.7 * sat
    arrivals = np.cumsum(rng.exponential(1.0 / lam, count))
    ctx = S.stark_create(0, hbm_budget_bytes=budget, max_slots=slots)
    # start the engine (device arena, slot streams) before the clock: its
    # first submission allocates the arena
    t_start = time.perf_counter()
    drain(ctx, [submit(ctx, i) for i in range(min(8, count))])
    log(f"serving: engine start and {min(8, count)} warm-up requests {1e3 * (time.perf_counter() - t_start):.1f} ms")
    S.stark_stats_reset(ctx)
    tickets = []
    t0 = time.perf_counter()
    for i in range(count):
        while time.perf_counter() - t0 < arrivals[i]:
            pass
        tickets.append(submit(ctx, i))
    drain(ctx, tickets)
    wall = time.perf_counter() - t0
    stt = S.stark_stats(ctx)
    S.stark_destroy(ctx)
    out = {"requests": count, "rate_req_s": lam, "saturation_req_s": sat, "p50_ms": stt.p50_ms,
           "p99_ms": stt.p99_ms, "throughput_tflops": stt.throughput_tflops, "completed": int(stt.completed),
           "failed": int(stt.failed), "max_concurrent": stt.max_concurrent,
           "max_inflight_gb": stt.max_inflight_bytes / 1e9, "wall_s": wall, "slots": slots,
           "budget_gb": budget / 2 ** 30, "offered_tflops": work / arrivals[-1] * 1e-12}
    log(f"serving: {count} requests at {lam:.0f} req/s: p50 {stt.p50_ms:.2f} ms, p99 {stt.p99_ms:.2f} ms, "
        f"{stt.throughput_tflops:.1f} TF/s, max concurrent {stt.max_concurrent}")
    return out


def run_batched(S, torch, st, count: int = 64, seed: int = 7) -> dict:
    """`count` independent products, sizes drawn from {256, 384, 1000, 1024,
    2048, 3000, 4096} (odd sizes padded), binary32 uniform[-1, 1] operands, in
    one stark_gemm_batched call (every leaf of every problem in one grouped
    launch, graph-captured), at depths 0..2 (clamped per problem) and with
    STARK_DEPTH_AUTO (the batch planner's depth, padding and tile class per
    problem); Freivalds' check on every product of the fastest setting."""
    from paper_1811_07325_amd import inputs
    rng = np.random.default_rng(seed)
    sizes = [int(x) for x in rng.choice([256, 384, 1000, 1024, 2048, 3000, 4096], count)]
    As = [torch.from_numpy(inputs.uniform(m, 2 * i)).cuda() for i, m in enumerate(sizes)]
    Bs = [torch.from_numpy(inputs.uniform(m, 2 * i + 1)).cuda() for i, m in enumerate(sizes)]
    Cs = [torch.empty((m, m), dtype=torch.float32, device="cuda") for m in sizes]
    flops = sum(2.0 * m ** 3 for m in sizes)
    ctx = S.stark_create(0)
    per_depth = []
    for depth in (0, 1, 2, S.STARK_DEPTH_AUTO):
        for _ in range(2):                     # eager, then captured
            S.stark_gemm_batched(ctx, As, Bs, Cs, sizes, depth, S.STARK_FP32, st)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(5):
            S.stark_gemm_batched(ctx, As, Bs, Cs, sizes, depth, S.STARK_FP32, st)
        e1.record(st)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / 5
        label = "auto" if depth == S.STARK_DEPTH_AUTO else depth
        per_depth.append({"depth": label, "ms": ms, "tflops": flops / (ms * 1e-3) * 1e-12})
        log(f"batched {count} fp32 depth {label}: {ms:.3f} ms, {flops / (ms * 1e-3) * 1e-12:.1f} TF/s")
    best = min(per_depth, key=lambda r: r["ms"])
    S.stark_gemm_batched(ctx, As, Bs, Cs, sizes, S.STARK_DEPTH_AUTO if best["depth"] == "auto" else best["depth"],
                         S.STARK_FP32, st)
    st.synchronize()
    worst = 0.0
    for i, m in enumerate(sizes):
        x = torch.from_numpy(inputs.gaussian_vector(m, 100 + i)).cuda()
        y = [torch.empty(m, dtype=torch.float64, device="cuda") for _ in range(3)]
        S.stark_matvec_f64(Bs[i], x, y[0], m, st)
        S.stark_matvec_f64(As[i], y[0], y[1], m, st)
        S.stark_matvec_f64(Cs[i], x, y[2], m, st)
        st.synchronize()
        worst = max(worst, float(torch.linalg.norm(y[2] - y[1]) / torch.linalg.norm(y[1])))
    S.stark_destroy(ctx)
    return {"problems": count, "sizes": sorted(set(sizes)), "precision": "fp32", "flops": flops,
            "depth": best["depth"], "ms": best["ms"], "tflops": best["tflops"], "per_depth": per_depth,
            "freivalds_max": worst}


COPY_BYTES = 1 << 30


def copy_calibration(torch) -> int:
    """A streaming kernel of known traffic: y = -x over 1 GiB of binary32
    (reads 1 GiB, writes 1 GiB), four times (the last three timed).  Hardware counters read on it
    give the factor that turns the same counters read on other kernels into
    bytes."""
    x = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.neg(x, out=y)
    e0.record()
    for _ in range(3):
        torch.neg(x, out=y)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / 3
    print(json.dumps({"copy_bytes": COPY_BYTES, "kernel": "neg", "reps": 4, "ms": ms,
                      "read_write_gbs": 2 * COPY_BYTES / (ms * 1e-3) * 1e-9}), flush=True)
    return 0


def read_traffic(path: str, key: str):
    """Leaf-GEMM HBM bytes per launch (fetch + write) recorded for `key`, or
    None when absent or taken on another version of the GEMM source."""
    if not os.path.exists(path):
        return None
    from paper_1811_07325_amd.profsum import source_digest
    digest = None
    for line in open(path):
        f = line.split()
        if line.startswith("# source_sha256"):
            digest = f[2]
        elif f and not line.startswith("#") and f[0] == key:
            if digest != source_digest():
                log(f"traffic for {key} was taken on another GEMM source: not reported")
                return None
            return float(f[1]) + float(f[2])
    return None


def cpu_table(oracle, inputs) -> dict:
    """The oracle's full FP64 products on the host, the analog of the
    single-node serial-naive / serial-Strassen columns of the paper's
    Table V: classical (i-t-j loop) and Strassen (Algorithm 1) at n = 512
    (depth 2) and 4096 (depth 3) on every OpenMP thread, and at n = 512 and
    1024 on one thread."""
    full = oracle.threads()
    rows = []
    for n_, d_, threads in ((512, 2, full), (4096, 3, full), (512, 2, 1), (1024, 2, 1)):
        A_, B_ = inputs.uniform(n_, 0), inputs.uniform(n_, 1)
        oracle.set_threads(threads)
        try:
            t0 = time.perf_counter()
            oracle.gemm_f64(A_, B_)
            tc = time.perf_counter() - t0
            t0 = time.perf_counter()
            oracle.strassen_f64(A_, B_, d_)
            ts = time.perf_counter() - t0
        finally:
            oracle.set_threads(full)
        f = 2.0 * n_ ** 3
        rows.append({"n": n_, "threads": threads, "classical_s": tc, "classical_gflops": f / tc * 1e-9,
                     "strassen_depth": d_, "strassen_s": ts, "strassen_gflops": f / ts * 1e-9})
        log(f"cpu oracle n={n_} threads={threads}: classical {tc:.2f} s ({f / tc * 1e-9:.2f} GF/s), "
            f"strassen depth {d_} {ts:.2f} s ({f / ts * 1e-9:.2f} GF/s)")
    return {"rows": rows, "note": "FP64, uniform[-1,1] inputs; the paper's Table V columns are serial naive "
                                  "and serial Strassen on one 2.60 GHz Xeon node (context only)"}


def host_info() -> dict:
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    return {"cpu_model": model, "nproc": nproc, "os_cpu_count": os.cpu_count()}


def main() -> int:
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1"}))
        return 2
    import torch

    if args.copy_calibration:
        return copy_calibration(torch)

    from paper_1811_07325_amd import inputs
    from paper_1811_07325_amd import stark as S

    n = args.n
    tol = args.tol
    dev = torch.device("cuda", 0)
    st = torch.cuda.Stream(device=dev)
    if args.batched_only:
        print(json.dumps(run_batched(S, torch, st)), flush=True)
        return 0
    if args.serving_only:
        print(json.dumps(run_serving(S, count=args.serving_requests)), flush=True)
        return 0

    log(f"generating inputs n={n}")
    A = torch.from_numpy(inputs.normal(n, 0)).to(dev)
    B = torch.from_numpy(inputs.normal(n, 1)).to(dev)
    C = torch.empty((n, n), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    ctx = S.stark_create(0)

    def timed(depth: int, precision: int, steps: int, warmup: int) -> float:
        """ms per multiply over `steps` back-to-back calls."""
        for _ in range(warmup):
            S.stark_gemm(ctx, A, B, C, n, depth, precision, st)
        st.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(st)
        for _ in range(steps):
            S.stark_gemm(ctx, A, B, C, n, depth, precision, st)
        e1.record(st)
        e1.synchronize()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    # -- autotune the headline configuration ---------------------------------
    # candidates: the three-product split paths (or the one precision asked
    # for); the headline is the fastest point within `tol`
    names = ["fp16x3", "bf16x3"] if args.precision == "split3" else [args.precision]
    tuned = {}        # precision name -> autotuner points (depth, ms, err, tile)
    if args.depth is None:
        for name in names:
            log(f"autotuning {name} depth in [{args.min_depth}, {args.max_depth}], target {tol:g}")
            tuned[name] = S.stark_tune(ctx, A, B, C, n, S.PRECISIONS[name], args.min_depth, args.max_depth, tol, st)
            for p in tuned[name]:
                log(f"  {name} depth {p[0]} tile {p[3]}: {p[1]:.3f} ms, freivalds {p[2]:.2e}"
                    f"{'' if p[2] <= tol else '  (outside the target)'}")
        within = [(p[1], name, p) for name, pts in tuned.items() for p in pts if p[2] <= tol]
        if within:
            _, hname, hp = min(within)
            run_depth = S.STARK_DEPTH_AUTO         # the autotuner recorded this point for hname
        else:                                       # nothing within the target: the most accurate point
            _, hname, hp = min((p[2], name, p) for name, pts in tuned.items() for p in pts)
            run_depth = hp[0]
            log("  no point within the target; timing the most accurate")
        depth, tile = hp[0], hp[3]
        log(f"  headline: {hname} depth {depth} tile {tile}")
    else:
        hname = names[0]
        depth, tile = args.depth, S.stark_plan_info(n, args.depth, S.PRECISIONS[hname]).gemm_tile
        run_depth = depth
    prec = S.PRECISIONS[hname]

    # -- timed region -----------------------------------------------------------
    log(f"timing {hname} depth {depth} tile {tile}: warmup {args.warmup}, steps {args.steps}")
    ms = timed(run_depth, prec, args.steps, args.warmup)
    eff = 2.0 * n ** 3 / (ms * 1e-3) * 1e-12
    log(f"  {ms:.3f} ms/step, {eff:.1f} effective TFLOP/s")

    # -- error of the headline result (C holds it) ------------------------------
    import oracle
    S.stark_gemm(ctx, A, B, C, n, run_depth, prec, st)
    st.synchronize()
    rows = inputs.sample_rows(n, args.rows, 2)
    Ah = A.cpu().numpy()
    Bh = B.cpu().numpy()
    log(f"oracle: {rows.size} sampled rows (FP64) on {oracle.threads()} host threads")
    t0 = time.perf_counter()
    ref = oracle.rows_f64(Ah, Bh, rows)
    t_rows = time.perf_counter() - t0
    Ch = C[torch.from_numpy(rows).to(dev)].cpu().numpy().astype(np.float64)
    d = Ch - ref
    rel_rows = float(np.sqrt(np.sum(d * d) / np.sum(ref * ref)))
    max_abs = float(np.max(np.abs(d)))
    x = torch.from_numpy(inputs.gaussian_vector(n, 3)).to(dev)
    y = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(3)]
    S.stark_matvec_f64(B, x, y[0], n, st)
    S.stark_matvec_f64(A, y[0], y[1], n, st)

    def freivalds() -> float:
        """||C x - A (B x)|| / ||A (B x)|| for the result now in C."""
        S.stark_matvec_f64(C, x, y[2], n, st)
        st.synchronize()
        return float(torch.linalg.norm(y[2] - y[1]) / torch.linalg.norm(y[1]))

    freiv = freivalds()
    log(f"  error: rel_frob(rows)={rel_rows:.3e} max_abs={max_abs:.3e} freivalds={freiv:.3e}")

    # -- per-phase times (live, HIP events on the launching stream) -----------
    def phases_of(d_: int, p_: int, reps: int) -> dict:
        """divide (+ split), leaf and combine phases launched one at a time
        (planner's tile class), with algorithmic bytes / flops and the
        fractions of the HBM and matrix-core peaks they reach."""
        plan_ = S.stark_plan_info(n, d_, p_)
        S.stark_gemm_phases(ctx, A, B, C, n, d_, p_, S.STARK_PHASE_DIVIDE, st)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record(st)
        for _ in range(reps):
            S.stark_gemm_phases(ctx, A, B, C, n, d_, p_, S.STARK_PHASE_DIVIDE, st)
        ev[1].record(st)
        for _ in range(reps):
            S.stark_gemm_phases(ctx, A, B, C, n, d_, p_, S.STARK_PHASE_LEAF, st)
        ev[2].record(st)
        for _ in range(reps):
            S.stark_gemm_phases(ctx, A, B, C, n, d_, p_, S.STARK_PHASE_COMBINE, st)
        ev[3].record(st)
        ev[3].synchronize()
        t_d, t_l, t_c = (ev[i].elapsed_time(ev[i + 1]) / reps for i in range(3))
        peak_l = PEAK["fp32"] if plan_.planes == 0 else PEAK["bf16"]
        sb = plan_.divide_bytes + plan_.split_bytes
        out_ = {"depth": d_, "leaf": plan_.leaf, "gemm_tile": plan_.gemm_tile,
                "divide_ms": t_d, "divide_bytes": sb,
                "divide_frac_hbm": sb / (t_d * 1e-3) / PEAK["hbm"] if t_d > 0 else None,
                "leaf_ms": t_l, "leaf_mfma_flops": plan_.mfma_flops, "leaf_useful_flops": plan_.leaf_flops,
                "leaf_tflops": plan_.mfma_flops / (t_l * 1e-3) * 1e-12,
                "leaf_frac_peak": plan_.mfma_flops / (t_l * 1e-3) / peak_l,
                "combine_ms": t_c, "combine_bytes": plan_.combine_bytes,
                "combine_frac_hbm": plan_.combine_bytes / (t_c * 1e-3) / PEAK["hbm"] if t_c > 0 else None,
                "sum_ms": t_d + t_l + t_c}
        return out_

    planes = S.stark_plan_info(n, depth, prec).planes
    ph = phases_of(depth, prec, max(1, args.phase_reps))
    plan = S.stark_plan_info(n, depth, prec)
    t_leaf = ph["leaf_ms"]
    L = plan.leaf
    nleaf = 7 ** depth
    prods = {0: 1, 2: 3, 3: 6}[planes]     # matrix-core products per leaf (FP16X3: 3)
    leaf_flops = plan.mfma_flops                      # matrix-core work of one launch
    assert leaf_flops == 2.0 * L ** 3 * nleaf * prods
    unit_peak = PEAK["fp32"] if planes == 0 else PEAK["bf16"]
    achieved = leaf_flops / (t_leaf * 1e-3)
    traffic = read_traffic(args.traffic, f"n{n}_d{depth}_{hname}")
    phases = {
        "divide_ms": ph["divide_ms"], "divide_gbs": ph["divide_bytes"] / (ph["divide_ms"] * 1e-3) * 1e-9,
        "leaf_ms": t_leaf, "leaf_tflops": achieved * 1e-12,
        "combine_ms": ph["combine_ms"],
        "combine_gbs": ph["combine_bytes"] / (ph["combine_ms"] * 1e-3) * 1e-9 if ph["combine_ms"] > 0 else None,
    }
    log(f"  phases: divide {ph['divide_ms']:.3f} ms ({phases['divide_gbs']:.0f} GB/s), leaf {t_leaf:.3f} ms "
        f"({achieved * 1e-12:.1f} TF/s of {unit_peak * 1e-12:.0f}), combine {ph['combine_ms']:.3f} ms")
    roofline = {"bound": "mfma", "achieved": achieved * 1e-12, "peak": unit_peak * 1e-12, "unit": "TFLOP/s",
                "frac": achieved / unit_peak, "traffic": traffic,
                "kernel": ("k_gemm_bf16" if planes else "k_gemm_f32") + ("_big" if plan.gemm_tile == 256 else ""),
                "gemm_tile": plan.gemm_tile,
                "work_per_launch": f"{nleaf} leaves x {prods} x 2*{L}^3 flops"}

    # -- per-depth phase table (where the time goes against the depth) ----------
    phase_table = {}
    if not args.no_phase_table:
        for name_ in dict.fromkeys([hname, "fp32"]):
            p_ = S.PRECISIONS[name_]
            rows_ = []
            for d_ in range(1, 5):
                r_ = phases_of(d_, p_, 3)
                rows_.append(r_)
                log(f"  phase table {name_} depth {d_}: divide {r_['divide_ms']:.3f} ms "
                    f"({r_['divide_frac_hbm']:.2f} of HBM), leaf {r_['leaf_ms']:.3f} ms "
                    f"({r_['leaf_frac_peak']:.2f} of peak), combine {r_['combine_ms']:.3f} ms "
                    f"({(r_['combine_frac_hbm'] or 0):.2f} of HBM)")
            phase_table[name_] = rows_

    # -- comparisons on the same GPU ----------------------------------------------
    compare = {}
    if not args.no_compare:
        legs = (("fp32_strassen", "fp32", 1, 4), ("fp32_classical", "fp32", 0, 0),
                ("fp16x3_strassen", "fp16x3", 2, 4), ("fp16x3_classical", "fp16x3", 0, 0),
                ("bf16x3_strassen", "bf16x3", 2, 4), ("bf16x3_strassen_depth1", "bf16x3", 1, 1),
                ("bf16x3_classical", "bf16x3", 0, 0), ("bf16x6_strassen", "bf16x6", 2, 4),
                ("bf16x3_winograd", "bf16x3_winograd", 2, 4), ("fp16x3_winograd", "fp16x3_winograd", 2, 4),
                ("fp32_winograd", "fp32_winograd", 1, 4))
        for leg, name_, dmin, dmax in legs:
            p_ = S.PRECISIONS[name_]
            if dmin == dmax:
                d_, t_ = dmin, S.stark_plan_info(n, dmin, p_).gemm_tile
                pts, run_d = [], dmin
            else:
                pts = tuned.get(name_) if (dmin, dmax) == (args.min_depth, args.max_depth) else None
                if pts is None:
                    pts = S.stark_tune(ctx, A, B, C, n, p_, dmin, dmax, tol, st)
                okp = [p for p in pts if p[2] <= tol]
                if okp:     # the autotuner recorded the fastest point within the target
                    d_, t_ = min(okp, key=lambda p: p[1])[::3]
                    run_d = S.STARK_DEPTH_AUTO
                else:       # nothing recorded: the fastest point, at its depth
                    d_ = min(pts, key=lambda p: p[1])[0]
                    t_ = S.stark_plan_info(n, d_, p_).gemm_tile
                    run_d = d_
            m_ = timed(run_d, p_, max(3, args.steps // 2), 1)
            fv = freivalds()
            compare[leg] = {"precision": name_, "depth": d_, "tile": t_, "ms": m_,
                            "tflops": 2.0 * n ** 3 / (m_ * 1e-3) * 1e-12, "freivalds": fv,
                            "meets_target": fv <= tol,
                            "tune": [{"depth": a, "ms": b, "err": c, "tile": t} for a, b, c, t in pts]}
            log(f"  {leg}: depth {d_} tile {t_}, {m_:.3f} ms, {compare[leg]['tflops']:.1f} TF/s, "
                f"freivalds {fv:.2e}{'' if fv <= tol else '  (outside the target)'}")
        # rectangular: (n/2) x n times n x (n/2), square-block partition,
        # operands are views of the headline A, B and C storage
        mr, kr, nr = n // 2, n, n // 2
        Ar = A[:mr]
        Br = B.view(-1)[:kr * nr].view(kr, nr)
        Cr = C.view(-1)[:mr * nr].view(mr, nr)
        rd = S.stark_model_depth(min(mr, kr, nr), prec)      # what STARK_DEPTH_AUTO takes
        for _ in range(2):
            S.stark_gemm_rect(ctx, Ar, Br, Cr, mr, kr, nr, S.STARK_DEPTH_AUTO, prec, st)
        tr = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        tr[0].record(st)
        for _ in range(3):
            S.stark_gemm_rect(ctx, Ar, Br, Cr, mr, kr, nr, S.STARK_DEPTH_AUTO, prec, st)
        tr[1].record(st)
        tr[1].synchronize()
        m_ = tr[0].elapsed_time(tr[1]) / 3
        compare["rect_" + hname] = {
            "shape": [mr, kr, nr], "depth": rd, "block_edge": S.stark_rect_block_edge(mr, kr, nr, rd), "ms": m_,
            "tflops": 2.0 * mr * kr * nr / (m_ * 1e-3) * 1e-12}
        log(f"  rect {mr}x{kr}x{nr} {hname} depth {rd} (automatic): {m_:.3f} ms, "
            f"{compare['rect_' + hname]['tflops']:.1f} TF/s")
        tt = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(st):
            for _ in range(2):
                torch.matmul(A, B, out=C)
            tt[0].record(st)
            for _ in range(3):
                torch.matmul(A, B, out=C)
            tt[1].record(st)
        tt[1].synchronize()
        m_ = tt[0].elapsed_time(tt[1]) / 3
        compare["torch_matmul_fp32_external"] = {"ms": m_, "tflops": 2.0 * n ** 3 / (m_ * 1e-3) * 1e-12,
                                                 "freivalds": freivalds()}

    # -- sizes off the 64 * 2^depth grid: peeled against zero-padded ----------------
    # n + 1 and n + 64 at the headline's precision and depth; the operands hold
    # the headline A and B in their leading n x n block and normal(0,1) values
    # from torch's seeded device generator in the border
    peeling = {}
    if not args.no_peeling:
        gen = torch.Generator(device=dev)
        for m in (n + 1, n + 64):
            gen.manual_seed(m)
            Am = torch.randn(m, m, generator=gen, device=dev)
            Bm = torch.randn(m, m, generator=gen, device=dev)
            Am[:n, :n] = A
            Bm[:n, :n] = B
            Cm = torch.empty((m, m), dtype=torch.float32, device=dev)
            xm = torch.randn(m, generator=gen, device=dev, dtype=torch.float64)
            ym = [torch.empty(m, dtype=torch.float64, device=dev) for _ in range(3)]
            # the operands are filled on torch's stream; the library's calls
            # below run on `st`, which does not wait for it
            torch.cuda.synchronize()
            S.stark_matvec_f64(Bm, xm, ym[0], m, st)
            S.stark_matvec_f64(Am, ym[0], ym[1], m, st)
            row = {"n": m, "depth": depth, "precision": hname}
            for mode, flag in (("peeled", S.STARK_PEEL), ("padded", S.STARK_PAD)):
                pm = prec | flag
                pl = S.stark_plan_info(m, depth, pm)
                for _ in range(2):
                    S.stark_gemm(ctx, Am, Bm, Cm, m, depth, pm, st)
                te = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                te[0].record(st)
                for _ in range(3):
                    S.stark_gemm(ctx, Am, Bm, Cm, m, depth, pm, st)
                te[1].record(st)
                te[1].synchronize()
                tm = te[0].elapsed_time(te[1]) / 3
                S.stark_matvec_f64(Cm, xm, ym[2], m, st)
                st.synchronize()
                fv = float(torch.linalg.norm(ym[2] - ym[1]) / torch.linalg.norm(ym[1]))
                row[mode] = {"ms": tm, "tflops": 2.0 * m ** 3 / (tm * 1e-3) * 1e-12, "peel": pl.peel,
                             "n_pad": pl.n_pad, "gemm_tile": pl.gemm_tile, "freivalds": fv}
                log(f"  n={m} {mode}: residue {pl.peel}, core/padded edge {pl.n_pad}, tile {pl.gemm_tile}: "
                    f"{tm:.3f} ms, {row[mode]['tflops']:.1f} TF/s, freivalds {fv:.2e}")
            row["default"] = "peeled" if S.stark_plan_info(m, depth, prec).peel else "padded"
            peeling[str(m)] = row
            del Am, Bm, Cm

    # -- CPU baseline: the oracle on a bounded sample of rows -----------------------
    # (the error-check rows plus more rows, about 10 s of host work in total),
    # and the Table V analog (full FP64 products at smaller n)
    cpu = None
    if not args.no_cpu_baseline:
        extra = inputs.sample_rows(n, args.cpu_rows, 7)
        t0 = time.perf_counter()
        oracle.rows_f64(Ah, Bh, extra)
        t_extra = time.perf_counter() - t0
        nrows, secs = rows.size + extra.size, t_rows + t_extra
        flops = 2.0 * nrows * n * n
        cpu = {"value": flops / secs * 1e-12, "unit": "TFLOP/s", "cores": oracle.threads(), "kind": "oracle",
               "sample": f"classical FP64 triple loop, {nrows} sampled rows of the n={n} product "
                         f"({flops:.3g} flops, {secs:.1f} s)"}
        cpu.update(host_info())
        log(f"cpu baseline: {cpu['value']:.4f} TFLOP/s on {cpu['cores']} threads ({secs:.1f} s); "
            f"host {cpu['cpu_model']}, nproc {cpu['nproc']}")
        cpu["full_products"] = cpu_table(oracle, inputs)

    # -- batched and serving -------------------------------------------------------
    batched = None
    if not args.no_batched:
        batched = run_batched(S, torch, st)
    serving = None
    if not args.no_serving:
        serving = run_serving(S, count=args.serving_requests)

    S.stark_destroy(ctx)
    bf = compare.get("bf16x3_strassen")
    out = {
        "metric": "effective TFLOP/s (2n^3/t) at n=16384 vs plain FP32 path; p50/p99 request latency",
        "value": eff, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": hname if planes else "f32", "data": "synthetic",
        "config": {"workload": (f"strassen C=AB n={n} normal(0,1), leaf products {hname} "
                                f"(three split products on 16-bit matrix cores, binary32 accumulation) "
                                f"depth={depth}" + (f" (fastest within rel. error {tol:g} among "
                                                    f"{'/'.join(names)} at depths {args.min_depth}..{args.max_depth})"
                                                    if args.depth is None else "")),
                   "n": n, "depth": depth, "gemm_tile": tile, "precision": hname, "leaf": L,
                   "n_pad": plan.n_pad,
                   "library": S.LIB_PATH if S.LIB_PATH != S.DEFAULT_LIB_PATH else "in-tree"},
        "error": {"rel_frob_sampled_rows": rel_rows, "max_abs_sampled_rows": max_abs, "freivalds": freiv,
                  "rows": int(rows.size), "target": tol, "meets_target": rel_rows <= tol,
                  # measured paths of this run within the target (Freivalds estimate), fastest first
                  "target_met_by": sorted(({"path": k, "tflops": v["tflops"], "freivalds": v["freivalds"]}
                                           for k, v in compare.items()
                                           if v.get("freivalds") is not None and v["freivalds"] <= tol),
                                          key=lambda r: -r["tflops"]),
                  "bf16x3_depths_2_4": ({"meets_target": False if bf is None else bf["meets_target"],
                                         "tune": None if bf is None else bf["tune"]})},
        "tune": {k: [{"depth": a, "ms": b, "err": c, "tile": t} for a, b, c, t in v] for k, v in tuned.items()},
        "phases": phases, "phase_table": phase_table, "roofline": roofline, "cpu_baseline": cpu,
        "compare": compare, "peeling": peeling, "batched": batched,
        # the paper's own figure for this size (distributed Spark, FP64; another machine): context only
        "paper_context": {"n": 16384, "stark_wall_clock_s": 161.0, "effective_tflops": 2.0 * 16384 ** 3 / 161.0 * 1e-12,
                          "source": "Fig. 6 and Table V (fastest partition, b = 16)",
                          "hardware": "3 nodes, each 2 x 6-core Xeon 2.60 GHz, 132 GB, 14 Gb/s InfiniBand; "
                                      "Spark 1.6.0 with 5 executors x 5 cores; FP64 leaf products through BLAS",
                          "serial_strassen_one_node_s": 2453.0},
        "serving": serving,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
