"""Summaries of rocprofv3 output for the measurements kept with the sources.

* `kernel_stats_md`: the `--kernel-trace --stats -f csv` kernel table as a
  short markdown table;
* `counter_per_kernel`: mean of one `--pmc` counter per dispatch for the
  kernels whose name contains a given string;
* `traffic_table_md`: the same for every kernel of a run, as markdown;
* `traffic`: leaf-GEMM HBM bytes per launch from FETCH_SIZE and WRITE_SIZE
  runs, each scaled by what the same counter reads for a plain copy of known
  size (the counters report KiB per dispatch);
* `mfma_md`: matrix-core busy fraction, hardware flops and clock of a kernel;
* `stream_overlap` / `overlap_md`: the share of GPU-busy time during which
  kernels of two or more streams run at once (served requests);
* `source_digest`: SHA-256 of the kernel source the counters were taken on,
  so a reader can tell when they are stale.

Command line:
  python -m paper_1811_07325_amd.profsum stats <kernel_stats.csv> <title> <command>
  python -m paper_1811_07325_amd.profsum traffic <key> <copy_fetch.csv> <copy_write.csv>
      <copy_bytes> <gemm_fetch.csv> <gemm_write.csv> <kernel substring> <command...>
  python -m paper_1811_07325_amd.profsum mfma <counters.csv> <kernel substring> <title> <command lines...>
  python -m paper_1811_07325_amd.profsum table <copy_fetch.csv> <copy_write.csv> <copy_bytes>
      <run_fetch.csv> <run_write.csv> <kernel,substrings> <title> <command lines...>
  python -m paper_1811_07325_amd.profsum overlap <kernel_trace.csv> <title> <command lines...>
"""
from __future__ import annotations

import csv
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
GEMM_SOURCE = os.path.join(HERE, "csrc", "k_gemm.hip")


def source_digest(path: str = GEMM_SOURCE) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def kernel_stats_md(path: str, title: str, command: str, top: int = 12) -> str:
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = [f"# {title}", "", "Command (from the repository root, on one MI355X):", "", "```", command, "```", "",
           "| kernel | calls | avg (ms) | min (ms) | max (ms) | share of GPU time |",
           "|---|---:|---:|---:|---:|---:|"]
    for r in rows[:top]:
        name = r["Name"].replace("|", "/")
        if len(name) > 90:
            name = name[:87] + "..."
        out.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.3f} | {float(r['MinNs']) / 1e6:.3f} "
                   f"| {float(r['MaxNs']) / 1e6:.3f} | {float(r['Percentage']):.1f} % |")
    return "\n".join(out) + "\n"


def counter_per_kernel(path: str, counter: str, name_part: str) -> tuple[float, int]:
    """(mean counter value per dispatch, dispatch count) over kernels whose
    name contains `name_part`."""
    vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
            if r["Counter_Name"] == counter and name_part in r["Kernel_Name"]]
    if not vals:
        raise ValueError(f"no {counter} rows for kernels matching {name_part!r} in {path}")
    return sum(vals) / len(vals), len(vals)


def traffic(copy_fetch: str, copy_write: str, copy_bytes: float, gemm_fetch: str, gemm_write: str,
            name_part: str, copy_name: str = "neg") -> dict:
    """Leaf-GEMM HBM bytes per launch.  The copy kernel reads and writes
    `copy_bytes` each; the factor per counter is known bytes / counted bytes."""
    cf, _ = counter_per_kernel(copy_fetch, "FETCH_SIZE", copy_name)
    cw, _ = counter_per_kernel(copy_write, "WRITE_SIZE", copy_name)
    ff = copy_bytes / (cf * 1024.0)
    fw = copy_bytes / (cw * 1024.0)
    gf, nf = counter_per_kernel(gemm_fetch, "FETCH_SIZE", name_part)
    gw, nw = counter_per_kernel(gemm_write, "WRITE_SIZE", name_part)
    return {"fetch_bytes": gf * 1024.0 * ff, "write_bytes": gw * 1024.0 * fw, "factor_fetch": ff,
            "factor_write": fw, "dispatches": (nf, nw)}


def traffic_table_md(copy_fetch: str, copy_write: str, copy_bytes: float, run_fetch: str, run_write: str,
                     kernels: list[str], title: str, commands: list[str]) -> str:
    """Measured HBM bytes per dispatch of the named kernels (distinct values
    with their dispatch counts), both counters scaled by the copy factors."""
    cf, _ = counter_per_kernel(copy_fetch, "FETCH_SIZE", "neg")
    cw, _ = counter_per_kernel(copy_write, "WRITE_SIZE", "neg")
    ff, fw = copy_bytes / (cf * 1024.0), copy_bytes / (cw * 1024.0)

    def per_dispatch(path, counter, part, factor):
        vals = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter and part in r["Kernel_Name"]:
                vals[int(r["Dispatch_Id"])] = float(r["Counter_Value"]) * 1024.0 * factor
        return [vals[k] for k in sorted(vals)]

    out = [f"# {title}", "", "Commands (from the repository root, on one MI355X):", "", "```"] + commands + [
        "```", "", f"Copy calibration: a 1 GiB elementwise copy reads as FETCH_SIZE x {ff:.3f} and "
        f"WRITE_SIZE x {fw:.3f} of its known bytes; every figure below is scaled by these factors.", "",
        "| kernel | dispatches | fetched GB per dispatch | written GB per dispatch |", "|---|---:|---:|---:|"]
    for k in kernels:
        f = per_dispatch(run_fetch, "FETCH_SIZE", k, ff)
        w = per_dispatch(run_write, "WRITE_SIZE", k, fw)
        shapes = {}
        for a, b in zip(f, w):
            key = (round(a / 1e9, 2), round(b / 1e9, 2))
            shapes[key] = shapes.get(key, 0) + 1
        for (a, b), c in sorted(shapes.items(), key=lambda t: -t[0][0]):
            out.append(f"| `{k}` | {c} | {a:.2f} | {b:.2f} |")
    return "\n".join(out) + "\n"


def mfma_md(path: str, name_part: str, simds: int, xccs: int, title: str, commands: list[str]) -> str:
    """Matrix-core counters of one kernel per dispatch: hardware flops
    (SQ_INSTS_VALU_MFMA_MOPS_BF16 + _F16 + _F32, whichever were collected,
    x 512),
    MFMA busy fraction
    (SQ_VALU_MFMA_BUSY_CYCLES summed over SIMDs / (active cycles per XCC x
    SIMDs); GRBM_GUI_ACTIVE is reported summed over the XCCs) and the average
    shader clock over the dispatch (active cycles per XCC / duration)."""
    per = {}
    for r in csv.DictReader(open(path)):
        if name_part in r["Kernel_Name"]:
            e = per.setdefault(int(r["Dispatch_Id"]), {})
            e[r["Counter_Name"]] = float(r["Counter_Value"])
            e["ns"] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    out = [f"# {title}", "", "Commands (from the repository root, on one MI355X):", "", "```"] + commands + [
        "```", "", "| dispatch | ms | MFMA flops | MFMA busy | clock (GHz) |", "|---:|---:|---:|---:|---:|"]
    for k in sorted(per):
        e = per[k]
        cyc = e["GRBM_GUI_ACTIVE"] / xccs
        mops = (e.get("SQ_INSTS_VALU_MFMA_MOPS_BF16", 0.0) + e.get("SQ_INSTS_VALU_MFMA_MOPS_F16", 0.0) +
                e.get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0))
        out.append(f"| {k} | {e['ns'] / 1e6:.3f} | {mops * 512:.4e} | "
                   f"{e['SQ_VALU_MFMA_BUSY_CYCLES'] / (cyc * simds):.3f} | {cyc / e['ns']:.2f} |")
    return "\n".join(out) + "\n"


def stream_overlap(path: str) -> dict:
    """Concurrency of kernels from different streams in a --kernel-trace
    csv: sweeping the dispatch start / end times, the share of the time with
    at least one kernel running during which kernels of k or more distinct
    streams run at once (k = 2, 3, 4), and the busy time itself."""
    ev = []
    for r in csv.DictReader(open(path)):
        s, e, sid = int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Stream_Id"]
        if e > s:
            ev.append((s, 1, sid))
            ev.append((e, -1, sid))
    ev.sort(key=lambda x: (x[0], x[1]))
    active: dict[str, int] = {}
    busy = 0
    at_least = {2: 0, 3: 0, 4: 0}
    last = None
    for t, d, sid in ev:
        if last is not None and active:
            span = t - last
            busy += span
            for k in at_least:
                if len(active) >= k:
                    at_least[k] += span
        last = t
        active[sid] = active.get(sid, 0) + d
        if active[sid] == 0:
            del active[sid]
    return {"busy_ms": busy / 1e6, **{f"frac_ge{k}_streams": (v / busy if busy else 0.0) for k, v in at_least.items()},
            "streams": len({x[2] for x in ev}), "dispatches": len(ev) // 2}


def overlap_md(path: str, title: str, commands: list[str]) -> str:
    o = stream_overlap(path)
    out = [f"# {title}", "", "Commands (from the repository root, on one MI355X):", "", "```"] + commands + [
        "```", "", "| quantity | value |", "|---|---:|",
        f"| kernel dispatches | {o['dispatches']} |", f"| streams with kernels | {o['streams']} |",
        f"| GPU busy time (at least one kernel running) | {o['busy_ms']:.1f} ms |"]
    for k in (2, 3, 4):
        out.append(f"| share of busy time with kernels of >= {k} streams running | {o[f'frac_ge{k}_streams']:.3f} |")
    return "\n".join(out) + "\n"


def main(argv: list[str]) -> int:
    if argv[0] == "stats":
        sys.stdout.write(kernel_stats_md(argv[1], argv[2], argv[3]))
        return 0
    if argv[0] == "traffic":
        key, cfe, cwr, cb, gfe, gwr, part = argv[1:8]
        t = traffic(cfe, cwr, float(cb), gfe, gwr, part)
        print(f"# source_sha256 {source_digest()}")
        print(f"# command: {' '.join(argv[8:])}")
        print("# key fetch_bytes write_bytes factor_fetch factor_write")
        print(f"{key} {t['fetch_bytes']:.6e} {t['write_bytes']:.6e} {t['factor_fetch']:.4f} {t['factor_write']:.4f}")
        return 0
    if argv[0] == "mfma":
        path, part, title = argv[1:4]
        sys.stdout.write(mfma_md(path, part, 1024, 8, title, argv[4:]))
        return 0
    if argv[0] == "overlap":
        sys.stdout.write(overlap_md(argv[1], argv[2], argv[3:]))
        return 0
    if argv[0] == "table":
        cfe, cwr, cb, rfe, rwr, kernels, title = argv[1:8]
        sys.stdout.write(traffic_table_md(cfe, cwr, float(cb), rfe, rwr, kernels.split(","), title, argv[8:]))
        return 0
    print(__doc__)
    return 2


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
