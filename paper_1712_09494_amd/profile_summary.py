"""Summarise rocprofv3 output of a benchmark run into the text summaries kept
under profiles/ (per-kernel counters per dispatch, HBM traffic scaled by a
plain copy of known size, and the kernel-trace statistics).

    python -m paper_1712_09494_amd.profile_summary --workload random_scaling_2p26 \
        --pmc out/pmc1 out/pmc2 ... --trace out/kt --commands-file out/prof_commands.txt

Counter passes: each --pmc directory holds the run_counter_collection.csv of
one rocprofv3 --pmc run of the same program.  FETCH_SIZE and WRITE_SIZE (KiB
per dispatch) are scaled by what they read for probe_copy_kernel, which
reads and writes a known number of bytes (--copy-bytes), so that the
scaled figures are HBM bytes.  Kernels are named by their function name;
probe_mix_kernel dispatches are split into consecutive groups of
--mix-group dispatches, one per find-or-put kernel the benchmark compares
(--mix-for, in the benchmark's order).  The JSON also records the sha256 of
the counted kernels' sources, so that a reader can tell whether the
counters are still current.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

# the sources that define or launch the counted find-or-put kernels
COUNTED_SOURCES = ("ht_device.h", "bucketed_dev.h", "bucketed.hip", "cuckoo_dev.h", "cuckoo.hip", "table.hip")


def source_hash() -> str:
    h = hashlib.sha256()
    for name in sorted(COUNTED_SOURCES):
        h.update(name.encode())
        with open(os.path.join(HERE, "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def short_name(full: str) -> str:
    """Function name without namespace, return type and arguments; template
    arguments kept for the probe kernels only."""
    s = full.strip().replace("(anonymous namespace)::", "")
    if s.startswith("void "):
        s = s[5:]
    s = s.split("(")[0].replace("ht::", "").replace("at::native::", "")
    base = s.split("<")[0]
    return s.replace(" ", "") if base.startswith("probe_") else base


def read_pmc(dirs, mix_group: int, mix_for: list[str]):
    """{kernel: {counter: [values per dispatch]}} over every pass."""
    out = defaultdict(lambda: defaultdict(list))
    for d in dirs:
        path = None
        for root, _, files in os.walk(d):
            for f in files:
                if f.endswith("counter_collection.csv"):
                    path = os.path.join(root, f)
        if path is None:
            raise SystemExit(f"no counter_collection.csv under {d}")
        rows = list(csv.DictReader(open(path)))
        mix_seen = defaultdict(list)
        for r in sorted(rows, key=lambda r: int(r["Dispatch_Id"])):
            name = short_name(r["Kernel_Name"])
            if name.startswith("probe_mix_kernel"):
                ids = mix_seen[name]
                if r["Dispatch_Id"] not in ids:
                    ids.append(r["Dispatch_Id"])
                g = ids.index(r["Dispatch_Id"]) // mix_group
                label = mix_for[g] if g < len(mix_for) else str(g)
                form = "same_line" if "true" in name else "other_line"
                name = f"probe_mix[{form},{label}]"
            out[name][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return out


def read_trace(d):
    """Kernel statistics of a --kernel-trace --stats run: {name: row}."""
    path = None
    for root, _, files in os.walk(d):
        for f in files:
            if f.endswith("kernel_stats.csv"):
                path = os.path.join(root, f)
    if path is None:
        return None
    stats = {}
    for r in csv.DictReader(open(path)):
        name = short_name(r["Name"])
        e = stats.setdefault(name, {"calls": 0, "total_ns": 0.0, "min_ns": None, "max_ns": 0.0})
        e["calls"] += int(r["Calls"])
        e["total_ns"] += float(r["TotalDurationNs"])
        mn, mx = float(r["MinNs"]), float(r["MaxNs"])
        e["min_ns"] = mn if e["min_ns"] is None else min(e["min_ns"], mn)
        e["max_ns"] = max(e["max_ns"], mx)
    total = sum(e["total_ns"] for e in stats.values()) or 1.0
    for e in stats.values():
        e["avg_us"] = e["total_ns"] / e["calls"] / 1e3
        e["share"] = e["total_ns"] / total
    return stats


def mean(v):
    return sum(v) / len(v) if v else None


def summarise(pmc, copy_bytes: float):
    cal = pmc.get("probe_copy_kernel", {})
    f_cal = mean(cal.get("FETCH_SIZE", []))
    w_cal = mean(cal.get("WRITE_SIZE", []))
    fetch_scale = copy_bytes / (f_cal * 1024) if f_cal else None
    write_scale = copy_bytes / (w_cal * 1024) if w_cal else None
    kernels = {}
    for name, cs in sorted(pmc.items()):
        k = {"dispatches": max(len(v) for v in cs.values())}
        for cname, vals in sorted(cs.items()):
            k[cname] = mean(vals)
        if k.get("FETCH_SIZE") is not None and k.get("WRITE_SIZE") is not None and fetch_scale and write_scale:
            k["hbm_bytes"] = k["FETCH_SIZE"] * 1024 * fetch_scale + k["WRITE_SIZE"] * 1024 * write_scale
            k["hbm_read_bytes"] = k["FETCH_SIZE"] * 1024 * fetch_scale
            k["hbm_write_bytes"] = k["WRITE_SIZE"] * 1024 * write_scale
        if k.get("TCC_HIT_sum") is not None and k.get("TCC_MISS_sum") is not None:
            tot = k["TCC_HIT_sum"] + k["TCC_MISS_sum"]
            k["l2_hit_rate"] = k["TCC_HIT_sum"] / tot if tot else None
        if k.get("TCP_TCC_READ_REQ_sum") and k.get("TCP_TCC_READ_REQ_LATENCY_sum") is not None:
            k["l2_read_latency_cycles"] = k["TCP_TCC_READ_REQ_LATENCY_sum"] / k["TCP_TCC_READ_REQ_sum"]
        if k.get("SQ_WAVE_CYCLES") and k.get("SQ_WAIT_INST_ANY") is not None:
            k["wave_wait_fraction"] = k["SQ_WAIT_INST_ANY"] / k["SQ_WAVE_CYCLES"]
        if k.get("SQ_INST_LEVEL_VMEM") is not None and k.get("SQ_WAVE_CYCLES"):
            k["vmem_in_flight_per_wave"] = k["SQ_INST_LEVEL_VMEM"] / k["SQ_WAVE_CYCLES"]
        kernels[name] = k
    return {"fetch_scale": fetch_scale, "write_scale": write_scale,
            "calibration": {"kernel": "probe_copy_kernel", "bytes_read": copy_bytes, "bytes_written": copy_bytes,
                            "fetch_kib": f_cal, "write_kib": w_cal},
            "kernels": kernels}


def fmt(x, nd=1):
    if x is None:
        return "-"
    if isinstance(x, float) and abs(x) >= 1e4:
        return f"{x:,.0f}"
    return f"{x:.{nd}f}" if isinstance(x, float) else str(x)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True)
    ap.add_argument("--pmc", nargs="*", default=[])
    ap.add_argument("--trace")
    ap.add_argument("--copy-bytes", type=float, default=float(1 << 29))
    ap.add_argument("--mix-group", type=int, default=6)
    ap.add_argument("--mix-for", default="bucketed_fop,cuckoo_probe")
    ap.add_argument("--commands-file", help="text file with the commands of the runs, one per line")
    ap.add_argument("--kernels", default="bucketed_fop_kernel,cuckoo_probe_kernel,cuckoo_evict_kernel,"
                                         "cuckoo_scrub_kernel,probe_mix,probe_copy_kernel")
    ap.add_argument("--outdir", default=os.path.join(ROOT, "profiles"))
    args = ap.parse_args()
    cmds = open(args.commands_file).read().strip().splitlines() if args.commands_file else []
    res = {"workload": args.workload, "kernel_source_sha256": source_hash(), "commands": cmds}
    if args.pmc:
        res.update(summarise(read_pmc(args.pmc, args.mix_group, args.mix_for.split(",")), args.copy_bytes))
        with open(os.path.join(args.outdir, f"counters_{args.workload}.json"), "w") as f:
            json.dump(res, f, indent=1)
            f.write("\n")
        keep = args.kernels.split(",")
        rows = [(n, k) for n, k in res["kernels"].items() if any(n.startswith(p) for p in keep)]
        lines = [f"# Counters per dispatch: {args.workload}", "",
                 "Commands (from the repository root, one counter pass per run):", "", "```"] + cmds + ["```", "",
                 f"HBM bytes = FETCH_SIZE x {fmt(res['fetch_scale'], 3)} + WRITE_SIZE x {fmt(res['write_scale'], 3)} "
                 f"(KiB x 1024; the factors make probe_copy_kernel's figures equal its "
                 f"{int(args.copy_bytes):,} bytes read and written).  L2 read latency = "
                 "TCP_TCC_READ_REQ_LATENCY / TCP_TCC_READ_REQ (cycles); wave wait = SQ_WAIT_INST_ANY / "
                 "SQ_WAVE_CYCLES; VMEM in flight = SQ_INST_LEVEL_VMEM / SQ_WAVE_CYCLES.  probe_mix rows are "
                 "the mixed memory-pattern probe run with the named kernel's lines and compare-and-swaps per key.",
                 f"Counted kernels' sources sha256: `{res['kernel_source_sha256']}`", "",
                 "| kernel | dispatches | HBM read MB | HBM write MB | L2 hit % | EA read req | EA 128B req | "
                 "EA atomics | DRAM credit stalls | L2 read latency (cyc) | wave wait % | VMEM in flight/wave |",
                 "|---|---|---|---|---|---|---|---|---|---|---|---|"]
        for n, k in rows:
            lines.append("| " + " | ".join([
                n, str(k["dispatches"]),
                fmt(k.get("hbm_read_bytes", 0) / 1e6 if k.get("hbm_read_bytes") is not None else None, 2),
                fmt(k.get("hbm_write_bytes", 0) / 1e6 if k.get("hbm_write_bytes") is not None else None, 2),
                fmt(100 * k["l2_hit_rate"] if k.get("l2_hit_rate") is not None else None),
                fmt(k.get("TCC_EA0_RDREQ_sum"), 0), fmt(k.get("TCC_EA0_RDREQ_128B_sum"), 0),
                fmt(k.get("TCC_EA0_ATOMIC_sum"), 0), fmt(k.get("TCC_EA0_RDREQ_DRAM_CREDIT_STALL_sum"), 0),
                fmt(k.get("l2_read_latency_cycles"), 0),
                fmt(100 * k["wave_wait_fraction"] if k.get("wave_wait_fraction") is not None else None),
                fmt(k.get("vmem_in_flight_per_wave"), 2)]) + " |")
        with open(os.path.join(args.outdir, f"counters_{args.workload}.md"), "w") as f:
            f.write("\n".join(lines) + "\n")
    if args.trace:
        st = read_trace(args.trace)
        if st:
            lines = [f"# Kernel trace: {args.workload}", "", "Command (from the repository root, on one MI355X):", "",
                     "```"] + [c for c in cmds if "--kernel-trace" in c] + ["```", "",
                     "| kernel | calls | avg us | min us | max us | share % |", "|---|---|---|---|---|---|"]
            for n, e in sorted(st.items(), key=lambda kv: -kv[1]["total_ns"])[:20]:
                lines.append(f"| {n} | {e['calls']} | {e['avg_us']:.2f} | {e['min_ns'] / 1e3:.2f} | "
                             f"{e['max_ns'] / 1e3:.2f} | {100 * e['share']:.2f} |")
            with open(os.path.join(args.outdir, f"kernel_trace_{args.workload}.md"), "w") as f:
                f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
