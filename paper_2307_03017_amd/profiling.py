"""Summaries of rocprofv3 output for the library's kernels.

    # kernel durations (rocprofv3 --kernel-trace --stats --output-format csv)
    python -m paper_2307_03017_amd.profiling stats <kernel_stats.csv> --cmd "<rocprofv3 command>" --md out.md

    # HBM traffic per launch from two counter runs (FETCH_SIZE, then WRITE_SIZE), scaled by
    # what the same counters read for the library's plain FP32 copy kernel (k_convert) over a
    # buffer of known size
    python -m paper_2307_03017_amd.profiling traffic --fetch <fetch counter_collection.csv> \\
        --write <write counter_collection.csv> --kernel k_grad_shift --copy-bytes 268435456 \\
        --cmd "<commands>" --json out.json --md out.md

    # instruction mix and issue-slot load per launch size (rocprofv3 --pmc of SQ_COUNTERS)
    python -m paper_2307_03017_amd.profiling sq <counter_collection.csv> --agent <agent_info.csv> \
        --kernel k_grad_shift --cmd "<commands>" --json out.json --md out.md
"""

from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
from collections import defaultdict

_PKG = os.path.dirname(os.path.abspath(__file__))


# the sources a kernel is compiled from (a recorded traffic figure holds while they are unchanged)
KERNEL_SOURCES = {
    "k_plane_sweep": ("hsgd_psv.hip", "hsgd_device.h", "hsgd_internal.h"),
}
DEFAULT_SOURCES = ("hsgd_kernels.hip", "hsgd_device.h", "hsgd_internal.h")


_COMMENT = re.compile(r"//[^\n]*|/\*.*?\*/", re.S)


def kernel_source_hash(kernel: str = "k_grad_shift") -> str:
    """Hash of the code a kernel is compiled from: its sources with comments removed and
    whitespace collapsed, so that editing a comment keeps the recorded figures valid."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(kernel, DEFAULT_SOURCES):
        with open(os.path.join(_PKG, "csrc", f), encoding="utf-8") as fh:
            code = " ".join(_COMMENT.sub(" ", fh.read()).split())
        h.update(code.encode())
        h.update(b"\0")
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    """'void hsgd::(anonymous namespace)::k_grad_shift<0, 32, true>(...)' -> 'k_grad_shift<0, 32, true>'"""
    name = name.split("(void")[0] if name.startswith("void ") else name
    name = re.sub(r"^void\s+", "", name)
    name = name.replace("hsgd::(anonymous namespace)::", "")
    depth = 0
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return name[:i]
    return name


def read_stats(path: str):
    rows = []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            keys = {k.lower(): k for k in r}
            name = r[keys.get("name", "Name")]
            calls = int(float(r[keys["calls"]]))
            tot = float(r[keys.get("totaldurationns", keys.get("duration (nsec)", "TotalDurationNs"))])
            avg = float(r[keys.get("averagens", keys.get("average (nsec)", "AverageNs"))])
            mn = float(r[keys.get("minns", keys.get("min (nsec)", "MinNs"))])
            mx = float(r[keys.get("maxns", keys.get("max (nsec)", "MaxNs"))])
            rows.append(dict(name=short_name(name), calls=calls, total_us=tot / 1e3, avg_us=avg / 1e3,
                             min_us=mn / 1e3, max_us=mx / 1e3))
    return rows


def stats_md(rows, cmd: str) -> str:
    total = sum(r["total_us"] for r in rows) or 1.0
    out = ["# Kernel durations", "", "Command:", "", "```", cmd, "```", "",
           "| kernel | calls | avg us | min us | max us | share |", "|---|---:|---:|---:|---:|---:|"]
    for r in sorted(rows, key=lambda r: -r["total_us"]):
        out.append(f"| `{r['name']}` | {r['calls']} | {r['avg_us']:.1f} | {r['min_us']:.1f} | "
                   f"{r['max_us']:.1f} | {100 * r['total_us'] / total:.1f}% |")
    return "\n".join(out) + "\n"


def _counter_rows(path: str, counter: str):
    """Per dispatch: (kernel short name, grid size, counter value)."""
    per = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            key = (r["Dispatch_Id"], short_name(r["Kernel_Name"]), int(r["Grid_Size"]))
            per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    return [(k[1], k[2], v) for k, v in per.items()]


def traffic(fetch_csv: str, write_csv: str, kernel: str, copy_bytes: int, copy_kernel: str = "k_convert<0, 0>"):
    f = _counter_rows(fetch_csv, "FETCH_SIZE")
    w = _counter_rows(write_csv, "WRITE_SIZE")
    cf = [v for n, g, v in f if n == copy_kernel]
    cw = [v for n, g, v in w if n == copy_kernel]
    if not cf or not cw:
        raise SystemExit("no copy-kernel dispatches in the counter files")
    # the copy reads and writes copy_bytes/2 each (copy_bytes counts both directions)
    f_factor = (copy_bytes / 2) / (1024.0 * sum(cf) / len(cf))
    w_factor = (copy_bytes / 2) / (1024.0 * sum(cw) / len(cw))
    fk = defaultdict(list)
    wk = defaultdict(list)
    for n, g, v in f:
        if n.startswith(kernel):
            fk[(n, g)].append(v * 1024.0 * f_factor)
    for n, g, v in w:
        if n.startswith(kernel):
            wk[(n, g)].append(v * 1024.0 * w_factor)
    launches = []
    for key in sorted(fk):
        rb = sum(fk[key]) / len(fk[key])
        wb = sum(wk.get(key, [0.0])) / max(len(wk.get(key, [])), 1)
        launches.append(dict(kernel=key[0], grid=key[1], read_bytes=rb, write_bytes=wb))
    mean = sum(l["read_bytes"] + l["write_bytes"] for l in launches) / max(len(launches), 1)
    return dict(kernel=kernel, fetch_factor=f_factor, write_factor=w_factor, launches=launches,
                hbm_bytes_per_launch=mean, kernel_source_hash=kernel_source_hash(kernel))


def traffic_md(t, cmd: str) -> str:
    out = ["# HBM traffic per launch", "", "Commands:", "", "```", cmd, "```", "",
           f"Calibration with the library's plain FP32 copy kernel over a buffer of known size: "
           f"FETCH_SIZE x {t['fetch_factor']:.3f}, WRITE_SIZE x {t['write_factor']:.3f}. "
           "Both counters count what leaves L2 towards memory: reads that the Infinity Cache "
           "serves are included.", "",
           f"Kernel source hash: `{t['kernel_source_hash']}`", "",
           "| kernel | grid | read MB | write MB |", "|---|---:|---:|---:|"]
    for l in t["launches"]:
        out.append(f"| `{l['kernel']}` | {l['grid']} | {l['read_bytes'] / 1e6:.1f} | {l['write_bytes'] / 1e6:.1f} |")
    out += ["", f"Mean over these launch sizes: {t['hbm_bytes_per_launch'] / 1e6:.1f} MB per launch."]
    return "\n".join(out) + "\n"


def l2(csv_path: str):
    """L2 (TCC) hit rate per kernel from a TCC_HIT_sum / TCC_MISS_sum counter run: hits over
    requests, summed over every dispatch of the kernel (all template instances of one
    kernel name pooled, grid sizes kept apart)."""
    hits = _counter_rows(csv_path, "TCC_HIT_sum")
    miss = _counter_rows(csv_path, "TCC_MISS_sum")
    agg = defaultdict(lambda: [0.0, 0.0, 0])
    for n, g, v in hits:
        agg[(n, g)][0] += v
        agg[(n, g)][2] += 1
    for n, g, v in miss:
        agg[(n, g)][1] += v
    rows = []
    for (n, g), (h, m, c) in sorted(agg.items()):
        rows.append(dict(kernel=n, grid=g, dispatches=c, hits=h, misses=m, hit_rate=h / (h + m) if h + m else None))
    by_kernel = defaultdict(lambda: [0.0, 0.0])
    for r in rows:
        base = r["kernel"].split("<")[0]
        by_kernel[base][0] += r["hits"]
        by_kernel[base][1] += r["misses"]
    return dict(rows=rows, hit_rate={k: h / (h + m) for k, (h, m) in by_kernel.items() if h + m},
                kernel_source_hash={k: kernel_source_hash(k) for k in by_kernel})


def l2_md(t, cmd: str) -> str:
    out = ["# L2 hit rate per kernel", "", "Command:", "", "```", cmd, "```", "",
           "TCC_HIT_sum / (TCC_HIT_sum + TCC_MISS_sum) over the dispatches of each kernel "
           "(summed over every L2 channel of the 8 XCDs).", "",
           "| kernel | grid | dispatches | hit rate |", "|---|---:|---:|---:|"]
    for r in t["rows"]:
        hr = "—" if r["hit_rate"] is None else f"{100 * r['hit_rate']:.1f}%"
        out.append(f"| `{r['kernel']}` | {r['grid']} | {r['dispatches']} | {hr} |")
    out += ["", "Per kernel (all launches): " + ", ".join(f"`{k}` {100 * v:.1f}%" for k, v in sorted(t["hit_rate"].items()))]
    return "\n".join(out) + "\n"


SQ_COUNTERS = ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_WAVES", "SQ_WAVE_CYCLES",
               "SQ_ACTIVE_INST_VALU", "SQ_WAIT_INST_ANY", "SQ_BUSY_CYCLES", "GRBM_GUI_ACTIVE")


def sq(csv_path: str, agent_csv: str, kernel: str):
    """Instruction mix and issue load of one kernel per launch size, from a rocprofv3 --pmc run
    of SQ_COUNTERS. A wave64 VALU (or SALU) instruction holds its SIMD's issue slot of that
    type for 4 cycles; GRBM_GUI_ACTIVE sums the busy cycles of every XCD, so a launch lasts
    GRBM_GUI_ACTIVE / XCDs cycles and the slot load is 4 * instructions / (SIMDs * cycles)."""
    gpu = [r for r in csv.DictReader(open(agent_csv)) if int(r.get("Simd_Count") or 0) > 0][0]
    simds, xcds = int(gpu["Simd_Count"]), int(gpu["Num_Xcc"])
    per = defaultdict(dict)
    for r in csv.DictReader(open(csv_path)):
        if short_name(r["Kernel_Name"]).split("<")[0] != kernel:
            continue
        d = per[r["Dispatch_Id"]]
        d[r["Counter_Name"]] = float(r["Counter_Value"])
        d["name"] = short_name(r["Kernel_Name"])
        d["grid"] = int(r["Grid_Size"])
        d["dur"] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    groups = defaultdict(list)
    for d in per.values():
        groups[(d["name"], d["grid"])].append(d)
    out = []
    for (name, grid), ds in sorted(groups.items(), key=lambda kv: kv[0][1]):
        m = {c: sum(d[c] for d in ds) / len(ds) for c in SQ_COUNTERS + ("dur",)}
        cyc = m["GRBM_GUI_ACTIVE"] / xcds
        out.append(dict(kernel=name, grid=grid, launches=len(ds), us=m["dur"] * 1e6,
                        clock_ghz=cyc / m["dur"] / 1e9, waves=m["SQ_WAVES"],
                        valu_per_wave=m["SQ_INSTS_VALU"] / m["SQ_WAVES"],
                        salu_per_wave=m["SQ_INSTS_SALU"] / m["SQ_WAVES"],
                        lds_per_wave=m["SQ_INSTS_LDS"] / m["SQ_WAVES"],
                        valu_slot_load=4 * m["SQ_INSTS_VALU"] / (simds * cyc),
                        salu_slot_load=4 * m["SQ_INSTS_SALU"] / (simds * cyc),
                        wait_share=m["SQ_WAIT_INST_ANY"] / m["SQ_WAVE_CYCLES"]))
    return dict(kernel=kernel, simds=simds, xcds=xcds, rows=out, kernel_source_hash=kernel_source_hash(kernel))


def sq_md(t, cmd: str) -> str:
    out = [f"# Instruction mix and issue load: `{t['kernel']}`", "", "Command:", "", "```", cmd, "```", "",
           f"Kernel source hash: `{t['kernel_source_hash']}`", "",
           f"{t['simds']} SIMDs in {t['xcds']} XCDs. A wave64 VALU or SALU instruction holds its SIMD's "
           "issue slot of that type for 4 cycles; a launch lasts GRBM_GUI_ACTIVE / XCDs cycles (the "
           "clock column is those cycles over the launch's timestamps). Slot load = 4 x instructions / "
           "(SIMDs x cycles); waiting = SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES (share of wave time spent "
           "waiting for a dependency before the next instruction could issue).", "",
           "| kernel | grid | launches | us | clock GHz | waves | VALU / wave | SALU / wave | LDS / wave "
           "| VALU slot load | SALU slot load | waiting |",
           "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for r in t["rows"]:
        out.append(f"| `{r['kernel']}` | {r['grid']} | {r['launches']} | {r['us']:.1f} | {r['clock_ghz']:.2f} "
                   f"| {r['waves']:.0f} | {r['valu_per_wave']:.0f} | {r['salu_per_wave']:.0f} "
                   f"| {r['lds_per_wave']:.0f} | {100 * r['valu_slot_load']:.1f}% | {100 * r['salu_slot_load']:.1f}% "
                   f"| {100 * r['wait_share']:.1f}% |")
    return "\n".join(out) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd_name", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("--cmd", default="")
    a.add_argument("--md")
    b = sub.add_parser("traffic")
    b.add_argument("--fetch", required=True)
    b.add_argument("--write", required=True)
    b.add_argument("--kernel", required=True)
    b.add_argument("--copy-bytes", type=int, required=True)
    b.add_argument("--cmd", default="")
    b.add_argument("--json")
    b.add_argument("--md")
    c = sub.add_parser("l2")
    c.add_argument("csv")
    c.add_argument("--cmd", default="")
    c.add_argument("--json")
    c.add_argument("--md")
    e = sub.add_parser("sq")
    e.add_argument("csv")
    e.add_argument("--agent", required=True, help="the run's agent_info.csv")
    e.add_argument("--kernel", default="k_grad_shift")
    e.add_argument("--cmd", default="")
    e.add_argument("--json")
    e.add_argument("--md")
    args = ap.parse_args(argv)
    if args.cmd_name == "sq":
        t = sq(args.csv, args.agent, args.kernel)
        if args.json:
            json.dump(t, open(args.json, "w"), indent=1)
        md = sq_md(t, args.cmd)
        if args.md:
            open(args.md, "w").write(md)
        print(md)
        return
    if args.cmd_name == "l2":
        t = l2(args.csv)
        if args.json:
            json.dump(t, open(args.json, "w"), indent=1)
        md = l2_md(t, args.cmd)
        if args.md:
            open(args.md, "w").write(md)
        print(md)
    elif args.cmd_name == "stats":
        md = stats_md(read_stats(args.csv), args.cmd)
        if args.md:
            open(args.md, "w").write(md)
        print(md)
    else:
        t = traffic(args.fetch, args.write, args.kernel, args.copy_bytes)
        if args.json:
            json.dump(t, open(args.json, "w"), indent=1)
        md = traffic_md(t, args.cmd)
        if args.md:
            open(args.md, "w").write(md)
        print(md)


if __name__ == "__main__":
    main()
