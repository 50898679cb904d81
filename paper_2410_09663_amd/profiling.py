"""Summaries of rocprofv3 output for the committed profiles.

Reads the CSV files rocprofv3 writes (``--kernel-trace --stats``: *_kernel_stats.csv and
*_kernel_trace.csv; ``--pmc``: *_counter_collection.csv) and prints the Markdown tables
kept under profiles/, and the per-class HBM traffic record the benchmark reads
(profiles/traffic.json).  Nothing here runs on the GPU.

  python -m paper_2410_09663_amd.profiling trace DIR
  python -m paper_2410_09663_amd.profiling traffic --fetch DIR --write DIR \
        --copy-fetch DIR --copy-write DIR [--tag C4_fp32 --json profiles/traffic.json]
  python -m paper_2410_09663_amd.profiling counters DIR [DIR ...]

Kernels map to the benchmark's kernel classes by name.  Dispatches of a class whose grid
is below 1/16 of the class's largest grid (the batch-1 plant step, or the one-workgroup
factorisation beside chip-wide launches) are listed on their own rows and left out of
the class's per-launch traffic.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import OrderedDict, defaultdict

PKG = os.path.dirname(os.path.abspath(__file__))

CLASS_OF = [  # kernel-name prefix -> class, first match wins
    ("k_conv_first", "conv_first"), ("k_conv_last", "conv_last"), ("k_conv_mfma", "conv_mid"),
    ("k_conv_f32r", "conv_mid"), ("k_conv_bf16r", "conv_mid"), ("k_center", "means"),
    ("k_conv_direct", "conv_mid"), ("k_lift", "lift"), ("k_stats_reduce", "stats_reduce"),
    ("k_stats", "stats"), ("k_update", "update"), ("k_chol", "chol"), ("k_potrf", "chol"),
    ("k_gain", "gain"), ("k_normals", "noise"), ("k_means", "means"), ("k_init_slice0", "init"),
    ("k_assemble", "assemble"), ("k_observe", "observe"), ("k_constraint", "observe"),
    ("k_extract", "extract"), ("k_copy_jobs", "copy"), ("k_zero_u32", "assemble"),
    ("k_split_gain", "update"),
]
SOURCE_OF = {"conv_first": "rollout.hip", "conv_mid": "rollout.hip", "conv_last": "rollout.hip",
             "stats": "stats.hip", "stats_reduce": "stats.hip", "means": "stats.hip", "chol": "gain.hip",
             "gain": "gain.hip", "update": "update.hip", "noise": "noise.hip", "assemble": "noise.hip",
             "observe": "noise.hip", "init": "noise.hip", "extract": "update.hip", "copy": "noise.hip",
             "lift": "rollout.hip"}


def _demangle_simple(name: str) -> str:
    """Names the profiler left mangled (e.g. with __bf16 parameters): the function
    identifier in the library's anonymous namespace and its integer / bool template
    arguments, as 'k_name<a, b>'."""
    m = re.match(r"_ZN3oic12_GLOBAL__N_1(\d+)", name)
    if not m:
        return name
    k = int(m.group(1))
    ident = name[m.end():m.end() + k]
    rest = name[m.end() + k:]
    args = []
    if rest.startswith("I"):
        for a in re.finditer(r"L([ib])(\d+)E", rest[1:rest.find("EE") + 2] if "EE" in rest else rest[1:]):
            args.append(("true" if a.group(2) == "1" else "false") if a.group(1) == "b" else a.group(2))
    return f"{ident}<{', '.join(args)}>" if args else ident


def kernel_class(name: str) -> str:
    name = _demangle_simple(name)
    base = name.replace("(anonymous namespace)::", "").split("(")[0].strip()
    base = re.sub(r"^(void\s+)?(\w+::)*", "", base)
    for prefix, cls in CLASS_OF:
        if base.startswith(prefix):
            return cls
    return "-"


def short_name(name: str) -> str:
    """Kernel name without namespaces, parameter list and 'void'."""
    name = _demangle_simple(name)
    s = re.sub(r"\(.*$", "", name.replace("(anonymous namespace)::", "").strip())
    s = re.sub(r"^void\s+", "", s)
    s = re.sub(r"\boic::(\(anonymous namespace\)::)?", "", s)
    return s.strip()


def _rows(directory, suffix):
    files = sorted(glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {directory}")
    out = []
    for f in files:
        with open(f, newline="") as fh:
            out.extend(csv.DictReader(fh))
    return out


def _col(row, *names):
    for n in names:
        if n in row and row[n] != "":
            return row[n]
    raise KeyError(f"none of {names} in {list(row)}")


def _grid(row):
    for n in ("Grid_Size", "Grid_Size_X"):
        if n in row and row[n] != "":
            g = int(float(row[n]))
            if n == "Grid_Size_X":
                g *= int(float(row.get("Grid_Size_Y", 1) or 1)) * int(float(row.get("Grid_Size_Z", 1) or 1))
            return g
    return 0


def _wg(row):
    for n in ("Workgroup_Size", "Workgroup_Size_X"):
        if n in row and row[n] != "":
            w = int(float(row[n]))
            if n == "Workgroup_Size_X":
                w *= int(float(row.get("Workgroup_Size_Y", 1) or 1)) * int(float(row.get("Workgroup_Size_Z", 1) or 1))
            return w
    return 0


def _small(grid, class_max):
    return class_max > 0 and grid * 16 < class_max


def trace_table(directory):
    """Per (kernel, launch size) rows from the kernel trace: calls, average and total
    duration, share, registers, LDS and workgroup size."""
    rows = _rows(directory, "_kernel_trace.csv")
    groups = OrderedDict()
    class_max = defaultdict(int)
    for r in rows:
        name = _col(r, "Kernel_Name")
        g = _grid(r)
        class_max[kernel_class(name)] = max(class_max[kernel_class(name)], g)
    total_all = 0.0
    for r in rows:
        name = _col(r, "Kernel_Name")
        dur = (int(_col(r, "End_Timestamp")) - int(_col(r, "Start_Timestamp"))) * 1e-3  # us
        total_all += dur
        cls = kernel_class(name)
        small = _small(_grid(r), class_max[cls])
        key = (short_name(name), small)
        e = groups.setdefault(key, {"calls": 0, "us": 0.0, "cls": cls,
                                    "vgpr": r.get("VGPR_Count", r.get("Arch_VGPR_Count", "")),
                                    "agpr": r.get("Accum_VGPR_Count", ""), "lds": r.get("LDS_Block_Size", ""),
                                    "scratch": r.get("Scratch_Size", ""), "wg": _wg(r), "grid": _grid(r)})
        e["calls"] += 1
        e["us"] += dur
    lines = ["| kernel | class | calls | avg us | total us | % | vgpr | agpr | lds B | scratch B | wg |",
             "|---|---|---|---|---|---|---|---|---|---|---|"]
    for (name, small), e in sorted(groups.items(), key=lambda kv: -kv[1]["us"]):
        label = f"`{name}`" + (" (small grid)" if small else "")
        lines.append(f"| {label} | {e['cls']} | {e['calls']} | {e['us'] / e['calls']:.1f} | {e['us']:.0f} | "
                     f"{100 * e['us'] / total_all:.1f} | {e['vgpr']} | {e['agpr']} | {e['lds']} | "
                     f"{e['scratch']} | {e['wg']} |")
    return "\n".join(lines), groups


def counter_values(directory):
    """{dispatch id: (kernel name, grid, {counter: value})} from a --pmc run."""
    out = {}
    for r in _rows(directory, "_counter_collection.csv"):
        d = int(_col(r, "Dispatch_Id", "Correlation_Id"))
        name = _col(r, "Kernel_Name")
        e = out.setdefault(d, (name, _grid(r), defaultdict(float)))
        e[2][_col(r, "Counter_Name")] += float(_col(r, "Counter_Value"))
    return out


def copy_factor(directory, counter, copy_bytes):
    """Counter value (KiB) per byte of a plain device copy of copy_bytes, from the copy
    kernels of a `bench.py --calibrate-copy` run."""
    vals = [v[counter] for name, g, v in counter_values(directory).values() if "copy" in name.lower()
            and v[counter] > 0]
    if not vals:
        raise SystemExit(f"no copy dispatch with {counter} under {directory}")
    vals.sort()
    return vals[len(vals) // 2] * 1024.0 / copy_bytes


def traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_bytes=256 << 20):
    ff = copy_factor(copy_fetch_dir, "FETCH_SIZE", copy_bytes)
    fw = copy_factor(copy_write_dir, "WRITE_SIZE", copy_bytes)
    per = OrderedDict()
    class_max = defaultdict(int)
    fetch, write = counter_values(fetch_dir), counter_values(write_dir)
    for vals in (fetch, write):
        for name, g, _ in vals.values():
            class_max[kernel_class(name)] = max(class_max[kernel_class(name)], g)
    for vals, counter in ((fetch, "FETCH_SIZE"), (write, "WRITE_SIZE")):
        for name, g, v in vals.values():
            cls = kernel_class(name)
            small = _small(g, class_max[cls])
            e = per.setdefault((short_name(name), small), {"cls": cls, "FETCH_SIZE": [], "WRITE_SIZE": []})
            e[counter].append(v[counter])
    lines = [f"Calibration: a plain {copy_bytes >> 20} MiB device copy reads FETCH_SIZE = "
             f"{ff * copy_bytes / 1024:.0f} KiB and WRITE_SIZE = {fw * copy_bytes / 1024:.0f} KiB, so the "
             f"factors are {ff:.4f} (fetch) and {fw:.4f} (write); HBM bytes = FETCH_SIZE / f + WRITE_SIZE / w.",
             "", "| kernel | class | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM MB per dispatch |",
             "|---|---|---|---|---|---|"]
    classes = defaultdict(lambda: [0.0, 0])
    rows = []
    for (name, small), e in per.items():
        nf, nw = len(e["FETCH_SIZE"]), len(e["WRITE_SIZE"])
        if not nf or not nw:
            continue
        f = sum(e["FETCH_SIZE"]) / nf
        w = sum(e["WRITE_SIZE"]) / nw
        mb = (f * 1024 / ff + w * 1024 / fw) / 1e6
        rows.append((mb * max(nf, nw), f"| `{name}`{' (small grid)' if small else ''} | {e['cls']} | "
                                       f"{max(nf, nw)} | {f:.1f} | {w:.1f} | {mb:.2f} |"))
        if not small and e["cls"] != "-":
            classes[e["cls"]][0] += mb * 1e6 * max(nf, nw)
            classes[e["cls"]][1] += max(nf, nw)
    lines += [r for _, r in sorted(rows, key=lambda x: -x[0])]
    return "\n".join(lines), {c: (b / n, n) for c, (b, n) in classes.items()}


def update_traffic_json(path, tag, per_class):
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        rec = {}
    if not isinstance(rec, dict) or any("hbm_bytes_per_launch" in v for v in rec.values()
                                          if isinstance(v, dict)):
        rec = {}  # older flat layout
    entry = {}
    for cls, (b, n) in sorted(per_class.items()):
        src = SOURCE_OF.get(cls)
        if not src:
            continue
        with open(os.path.join(PKG, "csrc", src), "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
        entry[cls] = {"hbm_bytes_per_launch": b, "launches_measured": n, "source": src,
                      "source_sha256": sha}
    rec[tag] = entry
    with open(path, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
        f.write("\n")


def counters_table(dirs):
    """Per kernel, every counter of one or more --pmc runs, summed over its dispatches and
    divided by the dispatch count."""
    per = OrderedDict()
    names = []
    class_max = defaultdict(int)
    runs = [counter_values(d) for d in dirs]
    for vals in runs:
        for name, g, _ in vals.values():
            class_max[kernel_class(name)] = max(class_max[kernel_class(name)], g)
    for vals in runs:
        for name, g, v in vals.values():
            small = _small(g, class_max[kernel_class(name)])
            e = per.setdefault((short_name(name), small), defaultdict(list))
            for c, x in v.items():
                e[c].append(x)
                if c not in names:
                    names.append(c)
    # derived: matrix-core busy fraction (GRBM_GUI_ACTIVE sums the 8 XCDs, the MFMA busy
    # cycles the 1024 SIMDs) and LDS bank-conflict cycles per LDS instruction
    derived = []
    if "GRBM_GUI_ACTIVE" in names and "SQ_VALU_MFMA_BUSY_CYCLES" in names:
        derived.append(("MFMA busy", lambda e: (_mean(e, "SQ_VALU_MFMA_BUSY_CYCLES") / 1024.0) /
                        max(_mean(e, "GRBM_GUI_ACTIVE") / 8.0, 1e-30), "{:.1%}"))
    if "SQ_INSTS_LDS" in names and "SQ_LDS_BANK_CONFLICT" in names:
        derived.append(("LDS conflict cycles / LDS instr", lambda e: _mean(e, "SQ_LDS_BANK_CONFLICT") /
                        max(_mean(e, "SQ_INSTS_LDS"), 1e-30), "{:.2f}"))
    lines = ["| kernel | dispatches | " + " | ".join(names + [d[0] for d in derived]) + " |",
             "|---|---|" + "---|" * (len(names) + len(derived))]
    for (name, small), e in per.items():
        cells = [f"{sum(e[c]) / len(e[c]):.4g}" if e.get(c) else "" for c in names]
        cells += [fmt.format(f(e)) if all(e.get(c) for c in names[:1]) else "" for _, f, fmt in derived]
        cnt = max(len(v) for v in e.values()) if e else 0
        lines.append(f"| `{name}`{' (small grid)' if small else ''} | {cnt} | " + " | ".join(cells) + " |")
    return "\n".join(lines)


def _mean(e, c):
    v = e.get(c) or [0.0]
    return sum(v) / len(v)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    tr = sub.add_parser("traffic")
    tr.add_argument("--fetch", required=True)
    tr.add_argument("--write", required=True)
    tr.add_argument("--copy-fetch", required=True)
    tr.add_argument("--copy-write", required=True)
    tr.add_argument("--tag")
    tr.add_argument("--json")
    c = sub.add_parser("counters")
    c.add_argument("dirs", nargs="+")
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        print(trace_table(a.dir)[0])
    elif a.cmd == "traffic":
        table, per_class = traffic(a.fetch, a.write, a.copy_fetch, a.copy_write)
        print(table)
        if a.json and a.tag:
            update_traffic_json(a.json, a.tag, per_class)
    else:
        print(counters_table(a.dirs))


if __name__ == "__main__":
    sys.exit(main())
