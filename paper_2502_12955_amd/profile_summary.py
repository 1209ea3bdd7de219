"""Summaries of rocprofv3 output for the committed profile records.

    python -m paper_2502_12955_amd.profile_summary kernels DIR OUT.md --cmd "..."
        kernel-trace statistics (``*_kernel_stats.csv``) as a short markdown table

    python -m paper_2502_12955_amd.profile_summary traffic FETCH_DIR WRITE_DIR OUT.json OUT.md \
        --copy-mib M --fluid F --alg-bytes B --cmd-fetch "..." --cmd-write "..."
        HBM bytes per step of the step kernels from two ``--pmc`` runs
        (FETCH_SIZE, WRITE_SIZE in KiB per dispatch), each scaled by what the
        same counter reads for a plain device copy of M MiB in the same run.

The traffic record carries the hash of the kernel sources it was measured on,
so the benchmark reports it only while the kernels are unchanged.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ("paper_2502_12955_amd/csrc/kernels.hip", "paper_2502_12955_amd/csrc/node.hpp",
                  "paper_2502_12955_amd/csrc/common.hpp")
STEP_KERNELS = ("k_density", "k_collide")


def kernel_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short(name):
    m = re.search(r"(\w+)(<[^()]*>)?\(", name)
    if not m:
        return name[:60]
    return m.group(1) + (m.group(2) or "")


def _one(pattern):
    hits = sorted(glob.glob(pattern, recursive=True))
    if not hits:
        raise FileNotFoundError(pattern)
    return hits[0]


def kernels(args):
    path = _one(os.path.join(args.dir, "**", "*kernel_stats.csv"))
    rows = list(csv.DictReader(open(path)))
    lines = [f"# Kernel statistics: {args.title}", "", "Command:", "", "```", args.cmd, "```", "",
             "| kernel | calls | avg (us) | min (us) | max (us) | share |", "|---|---|---|---|---|---|"]
    step_avg = 0.0
    for r in rows:
        n = short(r["Name"])
        avg = float(r["AverageNs"]) / 1e3
        if any(k in n for k in STEP_KERNELS):
            step_avg += avg
        lines.append(f"| `{n}` | {r['Calls']} | {avg:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} % |")
    if step_avg > 0:
        lines += ["", f"Sum of the average durations of the step kernels ({', '.join(STEP_KERNELS)}): "
                      f"{step_avg:.1f} us per step."]
    lines.append("")
    with open(args.out, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


def _counter(dirname, counter):
    path = _one(os.path.join(dirname, "**", "*counter_collection.csv"))
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return agg


def traffic(args):
    out = {}
    for counter, d in (("FETCH_SIZE", args.fetch_dir), ("WRITE_SIZE", args.write_dir)):
        agg = _counter(d, counter)
        copy = [v for k, v in agg.items() if "copyBuffer" in k]
        if not copy:
            raise RuntimeError(f"no copy kernel in the {counter} run")
        copy_kib = max(max(v) for v in copy)   # the calibration copy is the largest one
        factor = args.copy_mib * 1024.0 / copy_kib
        step = {}
        for k, v in agg.items():
            n = short(k)
            for sk in STEP_KERNELS:
                if sk in n:
                    step[sk] = sum(v) / len(v) * 1024.0 * factor
        out[counter] = dict(copy_kib=copy_kib, factor=factor, bytes_per_launch=step)
    fetch = sum(out["FETCH_SIZE"]["bytes_per_launch"].values())
    write = sum(out["WRITE_SIZE"]["bytes_per_launch"].values())
    rec = dict(kernel_hash=kernel_hash(), bytes_per_launch=round(fetch + write),
               fetch_bytes=round(fetch), write_bytes=round(write),
               per_kernel={k: dict(fetch=round(out["FETCH_SIZE"]["bytes_per_launch"].get(k, 0.0)),
                                   write=round(out["WRITE_SIZE"]["bytes_per_launch"].get(k, 0.0)))
                           for k in STEP_KERNELS},
               fetch_factor=out["FETCH_SIZE"]["factor"], write_factor=out["WRITE_SIZE"]["factor"],
               algorithmic_bytes=args.alg_bytes * args.fluid, fluid_nodes=args.fluid,
               copy_mib=args.copy_mib)
    with open(args.out_json, "w") as f:
        json.dump(rec, f, indent=1)
    lines = [f"# HBM traffic per step: {args.title}", "",
             "Counters: FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each from its own run, scaled by "
             f"the factor that makes a plain {args.copy_mib} MiB device copy in the same run read and "
             "write exactly its size.", "", "Commands:", "", "```", args.cmd_fetch, args.cmd_write, "```", "",
             f"| | fetch | write |", "|---|---|---|",
             f"| copy kernel reading / writing {args.copy_mib} MiB (KiB) | {out['FETCH_SIZE']['copy_kib']:.0f} | "
             f"{out['WRITE_SIZE']['copy_kib']:.0f} |",
             f"| scale factor | {rec['fetch_factor']:.3f} | {rec['write_factor']:.3f} |"]
    for k in STEP_KERNELS:
        pk = rec["per_kernel"][k]
        lines.append(f"| `{k}` bytes per launch | {pk['fetch'] / 1e9:.3f} GB | {pk['write'] / 1e9:.3f} GB |")
    lines += ["", f"Step total: {rec['bytes_per_launch'] / 1e9:.3f} GB per step; algorithmic "
                  f"{args.alg_bytes} B x {args.fluid} fluid nodes = {rec['algorithmic_bytes'] / 1e9:.3f} GB "
                  f"(ratio {rec['bytes_per_launch'] / rec['algorithmic_bytes']:.2f}).",
              f"Kernel source hash: `{rec['kernel_hash']}`.", ""]
    with open(args.out_md, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="what", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("dir")
    k.add_argument("out")
    k.add_argument("--cmd", required=True)
    k.add_argument("--title", default="")
    t = sub.add_parser("traffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    t.add_argument("out_json")
    t.add_argument("out_md")
    t.add_argument("--copy-mib", type=float, required=True)
    t.add_argument("--fluid", type=int, required=True)
    t.add_argument("--alg-bytes", type=int, required=True)
    t.add_argument("--cmd-fetch", required=True)
    t.add_argument("--cmd-write", required=True)
    t.add_argument("--title", default="")
    args = ap.parse_args(argv)
    (kernels if args.what == "kernels" else traffic)(args)


if __name__ == "__main__":
    main()
