#!/usr/bin/env python3
"""Throughput of the multi-component LBM step on one MI355X.

Workload (default): two-component D3Q19 Shan-Chen flow + D3Q7 reactive solute
in a 256^3 seeded Boolean sphere pack (porosity 0.4, R = 8), body force along
x, first-order wall reaction k = 1e-3, FP32 storage and arithmetic.  Inputs are
synthetic and already resident in HBM when the timed region starts.  A step is
one full pass of the path: densities and pseudo-potentials, interaction
forces, Guo velocity, BGK collision, streaming with bounce-back, the solute
collision with wet-node reaction and inlet/outlet, plus the FP64 monitors that
run every ``monitor_every`` steps.

Prints ONE JSON line (contract): metric MLUPS (box-node updates per second,
every component and the solute counted once per node), roofline of the step
kernel against the 8 TB/s HBM peak (algorithmic bytes: 361 B per fluid-node
update), and the CPU oracle timed on this host's cores on a bounded sample
(the first steps of the same 256^3 state).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per fluid-node update: populations read once and written
# once (2 x 19 flow + 7 solute values) plus one mask byte
ALG_BYTES = {"f32": 2 * (2 * 19 + 7) * 4 + 1, "f64": 2 * (2 * 19 + 7) * 8 + 1,
             "f16s": 2 * (2 * 19 + 7) * 2 + 1, "bf16s": 2 * (2 * 19 + 7) * 2 + 1}
def traffic_from_profiles(storage, n, nfluid):
    """HBM bytes per launch from committed rocprofv3 PMC summaries, if they were
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_step_{storage}_{n}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    from paper_2502_12955_amd.profile_summary import kernel_hash

    if d.get("kernel_hash") != kernel_hash():
        return None
    return d.get("bytes_per_launch")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(p, mask, rho, C, steps, steps_single):
    """The FP64 C oracle on this host: `steps` steps of the benchmark state with
    every host core, then `steps_single` steps with one thread (bounded samples
    of the same workload)."""
    import numpy as np

    import oracle

    m, _ = oracle.pinch_fill(p, mask)
    f, h = oracle.init(p, m, rho, None, C)
    N = int(np.prod(mask.shape))
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    all_cores = oracle.set_threads(cores)
    t0 = time.perf_counter()
    oracle.step(p, m, f, h, steps)
    dt = time.perf_counter() - t0
    one = oracle.set_threads(1)
    t1 = time.perf_counter()
    oracle.step(p, m, f, h, steps_single)
    dt1 = time.perf_counter() - t1
    oracle.set_threads(all_cores)
    shape = f"{mask.shape[2]}x{mask.shape[1]}x{mask.shape[0]}"
    return {"value": round(N * steps / dt / 1e6, 4), "unit": "MLUPS", "cores": all_cores, "kind": "oracle",
            "sample": f"{steps} steps of the same {shape} state (plain C FP64 oracle, OpenMP over nodes, "
                      f"{all_cores} threads), {dt:.1f} s",
            "single_thread": {"value": round(N * steps_single / dt1 / 1e6, 4), "unit": "MLUPS", "cores": one,
                              "sample": f"{steps_single} step(s) of the same state, 1 thread, {dt1:.1f} s"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--n", type=int, default=256, help="edge of the cubic sphere-pack box")
    ap.add_argument("--storage", default="f32", choices=["f32", "f64", "f16s", "bf16s"])
    ap.add_argument("--block", type=int, default=0,
                    help="threads per workgroup of the step kernels (0: the native tuner picks the launch shape)")
    ap.add_argument("--grid", type=int, default=0, help="persistent grid blocks with --block (0: one pass)")
    ap.add_argument("--cpu-steps", type=int, default=8, help="oracle steps timed on all host cores")
    ap.add_argument("--cpu-steps-single", type=int, default=1, help="oracle steps timed on one thread")
    ap.add_argument("--no-ceiling", action="store_true", help="skip the HBM probe kernels")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the path runs on a single GPU; sharding across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2502_12955_amd import inputs, mclbm

    rank = int(os.environ.get("RANK", "0"))
    torch.cuda.set_device(0)
    t0 = time.time()
    p, mask, rho, u, C = inputs.porous_case(n=args.n, storage=args.storage)
    log(f"[bench] workload generated in {time.time() - t0:.1f} s")

    lat = mclbm.Lattice(p)
    nrc = lat.set_geometry(mask)
    if args.block == 0:
        nb, blk, grd, ms = lat.autotune(trial_steps=10)
        log(f"[bench] tuned: {nb or 8} bands, block {blk}, grid {grd} ({ms:.3f} ms/step)")
    else:
        nb, blk, grd = 0, args.block, args.grid
        lat.set_launch(blk, grd)
    gmask, _, _ = lat.get_geometry()
    nfluid = int((gmask == 0).sum())
    lat.init_fields(rho, None, C)
    log(f"[bench] lattice ready: {args.n}^3, fluid {nfluid}, reclassified {nrc}")

    stream = lat.stream
    if args.calib_copy_mib:
        src = torch.ones(args.calib_copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    lat.step(args.warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t_start = time.perf_counter()
    ev0.record(stream)
    lat.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    gpu_ms = ev0.elapsed_time(ev1)
    log(f"[bench] {args.steps} steps: {gpu_ms:.1f} ms (events), {wall * 1e3:.1f} ms (wall)")
    mon = lat.monitors()

    N = args.n ** 3
    ms_per_step = max(gpu_ms, wall * 1e3) / args.steps
    mlups = N / (ms_per_step * 1e-3) / 1e6
    launch_ms = gpu_ms / args.steps
    alg_bytes = ALG_BYTES[args.storage] * nfluid
    achieved = alg_bytes / (launch_ms * 1e-3) / 1e9
    traffic = traffic_from_profiles(args.storage, args.n, nfluid)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "mcmp step (k_density + k_collide)", "alg_bytes_per_launch": alg_bytes,
                "launch_ms": round(launch_ms, 4)}

    if not args.no_ceiling:
        # measured HBM ceiling of this device (streaming kernels of the library)
        lat.close()
        torch.cuda.synchronize()
        ceiling = {k: round(max(mclbm.hbm_probe(k, nbytes=2 << 30, blocks_per_cu=b, iters=3)
                                for b in (2, 4, 8, 16)), 1)
                   for k in ("read", "write", "copy")}
        roofline["measured_ceiling_gbs"] = ceiling
        roofline["frac_of_copy_ceiling"] = round(achieved / ceiling["copy"], 4)

    cpu = None
    if rank == 0 and not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle ...")
        cpu = cpu_baseline(p, mask, rho, C, args.cpu_steps, args.cpu_steps_single)

    out = {
        "metric": "MLUPS", "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"f32": "f32", "f64": "f64", "f16s": "f16 storage / f32 arithmetic",
                  "bf16s": "bf16 storage / f32 arithmetic"}[args.storage],
        "data": "synthetic",
        "config": {"workload": f"D3Q19 two-component Shan-Chen + D3Q7 reactive solute, {args.n}^3 "
                               f"Boolean sphere pack porosity 0.4 R=8, Guo forcing, body force x 1e-5, "
                               f"wall reaction k=1e-3, inlet/outlet solute",
                   "nodes": N, "fluid_nodes": nfluid, "storage": args.storage,
                   "launch": {"block": blk, "grid": grd, "bands": nb or 8},
                   "mflups": round(nfluid / (ms_per_step * 1e-3) / 1e6, 1),
                   "monitor_every": p["monitor_every"], "final_residual": float(mon[9])},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    lat.close()
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
