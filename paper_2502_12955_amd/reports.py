"""Measurement studies beyond the single-lattice benchmark.

    python -m paper_2502_12955_amd.reports precision [--n 384 --steps 20000]
        Reduced-precision storage (FP16 / BF16 shifted, FP32) against an FP64
        run on the GPU from the same state: per-field max-abs and RMS error
        over fluid nodes after ``steps``, throughput of each storage, and the
        residual history of each storage on a smaller box (steps to the
        tolerance, or the floor reached).

    python -m paper_2502_12955_amd.reports thermal [--n 256 --steps 500]
        Conjugate heat transfer on the benchmark lattice: step time with and
        without the energy fields, node counts of the solid list and the
        interface, interface iterations per solve.

    python -m paper_2502_12955_amd.reports variants [--n 256 --steps 500]
        Step time of the benchmark lattice with the product species, the
        per-node rate field, both, one component, and of the 128 x 64 FP64
        droplet (latency: its state fits the caches).

    python -m paper_2502_12955_amd.reports batch [--count 64]
        A batch of samples with independent per-axis edges in {32, 48, 64,
        96, 128}: aggregate throughput of the batched, graph-replayed run
        against the samples run one after another, and the run to a residual
        tolerance with per-sample convergence.

Each prints one JSON line (and writes it to --out if given).
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import inputs, mclbm

FIELDS = ("rho1", "rho2", "phi", "u_x", "u_y", "u_z", "|u|", "C")


def _fields(rho, u, C, fluid):
    r0, r1 = rho[0][fluid], rho[1][fluid]
    tot = r0 + r1
    ux, uy, uz = u[0][fluid], u[1][fluid], u[2][fluid]
    return dict(rho1=r0, rho2=r1, phi=(r0 - r1) / tot, u_x=ux, u_y=uy, u_z=uz,
                **{"|u|": np.sqrt(ux * ux + uy * uy + uz * uz)}, C=C[0][fluid] if C.ndim > 1 else C[fluid])


def _timed_steps(lat, steps):
    import torch

    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(lat.stream)
    lat.step(steps)
    e1.record(lat.stream)
    torch.cuda.synchronize()
    return max(e0.elapsed_time(e1), (time.perf_counter() - t0) * 1e3)


def _residual_history(p, mask, rho, C, tol, cap):
    lat = mclbm.Lattice(p)
    lat.set_graph(True)
    lat.set_geometry(mask)
    lat.init_fields(rho, None, C)
    K = p["monitor_every"]
    hist, reached, floor = [], None, np.inf
    t0 = time.perf_counter()
    done = 0
    while done < cap:
        lat.step(K)
        done += K
        m = lat.monitors()
        r = float(m[9])
        if done > K:
            floor = min(floor, r)
            if done % (10 * K) == 0:
                hist.append((done, r, float(m[4]), float(m[5]), float(m[6])))
            if r <= tol and reached is None:
                reached = done
                break
    lat.synchronize()
    wall = time.perf_counter() - t0
    lat.close()
    return dict(steps_to_tol=reached, floor=floor, wall_s=wall, history=hist)


def precision(args):
    out = dict(study="reduced-precision storage", n=args.n, steps=args.steps)
    p, mask, rho, _, C = inputs.porous_case(n=args.n, config=3)
    ref = None
    res = {}
    for storage in ["f64"] + args.storages:
        q = dict(p, storage=storage)
        lat = mclbm.Lattice(q)
        lat.set_geometry(mask)
        gmask, _, _ = lat.get_geometry()
        fluid = gmask.reshape(-1) == 0
        lat.init_fields(rho, None, C)
        ms = _timed_steps(lat, args.steps)
        r, u, c = lat.moments()
        lat.close()
        f = _fields(r.reshape(2, -1), u.reshape(3, -1), c.reshape(1, -1), fluid)
        entry = dict(ms_per_step=ms / args.steps, mlups=args.n ** 3 / (ms / args.steps * 1e-3) / 1e6)
        if ref is None:
            ref = f
        else:
            err = {}
            for k in FIELDS:
                d = f[k] - ref[k]
                scale = float(np.abs(ref[k]).max())
                err[k] = dict(max_abs=float(np.abs(d).max()), rms=float(np.sqrt(np.mean(d * d))),
                              max_rel_to_field_max=float(np.abs(d).max() / scale) if scale else None)
            entry["error_vs_f64"] = err
        res[storage] = entry
        print(f"[precision] {storage}: {entry['ms_per_step']:.3f} ms/step", flush=True)
    out["runs"] = res
    # residual histories on a smaller box
    p2, mask2, rho2, _, C2 = inputs.porous_case(n=args.res_n, config=3, sample=1)
    out["residual"] = dict(n=args.res_n, tol=args.tol, cap=args.cap)
    for storage in ["f64"] + args.storages:
        out["residual"][storage] = _residual_history(dict(p2, storage=storage), mask2, rho2, C2, args.tol, args.cap)
        print(f"[precision] residual {storage}: {out['residual'][storage]['steps_to_tol']} "
              f"floor {out['residual'][storage]['floor']:.3e}", flush=True)
    return out


def thermal(args):
    """The 256^3 porous workload with conjugate heat transfer (FP32): the fluid
    energy populations ride with the flow, the solid ones on the solid list,
    the interface solve runs per interface node with the Arrhenius rate law of
    the interface temperature (k(1) equal to the benchmark's uniform rate)."""
    p, mask, rho, _, C = inputs.porous_case(n=args.n, config=2, storage=args.storage)
    E_over_R = 1.5
    th = dict(tau_ef=0.85, tau_es=1.4, rhocp_f=1.0, rhocp_s=2.5, h_r=0.5, arr_A=p["k_wall"] * np.exp(E_over_R),
              arr_E_over_R=E_over_R, T_tol=1e-6, T_maxit=50)
    out = dict(study="conjugate heat transfer", n=args.n, steps=args.steps, storage=args.storage, thermal=th)
    res = {}
    for on in (False, True):
        lat = mclbm.Lattice(p)
        if on:
            lat.set_thermal(th)
        lat.set_geometry(mask)
        lat.init_fields(rho, None, C)
        if on:
            lat.init_temperature(np.ones(mask.size))
        lat.set_graph(True)
        lat.step(100)                    # warm-up and graph capture
        ms = _timed_steps(lat, args.steps) / args.steps
        entry = dict(ms_per_step=ms)
        if on:
            stats = lat.thermal_stats()
            gm, _, _ = lat.get_geometry()
            solid = gm.reshape(-1) != 0
            nz, ny, nx = mask.shape
            s3 = solid.reshape(nz, ny, nx)
            near = np.zeros_like(s3)
            for dz in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        if abs(dx) + abs(dy) + abs(dz) in (1, 2):   # the D3Q19 neighbours
                            near |= np.roll(s3, (dz, dy, dx), axis=(0, 1, 2))
            iface = int(np.count_nonzero(near & ~s3))
            T = lat.temperature()
            entry.update(fluid_nodes=int(np.count_nonzero(~solid)), solid_nodes=int(np.count_nonzero(solid)),
                         interface_nodes=iface, iterations_total=stats[0], unsettled=stats[1],
                         degenerate=stats[2],
                         iterations_per_solve=stats[0] / max(1, iface * (100 + args.steps)),
                         T_min=float(T.min()), T_max=float(T.max()))
        lat.close()
        res["thermal" if on else "flow_and_solute"] = entry
        print(f"[thermal] {'on' if on else 'off'}: {ms:.3f} ms/step", flush=True)
    out["runs"] = res
    return out


def variants(args):
    """Step time of the kernel variants on the benchmark lattice (FP32): the
    reacting solute alone, with the product species (eq:reactCO2), with a
    per-node rate field k(x) (eq:reactO2, from a prescribed temperature), with
    both, and a single component (the diagonal cohesion of eq:1.12, G = -5
    with the solute); plus the 2-D two-component droplet in FP64."""
    p, mask, rho, _, C = inputs.porous_case(n=args.n, config=2, storage=args.storage)
    nz, ny, nx = mask.shape
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    T = 1.0 + 0.1 * np.sin(2 * np.pi * xx / nx) * np.cos(2 * np.pi * zz / nz)
    kfield = inputs.arrhenius_rate_field(T, p["k_wall"] * np.exp(1.5), 1.5).reshape(-1)
    one = np.where(mask == 0, 1.0, 0.0)[None] * 0.15   # outside the spinodal of G = -5
    cases = [("reacting solute", dict(), None, rho),
             ("product species", dict(product=1, D2=0.12, C_in2=0.0), None, rho),
             ("rate field", dict(), kfield, rho),
             ("product species and rate field", dict(product=1, D2=0.12, C_in2=0.0), kfield, rho),
             ("one component, G = -5", dict(ncomp=1, G=((-5.0, 0.0), (0.0, 0.0)), G_ads=(0.0, 0.0)), None, one)]
    out = dict(study="kernel variants", n=args.n, steps=args.steps, storage=args.storage, runs={})
    nodes = nx * ny * nz
    for name, upd, kf, r in cases:
        q = dict(p, **upd)
        if kf is not None:
            q["rate_field"] = 1
        lat = mclbm.Lattice(q)
        lat.set_geometry(mask)
        if kf is not None:
            lat.set_wall_rate(kf)
        lat.init_fields(r, None, C)
        lat.set_graph(True)
        lat.step(100)
        ms = _timed_steps(lat, args.steps) / args.steps
        lat.close()
        out["runs"][name] = dict(ms_per_step=ms, mlups=nodes / (ms * 1e-3) / 1e6)
        print(f"[variants] {name}: {ms:.3f} ms/step", flush=True)
    p2, m2, r2, _, _ = inputs.droplet_2d_case(nx=128, ny=64, radius=20.0, storage="f64")
    lat = mclbm.Lattice(p2)
    lat.set_geometry(m2)
    lat.init_fields(r2)
    lat.set_graph(True)
    lat.step(200)
    ms = _timed_steps(lat, 2000) / 2000
    lat.close()
    out["runs"]["2-D droplet 128 x 64, FP64"] = dict(us_per_step=ms * 1e3, mlups=128 * 64 / (ms * 1e-3) / 1e6)
    print(f"[variants] droplet: {ms * 1e3:.1f} us/step", flush=True)
    return out


def batch(args):
    edges = inputs.batch_edges(args.count)
    cases = []
    for s, (ez, ey, ex) in enumerate(edges):
        por = 0.3 + 0.2 * inputs.SplitMix64(inputs.seed_for(4, 1000 + s)).uniform(1)[0]
        p, mask, rho, _, C = inputs.porous_case(shape=(ez, ey, ex), porosity=por, config=4, sample=s,
                                               storage=args.storage)
        cases.append((p, mask, rho, C))
    nodes = sum(int(np.prod(c[1].shape)) for c in cases)
    out = dict(study="batch of uneven samples", count=args.count, box_nodes=nodes, storage=args.storage,
               edges=edges)

    b = mclbm.Batch([c[0] for c in cases])
    b.set_geometry([c[1] for c in cases])
    tuned = b.autotune(trial_steps=5)
    b.set_graph(True)
    b.init_fields([c[2] for c in cases], None, [c[3] for c in cases])
    b.step(args.steps)  # warm-up and graph capture
    fluid = int(b.monitors()[8])
    ms = _timed_steps(b, args.steps)
    out["fluid_nodes"] = fluid
    out["batched"] = dict(launch=dict(bands=tuned[0] or 8, block=tuned[1], grid=tuned[2]), ms_per_step=ms / args.steps,
                          mlups=nodes / (ms / args.steps * 1e-3) / 1e6,
                          mflups=fluid / (ms / args.steps * 1e-3) / 1e6)
    b.close()
    print(f"[batch] batched: {ms / args.steps:.3f} ms/step", flush=True)

    seq_ms = 0.0
    for p, mask, rho, C in cases:
        lat = mclbm.Lattice(p)
        lat.set_graph(True)
        lat.set_geometry(mask)
        lat.init_fields(rho, None, C)
        lat.step(min(args.steps, 200))
        seq_ms += _timed_steps(lat, args.steps)
        lat.close()
    out["sequential"] = dict(ms_per_step=seq_ms / args.steps, mlups=nodes / (seq_ms / args.steps * 1e-3) / 1e6,
                             mflups=fluid / (seq_ms / args.steps * 1e-3) / 1e6)
    print(f"[batch] sequential: {seq_ms / args.steps:.3f} ms/step", flush=True)

    b = mclbm.Batch([c[0] for c in cases])
    b.set_bands(tuned[0])
    b.set_geometry([c[1] for c in cases])
    b.set_launch(tuned[1], tuned[2])
    b.set_graph(True)
    b.init_fields([c[2] for c in cases], None, [c[3] for c in cases])
    b.synchronize()
    t0 = time.perf_counter()
    ok, steps = b.run_to_residual(args.tol, args.cap, allow_diverged=True)
    b.synchronize()
    wall = time.perf_counter() - t0
    mons = [b.sample_monitors(s) for s in range(args.count)]
    b.close()
    conv = [int(m[11]) for m in mons]
    div = [int(m[13]) for m in mons]
    done = [c for c in conv if c > 0]
    out["to_residual"] = dict(tol=args.tol, cap=args.cap, all_converged=bool(ok), steps=int(steps), wall_s=wall,
                              converged=len(done), conv_steps=conv,
                              diverged={s: d for s, d in enumerate(div) if d >= 0},
                              median_conv_step=float(np.median(done)) if done else None,
                              final_residual=[float(m[9]) for m in mons])
    # the same samples one after another, each to the same tolerance
    seq_wall = 0.0
    for p, mask, rho, C in cases:
        lat = mclbm.Lattice(p)
        lat.set_graph(True)
        lat.set_geometry(mask)
        lat.init_fields(rho, None, C)
        lat.synchronize()
        t1 = time.perf_counter()
        lat.run_to_residual(args.tol, args.cap, allow_diverged=True)
        lat.synchronize()
        seq_wall += time.perf_counter() - t1
        lat.close()
    out["to_residual"]["sequential_wall_s"] = seq_wall
    print(f"[batch] to residual: {len(done)}/{args.count} converged, {len(out['to_residual']['diverged'])} "
          f"diverged, {steps} steps, {wall:.1f} s batched, {seq_wall:.1f} s one after another", flush=True)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="what", required=True)
    a = sub.add_parser("precision")
    a.add_argument("--n", type=int, default=384)
    a.add_argument("--steps", type=int, default=20000)
    a.add_argument("--storages", nargs="+", default=["f32", "f16s", "bf16s"])
    a.add_argument("--res-n", type=int, default=128)
    a.add_argument("--tol", type=float, default=1e-6)
    a.add_argument("--cap", type=int, default=30000)
    a.add_argument("--out", default=None)
    t = sub.add_parser("thermal")
    t.add_argument("--n", type=int, default=256)
    t.add_argument("--steps", type=int, default=500)
    t.add_argument("--storage", default="f32")
    t.add_argument("--out", default=None)
    v = sub.add_parser("variants")
    v.add_argument("--n", type=int, default=256)
    v.add_argument("--steps", type=int, default=500)
    v.add_argument("--storage", default="f32")
    v.add_argument("--out", default=None)
    b = sub.add_parser("batch")
    b.add_argument("--count", type=int, default=64)
    b.add_argument("--steps", type=int, default=500)
    b.add_argument("--storage", default="f32")
    b.add_argument("--tol", type=float, default=1e-3)
    b.add_argument("--cap", type=int, default=40000)
    b.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    rep = {"precision": precision, "batch": batch, "thermal": thermal, "variants": variants}[args.what](args)
    line = json.dumps(rep)
    print(line)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
