"""Particle deposition study (sec:particle_deposition) on the HIP path.

The paper's set-up: D2Q9 lattices for the flow and for the particle mass
fraction on a 419 x 415 porous image, particle diffusivity 0.156 (relaxation
time 0.9687), deposition probability 0.002, inlet mass fraction 0.01 and a peak
inlet velocity of 5.65e-5.  The image itself is not available, so a seeded
Boolean disc pack of the same size stands in for it.  The flow is driven by a
body force along x (periodic), the particles enter through the plane x = 0 and
leave through x = nx-1, and the particle lattice is D2Q5 with rest weight 1/3
(c_s^2 = 1/3, so the paper's diffusivity gives its relaxation time).

Reported: the nodes turned solid over time and where they are along x (the
paper finds deposits near the inlet first, then further downstream), the mean
velocity (it drops as the pores clog), the outlet concentration, and the time
per step with deposition against the same lattice without it.

    python -m paper_2502_12955_amd.deposition [--steps N] [--out report.json]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import inputs, mclbm


def paper_case(nx=419, ny=415, porosity=0.6, radius=9, seed_sample=0, dep_prob=0.002, C_in=0.01,
               accel=3e-7, storage="f64", deposition=1):
    """Single-component flow + particle field on a seeded disc pack (the image's stand-in)."""
    shape = (1, ny, nx)
    mask, _, _ = inputs.sphere_pack(shape, porosity, radius, inputs.seed_for(8, seed_sample))
    p = inputs.base_params(lattice="D2Q9", nx=nx, ny=ny, nz=1, ncomp=1, tau=(1.0, 1.0),
                           G=((0.0, 0.0), (0.0, 0.0)), accel=(accel, 0.0, 0.0), forcing="guo",
                           solute="inlet_outlet_x", D=0.156, J0=1.0 / 3.0, k_wall=0.0, C_in=C_in,
                           storage=storage, monitor_every=1000, deposition=deposition, dep_prob=dep_prob)
    rho = np.where(mask == 0, 1.0, 0.0)[None]
    return p, mask, rho


def run(steps=100_000, every=10_000, dep_prob=0.002, C_in=0.01, storage="f64", nx=419, ny=415):
    out = dict(nx=nx, ny=ny, steps=steps, dep_prob=dep_prob, C_in=C_in, storage=storage, history=[])
    timings = {}
    for dep in (0, 1):
        p, mask, rho = paper_case(nx=nx, ny=ny, dep_prob=dep_prob, C_in=C_in, storage=storage, deposition=dep)
        lat = mclbm.Lattice(p)
        nrc = lat.set_geometry(mask)
        lat.init_fields(rho)
        solid0 = lat.get_geometry()[0].reshape(ny, nx) != 0
        N = nx * ny
        done = 0
        t_total = 0.0
        while done < steps:
            n = min(every, steps - done)
            t0 = time.perf_counter()
            lat.step(n)
            lat.synchronize()
            dt = time.perf_counter() - t0
            t_total += dt
            done += n
            if dep:
                r, u, C = lat.moments()
                mg, _, _ = lat.get_geometry()
                _, conv = lat.get_deposit()
                fluid = mg.reshape(ny, nx) == 0
                ux = u[0].reshape(ny, nx)
                Cout = C.reshape(ny, nx)[:, nx - 1][fluid[:, nx - 1]]
                # where the deposits are: x of the nodes that turned solid
                xs = np.nonzero(~fluid & ~solid0)[1]
                rec = dict(step=done, converted=int(conv), fluid_nodes=int(fluid.sum()), ms_per_step=1e3 * dt / n,
                           mean_ux=float(ux[fluid].mean()), max_ux=float(ux[fluid].max()),
                           outlet_C=float(Cout.mean()) if Cout.size else 0.0,
                           x_median=float(np.median(xs)) if xs.size else None,
                           x_p90=float(np.percentile(xs, 90)) if xs.size else None)
                out["history"].append(rec)
                print(f"[deposition] step {done}: {conv} nodes turned solid, mean u_x {rec['mean_ux']:.3e}, "
                      f"outlet C {rec['outlet_C']:.3e}, deposits at x median {rec['x_median']} / 90 % "
                      f"{rec['x_p90']}, {rec['ms_per_step']:.4f} ms/step", flush=True)
        timings["with" if dep else "without"] = dict(ms_per_step=1e3 * t_total / steps,
                                                      mlups=N * steps / t_total / 1e6)
        if not dep:
            out["initial_fluid_nodes"] = int((lat.get_geometry()[0] == 0).sum())
            out["reclassified"] = int(nrc)
        lat.close()
    out["timing"] = timings
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--steps", type=int, default=100_000)
    ap.add_argument("--every", type=int, default=10_000)
    ap.add_argument("--dep-prob", type=float, default=0.002)
    ap.add_argument("--c-in", type=float, default=0.01)
    ap.add_argument("--storage", default="f64")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    rep = run(args.steps, args.every, args.dep_prob, args.c_in, args.storage)
    line = json.dumps(rep)
    print(line)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
