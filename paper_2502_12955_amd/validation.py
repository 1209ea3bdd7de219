"""Multiphase validation cases of the paper, run on the HIP path.

* Phase separation (validation section, single component): eq:1.12 with a
  diagonal cohesion G = -5, psi = rho0 (1 - exp(-rho / rho0)) (eq:1.11), a
  box of uniform density with seeded random perturbations.  The liquid and
  vapour densities it settles to are compared with the flat-interface
  coexistence of the model (equal pressure and the Shan-Chen mechanical
  stability condition).
* Contact angle (contact-angle subsection): a two-component droplet on a
  flat wall with adhesion eq:1.15; the angle is measured with the paper's
  construction from the cap height h and contact length b and compared with
  the relation of Huang et al. between adhesion and cohesion.

    python -m paper_2502_12955_amd.validation [--out report.json]
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import inputs, mclbm


# ----------------------------------------------------------------------------- theory
def sc_coexistence(G, rho0=1.0):
    """Bulk (vapour, liquid) densities of a flat interface of the single-component
    model: p(rho) = rho / 3 + G psi(rho)^2 / 6 equal in both phases and
    integral_{rho_v}^{rho_l} (p0 - p) psi' / psi^2 d rho = 0."""
    from scipy.integrate import quad
    from scipy.optimize import fsolve

    psi = lambda r: rho0 * (1.0 - np.exp(-r / rho0))
    dpsi = lambda r: np.exp(-r / rho0)
    p = lambda r: r / 3.0 + G / 6.0 * psi(r) ** 2

    def eqs(v):
        rv, rl = v
        p0 = p(rl)
        return [p(rv) - p0, quad(lambda r: (p0 - p(r)) * dpsi(r) / psi(r) ** 2, rv, rl)[0]]

    rv, rl = fsolve(eqs, [0.15 * rho0, 1.9 * rho0])
    return float(rv), float(rl)


def cap_angle(h, b):
    """Contact angle of a circular cap of height h over a contact length b (the
    paper's construction: r = (4 h^2 + b^2) / (8 h); the angle between the wall
    and the cap at the contact line, inside the droplet, is atan2(b / 2, r - h),
    which is the paper's pi - arctan(b / (2 (h - r))) on the right branch)."""
    r = (4.0 * h * h + b * b) / (8.0 * h)
    return r, math.atan2(0.5 * b, r - h)


def huang_angle(g_ads, G_c, rho_main, rho_dissolved):
    """cos(theta) = (G_ads,2 - G_ads,1) / (G_c (rho_1 - rho_2) / 2), clipped to [-1, 1]."""
    c = (g_ads[1] - g_ads[0]) / (G_c * (rho_main - rho_dissolved) / 2.0)
    return math.acos(max(-1.0, min(1.0, c)))


def _crossings(v, level=0.0):
    """Positions (fractional indices) where the sampled profile v crosses ``level``."""
    s = v - level
    out = []
    for i in range(len(s) - 1):
        if s[i] == 0.0:
            out.append(float(i))
        elif s[i] * s[i + 1] < 0:
            out.append(i + s[i] / (s[i] - s[i + 1]))
    return out


def measure_cap(phi, wall_y=0.5):
    """(h, b) of the droplet (phi > 0) standing on the wall below row 1 of a
    [ny, nx] phase field (row 0 solid, halfway bounce-back puts the wall at
    y = 0.5): b from the phi = 0 crossings along the first fluid row, h from the
    crossing along the column through the droplet's centre."""
    row = phi[1]
    xs = _crossings(row)
    if len(xs) != 2:
        raise ValueError(f"expected two contact points, found {len(xs)}")
    b = xs[1] - xs[0]
    xc = 0.5 * (xs[0] + xs[1])
    col = np.array([np.interp(xc, np.arange(phi.shape[1]), phi[y]) for y in range(phi.shape[0])])
    ys = _crossings(col[1:])
    if not ys:
        raise ValueError("no top of the droplet")
    top = 1.0 + ys[0]
    return top - wall_y, b


# ----------------------------------------------------------------------------- runs
def phase_separation(n=128, G=-5.0, rho_mean=0.7, amp=0.1, steps=40000, seed=7, forcing="sc", storage="f64",
                     lattice="D2Q9"):
    """Uniform density rho_mean with seeded relative perturbations U(-amp, amp)."""
    nz = 1 if lattice == "D2Q9" else n
    p = inputs.base_params(lattice=lattice, nx=n, ny=n, nz=nz, ncomp=1, tau=(1.0, 1.0),
                           G=((G, 0.0), (0.0, 0.0)), forcing=forcing, solute="off", storage=storage,
                           monitor_every=1000)
    u01 = inputs.SplitMix64(inputs.seed_for(6, seed)).uniform(n * n * nz)
    rho = rho_mean * (1.0 + amp * (2.0 * u01 - 1.0))
    lat = mclbm.Lattice(p)
    lat.set_geometry(np.zeros(n * n * nz, np.uint8))
    lat.init_fields(rho.reshape(1, -1))
    t0 = time.perf_counter()
    lat.step(steps)
    r, u, _ = lat.moments()
    wall = time.perf_counter() - t0
    lat.close()
    r = np.asarray(r)[0]
    # bulk phases: the medians of the nodes clearly inside each phase
    liq = float(np.median(r[r > 0.5 * (r.max() + rho_mean)]))
    vap = float(np.median(r[r < 0.5 * (r.min() + rho_mean)]))
    return dict(n=n, lattice=lattice, G=G, steps=steps, forcing=forcing, liquid=liq, vapour=vap,
                mass_rel_change=float(r.sum() / rho.sum() - 1.0), max_u=float(np.abs(u).max()),
                mlups=n * n * nz * steps / wall / 1e6)


def two_component_bulk(G_c=5.0, nx=64, steps=20000):
    """Bulk (main, dissolved) densities of a component across a flat interface of
    the symmetric two-component model (a periodic D2Q9 slab on the HIP path)."""
    p = inputs.base_params(lattice="D2Q9", nx=nx, ny=1, nz=1, ncomp=2, tau=(1.0, 1.0),
                           G=((0.0, G_c), (G_c, 0.0)), forcing="guo", solute="off", storage="f64",
                           monitor_every=1000)
    x = np.arange(nx)
    inside = (x >= nx // 4) & (x < 3 * nx // 4)
    rho = np.stack([np.where(inside, 1.0, 0.03), np.where(inside, 0.03, 1.0)])
    lat = mclbm.Lattice(p)
    lat.set_geometry(np.zeros(nx, np.uint8))
    lat.init_fields(rho)
    lat.step(steps)
    r, _, _ = lat.moments()
    lat.close()
    r = np.asarray(r)
    return float(r[0][nx // 2]), float(r[0][0])


def contact_angle(g, nx=200, ny=80, radius=25.0, steps=30000, G_c=5.0, storage="f64", bulk=None):
    """Droplet of component 0 on the wall below row 1, both components started at
    their flat-interface bulk densities (so the droplet does not dissolve into the
    other phase); adhesion G_ads = (g, -g).  Returns the measured and the predicted
    angle (degrees) and the bulk densities used in the prediction."""
    main, dissolved = bulk if bulk is not None else two_component_bulk(G_c)
    p = inputs.base_params(lattice="D2Q9", nx=nx, ny=ny, nz=1, ncomp=2, tau=(1.0, 1.0),
                           G=((0.0, G_c), (G_c, 0.0)), G_ads=(g, -g), forcing="guo", solute="off",
                           storage=storage, monitor_every=1000)
    mask = np.zeros((1, ny, nx), np.uint8)
    mask[0, 0, :] = 1
    mask[0, ny - 1, :] = 1
    rho = inputs.droplet((1, ny, nx), radius, rho_in=(main, dissolved), rho_out=(dissolved, main),
                         centre=((nx - 1) / 2.0, 0.5, 0.0))
    rho[:, mask.astype(bool)] = 0.0
    lat = mclbm.Lattice(p)
    lat.set_geometry(mask)
    lat.init_fields(rho.reshape(2, -1))
    lat.step(steps)
    r, _, _ = lat.moments()
    lat.close()
    r = np.asarray(r).reshape(2, ny, nx)
    tot = r[0] + r[1]
    phi = np.where(tot > 0, (r[0] - r[1]) / np.where(tot > 0, tot, 1.0), 0.0)
    h, b = measure_cap(phi)
    _, theta = cap_angle(h, b)
    pred = huang_angle((g, -g), G_c, main, dissolved)
    return dict(g_ads=g, h=h, b=b, theta_deg=math.degrees(theta), huang_deg=math.degrees(pred),
                rho_main=main, rho_dissolved=dissolved, steps=steps)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", default=None)
    ap.add_argument("--steps", type=int, default=30000)
    args = ap.parse_args(argv)
    rv, rl = sc_coexistence(-5.0)
    rep = dict(coexistence_theory=dict(vapour=rv, liquid=rl))
    rep["phase_separation"] = [phase_separation(128, steps=40000, forcing=f) for f in ("sc", "guo")]
    rep["phase_separation_3d"] = phase_separation(128, steps=2000, lattice="D3Q19", storage="f32")
    for r in rep["phase_separation"]:
        print(f"[validation] phase separation {r['forcing']}: liquid {r['liquid']:.4f} vapour {r['vapour']:.4f} "
              f"(flat interface {rl:.4f} / {rv:.4f})", flush=True)
    rep["contact_angle"] = []
    bulk = two_component_bulk(5.0)
    rep["two_component_bulk"] = dict(main=bulk[0], dissolved=bulk[1])
    for g in (-0.15, -0.1, -0.05, 0.0, 0.05, 0.1, 0.15):
        c = contact_angle(g, steps=args.steps, bulk=bulk)
        rep["contact_angle"].append(c)
        print(f"[validation] contact angle G_ads = ({g}, {-g}): {c['theta_deg']:.1f} deg, "
              f"relation of Huang et al. {c['huang_deg']:.1f} deg", flush=True)
    line = json.dumps(rep)
    print(line)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
