"""Second, independent statement of one time step in vectorised numpy (np.roll).

TEST INFRASTRUCTURE ONLY.  It exists to cross-check the C oracle on tiny
lattices: it is written separately (array shifts instead of per-node loops)
from the same equations, with its own lattice tables, so that an indexing or
sign slip in either one shows up as a disagreement.  Arrays are indexed
[..., z, y, x].
"""
from __future__ import annotations

import numpy as np

# Paper tables ("3D and 2D LBM Models"), D2Q9 with w_4 = 1/9.
_D3Q19 = np.array([
    (0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
    (1, 1, 0), (-1, -1, 0), (1, 0, 1), (-1, 0, -1), (0, 1, 1), (0, -1, -1),
    (1, -1, 0), (-1, 1, 0), (1, 0, -1), (-1, 0, 1), (0, 1, -1), (0, -1, 1)])
_W19 = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
_D2Q9 = np.array([(0, 0, 0), (1, 0, 0), (0, 1, 0), (-1, 0, 0), (0, -1, 0),
                  (1, 1, 0), (-1, 1, 0), (-1, -1, 0), (1, -1, 0)])
_W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def _tables(p):
    if p["lattice"] in ("D3Q19", 1):
        c, w, cs = _D3Q19, _W19, _D3Q19[:7]
    else:
        c, w, cs = _D2Q9, _W9, _D2Q9[:5]
    J0 = p.get("J0", 0.1)
    ws = np.array([J0] + [(1 - J0) / (len(cs) - 1)] * (len(cs) - 1))
    opp = np.array([int(np.flatnonzero((c == -ci).all(1))[0]) for ci in c])
    opps = np.array([int(np.flatnonzero((cs == -ci).all(1))[0]) for ci in cs])
    return c, w, opp, cs, ws, opps


def _shift(a, d):
    """a(x - d) as an array over x (periodic): roll by +d along each axis."""
    return np.roll(a, shift=(int(d[2]), int(d[1]), int(d[0])), axis=(-3, -2, -1))


def _ahead(a, d):
    """a(x + d) (periodic)."""
    return _shift(a, -np.asarray(d))


def step(p, mask, f, h):
    """One step.  f: [ncomp, Q, nz, ny, nx], h: [QS, nz, ny, nx], mask [nz, ny, nx]."""
    c, w, opp, cs, ws, opps = _tables(p)
    nc = int(p.get("ncomp", 2))
    cs2 = 1.0 / 3.0
    solid = mask.astype(bool)
    fluid = ~solid
    tau = np.asarray(p["tau"], float)
    G = np.asarray(p["G"], float)
    Gads = np.asarray(p["G_ads"], float)
    acc = np.asarray(p["accel"], float)
    rho0 = p.get("rho0", 1.0)

    rho = np.where(fluid, f.sum(axis=1), 0.0)                      # [nc, z, y, x]
    psi = np.where(fluid, rho0 * (1.0 - np.exp(-rho / rho0)), 0.0)
    j = np.einsum("sqzyx,qa->sazyx", f, c.astype(float))          # [nc, 3, ...]

    # Forces: cohesion (eq:1.14), adhesion (eq:1.15), body.
    F = np.zeros((nc, 3) + mask.shape)
    for s in range(nc):
        coh = np.zeros((3,) + mask.shape)
        ads = np.zeros((3,) + mask.shape)
        for i in range(1, len(c)):
            nb_psi = sum(G[s, t] * _ahead(psi[t], c[i]) for t in range(nc))
            nb_sol = _ahead(solid.astype(float), c[i])
            for a in range(3):
                coh[a] += w[i] * nb_psi * c[i, a]
                ads[a] += w[i] * nb_sol * c[i, a]
        for a in range(3):
            F[s, a] = -psi[s] * coh[a] - Gads[s] * rho[s] * ads[a] + rho[s] * acc[a]
    F *= fluid

    rt = rho.sum(axis=0)
    rt_safe = np.where(fluid, rt, 1.0)
    u = (j.sum(axis=0) + 0.5 * F.sum(axis=0)) / rt_safe
    if p.get("forcing", "guo") in ("guo", 0):
        ueq = np.broadcast_to(u, (nc,) + u.shape)
    else:
        den = sum(rho[s] / tau[s] for s in range(nc))
        den = np.where(fluid, den, 1.0)
        up = sum(j[s] / tau[s] for s in range(nc)) / den
        ueq = np.stack([up + tau[s] * F[s] / np.where(fluid, rho[s], 1.0) for s in range(nc)])

    fstar = np.empty_like(f)
    for s in range(nc):
        v = ueq[s]
        vv = (v * v).sum(axis=0)
        uF = (u * F[s]).sum(axis=0)
        for i in range(len(c)):
            cv = sum(c[i, a] * v[a] for a in range(3))
            feq = w[i] * rho[s] * (1 + cv / cs2 + (cv * cv - cs2 * vv) / (2 * cs2 * cs2))
            if p.get("forcing", "guo") in ("guo", 0):
                cF = sum(c[i, a] * F[s, a] for a in range(3))
                cu = sum(c[i, a] * u[a] for a in range(3))
                S = w[i] * (cF / cs2 + (cF * cu - cs2 * uF) / (cs2 * cs2))
            else:
                S = 0.0
            fstar[s, i] = f[s, i] - (f[s, i] - feq) / tau[s] + (1 - 0.5 / tau[s]) * S

    new_f = np.empty_like(f)
    for s in range(nc):
        for i in range(len(c)):
            up_solid = _shift(solid, c[i])
            new_f[s, i] = np.where(up_solid, fstar[s, opp[i]], _shift(fstar[s, i], c[i]))
    new_f *= fluid

    new_h = h
    sol = p.get("solute", "off")
    if sol not in ("off", 0):
        csd = float(sum(ws[k] * cs[k, 0] ** 2 for k in range(len(cs))))
        tau_d = p["D"] / csd + 0.5
        C = h.sum(axis=0)
        hstar = np.empty_like(h)
        for k in range(len(cs)):
            eu = sum(cs[k, a] * u[a] for a in range(3))
            heq = ws[k] * C * (1 + eu / csd)
            hstar[k] = h[k] - (h[k] - heq) / tau_d
        new_h = np.empty_like(h)
        nx = mask.shape[-1]
        xs = np.arange(nx)[None, None, :]
        seam = sol in ("inlet_outlet_x", 2)
        kw = p["k_wall"]
        for k in range(len(cs)):
            kb = opps[k]
            plain = _shift(hstar[k], cs[k])
            hin = _ahead(hstar[kb], cs[k])
            up_solid = _shift(solid, cs[k])
            if seam and cs[k, 0] != 0:
                # upstream across the seam is not a node: not a wet link
                crosses = (xs == 0) if cs[k, 0] == 1 else (xs == nx - 1)
                up_solid = up_solid & ~crosses
            Cb = 2 * hin / (2 * ws[k] + kw * tau_d / (tau_d - 0.5))
            val = np.where(up_solid, 2 * ws[k] * Cb - hin, plain)
            if seam and cs[k, 0] == 1:
                val = np.where(xs == 0, 2 * ws[k] * p["C_in"] - hin, val)
            if seam and cs[k, 0] == -1:
                val = np.where(xs == nx - 1, hstar[k], val)
            new_h[k] = val
        new_h *= fluid
    return new_f, new_h
