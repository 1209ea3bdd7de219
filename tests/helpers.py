"""Shared test helpers: run the same seeded case through the HIP library and the oracle."""
import numpy as np

import oracle
from paper_2502_12955_amd import inputs


def nrel(a, b):
    """Normwise relative difference ||a - b||_2 / ||b||_2 (0 if both vanish)."""
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    den = np.linalg.norm(b)
    num = np.linalg.norm(a - b)
    return num / den if den else num


def maxrel(a, b):
    """Element-wise difference relative to the field's scale: max|a - b| / max|b|
    (max|a - b| if b vanishes).  One wrong value anywhere in the field shows up at
    its own size, unlike a norm over the whole field."""
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    num = float(np.max(np.abs(a - b), initial=0.0))
    den = float(np.max(np.abs(b), initial=0.0))
    return num / den if den else num


def gpu_lattice(p, mask, rho, u=None, C=None, block=None):
    from paper_2502_12955_amd import mclbm

    lat = mclbm.Lattice(p)
    if block is not None:
        lat.set_launch(block)
    lat.set_geometry(mask)
    lat.init_fields(rho, u, C)
    return lat


def oracle_state(p, mask, rho, u=None, C=None):
    m, n = oracle.pinch_fill(p, mask)
    f, h = oracle.init(p, m, rho, u, C)
    return m, f, h


def split_pops(p, pops):
    """Split get_populations output into (f [ncomp*Q, N], h [QS, N])."""
    N = p["nx"] * p["ny"] * p.get("nz", 1)
    Q = 19 if p["lattice"] == "D3Q19" else 9
    QS = 7 if p["lattice"] == "D3Q19" else 5
    nc = p.get("ncomp", 2)
    f = pops[: nc * Q * N].reshape(nc * Q, N)
    h = pops[nc * Q * N:].reshape(-1, N) if p.get("solute", "off") != "off" else np.zeros((QS, N))
    return f, h


def small_porous(shape=(14, 18, 22), seed_sample=3, porosity=0.55, radius=3, **kw):
    p, mask, rho, u, C = inputs.porous_case(shape=shape, porosity=porosity, radius=radius,
                                           blob_radius=2, sample=seed_sample)
    p.update(kw)
    rng = inputs.SplitMix64(inputs.seed_for(9, seed_sample))
    C = 0.5 * rng.uniform(int(np.prod(shape))).reshape(shape)
    return p, mask, rho, u, C
