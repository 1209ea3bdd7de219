"""Seeded synthetic inputs: geometries, initial fields and the workload parameter sets.

This module is the only code shared by the HIP path and the CPU oracle's
tests.  It holds no arithmetic of the method itself: it draws random
numbers, voxelises spheres and fills initial density fields.  Geometry
post-processing (pinch-fill, link masks) belongs to each side separately.

PRNG: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), seed = (12955 << 32) | (config << 24) | sample, where
config numbers the workload: 1 the 2-D droplet, 2 the 256^3 porous flow with
solute, 3 its 384^3 reduced-precision study, 4 the batch of uneven samples, 5
the warm-start samples.
"""
from __future__ import annotations

import numpy as np

_M64 = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


def seed_for(config: int, sample: int = 0) -> int:
    return ((12955 << 32) | (int(config) << 24) | int(sample)) & _M64


class SplitMix64:
    """SplitMix64 stream; ``next(n)`` returns n uint64 values as a numpy array."""

    def __init__(self, seed: int):
        self.state = int(seed) & _M64

    def next(self, n: int) -> np.ndarray:
        with np.errstate(over="ignore"):
            k = np.arange(1, n + 1, dtype=np.uint64)
            z = np.uint64(self.state) + k * np.uint64(_GAMMA)
            z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
            z = z ^ (z >> np.uint64(31))
        self.state = (self.state + n * _GAMMA) & _M64
        return z

    def uniform(self, n: int) -> np.ndarray:
        """Doubles in [0, 1) from the top 53 bits."""
        return (self.next(n) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))

    def integers(self, n: int, high: int) -> np.ndarray:
        return (self.next(n) % np.uint64(high)).astype(np.int64)


def _ball_offsets(radius: int, dims: int):
    r = int(radius)
    rng = np.arange(-r, r + 1)
    if dims == 3:
        dz, dy, dx = np.meshgrid(rng, rng, rng, indexing="ij")
        keep = dx * dx + dy * dy + dz * dz <= r * r
        return dx[keep], dy[keep], dz[keep]
    dy, dx = np.meshgrid(rng, rng, indexing="ij")
    keep = dx * dx + dy * dy <= r * r
    return dx[keep], dy[keep], np.zeros(int(keep.sum()), np.int64)


def sphere_pack(shape, porosity: float, radius: int, seed: int, max_spheres: int = 10_000_000):
    """Boolean (overlapping) sphere pack with distinct integer centres.

    shape = (nz, ny, nx).  A voxel is solid iff its minimum-image periodic
    squared distance to some centre is <= radius^2 (exact integers).  Spheres
    are added in PRNG order until the voxel porosity is <= ``porosity``.
    Returns (mask uint8 [nz, ny, nx] with 1 = solid, achieved porosity, count).
    """
    nz, ny, nx = (int(s) for s in shape)
    dims = 3 if nz > 1 else 2
    dx, dy, dz = _ball_offsets(radius, dims)
    N = nx * ny * nz
    mask = np.zeros(N, np.uint8)
    target_solid = int(np.ceil((1.0 - porosity) * N - 1e-9))
    rng = SplitMix64(seed)
    seen = set()
    solid = 0
    count = 0
    while solid < target_solid and count < max_spheres:
        batch = rng.integers(3 * 256, 1 << 62)
        cx = batch[0::3] % nx
        cy = batch[1::3] % ny
        cz = batch[2::3] % nz if dims == 3 else np.zeros_like(cx)
        for x0, y0, z0 in zip(cx.tolist(), cy.tolist(), cz.tolist()):
            key = (x0, y0, z0)
            if key in seen:
                continue
            seen.add(key)
            idx = ((x0 + dx) % nx) + nx * (((y0 + dy) % ny) + ny * ((z0 + dz) % nz))
            new = int(np.count_nonzero(mask[idx] == 0))
            mask[idx] = 1
            solid += new
            count += 1
            if solid >= target_solid:
                break
    return mask.reshape(nz, ny, nx), 1.0 - solid / N, count


def droplet(shape, radius: float, rho_in=(1.0, 0.03), rho_out=(0.03, 1.0), centre=None):
    """Two-component static droplet: inside iff squared distance < radius^2.

    Returns rho [2, nz, ny, nx]; default centre is the box centre ((n-1)/2).
    """
    nz, ny, nx = (int(s) for s in shape)
    if centre is None:
        centre = ((nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2
    inside = d2 < radius * radius
    rho = np.empty((2, nz, ny, nx))
    rho[0] = np.where(inside, rho_in[0], rho_out[0])
    rho[1] = np.where(inside, rho_in[1], rho_out[1])
    return rho


def blob_phase(mask, saturation: float, radius: int, seed: int,
               rho_blob=(0.03, 1.0), rho_rest=(1.0, 0.03)):
    """Non-wetting blobs: spheres of ``radius`` around seeded fluid voxels until the
    blob fraction of fluid voxels reaches ``saturation``.  Component 1 is the blob
    fluid.  Returns rho [2, *mask.shape] (0 on solid voxels) and the achieved fraction.
    """
    shape = mask.shape
    nz, ny, nx = shape if len(shape) == 3 else (1,) + tuple(shape)
    flat = mask.reshape(-1)
    fluid_idx = np.flatnonzero(flat == 0)
    nfluid = fluid_idx.size
    dims = 3 if nz > 1 else 2
    dx, dy, dz = _ball_offsets(radius, dims)
    blob = np.zeros(flat.size, bool)
    rng = SplitMix64(seed)
    nblob = 0
    guard = 0
    while nfluid and nblob < saturation * nfluid and guard < 10_000_000:
        picks = fluid_idx[rng.integers(64, nfluid)]
        for c in picks.tolist():
            guard += 1
            x0, y0, z0 = c % nx, (c // nx) % ny, c // (nx * ny)
            idx = ((x0 + dx) % nx) + nx * (((y0 + dy) % ny) + ny * ((z0 + dz) % nz))
            idx = idx[flat[idx] == 0]
            nblob += int(np.count_nonzero(~blob[idx]))
            blob[idx] = True
            if nblob >= saturation * nfluid:
                break
    rho = np.zeros((2, flat.size))
    fl = flat == 0
    rho[0] = np.where(blob, rho_blob[0], rho_rest[0]) * fl
    rho[1] = np.where(blob, rho_blob[1], rho_rest[1]) * fl
    return rho.reshape((2,) + tuple(shape)), (nblob / nfluid if nfluid else 0.0)


def random_state_fields(shape, ncomp, seed, rho_lo=0.2, rho_hi=1.2, u_amp=0.02, c_hi=1.0):
    """Smooth-free random densities, velocities and concentration for parity cases."""
    rng = SplitMix64(seed)
    n = int(np.prod(shape))
    rho = rho_lo + (rho_hi - rho_lo) * rng.uniform(ncomp * n).reshape((ncomp,) + tuple(shape))
    u = u_amp * (2.0 * rng.uniform(3 * n) - 1.0).reshape((3,) + tuple(shape))
    C = c_hi * rng.uniform(n).reshape(tuple(shape))
    return rho, u, C


# ----------------------------------------------------------------------------- workloads
def base_params(**kw):
    """Parameter dict understood by both the HIP binding and the oracle."""
    p = dict(lattice="D3Q19", nx=8, ny=8, nz=8, ncomp=2, tau=(1.0, 1.0),
             G=((0.0, 5.0), (5.0, 0.0)), G_ads=(0.0, 0.0), rho0=1.0,
             accel=(0.0, 0.0, 0.0), forcing="guo", solute="off",
             D=0.1, J0=0.1, k_wall=0.0, C_in=0.0, storage="f64", monitor_every=100)
    p.update(kw)
    return p


def droplet_2d_params(nx=128, ny=64, storage="f64", forcing="guo"):
    """Static droplet: D2Q9 two-component, periodic box, BGK tau = 1 both, G_c = 5."""
    return base_params(lattice="D2Q9", nx=nx, ny=ny, nz=1, forcing=forcing, storage=storage,
                       J0=0.4)


def droplet_2d_case(nx=128, ny=64, radius=20.0, storage="f64", forcing="guo"):
    p = droplet_2d_params(nx, ny, storage, forcing)
    mask = np.zeros((1, ny, nx), np.uint8)
    rho = droplet((1, ny, nx), radius)
    return p, mask, rho, None, None


def porous_params(n=256, storage="f32", nx=None, ny=None, nz=None):
    """Two-component D3Q19 + D3Q7 solute in a sphere pack, drive along x, wall reaction.

    G_c = 4.2 and G_ads = -+0.1: with G_c = 5 and G_ads = -+0.5 some packs develop
    runaway interface currents within 10,000-20,000 steps.  G_c = 4.2 is above the
    demixing point of a symmetric mixture under the pseudo-potential of eq:1.11
    (G psi psi' = 1, G = 4.16 at 0.515 per component), but the 15 % blob fluid of
    porous_case lies outside the two-phase region there: the blobs dissolve into the
    carrier as the run proceeds."""
    return base_params(lattice="D3Q19", nx=nx or n, ny=ny or n, nz=nz or n, ncomp=2,
                       tau=(1.0, 1.0), G=((0.0, 4.2), (4.2, 0.0)), G_ads=(-0.1, 0.1),
                       accel=(1e-5, 0.0, 0.0), forcing="guo", solute="inlet_outlet_x",
                       D=0.1, J0=0.1, k_wall=1e-3, C_in=1.0, storage=storage)


def porous_case(n=256, porosity=0.4, radius=8, config=2, sample=0, storage="f32",
                blob_radius=6, saturation=0.15, shape=None):
    """Sphere pack + non-wetting blobs; returns (params, raw mask, rho, u, C)."""
    if shape is None:
        shape = (n, n, n)
    nz, ny, nx = shape
    p = porous_params(storage=storage, nx=nx, ny=ny, nz=nz)
    mask, _, _ = sphere_pack(shape, porosity, radius, seed_for(config, sample))
    rho, _ = blob_phase(mask, saturation, blob_radius, seed_for(config, sample) ^ 0x5A5A)
    C = np.zeros(shape)
    return p, mask, rho, None, C


def batch_edges(count=64, seed=None, choices=(32, 48, 64, 96, 128)):
    """Independent per-axis edge lengths for a batch of samples."""
    rng = SplitMix64(seed_for(4, 0) if seed is None else seed)
    picks = rng.integers(3 * count, len(choices)).reshape(count, 3)
    return [tuple(int(choices[j]) for j in row) for row in picks]


def arrhenius_rate_field(T, A, E_over_R):
    """Per-node first-order wall reaction rate k = A exp(-E / (R_u T)) (the rate law of
    the O2 reaction, eq:reactO2) of a prescribed temperature field T [K]; E_over_R =
    E / R_u in K.  An input generator for the rate-field runs: both sides take the
    resulting k values as given."""
    return A * np.exp(-E_over_R / np.asarray(T, np.float64))
