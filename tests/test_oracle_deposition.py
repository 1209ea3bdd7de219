"""Oracle pins for particle deposition (sec:particle_deposition, eq:surface_deposition).

A fluid at rest with a uniform particle mass fraction c0 and a non-reacting wall
(k = 0) stays exactly uniform: halfway bounce-back returns every population
unchanged, and the wet-node rule with k = 0 reflects h_in as it came.  The
deposit of a node next to the substrate then grows by DP c0 per step, so it
first exceeds 1 after t* = floor(1 / (DP c0)) + 1 steps; the next layer only
starts to collect once the first has turned solid, so the deposit front moves
one node per t* steps.  These closed forms pin the update, the threshold, the
neighbourhood and the layer-by-layer growth; the pinch rule after a conversion
is pinned by a gap that closes once both of its sides have turned solid.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2502_12955_amd import inputs

DP, C0 = 0.01, 0.37            # 1 / (DP c0) = 270.27...: t* = 271, far from a tie


def _rest_box(lattice, shape, mask):
    nz, ny, nx = shape
    p = inputs.base_params(lattice=lattice, nx=nx, ny=ny, nz=nz, ncomp=1, G=((0, 0), (0, 0)),
                           tau=(0.8, 0.8), solute="periodic", D=0.15, J0=0.2, k_wall=0.0, storage="f64")
    m, _ = oracle.pinch_fill(p, mask)
    rho = np.where(m == 0, 1.0, 0.0)[None]
    C = np.where(m == 0, C0, 0.0)
    f, h = oracle.init(p, m, rho, None, C)
    return p, np.ascontiguousarray(m.reshape(-1)), f, h


@pytest.mark.parametrize("lattice,nz", [("D2Q9", 1), ("D3Q19", 3)])
def test_deposit_layers_grow_one_node_per_closed_form_period(lattice, nz):
    ny, nx = 12, 10
    mask = np.zeros((nz, ny, nx), np.uint8)
    mask[:, 0, :] = 1
    mask[:, ny - 1, :] = 1
    p, m, f, h = _rest_box(lattice, (nz, ny, nx), mask)
    QS = 7 if lattice == "D3Q19" else 5
    t_star = math.floor(1.0 / (DP * C0)) + 1
    assert t_star == 271
    Cps = np.zeros(nx * ny * nz)
    rows = lambda a: a.reshape(nz, ny, nx).transpose(1, 0, 2).reshape(ny, nz * nx)   # [y][z, x]
    n = oracle.step_deposit(p, m, f, h, Cps, DP, t_star - 1)
    assert n == 0
    # rows next to a wall hold (t*-1) DP c0; the rows further in hold nothing
    assert np.allclose(rows(Cps)[[1, ny - 2]], (t_star - 1) * DP * C0, rtol=1e-12, atol=0)
    assert np.all(rows(Cps)[2:ny - 2] == 0.0)
    # the particle field is still exactly uniform
    C = h[:QS].sum(axis=0)
    assert np.allclose(C[m == 0], C0, rtol=1e-13, atol=0)
    fluid_mass = f.sum()
    layer = nx * nz
    n = oracle.step_deposit(p, m, f, h, Cps, DP, 1)
    assert n == 2 * layer
    assert np.all(rows(m)[[0, 1, ny - 2, ny - 1]] == 1) and np.all(rows(m)[2:ny - 2] == 0)
    assert np.all(rows(Cps)[[1, ny - 2]] == 0.0) and np.all(f[:, m == 1] == 0.0)
    # the converted nodes took their fluid (rho = 1 each) and particles (c0 each) with them
    assert abs(f.sum() - (fluid_mass - 2 * layer)) < 1e-10
    assert abs(h[:QS].sum() - C0 * layer * (ny - 4)) < 1e-10
    # the next layer starts from zero and needs the same t* steps
    n = oracle.step_deposit(p, m, f, h, Cps, DP, t_star - 1)
    assert n == 0
    assert np.allclose(rows(Cps)[[2, ny - 3]], (t_star - 1) * DP * C0, rtol=1e-12, atol=0)
    n = oracle.step_deposit(p, m, f, h, Cps, DP, 1)
    assert n == 2 * layer
    assert int(m.sum()) == 6 * layer


@pytest.mark.parametrize("lattice,shape,nbrs", [("D2Q9", (1, 9, 9), 8), ("D3Q19", (7, 7, 7), 18)])
def test_only_flow_lattice_neighbours_of_a_solid_collect(lattice, shape, nbrs):
    """One solid voxel in a periodic box: exactly its flow-lattice neighbours
    (8 in D2Q9 with the diagonals, 18 in D3Q19 without the cube corners) collect."""
    mask = np.zeros(shape, np.uint8)
    c = tuple(s // 2 for s in shape)
    mask[c] = 1
    p, m, f, h = _rest_box(lattice, shape, mask)
    Cps = np.zeros(m.size)
    oracle.step_deposit(p, m, f, h, Cps, DP, 5)
    got = np.argwhere(Cps.reshape(shape) > 0)
    assert len(got) == nbrs
    cvec, _, _ = oracle.flow_lattice(lattice)
    want = {(c[0] + d[2], c[1] + d[1], c[2] + d[0]) for d in cvec[1:]}
    assert {tuple(g) for g in got} == want
    assert np.allclose(Cps[Cps > 0], 5 * DP * C0, rtol=1e-12, atol=0)


def test_a_gap_closed_by_deposits_on_both_sides_is_filled_by_the_pinch_rule():
    """Two solid columns at x = 3 and x = 7 across a periodic box leave a gap of
    three columns.  Columns 4 and 6 collect and turn solid at t*; column 5 never
    collected, but is then pinched between two solids along x and turns solid in
    the same step."""
    nz, ny, nx = 1, 6, 11
    mask = np.zeros((nz, ny, nx), np.uint8)
    mask[0, :, 3] = 1
    mask[0, :, 7] = 1
    p, m, f, h = _rest_box("D2Q9", (nz, ny, nx), mask)
    Cps = np.zeros(m.size)
    n = oracle.step_deposit(p, m, f, h, Cps, DP, 270)
    assert n == 0 and np.all(Cps.reshape(ny, nx)[:, 5] == 0.0)
    n = oracle.step_deposit(p, m, f, h, Cps, DP, 1)
    cols = m.reshape(ny, nx).all(axis=0)
    assert cols[2] and cols[3] and cols[4] and cols[5] and cols[6] and cols[7] and cols[8]
    assert not cols[0] and not cols[1] and not cols[9] and not cols[10]
    # columns 2, 4, 6, 8 by their deposits, column 5 by the pinch rule
    assert n == 5 * ny
    assert np.all(f[:, m == 1] == 0.0) and np.all(h[:, m == 1] == 0.0)


def test_deposit_collects_the_post_streaming_concentration():
    """With flow and a non-uniform field the increment of one step is DP times the
    concentration the moments report after that step, at every collecting node."""
    p, mask, rho, u, C = inputs.porous_case(shape=(1, 24, 30), porosity=0.6, radius=3, blob_radius=2, sample=4)
    p.update(lattice="D2Q9", nz=1, solute="inlet_outlet_x", C_in=0.8, k_wall=0.02, ncomp=1,
             G=((0, 0), (0, 0)), storage="f64")
    rho = rho[:1]
    m, _ = oracle.pinch_fill(p, mask)
    m = np.ascontiguousarray(m.reshape(-1))
    f, h = oracle.init(p, m, rho, None, 0.3 * np.ones(m.size))
    Cps = np.zeros(m.size)
    oracle.step_deposit(p, m, f, h, Cps, 1e-3, 20)
    before = Cps.copy()
    oracle.step(p, m, f, h, 1)
    _, _, Cnow = oracle.moments(p, m, f, h)
    n = oracle.deposit(p, m, f, h, Cps, 1e-3)
    assert n == 0
    fb, _ = oracle.link_masks(p, m)
    near = (m == 0) & (fb != 0)
    assert near.sum() > 0
    assert np.allclose(Cps[near] - before[near], 1e-3 * Cnow[near], rtol=1e-9, atol=1e-18)
    assert np.all(Cps[~near] == before[~near])
