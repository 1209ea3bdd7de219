"""GPU: degenerate and extreme inputs against the oracle (no fault, same results).

Periodic boxes of one or two nodes per axis (every neighbour is the node itself or
its one partner), zero steps, and a lattice whose fluid count is one more than a
whole 64-node chunk.
"""
import numpy as np
import pytest

import oracle
from paper_2502_12955_amd import inputs

from helpers import gpu_lattice, maxrel, oracle_state, split_pops

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("lattice,shape", [("D3Q19", (1, 1, 1)), ("D3Q19", (2, 1, 3)), ("D2Q9", (1, 1, 1)),
                                           ("D2Q9", (1, 2, 1))])
def test_tiny_periodic_boxes_match_oracle(lattice, shape):
    nz, ny, nx = shape
    p = inputs.base_params(lattice=lattice, nx=nx, ny=ny, nz=nz, ncomp=2, tau=(0.9, 1.2), G=((0.0, 1.5), (1.5, 0.0)),
                           accel=(1e-4, -2e-5, 0.0), solute="periodic", D=0.2, storage="f64")
    u01 = inputs.SplitMix64(inputs.seed_for(7, nx * 100 + ny * 10 + nz)).uniform(2 * nx * ny * nz)
    rho = (0.5 + u01).reshape((2,) + shape)
    C = np.linspace(0.1, 0.9, nx * ny * nz).reshape(shape)
    mask = np.zeros(shape, np.uint8)
    m, f, h = oracle_state(p, mask, rho, None, C)
    oracle.step(p, m, f, h, 25)
    lat = gpu_lattice(p, mask, rho, None, C)
    lat.step(0)                                       # zero steps: a no-op
    assert lat.monitors()[10] == 0
    lat.step(25)
    fg, hg = split_pops(p, lat.populations())
    assert maxrel(fg, f) < 1e-12 and maxrel(hg, h) < 1e-12
    lat.close()


def test_one_node_past_a_whole_chunk():
    """65 fluid nodes: one full 64-node chunk and a chunk with a single live lane."""
    nx = 67
    p = inputs.base_params(lattice="D2Q9", nx=nx, ny=1, nz=1, ncomp=1, G=((0, 0), (0, 0)), accel=(1e-5, 0, 0),
                           solute="inlet_outlet_x", D=0.3, k_wall=0.05, C_in=0.5, storage="f64")
    mask = np.zeros((1, 1, nx), np.uint8)
    mask[0, 0, nx - 2:] = 1                          # 65 fluid nodes, a reacting wall at the end
    rho = np.where(mask == 0, 1.0, 0.0)[None]
    m, f, h = oracle_state(p, mask, rho)
    assert int((m == 0).sum()) == 65
    oracle.step(p, m, f, h, 200)
    lat = gpu_lattice(p, mask, rho)
    lat.step(200)
    fg, hg = split_pops(p, lat.populations())
    assert maxrel(fg, f) < 1e-12 and maxrel(hg, h) < 1e-12
    lat.close()
