"""GPU: the multiphase validation cases of the paper on the HIP path.

Single component with a diagonal cohesion (eq:1.12, G = -5): FP64 parity
with the oracle (element by element, <= 1e-12 of the field's scale), a phase
separation that reaches the flat-interface coexistence densities, and the two-component contact angle
(eq:1.15) on the side of 90 degrees that the adhesion relation predicts.
"""
import numpy as np
import pytest

import oracle
from paper_2502_12955_amd import inputs, validation

from helpers import gpu_lattice, maxrel, oracle_state, split_pops

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("lattice,shape", [("D2Q9", (1, 48, 40)), ("D3Q19", (14, 12, 10))])
@pytest.mark.parametrize("forcing", ["sc", "guo"])
def test_single_component_cohesion_fp64_matches_oracle(lattice, shape, forcing):
    nz, ny, nx = shape
    p = inputs.base_params(lattice=lattice, nx=nx, ny=ny, nz=nz, ncomp=1, tau=(1.0, 1.0),
                           G=((-5.0, 0.0), (0.0, 0.0)), G_ads=(-0.3, 0.0), forcing=forcing, solute="off",
                           storage="f64")
    mask = np.zeros(shape, np.uint8)
    mask[:, 0, :] = 1                                       # one wall, adhesion on it
    u01 = inputs.SplitMix64(inputs.seed_for(6, 1)).uniform(nx * ny * nz).reshape(shape)
    rho = (0.7 * (1.0 + 0.1 * (2.0 * u01 - 1.0)))[None]
    m, f, h = oracle_state(p, mask, rho)
    oracle.step(p, m, f, h, 300)
    lat = gpu_lattice(p, mask, rho)
    lat.step(300)
    fg, _ = split_pops(p, lat.populations())
    print(lattice, forcing, maxrel(fg, f), flush=True)
    assert maxrel(fg, f) < 1e-12
    lat.close()


def test_phase_separation_reaches_the_coexistence_densities():
    """128^2, G = -5, uniform 0.7 with 10 % perturbations (the paper's phase-separation
    set-up), velocity-shift forcing at tau = 1: the bulk densities of the droplets
    and the vapour settle near the flat-interface coexistence (Laplace pressure of
    the curved interfaces shifts them by a few per cent)."""
    rv, rl = validation.sc_coexistence(-5.0)
    r = validation.phase_separation(128, steps=20000)
    print(r, rv, rl, flush=True)
    assert abs(r["mass_rel_change"]) < 1e-10
    assert abs(r["liquid"] / rl - 1) < 0.03
    assert abs(r["vapour"] / rv - 1) < 0.15


def test_contact_angle_side_of_90_degrees_follows_the_adhesion():
    """A neutral wall keeps the droplet near 90 degrees; adhesion that attracts the
    droplet's component (G_ads,1 < 0 < G_ads,2) spreads it, the opposite adhesion
    lifts it, on the sides of 90 degrees the relation of Huang et al. gives."""
    bulk = validation.two_component_bulk(5.0)
    assert 0.9 < bulk[0] < 1.0 and 0.08 < bulk[1] < 0.16
    neutral = validation.contact_angle(0.0, steps=20000, bulk=bulk)
    wet = validation.contact_angle(-0.1, steps=20000, bulk=bulk)
    dry = validation.contact_angle(0.1, steps=20000, bulk=bulk)
    print(neutral, wet, dry, flush=True)
    assert abs(neutral["theta_deg"] - 90.0) < 4.0
    assert wet["theta_deg"] < neutral["theta_deg"] - 5.0 and wet["huang_deg"] < 90.0
    assert dry["theta_deg"] > neutral["theta_deg"] + 5.0 and dry["huang_deg"] > 90.0
