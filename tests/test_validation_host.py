"""Host-side logic of the validation cases (no GPU): the coexistence condition
and the contact-angle construction."""
import math

import numpy as np

from paper_2502_12955_amd import validation


def test_coexistence_condition_textbook_values():
    """psi = 1 - exp(-rho), G = -5: vapour 0.156, liquid 1.932 (Shan-Chen
    mechanical stability; the values quoted in the lattice Boltzmann literature)."""
    rv, rl = validation.sc_coexistence(-5.0)
    assert abs(rv - 0.1564) < 5e-4 and abs(rl - 1.9324) < 5e-4
    # weaker cohesion: the two phases approach each other
    rv4, rl4 = validation.sc_coexistence(-4.5)
    assert rv4 > rv and rl4 < rl


def test_cap_construction_on_exact_circles():
    for theta in (30.0, 60.0, 90.0, 120.0, 150.0):
        r = 10.0
        t = math.radians(theta)
        h = r * (1 - math.cos(t))
        b = 2 * r * math.sin(t)
        rr, tt = validation.cap_angle(h, b)
        assert abs(rr - r) < 1e-12 and abs(math.degrees(tt) - theta) < 1e-9


def test_huang_relation():
    assert abs(math.degrees(validation.huang_angle((0.0, 0.0), 5.0, 1.0, 0.03)) - 90.0) < 1e-12
    c = math.cos(validation.huang_angle((-0.3, 0.3), 5.0, 1.0, 0.0))
    assert abs(c - 0.6 / 2.5) < 1e-12


def test_measure_cap_on_a_smooth_synthetic_droplet():
    """A tanh-smoothed circular cap of known angle on the wall at y = 0.5."""
    ny, nx = 60, 160
    for theta in (60.0, 90.0, 120.0):
        r = 22.0
        t = math.radians(theta)
        yc = 0.5 - r * math.cos(t)          # centre height: the cap meets the wall at angle theta
        y, x = np.mgrid[0:ny, 0:nx].astype(float)
        d = np.hypot(x - nx / 2, y - yc)
        phi = -np.tanh((d - r) / 2.0)
        phi[0] = 0.0
        h, b = validation.measure_cap(phi)
        _, tt = validation.cap_angle(h, b)
        assert abs(math.degrees(tt) - theta) < 4.0, (theta, math.degrees(tt))
