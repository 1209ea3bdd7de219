"""Pins of the oracle's lattice tables and local formulas (no GPU).

The tables are compared with the paper's printed tables (tests/golden), and
with exact rational moment identities; the equilibrium (eq:6), Guo term
(eq:1.21) and pseudo-potential (eq:1.11) with their defining moments.
"""
import json
import os
from fractions import Fraction
from itertools import product

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "lattice_tables.json")


def _golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


@pytest.mark.parametrize("name,lat", [("D3Q19", "D3Q19"), ("D2Q9", "D2Q9")])
def test_flow_tables_match_paper(name, lat):
    g = _golden()[name]
    c, w, opp = oracle.flow_lattice(lat)
    cz = g.get("cz", [0] * len(g["cx"]))
    assert c.tolist() == [list(t) for t in zip(g["cx"], g["cy"], cz)]
    assert np.array_equal(w * g["den"], np.array(g["w"], float))
    for i in range(len(w)):
        assert (c[opp[i]] == -c[i]).all()


def test_d2q5_table_matches_paper_at_J0_04():
    g = _golden()["D2Q5"]
    c, w, opp, cs2 = oracle.solute_lattice("D2Q9", 0.4)
    assert c[:, :2].tolist() == [list(t) for t in zip(g["cx"], g["cy"])]
    assert np.allclose(w * g["den"], g["w"], rtol=0, atol=1e-14)
    assert abs(cs2 - 0.3) < 1e-15


def test_d3q7_is_first_seven_d3q19_vectors():
    c19, _, _ = oracle.flow_lattice("D3Q19")
    c, w, opp, cs2 = oracle.solute_lattice("D3Q19", 0.1)
    assert (c == c19[:7]).all()
    assert abs(w.sum() - 1.0) < 1e-15 and abs(w[0] - 0.1) < 1e-15
    assert abs(cs2 - 0.3) < 1e-15  # keeps tau_d = (10/3) D + 1/2


@pytest.mark.parametrize("lat,dims", [("D3Q19", 3), ("D2Q9", 2)])
def test_exact_isotropy(lat, dims):
    """sum w = 1, sum w c = 0, sum w c c = cs2 I, sum w c^4 = cs2^2 (dd+dd+dd), in rationals."""
    c, w, _ = oracle.flow_lattice(lat)
    wf = [Fraction(x).limit_denominator(36) for x in w]
    cs2 = Fraction(1, 3)
    assert sum(wf) == 1
    ax = range(dims)
    for a in ax:
        assert sum(wf[i] * c[i][a] for i in range(len(w))) == 0
    for a, b in product(ax, ax):
        assert sum(wf[i] * c[i][a] * c[i][b] for i in range(len(w))) == (cs2 if a == b else 0)
    for a, b, cc in product(ax, ax, ax):
        assert sum(wf[i] * c[i][a] * c[i][b] * c[i][cc] for i in range(len(w))) == 0
    for a, b, cc, d in product(ax, ax, ax, ax):
        want = cs2 * cs2 * ((a == b) * (cc == d) + (a == cc) * (b == d) + (a == d) * (b == cc))
        assert sum(wf[i] * c[i][a] * c[i][b] * c[i][cc] * c[i][d] for i in range(len(w))) == want


@pytest.mark.parametrize("lat", ["D3Q19", "D2Q9"])
def test_equilibrium_moments(lat):
    c, w, _ = oracle.flow_lattice(lat)
    cs2 = 1.0 / 3.0
    rng = np.random.default_rng(1)
    for _ in range(5):
        rho = 0.3 + rng.random()
        v = 0.05 * (rng.random(3) - 0.5)
        if lat == "D2Q9":
            v[2] = 0.0
        fe = oracle.feq(lat, rho, v)
        assert abs(fe.sum() - rho) < 1e-15 * 10
        assert np.allclose(c.T @ fe, rho * v, atol=1e-16 * 10)
        P = np.einsum("i,ia,ib->ab", fe, c, c)
        want = rho * cs2 * np.eye(3) + rho * np.outer(v, v)
        if lat == "D2Q9":
            want[2, 2] = 0.0
        assert np.allclose(P, want, atol=1e-15)


@pytest.mark.parametrize("lat", ["D3Q19", "D2Q9"])
def test_guo_term_moments(lat):
    """sum F_i = 0, sum c F_i = F, sum c c F_i = u F + F u (Guo et al. 2002)."""
    c, _, _ = oracle.flow_lattice(lat)
    rng = np.random.default_rng(2)
    for _ in range(5):
        F = 1e-3 * (rng.random(3) - 0.5)
        u = 0.05 * (rng.random(3) - 0.5)
        if lat == "D2Q9":
            F[2] = u[2] = 0.0
        S = oracle.guo(lat, F, u)
        assert abs(S.sum()) < 1e-17
        assert np.allclose(c.T @ S, F, atol=1e-17)
        M2 = np.einsum("i,ia,ib->ab", S, c, c)
        assert np.allclose(M2, np.outer(u, F) + np.outer(F, u), atol=1e-17)


def test_psi_limits():
    assert oracle.psi(0.0) == 0.0
    assert abs(oracle.psi(50.0, 1.0) - 1.0) < 1e-15
    # derivative at 0 is 1; psi(rho0) = rho0 (1 - 1/e)
    assert abs(oracle.psi(1e-8) / 1e-8 - 1.0) < 1e-7
    assert abs(oracle.psi(2.0, 2.0) - 2.0 * (1 - np.exp(-1.0))) < 1e-15
