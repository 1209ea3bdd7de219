"""Pins of the oracle's conjugate heat transfer (Reactive LBM subsection; no GPU).

Energy populations in the fluid (eq:therpop, eq:therpopeq) and the solid
(eq:therpop_solid, eq:therpopeq_solid), coupled at interface nodes by the
thermal counter-slip conditions (eq:countSlipFluxCon, eq:countSlipTempCon)
with the reaction heat (eq:reacRate) and the wet-node reaction
(eq:wetnode9).  Each test states what fixes the expected value:
  - node classes against a brute-force neighbour scan;
  - a uniform temperature at rest is a fixed point;
  - a diffusing point pulse in pure fluid and in pure solid: the exact BGK
    second-moment recursion, drift u per step under uniform flow, and (the
    second-order equilibrium) the same spread under uniform flow as at rest;
  - two half-spaces brought into contact: the interface settles at the
    effusivity-weighted mean (e = rho c_p sqrt(alpha)), the classical
    conduction result, reached as t^-1/2;
  - after every step, at every interface node: equal temperatures on both
    sides, and the heat-flux balance with the reaction heat computed from
    the node's own solute populations;
  - on a flat wall the unknown populations equal the printed
    eq:unknownpopTempS and eq:unknownpopTempF;
  - the reaction heat raises the wall temperature, more so with a faster
    reaction.
"""
import numpy as np
import pytest

import oracle
from paper_2502_12955_amd import inputs


def _thermal_params(lat="D2Q9", nx=4, ny=60, nz=1, **kw):
    p = inputs.base_params(lattice=lat, nx=nx, ny=ny, nz=nz, ncomp=1, G=((0, 0), (0, 0)), tau=(1.0, 1.0),
                           solute="off", J0=0.4 if lat == "D2Q9" else 0.1)
    p.update(tau_ef=0.8, tau_es=1.3, rhocp_f=1.0, rhocp_s=2.5, h_r=0.0, arr_A=0.0, arr_E_over_R=0.0,
             T_tol=1e-14, T_maxit=100)
    p.update(kw)
    return p


def _slab(p, solid_rows, axis="y"):
    """Solid slab of the first `solid_rows` rows (y) or planes (z), periodic box."""
    nz, ny, nx = int(p.get("nz", 1)), int(p["ny"]), int(p["nx"])
    mask = np.zeros((nz, ny, nx), np.uint8)
    if axis == "y":
        mask[:, :solid_rows, :] = 1
    else:
        mask[:solid_rows, :, :] = 1
    return mask


def _weights(lat):
    c, w, opp = oracle.flow_lattice(lat)
    return c, w, opp


# ----------------------------------------------------------------------------- node classes
@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
def test_node_classes_match_a_neighbour_scan(lat):
    nz = 9 if lat == "D3Q19" else 1
    p = _thermal_params(lat, nx=11, ny=10, nz=nz)
    mask, _, _ = inputs.sphere_pack((nz, 10, 11), 0.6, 2, inputs.seed_for(9, 41))
    hs, it = oracle.thermal_nodes(p, mask)
    c, _, _ = _weights(lat)
    solid = mask.astype(bool)
    near = np.zeros_like(solid)
    for ci in c[1:]:
        near |= np.roll(solid, shift=(int(ci[2]), int(ci[1]), int(ci[0])), axis=(0, 1, 2))
    want_it = (~solid) & near
    assert np.array_equal(it.reshape(mask.shape).astype(bool), want_it)
    assert np.array_equal(hs.reshape(mask.shape).astype(bool), solid | want_it)


# ----------------------------------------------------------------------------- fixed point
@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
def test_uniform_temperature_at_rest_is_a_fixed_point(lat):
    nz = 10 if lat == "D3Q19" else 1
    p = _thermal_params(lat, nx=12, ny=11, nz=nz, solute="periodic", k_wall=0.0, h_r=0.0)
    mask, _, _ = inputs.sphere_pack((nz, 11, 12), 0.55, 3, inputs.seed_for(9, 42))
    mask, _ = oracle.pinch_fill(p, mask)
    N = mask.size
    rho = np.ones((1, N))
    f, h = oracle.init(p, mask, rho, None, np.full(N, 0.3))
    g, gs, Ti = oracle.thermal_init(p, mask, np.full(N, 0.7))
    oracle.step_thermal(p, mask, f, h, g, gs, Ti, 30)
    T = oracle.temperature(p, mask, g, gs)
    assert np.abs(T - 0.7).max() < 1e-13


# ----------------------------------------------------------------------------- pulses
def _pulse(p, mask, centre, u=None, steps=9):
    N = mask.size
    T0 = np.zeros(N)
    T0[np.ravel_multi_index(centre, mask.shape)] = 1.0
    rho = np.ones((1, N))
    uu = None
    if u is not None:
        uu = np.zeros((3, N))
        for a in range(3):
            uu[a] = u[a]
    f, h = oracle.init(p, mask, rho, uu)
    g, gs, Ti = oracle.thermal_init(p, mask, T0, uu)
    oracle.step_thermal(p, mask, f, h, g, gs, Ti, steps)
    E = (gs if mask.all() else g).sum(0).reshape(mask.shape)
    return E


@pytest.mark.parametrize("lat,phase", [("D2Q9", "fluid"), ("D2Q9", "solid"), ("D3Q19", "fluid"), ("D3Q19", "solid")])
def test_pulse_second_moment_exact(lat, phase):
    """Point pulse of energy at rest, equilibrium start, pure fluid (no solid
    node) or pure solid (no fluid node): per axis the variance grows as
    m2(n) = cs2 M [(2 tau - 1) n - 2 tau (tau - 1)(1 - (1 - 1/tau)^n)], cs2 = 1/3."""
    n = 24
    nz = n if lat == "D3Q19" else 1
    p = _thermal_params(lat, nx=n, ny=n, nz=nz, tau_ef=0.83, tau_es=1.45, rhocp_f=1.7, rhocp_s=0.6)
    mask = np.full((nz, n, n), 1 if phase == "solid" else 0, np.uint8)
    centre = (nz // 2, n // 2, n // 2)
    steps = 9
    E = _pulse(p, mask, centre, steps=steps)
    tau = p["tau_es"] if phase == "solid" else p["tau_ef"]
    M = E.sum()
    rc = p["rhocp_s"] if phase == "solid" else p["rhocp_f"]
    assert abs(M - rc) < 1e-13
    x = np.arange(n) - n // 2
    want = M / 3.0 * ((2 * tau - 1) * steps - 2 * tau * (tau - 1) * (1 - (1 - 1 / tau) ** steps))
    mx = (E.sum(axis=(0, 1)) * x * x).sum()
    my = (E.sum(axis=(0, 2)) * x * x).sum()
    assert abs(mx - want) < 1e-12 * want and abs(my - want) < 1e-12 * want


def test_fluid_pulse_drifts_with_uniform_flow():
    """With uniform u the fluid energy centroid moves exactly u per step (the
    first moment of eq:therpopeq is E u)."""
    u = (0.02, -0.01, 0.005)
    n = 24
    p = _thermal_params("D3Q19", nx=n, ny=n, nz=n)
    mask = np.zeros((n, n, n), np.uint8)
    steps = 8
    E = _pulse(p, mask, (n // 2, n // 2, n // 2), u=u, steps=steps)
    x = np.arange(n) - n // 2
    cen = [(E.sum(axis=(0, 1)) * x).sum(), (E.sum(axis=(0, 2)) * x).sum(), (E.sum(axis=(1, 2)) * x).sum()]
    assert np.allclose(np.array(cen) / E.sum(), np.array(u) * steps, rtol=1e-11, atol=1e-14)


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
def test_fluid_pulse_spreads_as_at_rest_under_uniform_flow(lat):
    """The second-order terms of eq:therpopeq make the second moment of the
    equilibrium E (cs2 I + u u), so under a uniform u the central variance of a
    pulse grows by exactly the closed form at rest (a first-order equilibrium
    would add a numerical diffusion of order u^2)."""
    n = 24
    nz = n if lat == "D3Q19" else 1
    u = (0.05, -0.03, 0.02 if lat == "D3Q19" else 0.0)
    tau = 0.83
    p = _thermal_params(lat, nx=n, ny=n, nz=nz, tau_ef=tau)
    mask = np.zeros((nz, n, n), np.uint8)
    steps = 8
    E = _pulse(p, mask, (nz // 2, n // 2, n // 2), u=u, steps=steps)
    x = np.arange(n) - n // 2
    M = E.sum()
    want = 1.0 / 3.0 * ((2 * tau - 1) * steps - 2 * tau * (tau - 1) * (1 - (1 - 1 / tau) ** steps))
    for ax in ((0, 1), (0, 2)):
        e = E.sum(axis=ax)
        c = (e * x).sum() / M
        var = (e * (x - c) ** 2).sum() / M
        assert abs(var - want) < 1e-12 * want


# ----------------------------------------------------------------------------- contact
@pytest.mark.parametrize("lat,taus,rcs", [("D2Q9", (0.8, 1.3), (1.0, 2.5)), ("D2Q9", (0.7, 2.0), (2.0, 1.0)),
                                          ("D3Q19", (0.9, 1.2), (1.0, 3.0))])
def test_contact_temperature_is_the_effusivity_mean(lat, taus, rcs):
    """Fluid at T = 1 and solid at T = 0, brought into contact along a flat
    interface: the interface temperature of two half-spaces is the constant
    (e_f T_f + e_s T_s) / (e_f + e_s), e = rho c_p sqrt(alpha), alpha =
    (tau - 1/2)/3.  The discrete interface approaches it as t^-1/2, so the
    extrapolation 2 T(4t) - T(t) from t = 400 and 1600 must hit it."""
    ny, ns = 600, 300
    if lat == "D2Q9":
        p = _thermal_params(lat, nx=4, ny=ny, nz=1, tau_ef=taus[0], tau_es=taus[1], rhocp_f=rcs[0], rhocp_s=rcs[1])
        mask = _slab(p, ns, "y")
        line = lambda T: T.reshape(mask.shape)[0, :, 0]
    else:
        p = _thermal_params(lat, nx=2, ny=2, nz=ny, tau_ef=taus[0], tau_es=taus[1], rhocp_f=rcs[0], rhocp_s=rcs[1])
        mask = _slab(p, ns, "z")
        line = lambda T: T.reshape(mask.shape)[:, 0, 0]
    N = mask.size
    m = mask.reshape(-1)
    rho = np.ones((1, N))
    f, h = oracle.init(p, mask, rho)
    g, gs, Ti = oracle.thermal_init(p, mask, np.where(m == 1, 0.0, 1.0))
    oracle.step_thermal(p, mask, f, h, g, gs, Ti, 400)
    T400 = line(oracle.temperature(p, mask, g, gs))[ns]
    oracle.step_thermal(p, mask, f, h, g, gs, Ti, 1200)
    T1600 = line(oracle.temperature(p, mask, g, gs))[ns]
    ef = rcs[0] * np.sqrt((taus[0] - 0.5) / 3)
    es = rcs[1] * np.sqrt((taus[1] - 0.5) / 3)
    want = ef / (ef + es)
    assert abs(T1600 - want) < abs(T400 - want)          # approaching
    assert abs(2 * T1600 - T400 - want) < 1.5e-3           # at the t^-1/2 rate


# ----------------------------------------------------------------------------- interface identities
def _reactive_wall(steps, h_r=0.8, A=5.0, EoR=2.0, lat="D2Q9", T0=1.0):
    """Flat reacting wall (solid rows 0..7 of 24), solute diffusing from a
    uniform initial C = 1, Arrhenius rate of the interface temperature."""
    p = _thermal_params(lat, nx=6, ny=24, solute="periodic", D=0.1, k_wall=0.0, h_r=h_r, arr_A=A,
                        arr_E_over_R=EoR, tau_ef=0.8, tau_es=1.2, rhocp_f=1.0, rhocp_s=2.0)
    mask = _slab(p, 8, "y")
    N = mask.size
    rho = np.ones((1, N))
    f, h = oracle.init(p, mask, rho, None, np.ones(N))
    g, gs, Ti = oracle.thermal_init(p, mask, np.full(N, T0))
    stats = oracle.step_thermal(p, mask, f, h, g, gs, Ti, steps)
    return p, mask, f, h, g, gs, Ti, stats


def test_interface_temperature_and_flux_balance_hold_after_each_step():
    p, mask, f, h, g, gs, Ti, stats = _reactive_wall(1)
    _, w, opp = _weights("D2Q9")
    _, W, sopp, cs2 = oracle.solute_lattice("D2Q9", p["J0"])
    hs, it = oracle.thermal_nodes(p, mask)
    nx, ny = p["nx"], p["ny"]
    tau_d = p["D"] / cs2 + 0.5
    kf, ks = 1 - 0.5 / p["tau_ef"], 1 - 0.5 / p["tau_es"]
    for step in range(6):
        if step:
            oracle.step_thermal(p, mask, f, h, g, gs, Ti, 1)
        for y, up in ((8, True), (23, False)):       # wall below row 8, wall above row 23 (row 0 solid)
            for x in range(nx):
                n = y * nx + x
                assert it[n] == 1
                Tf = g[:, n].sum() / p["rhocp_f"]
                Ts = gs[:, n].sum() / p["rhocp_s"]
                assert abs(Tf - Ts) < 1e-14 and abs(Tf - Ti[n]) < 1e-12
                # solute wet link: D2Q5 direction 2 (+y) from a wall below, 4 (-y) from above
                k = 2 if up else 4
                hin = h[sopp[k], n]
                Cb = (h[k, n] + hin) / (2 * W[k])      # from h_k = 2 W C_b - h_in
                kr = p["arr_A"] * np.exp(-p["arr_E_over_R"] / Ti[n])
                assert abs(Cb - 2 * hin / (2 * W[k] + kr * tau_d / (tau_d - 0.5))) < 1e-12 * abs(Cb)
                Hdot = p["h_r"] * kr * Cb
                into = [2, 5, 6] if up else [4, 7, 8]   # populations pointing away from the wall
                out = [opp[i] for i in into]
                flux_f = g[into, n].sum() - g[out, n].sum()
                flux_s = gs[into, n].sum() - gs[out, n].sum()
                assert abs(kf * flux_f - ks * flux_s - Hdot) < 1e-12 * max(1.0, abs(Hdot))
    assert stats[1] == 0 and stats[2] == 0


def test_flat_wall_unknowns_equal_the_printed_formulas():
    """Wall below (normal +y), D2Q9: the solid unknowns g_s,4/7/8 are the printed
    eq:unknownpopTempS, the fluid unknowns g_2/5/6 the printed eq:unknownpopTempF,
    evaluated from the node's known populations after the step."""
    p, mask, f, h, g, gs, Ti, _ = _reactive_wall(5)
    _, w, _ = _weights("D2Q9")
    _, W, sopp, cs2 = oracle.solute_lattice("D2Q9", p["J0"])
    cfs = p["rhocp_f"] / p["rhocp_s"]
    tf, ts = p["tau_ef"], p["tau_es"]
    ksf = (ts - 0.5) / ts * tf / (tf - 0.5)
    for x in range(p["nx"]):
        n = 8 * p["nx"] + x
        G = g[:, n]
        S = gs[:, n]
        Cb = (h[2, n] + h[sopp[2], n]) / (2 * W[2])
        kr = p["arr_A"] * np.exp(-p["arr_E_over_R"] / Ti[n])
        Hdot = p["h_r"] * kr * Cb
        bracket = (ksf * (S[2] + S[5] + S[6]) + (G[4] + G[7] + G[8])
                   + (G[0] + G[1] + G[3] + G[4] + G[7] + G[8])
                   - cfs * (S[0] + S[1] + S[2] + S[3] + S[5] + S[6])
                   + tf / (tf - 0.5) * Hdot)
        for a in (4, 7, 8):
            want = w[a] / ((w[4] + w[7] + w[8]) * (ksf + cfs)) * bracket
            assert abs(S[a] - want) < 1e-12 * abs(want)
        for a in (2, 5, 6):
            want = w[a] / (w[2] + w[5] + w[6]) * (cfs * S.sum() - (G[0] + G[1] + G[3] + G[4] + G[7] + G[8]))
            assert abs(G[a] - want) < 1e-12 * abs(want)


def test_reaction_heat_warms_the_wall():
    """With h_r > 0 the wall ends warmer than without, and warmer still with a
    faster reaction (larger pre-exponential factor)."""
    T = {}
    for key, hr, A in (("none", 0.0, 5.0), ("slow", 0.8, 1.0), ("fast", 0.8, 5.0)):
        p, mask, f, h, g, gs, Ti, _ = _reactive_wall(60, h_r=hr, A=A)
        T[key] = oracle.temperature(p, mask, g, gs).reshape(mask.shape)[0, 8, :].mean()
    assert abs(T["none"] - 1.0) < 1e-13
    assert 1.0 < T["slow"] < T["fast"]


def test_two_node_channel_interfaces_are_posed():
    """A fluid gap two nodes wide between solid slabs: every fluid node is an
    interface node; the solid populations that would stream across the gap
    from the other wall are unknowns of the counter-slip conditions, so the
    flux condition is posed at every node (no degenerate node) and the
    temperatures on both sides agree at every interface node."""
    p = _thermal_params("D2Q9", nx=5, ny=12, solute="periodic", D=0.1, h_r=0.6, arr_A=4.0, arr_E_over_R=1.0)
    mask = np.ones((1, 12, 5), np.uint8)
    mask[0, 5:7, :] = 0
    N = mask.size
    f, h = oracle.init(p, mask, np.ones((1, N)), None, np.ones(N))
    g, gs, Ti = oracle.thermal_init(p, mask, np.full(N, 1.0))
    stats = oracle.step_thermal(p, mask, f, h, g, gs, Ti, 20)
    assert stats[2] == 0 and stats[1] == 0
    _, it = oracle.thermal_nodes(p, mask)
    assert it.sum() == 10
    for n in np.nonzero(it)[0]:
        assert abs(g[:, n].sum() / p["rhocp_f"] - gs[:, n].sum() / p["rhocp_s"]) < 1e-14
    T = oracle.temperature(p, mask, g, gs).reshape(12, 5)
    assert T[5:7].min() > 1.0          # the reaction heat stays in the gap's walls and fluid
