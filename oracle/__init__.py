"""Plain FP64 CPU oracle for the multi-component Shan-Chen LBM with a reactive solute.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.  It
shares no code with the HIP library (``paper_2502_12955_amd``) and imports
nothing from it.

The arithmetic lives in ``mclbm_oracle.c`` (plain scalar C loops, FP64, no
fast-math), compiled to ``liboracle.so`` next to this file.  This module only
marshals numpy arrays.  Every function cites the part of the paper it
follows; see the C file for the formulas.

Parameters are plain dicts with the keys listed in ``PARAM_KEYS``; the same
dict drives the HIP library, each side converting it to its own struct.

Residual monitor (not in the paper, our definition): for a field ``a`` at
steps t and t-K over fluid nodes, ``r = ||a(t) - a(t-K)||_2 / ||a(t)||_2``.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "mclbm_oracle.c")

PARAM_KEYS = ("lattice", "nx", "ny", "nz", "ncomp", "forcing", "solute", "tau", "G",
              "G_ads", "rho0", "accel", "D", "J0", "k_wall", "C_in", "product", "D2", "C_in2", "k_node")

LATTICES = {"D2Q9": 0, "D3Q19": 1}
FORCINGS = {"guo": 0, "sc": 1}
SOLUTES = {"off": 0, "periodic": 1, "inlet_outlet_x": 2}


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (-O2 -fopenmp, no fast-math)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-std=c99", "-Wall", "-shared", "-fPIC",
           "-o", _SO + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_SO + ".tmp", _SO)
    return _SO


class _Params(ct.Structure):
    _fields_ = [("lattice", ct.c_int32), ("nx", ct.c_int32), ("ny", ct.c_int32),
                ("nz", ct.c_int32), ("ncomp", ct.c_int32), ("forcing", ct.c_int32),
                ("solute", ct.c_int32), ("pad_", ct.c_int32),
                ("tau", ct.c_double * 2), ("G", (ct.c_double * 2) * 2),
                ("G_ads", ct.c_double * 2), ("rho0", ct.c_double),
                ("accel", ct.c_double * 3), ("D", ct.c_double), ("J0", ct.c_double),
                ("k_wall", ct.c_double), ("C_in", ct.c_double),
                ("product", ct.c_int32), ("pad2_", ct.c_int32), ("D2", ct.c_double), ("C_in2", ct.c_double),
                ("k_node", ct.POINTER(ct.c_double))]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        _lib = ct.CDLL(_SO)
        _lib.orc_pinch_fill.restype = ct.c_int64
        _lib.orc_flow_lattice.restype = ct.c_int
        _lib.orc_solute_lattice.restype = ct.c_int
        _lib.orc_psi.restype = ct.c_double
        _lib.orc_psi.argtypes = [ct.c_double, ct.c_double]
    return _lib


def _enum(v, table):
    return table[v] if isinstance(v, str) else int(v)


def _struct(p: dict) -> _Params:
    s = _Params()
    s.lattice = _enum(p["lattice"], LATTICES)
    s.nx, s.ny, s.nz = int(p["nx"]), int(p["ny"]), int(p.get("nz", 1))
    s.ncomp = int(p.get("ncomp", 2))
    s.forcing = _enum(p.get("forcing", "guo"), FORCINGS)
    s.solute = _enum(p.get("solute", "off"), SOLUTES)
    tau = p.get("tau", (1.0, 1.0))
    s.tau[0], s.tau[1] = float(tau[0]), float(tau[1] if len(tau) > 1 else tau[0])
    G = p.get("G", ((0.0, 0.0), (0.0, 0.0)))
    for a in range(2):
        for b in range(2):
            s.G[a][b] = float(G[a][b])
    ga = p.get("G_ads", (0.0, 0.0))
    s.G_ads[0], s.G_ads[1] = float(ga[0]), float(ga[1])
    s.rho0 = float(p.get("rho0", 1.0))
    acc = p.get("accel", (0.0, 0.0, 0.0))
    for a in range(3):
        s.accel[a] = float(acc[a])
    s.D = float(p.get("D", 0.1))
    s.J0 = float(p.get("J0", 0.1))
    s.k_wall = float(p.get("k_wall", 0.0))
    s.C_in = float(p.get("C_in", 0.0))
    s.product = int(p.get("product", 0))
    s.D2 = float(p.get("D2", 0.1))
    s.C_in2 = float(p.get("C_in2", 0.0))
    kn = p.get("k_node")
    if kn is not None:     # per-node reaction rate [N]; the array must outlive the call
        s._k_node = np.ascontiguousarray(kn, np.float64).reshape(-1)
        s.k_node = s._k_node.ctypes.data_as(ct.POINTER(ct.c_double))
    return s


def _ptr(a, ctype):
    return a.ctypes.data_as(ct.POINTER(ctype))


def _q(p):
    return 19 if _enum(p["lattice"], LATTICES) == 1 else 9


def _qs(p):
    return 7 if _enum(p["lattice"], LATTICES) == 1 else 5


def n_species(p):
    """Solute species carried: 0 (solute off), 1 (O2), 2 (O2 and the product CO2)."""
    if _enum(p.get("solute", "off"), SOLUTES) == 0:
        return 0
    return 2 if int(p.get("product", 0)) else 1


def n_nodes(p):
    return int(p["nx"]) * int(p["ny"]) * int(p.get("nz", 1))


# ----------------------------------------------------------------------------- tables
def flow_lattice(lattice):
    """D2Q9 / D3Q19 velocities, weights and opposite directions (paper tables)."""
    lib = _load()
    c = np.zeros(19 * 3, np.int32)
    w = np.zeros(19)
    opp = np.zeros(19, np.int32)
    q = lib.orc_flow_lattice(_enum(lattice, LATTICES), _ptr(c, ct.c_int), _ptr(w, ct.c_double),
                             _ptr(opp, ct.c_int))
    return c[:3 * q].reshape(q, 3).copy(), w[:q].copy(), opp[:q].copy()


def solute_lattice(lattice, J0):
    """D2Q5 / D3Q7 velocities, weights (rest weight J0), opposites and c_s^2."""
    lib = _load()
    c = np.zeros(7 * 3, np.int32)
    w = np.zeros(7)
    opp = np.zeros(7, np.int32)
    cs2 = ct.c_double()
    q = lib.orc_solute_lattice(_enum(lattice, LATTICES), ct.c_double(J0), _ptr(c, ct.c_int),
                               _ptr(w, ct.c_double), _ptr(opp, ct.c_int), ct.byref(cs2))
    return c[:3 * q].reshape(q, 3).copy(), w[:q].copy(), opp[:q].copy(), cs2.value


def feq(lattice, rho, v):
    """Equilibrium of eq:6 at one node."""
    lib = _load()
    out = np.zeros(19)
    v = np.ascontiguousarray(v, np.float64)
    lib.orc_feq(_enum(lattice, LATTICES), ct.c_double(rho), _ptr(v, ct.c_double),
                _ptr(out, ct.c_double))
    return out[:_q({"lattice": lattice})].copy()


def guo(lattice, F, u):
    """Guo forcing term of eq:1.21 at one node."""
    lib = _load()
    out = np.zeros(19)
    F = np.ascontiguousarray(F, np.float64)
    u = np.ascontiguousarray(u, np.float64)
    lib.orc_guo(_enum(lattice, LATTICES), _ptr(F, ct.c_double), _ptr(u, ct.c_double),
                _ptr(out, ct.c_double))
    return out[:_q({"lattice": lattice})].copy()


def set_threads(n):
    """OpenMP threads of the oracle's loops (n <= 0: leave as is); returns the count in effect."""
    lib = _load()
    lib.orc_set_threads.restype = ct.c_int
    return int(lib.orc_set_threads(ct.c_int(int(n))))


def psi(rho, rho0=1.0):
    """Pseudo-potential of eq:1.11."""
    return _load().orc_psi(float(rho), float(rho0))


# ----------------------------------------------------------------------------- geometry
def pinch_fill(p, mask):
    """Reclassify pinched fluid voxels as solid, to a fixed point. Returns (mask, count)."""
    m = np.ascontiguousarray(mask, np.uint8).copy()
    s = _struct(p)
    n = _load().orc_pinch_fill(ct.byref(s), _ptr(m, ct.c_uint8))
    return m, int(n)


def link_masks(p, mask):
    """Per-node bit masks: bit i of flow = upstream n - c_i solid; bit k of solute = wet link."""
    m = np.ascontiguousarray(mask, np.uint8)
    N = n_nodes(p)
    fb = np.zeros(N, np.uint32)
    sb = np.zeros(N, np.uint32)
    s = _struct(p)
    _load().orc_link_masks(ct.byref(s), _ptr(m, ct.c_uint8), _ptr(fb, ct.c_uint32),
                           _ptr(sb, ct.c_uint32))
    return fb, sb


# ----------------------------------------------------------------------------- state
def init(p, mask, rho, u=None, C=None):
    """Equilibrium populations f^eq(rho_s, u), h^eq(C, u) without the force term."""
    N = n_nodes(p)
    nc = int(p.get("ncomp", 2))
    m = np.ascontiguousarray(mask, np.uint8)
    rho = np.ascontiguousarray(rho, np.float64).reshape(nc, N)
    f = np.zeros((nc * _q(p), N))
    h = np.zeros((_qs(p) * max(1, n_species(p)), N))
    up = None if u is None else np.ascontiguousarray(u, np.float64).reshape(3, N)
    Cp = None if C is None else np.ascontiguousarray(C, np.float64).reshape(N)
    s = _struct(p)
    _load().orc_init(ct.byref(s), _ptr(m, ct.c_uint8), _ptr(rho, ct.c_double),
                     None if up is None else _ptr(up, ct.c_double),
                     None if Cp is None else _ptr(Cp, ct.c_double),
                     _ptr(f, ct.c_double), _ptr(h, ct.c_double))
    return f, h


def step(p, mask, f, h, nsteps=1):
    """Advance the state (f, h) in place by nsteps time steps."""
    m = np.ascontiguousarray(mask, np.uint8)
    assert f.dtype == np.float64 and f.flags.c_contiguous
    assert h.dtype == np.float64 and h.flags.c_contiguous
    s = _struct(p)
    _load().orc_step(ct.byref(s), _ptr(m, ct.c_uint8), _ptr(f, ct.c_double),
                     _ptr(h, ct.c_double), ct.c_int64(int(nsteps)))
    return f, h


def deposit(p, mask, f, h, Cps, DP):
    """Particle deposition after a step (sec:particle_deposition,
    eq:surface_deposition): deposits grow at nodes next to a solid, nodes whose
    deposit exceeds 1 turn solid (then the pinch rule again).  mask (uint8),
    f, h and Cps ([N]) are updated in place; returns the nodes made solid."""
    for a, dt in ((mask, np.uint8), (f, np.float64), (h, np.float64), (Cps, np.float64)):
        assert a.dtype == dt and a.flags.c_contiguous
    s = _struct(p)
    lib = _load()
    lib.orc_deposit.restype = ct.c_int64
    return int(lib.orc_deposit(ct.byref(s), _ptr(mask, ct.c_uint8), _ptr(f, ct.c_double), _ptr(h, ct.c_double),
                               _ptr(Cps, ct.c_double), ct.c_double(float(DP))))


def step_deposit(p, mask, f, h, Cps, DP, nsteps):
    """nsteps of (one step, then deposit); returns the nodes made solid."""
    total = 0
    for _ in range(int(nsteps)):
        step(p, mask, f, h, 1)
        total += deposit(p, mask, f, h, Cps, DP)
    return total


def step_nodes(p, mask, f, h, nodes):
    """Populations after one step at the given fluid nodes, from the state at t."""
    m = np.ascontiguousarray(mask, np.uint8)
    nodes = np.ascontiguousarray(nodes, np.int64)
    nc = int(p.get("ncomp", 2))
    fo = np.zeros((len(nodes), nc * _q(p)))
    ho = np.zeros((len(nodes), _qs(p) * max(1, n_species(p))))
    f = np.ascontiguousarray(f, np.float64)
    h = np.ascontiguousarray(h, np.float64)
    s = _struct(p)
    _load().orc_step_nodes(ct.byref(s), _ptr(m, ct.c_uint8), _ptr(f, ct.c_double),
                           _ptr(h, ct.c_double), _ptr(nodes, ct.c_int64),
                           ct.c_int64(len(nodes)), _ptr(fo, ct.c_double), _ptr(ho, ct.c_double))
    return fo, ho


def forces(p, mask, f):
    """Total force F^s (cohesion eq:1.14 + adhesion eq:1.15 + body) as [ncomp][3][N]."""
    N = n_nodes(p)
    nc = int(p.get("ncomp", 2))
    m = np.ascontiguousarray(mask, np.uint8)
    out = np.zeros((nc, 3, N))
    f = np.ascontiguousarray(f, np.float64)
    s = _struct(p)
    _load().orc_forces(ct.byref(s), _ptr(m, ct.c_uint8), _ptr(f, ct.c_double),
                       _ptr(out, ct.c_double))
    return out


def moments(p, mask, f, h):
    """rho_s [ncomp][N], barycentric u with half force [3][N], C [N] (with the
    product species: [2][N], O2 then CO2); solid nodes -> 0."""
    N = n_nodes(p)
    nc = int(p.get("ncomp", 2))
    m = np.ascontiguousarray(mask, np.uint8)
    rho = np.zeros((nc, N))
    u = np.zeros((3, N))
    C = np.zeros((2, N)) if n_species(p) == 2 else np.zeros(N)
    f = np.ascontiguousarray(f, np.float64)
    h = np.ascontiguousarray(h, np.float64)
    s = _struct(p)
    _load().orc_moments(ct.byref(s), _ptr(m, ct.c_uint8), _ptr(f, ct.c_double),
                        _ptr(h, ct.c_double), _ptr(rho, ct.c_double), _ptr(u, ct.c_double),
                        _ptr(C, ct.c_double))
    return rho, u, C


def phase_field(rho):
    """phi = (rho_0 - rho_1)/(rho_0 + rho_1) (0 where both vanish); 1-component: 0."""
    if rho.shape[0] < 2:
        return np.zeros(rho.shape[1:])
    tot = rho[0] + rho[1]
    out = np.zeros_like(tot)
    nz = tot != 0
    out[nz] = (rho[0][nz] - rho[1][nz]) / tot[nz]
    return out


def residual(a_now, a_prev, fluid):
    """||a(t) - a(t-K)||_2 / ||a(t)||_2 over fluid nodes (0/0 -> 0)."""
    a = np.asarray(a_now, np.float64)[..., fluid]
    b = np.asarray(a_prev, np.float64)[..., fluid]
    num = float(np.sum((a - b) ** 2))
    den = float(np.sum(a ** 2))
    if den == 0.0:
        return 0.0 if num == 0.0 else float("inf")
    return (num / den) ** 0.5


# ----------------------------------------------------------------------------- conjugate heat transfer
class _Thermal(ct.Structure):
    _fields_ = [("tau_ef", ct.c_double), ("tau_es", ct.c_double), ("rhocp_f", ct.c_double),
                ("rhocp_s", ct.c_double), ("h_r", ct.c_double), ("A", ct.c_double), ("E_over_R", ct.c_double),
                ("T_tol", ct.c_double), ("T_maxit", ct.c_int32), ("pad_", ct.c_int32)]


THERMAL_KEYS = ("tau_ef", "tau_es", "rhocp_f", "rhocp_s", "h_r", "arr_A", "arr_E_over_R", "T_tol", "T_maxit")


def _thermal(p: dict) -> _Thermal:
    t = _Thermal()
    t.tau_ef = float(p.get("tau_ef", 1.0))
    t.tau_es = float(p.get("tau_es", 1.0))
    t.rhocp_f = float(p.get("rhocp_f", 1.0))
    t.rhocp_s = float(p.get("rhocp_s", 1.0))
    t.h_r = float(p.get("h_r", 0.0))
    t.A = float(p.get("arr_A", 0.0))
    t.E_over_R = float(p.get("arr_E_over_R", 0.0))
    t.T_tol = float(p.get("T_tol", 1e-14))
    t.T_maxit = int(p.get("T_maxit", 100))
    return t


def thermal_nodes(p, mask):
    """(holds_solid, interface) node classes of the conjugate heat transfer:
    solid and interface nodes carry solid energy populations; an interface node is
    a fluid node with a solid flow-lattice neighbour (Reactive LBM subsection)."""
    m = np.ascontiguousarray(mask, np.uint8).reshape(-1)
    N = n_nodes(p)
    hs = np.zeros(N, np.uint8)
    it = np.zeros(N, np.uint8)
    s = _struct(p)
    _load().orc_thermal_nodes(ct.byref(s), _ptr(m, ct.c_uint8), _ptr(hs, ct.c_uint8), _ptr(it, ct.c_uint8))
    return hs, it


def thermal_init(p, mask, T, u=None):
    """Energy populations at temperature T [N]: fluid g^eq(rho_f c_p,f T, u)
    (eq:therpopeq), solid w_i rho_s c_p,s T (eq:therpopeq_solid); returns (g, gs, Ti)."""
    N = n_nodes(p)
    Q = _q(p)
    m = np.ascontiguousarray(mask, np.uint8).reshape(-1)
    T = np.ascontiguousarray(T, np.float64).reshape(N)
    up = None if u is None else np.ascontiguousarray(u, np.float64).reshape(3, N)
    g = np.zeros((Q, N))
    gs = np.zeros((Q, N))
    Ti = np.zeros(N)
    s, t = _struct(p), _thermal(p)
    _load().orc_thermal_init(ct.byref(s), ct.byref(t), _ptr(m, ct.c_uint8), _ptr(T, ct.c_double),
                             None if up is None else _ptr(up, ct.c_double), _ptr(g, ct.c_double),
                             _ptr(gs, ct.c_double), _ptr(Ti, ct.c_double))
    return g, gs, Ti


def step_thermal(p, mask, f, h, g, gs, Ti, nsteps=1):
    """Advance (f, h, g, gs, Ti) in place by nsteps steps with conjugate heat
    transfer; returns (iterations, unsettled interface solves, degenerate
    interface nodes)."""
    m = np.ascontiguousarray(mask, np.uint8)
    for a in (f, h, g, gs, Ti):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    stats = np.zeros(3, np.int64)
    s, t = _struct(p), _thermal(p)
    _load().orc_step_thermal(ct.byref(s), ct.byref(t), _ptr(m, ct.c_uint8), _ptr(f, ct.c_double),
                             _ptr(h, ct.c_double), _ptr(g, ct.c_double), _ptr(gs, ct.c_double),
                             _ptr(Ti, ct.c_double), ct.c_int64(int(nsteps)), _ptr(stats, ct.c_int64))
    return tuple(int(v) for v in stats)


def temperature(p, mask, g, gs):
    """T [N]: fluid (and interface) nodes E_f / (rho c_p)_f, solid nodes E_s / (rho c_p)_s."""
    N = n_nodes(p)
    m = np.ascontiguousarray(mask, np.uint8).reshape(-1)
    T = np.zeros(N)
    s, t = _struct(p), _thermal(p)
    _load().orc_temperature(ct.byref(s), ct.byref(t), _ptr(m, ct.c_uint8), _ptr(g, ct.c_double),
                            _ptr(gs, ct.c_double), _ptr(T, ct.c_double))
    return T
