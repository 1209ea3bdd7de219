"""Thin ctypes binding of ``libmclbm.so`` (contract in ``include/mclbm.h``).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch provides the device arena (a uint8 CUDA tensor) and the stream; numpy
arrays carry host data.  There is no fallback: if the library is missing or
fails to load, ``load()`` raises.

The functions mirror the C names without the ``mclbm_`` prefix; ``Lattice``
bundles a handle with its arena.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmclbm.so")

OK, EINVAL, ENOMEM, EHIP, ESTATE, EDIVERGED = 0, -1, -2, -3, -4, -5
D2Q9, D3Q19 = 0, 1
FORCING = {"guo": 0, "sc": 1}
SOLUTE = {"off": 0, "periodic": 1, "inlet_outlet_x": 2}
STORAGE = {"f64": 0, "f32": 1, "f16s": 2, "bf16s": 3}
LATTICE = {"D2Q9": 0, "D3Q19": 1}
STORE_DTYPE = {0: np.float64, 1: np.float32, 2: np.uint16, 3: np.uint16}


class MclbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mclbm error {code}: {msg}")
        self.code = code


class Params(ct.Structure):
    _fields_ = [("lattice", ct.c_int32), ("nx", ct.c_int32), ("ny", ct.c_int32), ("nz", ct.c_int32),
                ("ncomp", ct.c_int32), ("forcing", ct.c_int32), ("solute", ct.c_int32),
                ("storage", ct.c_int32), ("monitor_every", ct.c_int32), ("reserved", ct.c_int32),
                ("tau", ct.c_double * 2), ("G", (ct.c_double * 2) * 2), ("G_ads", ct.c_double * 2),
                ("rho0", ct.c_double), ("accel", ct.c_double * 3), ("D", ct.c_double),
                ("J0", ct.c_double), ("k_wall", ct.c_double), ("C_in", ct.c_double),
                ("product", ct.c_int32), ("rate_field", ct.c_int32), ("D2", ct.c_double), ("C_in2", ct.c_double),
                ("deposition", ct.c_int32), ("reserved2", ct.c_int32), ("dep_prob", ct.c_double)]


class ThermalParams(ct.Structure):
    """mclbm_thermal: conjugate heat transfer parameters."""
    _fields_ = [("tau_ef", ct.c_double), ("tau_es", ct.c_double), ("rhocp_f", ct.c_double),
                ("rhocp_s", ct.c_double), ("h_r", ct.c_double), ("A", ct.c_double), ("E_over_R", ct.c_double),
                ("T_tol", ct.c_double), ("T_maxit", ct.c_int32), ("reserved", ct.c_int32)]


def thermal_from_dict(p: dict) -> ThermalParams:
    """Keys as the oracle's: tau_ef, tau_es, rhocp_f, rhocp_s, h_r, arr_A, arr_E_over_R, T_tol, T_maxit."""
    t = ThermalParams()
    t.tau_ef = float(p.get("tau_ef", 1.0))
    t.tau_es = float(p.get("tau_es", 1.0))
    t.rhocp_f = float(p.get("rhocp_f", 1.0))
    t.rhocp_s = float(p.get("rhocp_s", 1.0))
    t.h_r = float(p.get("h_r", 0.0))
    t.A = float(p.get("arr_A", 0.0))
    t.E_over_R = float(p.get("arr_E_over_R", 0.0))
    t.T_tol = float(p.get("T_tol", 1e-14))
    t.T_maxit = int(p.get("T_maxit", 100))
    t.reserved = 0
    return t


def _enum(v, table):
    return table[v] if isinstance(v, str) else int(v)


def params_from_dict(p: dict) -> Params:
    s = Params()
    s.lattice = _enum(p["lattice"], LATTICE)
    s.nx, s.ny, s.nz = int(p["nx"]), int(p["ny"]), int(p.get("nz", 1))
    s.ncomp = int(p.get("ncomp", 2))
    s.forcing = _enum(p.get("forcing", "guo"), FORCING)
    s.solute = _enum(p.get("solute", "off"), SOLUTE)
    s.storage = _enum(p.get("storage", "f64"), STORAGE)
    s.monitor_every = int(p.get("monitor_every", 100))
    s.reserved = 0
    tau = p.get("tau", (1.0, 1.0))
    s.tau[0] = float(tau[0])
    s.tau[1] = float(tau[1] if len(tau) > 1 else tau[0])
    G = p.get("G", ((0.0, 0.0), (0.0, 0.0)))
    for a in range(2):
        for b in range(2):
            s.G[a][b] = float(G[a][b])
    ga = p.get("G_ads", (0.0, 0.0))
    s.G_ads[0], s.G_ads[1] = float(ga[0]), float(ga[1])
    s.rho0 = float(p.get("rho0", 1.0))
    for a, v in enumerate(p.get("accel", (0.0, 0.0, 0.0))):
        s.accel[a] = float(v)
    s.D = float(p.get("D", 0.1))
    s.J0 = float(p.get("J0", 0.1))
    s.k_wall = float(p.get("k_wall", 0.0))
    s.C_in = float(p.get("C_in", 0.0))
    s.product = int(p.get("product", 0))
    s.rate_field = int(p.get("rate_field", 0))
    s.D2 = float(p.get("D2", 0.1))
    s.C_in2 = float(p.get("C_in2", 0.0))
    s.deposition = int(p.get("deposition", 0))
    s.reserved2 = 0
    s.dep_prob = float(p.get("dep_prob", 0.0))
    return s


def n_species(p: dict) -> int:
    """Solute species carried: 0 (solute off), 1, or 2 with the product."""
    if _enum(p.get("solute", "off"), SOLUTE) == 0:
        return 0
    return 2 if int(p.get("product", 0)) else 1


_lib = None

EXPORTS = ("mclbm_required_bytes", "mclbm_init_lattice", "mclbm_set_geometry", "mclbm_get_geometry",
           "mclbm_init_fields", "mclbm_step", "mclbm_get_moments", "mclbm_get_monitors",
           "mclbm_monitor_now", "mclbm_get_populations", "mclbm_set_populations",
           "mclbm_population_bytes", "mclbm_run_to_residual", "mclbm_set_launch", "mclbm_set_bands", "mclbm_set_graph",
           "mclbm_required_bytes_batch", "mclbm_init_batch", "mclbm_get_sample_monitors", "mclbm_get_step",
           "mclbm_synchronize", "mclbm_autotune", "mclbm_set_wall_rate", "mclbm_get_deposit", "mclbm_set_deposit", "mclbm_destroy",
           "mclbm_last_error", "mclbm_hbm_probe", "mclbm_set_addressing", "mclbm_set_thermal",
           "mclbm_init_temperature", "mclbm_get_temperature", "mclbm_get_thermal_populations",
           "mclbm_get_thermal_stats")


def load(path: str = LIB_PATH):
    """Load the HIP library; raises if it is not built or cannot be loaded."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2502_12955_amd/build.py")
    lib = ct.CDLL(path)
    vp, i32, i64, dbl, sz = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_double, ct.c_size_t
    P = ct.POINTER(Params)
    lib.mclbm_required_bytes.argtypes = [P, ct.POINTER(sz)]
    lib.mclbm_init_lattice.argtypes = [P, vp, sz, vp, ct.POINTER(vp)]
    lib.mclbm_set_geometry.argtypes = [vp, vp, ct.POINTER(i64)]
    lib.mclbm_set_wall_rate.argtypes = [vp, vp]
    lib.mclbm_get_deposit.argtypes = [vp, vp, ct.POINTER(i64)]
    lib.mclbm_set_deposit.argtypes = [vp, vp, i64]
    lib.mclbm_get_geometry.argtypes = [vp, vp, vp, vp]
    lib.mclbm_init_fields.argtypes = [vp, vp, vp, vp]
    lib.mclbm_step.argtypes = [vp, i64]
    lib.mclbm_get_moments.argtypes = [vp, vp, vp, vp, i32]
    lib.mclbm_get_monitors.argtypes = [vp, vp]
    lib.mclbm_monitor_now.argtypes = [vp]
    lib.mclbm_get_populations.argtypes = [vp, vp, i32]
    lib.mclbm_set_populations.argtypes = [vp, vp, i32]
    lib.mclbm_population_bytes.argtypes = [vp, i32, ct.POINTER(sz)]
    lib.mclbm_run_to_residual.argtypes = [vp, dbl, i64, ct.POINTER(i64)]
    lib.mclbm_set_launch.argtypes = [vp, i32, i32]
    lib.mclbm_set_bands.argtypes = [vp, i32]
    lib.mclbm_set_graph.argtypes = [vp, i32]
    lib.mclbm_set_addressing.argtypes = [vp, i32]
    lib.mclbm_set_thermal.argtypes = [vp, ct.POINTER(ThermalParams)]
    lib.mclbm_init_temperature.argtypes = [vp, vp, vp]
    lib.mclbm_get_temperature.argtypes = [vp, vp]
    lib.mclbm_get_thermal_populations.argtypes = [vp, vp, vp]
    lib.mclbm_get_thermal_stats.argtypes = [vp, vp]
    lib.mclbm_required_bytes_batch.argtypes = [P, i32, ct.POINTER(sz)]
    lib.mclbm_init_batch.argtypes = [P, i32, vp, sz, vp, ct.POINTER(vp)]
    lib.mclbm_get_sample_monitors.argtypes = [vp, i32, vp]
    lib.mclbm_get_step.argtypes = [vp, ct.POINTER(i64)]
    lib.mclbm_synchronize.argtypes = [vp]
    lib.mclbm_autotune.argtypes = [vp, i32, ct.POINTER(i32), ct.POINTER(i32), ct.POINTER(i32), ct.POINTER(dbl), vp,
                                   i32, ct.POINTER(i32)]
    lib.mclbm_hbm_probe.argtypes = [i32, vp, vp, sz, i32, i32, vp, ct.POINTER(dbl)]
    lib.mclbm_destroy.argtypes = [vp]
    lib.mclbm_destroy.restype = None
    lib.mclbm_last_error.argtypes = [vp]
    lib.mclbm_last_error.restype = ct.c_char_p
    for name in EXPORTS:
        if name not in ("mclbm_destroy", "mclbm_last_error"):
            getattr(lib, name).restype = ct.c_int
    _lib = lib
    return lib


def hbm_probe(kind: str, nbytes: int = 2 << 30, blocks_per_cu: int = 8, iters: int = 5) -> float:
    """Best GB/s of the library's streaming read / write / copy kernel over
    ``nbytes`` (device buffers allocated here with torch)."""
    import torch

    k = {"read": 0, "write": 1, "copy": 2}[kind]
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty(nbytes // 4 if k == 2 else 4096, dtype=torch.float32, device="cuda")
    out = ct.c_double()
    stream = ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    _check(load().mclbm_hbm_probe(k, ct.c_void_p(a.data_ptr()), ct.c_void_p(b.data_ptr()), nbytes, blocks_per_cu,
                                  iters, stream, ct.byref(out)))
    del a, b
    return out.value


def last_error(handle=None) -> str:
    return load().mclbm_last_error(handle).decode()


def _check(rc, handle=None, allow=(OK,)):
    if rc not in allow:
        raise MclbmError(rc, last_error(handle))
    return rc


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def required_bytes(p: dict) -> int:
    n = ct.c_size_t()
    s = params_from_dict(p)
    _check(load().mclbm_required_bytes(ct.byref(s), ct.byref(n)))
    return n.value


def init_lattice(p: dict, arena_ptr, arena_bytes: int, stream_ptr):
    s = params_from_dict(p)
    h = ct.c_void_p()
    _check(load().mclbm_init_lattice(ct.byref(s), arena_ptr, arena_bytes, stream_ptr, ct.byref(h)))
    return h


def set_geometry(h, mask) -> int:
    m = np.ascontiguousarray(mask, np.uint8)
    n = ct.c_int64()
    _check(load().mclbm_set_geometry(h, _ptr(m), ct.byref(n)), h)
    return n.value


def get_geometry(h, N):
    mask = np.zeros(N, np.uint8)
    fb = np.zeros(N, np.uint32)
    sb = np.zeros(N, np.uint32)
    _check(load().mclbm_get_geometry(h, _ptr(mask), _ptr(fb), _ptr(sb)), h)
    return mask, fb, sb


def init_fields(h, rho, u=None, C=None):
    r = np.ascontiguousarray(rho, np.float64)
    uu = None if u is None else np.ascontiguousarray(u, np.float64)
    cc = None if C is None else np.ascontiguousarray(C, np.float64)
    _check(load().mclbm_init_fields(h, _ptr(r), _ptr(uu), _ptr(cc)), h)


def step(h, n: int, allow_diverged=False):
    allow = (OK, EDIVERGED) if allow_diverged else (OK,)
    return _check(load().mclbm_step(h, int(n)), h, allow)


def set_wall_rate(h, k_box):
    """Per-node reaction rate [N] (box nodes; needs rate_field=1 and set_geometry first)."""
    k = np.ascontiguousarray(k_box, np.float64).reshape(-1)
    _check(load().mclbm_set_wall_rate(h, _ptr(k)), h)


def get_deposit(h, N):
    """Particle deposit C_ps per box node [N] (eq:surface_deposition; 0 on solid
    nodes) and the number of nodes deposition has turned solid."""
    Cps = np.zeros(N)
    n = ct.c_int64()
    _check(load().mclbm_get_deposit(h, _ptr(Cps), ct.byref(n)), h)
    return Cps, n.value


def set_deposit(h, Cps, converted=0):
    """Restore the deposits [N] (box nodes) and the converted-node count."""
    d = np.ascontiguousarray(Cps, np.float64).reshape(-1)
    _check(load().mclbm_set_deposit(h, _ptr(d), int(converted)), h)


def get_moments(h, ncomp, N, nspecies=1):
    """rho [ncomp][N], u [3][N], C [N] (or [2][N] with the product species)."""
    rho = np.zeros((ncomp, N))
    u = np.zeros((3, N))
    C = np.zeros((2, N)) if nspecies == 2 else np.zeros(N)
    _check(load().mclbm_get_moments(h, _ptr(rho), _ptr(u), _ptr(C), 0), h)
    return rho, u, C


def get_moments_device(h, rho_ptr, u_ptr, C_ptr):
    _check(load().mclbm_get_moments(h, rho_ptr, u_ptr, C_ptr, 1), h)


def get_monitors(h):
    out = np.zeros(16)
    _check(load().mclbm_get_monitors(h, _ptr(out)), h)
    return out


def monitor_now(h, allow_diverged=False):
    allow = (OK, EDIVERGED) if allow_diverged else (OK,)
    return _check(load().mclbm_monitor_now(h), h, allow)


def population_bytes(h, raw: bool) -> int:
    n = ct.c_size_t()
    _check(load().mclbm_population_bytes(h, int(bool(raw)), ct.byref(n)), h)
    return n.value


def get_populations(h, raw=False, storage="f64"):
    nb = population_bytes(h, raw)
    dt = np.dtype(STORE_DTYPE[_enum(storage, STORAGE)]) if raw else np.dtype(np.float64)
    out = np.zeros(nb // dt.itemsize, dt)
    _check(load().mclbm_get_populations(h, _ptr(out), int(bool(raw))), h)
    return out


def set_populations(h, src, raw=False):
    a = np.ascontiguousarray(src)
    if not raw:
        a = np.ascontiguousarray(a, np.float64)
    if a.nbytes != population_bytes(h, raw):
        raise ValueError("population array has the wrong size")
    _check(load().mclbm_set_populations(h, _ptr(a), int(bool(raw))), h)


def run_to_residual(h, tol: float, max_steps: int, allow_diverged=False):
    """Returns (every sample converged, steps taken).  With allow_diverged, a
    batch in which some sample went non-finite returns (False, steps) instead
    of raising; the sample monitors say which (out[13] >= 0)."""
    n = ct.c_int64()
    allow = (OK, 1, EDIVERGED) if allow_diverged else (OK, 1)
    rc = _check(load().mclbm_run_to_residual(h, float(tol), int(max_steps), ct.byref(n)), h, allow)
    return rc == OK, n.value


def set_launch(h, block_threads=256, grid_blocks=0):
    _check(load().mclbm_set_launch(h, int(block_threads), int(grid_blocks)), h)


def set_bands(h, bands=0):
    _check(load().mclbm_set_bands(h, int(bands)), h)


def set_addressing(h, flat: bool):
    _check(load().mclbm_set_addressing(h, int(bool(flat))), h)


def autotune(h, trial_steps=20):
    """Native tuner of the numbering and launch shape; returns (bands, block, grid,
    ms_per_step, table rows (bands, block, grid, ms))."""
    nb, b, g, n = ct.c_int32(), ct.c_int32(), ct.c_int32(), ct.c_int32()
    ms = ct.c_double()
    table = np.zeros((128, 4))
    _check(load().mclbm_autotune(h, int(trial_steps), ct.byref(nb), ct.byref(b), ct.byref(g), ct.byref(ms),
                                 _ptr(table), 128, ct.byref(n)), h)
    return nb.value, b.value, g.value, ms.value, table[: n.value].tolist()


def tune_key(plist):
    """Cache key of a launch-shape choice: physics class and box-node size class (powers of 2)."""
    p = plist[0]
    nodes = sum(int(q["nx"]) * int(q["ny"]) * int(q.get("nz", 1)) for q in plist)
    return (f"{p.get('lattice', 'D3Q19')}-{p.get('storage', 'f64')}-nc{p.get('ncomp', 2)}-"
            f"{p.get('solute', 'off')}-{p.get('forcing', 'guo')}-n2^{int(round(np.log2(max(nodes, 1))))}")


def set_graph(h, enable=True):
    _check(load().mclbm_set_graph(h, int(bool(enable))), h)


def required_bytes_batch(plist) -> int:
    arr = (Params * len(plist))(*[params_from_dict(p) for p in plist])
    n = ct.c_size_t()
    _check(load().mclbm_required_bytes_batch(arr, len(plist), ct.byref(n)))
    return n.value


def init_batch(plist, arena_ptr, arena_bytes, stream_ptr):
    arr = (Params * len(plist))(*[params_from_dict(p) for p in plist])
    h = ct.c_void_p()
    _check(load().mclbm_init_batch(arr, len(plist), arena_ptr, arena_bytes, stream_ptr, ct.byref(h)))
    return h


def get_sample_monitors(h, s):
    out = np.zeros(16)
    _check(load().mclbm_get_sample_monitors(h, int(s), _ptr(out)), h)
    return out


def get_step(h) -> int:
    n = ct.c_int64()
    _check(load().mclbm_get_step(h, ct.byref(n)), h)
    return n.value


def synchronize(h):
    _check(load().mclbm_synchronize(h), h)


def destroy(h):
    if h:
        load().mclbm_destroy(h)


class Lattice:
    """A solver handle plus the torch device arena it lives in.

    ``stream``: a torch.cuda.Stream (default: the current stream).  All work is
    queued on it.
    """

    def __init__(self, params: dict, device="cuda:0", stream=None):
        import torch

        load()
        self.params = dict(params)
        self.N = int(params["nx"]) * int(params["ny"]) * int(params.get("nz", 1))
        self.ncomp = int(params.get("ncomp", 2))
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = required_bytes(params)
        self.arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.arena.data_ptr()
        aligned = (base + 255) & ~255
        self.h = init_lattice(params, ct.c_void_p(aligned), nbytes, ct.c_void_p(self.stream.cuda_stream))

    def close(self):
        if getattr(self, "h", None):
            destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_geometry(self, mask):
        return set_geometry(self.h, np.asarray(mask).reshape(-1))

    def get_geometry(self):
        return get_geometry(self.h, self.N)

    def init_fields(self, rho, u=None, C=None):
        init_fields(self.h, np.asarray(rho).reshape(self.ncomp, self.N),
                    None if u is None else np.asarray(u).reshape(3, self.N),
                    None if C is None else np.asarray(C).reshape(self.N))

    def set_wall_rate(self, k_box):
        set_wall_rate(self.h, np.asarray(k_box).reshape(self.N))

    def get_deposit(self):
        return get_deposit(self.h, self.N)

    def set_deposit(self, Cps, converted=0):
        set_deposit(self.h, np.asarray(Cps).reshape(self.N), converted)

    def step(self, n=1, allow_diverged=False):
        return step(self.h, n, allow_diverged)

    def moments(self):
        return get_moments(self.h, self.ncomp, self.N, n_species(self.params))

    def monitors(self):
        return get_monitors(self.h)

    def monitor_now(self, allow_diverged=False):
        return monitor_now(self.h, allow_diverged)

    def populations(self, raw=False):
        return get_populations(self.h, raw, self.params.get("storage", "f64"))

    def set_populations(self, src, raw=False):
        set_populations(self.h, src, raw)

    def run_to_residual(self, tol, max_steps, allow_diverged=False):
        return run_to_residual(self.h, tol, max_steps, allow_diverged)

    def set_launch(self, block_threads=256, grid_blocks=0):
        set_launch(self.h, block_threads, grid_blocks)

    def set_bands(self, bands=0):
        set_bands(self.h, bands)

    def set_graph(self, enable=True):
        set_graph(self.h, enable)

    def set_addressing(self, flat=False):
        set_addressing(self.h, flat)

    # conjugate heat transfer
    def set_thermal(self, p: dict):
        t = thermal_from_dict(p)
        _check(load().mclbm_set_thermal(self.h, ct.byref(t)), self.h)

    def init_temperature(self, T, u=None):
        T = np.ascontiguousarray(np.asarray(T, np.float64).reshape(self.N))
        up = None if u is None else np.ascontiguousarray(np.asarray(u, np.float64).reshape(3, self.N))
        _check(load().mclbm_init_temperature(self.h, _ptr(T), _ptr(up)), self.h)

    def temperature(self):
        T = np.zeros(self.N)
        _check(load().mclbm_get_temperature(self.h, _ptr(T)), self.h)
        return T

    def thermal_populations(self):
        q = 19 if _enum(self.params["lattice"], LATTICE) == 1 else 9
        g = np.zeros((q, self.N))
        gs = np.zeros((q, self.N))
        _check(load().mclbm_get_thermal_populations(self.h, _ptr(g), _ptr(gs)), self.h)
        return g, gs

    def thermal_stats(self):
        out = np.zeros(3, np.int64)
        _check(load().mclbm_get_thermal_stats(self.h, _ptr(out)), self.h)
        return tuple(int(v) for v in out)



    def autotune(self, trial_steps=20, cache_path=None):
        """Choose the band count of the numbering and the launch shape (after
        set_geometry; init_fields must follow).

        With ``cache_path`` (a JSON file), a choice already made for the same
        physics and size class is reused without timing, and new choices are
        added to the file.  Returns (bands, block, grid, ms_per_step or None if
        cached)."""
        import json

        key = tune_key(getattr(self, "plist", [self.params]))
        cache = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
        if key in cache:
            nb, b, g = cache[key]["bands"], cache[key]["block"], cache[key]["grid"]
            self.set_bands(nb)
            self.set_launch(b, g)
            return nb, b, g, None
        nb, b, g, ms, table = autotune(self.h, trial_steps)
        if cache_path:
            cache[key] = dict(bands=nb, block=b, grid=g, ms_per_step=ms, table=table)
            with open(cache_path, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
        return nb, b, g, ms

    @property
    def step_count(self):
        return get_step(self.h)

    def synchronize(self):
        synchronize(self.h)


class Batch(Lattice):
    """A batch of independent samples sharing the physics (dimensions may differ).

    Host arrays are per-sample arrays concatenated in sample order; the helpers
    ``concat``/``split`` convert between lists of per-sample arrays and that layout.
    """

    def __init__(self, plist, device="cuda:0", stream=None):
        import torch

        load()
        self.plist = [dict(p) for p in plist]
        self.params = dict(plist[0])
        self.sizes = [int(p["nx"]) * int(p["ny"]) * int(p.get("nz", 1)) for p in plist]
        self.N = sum(self.sizes)
        self.ncomp = int(plist[0].get("ncomp", 2))
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = required_bytes_batch(self.plist)
        self.arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.arena.data_ptr() + 255) & ~255
        self.h = init_batch(self.plist, ct.c_void_p(aligned), nbytes, ct.c_void_p(self.stream.cuda_stream))

    def concat(self, per_sample, fields):
        """List of arrays [fields][N_s] (any shape with N_s trailing values) -> flat batch array."""
        return np.concatenate([np.asarray(a, np.float64).reshape(fields, n).ravel()
                               for a, n in zip(per_sample, self.sizes)])

    def split(self, flat, fields):
        out, off = [], 0
        for n in self.sizes:
            out.append(np.asarray(flat[off:off + fields * n]).reshape(fields, n))
            off += fields * n
        return out

    def set_geometry(self, masks):
        flat = np.concatenate([np.asarray(m, np.uint8).reshape(-1) for m in masks])
        return set_geometry(self.h, flat)

    def init_fields(self, rhos, us=None, Cs=None):
        init_fields(self.h, self.concat(rhos, self.ncomp),
                    None if us is None else self.concat(us, 3),
                    None if Cs is None else self.concat(Cs, 1))

    def moments(self):
        rho = np.zeros(self.ncomp * self.N)
        u = np.zeros(3 * self.N)
        nsp = max(1, n_species(self.plist[0]))
        C = np.zeros(nsp * self.N)
        _check(load().mclbm_get_moments(self.h, _ptr(rho), _ptr(u), _ptr(C), 0), self.h)
        return self.split(rho, self.ncomp), self.split(u, 3), self.split(C, nsp)

    def sample_monitors(self, s):
        return get_sample_monitors(self.h, s)
