"""The C oracle against the separately written numpy statement, and geometry pins (no GPU)."""
import numpy as np
import pytest

import oracle
from oracle import np_oracle
from paper_2502_12955_amd import inputs


def _noisy_state(p, mask, seed):
    shape = mask.shape
    nc = p["ncomp"]
    rho, u, C = inputs.random_state_fields(shape, nc, seed, rho_lo=0.3, rho_hi=1.1, u_amp=0.03)
    m, _ = oracle.pinch_fill(p, mask)
    f, h = oracle.init(p, m, rho * (m == 0), u, C * (m == 0))
    rng = inputs.SplitMix64(seed + 99)
    f *= 1.0 + 0.05 * (rng.uniform(f.size).reshape(f.shape) - 0.5)
    h *= 1.0 + 0.05 * (rng.uniform(h.size).reshape(h.shape) - 0.5)
    return m, f, h


CASES = [
    dict(lattice="D2Q9", nx=7, ny=6, nz=1, forcing="guo", solute="periodic", J0=0.4),
    dict(lattice="D2Q9", nx=8, ny=5, nz=1, forcing="sc", solute="inlet_outlet_x", J0=0.4),
    dict(lattice="D3Q19", nx=6, ny=5, nz=4, forcing="guo", solute="inlet_outlet_x"),
    dict(lattice="D3Q19", nx=5, ny=6, nz=4, forcing="sc", solute="periodic"),
    dict(lattice="D3Q19", nx=6, ny=4, nz=5, forcing="guo", solute="off", ncomp=1),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_c_oracle_matches_numpy_statement(case):
    kw = dict(CASES[case])
    nc = kw.pop("ncomp", 2)
    p = inputs.base_params(ncomp=nc, tau=(0.8, 1.3)[:nc] * (2 // nc) if nc == 1 else (0.8, 1.3),
                           G=((0.3, 1.9), (1.9, -0.2)), G_ads=(-0.3, 0.25), rho0=1.2,
                           accel=(2e-4, -1e-4, 5e-5), D=0.15, k_wall=0.05, C_in=0.8, **kw)
    if nc == 1:
        p["tau"] = (0.8, 0.8)
    shape = (p["nz"], p["ny"], p["nx"])
    rng = inputs.SplitMix64(1000 + case)
    mask = (rng.uniform(int(np.prod(shape))) < 0.25).astype(np.uint8).reshape(shape)
    m, f, h = _noisy_state(p, mask, 77 + case)
    assert (m == 0).sum() > 10
    Q = 19 if p["lattice"] == "D3Q19" else 9
    QS = 7 if p["lattice"] == "D3Q19" else 5
    fn = f.reshape((nc, Q) + shape).copy()
    hn = h.reshape((QS,) + shape).copy()
    for _ in range(5):
        oracle.step(p, m, f, h, 1)
        fn, hn = np_oracle.step(p, m, fn, hn)
        scale = np.max(np.abs(f))
        assert np.max(np.abs(f.reshape(fn.shape) - fn)) < 1e-13 * scale
        if p["solute"] != "off":
            assert np.max(np.abs(h.reshape(hn.shape) - hn)) < 1e-13 * max(1.0, np.max(np.abs(h)))


def test_step_nodes_matches_full_step():
    p = inputs.base_params(lattice="D3Q19", nx=7, ny=6, nz=5, G_ads=(-0.2, 0.3),
                           accel=(1e-4, 0, 0), solute="inlet_outlet_x", k_wall=0.02, C_in=1.0)
    shape = (5, 6, 7)
    rng = inputs.SplitMix64(5)
    mask = (rng.uniform(210) < 0.3).astype(np.uint8).reshape(shape)
    m, f, h = _noisy_state(p, mask, 3)
    nodes = np.flatnonzero(m.reshape(-1) == 0)
    fo, ho = oracle.step_nodes(p, m, f, h, nodes)
    oracle.step(p, m, f, h, 1)
    assert np.max(np.abs(fo.T - f[:, nodes])) < 1e-15
    assert np.max(np.abs(ho.T - h[:, nodes])) < 1e-15


# ----------------------------------------------------------------------------- geometry
def test_pinch_fill_hand_example():
    """Fluid voxels with solid on both sides along an axis become solid, to a fixed point."""
    p = inputs.base_params(lattice="D2Q9", nx=7, ny=5, nz=1)
    mask = np.zeros((1, 5, 7), np.uint8)
    mask[0, 2, 1] = 1
    mask[0, 2, 3] = 1          # x = 2 pinched along x -> solid
    mask[0, 0, 5] = 1
    mask[0, 2, 5] = 1          # (5, 1) pinched along y; (4, 2) pinched along x
    out, n = oracle.pinch_fill(p, mask)
    want = mask.copy()
    want[0, 2, 2] = 1
    want[0, 2, 4] = 1
    want[0, 1, 5] = 1
    assert n == 3 and np.array_equal(out, want)


def test_pinch_fill_cascades_and_seams():
    p = inputs.base_params(lattice="D2Q9", nx=6, ny=3, nz=1, solute="inlet_outlet_x")
    mask = np.zeros((1, 3, 6), np.uint8)
    mask[0, 1, 1] = 1          # x = 0 between the inlet seam and a solid -> solid
    out, n = oracle.pinch_fill(p, mask)
    assert out[0, 1, 0] == 1 and n == 1
    p2 = dict(p, solute="periodic")
    out2, n2 = oracle.pinch_fill(p2, mask)
    assert n2 == 0             # periodic: x = 0 has fluid at x = 5
    # a 1-wide corridor closed at one end fills up completely
    p3 = inputs.base_params(lattice="D2Q9", nx=8, ny=3, nz=1)
    m3 = np.zeros((1, 3, 8), np.uint8)
    m3[0, 0, :] = 1
    m3[0, 2, :] = 1
    out3, n3 = oracle.pinch_fill(p3, m3)
    assert n3 == 8 and out3.all()


def test_pinch_fill_is_order_independent_fixed_point():
    p = inputs.base_params(lattice="D3Q19", nx=12, ny=10, nz=9)
    rng = inputs.SplitMix64(12)
    mask = (rng.uniform(1080) < 0.45).astype(np.uint8).reshape(9, 10, 12)
    out, n = oracle.pinch_fill(p, mask)
    again, n2 = oracle.pinch_fill(p, out)
    assert n2 == 0 and np.array_equal(out, again)
    assert np.all(out >= mask) and n == int(out.sum() - mask.sum())
    # sequential in-place sweep (Gauss-Seidel order) reaches the same least fixed point
    m = mask.copy()
    changed = True
    while changed:
        changed = False
        for z in range(9):
            for y in range(10):
                for x in range(12):
                    if m[z, y, x]:
                        continue
                    for d in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
                        a = m[(z + d[2]) % 9, (y + d[1]) % 10, (x + d[0]) % 12]
                        b = m[(z - d[2]) % 9, (y - d[1]) % 10, (x - d[0]) % 12]
                        if a and b:
                            m[z, y, x] = 1
                            changed = True
                            break
    assert np.array_equal(m, out)


def test_link_masks_definition():
    p = inputs.base_params(lattice="D3Q19", nx=5, ny=5, nz=5, solute="inlet_outlet_x")
    mask = np.zeros((5, 5, 5), np.uint8)
    mask[2, 2, 2] = 1
    fb, sb = oracle.link_masks(p, mask)
    c, _, _ = oracle.flow_lattice("D3Q19")
    fb = fb.reshape(5, 5, 5)
    # node (3,2,2): upstream along c_i = (1,0,0) (i = 1) is the solid voxel
    assert fb[2, 2, 3] == (1 << 1)
    # node (3,3,2): upstream along (1,1,0) (i = 7)
    assert fb[2, 3, 3] == (1 << 7)
    assert sb.reshape(5, 5, 5)[2, 2, 3] == (1 << 1)
    assert sb.reshape(5, 5, 5)[2, 3, 3] == 0
    assert fb[2, 2, 2] == 0
    # seam: no wet link across x = 0 / x = nx-1 even if the wrapped node is solid
    m2 = np.zeros((1, 1, 5), np.uint8)
    m2[0, 0, 4] = 1
    p2 = inputs.base_params(lattice="D3Q19", nx=5, ny=1, nz=1, solute="inlet_outlet_x")
    _, sb2 = oracle.link_masks(p2, m2)
    assert sb2[0] == 0 and sb2[3] == (1 << 2)
