"""GPU: reduced-precision population storage (FP16 / BF16 weight-shifted deviations,
FP32 arithmetic) against the FP64 oracle, through the C ABI.

* Encoder, bit for bit: FP64 populations written with set_populations are stored
  by the step kernels' own store (round to FP32, subtract the shift w_i rhobar_s in
  FP32, round to nearest even into the 16-bit format).  The stored bits must equal
  torch's round-to-nearest-even conversion of the same FP32 deviation, over ties,
  FP16 and BF16 subnormals, overflow and +-Inf (NaN stays NaN).
* One step, element by element: from the same 16-bit representable state the
  stored result of a step may differ from the FP64 oracle's step by at most half a
  unit in the last place of the 16-bit deviation (11-bit significand for FP16, 8-bit
  for BF16) plus the FP32 arithmetic of the step and of the decode.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2502_12955_amd import inputs

from helpers import gpu_lattice, small_porous, split_pops

pytestmark = pytest.mark.gpu

TORCH_DT = {"f16s": torch.float16, "bf16s": torch.bfloat16}
WN19 = np.array([12, 2, 2, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1], np.float32)


def _bits(x32, storage):
    """torch's round-to-nearest-even FP32 -> 16-bit conversion, as raw bits."""
    t = torch.from_numpy(np.ascontiguousarray(x32, np.float32)).to(TORCH_DT[storage])
    return t.view(torch.int16).numpy().view(np.uint16)


def _decode(bits, storage):
    t = torch.from_numpy(bits.view(np.int16).copy()).view(TORCH_DT[storage])
    return t.to(torch.float32).numpy()


def _ulp16(x, storage):
    """Spacing of the 16-bit format at |x| (the subnormal spacing below the
    smallest normal)."""
    ax = np.abs(np.asarray(x, np.float64))
    mant, emin = (10, -14) if storage == "f16s" else (7, -126)
    e = np.floor(np.log2(np.maximum(ax, 2.0 ** emin)))
    return 2.0 ** (e - mant)


def _special_deviations(storage, rng):
    """Deviations (FP32 values) that exercise the encoder: exact ties between two
    neighbouring 16-bit numbers (normal and subnormal), values just off a tie,
    random values over many binades, zeros of both signs."""
    mant, emin = (10, -14) if storage == "f16s" else (7, -126)
    out = [0.0, -0.0]
    # ties and near-ties in the normal range, exponents from 2^-14 to 2^-7
    for e in range(-14, -6):
        for m in rng.integers(0, 2 ** mant, 12):
            a = (1.0 + m / 2.0 ** mant) * 2.0 ** e
            tie = a + 2.0 ** (e - mant - 1)
            for v in (tie, -tie, tie + 2.0 ** (e - mant - 8), tie - 2.0 ** (e - mant - 8)):
                out.append(v)
    # FP16 subnormals (spacing 2^-24) and their ties; BF16 needs FP32 subnormals,
    # which only unshifted (solute) planes can carry
    if storage == "f16s":
        for m in rng.integers(1, 2 ** 10, 24):
            out += [m * 2.0 ** -24, (m + 0.5) * 2.0 ** -24, -(m + 0.5) * 2.0 ** -24]
    out += list(rng.standard_normal(64) * 10.0 ** rng.uniform(-6, -2, 64))
    return np.array(out, np.float64)


@pytest.mark.parametrize("storage", ["f16s", "bf16s"])
def test_encoder_is_round_to_nearest_even_bit_for_bit(storage):
    nx, ny, nz = 8, 8, 6
    rng = np.random.default_rng(12955)
    p = inputs.base_params(lattice="D3Q19", nx=nx, ny=ny, nz=nz, ncomp=2, solute="periodic",
                           storage=storage, D=0.1, J0=0.1)
    N = nx * ny * nz
    mask = np.zeros((nz, ny, nx), np.uint8)
    rhobar = (0.75, 0.125)                          # uniform: the shift is exactly w_i rhobar_s
    rho = np.stack([np.full((nz, ny, nx), r) for r in rhobar])
    lat = gpu_lattice(p, mask, rho, None, np.zeros((nz, ny, nx)))
    Q, QS = 19, 7
    shift = np.zeros((2 * Q + QS,), np.float32)
    for s in range(2):
        shift[s * Q:(s + 1) * Q] = (WN19 / np.float32(36.0)) * np.float32(rhobar[s])
    vals = np.zeros((2 * Q + QS, N))
    dev = _special_deviations(storage, rng)
    for j in range(2 * Q):
        d = np.resize(np.roll(dev, 7 * j), N)
        vals[j] = (np.float64(shift[j]) + d).astype(np.float32).astype(np.float64)
    sol = list(_special_deviations(storage, rng))
    sol += [np.inf, -np.inf, np.nan, 7.0e4, -7.0e4, 65519.0, 65520.0, 1.0e-39, -3.0e-40,
            2.0 ** -130 * 3, 2.0 ** -133, 1.0e-45]
    for k in range(QS):
        vals[2 * Q + k] = np.resize(np.roll(np.array(sol), 5 * k), N)
    lat.set_populations(vals.ravel())
    got = lat.populations(raw=True).reshape(2 * Q + QS, N)
    x32 = vals.astype(np.float32) - shift[:, None]          # FP32 value, then FP32 shift
    want = _bits(x32, storage)
    nan = np.isnan(x32)
    assert np.array_equal(got[~nan], want[~nan])
    assert np.all(np.isnan(_decode(got[nan], storage)))
    # the cases were really hit: ties, subnormal results, overflow to Inf
    dec = _decode(got, storage).astype(np.float64)
    tiny = 2.0 ** (-14 if storage == "f16s" else -126)
    assert np.sum((np.abs(dec) < tiny) & (dec != 0)) > 10
    assert np.sum(np.isinf(dec)) >= (4 if storage == "f16s" else 2)
    lat.close()


@pytest.mark.parametrize("storage", ["f16s", "bf16s"])
@pytest.mark.parametrize("forcing", ["guo", "sc"])
def test_one_step_within_the_format_bound(storage, forcing):
    p, mask, rho, u, C = small_porous(storage=storage, forcing=forcing, k_wall=0.05, C_in=1.0,
                                      tau=(0.9, 1.3) if forcing == "sc" else (1.0, 1.0))
    lat = gpu_lattice(p, mask, rho, u, C)
    lat.step(5)
    state = lat.populations()
    f0, h0 = split_pops(p, state)
    m, _ = oracle.pinch_fill(p, mask)
    fo, ho = f0.copy(), h0.copy()
    oracle.step(p, m, fo, ho, 1)                   # FP64 step of the decoded 16-bit state
    lat.step(1)
    fg, hg = split_pops(p, lat.populations())
    fluid = m.reshape(-1) == 0
    rb = np.array([rho[s][m == 0].mean() for s in range(2)])
    sh = np.zeros((38, 1))
    for s in range(2):
        sh[s * 19:(s + 1) * 19, 0] = (WN19 / np.float32(36.0)) * np.float32(rb[s])
    scale = np.abs(fo[:, fluid]).max()
    # FP32 arithmetic of the step (as in the FP32 parity test) and of the decode
    a32 = 2e-6 * scale
    worst = 0.0
    for g, o, shv in ((fg, fo, sh), (hg, ho, 0.0)):
        g, o = g[:, fluid], o[:, fluid]
        dev = np.maximum(np.abs(o - shv), np.abs(g - shv))
        bound = 0.5 * _ulp16(dev, storage) + a32 + 1.2e-7 * np.abs(o)
        ratio = np.abs(g - o) / bound
        worst = max(worst, float(ratio.max()))
    print(storage, forcing, "max error / bound", worst, flush=True)
    assert worst <= 1.0
    # the bound is not vacuous: the rounding uses a good part of it
    assert worst > 0.25
    lat.close()
