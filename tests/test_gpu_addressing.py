"""GPU: the collide pass's two addressing forms give the same bits.

The step kernel addresses populations either with raw buffer instructions
(32-bit byte offsets, the default while every array is below 4 GiB) or with
flat 64-bit addresses (the form used for larger arrays).  Both must store the
same values into the same elements: every storage format, both forcing
schemes, the product species and the per-node rate field, after 30 steps,
compared bit for bit.
"""
import numpy as np
import pytest

from paper_2502_12955_amd import inputs, mclbm

from helpers import small_porous

pytestmark = pytest.mark.gpu


def _run(p, mask, rho, u, C, flat, k_node=None, steps=30):
    lat = mclbm.Lattice(p)
    lat.set_addressing(flat=flat)
    lat.set_geometry(mask)
    if k_node is not None:
        lat.set_wall_rate(k_node)
    lat.init_fields(rho, u, C)
    lat.step(steps)
    out = lat.populations(raw=True)
    lat.close()
    return out


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s", "bf16s"])
@pytest.mark.parametrize("forcing", ["guo", "sc"])
def test_buffer_and_flat_addressing_bit_identical(storage, forcing):
    print(f"addressing: {storage} {forcing}", flush=True)
    p, mask, rho, u, C = small_porous(storage=storage, forcing=forcing, solute="inlet_outlet_x",
                                      tau=(0.9, 1.3) if forcing == "sc" else (1.0, 1.0), k_wall=0.05,
                                      C_in=1.0)
    a = _run(p, mask, rho, u, C, flat=False)
    b = _run(p, mask, rho, u, C, flat=True)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("product,rate", [(1, 0), (0, 1), (1, 1)])
def test_addressing_with_product_and_rate_field(product, rate):
    print(f"addressing: product {product} rate field {rate}", flush=True)
    p, mask, rho, u, C = small_porous(storage="f32", k_wall=0.0 if rate else 0.05, C_in=1.0, product=product,
                                      D2=0.17, C_in2=0.2, rate_field=rate)
    k_node = None
    if rate:
        zz, yy, xx = np.meshgrid(*[np.arange(s) for s in mask.shape], indexing="ij")
        k_node = inputs.arrhenius_rate_field(700.0 + 15.0 * xx + 5.0 * np.sin(yy + zz), 1.0, 2500.0).reshape(-1)
    a = _run(p, mask, rho, u, C, flat=False, k_node=k_node)
    b = _run(p, mask, rho, u, C, flat=True, k_node=k_node)
    assert np.array_equal(a, b)
