"""Host-side pieces of the warm-start pipeline (no GPU): network save / load,
the mapping between solver fields and network tensors."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2502_12955_amd import warmnet, warmstart


def test_unet_save_and_load_round_trip(tmp_path):
    a = warmnet.UNet(cin=2, cout=4, widths=(8, 16), seed=1, device="cpu", residual=[(3, 1)])
    b = warmnet.UNet(cin=2, cout=4, widths=(8, 16), seed=2, device="cpu", residual=[(3, 1)])
    path = str(tmp_path / "w.npz")
    a.save(path)
    b.load_params(path)
    for la, lb in zip(a.layers(), b.layers()):
        assert torch.equal(la.W, lb.W) and torch.equal(la.b, lb.b)
    c = warmnet.UNet(cin=2, cout=4, widths=(8, 24), seed=1, device="cpu")
    with pytest.raises(ValueError):
        c.load_params(path)


def test_fields_round_trip_through_targets():
    rng = np.random.default_rng(0)
    shape = (4, 6, 8)
    solid = (rng.random(shape) < 0.3).astype(np.uint8)
    phi = np.clip(rng.uniform(-1, 1, shape), -0.9, 0.9)
    u = rng.standard_normal((3,) + shape) * 1e-3
    scale = 2e-3
    pred = np.concatenate([np.moveaxis(u / scale, 0, -1), phi[..., None]], axis=-1) * (1 - solid)[..., None]
    rho, uu = warmstart.fields_from_prediction(pred.astype(np.float32), solid, scale)
    assert rho.shape == (2, solid.size) and uu.shape == (3, solid.size)
    assert np.all(rho[:, solid.reshape(-1) == 1] == 0) and np.all(rho[:, solid.reshape(-1) == 0] > 0)
    back = warmstart.targets(rho, uu, shape, scale)
    fluid = solid == 0
    assert np.allclose(back[..., 3][fluid], phi[fluid], atol=1e-6)
    assert np.allclose(back[..., :3][fluid], (np.moveaxis(u, 0, -1) / scale)[fluid], atol=1e-5)
    # a prediction beyond the two phases' densities is clipped so both densities stay positive
    pred[..., 3] = 5.0
    rho2, _ = warmstart.fields_from_prediction(pred.astype(np.float32), solid, scale)
    assert np.all(rho2[:, solid.reshape(-1) == 0] > 0)
