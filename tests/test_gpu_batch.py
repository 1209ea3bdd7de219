"""GPU: batches of independent samples, persistent grids, graph replay and run-to-residual.

Every fluid node is updated by one thread with the same arithmetic whatever
the batch composition, launch shape or replay mechanism, so all of these are
required to be bit-identical to the plain single-lattice run.
"""
import numpy as np
import pytest

import oracle
from paper_2502_12955_amd import inputs, mclbm

from helpers import gpu_lattice, maxrel, split_pops

pytestmark = pytest.mark.gpu


def _samples(n=4, seed=0, storage="f32", k_wall=0.02):
    cases = []
    shapes = [(12, 14, 18), (9, 20, 16), (16, 10, 12), (10, 10, 10), (14, 9, 21)]
    for s in range(n):
        shape = shapes[s % len(shapes)]
        p, mask, rho, u, C = inputs.porous_case(shape=shape, porosity=0.5, radius=3, blob_radius=2,
                                               config=3, sample=seed + s, storage=storage)
        p.update(k_wall=k_wall, monitor_every=10)
        rng = inputs.SplitMix64(inputs.seed_for(3, 100 + s))
        C = 0.3 * rng.uniform(int(np.prod(shape))).reshape(shape)
        cases.append((p, mask, rho, C))
    return cases


def _batch(cases, **launch):
    b = mclbm.Batch([c[0] for c in cases])
    if launch:
        b.set_launch(**launch)
    b.set_geometry([c[1] for c in cases])
    b.init_fields([c[2] for c in cases], None, [c[3] for c in cases])
    return b


def _single_pops(case, steps):
    p, mask, rho, C = case
    lat = gpu_lattice(p, mask, rho, None, C)
    lat.step(steps)
    out = lat.populations(raw=True)
    lat.close()
    return out


def test_batch_samples_bit_identical_to_single_runs():
    cases = _samples(4)
    b = _batch(cases)
    b.step(25)
    pops = b.populations(raw=True)
    nplanes = 2 * 19 + 7
    off = 0
    for c, n in zip(cases, b.sizes):
        mine = pops[off: off + nplanes * n]
        off += nplanes * n
        assert np.array_equal(mine, _single_pops(c, 25))
    b.close()


@pytest.mark.parametrize("storage", ["f32", "f16s", "bf16s"])
def test_persistent_grid_and_block_sizes_bit_identical(storage):
    cases = _samples(3, seed=7, storage=storage)
    ref = _batch(cases)
    ref.step(20)
    want = ref.populations(raw=True)
    ref.close()
    for launch in (dict(block_threads=64, grid_blocks=8), dict(block_threads=128, grid_blocks=16),
                   dict(block_threads=256, grid_blocks=0)):
        b = _batch(cases, **launch)
        b.step(20)
        assert np.array_equal(b.populations(raw=True), want), launch
        b.close()


def test_graph_replay_matches_eager_steps():
    """Replays interleaved with eager steps and host reads; each compared bitwise."""
    cases = _samples(3, seed=11)
    eager = _batch(cases)
    graph = _batch(cases)
    graph.set_graph(True)
    for rep in range(4):
        eager.step(10)
        graph.step(10)          # first interval eager (no snapshot yet), then graph replays
        a = eager.populations(raw=True)
        g = graph.populations(raw=True)
        assert np.array_equal(a, g), rep
        assert np.array_equal(eager.monitors(), graph.monitors()), rep
    # an odd number of eager steps flips the A/B parity: the other graph is used
    eager.step(3)
    graph.step(3)
    eager.step(20)
    graph.step(20)
    assert np.array_equal(eager.populations(raw=True), graph.populations(raw=True))
    eager.close()
    graph.close()


def test_run_to_residual_freezes_each_sample():
    """Samples stop at their own convergence step; the batch result equals each
    sample run alone to the same tolerance.  FP64 storage: at this flow speed
    (|u| ~ 1e-4) FP32 round-off alone keeps the relative velocity change near
    1e-5, so the tolerance would test the arithmetic rather than the freezing."""
    cases = _samples(3, seed=21, k_wall=0.0, storage="f64")
    for p, *_ in cases:
        p.update(ncomp=1, G=((0, 0), (0, 0)), G_ads=(0, 0), solute="off", monitor_every=20,
                 accel=(1e-5, 0.0, 0.0))
    cases = [(p, m, r[:1] * 0 + 1.0, C) for p, m, r, C in cases]
    tol = 1e-5
    b = _batch(cases)
    b.set_graph(True)
    ok, steps = b.run_to_residual(tol, 20000)
    assert ok
    conv = [int(b.sample_monitors(s)[11]) for s in range(3)]
    assert all(c > 0 for c in conv) and max(conv) == steps
    pops = b.populations(raw=True)
    nplanes = 19
    off = 0
    for s, (c, n) in enumerate(zip(cases, b.sizes)):
        p, mask, rho, C = c
        lat = gpu_lattice(p, mask, rho)
        ok1, st1 = lat.run_to_residual(tol, 20000)
        assert ok1 and st1 == conv[s]
        assert np.array_equal(pops[off: off + nplanes * n], lat.populations(raw=True))
        off += nplanes * n
        lat.close()
    b.close()


def test_batch_fp64_matches_oracle_per_sample():
    cases = _samples(2, seed=31, storage="f64")
    b = _batch(cases)
    b.step(15)
    rhos, us, Cs = b.moments()
    for s, (p, mask, rho, C) in enumerate(cases):
        m, _ = oracle.pinch_fill(p, mask)
        f, h = oracle.init(p, m, rho, None, C)
        oracle.step(p, m, f, h, 15)
        ro, uo, Co = oracle.moments(p, m, f, h)
        assert maxrel(rhos[s], ro) < 1e-12
        assert maxrel(us[s], uo) < 1e-12
        assert maxrel(Cs[s][0], Co) < 1e-12
    b.close()


def test_autotune_picks_a_candidate_and_keeps_results_identical(tmp_path):
    cases = _samples(3, seed=41)
    b = mclbm.Batch([c[0] for c in cases])
    b.set_geometry([c[1] for c in cases])
    cache = str(tmp_path / "tune.json")
    nb, blk, grid, ms = b.autotune(trial_steps=4, cache_path=cache)
    assert nb in (0, 4, 16) and blk in (64, 128, 256) and grid % 8 == 0 and ms > 0
    with pytest.raises(mclbm.MclbmError) as e:      # populations were overwritten
        b.step(1)
    assert e.value.code == mclbm.ESTATE
    b.init_fields([c[2] for c in cases], None, [c[3] for c in cases])
    b.step(12)
    ref = _batch(cases)
    ref.step(12)
    assert np.array_equal(b.populations(raw=True), ref.populations(raw=True))
    # a second handle of the same class takes the cached shape without timing
    b2 = mclbm.Batch([c[0] for c in cases])
    b2.set_geometry([c[1] for c in cases])
    assert b2.autotune(trial_steps=4, cache_path=cache) == (nb, blk, grid, None)
    for x in (b, b2, ref):
        x.close()


def test_band_count_changes_the_numbering_not_the_results():
    """The fluid numbering's band count (1, 4, 16 bands, and 16 set again after
    the geometry, which numbers the nodes anew) leaves every population
    bit-identical to the default eight bands; monitors agree to rounding."""
    cases = _samples(3, seed=57)
    ref = _batch(cases)
    ref.step(12)
    want = ref.populations(raw=True)
    mref = ref.monitors()
    ref.close()
    for nb, after in ((1, False), (4, False), (16, False), (16, True)):
        b = mclbm.Batch([c[0] for c in cases])
        if not after:
            b.set_bands(nb)
        b.set_geometry([c[1] for c in cases])
        if after:
            b.set_bands(nb)
        b.init_fields([c[2] for c in cases], None, [c[3] for c in cases])
        b.step(12)
        assert np.array_equal(b.populations(raw=True), want), nb
        m = b.monitors()
        assert np.allclose(m[1:10], mref[1:10], rtol=1e-12, atol=0), nb
        b.close()
    b = mclbm.Batch([c[0] for c in cases])
    with pytest.raises(mclbm.MclbmError) as e:
        b.set_bands(65)
    assert e.value.code == mclbm.EINVAL
    b.close()


def test_a_diverged_sample_is_frozen_and_the_others_finish():
    """A NaN planted in one sample's populations (from the host) freezes that
    sample as diverged at the next monitor; the other samples run on to their
    own convergence, bit-identical to running them alone."""
    cases = _samples(3, seed=21, k_wall=0.0, storage="f64")
    for p, *_ in cases:
        p.update(ncomp=1, G=((0, 0), (0, 0)), G_ads=(0, 0), solute="off", monitor_every=20,
                 accel=(1e-5, 0.0, 0.0))
    cases = [(p, m, r[:1] * 0 + 1.0, C) for p, m, r, C in cases]
    b = _batch(cases)
    gmask, _, _ = b.get_geometry()
    n0 = b.sizes[0]
    n1 = int(np.flatnonzero(gmask[n0: n0 + b.sizes[1]] == 0)[0])   # a fluid node of sample 1
    pops = b.populations(raw=True)                   # [sample][plane][box node]
    pops[19 * n0 + n1] = np.nan                      # plane 0 of that node
    b.set_populations(pops, raw=True)
    ok, steps = b.run_to_residual(1e-5, 20000, allow_diverged=True)
    assert not ok
    mons = [b.sample_monitors(s) for s in range(3)]
    assert mons[1][13] == 20 and mons[1][11] == -1
    for s in (0, 2):
        assert mons[s][13] == -1 and mons[s][11] > 0
    with pytest.raises(mclbm.MclbmError) as e:
        b2 = _batch(cases)
        b2.set_populations(pops, raw=True)
        try:
            b2.run_to_residual(1e-5, 20000)
        finally:
            b2.close()
    assert e.value.code == mclbm.EDIVERGED
    out = b.populations(raw=True)
    sizes = []
    for s in (0, 2):
        p, mask, rho, C = cases[s]
        lat = gpu_lattice(p, mask, rho)
        ok1, st1 = lat.run_to_residual(1e-5, 20000)
        assert ok1 and st1 == mons[s][11]
        ref = lat.populations(raw=True)
        sizes.append(ref.size)
        off = 0 if s == 0 else out.size - ref.size
        assert np.array_equal(out[off: off + ref.size], ref)
        lat.close()
    b.close()


def test_tiny_samples_padded_beyond_their_box_match_the_oracle():
    """Samples of a few nodes each pad their fluid nodes to a whole 64-node
    chunk, so the batch holds more fluid slots than box nodes (the
    pseudo-potentials are stored per fluid slot); FP64 moments against the
    oracle and populations bit-identical to single-lattice runs."""
    shapes = [(1, 5, 6), (1, 3, 7), (1, 9, 9)]   # (nz, ny, nx)
    cases = []
    for s, shape in enumerate(shapes):
        nz, ny, nx = shape
        p = inputs.base_params(lattice="D2Q9", nx=nx, ny=ny, nz=1, G=((0.0, 4.2), (4.2, 0.0)),
                               G_ads=(-0.1, 0.1), accel=(1e-5, 0.0, 0.0), solute="periodic",
                               D=0.1, J0=0.4, k_wall=0.02, monitor_every=10)
        mask = np.zeros(shape, np.uint8)
        mask[0, 1, 2] = 1
        rho = inputs.droplet(shape, 1.6)
        rng = inputs.SplitMix64(inputs.seed_for(3, 700 + s))
        C = 0.3 * rng.uniform(int(np.prod(shape))).reshape(shape)
        cases.append((p, mask, rho, C))
    fluid = [int((oracle.pinch_fill(c[0], c[1])[0] == 0).sum()) for c in cases]
    assert sum(-(-nf // 64) * 64 for nf in fluid) > sum(int(np.prod(c[1].shape)) for c in cases)
    b = _batch(cases)
    b.step(12)
    rhos, us, Cs = b.moments()
    pops = b.populations(raw=True)
    nplanes = 2 * 9 + 5
    off = 0
    for s, (c, n) in enumerate(zip(cases, b.sizes)):
        p, mask, rho, C = c
        m, _ = oracle.pinch_fill(p, mask)
        f, h = oracle.init(p, m, rho, None, C)
        oracle.step(p, m, f, h, 12)
        ro, uo, Co = oracle.moments(p, m, f, h)
        assert maxrel(rhos[s], ro) < 1e-12
        assert maxrel(us[s], uo) < 1e-12
        assert maxrel(Cs[s][0], Co) < 1e-12
        mine = pops[off: off + nplanes * n]
        off += nplanes * n
        assert np.array_equal(mine, _single_pops(c, 12))
    b.close()
