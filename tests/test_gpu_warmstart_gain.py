"""GPU: what the trained warm start gains over the method without it.

The network is trained on the GPU by the project's own kernels on
geometry -> steady-field pairs that the solver itself generates (64^3 sphere
packs, the porous two-phase physics without solute, steady = residual <=
1e-3), then applied to held-out 64^3 samples whose seeds are disjoint from the
training seeds.  Each held-out sample runs to the same residual twice: from
rest (the method without the network) and from the prediction.  The solver
judges convergence both times.  Asserted: the median ratio of warm to cold
steps, over the samples that converge both ways, is below 0.8, and the warm
runs plus the inference take less wall time than the cold runs.
"""
import argparse

import numpy as np
import pytest

from paper_2502_12955_amd import warmstart

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_trained_warm_start_saves_steps_on_held_out_samples():
    args = argparse.Namespace(n=64, train=48, test=12, test_n=64, test_first=300000, phase="all", weights=None,
                              tol=1e-3, max_steps=40000, storage="f32", batch_solve=48, progress=0, epochs=15,
                              batch=2, lr=2e-3, widths=[16, 32, 64, 128], seed=0, out=None)
    print("warm-start gain: train 48 x 64^3, held-out 12 x 64^3 (seeds from 300000)", flush=True)
    rep = warmstart.run(args)
    pairs = [(w, c) for w, c in zip(rep["warm_steps"], rep["cold_steps"]) if w > 0 and c > 0]
    ratio = float(np.median([w / c for w, c in pairs]))
    wall = rep["wall_ratio_incl_inference"]
    print(f"trained on {rep['train_converged']} pairs; loss {rep['loss_history'][0]:.3e} -> "
          f"{rep['loss_history'][-1]:.3e}; held-out converged both ways {len(pairs)}/12; "
          f"median warm/cold steps {ratio:.3f}; wall (warm + inference) / cold {wall:.3f}", flush=True)
    assert rep["train_converged"] >= 40
    assert len(pairs) >= 9
    assert ratio < 0.8
    assert wall < 1.0
