"""Learned warm start for steady two-phase flow in porous media.

A 3-D U-Net (``warmnet.UNet``, every layer a HIP kernel of ``libwarmnet.so``)
maps [solid mask, initial phase field] to the steady [u_x, u_y, u_z, phi] of
the two-component Shan-Chen flow.  The lattice Boltzmann solver
(``libmclbm.so``) produces the training targets (batched run to a residual
tolerance), and then starts held-out samples from the prediction; it stays the
judge of convergence, so a poor prediction costs steps, never accuracy.

Workflow (``python -m paper_2502_12955_amd.warmstart --help``):

    1. ``make_samples``   seeded sphere packs + non-wetting blobs (inputs.porous_case)
    2. ``solve``          batched run to tolerance from rest -> steady fields, steps
    3. ``train``          mean squared error + Adam on the GPU
    4. ``evaluate``       held-out samples: steps to tolerance from rest vs from the prediction

The steady phase field of a two-phase flow depends on its history, so the
fields reached from a warm start may differ from those reached from rest; the
report gives both the step counts and that difference.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import inputs, mclbm, warmnet

RHO_MAJOR, RHO_MINOR = 1.0, 0.03     # densities of blob_phase's two phases


def u_scale(p, radius):
    """Velocity scale g R^2 / nu of a pore of radius R under body force g."""
    nu = (p["tau"][0] - 0.5) / 3.0
    return p["accel"][0] * radius * radius / nu


def make_samples(n, count, first, config=5, radius=8, blob_radius=6, saturation=0.15):
    """Seeded samples: porosity ~ U(0.3, 0.5) per sample, no solute."""
    out = []
    for s in range(first, first + count):
        por = 0.3 + 0.2 * inputs.SplitMix64(inputs.seed_for(config, s)).uniform(1)[0]
        p, mask, rho, _, _ = inputs.porous_case(n=n, porosity=por, radius=radius, config=config, sample=s,
                                               blob_radius=blob_radius, saturation=saturation)
        p.update(solute="off", k_wall=0.0, monitor_every=100)
        out.append(dict(params=p, mask=mask, rho=rho, seed=s))
    return out


def solve(samples, tol, max_steps, storage="f32", init=None):
    """Run a batch to tolerance.  ``init``: optional list of (rho, u) per sample
    (default: rest with the seeded phases).  Returns per-sample steps (-1: not
    converged within max_steps), per-sample divergence flags, the final fields
    and the wall time."""
    plist = [dict(s["params"], storage=storage) for s in samples]
    b = mclbm.Batch(plist)
    b.set_graph(True)
    b.set_geometry([s["mask"] for s in samples])
    if init is None:
        b.init_fields([s["rho"] for s in samples])
    else:
        b.init_fields([r for r, _ in init], [u for _, u in init])
    b.synchronize()
    t0 = time.perf_counter()
    ok, steps = b.run_to_residual(tol, max_steps, allow_diverged=True)
    b.synchronize()
    wall = time.perf_counter() - t0
    mons = [b.sample_monitors(i) for i in range(len(samples))]
    rhos, us, _ = b.moments()
    b.close()
    return dict(converged=ok, steps=[int(m[11]) for m in mons], diverged=[bool(m[13] >= 0) for m in mons],
                total_steps=steps, wall=wall, rho=rhos, u=us)


def features(mask, rho):
    """Network input [d, h, w, 2]: solid indicator and initial phase field (0 on solids)."""
    m = np.asarray(mask, np.float32).reshape(rho.shape[1:]) if np.ndim(mask) > 1 else None
    r0, r1 = rho[0], rho[1]
    tot = r0 + r1
    phi = np.where(tot > 0, (r0 - r1) / np.where(tot > 0, tot, 1.0), 0.0)
    solid = (tot == 0).astype(np.float32) if m is None else m
    return np.stack([solid, phi.astype(np.float32)], axis=-1)


def targets(rho, u, shape, scale):
    """Network target [d, h, w, 4]: u / scale and phi."""
    r0, r1 = rho[0].reshape(shape), rho[1].reshape(shape)
    tot = r0 + r1
    phi = np.where(tot > 0, (r0 - r1) / np.where(tot > 0, tot, 1.0), 0.0)
    uu = np.asarray(u).reshape((3,) + tuple(shape)) / scale
    return np.concatenate([np.moveaxis(uu, 0, -1), phi[..., None]], axis=-1).astype(np.float32)


def fields_from_prediction(pred, solid, scale):
    """(rho [2, N], u [3, N]) for init_fields from a prediction [d, h, w, 4]."""
    # the two phases' densities bound phi; clipping there keeps both densities >= RHO_MINOR > 0
    pmax = (RHO_MAJOR - RHO_MINOR) / (RHO_MAJOR + RHO_MINOR)
    phi = np.clip(pred[..., 3].astype(np.float64), -pmax, pmax)
    fluid = solid == 0
    tot = RHO_MAJOR + RHO_MINOR
    rho = np.stack([0.5 * tot * (1 + phi), 0.5 * tot * (1 - phi)]) * fluid
    u = np.moveaxis(pred[..., :3].astype(np.float64) * scale, -1, 0) * fluid
    return rho.reshape(2, -1), u.reshape(3, -1)


class Trainer:
    def __init__(self, net, x, t, wt, batch=2):
        import torch

        self.net, self.x, self.t, self.batch = net, x, t, batch
        self.wt = torch.tensor(np.asarray(wt, np.float32), device=x.device)
        self.flops = 0.0

    def epoch(self, lr, rng):
        import torch

        n = self.x.shape[0]
        order = rng.permutation(n)
        losses = []
        for i in range(0, n - self.batch + 1, self.batch):
            idx = torch.tensor(order[i: i + self.batch], device=self.x.device)
            xb = self.x.index_select(0, idx).contiguous()
            tb = self.t.index_select(0, idx).contiguous()
            y, acts = self.net.forward(xb)
            loss, g = warmnet.mse(y, tb, self.wt)
            self.net.backward(g, acts)
            self.net.adam_step(lr)
            losses.append(loss)
        return float(torch.stack(losses).mean().item())


def run(args):
    import torch

    t_all = time.perf_counter()
    dev = torch.device("cuda:0")
    rep = dict(n=args.n, train=args.train, test=args.test, tol=args.tol, storage=args.storage)
    train_s = make_samples(args.n, args.train, 0)
    test_s = make_samples(args.n, args.test, 100000)
    scale = u_scale(train_s[0]["params"], 8)
    shape = (args.n,) * 3

    def solve_all(samples, init=None):
        out = dict(steps=[], diverged=[], wall=0.0, rho=[], u=[])
        for i in range(0, len(samples), args.batch_solve):
            part = samples[i: i + args.batch_solve]
            r = solve(part, args.tol, args.max_steps, args.storage,
                      None if init is None else init[i: i + args.batch_solve])
            out["steps"] += r["steps"]
            out["diverged"] += r["diverged"]
            out["wall"] += r["wall"]
            out["rho"] += r["rho"]
            out["u"] += r["u"]
            print(f"[warmstart] solved {i + len(part)}/{len(samples)} steps {r['steps']} "
                  f"wall {r['wall']:.1f}s", flush=True)
        return out

    gen = solve_all(train_s)
    keep = [i for i, d in enumerate(gen["diverged"]) if not d]
    conv = [gen["steps"][i] for i in keep if gen["steps"][i] > 0]
    rep.update(train_converged=len(conv), train_diverged=len(train_s) - len(keep),
               train_steps_mean=float(np.mean(conv)) if conv else None, train_solve_wall_s=gen["wall"])
    X = np.stack([features(train_s[i]["mask"], train_s[i]["rho"].reshape((2,) + shape)) for i in keep])
    T = np.stack([targets(gen["rho"][i], gen["u"][i], shape, scale) for i in keep])
    var_u = float(np.mean(T[..., :3] ** 2))
    var_p = float(np.mean(T[..., 3] ** 2))
    wt = [var_p / max(var_u, 1e-30)] * 3 + [1.0]
    x = torch.tensor(X, device=dev)
    t = torch.tensor(T, device=dev)
    net = warmnet.UNet(cin=2, cout=4, widths=tuple(args.widths), seed=args.seed, residual=[(3, 1)],
                       zero_head=True)
    tr = Trainer(net, x, t, wt, batch=args.batch)
    rng = np.random.default_rng(args.seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = []
    for ep in range(args.epochs):
        lr = args.lr * (0.5 ** (ep // max(1, args.epochs // 3)))
        hist.append(tr.epoch(lr, rng))
        print(f"[warmstart] epoch {ep} loss {hist[-1]:.4e}", flush=True)
    torch.cuda.synchronize()
    train_wall = time.perf_counter() - t0
    it = args.epochs * (len(keep) // args.batch) * args.batch
    fl = 3.0 * warmnet.conv_flops(net, shape) * it
    rep.update(params=net.n_params(), loss_history=hist, train_wall_s=train_wall,
               train_tflops=fl / train_wall / 1e12)

    # held-out: from rest vs from the prediction
    cold = solve_all(test_s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    init = []
    for s in test_s:
        xf = torch.tensor(features(s["mask"], s["rho"].reshape((2,) + shape))[None], device=dev)
        y, _ = net.forward(xf)
        pred = y[0].cpu().numpy()
        init.append(fields_from_prediction(pred, (s["rho"].sum(0) == 0).astype(np.uint8), scale))
    torch.cuda.synchronize()
    infer = time.perf_counter() - t0
    warm = solve_all(test_s, init)
    ratio = [w / c for w, c in zip(warm["steps"], cold["steps"]) if w > 0 and c > 0]
    rep.update(cold_converged=sum(c > 0 for c in cold["steps"]), warm_converged=sum(w > 0 for w in warm["steps"]),
               cold_diverged=sum(cold["diverged"]), warm_diverged=sum(warm["diverged"]))
    dphi, du = [], []
    for i, (rc, rw, uc, uw) in enumerate(zip(cold["rho"], warm["rho"], cold["u"], warm["u"])):
        if cold["diverged"][i] or warm["diverged"][i]:
            continue      # non-finite fields: no comparison
        pc = targets(rc, uc, shape, scale)
        pw = targets(rw, uw, shape, scale)
        dphi.append(float(np.mean(np.abs(pc[..., 3] - pw[..., 3]))))
        du.append(float(np.linalg.norm(pc[..., :3] - pw[..., :3]) / max(np.linalg.norm(pc[..., :3]), 1e-30)))
    rep.update(cold_steps=cold["steps"], warm_steps=warm["steps"], cold_wall_s=cold["wall"],
               warm_wall_s=warm["wall"], inference_wall_s=infer,
               step_ratio_median=float(np.median(ratio)) if ratio else None,
               step_ratio_mean=float(np.mean(ratio)) if ratio else None,
               wall_ratio_incl_inference=(warm["wall"] + infer) / cold["wall"],
               final_phi_mean_abs_diff=dphi, final_u_rel_diff=du,
               total_wall_s=time.perf_counter() - t_all)
    return rep


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", type=int, default=64, help="cubic sample edge")
    ap.add_argument("--train", type=int, default=256)
    ap.add_argument("--test", type=int, default=32)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-steps", type=int, default=100000)
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--batch-solve", type=int, default=64)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--batch", type=int, default=2)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--widths", type=int, nargs="+", default=[16, 32, 64, 128])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    rep = run(args)
    line = json.dumps(rep)
    print(line)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
