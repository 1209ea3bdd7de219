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


def solve(samples, tol, max_steps, storage="f32", init=None, progress=0):
    """Run a batch to tolerance.  ``init``: optional list of (rho, u) per sample
    (default: rest with the seeded phases).  Returns per-sample steps (-1: not
    converged within max_steps), per-sample divergence flags, the final fields
    and the wall time.  With ``progress`` > 0 the run is cut into pieces of that
    many steps (a multiple of the monitor interval; the result is the same) and
    the number of settled samples is printed after each."""
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
    ok, steps, piece = False, 0, progress if progress > 0 else max_steps
    while steps < max_steps:
        ok, n = b.run_to_residual(tol, min(piece, max_steps - steps), allow_diverged=True)
        steps += n
        settled = sum(m[12] > 0 for m in (b.sample_monitors(i) for i in range(len(samples))))
        if progress > 0:
            print(f"[solve] step {steps}: {settled}/{len(samples)} settled, {time.perf_counter() - t0:.0f}s",
                  flush=True)
        if ok or n == 0 or settled == len(samples):
            break
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


def solve_all(samples, args, scale, init=None, tag=""):
    """``solve`` in batches of ``args.batch_solve``; keeps per sample the step
    count, the divergence flag and the steady fields as float32 targets."""
    out = dict(steps=[], diverged=[], wall=0.0, fields=[])
    for i in range(0, len(samples), args.batch_solve):
        part = samples[i: i + args.batch_solve]
        shape = part[0]["mask"].shape
        r = solve(part, args.tol, args.max_steps, args.storage,
                  None if init is None else init[i: i + args.batch_solve], progress=args.progress)
        out["steps"] += r["steps"]
        out["diverged"] += r["diverged"]
        out["wall"] += r["wall"]
        out["fields"] += [targets(rr, uu, shape, scale) for rr, uu in zip(r["rho"], r["u"])]
        print(f"[warmstart] {tag} solved {i + len(part)}/{len(samples)} median steps "
              f"{int(np.median(r['steps']))} wall {r['wall']:.1f}s", flush=True)
    return out


def train(args, rep):
    """Generate the training pairs with the solver and train the network."""
    import torch

    dev = torch.device("cuda:0")
    train_s = make_samples(args.n, args.train, 0)
    scale = u_scale(train_s[0]["params"], 8)
    shape = (args.n,) * 3
    gen = solve_all(train_s, args, scale, tag="train")
    keep = [i for i, d in enumerate(gen["diverged"]) if not d]
    conv = [gen["steps"][i] for i in keep if gen["steps"][i] > 0]
    rep.update(train_converged=len(conv), train_diverged=len(train_s) - len(keep),
               train_at_cap=len(keep) - len(conv),
               train_steps_median=float(np.median(conv)) if conv else None, train_solve_wall_s=gen["wall"])
    X = np.stack([features(train_s[i]["mask"], train_s[i]["rho"].reshape((2,) + shape)) for i in keep])
    T = np.stack([gen["fields"][i] for i in keep])
    del gen
    var_u = float(np.mean(T[..., :3] ** 2))
    var_p = float(np.mean(T[..., 3] ** 2))
    wt = [var_p / max(var_u, 1e-30)] * 3 + [1.0]
    x = torch.tensor(X, device=dev)
    t = torch.tensor(T, device=dev)
    del X, T
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
    if args.weights:
        net.save(args.weights)
    return net, scale


def evaluate(args, net, scale, rep):
    """Held-out samples of edge ``args.test_n``: steps to tolerance from rest
    and from the prediction, batch by batch (the network is fully
    convolutional with periodic padding, so it applies to any edge divisible
    by 2^(levels - 1))."""
    import torch

    dev = torch.device("cuda:0")
    test_s = make_samples(args.test_n, args.test, args.test_first)
    shape = (args.test_n,) * 3
    res = dict(cold_steps=[], warm_steps=[], cold_diverged=[], warm_diverged=[], cold_wall_s=0.0, warm_wall_s=0.0,
               inference_wall_s=0.0, final_phi_mean_abs_diff=[], final_u_rel_diff=[])
    for i in range(0, len(test_s), args.batch_solve):
        part = test_s[i: i + args.batch_solve]
        cold = solve_all(part, args, scale, tag="cold")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        init = []
        for s in part:
            xf = torch.tensor(features(s["mask"], s["rho"].reshape((2,) + shape))[None], device=dev)
            y, _ = net.forward(xf)
            init.append(fields_from_prediction(y[0].cpu().numpy(), (s["rho"].sum(0) == 0).astype(np.uint8), scale))
        torch.cuda.synchronize()
        res["inference_wall_s"] += time.perf_counter() - t0
        warm = solve_all(part, args, scale, init=init, tag="warm")
        for key in ("steps", "diverged"):
            res["cold_" + key] += cold[key]
            res["warm_" + key] += warm[key]
        res["cold_wall_s"] += cold["wall"]
        res["warm_wall_s"] += warm["wall"]
        for j in range(len(part)):
            if cold["diverged"][j] or warm["diverged"][j]:
                continue      # non-finite fields: no comparison
            pc, pw = cold["fields"][j], warm["fields"][j]
            res["final_phi_mean_abs_diff"].append(float(np.mean(np.abs(pc[..., 3] - pw[..., 3]))))
            res["final_u_rel_diff"].append(
                float(np.linalg.norm(pc[..., :3] - pw[..., :3]) / max(np.linalg.norm(pc[..., :3]), 1e-30)))
        del cold, warm, init
    ratio = [w / c for w, c in zip(res["warm_steps"], res["cold_steps"]) if w > 0 and c > 0]
    res.update(test_n=args.test_n, test=args.test, test_first=args.test_first,
               cold_converged=sum(c > 0 for c in res["cold_steps"]),
               warm_converged=sum(w > 0 for w in res["warm_steps"]),
               cold_steps_median=float(np.median([c for c in res["cold_steps"] if c > 0])) if ratio else None,
               warm_steps_median=float(np.median([w for w in res["warm_steps"] if w > 0])) if ratio else None,
               step_ratio_median=float(np.median(ratio)) if ratio else None,
               step_ratio_mean=float(np.mean(ratio)) if ratio else None,
               wall_ratio_incl_inference=(res["warm_wall_s"] + res["inference_wall_s"]) / max(res["cold_wall_s"], 1e-9))
    rep.update(res)


def run(args):
    t_all = time.perf_counter()
    rep = dict(n=args.n, tol=args.tol, storage=args.storage, phase=args.phase)
    if args.phase != "eval":
        rep["train"] = args.train
    if args.phase in ("all", "train"):
        net, scale = train(args, rep)
    else:
        net = warmnet.UNet(cin=2, cout=4, widths=tuple(args.widths), seed=args.seed, residual=[(3, 1)],
                           zero_head=True)
        net.load_params(args.weights)
        scale = u_scale(make_samples(args.n, 1, 0)[0]["params"], 8)
    if args.phase in ("all", "eval"):
        evaluate(args, net, scale, rep)
    rep["total_wall_s"] = time.perf_counter() - t_all
    return rep


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", type=int, default=64, help="cubic sample edge")
    ap.add_argument("--train", type=int, default=256)
    ap.add_argument("--test", type=int, default=32)
    ap.add_argument("--test-n", type=int, default=None, help="edge of the held-out samples (default: --n)")
    ap.add_argument("--test-first", type=int, default=100000, help="seed of the first held-out sample")
    ap.add_argument("--phase", choices=("all", "train", "eval"), default="all")
    ap.add_argument("--weights", default=None, help="network weights (.npz) written by train, read by eval")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-steps", type=int, default=100000)
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--batch-solve", type=int, default=64)
    ap.add_argument("--progress", type=int, default=5000, help="print the settled count every this many steps")
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--batch", type=int, default=2)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--widths", type=int, nargs="+", default=[16, 32, 64, 128])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    if args.test_n is None:
        args.test_n = args.n
    if args.phase == "eval" and not args.weights:
        ap.error("--phase eval needs --weights")
    rep = run(args)
    line = json.dumps(rep)
    print(line)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
