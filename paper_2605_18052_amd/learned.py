"""Training the learned inlier-weight network from the plain method.

The plain solve (IRLS weights, threshold filter) is run on training scenes;
at a few rounds the library's feature kernel gives the features of every
retained match, and each is labelled with whether the plain method still
retains it at the end of the solve.  The network is trained on those pairs
with the library's training kernels (mean binary cross-entropy, Adam).  This
module only marshals arrays between the C ABI calls.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np

from . import fastea

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "inlier_mlp.npy")


def load_weights(path: str = WEIGHTS) -> np.ndarray:
    """The shipped network (packed float32 parameters)."""
    p = np.load(path, allow_pickle=False)
    if p.dtype != np.float32 or p.shape != (4801,):
        raise ValueError(f"{path}: not a packed 8-64-64-1 network")
    return p


def he_init(seed: int = 0) -> np.ndarray:
    """Packed parameters with He-normal weights and zero biases."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(scale=math.sqrt(2.0 / 8), size=(64, 8))
    W2 = rng.normal(scale=math.sqrt(2.0 / 64), size=(64, 64))
    w3 = rng.normal(scale=math.sqrt(1.0 / 64), size=64)
    return np.concatenate([W1.ravel(), np.zeros(64), W2.ravel(), np.zeros(64), w3, [0.0]]).astype(
        np.float32)


def collect(scene, rounds=(0, 1, 2, 3, 5, 8, 12), per_round=150_000, seed=0, options=None):
    """(features [n,8], targets [n]) torch device tensors from a plain solve."""
    import torch
    opt = options if options is not None else fastea.default_options()
    ctx = fastea.Context(0, opt)
    ctx.load_intrinsics(scene.f_init, scene.cx, scene.cy)
    ctx.load_matches(scene.x1, scene.y1, scene.x2, scene.y2, scene.cam1, scene.cam2)
    ctx.init_poses(scene.R_init, scene.t_init)
    rng = np.random.default_rng(seed)
    feats, poss = [], []
    for r in range(opt.rounds):
        ctx.begin_round(max(opt.tau_px_init * opt.tau_decay ** r, opt.tau_px_min))
        if r in rounds:
            f, p = ctx.mlp_features()
            ok = torch.nonzero(p >= 0).flatten()
            if len(ok) > per_round:
                sel = torch.from_numpy(np.sort(rng.choice(len(ok), per_round, replace=False))).to(ok.device)
                ok = ok[sel]
            feats.append(f[ok].clone())
            poss.append(p[ok].clone())
        ctx.step(opt.iters_per_round)
    mask, _ = ctx.get_mask()
    perm, _, _, _ = ctx.get_segments()
    ctx.close()
    # label of a sorted position: is that match retained at the end
    kept_sorted = torch.from_numpy(mask[perm].astype(np.float32)).cuda()
    feat = torch.cat(feats).contiguous()
    target = kept_sorted[torch.cat(poss).long()].contiguous()
    return feat, target


def train(feat, target, epochs=6, batch=8192, lr=2e-3, seed=0, init_seed=0):
    import torch
    params = torch.from_numpy(he_init(init_seed)).cuda()
    losses = fastea.mlp_train(feat, target, params, epochs=epochs, batch=batch, lr=lr, seed=seed)
    return params.cpu().numpy(), losses


def bce(feat, target, params):
    import torch
    loss, _ = fastea.mlp_grad(feat, target, torch.from_numpy(params).cuda())
    return loss


def main(argv=None):
    """Trains the shipped network on the GPU: plain solves of trajectory
    scenes (500 cameras, 20 nearest neighbours, 20% outliers) give the
    features and labels; one held-out scene gives the validation loss."""
    import torch

    from . import synth
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--scenes", type=int, default=4)
    ap.add_argument("--matches", type=int, default=8_000_000)
    ap.add_argument("--seed", type=int, default=5000)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--lr", type=float, default=2e-3)
    a = ap.parse_args(argv)
    t0 = time.time()
    feats, targets = [], []
    for k in range(a.scenes):
        sc = synth.trajectory_scene(seed=a.seed + k, target_matches=a.matches, name=f"train{k}")
        f, t = collect(sc)
        feats.append(f)
        targets.append(t)
        print(f"[learned] scene {k}: {sc.n_matches} matches, {len(t)} samples ({time.time() - t0:.1f} s)",
              flush=True)
    feat = torch.cat(feats).contiguous()
    target = torch.cat(targets).contiguous()
    params, losses = train(feat, target, epochs=a.epochs, lr=a.lr)
    val = synth.trajectory_scene(seed=a.seed + a.scenes, target_matches=a.matches, name="val")
    vf, vt = collect(val)
    vloss = bce(vf, vt, params)
    print(f"[learned] train loss per epoch {np.round(losses, 4).tolist()}, validation {vloss:.4f}", flush=True)
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    np.save(a.out, params.astype(np.float32))
    meta = {"train_scenes": [f"trajectory_scene(seed={a.seed + k}, target_matches={a.matches})"
                             for k in range(a.scenes)],
            "validation_scene": f"trajectory_scene(seed={a.seed + a.scenes}, target_matches={a.matches})",
            "samples": int(len(target)), "positive_fraction": float(target.mean().item()),
            "epochs": a.epochs, "lr": a.lr, "train_loss": [float(x) for x in losses],
            "validation_loss": float(vloss)}
    with open(os.path.splitext(a.out)[0] + ".json", "w") as fh:
        json.dump(meta, fh, indent=1)
    print(f"[learned] wrote {a.out} ({time.time() - t0:.1f} s)", flush=True)


if __name__ == "__main__":
    main()
