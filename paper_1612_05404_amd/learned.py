"""Learned starter of the entropic alpha Newton iteration: sample collection,
training and the stored network.

The network (20 -> 32 -> 32 -> 1, SiLU) maps the 19 non-equilibrium ratios
of one node and component, given as z_p = (f_p/f_eq_p - 1)/s and
s = max_p |f_p/f_eq_p - 1|, to (alpha* - 2)/s, where alpha* is the root of
the entropy balance of the entropic collision.  In the update it serves the
nodes where the series starter is rejected.  Inference runs fused in the
collision kernel (BF16 matrix cores) and only moves the Newton starting
point: every node is still polished to the same stopping rule, and the plain
solve from alpha = 2 remains the fallback.

Samples are drawn by the library (``elbm_alpha_samples``) from states of the
method's own runs; forward, backward and Adam run in the library's own
kernels (``elbm_mlp_train``).  Everything here is orchestration.

Usage (GPU): ``python -m paper_1612_05404_amd.learned --out FILE`` trains on
the periodic drop (32^3, FP64) and the drop under a field (64x64x128, FP32)
and writes the 1761 FP32 parameters as a .npy file.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "alpha_mlp_weights.npy")
N_IN, N_H, NPARAM = 20, 32, 1761


def init_weights(seed: int) -> np.ndarray:
    """Glorot-uniform W1, W2 from a seeded generator, small w3, zero biases."""
    rng = np.random.default_rng(seed)
    l1 = np.sqrt(6.0 / (N_IN + N_H))
    l2 = np.sqrt(6.0 / (2 * N_H))
    w = np.concatenate([rng.uniform(-l1, l1, N_H * N_IN), np.zeros(N_H), rng.uniform(-l2, l2, N_H * N_H),
                        np.zeros(N_H), rng.uniform(-0.1, 0.1, N_H), [0.0]])
    assert w.size == NPARAM
    return w.astype(np.float32)


def load_weights(path: str = WEIGHTS) -> np.ndarray:
    w = np.load(path, allow_pickle=False)
    if w.dtype != np.float32 or w.shape != (NPARAM,):
        raise ValueError(f"{path}: expected float32[{NPARAM}], found {w.dtype}{list(w.shape)}")
    return w


def collect(lat, snapshots: int, every: int, box: int = 0, served_only: bool = True, tmax: float = 8.0,
            per_snapshot: int = 0, seed: int = 0):
    """Runs the lattice and gathers (z, target) samples of box `box` after
    every `every` steps.

    With `served_only` only the nodes where the series starter is rejected
    are kept: those are the nodes where the learned starter is used, mostly
    at the interface, where the non-equilibrium part is large.  Targets with
    |(alpha* - 2)/s| above `tmax` are dropped (rare nodes the network cannot
    help; Newton handles them from the fallback starter).  `per_snapshot` > 0
    caps the samples taken per snapshot (random subset).
    Returns device tensors X [M, 20], T [M]."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    xs, ts = [], []
    for _ in range(snapshots):
        lat.step(every, record=False)
        feat, tgt, scl, val = lat.alpha_samples(box)
        keep = (val == 2) if served_only else (val >= 1)
        keep &= tgt.abs() <= tmax
        X, T = feat[keep], tgt[keep]
        if per_snapshot > 0 and X.shape[0] > per_snapshot:
            pick = torch.randperm(X.shape[0], generator=g)[:per_snapshot].to(X.device)
            X, T = X[pick], T[pick]
        xs.append(X.clone())
        ts.append(T.clone())
    return torch.cat(xs), torch.cat(ts)


def train(lat, X, T, steps: int, batch: int = 8192, lr: float = 2e-3, lr_end: float = 1e-4, seed: int = 0,
          chunk: int = 500, log=None):
    """Adam on the library's kernels, reshuffling the samples every pass;
    the learning rate decays geometrically from lr to lr_end over the steps
    (constant within a chunk of at most `chunk` steps).
    Returns the per-step batch losses."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    M = X.shape[0]
    losses = []
    done = 0
    while done < steps:
        perm = torch.randperm(M, generator=g).to(X.device)
        Xs, Ts = X[perm].contiguous(), T[perm].contiguous()
        per_pass = max(1, M // batch)
        left = min(per_pass, steps - done)
        while left > 0:
            n = min(chunk, left)
            rate = lr * (lr_end / lr) ** (done / max(1, steps - 1))
            ls = lat.mlp_train(Xs, Ts, batch, n, rate)
            losses.append(ls)
            if log:
                log(f"[train] steps {done + n} lr {rate:.2e} loss {float(np.mean(ls[-50:])):.4e}")
            done += n
            left -= n
            # the next chunk continues where this one stopped in the shuffled order
            off = (n * batch) % M
            Xs = torch.roll(Xs, -off, 0).contiguous()
            Ts = torch.roll(Ts, -off, 0).contiguous()
    return np.concatenate(losses) if losses else np.zeros(0, np.float32)


def main():
    ap = argparse.ArgumentParser(description="train the learned alpha starter on the GPU")
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--samples", type=int, default=10_000_000,
                    help="samples to collect (served nodes of the periodic drop and the drop under a field)")
    ap.add_argument("--run-steps", type=int, default=2000, help="steps of each sampled run")
    ap.add_argument("--every", type=int, default=20, help="steps between two snapshots of a run")
    args = ap.parse_args()
    import torch
    from . import elbm, inputs
    t0 = time.time()
    log = lambda m: print(f"{m} ({time.time() - t0:.1f} s)", file=sys.stderr, flush=True)
    # runs of the two configurations the network serves, one seed after the
    # other (the jitter draws and the drop's charge differ), until the target
    # count is reached; a quarter of the samples from the FP64 periodic drop
    Xs, Ts = [], []
    have = {"drop32": 0, "efield_drop": 0}
    want = {"drop32": args.samples // 4, "efield_drop": args.samples - args.samples // 4}
    for name, base in (("drop32", 1234), ("efield_drop", 1235)):
        k = 0
        while have[name] < want[name] and k < 64:
            wl = inputs.WORKLOADS[name](seed=base + 1000 * k)
            lat = elbm.Lattice(wl.params, wl.boxes, wl.dtype, device="cuda:0", alpha_guess="standard")
            X, T = collect(lat, args.run_steps // args.every, args.every, seed=args.seed + k)
            lat.close()
            X, T = X[: want[name] - have[name]], T[: want[name] - have[name]]
            have[name] += X.shape[0]
            Xs.append(X)
            Ts.append(T)
            log(f"[samples] {name} seed {base + 1000 * k}: {X.shape[0]} samples (total {have[name]}), "
                f"target mean {T.mean().item():.4f} std {T.std().item():.4f}")
            k += 1
    X, T = torch.cat(Xs), torch.cat(Ts)
    log(f"[samples] {X.shape[0]} samples in all")
    wl = inputs.WORKLOADS["drop32"]()
    lat = elbm.Lattice(wl.params, wl.boxes, wl.dtype, device="cuda:0", alpha_guess="mlp")
    lat.mlp_set_weights(init_weights(args.seed))
    ls = train(lat, X, T, args.steps, log=log)
    w = lat.mlp_get_weights()
    np.save(args.out, w.astype(np.float32), allow_pickle=False)
    log(f"[train] final loss (mean of the last 500 steps) {float(np.mean(ls[-500:])):.4e}; wrote {args.out}")


if __name__ == "__main__":
    main()
