"""Train the learned shape-function surrogate on the GPU.

Samples are (features, exact shape functions) pairs of every (marker,
component): markers are drawn uniformly in the interior of the wall-bounded
stretched channel (x, y periodic and uniform, z between walls with tanh
clustering), their features and exact-MLS shape functions come from the HIP
library (mls_features, mls_build with MLS_EXACT).  The network is trained
with the library's own forward/backward kernels and Adam (mls_mlp_train_step)
on random mini-batches; the learning rate follows a cosine decay.

The result is an .npz checkpoint holding the FP32 parameters, the input
normalisation, the training configuration and seed, held-out metrics and a
SHA-256 of the parameters.

    python -m paper_1805_01113_amd.train_mlp --steps 60000 --out weights.npz
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
if os.path.dirname(HERE) not in sys.path:
    sys.path.insert(0, os.path.dirname(HERE))

from paper_1805_01113_amd import mls  # noqa: E402
from paper_1805_01113_amd import workloads as W  # noqa: E402

DEFAULT_WEIGHTS = os.path.join(HERE, "data", "mlp_stretched_channel.npz")
N_IN, N_H, N_OUT = 6, 128, 27


def channel_grid(nxy=512, nz=768, lz=1.5, beta=2.5):
    """The stretched-channel geometry: 512 x 512 x 768, tanh walls in z."""
    return W.GridSpec([W.uniform_faces(nxy), W.uniform_faces(nxy), W.tanh_faces(nz, lz, beta)],
                      [True, True, False])


def interior_markers(gs, n, seed):
    """n markers uniform in x, y and in z between the second faces from each wall."""
    r = np.random.default_rng(seed)
    fz = gs.faces[2]
    x = r.uniform(0.0, 1.0, n).astype(np.float32)
    y = r.uniform(0.0, 1.0, n).astype(np.float32)
    z = r.uniform(fz[2], fz[-3], n).astype(np.float32)
    return x, y, z


def init_params(seed):
    """He initialisation (normal, std sqrt(2 / fan_in)), zero biases, last layer x 0.1."""
    r = np.random.default_rng(seed)
    w1 = r.normal(0.0, math.sqrt(2.0 / N_IN), (N_IN, N_H))
    w2 = r.normal(0.0, math.sqrt(2.0 / N_H), (N_H, N_H))
    w3 = r.normal(0.0, math.sqrt(2.0 / N_H), (N_H, N_OUT)) * 0.1
    parts = [w1, np.zeros(N_H), w2, np.zeros(N_H), w3, np.zeros(N_OUT)]
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


def make_samples(ctx, gs, n_markers, seed, chunk=1 << 20):
    """Features [3 n, 6] and exact shape functions [3 n, 27] on the device."""
    import torch
    x, y, z = interior_markers(gs, n_markers, seed)
    feats, targs = [], []
    for a in range(0, n_markers, chunk):
        b = min(n_markers, a + chunk)
        xd, yd, zd = [torch.from_numpy(v[a:b]).cuda() for v in (x, y, z)]
        f = ctx.features(xd, yd, zd)
        _, phi, _ = ctx.build(xd, yd, zd, method=mls.MLS_EXACT)
        ctx.sync()
        feats.append(f.reshape(-1, N_IN))
        targs.append(mls.unpack_phi(phi, b - a).reshape(-1, N_OUT).contiguous())
    return torch.cat(feats), torch.cat(targs), (x, y, z)


def normalisation(feat_sample):
    """shift = mean, scale = 1 / std per feature (1 where a feature is constant)."""
    f = np.asarray(feat_sample, dtype=np.float64)
    mu = f.mean(0)
    sd = f.std(0)
    scale = np.where(sd > 1e-12, 1.0 / np.maximum(sd, 1e-12), 1.0)
    return np.concatenate([mu, scale]).astype(np.float32)


def evaluate(ctx, gs, held, tol=1e-4):
    """Held-out metrics: RMS error of the network against exact MLS, and the
    share of (marker, component) pairs the learned build keeps at tol."""
    import torch
    feat, targ, (x, y, z) = held
    y_net = ctx.mlp_forward(feat)
    ctx.sync()
    err = (y_net - targ).double()
    rms = float(torch.sqrt((err * err).mean()).item())
    emax = float(err.abs().max().item())
    ctx.stats_reset()
    xd, yd, zd = [torch.from_numpy(v).cuda() for v in (x, y, z)]
    ctx.build(xd, yd, zd, method=mls.MLS_LEARNED)
    ctx.sync()
    st = ctx.stats()
    kept = st["learned"] / max(1, st["learned"] + st["fallbacks"])
    return dict(rms=rms, max_abs=emax, kept=kept, tol=tol)


def train(steps=60000, batch=8192, lr=2e-3, lr_min=1e-5, mu=1.0, n_markers=3_333_334, n_held=100_000,
          seed=20180503, log_every=2000, out=DEFAULT_WEIGHTS, init=None):
    import torch
    gs = channel_grid()
    ctx = mls.Context(gs.faces, gs.periodic, fallback_tol=1e-4)
    t0 = time.time()
    feat, targ, _ = make_samples(ctx, gs, n_markers, seed)
    held = make_samples(ctx, gs, n_held, seed + 1)
    rows = feat.shape[0]
    print("samples: %d rows (%d markers x 3 components), held-out %d rows, %.1f s"
          % (rows, n_markers, held[0].shape[0], time.time() - t0), flush=True)
    sub = feat[torch.randperm(rows, device="cuda")[:1_000_000]].cpu().numpy()
    norm = normalisation(sub)
    params = init_params(seed) if init is None else np.asarray(init, dtype=np.float32)
    ctx.mlp_load(params, norm)
    m0 = evaluate(ctx, gs, held)
    print("start: held-out rms %.3e max %.3e kept %.4f" % (m0["rms"], m0["max_abs"], m0["kept"]), flush=True)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    t1 = time.time()
    history = []
    for s in range(steps):
        cur = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * s / max(1, steps)))
        idx = torch.randint(0, rows, (batch,), device="cuda", generator=gen)
        ctx.mlp_train_step(feat, targ, lr=cur, mu=mu, idx=idx, loss=loss)
        if (s + 1) % log_every == 0 or s + 1 == steps:
            ctx.sync()
            history.append((s + 1, float(loss.item())))
            print("step %d lr %.2e batch loss %.3e (%.1f steps/s)"
                  % (s + 1, cur, loss.item(), (s + 1) / (time.time() - t1)), flush=True)
    ctx.sync()
    train_s = time.time() - t1
    m1 = evaluate(ctx, gs, held)
    print("end: held-out rms %.3e max %.3e kept %.4f  (%.1f s training)"
          % (m1["rms"], m1["max_abs"], m1["kept"], train_s), flush=True)
    p, q = ctx.mlp_get()
    cfg = dict(steps=steps, batch=batch, lr=lr, lr_min=lr_min, mu=mu, n_markers=n_markers, n_held=n_held,
               seed=seed, grid="512x512x768 tanh beta 2.5 lz 1.5, x/y periodic", schedule="cosine",
               optimizer="adam(0.9, 0.999, 1e-8)", train_seconds=train_s)
    if out:
        os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
        np.savez(out, params=p, norm=q, config=json.dumps(cfg), start=json.dumps(m0), end=json.dumps(m1),
                 history=np.array(history, dtype=np.float64),
                 sha256=hashlib.sha256(p.tobytes() + q.tobytes()).hexdigest())
        print("wrote", out, flush=True)
    return p, q, m0, m1


def load_weights(path=DEFAULT_WEIGHTS):
    """(params, norm, metadata) of a checkpoint written by train()."""
    z = np.load(path, allow_pickle=False)
    p, q = z["params"], z["norm"]
    if hashlib.sha256(p.tobytes() + q.tobytes()).hexdigest() != str(z["sha256"]):
        raise ValueError("checkpoint %s: parameter hash mismatch" % path)
    meta = {k: json.loads(str(z[k])) for k in ("config", "start", "end")}
    return p, q, meta


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--steps", type=int, default=60000)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--lr-min", type=float, default=1e-5)
    ap.add_argument("--mu", type=float, default=1.0)
    ap.add_argument("--markers", type=int, default=3_333_334)
    ap.add_argument("--seed", type=int, default=20180503)
    ap.add_argument("--log-every", type=int, default=2000)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    a = ap.parse_args()
    train(a.steps, a.batch, a.lr, a.lr_min, a.mu, a.markers, seed=a.seed, log_every=a.log_every, out=a.out)


if __name__ == "__main__":
    main()
