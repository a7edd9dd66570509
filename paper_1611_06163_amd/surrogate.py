"""Training workflow of the membrane surrogate (network kernels and the
step integration live in libtdpd; this module only drives them).

collect() runs the plain model on the GPU and gathers per-vertex samples
(1-ring features and the plain bending + local-area force in the vertex's
local frame); train() fits the library's network to them with its own
forward, backward and Adam kernels.
"""
from __future__ import annotations

import numpy as np

from . import inputs as I
from . import tdpd


def collect(cfg, steps, every, skip=0):
    """Samples of every vertex that may use the network, every `every` steps
    of a plain run of `steps` steps (after `skip` unsampled steps)."""
    sysg = tdpd.System(cfg)
    sysg.step(skip)
    Xs, Ts = [], []
    for _ in range(max(steps // every, 1)):
        sysg.step(every)
        X, T, ok = sysg.surrogate_sample()
        Xs.append(X[ok])
        Ts.append(T[ok])
    sysg.close()
    return np.concatenate(Xs), np.concatenate(Ts)


def train(X, T, seed=0, batch=4096, steps=3000, lr=1e-3, holdout=0.05):
    """Fit a fresh network; returns (net, force_scale, report).  The samples
    are shuffled with a seeded permutation, a held-out share is kept for the
    error report, and targets are scaled by their RMS force."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(X.shape[0])
    X, T = X[perm], T[perm]
    nh = max(int(holdout * X.shape[0]), 1)
    Xh, Th, Xt, Tt = X[:nh], T[:nh], X[nh:], T[nh:]
    s_F = float(np.sqrt(np.mean(np.sum(Tt.astype(np.float64) ** 2, axis=1))))
    net = tdpd.Mlp(I.mlp_init_params(seed))
    losses = []
    # three stages of decreasing learning rate
    for frac, f in ((0.6, 1.0), (0.25, 0.3), (0.15, 0.1)):
        losses.append(net.train(Xt, Tt, s_F, min(batch, Xt.shape[0]), int(steps * frac), lr * f))
    losses = np.concatenate(losses)
    Y = net.forward(Xh) * s_F
    err = np.linalg.norm(Y - Th, axis=1)
    report = dict(samples=int(Xt.shape[0]), held_out=int(nh), force_scale=s_F,
                  loss_first=float(losses[:10].mean()), loss_last=float(losses[-10:].mean()),
                  heldout_rel_rms=float(np.sqrt(np.mean(err ** 2)) / s_F),
                  heldout_rel_p99=float(np.quantile(err, 0.99) / s_F),
                  heldout_within_1e2=float(np.mean(err <= 1e-2 * s_F)))
    return net, s_F, report
