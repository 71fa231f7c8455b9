"""Learned order of the RHS work queue.

A small network predicts, from 16 local-environment features of RHS j
(computed on the GPU by ``scocg_features``), the log of the number of outer
iterations its solve needs.  The predicted cost of RHS j is that iteration
count times the size of its local pattern (block entries); the work queue
hands out RHS longest-first, so the long solves start early and the tail of
the persistent launch is short.  The residual test stays the judge of
convergence: the order changes timing only, never results.

Training runs on the GPU through the library's own kernels
(``scocg_mlp_train_step``: forward, backward, Adam).  The host only
standardises the features (z-score), draws the batch order from a seeded
stream, and sorts predicted costs into a queue order.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import binding as B


@dataclass
class CostModel:
    w: np.ndarray            # float32 [5313]
    mu: np.ndarray           # feature means
    sd: np.ndarray           # feature standard deviations (1 where constant)
    history: list = field(default_factory=list)   # (epoch, train loss, validation loss)


def standardize(F, mu=None, sd=None):
    F = np.asarray(F, dtype=np.float64)
    if mu is None:
        mu = F.mean(0)
        sd = F.std(0)
        sd = np.where(sd > 0, sd, 1.0)
    return ((F - mu) / sd).astype(np.float32), mu, sd


def train(feats, log_iters, w0, shuffle_rng, epochs=200, batch=256, lr=1e-3, val_frac=0.2):
    """Fit the network to (feats, log_iters) with Adam on the GPU.

    ``w0``: initial weights (5313); ``shuffle_rng``: numpy Generator for the
    train/validation split and the batch order.  Returns a CostModel whose
    history lists (epoch, mean train-batch loss, validation loss)."""
    import torch
    X, mu, sd = standardize(feats)
    n = X.shape[0]
    perm = shuffle_rng.permutation(n)
    nval = int(round(val_frac * n))
    val, tr = perm[:nval], perm[nval:]
    dev = "cuda"
    Xd = torch.from_numpy(X).to(dev)
    td = torch.from_numpy(np.asarray(log_iters, dtype=np.float32)).to(dev)
    w = torch.from_numpy(np.asarray(w0, dtype=np.float32)).to(dev)
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    work = torch.empty(B.scocg_mlp_work_floats(), dtype=torch.float32, device=dev)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    vloss = torch.zeros(1, dtype=torch.float32, device=dev)
    vidx = torch.from_numpy(val.astype(np.int32)).to(dev) if nval else None
    stream = torch.cuda.current_stream()
    step = 0
    history = []
    best = (np.inf, w.cpu().numpy())
    for ep in range(epochs):
        order = tr[shuffle_rng.permutation(tr.size)]
        tot, nb = 0.0, 0
        batches = [order[i:i + batch] for i in range(0, order.size, batch)]
        for bidx in batches:
            step += 1
            idx = torch.from_numpy(bidx.astype(np.int32)).to(dev)
            B.scocg_mlp_train_step(w, m, v, Xd, td, idx, lr, step, loss, None, work, stream)
            tot += float(loss.item())
            nb += 1
        vl = float("nan")
        if vidx is not None:
            B.scocg_mlp_train_step(w, None, None, Xd, td, vidx, 0.0, 1, vloss, None, work, stream)
            vl = float(vloss.item())
            if vl < best[0]:
                best = (vl, w.cpu().numpy())
        history.append((ep, tot / max(1, nb), vl))
    w_final = best[1] if vidx is not None else w.cpu().numpy()    # weights of the best validation epoch
    return CostModel(w_final, mu, sd, history)


def predict(model: CostModel, feats):
    """Predicted log outer iterations for each row of ``feats`` (GPU forward)."""
    import torch
    X, _, _ = standardize(feats, model.mu, model.sd)
    Xd = torch.from_numpy(X).to("cuda")
    w = torch.from_numpy(model.w).to("cuda")
    y = torch.empty(X.shape[0], dtype=torch.float32, device="cuda")
    B.scocg_mlp_forward(w, Xd, y, torch.cuda.current_stream())
    return y.cpu().numpy().astype(np.float64)


def order_longest_first(cost):
    """Queue order: RHS by decreasing cost (stable for ties)."""
    return np.argsort(-np.asarray(cost, dtype=np.float64), kind="stable").astype(np.int32)


def entries_per_rhs(feats):
    """Block entries of each RHS's local pattern (features 0 and 1)."""
    F = np.asarray(feats, dtype=np.float64)
    return F[:, 0] * F[:, 1]
