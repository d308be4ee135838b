"""Training and evaluation driver of the learned centroider: marshals
clusters through tpx_centroid, tpx_patches and the tpx_mlp_* calls (every
step of the computation runs in the library's kernels), and scores refined
hits against generator truth on the host."""
from __future__ import annotations

import numpy as np

from . import Mlp, centroid_dev, load, patches, refine, to_device_events


def prepare(cl):
    """Device tensors (feat, hits, truth, mult) of a batch of generated
    clusters (dict with events, labels, truth, mult): every sample is its own
    shot with its trigger at tick 0."""
    import torch
    load()
    ev = to_device_events(cl["events"])
    labels = torch.from_numpy(np.asarray(cl["labels"], np.uint32).view(np.int32)).cuda()
    trig = np.zeros(cl["n"], np.uint64)
    hits = centroid_dev(ev, labels, trig)
    assert hits.shape[0] == cl["n"]
    feat = patches(ev, labels, hits)
    truth = torch.from_numpy(np.asarray(cl["truth"], np.float32).reshape(-1, 6)).cuda()
    mult = torch.from_numpy(np.asarray(cl["mult"], np.uint8)).cuda()
    return feat, hits, truth, mult


def fit(mlp: Mlp, data, epochs, lr, batch=None, lr_final=None):
    """Adam over consecutive minibatches (the generator draws samples i.i.d.,
    so the order needs no shuffle); lr decays geometrically to lr_final.
    Returns the loss of the last minibatch."""
    feat, hits, truth, mult = data
    n = feat.shape[0]
    b = batch or mlp.batch
    steps = epochs * ((n + b - 1) // b)
    lr_final = lr if lr_final is None else lr_final
    decay = (lr_final / lr) ** (1.0 / max(steps - 1, 1))
    k, loss = 0, None
    for e in range(epochs):
        for b0 in range(0, n, b):
            b1 = min(n, b0 + b)
            last = e == epochs - 1 and b1 == n
            loss = mlp.train_step(feat[b0:b1], hits[b0:b1], truth[b0:b1], mult[b0:b1],
                                  lr * decay ** k, want_loss=last)
            k += 1
    return loss


def predict(mlp: Mlp, feat, hits):
    return refine(hits, mlp.forward(feat))


def score(hits_np, refined_np, truth, mult):
    """Position and time RMSE vs truth of the weighted centroid (one hit per
    cluster) and of the network (one or two hits, as its multiplicity
    probability says; pairs matched the cheaper way round), over single hits
    and over the hits of pairs, and the multiplicity accuracy."""
    truth = np.asarray(truth, np.float64).reshape(-1, 2, 3)
    mult = np.asarray(mult)
    one = mult == 1
    cx, cy, ct = (hits_np[f].astype(np.float64) for f in ("x", "y", "tof_ns"))
    r = np.asarray(refined_np, np.float64)
    pa, pb = r[:, 0:3], r[:, 3:6]
    two_pred = r[:, 6] > 0.5
    out = {}

    def rms(a):
        return float(np.sqrt(np.mean(a))) if a.size else float("nan")

    # singles
    d_plain = (cx - truth[:, 0, 0]) ** 2 + (cy - truth[:, 0, 1]) ** 2
    d_net = ((pa[:, :2] - truth[:, 0, :2]) ** 2).sum(1)
    out["single_pos_rmse_px"] = {"centroid": rms(d_plain[one]), "learned": rms(d_net[one])}
    out["single_t_rmse_ns"] = {"centroid": rms(((ct - truth[:, 0, 2]) ** 2)[one]),
                               "learned": rms(((pa[:, 2] - truth[:, 0, 2]) ** 2)[one])}
    # pairs: the centroid is one hit for both
    pr = ~one
    dp = np.concatenate([((cx - truth[:, k, 0]) ** 2 + (cy - truth[:, k, 1]) ** 2)[pr]
                         for k in range(2)])
    def pos2(p, t):
        return ((p[:, :2] - t[:, :2]) ** 2).sum(1)
    c1 = pos2(pa, truth[:, 0]) + pos2(pb, truth[:, 1])
    c2 = pos2(pa, truth[:, 1]) + pos2(pb, truth[:, 0])
    both = np.where(c1 <= c2, c1, c2)
    as_one = pos2(pa, truth[:, 0]) + pos2(pa, truth[:, 1])
    dn = np.where(two_pred, both, as_one)[pr]
    out["pair_pos_rmse_px"] = {"centroid": rms(dp), "learned": float(np.sqrt(dn.sum() / (2 * max(
        dn.size, 1)))) if dn.size else float("nan")}
    out["multiplicity_accuracy"] = float(np.mean(two_pred == ~one))
    out["n_single"], out["n_pair"] = int(one.sum()), int(pr.sum())
    return out
