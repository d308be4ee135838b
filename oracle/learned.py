"""Oracle for the learned centroider / multiplicity splitter: 7 x 7 ToT/ToA
patch per cluster, a 98 -> 256 -> 256 -> 8 MLP, its loss, gradients and the
Adam update.

TEST INFRASTRUCTURE ONLY: the test suite and the benchmark's CPU-baseline leg
are the only callers.  The product library never imports anything from here.

Plain numpy in float64, written from the definitions:
  * the patch around a hit is centred on the pixel nearest to the hit's
    ToT-weighted centroid (Sec. V, Centroiding, Eq. 9), rounded as the fp32
    centroid (x + 1/2 rounded down, in fp32); plane 0 holds each pixel's
    summed ToT / 1024 (ToT is a 10-bit count, so this lies in [0, 1)), plane 1
    the pixel's earliest ToA minus the hit's earliest ToA, in units of
    64 ticks (100 ns); pixels outside the 7 x 7 window are left out; both
    planes are stored as bfloat16 (round to nearest even from fp32);
  * the network computes with bfloat16 inputs and weights and fp32 biases:
    h1 = relu(W1 f + b1), h2 = relu(W2 h1 + b2), o = W3 h2 + b3, with W stored
    row-major as [out][in] and the parameters packed W1, b1, W2, b2, W3, b3;
    here every product and sum is exact float64 and the hidden activations
    are not rounded;
  * outputs o[0:3] and o[3:6] are two hits as corrections to the weighted
    centroid (x - xc, y - yc in pixels, with (xc, yc) the fp32 centroid, and
    (t - ToA_first) / 10 ns), o[6] and o[7] the logits of one and two hits,
    so a network that outputs zeros reproduces the weighted centroid;
  * the loss of a sample is the squared error of hit A for a single hit, the
    smaller of the two assignments' summed squared errors for a pair (ties
    take A-first / B-second), plus the cross entropy of the two logits;
    the batch loss is the mean;
  * gradients treat the bfloat16 rounding of the weights as the identity
    (mixed-precision training with fp32 master weights);
  * Adam (Kingma and Ba, 2015) with bias-corrected moments.
The gradients are pinned by central finite differences of this loss, the
forward pass by networks whose output is known in closed form, the rounding
by torch's own bfloat16 conversion.
"""
from __future__ import annotations

import numpy as np

IN, HID, OUT = 98, 256, 8
PATCH, HALF = 7, 3
TICK_NS = 1.5625
T_UNIT_NS = 10.0
SHAPES = [("W1", (HID, IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("W3", (OUT, HID)), ("b3", (OUT,))]
N_PARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def bf16_bits(a):
    """fp32 -> bfloat16 bit pattern, round to nearest, ties to even."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    return ((u + 0x7FFF + lsb) >> 16).astype(np.uint16)


def bf16_value(bits):
    return (np.asarray(bits, np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def bf16_round(a):
    return bf16_value(bf16_bits(a))


def unpack(params):
    p = np.asarray(params, np.float64)
    assert p.size == N_PARAM
    out, k = {}, 0
    for name, shape in SHAPES:
        m = int(np.prod(shape))
        out[name] = p[k:k + m].reshape(shape)
        k += m
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in SHAPES])


def centre(hx, hy):
    """Patch centre of hits with fp32 centroids: floor(x + 1/2) in fp32."""
    h = np.float32(0.5)
    cx = np.floor(np.asarray(hx, np.float32) + h).astype(np.int64)
    cy = np.floor(np.asarray(hy, np.float32) + h).astype(np.int64)
    return cx, cy


def patches(x, y, tot, toa, shot, labels, hits):
    """bfloat16 bit patterns [n_hits, 98] of the clusters (events grouped by
    (shot, label)) whose hits are given (fields x, y as fp32 centroids, shot,
    label, toa_first)."""
    n_h = len(hits)
    idx = {(int(s), int(l)): k for k, (s, l) in enumerate(zip(hits["shot"], hits["label"]))}
    cx, cy = centre(hits["x"], hits["y"])
    tsum = np.zeros((n_h, PATCH * PATCH), np.int64)
    dmin = np.full((n_h, PATCH * PATCH), -1, np.int64)
    for i in range(len(x)):
        k = idx[(int(shot[i]), int(labels[i]))]
        ix = int(x[i]) - int(cx[k]) + HALF
        iy = int(y[i]) - int(cy[k]) + HALF
        if not (0 <= ix < PATCH and 0 <= iy < PATCH):
            continue
        c = iy * PATCH + ix
        tsum[k, c] += int(tot[i])
        d = int(toa[i]) - int(hits["toa_first"][k])
        dmin[k, c] = d if dmin[k, c] < 0 else min(dmin[k, c], d)
    f_tot = np.minimum(tsum, 1023).astype(np.float64) / 1024.0
    f_t = np.where(dmin >= 0, dmin, 0).astype(np.float64) / 64.0
    return np.concatenate([bf16_bits(f_tot), bf16_bits(f_t)], axis=1)


def forward(params, feat_bits, quantize=True):
    """(o, cache) for bfloat16 features; weights are used bfloat16-rounded
    and biases fp32-rounded (quantize=False keeps them exact, which makes the
    loss differentiable for finite-difference checks)."""
    P = unpack(params)
    X = bf16_value(feat_bits)
    q = bf16_round if quantize else (lambda a: a)
    qb = (lambda a: np.float32(a).astype(np.float64)) if quantize else (lambda a: a)
    W1, W2, W3 = (q(P[k]) for k in ("W1", "W2", "W3"))
    b1, b2, b3 = (qb(P[k]) for k in ("b1", "b2", "b3"))
    Z1 = X @ W1.T + b1
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ W2.T + b2
    H2 = np.maximum(Z2, 0.0)
    O = H2 @ W3.T + b3
    return O, dict(X=X, W1=W1, W2=W2, W3=W3, Z1=Z1, H1=H1, Z2=Z2, H2=H2)


def _centroid32(hits):
    return (np.asarray(hits["x"], np.float32).astype(np.float64),
            np.asarray(hits["y"], np.float32).astype(np.float64))


def targets(hits, truth):
    """Targets [n, 2, 3] of the truth hits (absolute x, y in pixels, t in ns)
    relative to each hit's fp32 centroid and earliest ToA."""
    xc, yc = _centroid32(hits)
    t0 = hits["toa_first"].astype(np.float64) * TICK_NS
    T = np.empty((len(hits), 2, 3))
    T[:, :, 0] = truth[:, :, 0] - xc[:, None]
    T[:, :, 1] = truth[:, :, 1] - yc[:, None]
    T[:, :, 2] = (truth[:, :, 2] - t0[:, None]) / T_UNIT_NS
    return T


def loss_grad(O, T, mult):
    """Mean loss and dL/dO."""
    O = np.asarray(O, np.float64)
    B = O.shape[0]
    pa, pb = O[:, 0:3], O[:, 3:6]
    ea = ((pa - T[:, 0]) ** 2).sum(1)
    c1 = ea + ((pb - T[:, 1]) ** 2).sum(1)
    c2 = ((pa - T[:, 1]) ** 2).sum(1) + ((pb - T[:, 0]) ** 2).sum(1)
    two = np.asarray(mult) == 2
    swap = two & (c2 < c1)
    lpos = np.where(two, np.minimum(c1, c2), ea)
    ta = np.where(swap[:, None], T[:, 1], T[:, 0])
    tb = np.where(swap[:, None], T[:, 0], T[:, 1])
    lse = np.logaddexp(O[:, 6], O[:, 7])
    ce = lse - np.where(two, O[:, 7], O[:, 6])
    loss = float(np.mean(lpos + ce))
    G = np.zeros_like(O)
    G[:, 0:3] = 2.0 * (pa - ta)
    G[:, 3:6] = np.where(two[:, None], 2.0 * (pb - tb), 0.0)
    p = np.exp(O[:, 6:8] - lse[:, None])
    G[:, 6] = p[:, 0] - (~two)
    G[:, 7] = p[:, 1] - two
    return loss, G / B


def backward(cache, G):
    """Parameter gradients (packed like the parameters) of dL/dO = G."""
    dW3 = G.T @ cache["H2"]
    db3 = G.sum(0)
    dZ2 = (G @ cache["W3"]) * (cache["Z2"] > 0)
    dW2 = dZ2.T @ cache["H1"]
    db2 = dZ2.sum(0)
    dZ1 = (dZ2 @ cache["W2"]) * (cache["Z1"] > 0)
    dW1 = dZ1.T @ cache["X"]
    db1 = dZ1.sum(0)
    return pack(dict(W1=dW1, b1=db1, W2=dW2, b2=db2, W3=dW3, b3=db3))


def grad(params, feat_bits, T, mult, quantize=True):
    O, cache = forward(params, feat_bits, quantize)
    loss, G = loss_grad(O, T, mult)
    return loss, backward(cache, G), O


def adam(params, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def refine(hits, O):
    """Absolute predictions: [n, 2, 3] (x, y in pixels, t in ns) and the
    probability of two hits; a cluster whose logit of two hits is not above
    that of one keeps the weighted centroid's position (the network's
    corrections apply to pairs), its time comes from the network."""
    xc, yc = _centroid32(hits)
    t0 = hits["toa_first"].astype(np.float64) * TICK_NS
    R = np.empty((len(hits), 2, 3))
    p2 = 1.0 / (1.0 + np.exp(O[:, 6] - O[:, 7]))
    # a cluster judged single (logit of two not above that of one) keeps the
    # centroid's position; the logits are compared as given
    keep = (O[:, 7] > O[:, 6]).astype(np.float64)
    for k in range(2):
        R[:, k, 0] = xc + keep * O[:, 3 * k]
        R[:, k, 1] = yc + keep * O[:, 3 * k + 1]
        R[:, k, 2] = t0 + T_UNIT_NS * O[:, 3 * k + 2]
    return R, p2
