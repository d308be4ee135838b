"""Pins of the learned-centroider oracle (oracle/learned.py): bfloat16
rounding against torch's conversion, patches against hand-computed cases and
invariants, the forward pass against networks with closed-form outputs, the
loss against closed forms, its gradients against central finite differences,
and the Adam update against its first steps in closed form."""
import numpy as np
import pytest

import synth
from oracle import learned as L


def test_bf16_matches_torch():
    import torch
    rng = np.random.default_rng(3)
    a = np.concatenate([rng.normal(0, 1, 4000), rng.normal(0, 1e-3, 1000), rng.normal(0, 300, 1000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 - 2 ** -9,
                         255.5, 1023 / 1024, 400 / 1024]]).astype(np.float32)
    ref = torch.from_numpy(a).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(L.bf16_bits(a), ref)
    # ties go to even: 1 + 2^-8 sits halfway between 1 and 1 + 2^-7
    assert L.bf16_bits(np.float32(1.0 + 2 ** -8)) == 0x3F80
    assert L.bf16_bits(np.float32(1.0 + 3 * 2 ** -8)) == 0x3F82


def _hits(x, y, shot, label, toa_first):
    h = np.zeros(len(x), [("x", "<f4"), ("y", "<f4"), ("shot", "<u8"), ("label", "<u8"),
                          ("toa_first", "<u8")])
    h["x"], h["y"], h["shot"], h["label"], h["toa_first"] = x, y, shot, label, toa_first
    return h


def test_patch_hand_example():
    """Three pixels of one cluster and a re-fired pixel, centroid at
    (100.4, 50.6) -> centre (100, 51)."""
    x = np.array([100, 101, 100, 103, 104])
    y = np.array([51, 51, 51, 48, 51])
    tot = np.array([400, 200, 1000, 50, 7])
    toa = np.array([1000, 1010, 1003, 990, 1100])
    lab = np.zeros(5)
    h = _hits([100.4], [50.6], [0], [0], [990])
    f = L.patches(x, y, tot, toa, np.zeros(5), lab, h)[0]
    tot_p, t_p = L.bf16_value(f[:49]).reshape(7, 7), L.bf16_value(f[49:]).reshape(7, 7)
    # (100, 51) is the centre cell (3, 3): ToT 400 + 1000 clipped to 1023
    assert tot_p[3, 3] == L.bf16_round(1023 / 1024)
    assert t_p[3, 3] == (1000 - 990) / 64
    assert tot_p[3, 4] == L.bf16_round(200 / 1024) and t_p[3, 4] == 20 / 64
    # (103, 48): dx = 3, dy = -3 -> cell (0, 6); (104, 51) is outside
    assert tot_p[0, 6] == L.bf16_round(50 / 1024) and t_p[0, 6] == 0.0
    assert np.count_nonzero(tot_p) == 3
    assert np.count_nonzero(t_p) == 2


def test_patch_single_pixel_and_translation():
    x, y = np.array([20]), np.array([30])
    f = L.patches(x, y, np.array([512]), np.array([77]), np.zeros(1), np.zeros(1),
                  _hits([20.0], [30.0], [0], [0], [77]))[0]
    assert f[24] == 0x3F00 and np.count_nonzero(f) == 1     # 512 / 1024 = 0.5
    rng = np.random.default_rng(9)
    for _ in range(20):
        n = int(rng.integers(1, 40))
        x = rng.integers(90, 100, n)
        y = rng.integers(90, 100, n)
        tot = rng.integers(1, 700, n)
        toa = rng.integers(1000, 1200, n)
        hx, hy = np.float32(rng.uniform(92, 97)), np.float32(rng.uniform(92, 97))
        a = L.patches(x, y, tot, toa, np.zeros(n), np.zeros(n), _hits([hx], [hy], [0], [0],
                                                                       [toa.min()]))
        dx, dy, dt = int(rng.integers(-50, 50)), int(rng.integers(-50, 50)), int(rng.integers(0, 10 ** 6))
        b = L.patches(x + dx, y + dy, tot, toa + dt, np.zeros(n), np.zeros(n),
                      _hits([hx + dx], [hy + dy], [0], [0], [toa.min() + dt]))
        assert np.array_equal(a, b)


def test_patch_centre_rounds_fp32():
    cx, cy = L.centre(np.float32([2.5, 2.4999998, -0.5, 7.0]), np.float32([0.0, 0.5, 1.49, 1.51]))
    assert list(cx) == [3, 2, 0, 7] and list(cy) == [0, 1, 1, 2]


def _feat_from_values(v):
    return L.bf16_bits(np.asarray(v, np.float32))


def test_forward_closed_form():
    """A network computing f_k, |f_k| and relu(f_j - 0.5) + 0.25 exactly."""
    P = {n: np.zeros(s) for n, s in L.SHAPES}
    k, j = 5, 60
    P["W1"][0, k], P["W1"][1, k], P["W1"][2, j] = 1.0, -1.0, 1.0
    P["b1"][2] = -0.5
    P["W2"][0, 0] = P["W2"][1, 1] = P["W2"][2, 2] = 1.0
    P["W3"][0, 0], P["W3"][0, 1] = 1.0, -1.0
    P["W3"][1, 0] = P["W3"][1, 1] = 1.0
    P["W3"][2, 2] = 1.0
    P["b3"][2] = 0.25
    rng = np.random.default_rng(1)
    v = rng.uniform(-2, 2, (50, L.IN))
    feat = _feat_from_values(v)
    fv = L.bf16_value(feat)
    O, _ = L.forward(L.pack(P), feat)
    assert np.array_equal(O[:, 0], fv[:, k])
    assert np.array_equal(O[:, 1], np.abs(fv[:, k]))
    assert np.array_equal(O[:, 2], np.maximum(fv[:, j] - 0.5, 0) + 0.25)
    assert np.all(O[:, 3:] == 0)


def test_forward_rounds_weights_to_bf16():
    P = {n: np.zeros(s) for n, s in L.SHAPES}
    P["W1"][0, 0] = 1.0 + 2 ** -9         # rounds to 1
    P["W2"][0, 0] = 3.0
    P["W3"][0, 0] = 1.0
    feat = _feat_from_values(np.ones((1, L.IN)))
    O, _ = L.forward(L.pack(P), feat)
    assert O[0, 0] == 3.0
    O, _ = L.forward(L.pack(P), feat, quantize=False)
    assert O[0, 0] == 3.0 * (1.0 + 2 ** -9)


def test_loss_closed_forms():
    T = np.array([[[0.1, -0.2, 0.3], [1.0, 2.0, -1.0]]])
    O = np.zeros((1, 8))
    O[0, 0:3] = T[0, 0]
    loss, G = L.loss_grad(O, T, [1])
    assert loss == pytest.approx(np.log(2.0), abs=1e-15)
    assert np.all(G[0, :6] == 0) and G[0, 6] == pytest.approx(-0.5) and G[0, 7] == pytest.approx(0.5)
    # a single hit ignores output B
    O2 = O.copy()
    O2[0, 3:6] = [5, 6, 7]
    assert L.loss_grad(O2, T, [1])[0] == loss
    # a pair is matched either way round
    O3 = np.zeros((1, 8))
    O3[0, 0:3], O3[0, 3:6] = T[0, 1], T[0, 0]
    l3, G3 = L.loss_grad(O3, T, [2])
    assert l3 == pytest.approx(np.log(2.0)) and np.all(G3[0, :6] == 0)
    l4, _ = L.loss_grad(O3, T[:, ::-1], [2])
    assert l4 == l3
    # squared error and the mean over the batch
    O4 = np.zeros((2, 8))
    l5, G5 = L.loss_grad(O4, np.repeat(T, 2, 0), [1, 1])
    assert l5 == pytest.approx(np.log(2.0) + (T[0, 0] ** 2).sum())
    assert np.allclose(G5[:, 0:3], -2.0 * T[0, 0] / 2)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(12)
    B = 6
    params = synth.init_mlp_params(4).astype(np.float64)
    params[L.N_PARAM - 8:] = rng.normal(0, 0.3, 8)
    feat = _feat_from_values(rng.uniform(0, 1, (B, L.IN)))
    T = rng.normal(0, 1, (B, 2, 3))
    mult = np.array([1, 2, 1, 2, 2, 1])
    loss, g, _ = L.grad(params, feat, T, mult, quantize=False)
    # probe every bias and a random subset of weights
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in L.SHAPES])
    probe = list(range(offs[1], offs[2])) + list(range(offs[3], offs[4])) + \
        list(range(offs[5], offs[6])) + list(rng.choice(L.N_PARAM, 400, replace=False))
    h = 1e-6
    for i in probe:
        p1, p2 = params.copy(), params.copy()
        p1[i] += h
        p2[i] -= h
        fd = (L.grad(p1, feat, T, mult, False)[0] - L.grad(p2, feat, T, mult, False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_gradient_of_input_layer_zero_for_empty_features():
    """Features that are zero everywhere give no W1 gradient in their
    columns (dW1 = dZ1^T X)."""
    rng = np.random.default_rng(2)
    feat = _feat_from_values(rng.uniform(0, 1, (8, L.IN)))
    feat[:, 10] = 0
    _, g, _ = L.grad(synth.init_mlp_params(1), feat, rng.normal(0, 1, (8, 2, 3)), np.ones(8, int))
    W1g = L.unpack(g)["W1"]
    assert np.all(W1g[:, 10] == 0) and np.any(W1g[:, 11] != 0)


def test_adam_first_steps():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 0.0])
    p1, m, v = L.adam(p, np.zeros(3), np.zeros(3), g, 1, 0.01, eps=0.0 + 1e-30)
    assert np.allclose(p1, p - 0.01 * np.sign(g))
    # second step with the same gradient still moves by lr * sign(g)
    p2, m, v = L.adam(p1, m, v, g, 2, 0.01, eps=1e-30)
    assert np.allclose(p2, p - 0.02 * np.sign(g))
    # and with gradient g2 after g1: m and v by their recurrences
    g2 = np.array([0.1, 1.0, 2.0])
    p1, m1, v1 = L.adam(p, np.zeros(3), np.zeros(3), g, 1, 0.01)
    p2, m2, v2 = L.adam(p1, m1, v1, g2, 2, 0.01)
    mh = (0.9 * 0.1 * g + 0.1 * g2) / (1 - 0.81)
    vh = (0.999 * 0.001 * g * g + 0.001 * g2 * g2) / (1 - 0.999 ** 2)
    assert np.allclose(p2, p1 - 0.01 * mh / (np.sqrt(vh) + 1e-8))


def test_targets_and_refine_invert():
    rng = np.random.default_rng(5)
    n = 30
    h = _hits(rng.uniform(10, 200, n).astype(np.float32), rng.uniform(10, 200, n).astype(np.float32),
              np.arange(n), np.zeros(n), rng.integers(0, 6000, n))
    truth = rng.uniform(0, 200, (n, 2, 3))
    T = L.targets(h, truth)
    O = np.zeros((n, 8))
    O[:, 0:3], O[:, 3:6] = T[:, 0], T[:, 1]
    O[:, 7] = 1.0                               # judged a pair: corrections apply
    R, p2 = L.refine(h, O)
    assert np.allclose(R, truth, atol=1e-9) and np.all(p2 > 0.5)
    # judged single: the centroid's position, the network's time
    O[:, 7] = -1.0
    R1, _ = L.refine(h, O)
    assert np.array_equal(R1[:, :, 0], np.repeat(h["x"].astype(np.float64)[:, None], 2, 1))
    assert np.allclose(R1[:, :, 2], truth[:, :, 2], atol=1e-9)
    # zero outputs are the weighted centroid itself (the fallback)
    R0, _ = L.refine(h, np.zeros((n, 8)))
    assert np.array_equal(R0[:, 0, 0], h["x"].astype(np.float64))
    assert np.array_equal(R0[:, 1, 1], h["y"].astype(np.float64))
    assert np.array_equal(R0[:, 0, 2], h["toa_first"] * 1.5625)
