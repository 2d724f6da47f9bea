"""Pins of the oracle's network forward (Sec. 4.3, Fig. 6), loss and gradient
(Sec. 5.2), Adam (Sec. 5.2 / Kingma and Ba) and Philox generator."""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_1709_05418_amd import synth

HERE = os.path.dirname(__file__)


def unpack(theta, K, W, H):
    out, off = {}, 0
    for name, r, c in synth.layer_shapes(K, W, H):
        n = r * (c if c else 1)
        out[name] = theta[off:off + n].reshape((r, c) if c else (r,))
        off += n
    assert off == theta.size
    return out


def numpy_forward(theta, K, W, H, z):
    """Matrix form of the network with numpy's float64 matmul (a library routine)."""
    p = unpack(np.asarray(theta, np.float64), K, W, H)
    P = z.shape[0]
    relu = lambda a: np.maximum(a, 0.0)
    o = np.zeros((P, W))
    gamma = z[:, -1:]
    for k in range(K):
        zk = np.concatenate([z[:, k * 225:(k + 1) * 225], gamma], axis=1)
        h = zk @ p[f"V{k}"].T + p[f"b1_{k}"]
        if k > 0:
            h = h + o @ p[f"W1_{k}"].T
        F1 = relu(h)
        o = relu(F1 @ p[f"W2_{k}"].T + p[f"b2_{k}"] + o)
    pre = None
    for m in range(H):
        pre = o @ p[f"Wh{m}"].T + p[f"bh{m}"]
        o = relu(pre)
    return o[:, 0], pre[:, 0]


def test_param_count_formula_and_paper_size():
    gold = json.load(open(os.path.join(HERE, "golden", "paper_structure.json")))
    K, W = gold["levels_K"]["value"], gold["hidden_width"]["value"]
    n = O.param_count(K, W, 3)
    assert n == synth.n_params(K, W, 3) == 1_296_601
    assert gold["param_count_approx"]["low"] <= n <= gold["param_count_approx"]["high"]
    assert 2 * K + 3 == gold["total_layers"]["value"]
    assert O.param_count(6, 64, 3) == 140_993


@pytest.mark.parametrize("K,W,H", [(1, 4, 3), (2, 8, 3), (3, 16, 2), (6, 64, 3)])
def test_forward_matches_numpy(K, W, H):
    rng = np.random.default_rng(K * 100 + W)
    theta = synth.init_params(K, W, H, seed=K + W, bias=0.01).astype(np.float64)
    z = rng.random((33, 225 * K + 1))
    z[:, -1] *= np.pi
    g, pre = O.forward(theta, K, W, H, z)
    g2, pre2 = numpy_forward(theta, K, W, H, z)
    np.testing.assert_allclose(pre, pre2, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(g, g2, rtol=1e-12, atol=1e-12)
    assert (g > 0).any()


def test_forward_bias_only_closed_form():
    K, W, H = 3, 5, 3
    theta = np.zeros(O.param_count(K, W, H))
    p = unpack(theta, K, W, H)
    for k in range(K):
        p[f"b1_{k}"][:] = 0.3
        p[f"b2_{k}"][:] = -0.1 + 0.2 * k
    p["bh0"][:] = 0.5
    p["bh1"][:] = 0.7
    p["bh2"][:] = 1.25
    g, pre = O.forward(theta, K, W, H, np.random.default_rng(0).random((4, 225 * K + 1)))
    # weights vanish, so every layer outputs relu(its bias); the final layer gives relu(1.25)
    np.testing.assert_array_equal(g, 1.25)
    p["bh2"][:] = -2.0
    g, pre = O.forward(theta, K, W, H, np.zeros((2, 225 * K + 1)))
    np.testing.assert_array_equal(g, 0.0)
    np.testing.assert_array_equal(pre, -2.0)


def test_forward_hand_computed_k1_w2():
    # K = 1, W = 2, H = 2 (one 2x2 trailing layer, then the 1x2 output layer)
    K, W, H = 1, 2, 2
    theta = np.zeros(O.param_count(K, W, H))
    p = unpack(theta, K, W, H)
    p["V0"][0, 0] = 2.0      # F1_0 from Sigma_0
    p["V0"][1, 225] = -1.0   # F1_1 from gamma
    p["b1_0"][:] = [0.5, 3.0]
    p["W2_0"][:] = [[1.0, 1.0], [0.0, -2.0]]
    p["b2_0"][:] = [0.0, 1.0]
    p["Wh0"][:] = [[1.0, -1.0], [0.5, 0.5]]
    p["bh0"][:] = [0.0, 0.25]
    p["Wh1"][:] = [[2.0, 1.0]]
    p["bh1"][:] = [-1.0]
    z = np.zeros((1, 226))
    z[0, 0], z[0, 225] = 1.5, 1.0
    # F1 = relu([2*1.5+0.5, -1+3]) = [3.5, 2]; a = [5.5, -4+1] -> o = [5.5, 0]
    # head: relu([5.5, 2.75+0.25]) = [5.5, 3]; out = relu(11 + 3 - 1) = 13
    g, pre = O.forward(theta, K, W, H, z)
    assert g[0] == 13.0 and pre[0] == 13.0


def test_backward_matches_central_differences():
    K, W, H = 2, 16, 3
    rng = np.random.default_rng(42)
    theta = synth.init_params(K, W, H, seed=7, bias=0.05).astype(np.float64)
    theta[-1] = 1.0  # keep the output ReLU alive so the gradient is not trivially zero
    B = 6
    z = rng.random((B, 225 * K + 1))
    t = np.log1p(rng.random(B) * 2)
    loss, grad = O.loss_grad(theta, K, W, H, z, t)
    g, _ = O.forward(theta, K, W, H, z)
    assert loss == pytest.approx(np.mean((np.log1p(g) - t) ** 2), rel=1e-14)
    h = 1e-6
    idx = rng.choice(theta.size, size=600, replace=False)
    idx = np.concatenate([idx, np.arange(theta.size - 300, theta.size)])  # all of the head's tail
    bad = []
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        lp, _ = O.loss_grad(tp, K, W, H, z, t, want_grad=False)
        lm, _ = O.loss_grad(tm, K, W, H, z, t, want_grad=False)
        fd = (lp - lm) / (2 * h)
        if abs(fd - grad[i]) > 1e-6 * max(abs(fd), abs(grad[i])) + 1e-9:
            bad.append((i, fd, grad[i]))
    # a perturbation that crosses a ReLU kink breaks the difference quotient; allow a handful
    assert len(bad) <= 3, bad[:5]
    assert np.abs(grad).max() > 1e-4


def test_loss_gradient_wrt_output_closed_form():
    # single-sample K=1 net whose output equals relu(bias): dL/db = 2 r / (1 + g)
    K, W, H = 1, 3, 1
    theta = np.zeros(O.param_count(K, W, H))
    theta[-1] = 0.8
    z = np.zeros((1, 226))
    t = np.array([0.1])
    loss, grad = O.loss_grad(theta, K, W, H, z, t)
    r = np.log1p(0.8) - 0.1
    assert loss == pytest.approx(r * r, rel=1e-15)
    assert grad[-1] == pytest.approx(2 * r / 1.8, rel=1e-14)


def test_adam_first_step_and_constant_gradient():
    rng = np.random.default_rng(0)
    n = 1000
    theta0 = rng.normal(size=n)
    g = rng.normal(size=n) * 10.0 ** rng.uniform(-6, 2, size=n)
    th, m, v = theta0.copy(), np.zeros(n), np.zeros(n)
    O.adam(th, m, v, g.copy(), 1)
    np.testing.assert_allclose(th - theta0, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-18)
    # constant gradient: bias correction makes every step the same size
    th, m, v = theta0.copy(), np.zeros(n), np.zeros(n)
    for t in range(1, 51):
        O.adam(th, m, v, g.copy(), t)
    np.testing.assert_allclose(th - theta0, -50e-3 * g / (np.abs(g) + 1e-8), rtol=1e-7, atol=1e-15)


def test_philox_known_answers():
    for line in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        f = [int(x, 16) for x in line.split()]
        np.testing.assert_array_equal(O.philox(f[0:4], f[4:6]), np.array(f[6:10], np.uint32))
