"""Pins of the oracle's all-at-once MLP baselines (Sec. 7, Fig. 10): a K = 1 RPNN is
exactly an MLP (no residual input, no W1), so on the same parameter vector the numpy MLP
must reproduce the C oracle's network and gradient; central finite differences check the
backward pass of deeper and wider MLPs.  CPU only."""
import numpy as np
import pytest

import oracle as O
from paper_1709_05418_amd import synth


def test_k1_rpnn_is_an_mlp():
    W, H, P = 24, 3, 37
    theta = synth.init_params(1, W, H, 5, bias=0.05, branch_scale=1.0)
    z = np.random.default_rng(1).random((P, 226))
    widths = [226, W, W, W, W, 1]
    assert O.mlp_param_count(widths) == O.param_count(1, W, H) == theta.size
    g, pre = O.mlp_forward(theta, widths, z)
    go, preo = O.forward(theta, 1, W, H, z)
    np.testing.assert_allclose(pre, preo, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(g, go, rtol=1e-12, atol=1e-12)
    t = np.log1p(np.abs(go) + 0.1 * np.random.default_rng(2).random(P))
    loss, grad = O.mlp_loss_grad(theta, widths, z, t)
    loss_o, grad_o = O.loss_grad(theta, 1, W, H, z, t)
    assert loss == pytest.approx(loss_o, rel=1e-12)
    np.testing.assert_allclose(grad, grad_o, rtol=1e-9, atol=1e-13)


@pytest.mark.parametrize("widths", [[9, 7, 5, 1], [12, 16, 16, 8, 8, 8, 1], [30] + [6] * 9 + [1]])
def test_mlp_gradient_finite_differences(widths):
    rng = np.random.default_rng(len(widths))
    n = O.mlp_param_count(widths)
    theta = rng.normal(0, 0.5, n) + 0.05
    z = rng.random((11, widths[0]))
    g, _ = O.mlp_forward(theta, widths, z)
    t = np.log1p(g) + 0.3 * rng.standard_normal(11)
    _, grad = O.mlp_loss_grad(theta, widths, z, t)
    h = 1e-6
    idx = rng.choice(n, size=min(n, 60), replace=False)
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (O.mlp_loss_grad(tp, widths, z, t)[0] - O.mlp_loss_grad(tm, widths, z, t)[0]) / (2 * h)
        assert grad[i] == pytest.approx(fd, rel=1e-5, abs=1e-9), i


def test_paper_sized_comparison_networks():
    # Sec. 7: 23 layers of 200 fed all at once, and 5 layers [400, 400, 200, 200, 200],
    # both with a scalar output layer after them, on the 2251-wide descriptor
    D = 225 * 10 + 1
    deep = [D] + [200] * 22 + [1]
    wide = [D, 400, 400, 200, 200, 200, 1]
    assert len(deep) - 1 == 23 and O.mlp_param_count(deep) == 1_294_801
    assert O.mlp_param_count(wide) == 1_222_001
    assert O.param_count(10, 200, 3) == 1_296_601
