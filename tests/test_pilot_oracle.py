"""Pins for the learned-pilot oracle: convolution against scipy, bf16
rounding against torch's conversion, gradients against finite differences."""
import numpy as np
import pytest
import scipy.signal

from oracle import pilot_oracle as P


def test_param_count():
    # 2*32*9+32 + 4*(32*32*9+32) + 32*9+1
    assert P.n_params() == 37889


def test_conv3x3_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 7, 9, 3))
    W = rng.standard_normal((3, 3, 3, 4))
    b = rng.standard_normal(4)
    y = P.conv3x3(x, W, b)
    for n in range(2):
        for co in range(4):
            ref = b[co] + sum(scipy.signal.correlate2d(x[n, :, :, ci], W[:, :, ci, co], mode="same",
                                                       boundary="fill", fillvalue=0) for ci in range(3))
            assert np.allclose(y[n, :, :, co], ref, atol=1e-12)


def test_bf16_round_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(5000) * 10 ** rng.uniform(-6, 3, 5000),
                        [1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -9, -0.0, 0.0, 65504.0, 1e-40]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    assert np.array_equal(P.bf16_round(x), ref)
    # ties go to even: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7
    assert P.bf16_round(np.float32(1 + 2 ** -8)) == 1.0
    assert P.bf16_round(np.float32(1 + 3 * 2 ** -8)) == 1 + 2 ** -6


@pytest.mark.parametrize("weight", [None, [0.3, 2.5]])
def test_gradient_finite_differences(weight):
    rng = np.random.default_rng(2)
    theta = rng.standard_normal(P.n_params()) * 0.2
    z = rng.random((2, 6, 5))
    sigma = np.array([0.1, 0.2])
    target = rng.random((2, 6, 5))
    loss, g = P.loss_and_grad(theta, z, sigma, target, bf16=False, weight=weight)
    idx = rng.choice(P.n_params(), 40, replace=False)
    # include every layer's bias and the last layer's weights
    idx = np.concatenate([idx, [608 - 1, P.n_params() - 1, P.n_params() - 2]])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (P.loss_and_grad(tp, z, sigma, target, False, weight)[0] -
              P.loss_and_grad(tm, z, sigma, target, False, weight)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-4 * abs(fd), (i, fd, g[i])


def test_weighted_loss_is_the_weighted_mean_of_image_losses():
    """Per-image weights: loss = (sum_b w_b * n_b * loss_b) / n, where loss_b is
    image b's own (unweighted) mean squared error."""
    rng = np.random.default_rng(5)
    theta = rng.standard_normal(P.n_params()) * 0.2
    z = rng.random((3, 5, 7))
    sigma = np.array([0.05, 0.1, 0.2])
    target = rng.random((3, 5, 7))
    w = np.array([0.5, 1.0, 4.0])
    lw, gw = P.loss_and_grad(theta, z, sigma, target, bf16=False, weight=w)
    parts = [P.loss_and_grad(theta, z[b:b + 1], sigma[b:b + 1], target[b:b + 1], bf16=False) for b in range(3)]
    assert abs(lw - sum(w[b] * parts[b][0] for b in range(3)) / 3) <= 1e-12 * abs(lw)
    g_sum = sum(w[b] * parts[b][1] for b in range(3)) / 3
    assert np.allclose(gw, g_sum, rtol=1e-10, atol=1e-14)


def test_residual_output_and_zero_network():
    z = np.random.default_rng(3).random((1, 5, 5))
    theta = np.zeros(P.n_params())
    pilot, _ = P.forward(theta, z, [0.1], bf16=False)
    assert np.array_equal(pilot, z)
