"""Pins for the classifier oracle (FP64 forward/backward of the 3-D CNN)."""
import numpy as np
import pytest
import torch
from scipy import ndimage

from oracle import cnn


def tiny(seed, n=2, T=3, Y=3, X=4):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, T, Y, X, cnn.C_IN))
    theta = cnn.init_params(seed)
    theta += rng.normal(0, 0.05, theta.size)          # non-zero biases
    labels = rng.integers(0, 2, n).astype(np.float64)
    return x, theta, labels


def test_parameter_count():
    assert cnn.n_params() == 97985


def test_conv_matches_brute_force_and_scipy():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, 3, 4, 5, 2))
    W = rng.standard_normal((3, 27, 2))
    b = rng.standard_normal(3)
    out = cnn.conv3(x, W, b)
    # brute force from the definition
    ref = np.zeros_like(out)
    for co in range(3):
        for t in range(3):
            for y in range(4):
                for xx in range(5):
                    acc = b[co]
                    for tap in range(27):
                        kt, ky, kx = tap // 9, (tap // 3) % 3, tap % 3
                        tt, yy, xz = t + kt - 1, y + ky - 1, xx + kx - 1
                        if 0 <= tt < 3 and 0 <= yy < 4 and 0 <= xz < 5:
                            acc += W[co, tap, :] @ x[0, tt, yy, xz, :]
                    ref[0, t, y, xx, co] = acc
    np.testing.assert_allclose(out, ref, atol=1e-12)
    # scipy's N-d correlation with zero padding, summed over input channels
    for co in range(3):
        s = sum(ndimage.correlate(x[0, ..., ci], W[co, :, ci].reshape(3, 3, 3), mode="constant", cval=0.0)
                for ci in range(2))
        np.testing.assert_allclose(out[0, ..., co], s + b[co], atol=1e-12)


def test_bce_matches_torch():
    z = np.array([-30.0, -2.0, -0.1, 0.0, 0.3, 5.0, 40.0])
    y = np.array([0, 1, 1, 0, 1, 0, 1], dtype=np.float64)
    ref = torch.nn.functional.binary_cross_entropy_with_logits(torch.tensor(z), torch.tensor(y)).item()
    assert cnn.bce_logits(z, y) == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_central_differences(seed):
    x, theta, labels = tiny(seed)
    loss, g, _ = cnn.loss_and_grad(theta, x, labels)
    rng = np.random.default_rng(100 + seed)
    sizes = [int(np.prod(s)) for s in cnn.param_shapes()]
    starts = np.cumsum([0] + sizes[:-1])
    idx = []
    for st, sz in zip(starts, sizes):                # a few entries of every tensor
        idx += list(st + rng.choice(sz, size=min(sz, 4), replace=False))
    h = 1e-5
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        num = (cnn.loss_and_grad(tp, x, labels)[0] - cnn.loss_and_grad(tm, x, labels)[0]) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 + 1e-5 * abs(num), (i, num, g[i])


def test_input_gradient_through_all_layers():
    """d loss / d x via the chain of conv backward passes, against differences."""
    x, theta, labels = tiny(3, n=1)
    P = cnn.unpack(theta)
    f = cnn.forward(theta, x)
    loss0 = cnn.bce_logits(f["z"], labels)

    def loss_at(xx):
        return cnn.bce_logits(cnn.forward(theta, xx)["z"], labels)

    # analytic dx: rerun the backward keeping the layer-1 input gradient
    y = labels
    dz = (1 / (1 + np.exp(-f["z"])) - y) / y.size
    du = np.outer(dz, P[10]) * (f["u"] > 0)
    dh = du @ P[8]
    a4 = f["acts"][4]
    dpost = np.broadcast_to((dh / np.prod(a4.shape[1:4]))[:, None, None, None, :], a4.shape)
    for l in (3, 2, 1, 0):
        dpre = dpost * (f["acts"][l + 1] > 0)
        _, _, dpost = cnn.conv3_backward(f["acts"][l], P[2 * l], dpre, need_dx=True)
    rng = np.random.default_rng(4)
    for _ in range(6):
        i = tuple(rng.integers(0, s) for s in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[i] += 1e-5
        xm[i] -= 1e-5
        num = (loss_at(xp) - loss_at(xm)) / 2e-5
        assert abs(num - dpost[i]) <= 1e-7 + 1e-5 * abs(num)
    assert np.isfinite(loss0)


def test_bf16_rounding_points_change_little():
    x, theta, labels = tiny(5)
    l0, g0, _ = cnn.loss_and_grad(theta, x, labels)
    l1, g1, _ = cnn.loss_and_grad(theta, x, labels, bf16_points=True)
    assert abs(l0 - l1) < 2e-2
    assert np.linalg.norm(g1 - g0) < 0.15 * np.linalg.norm(g0)
    v = np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 3.14159])
    np.testing.assert_array_equal(cnn.bf16(v), torch.tensor(v, dtype=torch.float32).to(torch.bfloat16).double().numpy())
