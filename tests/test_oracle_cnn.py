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
    # 4 conv layers (27 taps x cin x 32 + 32) + fc1 64 -> 32 + fc2 32 -> 1
    assert cnn.n_params() == (27 * 16 * 32 + 32) + 3 * (27 * 32 * 32 + 32) + (64 * 32 + 32) + (32 + 1) == 99009


def test_head_features_by_brute_force():
    """h = [per-channel maximum (first position on ties), features at the centre]."""
    x, theta, _ = tiny(8, n=2, T=4, Y=4, X=6)
    f = cnn.forward(theta, x)
    a4 = f["acts"][4]
    n, T, Y, X, C = a4.shape
    for i in range(n):
        for c in range(C):
            best, pos = -np.inf, None
            for t in range(T):
                for y in range(Y):
                    for xx in range(X):
                        if a4[i, t, y, xx, c] > best:
                            best, pos = a4[i, t, y, xx, c], (t * Y + y) * X + xx
            assert f["h"][i, c] == best and f["arg"][i, c] == pos
            assert f["h"][i, C + c] == a4[i, 2, 2, 3, c]


def test_pool_backward_ties_go_to_the_first_position():
    a4 = np.zeros((1, 2, 2, 2, 3))
    a4[0, 0, 1, 1, 0] = a4[0, 1, 0, 0, 0] = 2.0            # tie in channel 0
    a4[0, 1, 1, 1, 1] = 1.0
    flat = a4.reshape(1, 8, 3)
    arg = np.argmax(flat, axis=1)
    d = cnn.pool_backward(a4.shape, arg, np.arange(1.0, 7.0)[None, :])
    want = np.zeros_like(a4)
    want[0, 0, 1, 1, 0] += 1.0                                # first of the tied maxima, (t, y, x) order
    want[0, 1, 1, 1, 1] += 2.0
    want[0, 0, 0, 0, 2] += 3.0                                # all-equal channel: position 0
    want[0, 1, 1, 1, :] += [4.0, 5.0, 6.0]                    # centre (T/2, Y/2, X/2) = (1, 1, 1)
    np.testing.assert_array_equal(d, want)


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
    """d loss / d x through the head, the pool and every conv backward pass, against differences."""
    x, theta, labels = tiny(3, n=1)
    _, _, _, dx = cnn.loss_and_grad(theta, x, labels, input_grad=True)

    def loss_at(xx):
        return cnn.bce_logits(cnn.forward(theta, xx)["z"], labels)

    rng = np.random.default_rng(4)
    checked = 0
    for _ in range(40):
        i = tuple(rng.integers(0, s) for s in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[i] += 1e-6
        xm[i] -= 1e-6
        num = (loss_at(xp) - loss_at(xm)) / 2e-6
        assert abs(num - dx[i]) <= 1e-7 + 1e-5 * abs(num), (i, num, dx[i])
        checked += dx[i] != 0
    assert checked >= 5                          # the path reaches the input


def test_bf16_rounding_points_change_little():
    x, theta, labels = tiny(5)
    l0, g0, _ = cnn.loss_and_grad(theta, x, labels)
    l1, g1, _ = cnn.loss_and_grad(theta, x, labels, bf16_points=True)
    assert abs(l0 - l1) < 2e-2
    assert np.linalg.norm(g1 - g0) < 0.15 * np.linalg.norm(g0)
    v = np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 3.14159])
    np.testing.assert_array_equal(cnn.bf16(v), torch.tensor(v, dtype=torch.float32).to(torch.bfloat16).double().numpy())
