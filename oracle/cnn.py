"""Candidate classifier, forward and backward in FP64 (oracle; test infrastructure).

Paper section 2.3 classifies candidates with a CNN over the image cube
centred on the TOA (position, time, frequency): convolution blocks with
nonlinearities and max-pooling, a small fully connected head, a single logit
whose sigmoid is the RFI probability, trained with Adam on a binary
cross-entropy loss. The network here has the fixed shape of the workload this
project targets:

  input   x[n][t][y][x][s]           64 x 32 x 32 samples, 16 sub-bands as channels
  conv_l  a_l = relu(b_l + sum_{tap, ci} W_l[co][tap][ci] * a_{l-1}[pos + tap - 1][ci])
          3x3x3 taps over (t, y, x), zero padding, 32 output channels, l = 1..4
  pool    m[n][c] = max over (t, y, x) of a_4 (ties: first position in (t, y, x) order)
          q[n][c] = a_4 at the candidate's own position (T/2, Y/2, X/2): the cutout
                    puts the candidate's TOA at sample T/2 and its pixel at the centre
          h = [m, q]                 (64 features)
  fc1     r = relu(W1 h + c1)   (64 -> 32)
  fc2     z = w2 . r + c2        (32 -> 1), p_rfi = sigmoid(z)
  loss    mean_n [max(z, 0) - z*label + log(1 + exp(-|z|))]

The global max pool follows the paper's max-pooling; the candidate-position
features are there because any global pool is blind to where in the cutout a
feature sits, so it cannot tell a source at the centre from a bright source
beside a faint sidelobe copy at the centre.

Parameters are one flat FP32 vector in the order
  W_1[32][27][16], b_1[32], W_2[32][27][32], b_2[32], W_3, b_3, W_4, b_4,
  W1[32][64], c1[32], w2[32], c2[1]   (99,009 values),
with tap index kt*9 + ky*3 + kx.

`bf16=True` reproduces the rounding points of the GPU path: inputs, conv
weights, every stored activation a_l and every back-propagated pre-activation
gradient into a convolution are rounded to BF16 (round to nearest even);
everything else stays FP64. With bf16=False the network is exact FP64, which
the finite-difference pins check.
"""
import numpy as np

C_IN, C_HID, N_TAP = 16, 32, 27
LAYER_CIN = (C_IN, C_HID, C_HID, C_HID)


def param_shapes():
    shapes = []
    for cin in LAYER_CIN:
        shapes += [(C_HID, N_TAP, cin), (C_HID,)]
    shapes += [(C_HID, 2 * C_HID), (C_HID,), (C_HID,), (1,)]
    return shapes


def n_params():
    return int(sum(np.prod(s) for s in param_shapes()))


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = [], 0
    for s in param_shapes():
        n = int(np.prod(s))
        out.append(theta[o:o + n].reshape(s))
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def bf16(a):
    """Round to BF16 (nearest even), returned as float64 values."""
    a32 = np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))
    u = a32.view(np.uint32).astype(np.uint64)
    r = ((u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) >> np.uint64(16)) << np.uint64(16)
    out = (r & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(a32), np.nan, out)


def _shifted(x, kt, ky, kx):
    """x[n][t+kt-1][y+ky-1][x+kx-1][c] with zeros outside."""
    n, T, Y, X, c = x.shape
    p = np.zeros((n, T + 2, Y + 2, X + 2, c))
    p[:, 1:-1, 1:-1, 1:-1] = x
    return p[:, kt:kt + T, ky:ky + Y, kx:kx + X]


def conv3(x, W, b):
    """'Same' 3x3x3 convolution, channels last; W[co][tap][ci]."""
    out = np.zeros(x.shape[:4] + (W.shape[0],))
    for tap in range(N_TAP):
        kt, ky, kx = tap // 9, (tap // 3) % 3, tap % 3
        out += _shifted(x, kt, ky, kx) @ W[:, tap, :].T
    return out + b


def conv3_backward(x, W, dpre, need_dx=True):
    """Gradients of conv3 given d(loss)/d(pre-activation)."""
    n, T, Y, X, cin = x.shape
    dW = np.zeros_like(W)
    dx = np.zeros_like(x) if need_dx else None
    dpad = np.zeros((n, T + 2, Y + 2, X + 2, W.shape[0]))
    dpad[:, 1:-1, 1:-1, 1:-1] = dpre
    for tap in range(N_TAP):
        kt, ky, kx = tap // 9, (tap // 3) % 3, tap % 3
        xs = _shifted(x, kt, ky, kx)
        dW[:, tap, :] = np.einsum("ntyxo,ntyxc->oc", dpre, xs)
        if need_dx:
            # x[pos'] feeds out[pos' - tap + 1]
            dx += dpad[:, 2 - kt:2 - kt + T, 2 - ky:2 - ky + Y, 2 - kx:2 - kx + X] @ W[:, tap, :]
    return dW, dpre.sum(axis=(0, 1, 2, 3)), dx


def forward(theta, x, bf16_points=False):
    P = unpack(theta)
    rnd = bf16 if bf16_points else (lambda a: a)
    acts = [rnd(x)]
    for l in range(4):
        W, b = P[2 * l], P[2 * l + 1]
        acts.append(rnd(np.maximum(conv3(acts[-1], rnd(W), b), 0.0)))
    return dict(acts=acts, **head_forward(theta, acts[-1]))


def pool_backward(a4_shape, arg, dh):
    """d(loss)/d(a_4) from d(loss)/d(h): the max half goes to each channel's
    first maximum, the other half to the candidate position."""
    n, T, Y, X, C = a4_shape
    d = np.zeros((n, T * Y * X, C))
    for i in range(n):
        d[i, arg[i], np.arange(C)] += dh[i, :C]
    d = d.reshape(a4_shape)
    d[:, T // 2, Y // 2, X // 2, :] += dh[:, C:]
    return d


def bce_logits(z, y):
    return float(np.mean(np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z)))))


def head_backward(theta, f, labels):
    """From a forward record f (its h, u, r, z, arg and a_4): the mean BCE loss,
    the head's parameter gradients (W1, c1, w2, c2) and d(loss)/d(a_4)."""
    P = unpack(theta)
    y = np.asarray(labels, dtype=np.float64)
    n = y.size
    loss = bce_logits(f["z"], y)
    dz = (1.0 / (1.0 + np.exp(-f["z"])) - y) / n
    W1, w2 = P[8], P[10]
    g_w2 = f["r"].T @ dz
    g_c2 = np.array([dz.sum()])
    du = np.outer(dz, w2) * (f["u"] > 0)
    g_W1 = du.T @ f["h"]
    g_c1 = du.sum(axis=0)
    dh = du @ W1
    return loss, (g_W1, g_c1, g_w2, g_c2), pool_backward(f["acts"][4].shape, f["arg"], dh)


def head_forward(theta, a4):
    """The head on conv-4 outputs a4: the forward record fields h, u, r, z, arg."""
    P = unpack(theta)
    n, T, Y, X, C = a4.shape
    flat = a4.reshape(n, T * Y * X, C)
    arg = np.argmax(flat, axis=1)                      # first maximum along (t, y, x)
    m = np.take_along_axis(flat, arg[:, None, :], axis=1)[:, 0, :]
    q = a4[:, T // 2, Y // 2, X // 2, :]
    h = np.concatenate([m, q], axis=1)
    u = h @ P[8].T + P[9]
    r = np.maximum(u, 0.0)
    z = r @ P[10] + P[11][0]
    return dict(arg=arg, h=h, u=u, r=r, z=z)


def loss_and_grad(theta, x, labels, bf16_points=False, input_grad=False):
    """Mean BCE-with-logits loss and its gradient w.r.t. the flat parameters
    (and, with input_grad, w.r.t. the input cutouts as a fourth value)."""
    P = unpack(theta)
    rnd = bf16 if bf16_points else (lambda a: a)
    f = forward(theta, x, bf16_points)
    loss, head_grads, dpost = head_backward(theta, f, labels)
    grads = [None] * 12
    grads[8], grads[9], grads[10], grads[11] = head_grads
    for l in (3, 2, 1, 0):
        dpre = rnd(dpost * (f["acts"][l + 1] > 0))
        dW, db, dx = conv3_backward(f["acts"][l], rnd(P[2 * l]), dpre, need_dx=l > 0 or input_grad)
        grads[2 * l], grads[2 * l + 1] = dW, db
        dpost = dx
    if input_grad:
        return loss, pack(grads), f, dpost
    return loss, pack(grads), f


def init_params(seed):
    """He-uniform conv weights, small MLP weights, zero biases (host RNG)."""
    rng = np.random.default_rng(seed)
    parts = []
    for cin in LAYER_CIN:
        lim = np.sqrt(6.0 / (N_TAP * cin))
        parts += [rng.uniform(-lim, lim, (C_HID, N_TAP, cin)), np.zeros(C_HID)]
    lim1, lim2 = np.sqrt(6.0 / (2 * C_HID)), np.sqrt(6.0 / C_HID)
    parts += [rng.uniform(-lim1, lim1, (C_HID, 2 * C_HID)), np.zeros(C_HID),
              rng.uniform(-lim2, lim2, C_HID), np.zeros(1)]
    return pack(parts)
