"""GPU tests of the candidate classifier (needs an MI355X).

* gradients of one BF16 MFMA training step against the FP64 oracle with the
  same BF16 rounding points, per parameter tensor (reduced cutouts, t x y x 32
  with t x y from 4 x 4 to 40 x 8);
* the first Adam step against its closed form;
* inference probabilities against the oracle's sigmoid(logit);
* cutout extraction against its definition written out in NumPy;
* a small batch is memorised (loss falls), as a training smoke check.
Inputs are generated on the host from seeds; nothing the oracle sees comes
from the GPU.
"""
import numpy as np
import pytest

from oracle import cnn
from oracle.delays import delay_table
from paper_2510_18136_amd import nsfrb, synth
from tests._lib import ensure_built

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()
    assert torch.cuda.is_available()


def bf16_device(x):
    bits = (np.ascontiguousarray(cnn.bf16(x).astype(np.float32)).view(np.uint32) >> 16).astype(np.uint16)
    return torch.from_numpy(bits.view(np.int16)).cuda()


def make_case(seed, n=3, T=4, Y=4):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, T, Y, 32, 16))
    theta = cnn.init_params(seed).astype(np.float32).astype(np.float64)
    theta = theta + rng.normal(0, 0.02, theta.size).astype(np.float32)
    theta = theta.astype(np.float32).astype(np.float64)
    labels = rng.integers(0, 2, n).astype(np.float64)
    return x, theta, labels


def tensor_slices():
    sizes = [int(np.prod(s)) for s in cnn.param_shapes()]
    starts = np.cumsum([0] + sizes)
    names = [f"conv{l}.{k}" for l in range(1, 5) for k in ("W", "b")] + ["fc1.W", "fc1.b", "fc2.w", "fc2.b"]
    return [(nm, slice(starts[i], starts[i + 1])) for i, nm in enumerate(names)]


# the larger cutouts split the pooling pass over several position chunks (the
# last one ragged): 4 x 4 -> one chunk, 16 x 8 -> 4, 13 x 5 -> 3 uneven, 40 x 8 -> 10
@pytest.mark.parametrize("seed,n,T,Y", [(0, 3, 4, 4), (1, 3, 4, 4), (2, 2, 16, 8), (6, 2, 13, 5), (7, 1, 40, 8)])
def test_gradients_match_oracle(seed, n, T, Y):
    x, theta, labels = make_case(seed, n=n, T=T, Y=Y)
    n, T, Y = x.shape[:3]
    with nsfrb.Classifier(max_batch=n, n_time=T, ny=Y, lr=0.0) as c:
        c.set_params(theta)
        xd = bf16_device(x)
        yd = torch.from_numpy(labels.astype(np.float32)).cuda()
        print(f"[gpu] classifier grad check seed={seed} n={n} T={T} Y={Y}", flush=True)
        loss = c.train_step(xd.data_ptr(), yd.data_ptr(), n, update=False,
                            stream=torch.cuda.current_stream().cuda_stream)
        g = c.grads().astype(np.float64)
    l_ref, g_ref, _ = cnn.loss_and_grad(theta, x, labels, bf16_points=True)
    assert abs(loss - l_ref) <= 1e-3 * max(1.0, abs(l_ref))
    bad = []
    for name, sl in tensor_slices():
        err = np.linalg.norm(g[sl] - g_ref[sl])
        ref = np.linalg.norm(g_ref[sl])
        print(f"{name:10s} |g-g_ref| = {err:.3e}  |g_ref| = {ref:.3e}", flush=True)
        if not err <= 2e-2 * ref + 1e-6:
            bad.append(name)
    assert not bad, bad


def test_first_adam_step_closed_form():
    x, theta, labels = make_case(3, n=2)
    lr, eps = 1e-3, 1e-8
    with nsfrb.Classifier(max_batch=2, n_time=4, ny=4, lr=lr, eps=eps) as c:
        c.set_params(theta)
        xd, yd = bf16_device(x), torch.from_numpy(labels.astype(np.float32)).cuda()
        c.train_step(xd.data_ptr(), yd.data_ptr(), 2, update=True, stream=torch.cuda.current_stream().cuda_stream)
        g = c.grads().astype(np.float64)
        after = c.params().astype(np.float64)
    # step 1: m_hat = g, v_hat = g^2  =>  delta = -lr * g / (|g| + eps)
    expect = theta - lr * g / (np.abs(g) + eps)
    np.testing.assert_allclose(after, expect, rtol=0, atol=1e-6)


def test_inference_matches_oracle():
    x, theta, _ = make_case(4, n=5)
    with nsfrb.Classifier(max_batch=5, n_time=4, ny=4) as c:
        c.set_params(theta)
        xd = bf16_device(x)
        prob = torch.zeros(5, device="cuda")
        c.infer(xd.data_ptr(), 5, prob.data_ptr(), stream=torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        p = prob.cpu().numpy().astype(np.float64)
    z = cnn.forward(theta, x, bf16_points=True)["z"]
    np.testing.assert_allclose(p, 1 / (1 + np.exp(-z)), atol=2e-3)


def test_cutouts_match_definition():
    rng = np.random.default_rng(6)
    nx = ny = 40
    ns, nt, ct = 16, 160, 64
    freqs = np.linspace(1.311, 1.499, ns)
    delays = delay_table(freqs, freqs.max(), 134.2, np.linspace(0, 1000, 8))
    cubes = [rng.standard_normal((nx * ny, ns, nt)).astype(np.float16) for _ in range(2)]
    zd = [torch.from_numpy(c.ravel()).cuda() for c in cubes]
    descs = [(0, 3, 37, 5, 40), (1, 20, 20, 7, 130), (1, 0, 0, 0, 10), (0, 39, 0, 3, 150)]
    out = torch.zeros(len(descs) * ct * 32 * 32 * 16, dtype=torch.int16, device="cuda")
    with nsfrb.Classifier(max_batch=4, n_time=ct, ny=32) as c:
        c.cutouts([z.data_ptr() for z in zd], "f16", nx, ny, ns, nt, delays, descs, out.data_ptr(),
                  stream=torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
    got = (out.cpu().numpy().view(np.uint16).astype(np.uint32) << 16).view(np.float32).reshape(len(descs), ct, 32, 32, 16)
    for k, (cube, px, py, d, toa) in enumerate(descs):
        z = cubes[cube]
        ref = np.zeros((ct, 32, 32, 16), np.float32)
        for tt in range(ct):
            for y in range(32):
                for x in range(32):
                    xi, yi = px + x - 16, py + y - 16
                    if not (0 <= xi < nx and 0 <= yi < ny):
                        continue
                    for s in range(ns):
                        t = toa - ct // 2 + tt + delays[d, s]
                        if 0 <= t < nt:
                            ref[tt, y, x, s] = float(z[yi * nx + xi, s, t])
        np.testing.assert_array_equal(got[k], cnn.bf16(ref).astype(np.float32))


def test_memorises_a_small_batch():
    rng = np.random.default_rng(7)
    n = 16
    x = rng.standard_normal((n, 8, 4, 32, 16))
    labels = (np.arange(n) % 2).astype(np.float32)
    x[labels == 0, 3:5, :, 10:14, :] += 2.0            # a pulse-like blob for one class
    with nsfrb.Classifier(max_batch=n, n_time=8, ny=4, lr=3e-3, seed=5) as c:
        xd, yd = bf16_device(x), torch.from_numpy(labels).cuda()
        st = torch.cuda.current_stream().cuda_stream
        first = c.train_step(xd.data_ptr(), yd.data_ptr(), n, stream=st)
        for _ in range(60):
            last = c.train_step(xd.data_ptr(), yd.data_ptr(), n, stream=st)
    assert np.isfinite(first) and last < 0.2 * first


U_F32 = 2.0 ** -24          # FP32 unit roundoff


def bf16_ulp(v):
    """Spacing of BF16 numbers at |v|: 2^(floor(log2 |v|) - 7) (0 for v = 0)."""
    a = np.abs(v)
    return np.where(a > 0, np.exp2(np.floor(np.log2(np.maximum(a, 1e-300))) - 7), 0.0)


def rounding_bound(terms):
    """Worst-case error of an FP32 sum of `terms` products: terms * u * sum|products|."""
    return terms * U_F32


def check_rounded(name, got, ref, abs_sum, terms, min_equal=0.999):
    """got = BF16(FP32 sum), ref = BF16(FP64 sum) of the same inputs: they may
    differ only where the sum lies within the FP32 error of a BF16 rounding
    boundary, by at most one BF16 spacing plus that error."""
    d = np.abs(got - ref)
    allow = bf16_ulp(np.maximum(np.abs(got), np.abs(ref))) + rounding_bound(terms) * abs_sum
    equal = float((got == ref).mean())
    print(f"{name}: bit-equal {equal:.5f}, max |d| {d.max():.3e}, worst d/allow {(d / np.maximum(allow, 1e-300)).max():.3f}",
          flush=True)
    assert (d <= allow).all(), name
    assert equal >= min_equal, name


def test_real_cutout_shape_layer_by_layer():
    """The workload's cutout shape (64 x 32 x 32 x 16, two cutouts), so the conv
    row blocks beyond the first (and their halos) and the full pooling pass run.

    Each stage is checked element by element against the FP64 oracle fed with
    the GPU's own inputs to that stage (a flip in one layer would otherwise
    cascade into the next): every conv layer's BF16 output, every back-propagated
    BF16 pre-activation gradient, every weight and bias gradient, the logits of
    training and of inference, and the probabilities. The bounds come from the
    arithmetic: one BF16 spacing where the GPU's FP32 sum and the oracle's FP64
    sum round differently, plus the worst-case FP32 error of the sum
    (terms x 2^-24 x sum of |products|, computed by the oracle on absolute
    values). The end-to-end activations (oracle on its own inputs throughout)
    are reported, their flips cascading through the layers."""
    n, T, Y = 2, 64, 32
    x, theta, labels = make_case(11, n=n, T=T, Y=Y)
    P = cnn.unpack(theta)
    with nsfrb.Classifier(max_batch=n, n_time=T, ny=Y, lr=0.0) as c:
        c.set_params(theta)
        xd = bf16_device(x)
        yd = torch.from_numpy(labels.astype(np.float32)).cuda()
        print(f"[gpu] classifier at the real cutout shape n={n} T={T} Y={Y}", flush=True)
        c.train_step(xd.data_ptr(), yd.data_ptr(), n, update=False, want_loss=False,
                     stream=torch.cuda.current_stream().cuda_stream)
        g = c.grads().astype(np.float64)
        acts = [cnn.bf16(x)] + [c.activations(l, n).astype(np.float64) for l in range(1, 5)]
        dpre = [None] + [c.grad_pre(l, n).astype(np.float64) for l in range(1, 5)]
        z_train = c.logits(n).astype(np.float64)
        prob = torch.zeros(n, device="cuda")
        c.infer(xd.data_ptr(), n, prob.data_ptr(), stream=torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        p = prob.cpu().numpy().astype(np.float64)
        z_inf = c.logits(n).astype(np.float64)
    print("[gpu] FP64 oracle, stage by stage on the GPU's inputs (about a minute)", flush=True)
    # forward, layer by layer
    for l in range(4):
        W, b = cnn.bf16(P[2 * l]), P[2 * l + 1]
        ref = cnn.bf16(np.maximum(cnn.conv3(acts[l], W, b), 0.0))
        abs_sum = cnn.conv3(np.abs(acts[l]), np.abs(W), np.abs(b))
        check_rounded(f"a{l + 1}", acts[l + 1], ref, abs_sum, 27 * W.shape[2] + 1)
    # head on the GPU's a4: logits (training and inference) and probabilities
    f = cnn.head_forward(theta, acts[4])
    zb = 1e-5 * (1.0 + (np.abs(f["h"]) @ np.abs(P[8]).T + np.abs(P[9])) @ np.abs(P[10]) + abs(P[11][0]))
    for name, z in (("train", z_train), ("infer", z_inf)):
        dz = np.abs(z - f["z"])
        print(f"logits ({name}): max |dz| {dz.max():.3e} (bound {zb.min():.3e})", flush=True)
        assert (dz <= zb).all(), name
    np.testing.assert_allclose(p, 1.0 / (1.0 + np.exp(-z_inf)), rtol=0, atol=1e-6)
    # backward: the head's gradients and d(loss)/d(a4), then each layer on the GPU's pre-activation gradient
    f["acts"] = acts
    _, head_g, dpost = cnn.head_backward(theta, f, labels)
    sl = dict(tensor_slices())
    for name, ref in zip(("fc1.W", "fc1.b", "fc2.w", "fc2.b"), head_g):
        d = np.abs(g[sl[name]] - ref.ravel())
        allow = 1e-5 * (np.abs(ref.ravel()) + np.sqrt(np.mean(ref ** 2))) + 1e-9
        print(f"{name:10s} max |d| {d.max():.3e}  worst d/allow {(d / allow).max():.3f}", flush=True)
        assert (d <= allow).all(), name
    # |d(loss)/d(a4)| bound: the head's backward on absolute values; 128 terms cover the FP32
    # sums of the head (64 + 32) and the logit's own FP32 error entering sigmoid(z) - label
    du_abs = np.abs(np.outer((1.0 / (1.0 + np.exp(-f["z"])) - labels) / n, P[10])) * (f["u"] > 0)
    adpost = cnn.pool_backward(acts[4].shape, f["arg"], du_abs @ np.abs(P[8]))
    check_rounded("dpre4", dpre[4], cnn.bf16(dpost * (acts[4] > 0)), adpost, 128)
    for l in (3, 2, 1, 0):
        W = cnn.bf16(P[2 * l])
        dW, db, dx = cnn.conv3_backward(acts[l], W, dpre[l + 1], need_dx=l > 0)
        aW, ab, adx = cnn.conv3_backward(np.abs(acts[l]), np.abs(W), np.abs(dpre[l + 1]), need_dx=l > 0)
        n_pos = n * T * Y * 32
        for name, got, ref, a in ((f"conv{l + 1}.W", g[sl[f"conv{l + 1}.W"]], dW.ravel(), aW.ravel()),
                                  (f"conv{l + 1}.b", g[sl[f"conv{l + 1}.b"]], db.ravel(), ab.ravel())):
            d = np.abs(got - ref)
            allow = rounding_bound(n_pos) * a + 1e-12
            print(f"{name:10s} max |d| {d.max():.3e}  max rel {(d / np.maximum(np.abs(ref), 1e-30)).max():.3e}  "
                  f"worst d/allow {(d / allow).max():.3f}", flush=True)
            assert (d <= allow).all(), name
        if l > 0:
            check_rounded(f"dpre{l}", dpre[l], cnn.bf16(dx * (acts[l] > 0)), adx, 27 * 32)
    # end to end (the oracle on its own inputs throughout), for the record
    _, g_ref, fo = cnn.loss_and_grad(theta, x, labels, bf16_points=True)
    for l in range(1, 5):
        print(f"end to end a{l}: bit-equal {float((acts[l] == fo['acts'][l]).mean()):.5f}", flush=True)
    for name, s_ in tensor_slices():
        rel = np.linalg.norm(g[s_] - g_ref[s_]) / max(np.linalg.norm(g_ref[s_]), 1e-30)
        print(f"end to end {name:10s} relative L2 {rel:.3e}", flush=True)
