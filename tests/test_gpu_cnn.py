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
