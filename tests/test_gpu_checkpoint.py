"""GPU tests of classifier checkpoints (training with Adam, section 2.3, resumed).

2N Adam steps on one classifier must equal N steps, a checkpoint, a fresh
classifier that loads it, and N more steps, bit for bit (weights and both Adam
moments; the step count drives the bias corrections). Malformed checkpoints are
refused without changing the classifier.
"""
import ctypes

import numpy as np
import pytest

from paper_2510_18136_amd import nsfrb
from tests._lib import ensure_built

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N, T, Y = 2, 8, 8


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()
    assert torch.cuda.is_available()


def batch(step):
    """Seeded BF16 cutouts and labels of one step (the same for every run)."""
    rng = np.random.default_rng(1000 + step)
    x = rng.standard_normal((N, T, Y, 32, 16)).astype(np.float32)
    bits = (x.view(np.uint32) >> 16).astype(np.uint16)          # truncation to BF16 is fine for inputs
    y = rng.integers(0, 2, N).astype(np.float32)
    return torch.from_numpy(bits.view(np.int16)).cuda(), torch.from_numpy(y).cuda()


def run_steps(c, first, count):
    for k in range(first, first + count):
        x, y = batch(k)
        c.set_lr(1e-3 * (1.0 - 0.1 * k))            # a schedule, so the saved lr matters
        c.train_step(x.data_ptr(), y.data_ptr(), N, update=True, want_loss=False,
                     stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()


def test_resume_from_checkpoint_is_bit_exact(tmp_path):
    steps = 3
    print("[gpu] classifier checkpoint: 2N steps straight", flush=True)
    with nsfrb.Classifier(max_batch=N, n_time=T, ny=Y, seed=5) as a:
        run_steps(a, 0, 2 * steps)
        ref_params, ref_state = a.params(), a.state(user_counter=2 * steps)
    print("[gpu] classifier checkpoint: N steps, save, load into a fresh classifier, N steps", flush=True)
    with nsfrb.Classifier(max_batch=N, n_time=T, ny=Y, seed=5) as b:
        run_steps(b, 0, steps)
        b.save(str(tmp_path / "ck.bin"), user_counter=steps)
    with nsfrb.Classifier(max_batch=N, n_time=T, ny=Y, seed=99) as c:   # other initial weights
        assert c.load(str(tmp_path / "ck.bin")) == steps
        run_steps(c, steps, steps)
        params, state = c.params(), c.state(user_counter=2 * steps)
    assert np.array_equal(params.view(np.uint32), ref_params.view(np.uint32))
    assert state == ref_state                        # moments, step count and settings too


def test_malformed_checkpoints_are_refused():
    with nsfrb.Classifier(max_batch=N, n_time=T, ny=Y, seed=5) as c:
        before = c.params()
        blob = bytearray(c.state())
        n = int(nsfrb.lib().nsfrb_classifier_state_bytes())
        assert len(blob) == n == 56 + 3 * 4 * c.n_params
        for bad in (bytes(blob[:-4]), b"X" + bytes(blob[1:])):
            with pytest.raises(nsfrb.NsfrbError) as e:
                c.load_state(bad)
            assert e.value.status == nsfrb.INVALID_ARG
        # a checkpoint of another cutout shape
        with nsfrb.Classifier(max_batch=N, n_time=2 * T, ny=Y, seed=5) as other:
            with pytest.raises(nsfrb.NsfrbError) as e:
                other.load_state(bytes(blob))
            assert e.value.status == nsfrb.INVALID_ARG
        assert np.array_equal(c.params().view(np.uint32), before.view(np.uint32))
        # capacity too small: TRUNCATED, with the needed size reported
        small = np.zeros(16, np.uint8)
        written = ctypes.c_int64(0)
        st = nsfrb.lib().nsfrb_classifier_save(c.h, ctypes.c_uint64(0), small.ctypes.data_as(ctypes.c_void_p), 16,
                                               ctypes.byref(written))
        assert st == nsfrb.TRUNCATED and written.value == n


def test_training_driver_resumes_bit_exact(tmp_path):
    """The training driver stopped after one round of cubes and resumed from its
    checkpoint ends with the weights of an uninterrupted run."""
    from paper_2510_18136_amd import train_classifier as tc
    n_train, seed = 300, 7
    print("[gpu] training driver: uninterrupted run", flush=True)
    with nsfrb.Classifier(max_batch=64, n_time=tc.CUT_T, ny=32, seed=3) as a:
        tr = tc.train(a, n_train, seed=seed, log=lambda m: None)
        ref = a.params()
    assert tr["cutouts"] == n_train
    ck = str(tmp_path / "ck.bin")
    print("[gpu] training driver: one round, stop, resume", flush=True)
    with nsfrb.Classifier(max_batch=64, n_time=tc.CUT_T, ny=32, seed=3) as b:
        part = tc.train(b, n_train, seed=seed, log=lambda m: None, ckpt=ck, stop_after_rounds=1)
    assert 0 < part["cutouts"] < n_train
    with nsfrb.Classifier(max_batch=64, n_time=tc.CUT_T, ny=32, seed=11) as c:
        rest = tc.train(c, n_train, seed=seed, log=lambda m: None, ckpt=ck, resume=True)
        got = c.params()
    assert rest["cutouts"] == n_train and rest["steps"] == tr["steps"]
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
