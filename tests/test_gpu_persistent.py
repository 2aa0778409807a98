"""GPU tests of every search kernel form, each forced in turn (needs an MI355X).

The per-DM kernel and the persistent kernel (one pixel per workgroup at a time,
the next pixel's rows fetched during the current one), with 16 and with 8
waves, must give maps, per-pixel best trials and candidates bitwise equal to
each other: they sum in the same order and differ only in which wave does
what, when. The per-DM results are held to the oracle. Shapes cover one, two and three DM
rounds per wave, pixel counts that are not multiples of the 32-pixel chunks,
one and two LDS buffers, and FP32 and FP16 stores.
"""
import numpy as np
import pytest

from oracle.delays import delay_table
from paper_2510_18136_amd import nsfrb, synth
from tests._lib import ensure_built
from tests.test_gpu_search import compare, oracle_run, run_gpu

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FREQS = np.linspace(1.311, 1.499, 16)


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()
    assert torch.cuda.is_available()


def pulsed_cube(nt, npix, seed):
    cube = synth.noise_cube(nt, 16, npix, seed=seed)
    rng = np.random.default_rng(seed)
    for p in rng.choice(npix, size=12, replace=False):
        dm = float(rng.uniform(0, 4000))
        off = delay_table(FREQS, FREQS.max(), 134.2, [dm])[0]
        w = int(rng.choice([1, 3, 16, 100]))
        synth.inject_boxcar(cube, int(p), int(rng.integers(0, nt - int(off.max()) - w)), off, w, 2.0)
    return cube


def forms(monkeypatch, cfg, cube):
    """Results of each kernel form the plan offers, keyed by form."""
    out = {}
    for mode in ("0", "16", "8"):
        monkeypatch.setenv("NSFRB_PERSISTENT", mode)
        with nsfrb.Search(cfg) as s:
            info = s.plan_info()
        if info["persistent"] != (mode != "0"):
            continue                     # this shape has no such kernel (e.g. 16 waves with fewer DMs)
        if mode != "0":
            assert info["threads_per_workgroup"] == 64 * int(mode)
        print(f"[gpu] form {mode}: {info}", flush=True)
        out[mode] = run_gpu(cube, cfg)
    monkeypatch.delenv("NSFRB_PERSISTENT")
    return out


@pytest.mark.parametrize("n_dm,nx,ny,nt,store", [(32, 47, 45, 512, "f32"), (8, 33, 31, 512, "f32"),
                                                 (40, 40, 40, 512, "f32"), (32, 45, 47, 512, "f16"),
                                                 (32, 33, 31, 2048, "f32")])
def test_every_kernel_form_gives_the_same_results(monkeypatch, n_dm, nx, ny, nt, store):
    """(2048 samples in FP32: one LDS buffer, the next pixel's rows requested
    after the last de-dispersion; 512 samples: two buffers.)"""
    cube = pulsed_cube(nt, nx * ny, seed=n_dm + nx)
    widths = [1, 2, 4, 8, 16, 64, 100, 256]
    cfg = nsfrb.SearchConfig(nx, ny, nt, FREQS, np.linspace(0, 4000, n_dm), widths, store_dtype=store,
                             snr_threshold=6.0, max_candidates=64)
    res = forms(monkeypatch, cfg, cube)
    assert "0" in res and len(res) >= 2, sorted(res)
    ref = res["0"]
    for mode, g in res.items():
        assert np.array_equal(g["snr"], ref["snr"], equal_nan=True), mode
        assert np.array_equal(g["toa"], ref["toa"]), mode
        for key in ("best", "best_d", "best_w", "best_t"):
            assert np.array_equal(g[key], ref[key], equal_nan=True), (mode, key)
        assert g["cands"] == ref["cands"] and g["n_total"] == ref["n_total"], mode
    if store == "f32" and nt <= 512:
        compare(ref, oracle_run(cube, cfg), cfg)
