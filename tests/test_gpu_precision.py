"""Precision forms of the search against an FP64 oracle on unquantised z (GPU).

The workload is the tiny search (32 x 32 pixels, 4 sub-bands, 64 samples,
8 DMs, widths 1-16; 40,960 S/N maxima per cube) with z stored in FP16 or BF16
after normalisation to unit sigma; sums are FP32 and the noise statistics FP64.

Two errors are separated:
  * accumulation: the GPU against the oracle given the same quantised z -- the
    kernels' own arithmetic, bound 1e-4;
  * total: the GPU against the FP64 oracle on unquantised z. Each maximum may
    move by at most the storage cast's error over its window plus the
    accumulation bound: |max_t S_q - max_t S| <= max_t sum_window |z_q - z| /
    sqrt(n_sub w) + 1e-4, the first term computed exactly by the oracle's own
    window sums applied to |z_q - z| (a bound from the arithmetic, not from a
    measurement).
  * the 1e-3 target for the total error: met by FP32; missed by FP16 (about
    1.3e-3 on noise, 1.9e-3 with a S/N 16 pulse: each maximum sits on the
    largest samples of its window, where FP16's spacing is widest) and by BF16.
    The miss is recorded as an expected failure that must keep failing
    (strict), not as a loosened bound.
  * candidate-set agreement: for every pixel whose best (DM, width) leads the
    runner-up by more than the form's margin in the FP64 oracle (1e-3 for FP32
    and FP16, 3e-2 for BF16), the GPU picks the same trial, and threshold
    membership agrees wherever |S/N - theta| exceeds that margin.
"""
import numpy as np
import pytest

from oracle import search as osr
from paper_2510_18136_amd import synth
from tests._lib import ensure_built
from tests.test_gpu_search import c1_cfg, dw_margin, oracle_run, run_gpu

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ACCUM = 1e-4          # the kernels' own accumulation error
TARGET = 1e-3         # stated target for the total error against FP64 on unquantised z
MARGIN = {"f32": 1e-3, "f16": 1e-3, "bf16": 3e-2}


def cast_bound(cube, meta, store):
    """Per maximum: max over windows of sum |z_store - z_fp64| / sqrt(n_sub w), in FP64."""
    x = cube.astype(np.float32).astype(np.float64)
    zq = osr.normalize(x, "pixel_subband", store)[0]
    z64 = osr.normalize(x, "pixel_subband", "f64")[0]
    delays = osr.delay_table(meta["freqs"], meta["f_ref"], meta["dt_ms"], meta["dms"])
    return osr.snr_toa_maps(np.abs(zq - z64), delays, meta["widths"])[0]


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()
    assert torch.cuda.is_available()


@pytest.mark.parametrize("store", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("seed,amp", [(0, 1.0), (1, 4.0)])
def test_precision_form_against_fp64(store, seed, amp):
    cube, meta = synth.config1(seed=seed, amp=amp)
    cfg = c1_cfg(store_dtype=store)
    g = run_gpu(cube, cfg)
    x = cube.astype(np.float32).astype(np.float64)
    o64 = osr.search(x, meta["freqs"], meta["f_ref"], meta["dt_ms"], meta["dms"], meta["widths"], meta["nx"],
                     store="f64")
    oq = oracle_run(cube, cfg)
    fin = np.isfinite(o64["snr_max"])
    assert np.array_equal(np.isfinite(g["snr"]), fin)
    d_total = np.abs(g["snr"][fin] - o64["snr_max"][fin])
    total = d_total.max()
    accum = np.abs(g["snr"][fin] - oq["snr_max"][fin]).max()
    cast_only = np.abs(oq["snr_max"][fin] - o64["snr_max"][fin]).max()
    print(f"[precision] store={store} seed={seed} amp={amp}: max|dS/N| vs FP64 {total:.3e} "
          f"(cast alone {cast_only:.3e}, accumulation {accum:.3e}) over {fin.sum()} maxima", flush=True)
    assert accum <= ACCUM
    bound = cast_bound(cube, meta, store)[fin] + ACCUM
    assert (d_total <= bound).all()
    m = dw_margin(o64["snr_max"])
    clear = np.isfinite(o64["best"]) & (m > MARGIN[store])
    assert np.array_equal(g["best_d"][clear], o64["best_d"][clear])
    assert np.array_equal(g["best_w"][clear], o64["best_w"][clear])
    theta = 6.0
    sure = np.isfinite(o64["best"]) & (np.abs(o64["best"] - theta) > MARGIN[store])
    assert np.array_equal(g["best"][sure] >= theta, o64["best"][sure] >= theta)
    if amp > 1.0:
        assert (o64["best"] >= theta).any()                # a bright pulse makes a candidate


@pytest.mark.parametrize("store", [
    "f32",
    pytest.param("f16", marks=pytest.mark.xfail(strict=True, reason="FP16 storage alone moves S/N maxima by "
                                                "1.3e-3 to 1.9e-3: the 1e-3 target is missed")),
    pytest.param("bf16", marks=pytest.mark.xfail(strict=True, reason="BF16 storage moves S/N maxima by ~1e-2")),
])
def test_total_error_target(store):
    """The 1e-3 target on the total error, on noise and with a S/N 16 pulse."""
    worst = 0.0
    for seed, amp in ((0, 1.0), (1, 4.0)):
        cube, meta = synth.config1(seed=seed, amp=amp)
        g = run_gpu(cube, c1_cfg(store_dtype=store))
        x = cube.astype(np.float32).astype(np.float64)
        o64 = osr.search(x, meta["freqs"], meta["f_ref"], meta["dt_ms"], meta["dms"], meta["widths"], meta["nx"],
                         store="f64")
        fin = np.isfinite(o64["snr_max"])
        worst = max(worst, float(np.abs(g["snr"][fin] - o64["snr_max"][fin]).max()))
    print(f"[precision] store={store}: max |dS/N| vs FP64 on unquantised z = {worst:.3e} (target {TARGET})",
          flush=True)
    assert worst <= TARGET
