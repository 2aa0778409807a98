"""Pins for the oracle's de-dispersion / boxcar / S/N / candidate search.

Each test checks the oracle against something other than itself: brute-force
loops, exact integer arithmetic, closed forms for injected boxcars, the DM=0 /
width=1 identity, and N(0,1) statistics of the S/N on pure noise.
"""
import math

import numpy as np
import pytest

from oracle import brute
from oracle import search as osr
from oracle.delays import delay_table
from paper_2510_18136_amd import synth


def random_delays(rng, nd, ns, dmax):
    d = np.sort(rng.integers(0, dmax + 1, size=(nd, ns)), axis=1)[:, ::-1].copy()
    d[:, -1] = 0
    return d.astype(np.int32)


@pytest.mark.parametrize("seed", range(6))
def test_vectorised_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    nt, ns, npix = int(rng.integers(12, 33)), int(rng.integers(1, 5)), int(rng.integers(1, 9))
    z = rng.standard_normal((nt, ns, npix))
    delays = random_delays(rng, 3, ns, 6)
    widths = [1, 2, 3, 5, 8]
    smax, toa = osr.snr_toa_maps(z, delays, widths)
    bs, bt = brute.dedisperse_boxcar_brute(z.tolist(), delays.tolist(), widths)
    np.testing.assert_allclose(smax, np.array(bs), rtol=0, atol=1e-12)
    np.testing.assert_array_equal(toa, np.array(bt))
    best, bd, bw, btoa = osr.best_per_pixel(smax, toa)
    for p, (b, d, w, t) in enumerate(brute.best_brute(bs, bt)):
        assert (bd[p], bw[p], btoa[p]) == (d, w, t)
        assert best[p] == pytest.approx(b, abs=1e-12)


def test_integer_cube_sums_exact():
    rng = np.random.default_rng(11)
    z = rng.integers(-8, 9, size=(40, 4, 6)).astype(np.float64)
    delays = random_delays(rng, 4, 4, 7)
    widths = [1, 4, 7, 16]
    for d, D in enumerate(osr.dedisperse(z, delays)):
        for w in widths:
            B = osr.boxcar_sums(D, w)
            for t in range(B.shape[0]):
                for p in range(6):
                    exact = sum(int(z[t + k + delays[d, s], s, p]) for k in range(w) for s in range(4))
                    assert B[t, p] == exact


def closed_form_cube(A, w, t0, offsets, nt, ns, sigma):
    x = np.zeros((nt, ns, 1), dtype=np.float32)
    synth.inject_boxcar(x, 0, t0, offsets, w, A * sigma)
    return x


@pytest.mark.parametrize("A,w,sigma", [(1.0, 4, 1.0), (0.7, 13, 2.0), (3.0, 1, 0.5)])
def test_closed_form_injected_snr(A, w, sigma):
    """Noiseless injection with known statistics: S/N = A*sqrt(w*n_sub)/sigma (in units of sigma)."""
    ns, nt = 8, 96
    freqs = np.linspace(1.311, 1.499, ns)
    dms = np.linspace(0, 2000, 9)
    delays = delay_table(freqs, freqs.max(), 134.2, dms)
    d_true = 6
    x = closed_form_cube(A, w, 30, delays[d_true], nt, ns, sigma)
    med = np.zeros((1, ns))
    sig = np.full((1, ns), sigma)
    widths = [1, w, 2 * w]
    r = osr.search(x, freqs, freqs.max(), 134.2, dms, widths, 1, norm="external",
                   med=med, sigma=sig, theta=0.0)
    s = r["snr_max"]
    expect = A * math.sqrt(w * ns)            # amplitude A*sigma, noise sigma
    assert s[d_true, 1, 0] == pytest.approx(expect, rel=1e-6)
    assert r["toa"][d_true, 1, 0] == 30
    # width mismatch: A*n_sub*min(w, w')/sqrt(n_sub*w')  (w' = 1 and 2w)
    for iw, w2 in ((0, 1), (2, 2 * w)):
        assert s[d_true, iw, 0] == pytest.approx(A * ns * min(w, w2) / math.sqrt(ns * w2), rel=1e-6)
    # DM mismatch: integer-shift overlaps of the sub-band boxcars
    for d in range(len(dms)):
        best = -np.inf
        for t in range(nt - int(delays[d].max()) - w + 1):
            ov = 0
            for sb in range(ns):
                a = t + delays[d, sb]
                b = 30 + delays[d_true, sb]
                ov += max(0, min(a + w, b + w) - max(a, b))
            best = max(best, A * ov / math.sqrt(ns * w))
        assert s[d, 1, 0] == pytest.approx(best, rel=1e-6)
    assert s[d_true, 1, 0] <= r["best"][0]


def test_dm0_width1_identity():
    rng = np.random.default_rng(7)
    z = rng.standard_normal((50, 4, 9))
    delays = np.vstack([np.zeros(4, np.int32), np.array([3, 2, 1, 0], np.int32)])
    smax, toa = osr.snr_toa_maps(z, delays, [1, 2])
    s = z.sum(axis=1) / 2.0
    np.testing.assert_allclose(smax[0, 0], s.max(axis=0), atol=1e-14)
    np.testing.assert_array_equal(toa[0, 0], s.argmax(axis=0))


def test_pure_noise_snr_is_unit_normal():
    rng = np.random.default_rng(8)
    nt, ns, npix = 1024, 16, 64
    x = rng.standard_normal((nt, ns, npix)).astype(np.float32)
    z, *_ = osr.normalize(x, "pixel_subband", "f32")
    delays = delay_table(np.linspace(1.311, 1.499, ns), 1.499, 134.2, [0.0, 2000.0])
    D = osr.dedisperse(z, delays)
    for d in range(2):
        for w in (1, 8, 64):
            S = osr.snr_series(D[d], w, ns)
            # use non-overlapping windows so the samples are independent
            v = S[::w].ravel()
            assert abs(v.mean()) < 0.06
            assert abs(v.std() - 1.0) < 0.06


def test_no_valid_window_gives_minus_inf():
    z = np.ones((10, 2, 1))
    delays = np.array([[0, 0], [8, 0]], dtype=np.int32)
    smax, toa = osr.snr_toa_maps(z, delays, [1, 2, 3])
    assert np.isinf(smax[1, 2, 0]) and toa[1, 2, 0] == -1
    assert smax[1, 1, 0] == pytest.approx(4 / 2.0) and toa[1, 1, 0] == 0


def test_candidates_threshold_sort_and_ties():
    best = np.array([5.0, 7.0, 6.0, 7.0, np.nan, -np.inf, 9.0, 6.0 - 1e-9])
    bd = np.arange(8, dtype=np.int32)
    bw = np.zeros(8, np.int32)
    bt = np.zeros(8, np.int32)
    recs, ntot = osr.candidates(best, bd, bw, bt, nx=4, theta=6.0, k_max=3)
    assert ntot == 4                       # 7, 6 (inclusive), 7, 9
    assert [(r["x"], r["y"]) for r in recs] == [(2, 1), (1, 0), (3, 0)]   # 9; 7 at p=1 before p=3
    recs, ntot = osr.candidates(best, bd, bw, bt, nx=4, theta=6.0, k_max=10)
    assert [r["dm_index"] for r in recs] == [6, 1, 3, 2]


def test_best_tie_break_smallest_dm_then_width():
    smax = np.array([[[1.0], [3.0]], [[3.0], [3.0]]])
    toa = np.array([[[0], [1]], [[2], [3]]], dtype=np.int32)
    best, bd, bw, bt = osr.best_per_pixel(smax, toa)
    assert (bd[0], bw[0], bt[0]) == (0, 1, 1)


def test_config1_pulse_has_expected_snr_and_no_candidates():
    """The tiny workload's pulse (A = 1, w = 4, n_sub = 4) has expected S/N 4 < 6."""
    cube, m = synth.config1()
    r = osr.search(cube, m["freqs"], m["f_ref"], m["dt_ms"], m["dms"], m["widths"], m["nx"])
    p = m["injections"][0]["p"]
    assert r["delays"][3].tolist() == m["injections"][0]["offsets"].tolist()   # DM 500 -> trial 3
    assert 2.0 < r["snr_max"][3, 2, p] < 7.0
    np.testing.assert_array_equal(r["delays"], np.loadtxt(
        __file__.replace("test_oracle_search.py", "golden/delays_c1.txt"), dtype=np.int64)[:, 1:])


def test_unquantised_store_keeps_fp64_values():
    rng = np.random.default_rng(12)
    z = rng.standard_normal((5, 3, 7)) * 1e-3 + 1.0 / 3.0
    assert np.array_equal(osr.cast_store(z, "f64"), z)
    assert not np.array_equal(osr.cast_store(z, "f32"), z)
    # the FP32 store differs from the unquantised one by at most half an FP32 ulp per value
    assert np.abs(osr.cast_store(z, "f32") - z).max() <= 2.0 ** -25


# ------------------------------------------------------------ time binning
def test_bin_time_matches_explicit_loops():
    rng = np.random.default_rng(21)
    x = rng.standard_normal((23, 3, 4)).astype(np.float32)
    for f in (1, 2, 5, 7, 23):
        got = osr.bin_time(x, f)
        assert got.shape == (23 // f, 3, 4) and got.dtype == np.float32
        for tb in range(23 // f):
            for s in range(3):
                for p in range(4):
                    acc = 0.0
                    for k in range(f):
                        acc += float(x[tb * f + k, s, p])       # Python floats are FP64
                    assert got[tb, s, p] == np.float32(acc)


def test_bin_time_integer_totals_and_identity():
    rng = np.random.default_rng(22)
    x = rng.integers(-50, 51, size=(301, 2, 5)).astype(np.float32)
    b = osr.bin_time(x, 75)                       # 4 whole bins, one sample dropped
    assert b.shape == (4, 2, 5)
    np.testing.assert_array_equal(b.astype(np.int64).sum(axis=0), x[:300].astype(np.int64).sum(axis=0))
    np.testing.assert_array_equal(osr.bin_time(x, 1), x)
    np.testing.assert_array_equal(osr.bin_time(np.full((10, 1, 1), 0.25, np.float32), 5), np.full((2, 1, 1), 1.25))


def test_shift_table_reused_at_five_times_dm():
    """The paper's footnote: searching 5x-binned data at 5x the DMs keeps the shifts."""
    freqs = np.linspace(1.311, 1.499, 16)
    for dms in (np.linspace(0, 4000, 32), np.linspace(171, 4000, 16)):
        native = delay_table(freqs, freqs.max(), 134.2, dms)
        binned = delay_table(freqs, freqs.max(), 5 * 134.2, 5 * dms)
        np.testing.assert_array_equal(native, binned)


def test_binned_boxcar_snr_closed_form():
    """A bin-aligned boxcar of width f*w at DM 0, noiseless with external statistics
    sqrt(f)*sigma for the binned series, has S/N = A*sqrt(n_sub*f*w) at the coarse
    timescale: the same as the exact native boxcar of width f*w."""
    ns, nt, f, w, A, sigma = 4, 600, 75, 4, 0.8, 1.3
    freqs = np.linspace(1.311, 1.499, ns)
    x = np.zeros((nt, ns, 1), np.float32)
    synth.inject_boxcar(x, 0, 150, np.zeros(ns, np.int64), f * w, A * sigma)
    rs = osr.multiscale_search(x, freqs, freqs.max(), 134.2, [0.0, 500.0], [1, 2, 4, 8], 1,
                               factors=[1, f], dm_scales=[1.0, 0.0], norm="external",
                               med=np.zeros((1, ns)), sigma=np.full((1, ns), sigma), theta=0.0)
    # the coarse search used sigma, not sqrt(f) sigma: rescale its S/N by 1/sqrt(f)
    coarse = rs[1]["snr_max"][0, 2, 0] / math.sqrt(f)
    assert coarse == pytest.approx(A * math.sqrt(ns * f * w), rel=1e-6)
    assert rs[1]["toa"][0, 2, 0] == 150 // f
    assert rs[1]["delays"].shape == (1, ns) and not rs[1]["delays"].any()


def test_time_margin_on_hand_built_series():
    """The S/N margin over time (best minus second best window of one trial),
    which decides where TOAs are compared, on series worked out by hand:
    one sub-band, DM 0, so S/N = window sum / sqrt(w)."""
    z = np.array([1.0, 7.0, 3.0, 5.0, 5.0, -2.0])[:, None, None]
    delays = np.zeros((1, 1), np.int32)
    smax, toa, margin = osr.snr_toa_margin_maps(z, delays, [1, 2, 5, 6, 7])
    # width 1: best 7 at t=1, next 5 -> margin 2
    assert smax[0, 0, 0] == 7.0 and toa[0, 0, 0] == 1 and margin[0, 0, 0] == 2.0
    # width 2: sums 8, 10, 8, 10, 3 -> exact tie at 10: margin 0, first maximum t=1
    assert toa[0, 1, 0] == 1 and margin[0, 1, 0] == 0.0
    assert smax[0, 1, 0] == pytest.approx(10 / math.sqrt(2), abs=0)
    # width 5: sums 21 (t=0), 18 (t=1) -> margin 3/sqrt(5)
    assert toa[0, 2, 0] == 0 and margin[0, 2, 0] == pytest.approx(3 / math.sqrt(5), rel=1e-15)
    # width 6: one window -> inf; width 7: no window -> nan, -inf, -1
    assert margin[0, 3, 0] == np.inf and smax[0, 3, 0] == pytest.approx(19 / math.sqrt(6))
    assert np.isnan(margin[0, 4, 0]) and smax[0, 4, 0] == -np.inf and toa[0, 4, 0] == -1


def test_time_margin_with_delays_and_pixels():
    """Two sub-bands, delays (2, 0): D[t] = z0[t+2] + z1[t]; two pixels whose best
    windows are a clear peak and an exact tie."""
    z = np.zeros((8, 2, 2))
    z[:, 0, 0] = [0, 0, 0, 4, 0, 0, 0, 0]      # D: z0 shifted by 2 -> peak at t=1
    z[:, 1, 0] = [0, 3, 0, 0, 0, 1, 0, 0]      # D[1] = 4 + 3 = 7, D[5] = 1
    z[:, 0, 1] = [0, 0, 2, 0, 0, 2, 0, 0]      # D[0] = 2, D[3] = 2 (tie) for pixel 1
    delays = np.array([[2, 0]], np.int32)
    smax, toa, margin = osr.snr_toa_margin_maps(z, delays, [1])
    r2 = math.sqrt(2)
    assert smax[0, 0, 0] == pytest.approx(7 / r2) and toa[0, 0, 0] == 1
    assert margin[0, 0, 0] == pytest.approx(6 / r2)
    assert toa[0, 0, 1] == 0 and margin[0, 0, 1] == 0.0


def test_trial_margin_on_hand_built_maps():
    """Margin between the best and second-best (DM, width) trial of a pixel."""
    inf = np.inf
    smax = np.array([[[5.0, 1.0, -inf, -inf, 2.0]],
                     [[3.0, 1.0, -inf, 4.0, 2.0]]])        # [d=2][w=1][p=5]
    m = osr.trial_margin(smax)
    assert m[0] == 2.0                 # 5 vs 3
    assert m[1] == 0.0                 # exact tie 1 vs 1
    assert np.isnan(m[2])              # no trial has a window
    assert m[3] == inf                 # a single trial has a window: unambiguous
    assert m[4] == 0.0
    assert (osr.trial_margin(smax[:1]) == inf).all()   # one trial in total
    # agrees with the per-pixel best: the best trial is unique wherever m > 0
    best, bd, bw, _ = osr.best_per_pixel(smax, np.zeros(smax.shape, np.int32))
    assert bd[0] == 0 and best[0] == 5.0
