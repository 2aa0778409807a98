"""Pins for the oracle's robust statistics and cast chain."""
import numpy as np
import pytest
import torch
from scipy import stats as sst

from oracle import stats as ost
from oracle import brute
from oracle.search import cast_store, round_f32_to_bf16, normalize


def test_mad_constant_is_inverse_normal_quartile():
    assert ost.MAD_TO_SIGMA == 1.0 / sst.norm.ppf(0.75)


@pytest.mark.parametrize("n", [1, 2, 3, 7, 8, 64, 65, 2048])
def test_median_matches_library_and_sort(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n).astype(np.float32)
    m = ost.median_fp64(x)
    assert m == np.median(x.astype(np.float64))
    assert m == brute.median_brute(x.tolist())
    vec = ost.median_axis0(np.stack([x, -x], axis=1))
    assert vec[0] == m and vec[1] == np.median(-x.astype(np.float64))


def test_median_even_uses_fp64_midpoint():
    # two FP32 values whose FP32 mean would round differently from FP64
    a, b = np.float32(16777216.0), np.float32(16777218.0)
    assert ost.median_fp64(np.array([a, b])) == 16777217.0


def test_mad_against_library():
    rng = np.random.default_rng(5)
    x = rng.standard_normal(1001)
    med = np.median(x)
    assert ost.mad_fp64(x, med) == np.median(np.abs(x - med))
    assert ost.mad_fp64(x, med) * ost.MAD_TO_SIGMA == pytest.approx(
        sst.median_abs_deviation(x, scale="normal"), rel=1e-14)


def test_robust_stats_gaussian_sigma():
    rng = np.random.default_rng(1)
    cube = (rng.standard_normal((4096, 2, 8)) * 1.7 + 3.0).astype(np.float32)
    med, sig = ost.robust_stats(cube)
    assert med.shape == (8, 2)
    np.testing.assert_allclose(med, 3.0, atol=0.1)
    np.testing.assert_allclose(sig, 1.7, rtol=0.06)
    # per (p, s): matches the scalar definition exactly
    assert med[3, 1] == ost.median_fp64(cube[:, 1, 3])
    assert sig[3, 1] == ost.MAD_TO_SIGMA * ost.mad_fp64(cube[:, 1, 3], med[3, 1])


def test_pixel_mode_pools_subbands():
    rng = np.random.default_rng(2)
    cube = rng.standard_normal((33, 3, 5)).astype(np.float32)
    med, sig = ost.robust_stats(cube, "pixel")
    for p in range(5):
        v = cube[:, :, p].ravel()
        assert (med[p] == ost.median_fp64(v)).all()
        assert (sig[p] == ost.MAD_TO_SIGMA * ost.mad_fp64(v, ost.median_fp64(v))).all()


def test_wide_pulse_biases_std_not_mad():
    """Section 3.2: a plain noise estimate is biased high by 8-16 sample pulses."""
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2048, 1, 1)).astype(np.float32)
    x[1000:1016, 0, 0] += 12.0
    _, sig = ost.robust_stats(x)
    assert abs(sig[0, 0] - 1.0) < 0.06
    assert np.std(x) > 1.15 * sig[0, 0]


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(4)
    x = (rng.standard_normal(100000) * 3).astype(np.float32)
    x = np.concatenate([x, np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 65504.0,
                                     1e-40, -0.0, np.inf, -np.inf], dtype=np.float32)])
    ours = round_f32_to_bf16(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(ours.view(np.uint32), ref.view(np.uint32))


def test_cast_chain_is_fp64_fp32_store():
    z = np.array([1.0 + 2 ** -30, 0.1, -2.5e-5, 1e5 / 3])
    np.testing.assert_array_equal(cast_store(z, "f32"), z.astype(np.float32).astype(np.float64))
    np.testing.assert_array_equal(cast_store(z, "f16"),
                                  z.astype(np.float32).astype(np.float16).astype(np.float64))
    # a value where direct FP64->FP16 rounding differs from FP64->FP32->FP16
    v = np.float64(1.0) + np.float64(2 ** -11) + np.float64(2 ** -40)
    assert np.float16(v) != np.float16(np.float32(v))
    assert cast_store(np.array([v]), "f16")[0] == float(np.float16(np.float32(v)))


def test_normalize_flags_constant_and_nonfinite_series():
    x = np.zeros((16, 2, 3), dtype=np.float32)
    x[:, 1, :] = np.arange(16, dtype=np.float32)[:, None]
    x[5, 1, 2] = np.nan
    z, med, sig, nflag = normalize(x, "pixel_subband", "f32")
    assert nflag == 3 + 1        # three constant series, one with a NaN
    assert (z[:, 0, :] == 0).all() and (z[:, 1, 2] == 0).all()
    assert np.isnan(sig[2, 1]) and sig[0, 0] == 0
    assert z[:, 1, 0].tolist() == [float(np.float32((t - 7.5) / (1.482602218505602 * 4.0)))
                                  for t in range(16)]
