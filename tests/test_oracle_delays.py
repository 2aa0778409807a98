"""Pins for the oracle's delay table (section 2.2 delay law and its footnote)."""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle.delays import delay_table, delay_samples_real

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def paper_values():
    vals = {}
    for line in open(os.path.join(GOLD, "paper_values.txt")):
        line = line.split("#")[0].strip()
        if line:
            k, v = (a.strip() for a in line.split("="))
            vals[k] = float(v)
    return vals


def exact_delay(dm, f, fr, dt, k="4.15"):
    """Exact rational delay, then round half to even (independent of FP64)."""
    q = Fraction(k) * Fraction(dm) * (1 / (Fraction(f) ** 2) - 1 / (Fraction(fr) ** 2)) / Fraction(dt)
    fl = q.numerator // q.denominator
    rem = q - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return fl


def test_c1_table_matches_hand_values():
    rows = np.loadtxt(os.path.join(GOLD, "delays_c1.txt"), dtype=np.int64)
    got = delay_table(np.linspace(1.311, 1.499, 4), 1.499, 134.2, np.linspace(0, 1000, 8))
    assert got.dtype == np.int32
    np.testing.assert_array_equal(got, rows[:, 1:])


def test_exact_rational_agreement_c2_grid():
    freqs = np.linspace(1.311, 1.499, 16)
    dms = np.linspace(0, 4000, 32)
    got = delay_table(freqs, freqs.max(), 134.2, dms)
    real = delay_samples_real(freqs, freqs.max(), 134.2, dms)
    for d in range(32):
        for s in range(16):
            # the FP64 value is within 1e-9 of the exact one; compare the rounded
            # result wherever the value is not within that distance of a half
            frac = real[d, s] - np.floor(real[d, s])
            if abs(frac - 0.5) > 1e-9:
                assert got[d, s] == exact_delay(Fraction(float(dms[d])), Fraction(float(freqs[s])),
                                                Fraction(float(freqs.max())), Fraction("134.2"))
    # survey-shape spot value at the top DM (hand evaluation of the law)
    assert got[-1].tolist() == [17, 16, 14, 13, 12, 11, 9, 8, 7, 6, 5, 4, 3, 2, 1, 0]


def test_dm_zero_row_and_monotonicity():
    freqs = np.linspace(1.311, 1.499, 16)
    dms = np.linspace(0, 4000, 32)
    t = delay_table(freqs, freqs.max(), 134.2, dms)
    assert (t[0] == 0).all()
    assert (np.diff(t, axis=0) >= 0).all()   # non-decreasing in DM
    assert (np.diff(t, axis=1) <= 0).all()   # non-increasing in frequency
    assert (t[:, -1] == 0).all()             # reference sub-band has no delay


def test_delay_law_constant_and_sign():
    # a single sub-band pair: 4.15 ms * DM * (lo^-2 - hi^-2), positive at the low frequency
    r = delay_samples_real([1.311, 1.499], 1.499, 1.0, [100.0])
    assert r[0, 1] == 0.0
    assert r[0, 0] == pytest.approx(4.15 * 100 * (1.311 ** -2 - 1.499 ** -2), rel=1e-14)
    assert r[0, 0] > 0


def test_x5_shift_reuse_identity():
    """Footnote of section 2.2: DM range x5 at 5x coarser sampling reuses the shifts."""
    pv = paper_values()
    assert pv["dm5_lo"] == 5 * pv["dm_lo"] and pv["dm5_hi"] == 5 * pv["dm_hi"]
    freqs = np.linspace(pv["band_lo_ghz"], pv["band_hi_ghz"], 16)
    dms = np.linspace(pv["dm_lo"], pv["dm_hi"], int(pv["n_dm_trials"]))
    a = delay_table(freqs, freqs.max(), 134.2, dms)
    b = delay_table(freqs, freqs.max(), 5 * 134.2, 5 * dms)
    np.testing.assert_array_equal(a, b)
    dms32 = np.linspace(0, 4000, 32)
    np.testing.assert_array_equal(delay_table(freqs, freqs.max(), 134.2, dms32),
                                  delay_table(freqs, freqs.max(), 671.0, 5 * dms32))


def test_pulsar_nearest_trial_is_dm_zero():
    """Section 3.3: B0329+54 (DM 26.76) is detected at the DM=0 trial; next trial 213.72."""
    pv = paper_values()
    freqs = np.linspace(pv["band_lo_ghz"], pv["band_hi_ghz"], 16)
    t = delay_table(freqs, freqs.max(), 134.2, [0.0, pv["psr_dm"], pv["psr_next_trial"]])
    np.testing.assert_array_equal(t[1], t[0])      # its own shifts equal the DM=0 trial
    assert (t[2] != t[0]).any()                    # the next trial is distinguishable


def test_width_and_timescale_arithmetic():
    pv = paper_values()
    dt = pv["dt_ms"] / 1000.0
    assert 1 * dt == pytest.approx(pv["width_min_s"], abs=1e-3)
    assert 16 * dt == pytest.approx(pv["width_max_s"], abs=1e-2)
    assert 5 * dt == pytest.approx(pv["w5_min_s"], abs=1e-2)
    assert 80 * dt == pytest.approx(pv["w5_max_s"], abs=1e-2)
    assert 75 * dt == pytest.approx(pv["w75_min_s"], abs=1e-2)
    assert 1200 * dt == pytest.approx(pv["w75_max_s"], abs=0.2)   # 160.8 s = 1200 samples
