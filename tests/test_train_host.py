"""Host logic of the classifier training pipeline (CPU): the injection plans,
the candidate records taken from the search's per-pixel best arrays, and the
operating-point / recall / false-candidate bookkeeping."""
import math

import numpy as np
import pytest

from oracle.delays import delay_table
from paper_2510_18136_amd import train_classifier as tc
from tests._lib import ensure_built


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()


def cheb(a, b):
    return max(abs(a[0] - b[0]), abs(a[1] - b[1]))


def test_sky_plans_follow_the_recipe():
    rng = np.random.default_rng(3)
    for _ in range(50):
        plan = tc.plan_cube(rng, 7, "sky")
        pulses = [(r, b, o) for r, b, o in zip(plan["req"], plan["boxcars"], plan["offsets"]) if r[1] == "pulse"]
        assert len(pulses) == 4
        mains = [r[0] for r, _, _ in pulses]
        assert all(cheb(a, b) >= 17 for i, a in enumerate(mains) for b in mains[i + 1:])
        last = None
        for (xy, kind, snr), (k, pix, t0, w, amp), off in zip(plan["req"], plan["boxcars"], plan["offsets"]):
            assert k == 7 and pix == xy[1] * tc.NX + xy[0]
            assert 1 <= w <= 16 and 40 <= t0 < tc.NT - 40 - w + 1
            if kind == "pulse":
                assert 5 <= snr <= 50 and amp == pytest.approx(snr / math.sqrt(16 * w), rel=1e-12)
                last = (xy, t0, w, amp, off)
            else:                                    # a ghost copies the pulse placed just before it
                pxy, pt0, pw, pamp, poff = last
                assert 3 <= cheb(xy, pxy) <= 12 and (t0, w) == (pt0, pw)
                assert 0.1 <= amp / pamp <= 0.3 and np.array_equal(off, poff)
                assert all(cheb(xy, m) >= 17 for m in mains if m != pxy)
        assert len({r[0] for r in plan["req"]}) == len(plan["req"])         # distinct pixels


def test_pulse_offsets_follow_the_dispersion_law():
    for dm in (0.0, 137.5, 999.0):
        want = delay_table(tc.FREQS, tc.FREQS.max(), 134.2, np.array([dm]))[0]
        assert np.array_equal(tc.pulse_offsets(dm), want)


@pytest.mark.parametrize("kind", ["spike", "stripe"])
def test_rfi_plans(kind):
    rng = np.random.default_rng(4)
    for _ in range(30):
        plan = tc.plan_cube(rng, 0, kind)
        assert not plan["boxcars"] and 1 <= len(plan["rfi"]) <= 3
        for ev, t0, ln, sb, amp in plan["rfi"]:
            assert ev == kind
            if kind == "spike":
                assert ln == 1 and 1.5 <= amp <= 10 and 0 <= t0 < tc.NT
            else:
                assert 8 <= ln <= 96 and 0 <= t0 and t0 + ln <= tc.NT and 0 <= sb < 16 and 3 <= amp <= 15


def test_candidate_records_label_and_place():
    rng = np.random.default_rng(5)
    plan = tc.plan_cube(rng, 2, "sky")
    n = tc.NX * tc.NY
    snr = rng.standard_normal(n).astype(np.float32)
    dmi = rng.integers(0, 8, n).astype(np.int32)
    toa = rng.integers(0, 256, n).astype(np.int32)
    recs = tc.candidate_records(rng, 2, plan, snr, dmi, toa)
    inj = {r[0]: r[1] for r in plan["req"]}
    noise = [r for r in recs if r[7] == "noise"]
    assert len(noise) == 3 and len(recs) == len(inj) + 3
    for k, x, y, d, t, label, s, kind in recs:
        p = y * tc.NX + x
        assert k == 2 and (d, t) == (dmi[p], toa[p]) and s == pytest.approx(snr[p])
        if kind == "noise":
            assert label == 1 and all(cheb((x, y), o) > 3 for o in plan["occupied"])
        else:
            assert inj[(x, y)] == kind and label == (0 if kind == "pulse" else 1)
    far = [p for p in range(n) if all(cheb((p % tc.NX, p // tc.NX), o) > 3 for o in plan["occupied"])]
    top2 = sorted(far, key=lambda p: (-snr[p], p))[:2]
    assert [r[2] * tc.NX + r[1] for r in noise[:2]] == top2
    rfi = tc.candidate_records(rng, 0, dict(kind="spike"), snr, dmi, toa)
    assert len(rfi) == 8 and all(r[5] == 1 and r[7] == "spike" for r in rfi)
    assert len({(r[1], r[2]) for r in rfi}) == 8


def test_operating_point_and_summary():
    p = np.array([0.1, 0.2, 0.3, 0.4, 0.9, 0.05, 0.6])
    label = np.array([0, 0, 0, 0, 0, 1, 1])
    cut = tc.operating_point(p, label, 0.8)              # 4 of 5 positives: keep p < cut with cut just above 0.4
    assert 0.4 < cut < 0.4 + 1e-12
    kinds = np.array(["pulse"] * 5 + ["noise", "spike"])
    s = tc.summarise(p < cut, label, kinds)
    assert s["recall"] == 0.8 and s["detected"] == 4 and s["false_candidates"] == 1
    assert s["false_by_kind"]["noise"] == 1 and s["false_by_kind"]["spike"] == 0


def test_evaluate_counts_threshold_and_classifier():
    rng = np.random.default_rng(6)
    n = 400
    label = (rng.random(n) < 0.5).astype(int)
    snr = np.where(label == 0, rng.uniform(5, 50, n), rng.uniform(0, 20, n))
    p = np.where(label == 0, rng.uniform(0, 0.6, n), rng.uniform(0.4, 1, n))
    kinds = np.where(label == 0, "pulse", "ghost")
    val = (p, snr, label, kinds)
    res = tc.evaluate(val, val)
    thr = res["snr_threshold"]
    assert thr["recall"] == pytest.approx(np.mean(snr[label == 0] >= 6))
    assert thr["false_candidates"] == int(np.sum((snr >= 6) & (label == 1)))
    m = res["classifier_matched"]
    assert m["recall"] >= m["validation_target_recall"] >= thr["recall"]
    assert m["false_candidates"] == int(np.sum((p < m["p_rfi_below"]) & (label == 1)))
