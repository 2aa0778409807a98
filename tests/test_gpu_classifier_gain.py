"""What the trained classifier gains over the plain S/N >= 6 threshold (GPU).

A short run of the whole learned path: device cubes with pulses, sidelobe
ghosts and RFI -> batched search -> cutouts -> BF16 MFMA training with Adam ->
inference on fresh held-out cutouts. At an operating point chosen on a
validation split for recall at least the threshold's, the classifier must keep
at most half the threshold's false candidates with recall within two points of
it, and it must reject every zero-DM spike that the threshold lets through.
(The full-size run, 200k training cutouts and 10k held-out, is the module's
command line.)
"""
import numpy as np
import pytest

from paper_2510_18136_amd import nsfrb, train_classifier as tc
from tests._lib import ensure_built

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()
    assert torch.cuda.is_available()


def test_classifier_beats_the_snr_threshold():
    print("[gpu] classifier gain: train 24k cutouts", flush=True)
    with nsfrb.Classifier(max_batch=64, n_time=tc.CUT_T, ny=32, lr=1e-3, seed=3) as clf:
        tr = tc.train(clf, 24000, seed=301, lr=1e-3, log=lambda m: None)
        print(f"[gpu] trained {tr['cutouts']} cutouts in {tr['seconds']:.1f}s", flush=True)
        val = tc.score(clf, 3000, seed=302)
        held = tc.score(clf, 4000, seed=303)
    res = tc.evaluate(val, held)
    thr, clf_m = res["snr_threshold"], res["classifier_matched"]
    print(f"[gpu] threshold recall {thr['recall']:.3f} false {thr['false_candidates']}; "
          f"classifier recall {clf_m['recall']:.3f} false {clf_m['false_candidates']} {clf_m['false_by_kind']}",
          flush=True)
    assert thr["false_candidates"] > 100
    assert clf_m["false_candidates"] <= 0.5 * thr["false_candidates"]
    assert clf_m["recall"] >= thr["recall"] - 0.02
    assert thr["false_by_kind"]["spike"] > 0
    assert res["classifier_p50"]["false_by_kind"]["spike"] == 0
