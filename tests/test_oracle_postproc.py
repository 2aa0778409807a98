"""Pins for the PSF reduction oracle (section 2.3): hand-worked cases, the
single-candidate identity, translation invariance, and the property that a
source with its own sidelobes beats each of those sidelobes."""
import numpy as np
import pytest

from oracle import postproc
from paper_2510_18136_amd import synth


def tiny_psf():
    p = np.zeros((5, 5), np.float32)
    p[2, 2] = 1.0
    p[2, 4] = p[2, 0] = 0.5          # sidelobes two pixels east and west
    p[0, 2] = p[4, 2] = 0.25         # weaker ones two pixels north and south
    return p


def test_single_candidate_is_kept():
    assert postproc.psf_reduce([(7, 3, 9.5)], tiny_psf()) == (0, 9.5)


def test_hand_worked_case():
    # 90th percentile of the 25 pixels {0 x 20, 0.25 x 2, 0.5 x 2, 1}: sorted index 21.6
    # lies between 0.25 (index 21) and 0.5 (index 22): q = 0.25 + 0.6 * 0.25 = 0.4, so the
    # mask holds the centre and the two 0.5 sidelobes only.
    assert np.percentile(tiny_psf(), 90) == pytest.approx(0.4)
    cands = [(10, 10, 8.0), (12, 10, 6.0), (10, 12, 7.0)]
    i, s = postproc.psf_reduce(cands, tiny_psf())
    # S/N of the weighted mean: sum(w S) / sqrt(sum(w^2))
    # centre 0: member 1 at (+2, 0), weight 0.5 -> (8 + 3) / sqrt(1.25) = 9.839; member 2 at (0, +2) not in mask
    # centre 1: member 0 at (-2, 0), weight 0.5 -> (6 + 4) / sqrt(1.25) = 8.944
    # centre 2: no members -> 7.0
    assert i == 0 and s == pytest.approx(11.0 / np.sqrt(1.25))


def test_weighted_mean_snr_is_the_snr_of_the_weighted_mean():
    """Members with unit-noise S/N values: the score equals the weighted mean
    divided by its standard deviation, checked against a Monte Carlo of noise-only
    S/N values (the score of pure noise has unit variance)."""
    p = tiny_psf()
    cands = [(10, 10, 0.0), (12, 10, 0.0), (8, 10, 0.0)]      # centre 0 has two 0.5-weight members
    rng = np.random.default_rng(4)
    scores = []
    for _ in range(4000):
        s = rng.standard_normal(3)
        c = [(x, y, float(v)) for (x, y, _), v in zip(cands, s)]
        scores.append(((s[0] + 0.5 * s[1] + 0.5 * s[2]) / np.sqrt(1.5), postproc.psf_reduce(c, p)))
    direct = np.array([a for a, _ in scores])
    assert abs(direct.std() - 1.0) < 0.05
    # whenever the first candidate wins, its score is that unit-noise statistic
    for a, (i, s) in scores:
        if i == 0:
            assert s == pytest.approx(a, rel=1e-12)


def test_point_source_beats_its_own_sidelobes():
    """Candidates at a point source and at its brightest sidelobes, with S/N in
    proportion to the beam: the source is kept, wherever the sidelobes are."""
    psf = synth.snapshot_psf(half=20)
    h = 20
    order = np.argsort(psf.ravel())[::-1]
    for s_c in (8.0, 15.0, 40.0):
        cands = [(100, 100, s_c)]
        for k in order[1:10]:                             # the nine brightest other beam pixels
            dy, dx = divmod(int(k), psf.shape[1])
            cands.append((100 + dx - h, 100 + dy - h, s_c * float(psf.ravel()[k])))
        cands.sort(key=lambda c: -c[2])
        i, _ = postproc.psf_reduce(cands, psf)
        assert (cands[i][0], cands[i][1]) == (100, 100)


def test_translation_invariance():
    rng = np.random.default_rng(3)
    psf = synth.snapshot_psf(half=8)
    c = [(int(rng.integers(0, 30)), int(rng.integers(0, 30)), float(rng.uniform(6, 20))) for _ in range(10)]
    a = postproc.psf_reduce(c, psf)
    b = postproc.psf_reduce([(x + 13, y - 4, s) for x, y, s in c], psf)
    assert a[0] == b[0] and a[1] == pytest.approx(b[1], rel=1e-12)


def test_candidate_outside_every_mask_changes_nothing():
    rng = np.random.default_rng(5)
    psf = synth.snapshot_psf(half=8)
    c = [(int(rng.integers(20, 40)), int(rng.integers(20, 40)), float(rng.uniform(6, 20))) for _ in range(8)]
    i, s = postproc.psf_reduce(c, psf)
    far = c + [(200, 200, 0.5 * s)]                 # beyond the PSF from every candidate, lower score
    assert postproc.psf_reduce(far, psf) == (i, s)


def test_point_mirror_with_a_symmetric_beam():
    """B(-l, -m) = B(l, m): mirroring every candidate through a point mirrors the choice."""
    rng = np.random.default_rng(6)
    psf = synth.snapshot_psf(half=8)
    c = [(int(rng.integers(0, 20)), int(rng.integers(0, 20)), float(rng.uniform(6, 20))) for _ in range(10)]
    i, s = postproc.psf_reduce(c, psf)
    j, t = postproc.psf_reduce([(50 - x, 50 - y, v) for x, y, v in c], psf)
    assert i == j and s == pytest.approx(t, rel=1e-12)


def test_snapshot_psf_is_a_normalised_symmetric_beam():
    p = synth.snapshot_psf(half=10)
    assert p.shape == (21, 21) and p[10, 10] == 1.0
    np.testing.assert_allclose(p, p[::-1, ::-1], atol=1e-6)      # real beam: B(-l, -m) = B(l, m)
    assert p.max() == 1.0 and p.min() < 0.0
