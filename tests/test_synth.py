"""Input generator checks (CPU): Philox known answers, seeding, sky model."""
import os

import numpy as np

from paper_2510_18136_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    for line in open(os.path.join(GOLD, "philox_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(a, 16) for a in line.split()]
        out = synth.philox4x32_10([v[0:4]], (v[4], v[5]))[0]
        assert [int(a) for a in out] == v[6:10]


def test_philox_normals_are_standard():
    x = synth.philox_normals(200_000, seed=11)
    assert abs(x.mean()) < 0.01 and abs(x.std() - 1) < 0.01
    assert np.array_equal(x, synth.philox_normals(200_000, seed=11))


def test_noise_cube_independent_of_threads_and_seeded():
    a = synth.noise_cube(300, 2, 40, seed=5)
    b = synth.noise_cube(300, 2, 40, seed=5)
    assert np.array_equal(a, b) and not np.array_equal(a, synth.noise_cube(300, 2, 40, seed=6))
    big = synth.noise_cube(256, 4, 8192, seed=1)         # threaded path
    small = np.concatenate([synth.noise_cube(256, 4, 8192, seed=1, block=64)[i:i + 64] for i in range(0, 256, 64)])
    assert np.array_equal(big, small)


def test_injection_lands_on_dispersed_samples():
    cube = np.zeros((50, 4, 3), dtype=np.float32)
    off = synth.arrival_offsets(500.0, synth.C1_FREQS, synth.C1_FREQS.max(), synth.DT_MS)
    synth.inject_boxcar(cube, 1, 10, off, 4, 2.0)
    for s in range(4):
        assert (cube[10 + off[s]:14 + off[s], s, 1] == 2.0).all()
    assert cube.sum() == 4 * 4 * 2.0
