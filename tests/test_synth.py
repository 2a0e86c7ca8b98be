"""Input generators: determinism, the spectrum's rank-one structure, Philox KAT."""
import numpy as np

import synth


def test_blobs_deterministic_and_shape():
    a = synth.blobs2d(nx=32, ny=24, nt=5, seed=4)
    b = synth.blobs2d(nx=32, ny=24, nt=5, seed=4)
    c = synth.blobs2d(nx=32, ny=24, nt=5, seed=5)
    assert a.shape == (1, 5, 1, 24, 32) and a.dtype == np.float64
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_blob_noise_level():
    f = synth.blobs2d(nx=64, ny=64, nt=4, nblobs=0, seed=1, noise_std=1e-4)
    assert abs(f.std() - 1e-4) < 5e-6


def test_spectrum_without_drift_is_rank_one_in_time():
    f = synth.spectrum(16, 12, 8, 6, nmodes=8, seed=3, dtype=np.float64)[0]
    X = f.reshape(6, -1)
    s = np.linalg.svd(X, compute_uv=False)
    assert s[1] <= 1e-12 * s[0]
    g = synth.spectrum(16, 12, 8, 6, nmodes=8, seed=3, drift=True, dtype=np.float64)[0]
    s2 = np.linalg.svd(g.reshape(6, -1), compute_uv=False)
    assert s2[1] > 1e-3 * s2[0]


def test_spectrum_modes_nonzero_and_bounded():
    k, phi, om = synth.spectrum_params((64, 64, 64), 64, 11)
    assert np.all(np.abs(k).sum(axis=1) > 0) and np.abs(k).max() <= 4
    assert np.all((phi >= 0) & (phi < 2 * np.pi)) and np.all((om >= 0) & (om <= 0.2))


def test_philox_known_answers():
    """Known-answer vectors published with Random123 (Philox4x32-10)."""
    cases = [
        ([0, 0, 0, 0], (0, 0), [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]),
        ([0xffffffff] * 4, (0xffffffff, 0xffffffff),
         [0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd]),
        ([0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344], (0xa4093822, 0x299f31d0),
         [0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1]),
    ]
    for ctr, key, want in cases:
        got = synth.philox4x32(np.array([ctr], np.uint32), *key)[0]
        assert [int(v) for v in got] == want


def test_philox_normal_moments():
    z = synth.philox_normal(np.arange(200000, dtype=np.uint64), seed=9, std=2.0)
    assert abs(z.mean()) < 0.02 and abs(z.std() - 2.0) < 0.02
