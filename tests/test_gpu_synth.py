"""The device generator writes the same field as the NumPy generator."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("drift", [False, True])
def test_gpu_spectrum_matches_numpy(drift):
    from synth import gpu as sg
    ref = synth.spectrum(24, 20, 12, 5, nmodes=16, seed=11, drift=drift, dtype=np.float64)[0]
    t = torch.empty((5, 12, 20, 24), dtype=torch.float64, device="cuda")
    sg.spectrum_into(t, seed=11, nmodes=16, drift=drift)
    got = t.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    t32 = torch.empty((5, 12, 20, 24), dtype=torch.float32, device="cuda")
    sg.spectrum_into(t32, seed=11, nmodes=16, drift=drift)
    ref32 = synth.spectrum(24, 20, 12, 5, nmodes=16, seed=11, drift=drift, dtype=np.float32)[0]
    assert np.mean(t32.cpu().numpy() == ref32) > 0.999


def test_gpu_blobs_match_numpy():
    from synth import gpu as sg
    ref = synth.blobs2d_truncated(150, 90, 4, nblobs=30, seed=3, dtype=np.float64)[0]
    t = torch.empty((4, 1, 90, 150), dtype=torch.float64, device="cuda")
    sg.blobs_into(t, nblobs=30, seed=3)
    assert np.abs(t.cpu().numpy() - ref).max() <= 1e-12
