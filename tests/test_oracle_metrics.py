"""Pins for the SNR definitions of eq. (11) and eq. (12) (Section V-B):
hand-computed cases whose every term is known, chosen so that a wrong
axis, a variance in place of a deviation, the region's own deviation in
place of the background's, or the sample divisor changes the value."""
import math

import numpy as np
import pytest

from oracle.metrics import snr_fhr, snr_fmd


def _volume():
    # 8 voxels x 2 bins.  Material 0 = voxels 0-3, material 1 = voxels 4-5,
    # background = voxels 6-7.
    r = np.zeros((8, 2))
    r[0:4, 0] = [0.5, 1.5, 1.0, 1.0]   # mean 1 (its own deviation is not 0)
    r[0:4, 1] = 2.0                    # mean 2
    r[4:6, 0] = [2.0, 4.0]             # mean 3
    r[4:6, 1] = 4.0                    # mean 4
    r[6:8, 0] = [-1.0, 1.0]            # population deviation 1 (sample: sqrt 2)
    r[6:8, 1] = [-2.0, 2.0]            # population deviation 2
    regions = [np.arange(0, 4), np.arange(4, 6)]
    return r, regions, np.arange(6, 8)


def test_snr_fhr_hand_case():
    r, regions, bg = _volume()
    # (1/1)^2 + (3/1)^2 + (2/2)^2 + (4/2)^2 = 15, over N_k N_m = 4
    assert snr_fhr(r, regions, bg) == pytest.approx(10 * math.log10(15 / 4), rel=1e-14)


def test_snr_fhr_single_term_and_scale_invariance():
    r, regions, bg = _volume()
    one = r[:, :1]
    # bin 0 alone: (1 + 9) / 2
    assert snr_fhr(one, regions, bg) == pytest.approx(10 * math.log10(5.0), rel=1e-14)
    # a common gain changes neither the means' ratios nor the value
    assert snr_fhr(7.5 * r, regions, bg) == pytest.approx(snr_fhr(r, regions, bg), rel=1e-13)
    # a tenfold signal gain in every region adds exactly 20 dB
    r2 = r.copy()
    r2[:6] *= 10
    assert snr_fhr(r2, regions, bg) == pytest.approx(snr_fhr(r, regions, bg) + 20.0, rel=1e-13)


def test_snr_fmd_hand_case():
    xm = np.zeros((6, 2))
    xm[0:2, 0] = [3.0, 5.0]    # material 0 image: region mean 4
    xm[4:6, 0] = [-0.5, 0.5]   # background deviation 0.5 -> ratio 8
    xm[2:4, 1] = [1.0, 1.0]    # material 1 image: region mean 1
    xm[4:6, 1] = [0.0, 2.0]    # background deviation 1 -> ratio 1
    regions = [np.array([0, 1]), np.array([2, 3])]
    assert snr_fmd(xm, regions, np.array([4, 5])) == pytest.approx(10 * math.log10((64 + 1) / 2), rel=1e-14)
