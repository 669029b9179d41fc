"""Pins of the oracle's escape binning (the SEDs of paper Sec. 2 and Fig. 1):
n_theta bins equal in cos(theta) about +z, times n_phi bins equal in the
azimuth phi = atan2(d_y, d_x) in [0, 2 pi).

* A star in a dust-free grid: every packet escapes in its launch direction,
  which is isotropic, so each (theta, phi) bin holds Binomial(N, 1/(n_theta
  n_phi)) packets; bins equal in theta instead of cos(theta) would put 2.4 %
  instead of 10 % of the packets in the bottom theta bin.
* Pencil beams along hand-chosen directions, one per phi bin: the bin of each
  was worked out by hand (below), which pins the azimuth's axes, sense and
  range, and the theta bins' orientation.
"""
import math

import numpy as np
from scipy import stats

import oracle
import synth


def dust_free(n_packets, n_theta=10, n_phi=8, nl=4):
    w = synth.uniform_cube(4, 0.0, albedo=0.0, nl=nl, n_packets=n_packets)
    w.grid.rho = np.zeros(w.grid.n_cells)
    w.n_theta, w.n_phi = n_theta, n_phi
    return w


def test_isotropic_escapes_fill_equal_cos_and_phi_bins():
    N = 160_000
    w = dust_free(N)
    r = oracle.Session(w, n_threads=4).transport()
    assert int(r["counters"][oracle.CNT["escaped"]]) == N
    assert int(r["counters"][oracle.CNT["crossings"]]) > 0
    sed = r["sed"].sum(axis=2).astype(np.float64)          # [theta][phi], summed over bins
    n_bins = sed.size
    p = 1.0 / n_bins
    z = (sed - N * p) / math.sqrt(N * p * (1 - p))
    assert np.max(np.abs(z)) < 4.5, z
    chi2 = float(((sed - N * p) ** 2 / (N * p)).sum())
    assert stats.chi2.sf(chi2, n_bins - 1) > 1e-4, chi2
    # marginals: Binomial(N, 1/10) per theta bin and Binomial(N, 1/8) per phi bin
    for marg, k in ((sed.sum(1), w.n_theta), (sed.sum(0), w.n_phi)):
        q = 1.0 / k
        assert np.max(np.abs(marg - N * q)) < 4.5 * math.sqrt(N * q * (1 - q)), marg
    # equal-theta bins would give the bottom bin (1 - cos 18 deg) / 2 of the packets
    assert abs(sed.sum(1)[0] / N - 0.1) < 0.005 and (1 - math.cos(math.radians(18))) / 2 < 0.025


# direction (unnormalised) -> (theta bin, phi bin) with 10 x 8 bins, worked by hand:
# theta bin = floor((mu + 1) / 2 * 10), mu = d_z / |d|; phi bin = floor(phi / 45 deg)
HAND_BEAMS = [
    ((1.0, 0.0, 0.0), 5, 0),        # mu = 0 exactly: (0 + 1) / 2 * 10 = 5.0 -> 5; phi = 0 -> 0
    ((0.3, 0.5, 0.8), 9, 1),        # |d| = 0.98995, mu = 0.80812 -> 9.04; phi = 59.04 deg -> 1.31
    ((-0.5, 0.9, -0.1), 4, 2),      # |d| = 1.03441, mu = -0.09667 -> 4.52; phi = 119.05 deg -> 2.65
    ((-0.9, 0.3, -0.95), 1, 3),     # |d| = 1.34257, mu = -0.70760 -> 1.46; phi = 161.57 deg -> 3.59
    ((-1.0, -0.2, 0.3), 6, 4),      # |d| = 1.06301, mu = 0.28222 -> 6.41; phi = 191.31 deg -> 4.25
    ((-0.4, -0.9, 0.05), 5, 5),     # |d| = 0.98615, mu = 0.05070 -> 5.25; phi = 246.04 deg -> 5.47
    ((0.2, -1.0, -0.9), 1, 6),      # |d| = 1.36015, mu = -0.66169 -> 1.69; phi = 281.31 deg -> 6.25
    ((0.6, -0.1, 0.2), 6, 7),       # |d| = 0.64031, mu = 0.31235 -> 6.56; phi = 350.54 deg -> 7.79
]


def test_beams_land_in_hand_computed_bins():
    for d, bt, bp in HAND_BEAMS:
        w = dust_free(50)
        w.source.pos = np.array([1.7, 2.2, 2.9])
        w.source.beam = np.asarray(d) / np.linalg.norm(d)
        r = oracle.Session(w).transport()
        sed = r["sed"].sum(axis=2)
        assert int(sed[bt, bp]) == 50, (d, bt, bp, np.argwhere(sed))
    # one theta bin only: every beam of a phi sweep lands in that phi's bin
    w = dust_free(20, n_theta=1, n_phi=8)
    for k in range(8):
        phi = math.radians(45.0 * k + 22.5)
        w.source.pos = np.array([2.1, 1.9, 2.3])
        w.source.beam = np.array([math.cos(phi), math.sin(phi), 0.0])
        sed = oracle.Session(w).transport()["sed"].sum(axis=2)
        assert int(sed[0, k]) == 20, (k, sed)
