"""Pins of the oracle's point-spread-function convolution (paper Sec. 4,
Fig. 2: disk images seen with the ELT's 50 mas PSF at 10 um): the response to
a point source is the normalised Gaussian, its half maximum lies at half the
FWHM, flux is conserved away from the edges, and FWHM 0 is the identity."""
import math

import numpy as np

import oracle


def test_point_source_gives_the_normalised_gaussian():
    n, fwhm = 41, 5.0
    sigma = fwhm / (2 * math.sqrt(2 * math.log(2)))
    r = math.ceil(3 * sigma)
    img = np.zeros((n, n))
    img[20, 17] = 7.0
    out = oracle.psf_convolve(img, 2.0, fwhm)
    z = math.fsum(math.exp(-d * d / (2 * sigma * sigma)) for d in range(-r, r + 1))
    for dy in range(-r - 1, r + 2):
        for dx in range(-r - 1, r + 2):
            want = 0.0
            if abs(dx) <= r and abs(dy) <= r:
                want = 14.0 * math.exp(-(dx * dx + dy * dy) / (2 * sigma * sigma)) / (z * z)
            assert abs(out[20 + dy, 17 + dx] - want) <= 1e-14 * 14.0
    assert abs(out.sum() - 14.0) < 1e-12
    # half maximum at +-FWHM/2 along a row (linear interpolation between pixels)
    row = out[20, 17:] / out[20, 17]
    k = int(np.argmax(row < 0.5))
    x_half = (k - 1) + (row[k - 1] - 0.5) / (row[k - 1] - row[k])
    assert abs(2 * x_half - fwhm) < 0.15


def test_flux_conserved_inside_and_identity_at_zero_width():
    rng = np.random.default_rng(3)
    img = np.zeros((2, 60, 60))
    img[:, 15:45, 15:45] = rng.integers(0, 1000, (2, 30, 30))
    out = oracle.psf_convolve(img, 0.5, 8.0)          # r = 11 < 15: nothing leaves the image
    assert np.allclose(out.sum(axis=(1, 2)), 0.5 * img.sum(axis=(1, 2)), rtol=1e-13)
    assert np.array_equal(oracle.psf_convolve(img, 1.0, 0.0), img)
