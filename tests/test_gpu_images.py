"""Telescope images on the GPU: the PSF convolution against the oracle's
plain sum over shifts, across image sizes and widths up to the largest
supported (which needs the most local memory)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1201_3588_amd import mcrt

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("npix,fwhm", [(1, 0.0), (1, 4.0), (17, 2.5), (100, 7.3), (61, 32.0)])
def test_psf_matches_oracle(npix, fwhm):
    rng = np.random.default_rng(npix + int(fwhm))
    img = rng.integers(0, 1 << 40, (3, npix, npix), dtype=np.int64)
    img[1] = 0
    img[1, npix // 2, npix // 3] = 1 << 30                 # a point source
    g = mcrt.image_psf(torch.as_tensor(img).cuda(), npix, 2.0 ** -24, fwhm).cpu().numpy()
    o = oracle.psf_convolve(img, 2.0 ** -24, fwhm)
    assert g.shape == o.shape
    assert np.allclose(g, o, rtol=1e-13, atol=1e-13 * np.abs(o).max())


def test_psf_rejects_bad_arguments():
    img = torch.zeros((1, 8, 8), dtype=torch.int64, device="cuda")
    for fwhm in (-1.0, 33.0, float("nan")):
        with pytest.raises(mcrt.MCRTError):
            mcrt.image_psf(img, 8, 1.0, fwhm)
    with pytest.raises(mcrt.MCRTError):
        mcrt.image_psf(img, 7, 1.0, 2.0)
    L = mcrt.lib()
    assert L.mcrt_image_psf(None, 1, 8, 1.0, 2.0, None, None, None) == -1
