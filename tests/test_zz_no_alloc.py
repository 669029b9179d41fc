"""The allocation-free PSF entry point (mcrt_image_psf_static, weights in the
library's static device array) against mcrt_image_psf (caller-given weights)
and the oracle's plain sum over shifts: two calls in a row, the second with a
smaller image and a narrower PSF, each bit-identical to the allocating entry
point and within 1e-13 of the oracle."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
from paper_1201_3588_amd import mcrt

pytestmark = pytest.mark.gpu


def test_static_psf_matches_allocating_entry_point():
    L = mcrt.lib()
    rng = np.random.default_rng(11)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    for n_img, npix, fwhm in ((3, 97, 19.5), (2, 33, 3.0)):
        img = rng.integers(0, 1 << 40, (n_img, npix, npix), dtype=np.int64)
        img[0, npix // 2, npix // 3] = 1 << 41
        dimg = torch.as_tensor(img).cuda()
        out = torch.full((n_img, npix, npix), float("nan"), dtype=torch.float64, device="cuda")
        rc = L.mcrt_image_psf_static(C.c_void_p(dimg.data_ptr()), n_img, npix, 2.0 ** -24, fwhm,
                                     C.c_void_p(out.data_ptr()), stream)
        assert rc == 0
        ref = mcrt.image_psf(dimg, npix, 2.0 ** -24, fwhm)
        torch.cuda.synchronize()
        g, r = out.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(g, r), (npix, fwhm)
        o = oracle.psf_convolve(img, 2.0 ** -24, fwhm)
        assert np.allclose(g, o, rtol=1e-13, atol=1e-13 * np.abs(o).max())
    # the binding, and the errors: out-of-range width, bad sizes
    small = torch.zeros((1, 8, 8), dtype=torch.int64, device="cuda")
    o8 = torch.empty((1, 8, 8), dtype=torch.float64, device="cuda")
    mcrt.image_psf_static(small, 8, 1.0, 2.0, o8)
    assert L.mcrt_image_psf_static(C.c_void_p(small.data_ptr()), 1, 8, 1.0, 40.0,
                                   C.c_void_p(o8.data_ptr()), stream) == -1
    assert L.mcrt_image_psf_static(None, 1, 8, 1.0, 2.0, None, stream) == -1
    torch.cuda.synchronize()
    assert float(o8.abs().sum()) == 0.0
