// Images seen through a telescope: the fixed-point image sums convolved with
// the instrument's point spread function (paper Sec. 4, Fig. 2: the ELT's
// 50 mas at 10 um), a Gaussian of given full width at half maximum.
//
// One 16 x 16 output tile per workgroup: the tile and its halo of r pixels are
// staged in LDS as doubles (scaled, zero outside the image), filtered along x
// into a second LDS array, then along y into the output; the 1-D weights are
// shared by both passes (the 2-D kernel is their outer product).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>

#include "mcrt.h"

namespace {

constexpr int kTile = 16;

__global__ void __launch_bounds__(256) k_psf(const unsigned long long* __restrict__ img, int npix, double scale,
                                            int r, const double* __restrict__ wts, double* __restrict__ out) {
  extern __shared__ double lds[];
  const int side = kTile + 2 * r;
  double* tin = lds;                    // [side][side]
  double* tx = tin + side * side;       // [side][kTile]
  double* w = tx + side * kTile;        // [2r + 1]
  const int im = blockIdx.z;
  const int x0 = blockIdx.x * kTile - r, y0 = blockIdx.y * kTile - r;
  const unsigned long long* src = img + (int64_t)im * npix * npix;
  const int tid = threadIdx.y * kTile + threadIdx.x;
  for (int q = tid; q <= 2 * r; q += kTile * kTile) w[q] = wts[q];
  for (int q = tid; q < side * side; q += kTile * kTile) {
    const int yy = y0 + q / side, xx = x0 + q % side;
    tin[q] = (xx >= 0 && yy >= 0 && xx < npix && yy < npix)
                 ? scale * (double)src[(int64_t)yy * npix + xx] : 0.0;
  }
  __syncthreads();
  for (int q = tid; q < side * kTile; q += kTile * kTile) {
    const int row = q / kTile, col = q % kTile;
    const double* p = tin + row * side + col;
    double acc = 0.0;
    for (int k = 0; k <= 2 * r; ++k) acc += w[k] * p[k];
    tx[q] = acc;
  }
  __syncthreads();
  const int ox = blockIdx.x * kTile + threadIdx.x, oy = blockIdx.y * kTile + threadIdx.y;
  if (ox >= npix || oy >= npix) return;
  double acc = 0.0;
  for (int k = 0; k <= 2 * r; ++k) acc += w[k] * tx[(threadIdx.y + k) * kTile + threadIdx.x];
  out[((int64_t)im * npix + oy) * npix + ox] = acc;
}

// normalised 1-D weights exp(-d^2 / (2 sigma^2)), |d| <= r
__global__ void k_psf_weights(double sigma, int r, double* wts) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int d = -r; d <= r; ++d) {
    const double v = sigma > 0.0 ? exp(-(double)(d * d) / (2.0 * sigma * sigma)) : (d == 0 ? 1.0 : 0.0);
    wts[d + r] = v;
    s += v;
  }
  for (int d = 0; d <= 2 * r; ++d) wts[d] /= s;
}

// Weights of the allocation-free entry point: one copy per device, held from
// the library's load to the end of the process.  In host code this name is
// not a device address; the entry point uses the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[MCRT_PSF_STATIC_TAPS];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// address of the current device's copy of `scratch`, looked up once per device
hipError_t scratch_ptr(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

int32_t psf_launch(const uint64_t* image, int32_t n_images, int32_t npix, double scale, double fwhm_pix,
                   double* weights, double* out, hipStream_t stream) {
  const int32_t r = mcrt_psf_radius(fwhm_pix);
  const double sigma = fwhm_pix / (2.0 * sqrt(2.0 * log(2.0)));
  k_psf_weights<<<1, 64, 0, stream>>>(sigma, r, weights);
  const int side = kTile + 2 * r;
  const size_t lds = sizeof(double) * ((size_t)side * side + (size_t)side * kTile + (size_t)(2 * r + 1));
  const dim3 grid((npix + kTile - 1) / kTile, (npix + kTile - 1) / kTile, n_images);
  k_psf<<<grid, dim3(kTile, kTile), lds, stream>>>(reinterpret_cast<const unsigned long long*>(image), npix,
                                                   scale, r, weights, out);
  return hipGetLastError() == hipSuccess ? MCRT_OK : MCRT_E_HIP;
}

}  // namespace

extern "C" int32_t mcrt_psf_radius(double fwhm_pix) {
  if (!(fwhm_pix >= 0.0) || fwhm_pix > MCRT_PSF_MAX_FWHM) return -1;
  const double sigma = fwhm_pix / (2.0 * sqrt(2.0 * log(2.0)));
  return (int32_t)ceil(3.0 * sigma);
}

extern "C" int32_t mcrt_image_psf(const uint64_t* image, int32_t n_images, int32_t npix, double scale,
                                  double fwhm_pix, double* weights, double* out, hipStream_t stream) {
  if (!image || !out || !weights || n_images < 1 || npix < 1 || npix > 4096) return MCRT_E_INVALID;
  if (!std::isfinite(scale)) return MCRT_E_NUMERIC;
  const int32_t r = mcrt_psf_radius(fwhm_pix);
  if (r < 0) return MCRT_E_INVALID;
  return psf_launch(image, n_images, npix, scale, fwhm_pix, weights, out, stream);
}

extern "C" int32_t mcrt_image_psf_static(const uint64_t* image, int32_t n_images, int32_t npix, double scale,
                                         double fwhm_pix, double* out, hipStream_t stream) {
  if (!image || !out || n_images < 1 || npix < 1 || npix > 4096) return MCRT_E_INVALID;
  if (!std::isfinite(scale)) return MCRT_E_NUMERIC;
  const int32_t r = mcrt_psf_radius(fwhm_pix);
  if (r < 0) return MCRT_E_INVALID;
  if (2 * r + 1 > MCRT_PSF_STATIC_TAPS) return MCRT_E_CAPACITY;
  double* w = nullptr;
  if (scratch_ptr(&w) != hipSuccess) return MCRT_E_HIP;
  return psf_launch(image, n_images, npix, scale, fwhm_pix, w, out, stream);
}
