// Elementwise kernels around the 2D FFTs.
//
// The centred transforms are reduced to rocFFT's unshifted ones.  For even n,
//   sum_X G[X] exp(+2 pi i (X - n/2)(x - n/2)/n) = (-1)^k IFFT(G)[k],  k = (x + n/2) mod n,
// because exp(2 pi i (X - n/2) k / n) = exp(2 pi i X k / n) (-1)^k; in 2D the two signs
// combine to (-1)^(x + y).  So grid -> image is an in-place unshifted inverse FFT followed
// by one pass that reads the shifted element, applies the sign, keeps the real part and
// multiplies by the grid correction kappa(x) kappa(y) / sumW (the taper divided out of
// the image).  Image -> grid runs the same identity backwards: one pass writes
// (-1)^(kx+ky) kappa kappa I at the shifted position, then an in-place forward FFT.
#include "wproj_internal.h"

namespace wproj {
namespace {

template <typename Real>
__global__ void g2i_kernel(int n, int n_images, const Real *__restrict__ F,
                           const double *__restrict__ kappa, const double *__restrict__ wsum,
                           Real *__restrict__ img) {
  const int64_t cells = (int64_t)n * n;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cells * n_images) return;
  const int i = (int)(t / cells);
  const int64_t r = t - (int64_t)i * cells;
  const int y = (int)(r / n), x = (int)(r - (int64_t)y * n);
  const int h = n / 2;
  const int ys = y + h < n ? y + h : y - h;
  const int xs = x + h < n ? x + h : x - h;
  const double re = (double)F[2 * (cells * i + (int64_t)ys * n + xs)];
  double scale = kappa[x] * kappa[y];
  if (wsum != nullptr) {
    const double s = wsum[i];
    scale = s != 0.0 ? scale / s : 0.0;
  }
  const double v = ((x + y) & 1) ? -re : re;
  img[t] = (Real)(v * scale);
}

template <typename Real>
__global__ void i2g_kernel(int n, int n_images, const Real *__restrict__ img,
                           const double *__restrict__ kappa, Real *__restrict__ G) {
  const int64_t cells = (int64_t)n * n;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cells * n_images) return;
  const int i = (int)(t / cells);
  const int64_t r = t - (int64_t)i * cells;
  const int ky = (int)(r / n), kx = (int)(r - (int64_t)ky * n);
  const int h = n / 2;
  const int y = ky + h < n ? ky + h : ky - h;
  const int x = kx + h < n ? kx + h : kx - h;
  const double v = (double)img[cells * i + (int64_t)y * n + x] * (kappa[x] * kappa[y]);
  G[2 * t] = (Real)(((kx + ky) & 1) ? -v : v);
  G[2 * t + 1] = (Real)0;
}

}  // namespace

hipError_t launch_g2i_correct(const wproj_kernels *k, const void *fgrid, void *image,
                              const double *wsum, hipStream_t s) {
  const int n = k->params.n, ni = k->params.n_images;
  const int64_t total = (int64_t)n * n * ni;
  const unsigned blocks = (unsigned)((total + 255) / 256);
  if (k->params.precision == WPROJ_F64)
    hipLaunchKernelGGL(g2i_kernel<double>, dim3(blocks), dim3(256), 0, s, n, ni,
                       (const double *)fgrid, k->d_kappa, wsum, (double *)image);
  else
    hipLaunchKernelGGL(g2i_kernel<float>, dim3(blocks), dim3(256), 0, s, n, ni,
                       (const float *)fgrid, k->d_kappa, wsum, (float *)image);
  return hipGetLastError();
}

hipError_t launch_i2g_precorrect(const wproj_kernels *k, const void *image, void *grid,
                                 hipStream_t s) {
  const int n = k->params.n, ni = k->params.n_images;
  const int64_t total = (int64_t)n * n * ni;
  const unsigned blocks = (unsigned)((total + 255) / 256);
  if (k->params.precision == WPROJ_F64)
    hipLaunchKernelGGL(i2g_kernel<double>, dim3(blocks), dim3(256), 0, s, n, ni,
                       (const double *)image, k->d_kappa, (double *)grid);
  else
    hipLaunchKernelGGL(i2g_kernel<float>, dim3(blocks), dim3(256), 0, s, n, ni,
                       (const float *)image, k->d_kappa, (float *)grid);
  return hipGetLastError();
}

}  // namespace wproj
