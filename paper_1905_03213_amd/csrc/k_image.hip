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
// With w-stacking an image has one grid per layer: the grid -> image pass combines the
// layers' transforms with their phase factors, and image -> grid writes every layer.
#include <algorithm>

#include "wproj_internal.h"

namespace wproj {
namespace {

// Launch shape of the per-pixel kernels: blockIdx.x * 256 + threadIdx.x is the column,
// blockIdx.y the row, and blockIdx.z steps through the images (or grids) by gridDim.z;
// no per-element integer division.  The correction kernels take up to kPixZ images per
// launch row, so that a thread corrects several images' pixels with one kappa lookup
// (64 images of 1024^2: 0.24 ms with one image per thread, 0.16 ms with a z extent of 16,
// the same with 4); the Hermitian-half kernel keeps one grid per thread (its transform
// phase was 0.01-0.03 ms slower with the smaller extents).
constexpr int kPixThreads = 256;
constexpr unsigned kMaxGridZ = 65535;
constexpr unsigned kPixZ = 16;

template <typename Real>
__global__ void __launch_bounds__(kPixThreads)
    g2i_kernel(int n, int n_images, const Real *__restrict__ F, const double *__restrict__ kappa,
               const double *__restrict__ wsum, Real *__restrict__ img) {
  const int x = (int)(blockIdx.x * kPixThreads + threadIdx.x), y = (int)blockIdx.y;
  if (x >= n) return;
  const int64_t cells = (int64_t)n * n;
  const int h = n / 2;
  const int ys = y + h < n ? y + h : y - h;
  const int xs = x + h < n ? x + h : x - h;
  const double kk = kappa[x] * kappa[y];
  for (int i = (int)blockIdx.z; i < n_images; i += (int)gridDim.z) {
    const double re = (double)F[2 * (cells * i + (int64_t)ys * n + xs)];
    double scale = kk;
    if (wsum != nullptr) {
      const double s = wsum[i];
      scale = s != 0.0 ? scale / s : 0.0;
    }
    const double v = ((x + y) & 1) ? -re : re;
    img[cells * i + (int64_t)y * n + x] = (Real)(v * scale);
  }
}

// Twice the Hermitian part of each grid on the half spectrum the complex-to-real
// transform reads: H[ky][kx] = G[ky][kx] + conj(G[-ky][-kx]) (indices mod n), kx in
// [0, n/2].  The inverse transform of the Hermitian part is the real part of the inverse
// transform of G.
template <typename Real>
__global__ void __launch_bounds__(kPixThreads)
    hermitian_half_kernel(int n, int n_grids, const Real *__restrict__ G, Real *__restrict__ H) {
  const int kx = (int)(blockIdx.x * kPixThreads + threadIdx.x), ky = (int)blockIdx.y;
  const int hw = n / 2 + 1;
  if (kx >= hw) return;
  const int64_t cells = (int64_t)n * n, half = (int64_t)n * hw;
  const int my = ky == 0 ? 0 : n - ky, mx = kx == 0 ? 0 : n - kx;
  for (int i = (int)blockIdx.z; i < n_grids; i += (int)gridDim.z) {
    const Real *g = G + 2 * cells * i;
    const int64_t a = 2 * ((int64_t)ky * n + kx), b = 2 * ((int64_t)my * n + mx);
    Real *h = H + 2 * (half * i + (int64_t)ky * hw + kx);
    h[0] = g[a] + g[b];
    h[1] = g[a + 1] - g[b + 1];
  }
}

// g2i_kernel on the real output R = 2 Re IFFT(G) of the complex-to-real transform.
template <typename Real>
__global__ void __launch_bounds__(kPixThreads)
    g2i_real_kernel(int n, int n_images, const Real *__restrict__ R, const double *__restrict__ kappa,
                    const double *__restrict__ wsum, Real *__restrict__ img) {
  const int x = (int)(blockIdx.x * kPixThreads + threadIdx.x), y = (int)blockIdx.y;
  if (x >= n) return;
  const int64_t cells = (int64_t)n * n;
  const int h = n / 2;
  const int ys = y + h < n ? y + h : y - h;
  const int xs = x + h < n ? x + h : x - h;
  const double kk = 0.5 * kappa[x] * kappa[y];
  for (int i = (int)blockIdx.z; i < n_images; i += (int)gridDim.z) {
    const double re = (double)R[cells * i + (int64_t)ys * n + xs];
    double scale = kk;
    if (wsum != nullptr) {
      const double s = wsum[i];
      scale = s != 0.0 ? scale / s : 0.0;
    }
    const double v = ((x + y) & 1) ? -re : re;
    img[cells * i + (int64_t)y * n + x] = (Real)(v * scale);
  }
}

template <typename Real>
__global__ void __launch_bounds__(kPixThreads)
    i2g_kernel(int n, int n_images, const Real *__restrict__ img, const double *__restrict__ kappa,
               Real *__restrict__ G) {
  const int kx = (int)(blockIdx.x * kPixThreads + threadIdx.x), ky = (int)blockIdx.y;
  if (kx >= n) return;
  const int64_t cells = (int64_t)n * n;
  const int h = n / 2;
  const int y = ky + h < n ? ky + h : ky - h;
  const int x = kx + h < n ? kx + h : kx - h;
  const double kk = kappa[x] * kappa[y];
  const bool odd = (kx + ky) & 1;
  for (int i = (int)blockIdx.z; i < n_images; i += (int)gridDim.z) {
    const double v = (double)img[cells * i + (int64_t)y * n + x] * kk;
    const int64_t t = cells * i + (int64_t)ky * n + kx;
    G[2 * t] = (Real)(odd ? -v : v);
    G[2 * t + 1] = (Real)0;
  }
}

// w-stacking: n - 1 at pixel (x, y), n = sqrt(1 - l^2 - m^2), l = (x - n/2) cell,
// m = (y - n/2) cell; false outside the unit circle (no sky there: the layer factor is 0).
__device__ inline bool n_minus_1(const Geometry &G, int x, int y, double &nm1) {
#pragma clang fp contract(off)
  const double l = ((double)x - (double)G.n / 2.0) * G.cell;
  const double m = ((double)y - (double)G.n / 2.0) * G.cell;
  const double r2 = l * l + m * m;
  if (!(r2 < 1.0)) return false;
  nm1 = sqrt(1.0 - r2) - 1.0;
  return true;
}

// Layer centre w_l = -w_max + (l + 1/2) D, the same operations as the footprint rule.
__device__ inline double layer_centre(const Geometry &G, int layer) {
#pragma clang fp contract(off)
  return -G.w_max + ((double)layer + 0.5) * G.layer_w;
}

// Grid -> image with w-stacking: for image i, Re(sum over layers l of
// IDFT(G_{i,l})[y][x] exp(+2 pi i w_l (n - 1))) kappa(x) kappa(y) / sumW_i.  F holds the
// unshifted inverse FFTs of the n_images L grids (layer fastest).
template <typename Real>
__global__ void __launch_bounds__(kPixThreads)
    g2i_stack_kernel(Geometry G, const Real *__restrict__ F, const double *__restrict__ kappa,
                     const double *__restrict__ wsum, Real *__restrict__ img) {
  const int n = G.n, L = G.n_layers;
  const int x = (int)(blockIdx.x * kPixThreads + threadIdx.x), y = (int)blockIdx.y;
  if (x >= n) return;
  const int64_t cells = (int64_t)n * n;
  const int h = n / 2;
  const int ys = y + h < n ? y + h : y - h;
  const int xs = x + h < n ? x + h : x - h;
  double nm1 = 0.0;
  const bool sky = n_minus_1(G, x, y, nm1);
  const double kk = kappa[x] * kappa[y];
  for (int i = (int)blockIdx.z; i < G.n_images; i += (int)gridDim.z) {
    double acc = 0.0;
    if (sky) {
      for (int l = 0; l < L; ++l) {
        const int64_t e = 2 * (cells * ((int64_t)i * L + l) + (int64_t)ys * n + xs);
        const double re = (double)F[e], im = (double)F[e + 1];
        double sn, cs;
        sincospi(2.0 * layer_centre(G, l) * nm1, &sn, &cs);
        acc += re * cs - im * sn;  // Re((re + i im)(cs + i sn))
      }
    }
    double scale = kk;
    if (wsum != nullptr) {
      const double s = wsum[i];
      scale = s != 0.0 ? scale / s : 0.0;
    }
    const double v = ((x + y) & 1) ? -acc : acc;
    img[cells * i + (int64_t)y * n + x] = (Real)(v * scale);
  }
}

// Image -> grids with w-stacking: layer l of image i gets the shifted, sign-flipped
// kappa kappa I exp(-2 pi i w_l (n - 1)) (then forward FFTs, as for one grid).
template <typename Real>
__global__ void __launch_bounds__(kPixThreads)
    i2g_stack_kernel(Geometry G, const Real *__restrict__ img, const double *__restrict__ kappa,
                     Real *__restrict__ Gr) {
  const int n = G.n, L = G.n_layers;
  const int kx = (int)(blockIdx.x * kPixThreads + threadIdx.x), ky = (int)blockIdx.y;
  if (kx >= n) return;
  const int64_t cells = (int64_t)n * n;
  const int h = n / 2;
  const int y = ky + h < n ? ky + h : ky - h;
  const int x = kx + h < n ? kx + h : kx - h;
  const double kk = kappa[x] * kappa[y];
  double nm1 = 0.0;
  const bool sky = n_minus_1(G, x, y, nm1);
  const bool odd = (kx + ky) & 1;
  for (int g = (int)blockIdx.z; g < G.n_grids; g += (int)gridDim.z) {
    const int i = g / L, l = g - i * L;
    const double v = (double)img[cells * i + (int64_t)y * n + x] * kk;
    double re = 0.0, im = 0.0;
    if (sky) {
      double sn, cs;
      sincospi(2.0 * layer_centre(G, l) * nm1, &sn, &cs);
      re = v * cs;
      im = -v * sn;
    }
    const int64_t t = cells * g + (int64_t)ky * n + kx;
    Gr[2 * t] = (Real)(odd ? -re : re);
    Gr[2 * t + 1] = (Real)(odd ? -im : im);
  }
}

inline dim3 pixel_grid(int n, int planes) {
  return dim3((unsigned)((n + kPixThreads - 1) / kPixThreads), (unsigned)n, std::min((unsigned)planes, kPixZ));
}

}  // namespace

hipError_t launch_g2i_correct(const wproj_kernels *k, const void *fgrid, void *image,
                              const double *wsum, hipStream_t s) {
  const int n = k->params.n, ni = k->params.n_images;
  const dim3 grid = pixel_grid(n, ni), block(kPixThreads);
  if (k->params.w_mode == WPROJ_W_STACK) {
    if (k->params.precision == WPROJ_F64)
      hipLaunchKernelGGL(g2i_stack_kernel<double>, grid, block, 0, s, k->geo, (const double *)fgrid,
                         k->d_kappa, wsum, (double *)image);
    else
      hipLaunchKernelGGL(g2i_stack_kernel<float>, grid, block, 0, s, k->geo, (const float *)fgrid,
                         k->d_kappa, wsum, (float *)image);
    return hipGetLastError();
  }
  if (k->params.precision == WPROJ_F64)
    hipLaunchKernelGGL(g2i_kernel<double>, grid, block, 0, s, n, ni, (const double *)fgrid, k->d_kappa,
                       wsum, (double *)image);
  else
    hipLaunchKernelGGL(g2i_kernel<float>, grid, block, 0, s, n, ni, (const float *)fgrid, k->d_kappa,
                       wsum, (float *)image);
  return hipGetLastError();
}

hipError_t launch_hermitian_half(const wproj_kernels *k, const void *grid, void *half, hipStream_t s) {
  const int n = k->params.n, ng = k->geo.n_grids;
  const dim3 g3((unsigned)((n / 2 + 1 + kPixThreads - 1) / kPixThreads), (unsigned)n,
                std::min((unsigned)ng, kMaxGridZ));
  if (k->params.precision == WPROJ_F64)
    hipLaunchKernelGGL(hermitian_half_kernel<double>, g3, dim3(kPixThreads), 0, s, n, ng, (const double *)grid,
                       (double *)half);
  else
    hipLaunchKernelGGL(hermitian_half_kernel<float>, g3, dim3(kPixThreads), 0, s, n, ng, (const float *)grid,
                       (float *)half);
  return hipGetLastError();
}

hipError_t launch_g2i_correct_real(const wproj_kernels *k, const void *real, void *image,
                                   const double *wsum, hipStream_t s) {
  const int n = k->params.n, ni = k->params.n_images;
  const dim3 grid = pixel_grid(n, ni), block(kPixThreads);
  if (k->params.precision == WPROJ_F64)
    hipLaunchKernelGGL(g2i_real_kernel<double>, grid, block, 0, s, n, ni, (const double *)real, k->d_kappa,
                       wsum, (double *)image);
  else
    hipLaunchKernelGGL(g2i_real_kernel<float>, grid, block, 0, s, n, ni, (const float *)real, k->d_kappa,
                       wsum, (float *)image);
  return hipGetLastError();
}

hipError_t launch_i2g_precorrect(const wproj_kernels *k, const void *image, void *grid,
                                 hipStream_t s) {
  const int n = k->params.n, ni = k->params.n_images;
  const dim3 block(kPixThreads);
  if (k->params.w_mode == WPROJ_W_STACK) {
    const dim3 g3 = pixel_grid(n, k->geo.n_grids);
    if (k->params.precision == WPROJ_F64)
      hipLaunchKernelGGL(i2g_stack_kernel<double>, g3, block, 0, s, k->geo, (const double *)image,
                         k->d_kappa, (double *)grid);
    else
      hipLaunchKernelGGL(i2g_stack_kernel<float>, g3, block, 0, s, k->geo, (const float *)image,
                         k->d_kappa, (float *)grid);
    return hipGetLastError();
  }
  const dim3 g3 = pixel_grid(n, ni);
  if (k->params.precision == WPROJ_F64)
    hipLaunchKernelGGL(i2g_kernel<double>, g3, block, 0, s, n, ni, (const double *)image, k->d_kappa,
                       (double *)grid);
  else
    hipLaunchKernelGGL(i2g_kernel<float>, g3, block, 0, s, n, ni, (const float *)image, k->d_kappa,
                       (float *)grid);
  return hipGetLastError();
}

}  // namespace wproj
