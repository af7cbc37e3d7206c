// Plain gridder and degridder: no binning, every tap goes straight to the grid in HBM
// with a global atomic add (gridding) or a gather (degridding).  This is a per-tap
// atomic baseline, not the paper's GPU gridder: that one (Section 2.2) also spreads
// threads over convolution taps with atomic writes to global memory, but each thread
// first sums consecutive timestamps of one baseline in a register and writes only when
// the baseline changes.  It serves as the comparison path for the tiled gridder; in
// FP64 it is the double-precision baseline.
//
// One 64-lane wavefront owns a contiguous range of visibilities and handles them one
// at a time, its lanes covering the S_p x S_p taps (64 at a time).
#include "wproj_internal.h"

namespace wproj {
namespace {

__device__ inline double2 load_tap(const double2 *t, int64_t i) { return t[i]; }
__device__ inline float2 load_tap(const float2 *t, int64_t i) { return t[i]; }
__device__ inline float2 load_tap(const half2c *t, int64_t i) {
  half2c h = t[i];
  return make_float2((float)h.re, (float)h.im);
}

template <typename Real, typename Cplx, typename Tab>
__global__ void __launch_bounds__(256)
    plain_grid_kernel(Geometry G, const Tab *__restrict__ tab, int64_t nvis,
                      const double *__restrict__ uvw, const Cplx *__restrict__ vis,
                      const Real *__restrict__ wt, const int64_t *__restrict__ img_off,
                      Real *grid, double *wsum, unsigned long long *counters, int64_t per_wave) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t j0 = wave * per_wave;
  const int64_t j1 = min(nvis, j0 + per_wave);
  const int64_t cells = (int64_t)G.n * G.n;
  double wacc = 0.0;
  int wimg = -1;
  unsigned long long c_drop = 0, c_clamp = 0, c_bad = 0;
  for (int64_t j = j0; j < j1; ++j) {
    const int img = image_of(img_off, G.n_images, j);
    if (img < 0) continue;
    const Real w = wt[j];
    Footprint f;
    const int c = classify(G, uvw + 3 * j, w, f);
    if (c != kGridded) {
      c_drop += (c == kDropped);
      c_bad += (c == kBadWeight);
      continue;
    }
    if (w_clamped(G, uvw[3 * j + 2])) ++c_clamp;
    if (img != wimg) {
      if (wimg >= 0 && wsum && lane == 0) unsafeAtomicAdd(&wsum[wimg], wacc);
      wacc = 0.0;
      wimg = img;
    }
    wacc += (double)w;
    const Cplx v = vis[j];
    const Real ar = w * v.x, ai = (f.fold ? -w : w) * v.y;  // a folded row enters conjugated
    const int S = G.supp[f.p];
    const Tab *T = tab + G.tab_off[f.p] + ((int64_t)f.ov * G.O + f.ou) * S * S;
    Real *gimg = grid + 2 * cells * grid_of(G, img, f);
    for (int t = lane; t < S * S; t += 64) {
      const int kv = t / S, ku = t - kv * S;
      const auto k = load_tap(T, t);
      const Real gr = ar * k.x - ai * k.y;
      const Real gi = ar * k.y + ai * k.x;
      const int64_t cell = (int64_t)(f.y0 + kv) * G.n + (f.x0 + ku);
      unsafeAtomicAdd(&gimg[2 * cell], gr);
      unsafeAtomicAdd(&gimg[2 * cell + 1], gi);
    }
  }
  if (lane == 0) {
    if (wimg >= 0 && wsum) unsafeAtomicAdd(&wsum[wimg], wacc);
    if (counters) {
      if (c_drop) atomicAdd(&counters[0], c_drop);
      if (c_clamp) atomicAdd(&counters[1], c_clamp);
      if (c_bad) atomicAdd(&counters[2], c_bad);
    }
  }
}

// Degridding: 8 visibilities per wavefront pass, a group of 8 lanes per visibility.
// Lane r of a group takes footprint rows kv = r, r + 8, ... and walks each row's taps:
// the row's S taps are contiguous in the sub-kernel and the row's S cells contiguous in
// the grid, so a group reads whole 64-byte runs.  The 8 partial sums of a visibility are
// combined with three butterfly shuffles inside the group.  Each lane works out its own
// visibility's footprint (the same FP64 rule as gridding).
template <typename Real, typename Cplx, typename Tab>
__global__ void __launch_bounds__(256)
    plain_degrid_kernel(Geometry G, const Tab *__restrict__ tab, int64_t nvis,
                        const double *__restrict__ uvw, const Cplx *__restrict__ grid,
                        const int64_t *__restrict__ img_off, Cplx *__restrict__ out,
                        int64_t per_wave) {
  const int lane = threadIdx.x & 63;
  const int grp = lane >> 3, r = lane & 7;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t j0 = wave * per_wave;
  const int64_t j1 = min(nvis, j0 + per_wave);
  const int64_t cells = (int64_t)G.n * G.n;
  for (int64_t jb = j0; jb < j1; jb += 8) {
    const int64_t j = jb + grp;
    Real re = 0, im = 0;
    bool fold = false;
    if (j < j1) {
      const int img = image_of(img_off, G.n_images, j);
      Footprint f;
      if (img >= 0 && classify(G, uvw + 3 * j, 1.0, f) == kGridded) {
        fold = f.fold;
        const int S = G.supp[f.p];
        const Tab *T = tab + G.tab_off[f.p] + ((int64_t)f.ov * G.O + f.ou) * S * S;
        const Cplx *gimg = grid + cells * grid_of(G, img, f);
        for (int kv = r; kv < S; kv += 8) {
          const Tab *trow = T + kv * S;
          const Cplx *grow = gimg + (int64_t)(f.y0 + kv) * G.n + f.x0;
          for (int ku = 0; ku < S; ++ku) {
            const auto k = load_tap(trow, ku);
            const Cplx m = grow[ku];
            re += k.x * m.x + k.y * m.y;  // conj(k) * m
            im += k.x * m.y - k.y * m.x;
          }
        }
      }
    }
    re += __shfl_xor(re, 1, 64);
    im += __shfl_xor(im, 1, 64);
    re += __shfl_xor(re, 2, 64);
    im += __shfl_xor(im, 2, 64);
    re += __shfl_xor(re, 4, 64);
    im += __shfl_xor(im, 4, 64);
    if (r == 0 && j < j1) {
      Cplx o;
      o.x = re;
      o.y = fold ? -im : im;  // a Hermitian-folded row predicts the conjugate
      out[j] = o;
    }
  }
}

inline void plain_shape(int64_t nvis, unsigned &blocks, int64_t &per_wave) {
  const int64_t max_waves = 256 * 32;  // 256 CUs x 32 waves
  int64_t waves = nvis < max_waves ? (nvis > 0 ? nvis : 1) : max_waves;
  per_wave = (nvis + waves - 1) / waves;
  if (per_wave < 1) per_wave = 1;
  waves = (nvis + per_wave - 1) / per_wave;
  if (waves < 1) waves = 1;
  blocks = (unsigned)((waves + 3) / 4);  // 4 waves per 256-thread block
}

}  // namespace

hipError_t launch_plain_grid(const wproj_kernels *k, int64_t nvis, const double *uvw,
                             const void *vis, const void *wt, const int64_t *img_off, void *grid,
                             double *wsum, int64_t *counters, hipStream_t s) {
  unsigned blocks;
  int64_t per_wave;
  plain_shape(nvis, blocks, per_wave);
  auto *cnt = reinterpret_cast<unsigned long long *>(counters);
  switch (k->params.precision) {
    case WPROJ_F64:
      hipLaunchKernelGGL((plain_grid_kernel<double, double2, double2>), dim3(blocks), dim3(256), 0,
                         s, k->geo, (const double2 *)k->d_tab, nvis, uvw, (const double2 *)vis,
                         (const double *)wt, img_off, (double *)grid, wsum, cnt, per_wave);
      break;
    case WPROJ_F32:
      hipLaunchKernelGGL((plain_grid_kernel<float, float2, float2>), dim3(blocks), dim3(256), 0, s,
                         k->geo, (const float2 *)k->d_tab, nvis, uvw, (const float2 *)vis,
                         (const float *)wt, img_off, (float *)grid, wsum, cnt, per_wave);
      break;
    default:
      hipLaunchKernelGGL((plain_grid_kernel<float, float2, half2c>), dim3(blocks), dim3(256), 0, s,
                         k->geo, (const half2c *)k->d_tab, nvis, uvw, (const float2 *)vis,
                         (const float *)wt, img_off, (float *)grid, wsum, cnt, per_wave);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_plain_degrid(const wproj_kernels *k, int64_t nvis, const double *uvw,
                               const void *grid, const int64_t *img_off, void *vis_out,
                               hipStream_t s) {
  unsigned blocks;
  int64_t per_wave;
  plain_shape(nvis, blocks, per_wave);
  switch (k->params.precision) {
    case WPROJ_F64:
      hipLaunchKernelGGL((plain_degrid_kernel<double, double2, double2>), dim3(blocks), dim3(256),
                         0, s, k->geo, (const double2 *)k->d_tab, nvis, uvw,
                         (const double2 *)grid, img_off, (double2 *)vis_out, per_wave);
      break;
    case WPROJ_F32:
      hipLaunchKernelGGL((plain_degrid_kernel<float, float2, float2>), dim3(blocks), dim3(256), 0,
                         s, k->geo, (const float2 *)k->d_tab, nvis, uvw, (const float2 *)grid,
                         img_off, (float2 *)vis_out, per_wave);
      break;
    default:
      hipLaunchKernelGGL((plain_degrid_kernel<float, float2, half2c>), dim3(blocks), dim3(256), 0,
                         s, k->geo, (const half2c *)k->d_tab, nvis, uvw, (const float2 *)grid,
                         img_off, (float2 *)vis_out, per_wave);
      break;
  }
  return hipGetLastError();
}

namespace {

// One thread per visibility: its footprint and class, exactly as every gridding and
// degridding kernel decides them.
template <typename Real>
__global__ void __launch_bounds__(256)
    footprint_kernel(Geometry G, int64_t nvis, const double *__restrict__ uvw,
                     const Real *__restrict__ wt, int32_t *__restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nvis) return;
  Footprint f;
  const int cls = classify(G, uvw + 3 * j, wt ? wt[j] : Real(1), f);
  int32_t *o = out + 6 * j;
  const bool on = cls == kGridded;
  o[0] = on ? f.x0 : -1;
  o[1] = on ? f.y0 : -1;
  o[2] = on ? f.ou : -1;
  o[3] = on ? f.ov : -1;
  o[4] = on ? f.layer * G.n_w + f.p : -1;  // w-stacking: plane counted across layers
  o[5] = on && f.fold ? kGriddedFolded : cls;
}

}  // namespace

hipError_t launch_footprints(const wproj_kernels *k, int64_t nvis, const double *uvw,
                             const void *wt, int32_t *out, hipStream_t s) {
  if (nvis == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((nvis + 255) / 256);
  if (k->params.precision == WPROJ_F64)
    hipLaunchKernelGGL(footprint_kernel<double>, dim3(blocks), dim3(256), 0, s, k->geo, nvis, uvw,
                       (const double *)wt, out);
  else
    hipLaunchKernelGGL(footprint_kernel<float>, dim3(blocks), dim3(256), 0, s, k->geo, nvis, uvw,
                       (const float *)wt, out);
  return hipGetLastError();
}

}  // namespace wproj
