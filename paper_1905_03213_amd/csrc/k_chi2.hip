// chi^2 of predicted visibilities against observed ones, and its gradient: the loss of the
// differentiable forward model (model image -> degridded visibilities), fused into one
// pass over the visibilities.
//   chi2 = sum_j w_j |o_j - p_j|^2,   g_j = d chi2 / d Re p_j + i d chi2 / d Im p_j
//        = -2 w_j (o_j - p_j).
// The sum is taken in FP64 in a fixed order (each thread of a fixed grid strides through
// the visibilities, blocks reduce in LDS, one block adds the block sums in index order),
// so its value does not depend on scheduling.
#include <algorithm>

#include "wproj_internal.h"

namespace wproj {
namespace {

constexpr int kChi2Threads = 256;
constexpr int kChi2Blocks = 1024;

template <typename Real>
struct Cplx2;
template <>
struct Cplx2<float> {
  using T = float2;
};
template <>
struct Cplx2<double> {
  using T = double2;
};

template <typename Real>
__global__ void __launch_bounds__(kChi2Threads)
    chi2_partial_kernel(int64_t nvis, const typename Cplx2<Real>::T *__restrict__ obs,
                        const typename Cplx2<Real>::T *__restrict__ pred, const Real *__restrict__ wt,
                        typename Cplx2<Real>::T *__restrict__ grad, double *__restrict__ partial) {
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kChi2Threads;
  for (int64_t j = (int64_t)blockIdx.x * kChi2Threads + threadIdx.x; j < nvis; j += stride) {
    const auto o = obs[j];
    const auto p = pred[j];
    const Real w = wt ? wt[j] : Real(1);
    const Real rr = o.x - p.x, ri = o.y - p.y;
    acc += (double)w * ((double)rr * (double)rr + (double)ri * (double)ri);
    if (grad) {
      typename Cplx2<Real>::T g;
      g.x = Real(-2) * w * rr;
      g.y = Real(-2) * w * ri;
      grad[j] = g;
    }
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  __shared__ double s[kChi2Threads / 64];
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < kChi2Threads / 64; ++i) t += s[i];
    partial[blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(64) chi2_final_kernel(const double *__restrict__ partial, int n, double *chi2) {
  if (threadIdx.x != 0) return;
  double t = 0.0;
  for (int i = 0; i < n; ++i) t += partial[i];
  chi2[0] = t;
}

}  // namespace
}  // namespace wproj

extern "C" {

int64_t wproj_chi2_workspace_size(void) { return (int64_t)wproj::kChi2Blocks * (int64_t)sizeof(double); }

int wproj_chi2(int precision, int64_t nvis, const void *vis_obs, const void *pred, const void *weight,
               double *chi2, void *grad, void *workspace, int64_t workspace_bytes, void *stream) {
  using namespace wproj;
  if (precision < WPROJ_F64 || precision > WPROJ_F32_F16TABLE)
    return set_error(WPROJ_EINVAL, "wproj_chi2: unknown precision");
  if (nvis < 0) return set_error(WPROJ_EINVAL, "wproj_chi2: nvis < 0");
  if (!chi2) return set_error(WPROJ_EINVAL, "wproj_chi2: chi2 is NULL");
  if (nvis > 0 && (!vis_obs || !pred)) return set_error(WPROJ_EINVAL, "wproj_chi2: vis_obs and pred are required");
  if (!workspace || workspace_bytes < wproj_chi2_workspace_size())
    return set_error(WPROJ_EWORKSPACE, "wproj_chi2: the workspace needs wproj_chi2_workspace_size() bytes");
  hipStream_t s = (hipStream_t)stream;
  double *partial = (double *)workspace;
  const unsigned blocks = (unsigned)std::min<int64_t>(kChi2Blocks, std::max<int64_t>(1, (nvis + kChi2Threads - 1) / kChi2Threads));
  if (precision == WPROJ_F64)
    hipLaunchKernelGGL(chi2_partial_kernel<double>, dim3(blocks), dim3(kChi2Threads), 0, s, nvis,
                       (const double2 *)vis_obs, (const double2 *)pred, (const double *)weight, (double2 *)grad,
                       partial);
  else
    hipLaunchKernelGGL(chi2_partial_kernel<float>, dim3(blocks), dim3(kChi2Threads), 0, s, nvis,
                       (const float2 *)vis_obs, (const float2 *)pred, (const float *)weight, (float2 *)grad,
                       partial);
  hipLaunchKernelGGL(chi2_final_kernel, dim3(1), dim3(64), 0, s, partial, (int)blocks, chi2);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(WPROJ_EHIP, hipGetErrorString(e));
  return WPROJ_OK;
}

}  // extern "C"
