// Data-rate measurements on the device: LDS (the denominator of the tile gridder's
// LDS roofline) and the vector-memory return path from L1 (the path the kernel-table
// taps of the gridder and degridder take).
//
// LDS:
// Every workgroup streams 64-bit accesses through its own LDS buffer with the access
// shape of the gridder's private tiles: each lane of a wavefront touches its own 8-byte
// word, the 64 words of one instruction are consecutive (no bank conflicts), and each
// lane keeps kChains independent accesses in flight.  Modes:
//   0  reads   (ds_read_b64; the values are summed so that none is dead)
//   1  writes  (ds_write_b64)
//   2  read, add, write of the same word (the gridder's accumulation)
// The address moves by a runtime stride every round so that nothing can be hoisted out
// of the loop.  Bytes moved = blocks x threads x rounds x kChains x 8 (x 2 for mode 2).
#include <algorithm>

#include "wproj_internal.h"

namespace wproj {
namespace {

constexpr int kRateThreads = 256;
constexpr int kChains = 8;
constexpr int kRateWords = 2048;  // float2 words per workgroup: 16 KiB of LDS

template <int MODE>
__global__ void __launch_bounds__(kRateThreads)
    lds_rate_kernel(int rounds, int stride, float seed, float2 *__restrict__ sink) {
  __shared__ float2 buf[kRateWords];
  const int t = threadIdx.x;
  for (int i = t; i < kRateWords; i += kRateThreads) buf[i] = make_float2(seed * i, seed);
  __syncthreads();
  const int wave = t >> 6, lane = t & 63;
  // each wavefront walks its own quarter of the buffer (512 words, 8 chains x 64 lanes)
  float2 *mine = buf + wave * (kRateWords / 4);
  float ax = 0.0f, ay = 0.0f;
  int off = 0;
  for (int r = 0; r < rounds; ++r) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      const int a = ((c * 64 + off) & (kRateWords / 4 - 1) & ~63) + lane;
      if constexpr (MODE == 0) {
        const float2 v = mine[a];
        ax += v.x;
        ay += v.y;
      } else if constexpr (MODE == 1) {
        mine[a] = make_float2(ax + (float)c, ay);
      } else {
        float2 v = mine[a];
        v.x += seed;
        v.y += seed;
        mine[a] = v;
      }
    }
    off += stride;
    if constexpr (MODE == 1) ax += seed;
  }
  __syncthreads();
  if constexpr (MODE != 0) {
    ax += mine[lane].x;
    ay += mine[lane].y;
  }
  // never true for the seeds the host passes; keeps every access live
  if (ax == -1.0f && ay == -1.0f) sink[blockIdx.x * kRateThreads + t] = make_float2(ax, ay);
}

hipError_t launch_lds_rate(int mode, int n_cu, int rounds, float2 *sink, int64_t *bytes,
                           unsigned *blocks_out, hipStream_t s) {
  auto kern = mode == 0 ? lds_rate_kernel<0> : mode == 1 ? lds_rate_kernel<1> : lds_rate_kernel<2>;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kRateThreads, 0);
  if (e != hipSuccess) return e;
  // at most 64 workgroups per CU: the sink the caller passes holds that many
  const unsigned blocks = (unsigned)(n_cu * std::min(std::max(per_cu, 1), 64));
  *blocks_out = blocks;
  *bytes = (int64_t)blocks * kRateThreads * rounds * kChains * 8 * (mode == 2 ? 2 : 1);
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(kRateThreads), 0, s, rounds, 64 * 3, 0.5f, sink);
  return hipGetLastError();
}

// Vector-memory return rate: every lane loads W bytes per instruction (buffer loads of
// 4, 8 or 16 bytes, as the tap fetches are) from a 16 KiB window that stays in L1,
// kChains loads in flight per lane; 64 consecutive lanes read consecutive words, and
// the address moves by a runtime stride each round.  The dwords are folded with XOR so
// that none is dead.  Bytes moved = blocks x threads x rounds x kChains x W.
constexpr uint32_t kVmemWindow = 16384;

template <int W>
__global__ void __launch_bounds__(kRateThreads)
    vmem_rate_kernel(const uint32_t *__restrict__ win, int rounds, uint32_t stride, uint32_t *__restrict__ sink) {
  const __amdgpu_buffer_rsrc_t r =
      __builtin_amdgcn_make_buffer_rsrc((void *)win, (short)0, (int)kVmemWindow, 0x00020000);
  const int t = threadIdx.x;
  const uint32_t wave = (uint32_t)(t >> 6), lane = (uint32_t)(t & 63);
  uint32_t acc = 0, off = wave * 64u * (uint32_t)W * kChains;
  for (int i = 0; i < rounds; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      const uint32_t a = (off + (uint32_t)c * 64u * (uint32_t)W + lane * (uint32_t)W) & (kVmemWindow - 1u);
      if constexpr (W == 16) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, a, 0, 0);
        acc ^= v[0] ^ v[1] ^ v[2] ^ v[3];
      } else if constexpr (W == 8) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, a, 0, 0);
        acc ^= v[0] ^ v[1];
      } else {
        acc ^= __builtin_amdgcn_raw_buffer_load_b32(r, a, 0, 0);
      }
    }
    off += stride;
  }
  // the window holds zeros, so acc is 0 and nothing is stored; keeps every load live
  if (acc == 0xdeadbeefu) sink[blockIdx.x * kRateThreads + t] = acc;
}

hipError_t launch_vmem_rate(int width, int n_cu, int rounds, const uint32_t *win, uint32_t *sink,
                            int64_t *bytes, hipStream_t s) {
  auto kern = width == 16 ? vmem_rate_kernel<16> : width == 8 ? vmem_rate_kernel<8> : vmem_rate_kernel<4>;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kRateThreads, 0);
  if (e != hipSuccess) return e;
  const unsigned blocks = (unsigned)(n_cu * std::min(std::max(per_cu, 1), 64));
  *bytes = (int64_t)blocks * kRateThreads * rounds * kChains * width;
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(kRateThreads), 0, s, win, rounds, 3u * 64u * 16u, sink);
  return hipGetLastError();
}

}  // namespace
}  // namespace wproj

extern "C" int wproj_measure_vmem(int width, int32_t rounds, double *bytes_per_second, double *ms,
                                  void *stream) {
  using namespace wproj;
  if (width != 4 && width != 8 && width != 16) return set_error(WPROJ_EINVAL, "width must be 4, 8 or 16 bytes");
  if (rounds < 1 || rounds > (1 << 20)) return set_error(WPROJ_EINVAL, "rounds must be in [1, 2^20]");
  if (!bytes_per_second) return set_error(WPROJ_EINVAL, "bytes_per_second is NULL");
  hipStream_t s = (hipStream_t)stream;
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return set_error(WPROJ_EHIP, "device query failed");
  const int n_cu = prop.multiProcessorCount;
  uint32_t *win = nullptr, *sink = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  struct Guard {
    uint32_t *&w, *&k;
    hipEvent_t &a, &b;
    ~Guard() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
      (void)hipFree(w);
      (void)hipFree(k);
    }
  } guard{win, sink, e0, e1};
  const size_t sink_bytes = (size_t)n_cu * 64 * kRateThreads * sizeof(uint32_t);
  if (hipMalloc(&win, kVmemWindow) != hipSuccess || hipMalloc(&sink, sink_bytes) != hipSuccess)
    return set_error(WPROJ_ENOMEM, "buffer allocation failed");
  if (hipMemset(win, 0, kVmemWindow) != hipSuccess) return set_error(WPROJ_EHIP, "hipMemset failed");
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return set_error(WPROJ_EHIP, "hipEventCreate failed");
  int64_t bytes = 0;
  if (launch_vmem_rate(width, n_cu, rounds, win, sink, &bytes, s) != hipSuccess)  // warm-up
    return set_error(WPROJ_EHIP, "vector-memory rate kernel launch failed");
  if (hipEventRecord(e0, s) != hipSuccess || launch_vmem_rate(width, n_cu, rounds, win, sink, &bytes, s) != hipSuccess ||
      hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
    return set_error(WPROJ_EHIP, "vector-memory rate measurement failed");
  float t = 0.0f;
  if (hipEventElapsedTime(&t, e0, e1) != hipSuccess || !(t > 0.0f))
    return set_error(WPROJ_EHIP, "hipEventElapsedTime failed");
  *bytes_per_second = (double)bytes / ((double)t * 1e-3);
  if (ms) *ms = t;
  return WPROJ_OK;
}

extern "C" int wproj_measure_lds(int mode, int32_t rounds, double *bytes_per_second, double *ms,
                                 void *stream) {
  using namespace wproj;
  if (mode < 0 || mode > 2) return set_error(WPROJ_EINVAL, "mode must be 0 (read), 1 (write) or 2 (read-add-write)");
  if (rounds < 1 || rounds > (1 << 20)) return set_error(WPROJ_EINVAL, "rounds must be in [1, 2^20]");
  if (!bytes_per_second) return set_error(WPROJ_EINVAL, "bytes_per_second is NULL");
  hipStream_t s = (hipStream_t)stream;
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return set_error(WPROJ_EHIP, "device query failed");
  const int n_cu = prop.multiProcessorCount;
  float2 *sink = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  struct Guard {
    float2 *&p;
    hipEvent_t &a, &b;
    ~Guard() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
      (void)hipFree(p);
    }
  } guard{sink, e0, e1};
  // the sink is written only if a lane's sum hits an impossible value; sized for every lane
  const size_t sink_bytes = (size_t)n_cu * 64 * kRateThreads * sizeof(float2);
  if (hipMalloc(&sink, sink_bytes) != hipSuccess) return set_error(WPROJ_ENOMEM, "sink allocation failed");
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return set_error(WPROJ_EHIP, "hipEventCreate failed");
  int64_t bytes = 0;
  unsigned blocks = 0;
  if (launch_lds_rate(mode, n_cu, rounds, sink, &bytes, &blocks, s) != hipSuccess)  // warm-up
    return set_error(WPROJ_EHIP, "LDS rate kernel launch failed");
  if (hipEventRecord(e0, s) != hipSuccess ||
      launch_lds_rate(mode, n_cu, rounds, sink, &bytes, &blocks, s) != hipSuccess ||
      hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
    return set_error(WPROJ_EHIP, "LDS rate measurement failed");
  float t = 0.0f;
  if (hipEventElapsedTime(&t, e0, e1) != hipSuccess || !(t > 0.0f))
    return set_error(WPROJ_EHIP, "hipEventElapsedTime failed");
  *bytes_per_second = (double)bytes / ((double)t * 1e-3);
  if (ms) *ms = t;
  return WPROJ_OK;
}
