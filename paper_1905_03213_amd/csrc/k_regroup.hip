// Rows regrouped by baseline (Section 2.2, Eqs. 5 and 6): the paper's GPU imager reads
// a measurement set whose rows (one timestamp of one baseline, all channels) are in time
// order and regroups them so that each baseline's rows are contiguous and in time order.
// It numbers baselines from the antenna pair (Eq. 5), counts the rows per baseline (the
// array C) and takes an exclusive prefix sum of C for each baseline's first row (Eq. 6).
//
// On the device this is a stable counting sort with blocks of R consecutive rows:
//   count   per block, a histogram of its rows' baseline numbers in LDS, written out
//           baseline-major: cnt[b * n_blocks + block];
//   scan    exclusive prefix sum of cnt: offs[b * n_blocks + block] is where the block's
//           first row of baseline b goes (all earlier baselines, then the same baseline
//           in earlier blocks), so offs[b * n_blocks] is Eq. 6's start of baseline b;
//   place   one wavefront per block walks its rows in order, 64 at a time, with running
//           per-baseline positions in LDS; lanes that share a baseline number take
//           consecutive positions in lane order, so the order inside a baseline is the
//           original row order.
// Rows whose antenna IDs fall outside [0, n_ant) get the extra number n_b and go last.
#include <algorithm>

#include "wproj_tiled.h"

namespace wproj {
namespace {

__device__ inline uint32_t baseline_number(int32_t a1, int32_t a2, int32_t n_ant, uint32_t n_b) {
  if (a1 < 0 || a2 < 0 || a1 >= n_ant || a2 >= n_ant) return n_b;
  const int64_t s = a1 < a2 ? a1 : a2;
  const int64_t d = a1 < a2 ? (int64_t)a2 - a1 : (int64_t)a1 - a2;
  return (uint32_t)((-s * s + 2 * s * n_ant + s) / 2 + d);  // Eq. 5, 0-based IDs
}

__device__ inline uint64_t lanes_below() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// One wavefront per block of R rows: LDS histogram of the block's baseline numbers.
__global__ void __launch_bounds__(64)
    regroup_count_kernel(int64_t n_rows, int64_t rows_per_block, const int32_t *__restrict__ ant1,
                         const int32_t *__restrict__ ant2, int32_t n_ant, uint32_t n_keys,
                         int64_t n_blocks, uint32_t *__restrict__ cnt) {
  extern __shared__ uint32_t hist[];
  for (uint32_t b = threadIdx.x; b < n_keys; b += 64) hist[b] = 0u;
  __syncthreads();
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = std::min(n_rows, r0 + rows_per_block);
  for (int64_t j = r0 + threadIdx.x; j < r1; j += 64)
    atomicAdd(&hist[baseline_number(ant1[j], ant2[j], n_ant, n_keys - 1)], 1u);
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < n_keys; b += 64) cnt[(int64_t)b * n_blocks + blockIdx.x] = hist[b];
}

// Eq. 6 per baseline and the counts C, as int64: start[b] = offs[b * n_blocks],
// counts[b] = start[b + 1] - start[b] (start[n_keys] = n_rows).
__global__ void __launch_bounds__(256)
    regroup_start_kernel(const uint32_t *__restrict__ offs, uint32_t n_keys, int64_t n_blocks,
                         int64_t n_rows, int64_t *__restrict__ start, int64_t *__restrict__ counts) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_keys) return;
  const int64_t s0 = offs[(int64_t)b * n_blocks];
  const int64_t s1 = b + 1 < n_keys ? (int64_t)offs[(int64_t)(b + 1) * n_blocks] : n_rows;
  start[b] = s0;
  counts[b] = s1 - s0;
}

// One wavefront per block: places the block's rows in order.
__global__ void __launch_bounds__(64)
    regroup_place_kernel(int64_t n_rows, int64_t rows_per_block, const int32_t *__restrict__ ant1,
                         const int32_t *__restrict__ ant2, int32_t n_ant, uint32_t n_keys,
                         int64_t n_blocks, const uint32_t *__restrict__ offs,
                         int64_t *__restrict__ perm) {
  extern __shared__ uint32_t next[];
  for (uint32_t b = threadIdx.x; b < n_keys; b += 64) next[b] = offs[(int64_t)b * n_blocks + blockIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = std::min(n_rows, r0 + rows_per_block);
  for (int64_t c = r0; c < r1; c += 64) {
    const int64_t j = c + lane;
    const bool valid = j < r1;
    const uint32_t key = valid ? baseline_number(ant1[j], ant2[j], n_ant, n_keys - 1) : 0xffffffffu;
    // lanes grouped by baseline number; each group takes consecutive positions in lane order
    uint64_t pending = __ballot(valid);
    uint32_t pos = 0;
    while (pending) {
      const int leader = __ffsll((unsigned long long)pending) - 1;
      const uint32_t lk = (uint32_t)__shfl((int)key, leader, 64);
      const uint64_t same = __ballot(key == lk) & pending;
      const uint32_t base = next[lk];  // every lane reads the same LDS word
      if (key == lk && valid) pos = base + (uint32_t)__popcll(same & lanes_below());
      __syncthreads();  // one wavefront: orders the read above before the update below
      if (lane == leader) next[lk] = base + (uint32_t)__popcll(same);
      __syncthreads();
      pending &= ~same;
    }
    if (valid) perm[pos] = j;
  }
}

// Channel-major visibility order of regrouped rows: baseline b's count_b rows (starting
// at start_b in the row permutation) become n_chan runs of count_b visibilities, one run
// per channel, each in time order.  gridDim.y = baselines, gridDim.x blocks per baseline
// stride over its count_b n_chan outputs (writes and perm reads both coalesced).
__global__ void __launch_bounds__(256)
    channel_order_kernel(int32_t n_chan, const int64_t *__restrict__ perm,
                         const int64_t *__restrict__ start, const int64_t *__restrict__ counts,
                         int64_t *__restrict__ vis_perm) {
  const int64_t b = blockIdx.y;
  const int64_t s0 = start[b], cnt = counts[b];
  const int64_t total = cnt * n_chan;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = k / cnt, t = k - c * cnt;
    vis_perm[s0 * n_chan + k] = perm[s0 + t] * n_chan + c;
  }
}

// Small rows (at most 4 words): one thread per row.
__global__ void __launch_bounds__(256)
    gather_small_rows_kernel(int64_t n_rows, int words, const int64_t *__restrict__ perm,
                             int64_t n_src_rows, const uint32_t *__restrict__ src,
                             uint32_t *__restrict__ dst, unsigned long long *bad) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_rows) return;
  const int64_t p = perm[k];
  if (p < 0 || p >= n_src_rows) {
    if (bad) atomicAdd(bad, 1ull);
    return;
  }
  for (int i = 0; i < words; ++i) dst[k * words + i] = src[p * words + i];
}

// dst row k <- src row perm[k], rows of `words` elements of type V (4 or 16 bytes); each
// wavefront copies one row at a time.
template <typename V>
__global__ void __launch_bounds__(256)
    gather_rows_kernel(int64_t n_rows, int64_t words, const int64_t *__restrict__ perm,
                       int64_t n_src_rows, const V *__restrict__ src, V *__restrict__ dst,
                       unsigned long long *bad) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t k = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); k < n_rows; k += waves) {
    const int64_t p = perm[k];
    if (p < 0 || p >= n_src_rows) {
      if (bad && lane == 0) atomicAdd(bad, 1ull);
      continue;
    }
    const V *s = src + p * words;
    V *d = dst + k * words;
    for (int64_t i = lane; i < words; i += 64) d[i] = s[i];
  }
}

}  // namespace

RegroupShape regroup_shape(int64_t n_rows, int32_t n_ant) {
  RegroupShape r;
  r.n_keys = (uint32_t)((int64_t)n_ant * (n_ant + 1) / 2 + 1);
  // at most 2^26 per-block counts: blocks grow with rows x baselines
  const int64_t min_rows = (n_rows * (int64_t)r.n_keys + (1ll << 26) - 1) >> 26;
  r.rows_per_block = std::max<int64_t>(2048, (min_rows + 63) / 64 * 64);
  r.n_blocks = std::max<int64_t>(1, (n_rows + r.rows_per_block - 1) / r.rows_per_block);
  r.n_counts = (int64_t)r.n_keys * r.n_blocks;
  return r;
}

int64_t regroup_workspace_bytes(const RegroupShape &r) {
  const int64_t words = r.n_counts + (r.n_counts + 1) + scan_temp_words(r.n_counts);
  return words * 4;
}

hipError_t launch_regroup(const RegroupShape &r, int64_t n_rows, const int32_t *ant1,
                          const int32_t *ant2, int32_t n_ant, int64_t *perm, int64_t *start,
                          int64_t *counts, void *workspace, hipStream_t s) {
  uint32_t *cnt = (uint32_t *)workspace;
  uint32_t *offs = cnt + r.n_counts;
  uint32_t *tmp = offs + r.n_counts + 1;
  const size_t lds = sizeof(uint32_t) * r.n_keys;
  hipError_t e = hipFuncSetAttribute((const void *)regroup_count_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void *)regroup_place_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(regroup_count_kernel, dim3((unsigned)r.n_blocks), dim3(64), lds, s, n_rows,
                     r.rows_per_block, ant1, ant2, n_ant, r.n_keys, r.n_blocks, cnt);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_exclusive_scan(cnt, offs, r.n_counts, tmp, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(regroup_start_kernel, dim3((r.n_keys + 255) / 256), dim3(256), 0, s, offs,
                     r.n_keys, r.n_blocks, n_rows, start, counts);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (n_rows == 0) return hipSuccess;
  hipLaunchKernelGGL(regroup_place_kernel, dim3((unsigned)r.n_blocks), dim3(64), lds, s, n_rows,
                     r.rows_per_block, ant1, ant2, n_ant, r.n_keys, r.n_blocks, offs, perm);
  return hipGetLastError();
}

hipError_t launch_channel_order(int64_t n_keys, int32_t n_chan, const int64_t *perm,
                                const int64_t *start, const int64_t *counts, int64_t *vis_perm,
                                hipStream_t s) {
  if (n_keys == 0) return hipSuccess;
  hipLaunchKernelGGL(channel_order_kernel, dim3(16, (unsigned)n_keys), dim3(256), 0, s, n_chan, perm,
                     start, counts, vis_perm);
  return hipGetLastError();
}

hipError_t launch_gather_rows(int64_t n_rows, int64_t row_bytes, const int64_t *perm,
                              int64_t n_src_rows, const void *src, void *dst, int64_t *bad,
                              hipStream_t s) {
  if (n_rows == 0) return hipSuccess;
  auto *b = reinterpret_cast<unsigned long long *>(bad);
  if (row_bytes <= 16) {
    hipLaunchKernelGGL(gather_small_rows_kernel, dim3((unsigned)((n_rows + 255) / 256)), dim3(256), 0, s,
                       n_rows, (int)(row_bytes / 4), perm, n_src_rows, (const uint32_t *)src,
                       (uint32_t *)dst, b);
    return hipGetLastError();
  }
  const unsigned blocks = (unsigned)std::min<int64_t>((n_rows + 3) / 4, 1 << 16);
  // 16-byte moves when rows and both buffers allow them
  if (row_bytes % 16 == 0 && (reinterpret_cast<uintptr_t>(src) & 15) == 0 &&
      (reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
    hipLaunchKernelGGL(gather_rows_kernel<uint4>, dim3(blocks), dim3(256), 0, s, n_rows, row_bytes / 16,
                       perm, n_src_rows, (const uint4 *)src, (uint4 *)dst, b);
  } else {
    hipLaunchKernelGGL(gather_rows_kernel<uint32_t>, dim3(blocks), dim3(256), 0, s, n_rows, row_bytes / 4,
                       perm, n_src_rows, (const uint32_t *)src, (uint32_t *)dst, b);
  }
  return hipGetLastError();
}

}  // namespace wproj
