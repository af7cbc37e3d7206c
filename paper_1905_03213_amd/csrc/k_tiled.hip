// Tiled gridder: each work item is a run of binned records of one uv-tile; its
// workgroup accumulates them in an LDS copy of the tile plus an (S_max - 1)-cell halo
// on the high-x / high-y sides, then adds the non-zero cells to the grid in HBM with
// global atomics.  Most of the read-modify-write traffic of gridding therefore stays
// in LDS instead of going to HBM (the paper's CUDA gridder writes every tap of every
// visibility to global memory atomically, Section 2.2).
//
// Launch is persistent: one wave of workgroups sized to fill every CU pulls work items
// from a queue head in HBM until the queue is empty, which evens out the very uneven
// per-tile visibility counts of Earth-rotation tracks.
//
// Inside a workgroup each wavefront takes 64 consecutive records with one coalesced
// load, then walks them one at a time, broadcasting each record's fields from its
// owning lane (readlane); the 64 lanes cover the S x S taps of the record: lane t loads
// tap t of the sub-kernel (one coalesced 8-byte load per lane) and adds
// W V C into LDS at (y0 + kv, x0 + ku).  The LDS tile is stored as separate real and
// imaginary planes with a row pitch chosen so that the rows of a footprint land in
// different banks.
#include "wproj_tiled.h"

namespace wproj {
namespace {

__device__ inline float2 tab_load(const float2 *t, uint32_t i) { return t[i]; }
__device__ inline double2 tab_load(const double2 *t, uint32_t i) { return t[i]; }
__device__ inline float2 tab_load(const half2c *t, uint32_t i) {
  const half2c h = t[i];
  return make_float2((float)h.re, (float)h.im);
}

__device__ inline uint32_t bcast(uint32_t v, int j) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, j);
}
__device__ inline float bcast(float v, int j) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}
__device__ inline double bcast(double v, int j) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), j);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), j);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <typename Real, typename Rec, typename Tab, int S, int BS>
__global__ void __launch_bounds__(BS)
    tiled_grid_kernel(Geometry G, BinShape B, int pitch, int rows, const Tab *__restrict__ tab,
                      const Rec *__restrict__ rec, const WorkItem *__restrict__ items,
                      const uint32_t *__restrict__ n_items_ptr, uint32_t *counter, Real *grid) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Real *sre = reinterpret_cast<Real *>(smem_raw);
  const int plane = rows * pitch;
  Real *sim = sre + plane;
  __shared__ uint32_t s_item;
  constexpr int NW = BS / 64;
  const uint32_t n_items = *n_items_ptr;
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int64_t cells = (int64_t)G.n * G.n;
  const int tiles_per_img = B.ntx * B.nty;
  // fixed-support lanes: tap (kv, ku) of lane t = kv S + ku
  const int lane_kv = S > 0 ? lane / (S > 0 ? S : 1) : 0;
  const int lane_ku = S > 0 ? lane - lane_kv * S : 0;

  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t it = s_item;
    if (it >= n_items) break;
    const WorkItem w = items[it];
    const int img = (int)(w.tile / (uint32_t)tiles_per_img);
    const int rt = (int)(w.tile - (uint32_t)img * tiles_per_img);
    const int ty = rt / B.ntx, tx = rt - ty * B.ntx;
    const int ox = tx * B.tile, oy = ty * B.tile;
    for (int i = threadIdx.x; i < 2 * plane; i += BS) sre[i] = Real(0);
    __syncthreads();

    for (uint32_t r0 = w.begin + (uint32_t)wid * 64u; r0 < w.end; r0 += NW * 64u) {
      Rec mine;
      if (r0 + lane < w.end) {
        mine = rec[r0 + lane];
      } else {
        mine.xy = 0;
        mine.tap = 0;
        mine.wr = Real(0);
        mine.wi = Real(0);
      }
      const int cnt = (int)min(64u, w.end - r0);
      for (int j = 0; j < cnt; ++j) {
        const uint32_t xy = bcast(mine.xy, j);
        const uint32_t tp = bcast(mine.tap, j);
        const Real wr = bcast(mine.wr, j);
        const Real wi = bcast(mine.wi, j);
        const int lx = (int)(xy & 0xffffu) - ox;
        const int ly = (int)(xy >> 16) - oy;
        const uint32_t tb = tp & kTapMask;
        const int base = ly * pitch + lx;
        if (S > 0 && S * S <= 64) {
          if (lane < S * S) {
            const auto c = tab_load(tab, tb + lane);
            const Real gr = wr * c.x - wi * c.y;
            const Real gi = wr * c.y + wi * c.x;
            const int a = base + lane_kv * pitch + lane_ku;
            atomicAdd(&sre[a], gr);
            atomicAdd(&sim[a], gi);
          }
        } else {
          const int Sr = S > 0 ? S : (int)(tp >> kTapBits) + 1;
          for (int t = lane; t < Sr * Sr; t += 64) {
            const int kv = t / Sr, ku = t - kv * Sr;
            const auto c = tab_load(tab, tb + t);
            const Real gr = wr * c.x - wi * c.y;
            const Real gi = wr * c.y + wi * c.x;
            const int a = base + kv * pitch + ku;
            atomicAdd(&sre[a], gr);
            atomicAdd(&sim[a], gi);
          }
        }
      }
    }
    __syncthreads();

    Real *g = grid + 2 * cells * img;
    for (int i = threadIdx.x; i < plane; i += BS) {
      const Real vr = sre[i], vi = sim[i];
      if (vr != Real(0) || vi != Real(0)) {
        const int ry = i / pitch, rx = i - ry * pitch;
        const int gx = ox + rx, gy = oy + ry;
        if (rx < rows && gx < G.n && gy < G.n) {
          const int64_t c = (int64_t)gy * G.n + gx;
          unsafeAtomicAdd(&g[2 * c], vr);
          unsafeAtomicAdd(&g[2 * c + 1], vi);
        }
      }
    }
    __syncthreads();
  }
}

template <typename Real, typename Rec, typename Tab, int S, int BS>
hipError_t launch_one(const wproj_kernels *k, const BinShape &B, const TileShape &ts,
                      const BinWorkspace &W, void *grid, hipStream_t s) {
  auto kern = tiled_grid_kernel<Real, Rec, Tab, S, BS>;
  hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)ts.lds_bytes);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, BS, ts.lds_bytes);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  const unsigned blocks = (unsigned)(k->n_cu * per_cu);
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(BS), ts.lds_bytes, s, k->geo, B, ts.pitch, ts.rows,
                     (const Tab *)k->d_tab, (const Rec *)W.rec, W.items, W.choff + B.n_tiles,
                     W.counter, (Real *)grid);
  return hipGetLastError();
}

template <typename Real, typename Rec, typename Tab>
hipError_t dispatch_support(const wproj_kernels *k, const BinShape &B, const TileShape &ts,
                            const BinWorkspace &W, void *grid, hipStream_t s) {
  constexpr int BS = 512;
  if (k->uniform_support && k->s_max == 8)
    return launch_one<Real, Rec, Tab, 8, BS>(k, B, ts, W, grid, s);
  if (k->uniform_support && k->s_max == 7)
    return launch_one<Real, Rec, Tab, 7, BS>(k, B, ts, W, grid, s);
  return launch_one<Real, Rec, Tab, 0, BS>(k, B, ts, W, grid, s);
}

}  // namespace

TileShape tile_shape(const wproj_kernels *k, int tile) {
  TileShape t;
  t.tile = tile;
  t.rows = tile + k->s_max - 1;
  const int sref = k->uniform_support ? (k->s_max & 31) : 16;
  int pitch = t.rows;
  while ((pitch & 31) != sref) ++pitch;
  t.pitch = pitch;
  const size_t real = k->params.precision == WPROJ_F64 ? 8 : 4;
  t.lds_bytes = 2 * (size_t)t.rows * t.pitch * real;
  return t;
}

hipError_t launch_tiled_grid(const wproj_kernels *k, const BinShape &B, const BinWorkspace &W,
                             void *grid, hipStream_t s) {
  const TileShape ts = tile_shape(k, B.tile);
  hipError_t e = launch_fill_u32(W.counter, 1, 0u, s);
  if (e != hipSuccess) return e;
  switch (k->params.precision) {
    case WPROJ_F64:
      return dispatch_support<double, RecordF64, double2>(k, B, ts, W, grid, s);
    case WPROJ_F32:
      return dispatch_support<float, RecordF32, float2>(k, B, ts, W, grid, s);
    default:
      return dispatch_support<float, RecordF32, half2c>(k, B, ts, W, grid, s);
  }
}

}  // namespace wproj
