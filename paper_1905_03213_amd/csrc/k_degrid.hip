// Tiled degridder (the gather that is the adjoint of gridding):
//   V_j = sum_{kv,ku} conj(T_p[ov][ou][kv][ku]) M[y0+kv][x0+ku].
// Visibilities are binned by (image, uv-tile, w-plane) exactly as for gridding, but each
// record carries its visibility's row instead of W V.  A wavefront takes one work item
// (a run of records of one tile), copies that tile of the model grid plus its
// (S_max - 1)-cell halo into its private LDS with coalesced row loads, and then serves
// every record's footprint from LDS instead of gathering it from HBM.
//
// Records go 8 at a time, a group of 8 lanes per record; lane r of a group takes
// footprint rows kv = r, r + 8, ...: a row's S taps are contiguous in the sub-kernel and
// its S cells contiguous in the LDS tile.  The group's partial sums are combined across
// its 8 lanes and the first lane of the group stores V_j.  Binned for degridding alone,
// the tile copy has an odd row pitch (degrid_pitch), so the rows of a footprint start on
// different LDS banks whatever the bank count; plans share their records with the
// gridder and keep its pitch (an odd multiple of 8 cells, which suits the gridder's
// one-tap-per-lane pattern).
#include <algorithm>
#include <type_traits>

#include "wproj_tiled.h"

namespace wproj {
namespace {

template <typename Real> struct Cd;
template <> struct Cd<float> { using T = float2; };
template <> struct Cd<double> { using T = double2; };

__device__ inline float2 tap_at(const float2 *t, uint32_t i) { return t[i]; }
__device__ inline double2 tap_at(const double2 *t, uint32_t i) { return t[i]; }
__device__ inline float2 tap_at(const half2c *t, uint32_t i) {
  const half2c h = t[i];
  return make_float2((float)h.re, (float)h.im);
}

constexpr int kDegridWaves = 4;

// (re, im) += conj(k) m as four fused multiply-adds (written out, because the compiler
// otherwise forms a product, a fused multiply-add and an add per component)
__device__ inline float fma_r(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fma_r(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <typename Real, typename C2>
__device__ inline void mac_conj(Real &re, Real &im, Real kx, Real ky, const C2 &m) {
  re = fma_r(kx, m.x, re);
  re = fma_r(ky, m.y, re);
  im = fma_r(kx, m.y, im);
  im = fma_r(-ky, m.x, im);
}

// Sum over each aligned group of 8 lanes, valid in the group's first lane: DPP quad
// permutes pair lanes 1 and 2 apart, then a row shift brings lane +4.
__device__ inline float dpp_f(float v, int ctrl) {
  switch (ctrl) {
    case 0xB1: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
    case 0x4E: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));
    default: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x104, 0xF, 0xF, false));
  }
}
__device__ inline float group8_sum(float v) {
  v += dpp_f(v, 0xB1);  // quad_perm [1,0,3,2]
  v += dpp_f(v, 0x4E);  // quad_perm [2,3,0,1]
  v += dpp_f(v, 0x104); // row_shl:4 (lane i reads lane i + 4 of its row of 16)
  return v;
}
__device__ inline double group8_sum(double v) {
  v += __shfl_xor(v, 1, 64);
  v += __shfl_xor(v, 2, 64);
  v += __shfl_xor(v, 4, 64);
  return v;
}

template <typename Real, typename Rec, typename Tab, int S>
__global__ void __launch_bounds__(64 * kDegridWaves)
    tiled_degrid_kernel(Geometry G, BinShape B, int pitch, int rows, int wave_lds,
                        const Tab *__restrict__ tab, const Rec *__restrict__ rec,
                        const WorkItem *__restrict__ items, const uint32_t *__restrict__ order,
                        const uint32_t *__restrict__ n_items_ptr,
                        uint32_t *counter, const typename Cd<Real>::T *__restrict__ model,
                        typename Cd<Real>::T *__restrict__ out) {
  using C2 = typename Cd<Real>::T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  C2 *tile = reinterpret_cast<C2 *>(smem_raw) + (size_t)wid * wave_lds;
  const int grp = lane >> 3, r = lane & 7;
  const uint32_t n_items = *n_items_ptr;
  const int64_t cells = (int64_t)G.n * G.n;
  const int tiles_per_img = B.ntx * B.nty;
  const bool folding = G.w_mode != WPROJ_W_LINEAR;

  for (;;) {
    uint32_t got = 0;
    if (lane == 0) got = atomicAdd(counter, 1u);
    const uint32_t it = (uint32_t)__builtin_amdgcn_readlane((int)got, 0);
    if (it >= n_items) break;
    const WorkItem w = items[order[it]];  // largest items first
    const int img = (int)(w.tile / (uint32_t)tiles_per_img);
    const int rt = (int)(w.tile - (uint32_t)img * tiles_per_img);
    const int ty = rt / B.ntx, tx = rt - ty * B.ntx;
    const int ox = tx * B.tile, oy = ty * B.tile;
    const C2 *mimg = model + cells * img;
    // this wavefront's earlier reads of the previous tile precede these writes: LDS
    // executes one wavefront's instructions in order; the barrier keeps the compiler
    // from moving accesses across
    __builtin_amdgcn_wave_barrier();
    for (int i = lane; i < rows * rows; i += 64) {
      const int ry = i / rows, rx = i - ry * rows;
      const int gy = oy + ry, gx = ox + rx;
      C2 v;
      v.x = Real(0);
      v.y = Real(0);
      if (gy < G.n && gx < G.n) v = mimg[(int64_t)gy * G.n + gx];
      tile[ry * pitch + rx] = v;
    }
    __builtin_amdgcn_wave_barrier();

    if constexpr (S > 0 && S <= 8) {
      // Fixed support: records arrive 64 at a time in one coalesced load (lane i holds
      // record i of the batch; the next batch loads while this one is processed).  Group g
      // of 8 lanes takes record 8 t + g in step t, fetched from its holder lane with a
      // shuffle, and its lane r the footprint row kv = r.  A step's taps are loaded one
      // step ahead, and the group's partial sums are combined with DPP moves.
      const uint32_t n_rec = w.end - w.begin;
      auto load_batch = [&](uint32_t b, Rec &dst) {
        const uint32_t i = b + (uint32_t)lane;
        dst = rec[w.begin + (i < n_rec ? i : n_rec - 1)];  // padding lanes repeat the last record
      };
      auto fetch = [&](const Rec &c, int t, C2 *tap_row, uint32_t &tb_out, int &base_out, uint32_t &row_out,
                       bool &fold_out) {
        const int j = t * 8 + grp;
        const uint32_t tp = (uint32_t)__shfl((int)c.tap, j, 64);
        base_out = __shfl((int)c.lds, j, 64) & (int)kLdsMask;
        row_out = (uint32_t)__shfl((int)get_row(c), j, 64);
        // a Hermitian-folded row (negative weight in its record) predicts the conjugate
        fold_out = folding && __shfl(c.wr, j, 64) < Real(0);
        tb_out = tp & kTapMask;
        const uint32_t kv = r < S ? (uint32_t)r : 0u;
#pragma unroll
        for (int ku = 0; ku < S; ++ku) {
          const auto k = tap_at(tab + tb_out + kv * (uint32_t)S, (uint32_t)ku);
          tap_row[ku].x = k.x;
          tap_row[ku].y = k.y;
        }
      };
      Rec cur;
      if (n_rec > 0) load_batch(0, cur);
      for (uint32_t b = 0; b < n_rec; b += 64) {
        Rec nxt;
        const bool more = b + 64 < n_rec;
        if (more) load_batch(b + 64, nxt);
        // taps are loaded kAhead steps ahead: one with FP32/FP64 tables, two with FP16
        // tables, whose half-size loads leave registers and bandwidth for the deeper
        // prefetch (measured: FP16 1.66 -> 1.57 ms on the 2048^2 benchmark rows; FP32 got
        // slower, 2.30 -> 2.39 ms)
        constexpr int kAhead = std::is_same_v<Tab, half2c> ? 2 : 1;
        constexpr int kSlots = kAhead + 1;
        C2 taps[kSlots][S];
        uint32_t tb[kSlots], row[kSlots];
        int base[kSlots];
        bool fl[kSlots];
#pragma unroll
        for (int t = 0; t < kAhead; ++t) fetch(cur, t, taps[t], tb[t], base[t], row[t], fl[t]);
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int q = t % kSlots;
          if (t + kAhead < 8) {
            const int qn = (t + kAhead) % kSlots;
            fetch(cur, t + kAhead, taps[qn], tb[qn], base[qn], row[qn], fl[qn]);
          }
          Real re = 0, im = 0;
          if (r < S) {
            const C2 *mrow = tile + base[q] + r * pitch;
#pragma unroll
            for (int ku = 0; ku < S; ++ku) {
              const C2 m = mrow[ku];
              mac_conj(re, im, taps[q][ku].x, taps[q][ku].y, m);
            }
          }
          re = group8_sum(re);
          im = group8_sum(im);
          const uint32_t jr = b + (uint32_t)(t * 8 + grp);
          if (r == 0 && jr < n_rec) {
            C2 o;
            o.x = re;
            o.y = fl[q] ? -im : im;
            out[row[q]] = o;
          }
        }
        if (more) cur = nxt;
      }
    } else {
      for (uint32_t b = w.begin; b < w.end; b += 8) {
        const uint32_t jr = b + (uint32_t)grp;
        const bool valid = jr < w.end;
        const Rec rr = rec[valid ? jr : w.begin];
        const int Sr = S > 0 ? S : (int)(rr.tap >> kTapBits) + 1;
        const uint32_t tb = rr.tap & kTapMask;
        const int base = (int)(rr.lds & kLdsMask);
        Real re = 0, im = 0;
        if (valid) {
          for (int kv = r; kv < Sr; kv += 8) {
            const Tab *trow = tab + tb + (uint32_t)(kv * Sr);
            const C2 *mrow = tile + base + kv * pitch;
            for (int ku = 0; ku < Sr; ++ku) {
              const auto k = tap_at(trow, (uint32_t)ku);
              const C2 m = mrow[ku];
              mac_conj(re, im, (Real)k.x, (Real)k.y, m);
            }
          }
        }
        re = group8_sum(re);
        im = group8_sum(im);
        if (r == 0 && valid) {
          C2 o;
          o.x = re;
          o.y = rr.wr < Real(0) ? -im : im;  // a Hermitian-folded row predicts the conjugate
          out[get_row(rr)] = o;
        }
      }
    }
  }
}

template <typename Real, typename Rec, typename Tab, int S>
hipError_t launch_one(const wproj_kernels *k, const BinShape &B, const TileShape &ts,
                      const BinWorkspace &W, const void *model, void *out, hipStream_t s) {
  using C2 = typename Cd<Real>::T;
  auto kern = tiled_degrid_kernel<Real, Rec, Tab, S>;
  const int wpb = (int)std::max<size_t>(1, std::min<size_t>(kDegridWaves, k->max_lds / ts.lds_bytes));
  const size_t lds = ts.lds_bytes * wpb;
  hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * wpb, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  const int wave_lds = (int)(ts.lds_bytes / sizeof(C2));
  hipLaunchKernelGGL(kern, dim3((unsigned)(k->n_cu * per_cu)), dim3(64 * wpb), lds, s, k->geo, B,
                     ts.pitch, ts.rows, wave_lds, (const Tab *)k->d_tab, (const Rec *)W.rec,
                     W.items, W.order, W.choff + B.n_tiles, W.counter, (const C2 *)model, (C2 *)out);
  return hipGetLastError();
}

template <typename Real, typename Rec, typename Tab, int S>
hipError_t dispatch_fixed(const wproj_kernels *k, const BinShape &B, const TileShape &ts,
                          const BinWorkspace &W, const void *model, void *out, hipStream_t s) {
  if constexpr (S > 8) {
    return launch_one<Real, Rec, Tab, 0>(k, B, ts, W, model, out, s);
  } else {
    if (k->s_max == S) return launch_one<Real, Rec, Tab, S>(k, B, ts, W, model, out, s);
    return dispatch_fixed<Real, Rec, Tab, S + 1>(k, B, ts, W, model, out, s);
  }
}

// a fixed support from 3 to 8 (one footprint row per lane of a group) has its own kernel
template <typename Real, typename Rec, typename Tab>
hipError_t dispatch(const wproj_kernels *k, const BinShape &B, const TileShape &ts,
                    const BinWorkspace &W, const void *model, void *out, hipStream_t s) {
  if (k->uniform_support && k->s_max >= 3 && k->s_max <= 8)
    return dispatch_fixed<Real, Rec, Tab, 3>(k, B, ts, W, model, out, s);
  return launch_one<Real, Rec, Tab, 0>(k, B, ts, W, model, out, s);
}

}  // namespace

hipError_t launch_tiled_degrid(const wproj_kernels *k, const BinShape &B, const BinWorkspace &W,
                               const void *model_grid, void *vis_out, int64_t nvis, hipStream_t s) {
  // the tile copy uses the row pitch the records' LDS offsets were binned with
  TileShape ts = tile_shape(k, B.tile);
  ts.pitch = B.pitch;
  ts.lds_bytes = (size_t)ts.rows * ts.pitch * (k->params.precision == WPROJ_F64 ? 16 : 8);
  // rows that are dropped or belong to no image keep a zero prediction
  const int64_t words = nvis * (k->params.precision == WPROJ_F64 ? 4 : 2);
  hipError_t e = launch_fill_u32((uint32_t *)vis_out, words, 0u, s);
  if (e != hipSuccess) return e;
  if ((e = launch_fill_u32(W.counter, 1, 0u, s)) != hipSuccess) return e;
  switch (k->params.precision) {
    case WPROJ_F64:
      return dispatch<double, RecordF64, double2>(k, B, ts, W, model_grid, vis_out, s);
    case WPROJ_F32:
      return dispatch<float, RecordF32, float2>(k, B, ts, W, model_grid, vis_out, s);
    default:
      return dispatch<float, RecordF32, half2c>(k, B, ts, W, model_grid, vis_out, s);
  }
}

}  // namespace wproj
