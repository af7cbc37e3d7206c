// Tiled degridder (the gather that is the adjoint of gridding):
//   V_j = sum_{kv,ku} conj(T_p[ov][ou][kv][ku]) M[y0+kv][x0+ku].
// Visibilities are binned by (image, uv-tile, w-plane) exactly as for gridding, but each
// record carries its visibility's row instead of W V.  A workgroup takes one work item
// (a run of records of one tile), copies that tile of the model grid plus its
// (S_max - 1)-cell halo into LDS with coalesced row loads, and then serves every
// record's footprint from LDS instead of gathering it from HBM.  The copy is only read,
// so the workgroup's wavefronts share it and split the item's records between them.
//
// Two kernels serve the records.  With FP32 arithmetic and tables and a fixed support
// up to 8, tap_lane_degrid_kernel (below) gives each lane one tap of a record, as the
// gridder does, and sums a record's products across lanes.  Otherwise (FP64, FP16
// tables, larger or per-plane supports) records go 8 at a time, a group of 8 lanes per
// record; lane r of a group takes footprint rows kv = r, r + 8, ...: a row's S taps are
// contiguous in the sub-kernel and its S cells contiguous in the LDS tile.  The group's
// partial sums are combined across its 8 lanes and the first lane of the group stores
// V_j.  Binned for that kernel alone, the tile copy has an odd row pitch (degrid_pitch),
// so the rows of a footprint start on different LDS banks whatever the bank count; plans
// share their records with the gridder and keep its pitch (an odd multiple of 8 cells,
// which suits the one-tap-per-lane pattern).
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

// Wavefronts sharing one work item (and one tile copy) in the row-per-lane degridder
// (2048^2 benchmark rows, tile 32, FP16 tables: 1.58 ms with a copy per wavefront, 1.44
// with four per copy, 1.34 with eight, 1.37 with sixteen; FP64 7.06 -> 6.65 ms).
constexpr int kDegridWaves = 8;
// Wavefronts sharing one work item (and one tile copy) in the one-tap-per-lane degridder
// (2048^2 benchmark rows, tile 32: 1.95 ms with one, 1.82 with four, 1.75 with eight,
// 1.80 with sixteen).
constexpr int kTeamWaves = 8;

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
    tiled_degrid_kernel(Geometry G, BinShape B, int pitch, int rows,
                        const Tab *__restrict__ tab, const Rec *__restrict__ rec,
                        const WorkItem *__restrict__ items, const uint32_t *__restrict__ order,
                        const uint32_t *__restrict__ n_items_ptr,
                        uint32_t *counter, const typename Cd<Real>::T *__restrict__ model,
                        typename Cd<Real>::T *__restrict__ out) {
  using C2 = typename Cd<Real>::T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ uint32_t s_item;
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  C2 *tile = reinterpret_cast<C2 *>(smem_raw);  // one copy for the workgroup's wavefronts
  const int grp = lane >> 3, r = lane & 7;
  const uint32_t n_items = *n_items_ptr;
  const int64_t cells = (int64_t)G.n * G.n;
  const int tiles_per_img = B.ntx * B.nty;
  const bool folding = G.w_mode != WPROJ_W_LINEAR;

  for (;;) {
    __syncthreads();  // every wave is done with the previous tile and item
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t it = s_item;
    if (it >= n_items) break;
    const WorkItem w = items[order[it]];  // largest items first
    const int img = (int)(w.tile / (uint32_t)tiles_per_img);
    const int rt = (int)(w.tile - (uint32_t)img * tiles_per_img);
    const int ty = rt / B.ntx, tx = rt - ty * B.ntx;
    const int ox = tx * B.tile, oy = ty * B.tile;
    const C2 *mimg = model + cells * img;
    for (int i = threadIdx.x; i < rows * rows; i += blockDim.x) {
      const int ry = i / rows, rx = i - ry * rows;
      const int gy = oy + ry, gx = ox + rx;
      C2 v;
      v.x = Real(0);
      v.y = Real(0);
      if (gy < G.n && gx < G.n) v = mimg[(int64_t)gy * G.n + gx];
      tile[ry * pitch + rx] = v;
    }
    __syncthreads();

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
      // wavefront wid takes batches wid, wid + kDegridWaves, ...
      constexpr uint32_t kStep = 64u * kDegridWaves;
      Rec cur;
      if ((uint32_t)wid * 64u < n_rec) load_batch((uint32_t)wid * 64u, cur);
      for (uint32_t b = (uint32_t)wid * 64u; b < n_rec; b += kStep) {
        Rec nxt;
        const bool more = b + kStep < n_rec;
        if (more) load_batch(b + kStep, nxt);
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
      for (uint32_t b = w.begin + (uint32_t)wid * 8u; b < w.end; b += 8u * kDegridWaves) {
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

// Fixed support S <= 8 with FP32 arithmetic and FP32 tables, packed records: the
// gridder's layout run backwards.  A work item is taken by a team of kTeamWaves
// wavefronts that share one tile copy, each taking every kTeamWaves-th batch of 64
// records (a copy per wavefront would leave room for 12 wavefronts per CU at tile 32).  Records go in pairs, one per
// half wavefront: lane
// j of a half takes taps j and h + j (h = ceil(S^2 / 2)) of its half's record, which one
// load from the pair-ordered table brings (entries 2j and 2j + 1 of a sub-kernel), and
// reads the two footprint cells they weight from the tile copy.  A half wavefront's
// cells are four footprint rows of one record, which the gridder's row pitch keeps free
// of bank conflicts (the records are binned with it).  Each lane sums conj(tap) * cell
// over its two taps; a record's prediction is the sum of those partial sums over its
// half wavefront.  The sums of a batch of 64 records are formed together by a
// transpose-reduce: each step combines two values into one, halving both the values a
// lane holds and the lanes each value spans (lanes 16 apart through the quarter-
// wavefront swap, then 8, 4, 2 and 1 apart through DPP moves), so that lane L ends with
// the prediction of the batch's record bitrev6(L).  The steps run as the pairs arrive,
// in the order of a binary counter over them, and a lane holds one pending value per step.
template <int STEP>
__device__ inline float combine(float a, float b, int lane) {
  if constexpr (STEP == 1) {  // lanes 16 apart: rows 1, 3 of a with rows 0, 2 of b
    const auto x = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(x[0]) + __uint_as_float(x[1]);
  } else {
    // lanes with the step's bit set keep b and receive the partner's b; the others keep a
    constexpr int bit = 5 - STEP;  // 8, 4, 2, 1 lanes apart
    constexpr int ctrl = STEP == 2 ? 0x128 : STEP == 3 ? 0x141 : STEP == 4 ? 0x4E : 0xB1;
    const bool hi = (lane >> bit) & 1;
    const float send = hi ? a : b, keep = hi ? b : a;
    return keep + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(send), ctrl, 0xF, 0xF, false));
  }
}

// The lane's two taps of its record from one pair-ordered load (FP32 table).
__device__ inline void tap_pair(const TapPair<float2>::Raw &v, float2 &a, float2 &b) {
  a = make_float2(__uint_as_float(v[0]), __uint_as_float(v[1]));
  b = make_float2(__uint_as_float(v[2]), __uint_as_float(v[3]));
}

template <typename Tab, int S>
__global__ void __launch_bounds__(64 * kTeamWaves)
    tap_lane_degrid_kernel(Geometry G, BinShape B, int pitch, int rows,
                           const Tab *__restrict__ tab, uint32_t tab_bytes,
                           const RecordF32 *__restrict__ rec, const WorkItem *__restrict__ items,
                           const uint32_t *__restrict__ order, const uint32_t *__restrict__ n_items_ptr,
                           uint32_t *counter, const float2 *__restrict__ model, float2 *__restrict__ out) {
  static_assert(S * S <= 64, "one pass of 64 taps");
  using P = TapPair<Tab>;
  using Raw = typename P::Raw;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ uint32_t s_item;
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  float2 *tile = reinterpret_cast<float2 *>(smem_raw);
  const uint32_t n_items = *n_items_ptr;
  const int64_t cells = (int64_t)G.n * G.n;
  const int tiles_per_img = B.ntx * B.nty;
  const bool folding = G.w_mode != WPROJ_W_LINEAR;
  const __amdgpu_buffer_rsrc_t tab_rsrc =
      __builtin_amdgcn_make_buffer_rsrc((void *)tab, (short)0, (int)tab_bytes, kBufferWord3);
  constexpr int kN = S * S, kH = (kN + 1) / 2;
  constexpr uint32_t kSubBytes = (uint32_t)(2 * kH) * P::kTapBytes;
  const int half = lane >> 5, j = lane & 31;
  uint32_t upper = half ? 0xffffffffu : 0u;
  asm volatile("" : "+v"(upper));  // keeps the selects below one vector AND each
  // taps j and h + j of the half's record, where they exist (lanes past the sub-kernel
  // read entry pair 0 and contribute nothing)
  const bool on1 = j < kH, on2 = j < kN - kH;
  uint32_t p_pair = (on1 ? (uint32_t)(2 * j) : 0u) * P::kTapBytes;
  asm volatile("" : "+v"(p_pair));
  // byte offsets (from smem_raw) of the lane's two cells in a footprint whose first cell
  // is the copy's cell 0
  const uint32_t tile0 = 0u;
  const int t1 = on1 ? j : 0, t2 = on2 ? kH + j : 0;
  uint32_t c1 = tile0 + (uint32_t)((t1 / S) * pitch + t1 % S) * 8u;
  uint32_t c2 = tile0 + (uint32_t)((t2 / S) * pitch + t2 % S) * 8u;
  asm volatile("" : "+v"(c1));
  asm volatile("" : "+v"(c2));
  // lane L ends with record bitrev6(L) of the batch
  const int mine = (int)(__builtin_bitreverse32((uint32_t)lane) >> 26);

  for (;;) {
    __syncthreads();  // every wave is done with the previous tile and item
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t it = s_item;
    if (it >= n_items) break;
    const WorkItem w = items[order[it]];  // largest items first
    const int img = (int)(w.tile / (uint32_t)tiles_per_img);
    const int rt = (int)(w.tile - (uint32_t)img * tiles_per_img);
    const int ty = rt / B.ntx, tx = rt - ty * B.ntx;
    const int ox = tx * B.tile, oy = ty * B.tile;
    const float2 *mimg = model + cells * img;
    for (int i = threadIdx.x; i < rows * rows; i += blockDim.x) {
      const int ry = i / rows, rx = i - ry * rows;
      const int gy = oy + ry, gx = ox + rx;
      float2 v = make_float2(0.0f, 0.0f);
      if (gy < G.n && gx < G.n) v = mimg[(int64_t)gy * G.n + gx];
      tile[ry * pitch + rx] = v;
    }
    __syncthreads();

    const uint32_t n_rec = w.end - w.begin;
    // records 64 at a time, lane i holding record i of the batch; padding lanes repeat
    // the last record and their predictions are not stored
    auto load_batch = [&](uint32_t b, RecordF32 &dst) {
      const uint32_t i = b + (uint32_t)lane;
      dst = rec[w.begin + (i < n_rec ? i : n_rec - 1)];
    };
    // the lane's two taps of record k (lower half) or k + 1 (upper half) of the batch
    // (sub-kernel numbers above the LDS offsets)
    auto fetch = [&](const RecordF32 &c, int k) {
      const uint32_t a = (bcast(c.lds, k) >> kLdsBits) * kSubBytes;
      const uint32_t d = (bcast(c.lds, k + 1) >> kLdsBits) * kSubBytes - a;
      return P::load(tab_rsrc, a + (upper & d) + p_pair);
    };
    // the lane's two footprint cells of record k (lower half) or k + 1 (upper half)
    auto cells = [&](const RecordF32 &c, int k, float2 &m1, float2 &m2) {
      const uint32_t a = (bcast(c.lds, k) & kLdsMask) * 8u;
      const uint32_t d = (bcast(c.lds, k + 1) & kLdsMask) * 8u - a;
      const uint32_t sel = (upper & d) + a;
      m1 = *reinterpret_cast<const float2 *>(smem_raw + (c1 + sel));
      m2 = *reinterpret_cast<const float2 *>(smem_raw + (c2 + sel));
    };
    // sum of conj(tap) * cell over the lane's two taps
    auto partial = [&](const Raw &v, const float2 &m1, const float2 &m2, float &re, float &im) {
      float2 ta, tb;
      tap_pair(v, ta, tb);
      if constexpr (kN < 64) {
        if (!on1) ta = make_float2(0.0f, 0.0f);
        if (!on2) tb = make_float2(0.0f, 0.0f);
      }
      re = __builtin_fmaf(ta.x, m1.x, ta.y * m1.y);
      re = __builtin_fmaf(tb.x, m2.x, re);
      re = __builtin_fmaf(tb.y, m2.y, re);
      im = __builtin_fmaf(ta.x, m1.y, -(ta.y * m1.x));
      im = __builtin_fmaf(tb.x, m2.y, im);
      im = __builtin_fmaf(-tb.y, m2.x, im);
    };
    constexpr uint32_t kStep = 64u * kTeamWaves;
    RecordF32 cur;
    if ((uint32_t)wid * 64u < n_rec) load_batch((uint32_t)wid * 64u, cur);
    for (uint32_t b = (uint32_t)wid * 64u; b < n_rec; b += kStep) {
      RecordF32 nxt;
      const bool more = b + kStep < n_rec;
      if (more) load_batch(b + kStep, nxt);
      // pending value of each step (1 .. 5), real and imaginary parts; [0]: the result
      float pr[6], pi[6];
      // pairs in groups of 4; a group's taps and cells load while the previous group is
      // reduced
      Raw c[2][4];
      float2 m[2][4][2];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        c[0][i] = fetch(cur, 2 * i);
        cells(cur, 2 * i, m[0][i][0], m[0][i][1]);
      }
#pragma unroll
      for (int g = 0; g < 8; ++g) {
        if (g + 1 < 8) {
#pragma unroll
          for (int i = 0; i < 4; ++i) c[(g + 1) & 1][i] = fetch(cur, 8 * (g + 1) + 2 * i);
        }
        if (g + 1 < 8) {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            cells(cur, 8 * (g + 1) + 2 * i, m[(g + 1) & 1][i][0], m[(g + 1) & 1][i][1]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int pair = 4 * g + i;
          // records 2 pair (lower half) and 2 pair + 1 (upper half)
          float vr, vi;
          partial(c[g & 1][i], m[g & 1][i][0], m[g & 1][i][1], vr, vi);
          // carry: step s combines the pending value (the earlier pairs) with this one
#pragma unroll
          for (int s = 1; s <= 5; ++s) {
            if (((pair >> (s - 1)) & 1) == 0) {
              pr[s] = vr;
              pi[s] = vi;
              break;
            }
            switch (s) {
              case 1: vr = combine<1>(pr[1], vr, lane); vi = combine<1>(pi[1], vi, lane); break;
              case 2: vr = combine<2>(pr[2], vr, lane); vi = combine<2>(pi[2], vi, lane); break;
              case 3: vr = combine<3>(pr[3], vr, lane); vi = combine<3>(pi[3], vi, lane); break;
              case 4: vr = combine<4>(pr[4], vr, lane); vi = combine<4>(pi[4], vi, lane); break;
              default: vr = combine<5>(pr[5], vr, lane); vi = combine<5>(pi[5], vi, lane); break;
            }
            if (s == 5) {
              pr[0] = vr;
              pi[0] = vi;
            }
          }
        }
      }
      const uint32_t row = (uint32_t)__shfl((int)get_row(cur), mine, 64);
      const bool fold = folding && __shfl(cur.wr, mine, 64) < 0.0f;
      if (b + (uint32_t)mine < n_rec) out[row] = make_float2(pr[0], fold ? -pi[0] : pi[0]);
      if (more) cur = nxt;
    }
  }
}

template <typename Tab, int S>
hipError_t launch_tap_lane(const wproj_kernels *k, const BinShape &B, const TileShape &ts,
                           const BinWorkspace &W, const void *model, void *out, hipStream_t s) {
  auto kern = tap_lane_degrid_kernel<Tab, S>;
  const int wpb = kTeamWaves;
  const size_t lds = ts.lds_bytes;
  hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * wpb, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  if (!k->d_tab_pair || k->pair_stride != pair_table_stride(S)) return hipErrorInvalidValue;
  const int64_t n_sub = (int64_t)k->params.n_wplanes * k->params.oversample * k->params.oversample;
  hipLaunchKernelGGL(kern, dim3((unsigned)(k->n_cu * per_cu)), dim3(64 * wpb), lds, s, k->geo, B,
                     ts.pitch, ts.rows, (const Tab *)k->d_tab_pair,
                     (uint32_t)(n_sub * k->pair_stride * (int64_t)sizeof(Tab)), (const RecordF32 *)W.rec,
                     W.items, W.order, W.choff + B.n_tiles, W.counter, (const float2 *)model, (float2 *)out);
  return hipGetLastError();
}

template <typename Real, typename Rec, typename Tab, int S>
hipError_t launch_one(const wproj_kernels *k, const BinShape &B, const TileShape &ts,
                      const BinWorkspace &W, const void *model, void *out, hipStream_t s) {
  using C2 = typename Cd<Real>::T;
  auto kern = tiled_degrid_kernel<Real, Rec, Tab, S>;
  const int wpb = kDegridWaves;
  const size_t lds = ts.lds_bytes;
  hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * wpb, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(kern, dim3((unsigned)(k->n_cu * per_cu)), dim3(64 * wpb), lds, s, k->geo, B,
                     ts.pitch, ts.rows, (const Tab *)k->d_tab, (const Rec *)W.rec,
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

template <typename Tab, int S>
hipError_t dispatch_tap_lane(const wproj_kernels *k, const BinShape &B, const TileShape &ts,
                             const BinWorkspace &W, const void *model, void *out, hipStream_t s) {
  if constexpr (S > 8) {
    return hipErrorInvalidValue;
  } else {
    if (k->s_max == S) return launch_tap_lane<Tab, S>(k, B, ts, W, model, out, s);
    return dispatch_tap_lane<Tab, S + 1>(k, B, ts, W, model, out, s);
  }
}

}  // namespace

bool tap_lane_degrid(const wproj_kernels *k, const BinShape &B) {
  return k->params.precision == WPROJ_F32 && B.pack_sub && k->s_max <= 8 && k->d_tab_pair != nullptr &&
         k->pair_stride == pair_table_stride(k->s_max);
}

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
  if (tap_lane_degrid(k, B)) return dispatch_tap_lane<float2, kMinFixedSupport>(k, B, ts, W, model_grid, vis_out, s);
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
