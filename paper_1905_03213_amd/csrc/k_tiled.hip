// Tiled gridder: each work item is a run of binned records of one uv-tile.  One
// wavefront owns the work item and accumulates its records in a private LDS copy of
// the tile plus an (S_max - 1)-cell halo on the high-x / high-y sides, then stores the
// copy to the work item's slot of a partial-tile buffer; tile_reduce_kernel adds the
// slots to the grid, one thread per cell in a fixed order (no atomics; the sum over the
// partial tiles does not depend on scheduling, though the order of records inside a bin,
// and so the FP32 rounding inside a partial tile, follows the binning's count atomics).
// The read-modify-write traffic of gridding therefore stays in LDS instead of going to
// HBM (the paper's CUDA gridder, Section 2.2, keeps one thread per kernel tap and
// baseline, sums that baseline's consecutive timestamps in a register and writes to the
// grid in global memory with an atomic add when it moves to the next baseline).
//
// Because the tile is private to one wavefront and its 64 lanes always touch 64
// distinct cells of a record's footprint, the accumulation is a plain LDS read, add and
// write: instructions of one wavefront reach LDS in order, so a later record sees the
// earlier record's update without atomics.  (LDS floating-point atomics on this chip
// retire at only a few lanes per clock; plain 64-bit reads and writes run at full
// LDS bandwidth.)  Tiles are small (16 or 32 cells) so that a CU holds many wavefronts,
// each with its own tile, to hide LDS and memory latency.
//
// Launch is persistent: enough wavefronts to fill every CU pull work items from a queue
// head in HBM until the queue is empty, which evens out the very uneven per-tile
// visibility counts of Earth-rotation tracks.  With a fixed support, records are loaded
// 64 at a time and broadcast with readlane, and each lane handles one tap of every record
// per pass of 64 taps.  The table fetches (64 x 8 bytes per record returned to registers,
// mostly from L1) bound a one-record-per-load loop on this chip, so with FP32 arithmetic
// two records share a load: two adjacent taps per lane, one record per half wavefront,
// then a half-wavefront swap.  What is left is mostly vector-ALU issue (the four FMAs,
// the broadcasts and the addressing per record and tap lane).
#include <algorithm>
#include <type_traits>

#include "wproj_tiled.h"

namespace wproj {
namespace {

__device__ inline float2 tab_load(const float2 *t, uint32_t i) { return t[i]; }
__device__ inline double2 tab_load(const double2 *t, uint32_t i) { return t[i]; }
__device__ inline float2 tab_load(const half2c *t, uint32_t i) {
  const half2c h = t[i];
  return make_float2((float)h.re, (float)h.im);
}

// FP64 table fetch through a buffer resource (one record per load): the sub-kernel's
// first tap is wave-uniform and goes in the scalar offset, the lane's tap in the vector
// offset, so the address costs no vector instructions.  The hardware range check covers
// the vector offset only: callers keep the scalar offset inside the table.
__device__ inline double2 tab_fetch(__amdgpu_buffer_rsrc_t r, uint32_t lane, uint32_t tap, const double2 *) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, lane * 16u, tap * 16u, 0);
  const uint32_t w0 = v[0], w1 = v[1], w2 = v[2], w3 = v[3];
  const uint64_t re = (uint64_t)w0 | ((uint64_t)w1 << 32);
  const uint64_t im = (uint64_t)w2 | ((uint64_t)w3 << 32);
  return make_double2(__longlong_as_double((long long)re), __longlong_as_double((long long)im));
}
__device__ inline float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename Real> struct Cx;
template <> struct Cx<float> { using T = float2; };
template <> struct Cx<double> { using T = double2; };

// Records processed per group by one wavefront in the direct-fetch path: their table
// loads are all issued before the first is consumed, so up to kGroup memory latencies
// overlap per wave.
constexpr int kGroup = 8;
// The same for the per-record-support path, whose table misses reach past L2 (cfg3's
// 4096^2 rows: 4.03 ms with 8, 3.94 with 16, 4.72 with 32).
constexpr int kVarGroup = 16;

// One tap of an FP32 or FP16 table loaded through a buffer resource (lane's byte offset
// in the vector offset, the sub-kernel's in the scalar offset), kept raw until use.
template <typename Tab> struct TapRaw;
template <> struct TapRaw<float2> {
  typedef uint32_t T __attribute__((ext_vector_type(2)));
  __device__ static T load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
  }
  __device__ static float2 value(const T &v) { return make_float2(__uint_as_float(v[0]), __uint_as_float(v[1])); }
};
template <> struct TapRaw<half2c> {
  typedef uint32_t T;
  __device__ static T load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
  }
  __device__ static float2 value(const T &v) {
    half2c h;
    __builtin_memcpy(&h, &v, 4);
    return make_float2((float)h.re, (float)h.im);
  }
};
template <> struct TapRaw<double2> {  // the per-record-support fast path is FP32 only
  typedef double2 T;
};
constexpr int kMaxWavesPerBlock = 4;

// A row-carrying record (weight, row) turned into W V from the visibility it names; a
// negative weight marks a Hermitian-folded row, which enters as W conj(V).
template <typename Rec, typename C2>
__device__ inline void to_weighted(Rec &r, const C2 *vis) {
  const C2 v = vis[get_row(r)];
  const auto wgt = r.wr;
  r.wr = fabs(wgt) * v.x;
  r.wi = wgt * v.y;
}

// One record's read-add-write of its 64-cell footprint (lane = tap) in the private tile.
template <typename C2, typename Real, typename Tap>
__device__ inline void accumulate(C2 *acc, int a, Real wr, Real wi, const Tap &t) {
  C2 v = acc[a];
  v.x = fmadd(wr, (Real)t.x, v.x);
  v.x = fmadd(-wi, (Real)t.y, v.x);
  v.y = fmadd(wr, (Real)t.y, v.y);
  v.y = fmadd(wi, (Real)t.x, v.y);
  acc[a] = v;
}

// S = fixed support (0 = per-record support).  PLANNED: the records are row-carrying
// (weight, row) and W V is formed from vis[row] as each record is loaded.  RUNS (paired
// fixed-support path only): while consecutive records of the work item share the
// footprint origin, each lane keeps its cell of the footprint in a register and writes it
// back to the tile only when the origin changes.  The multiply-adds and their order are
// those of the plain read-add-write, so the result is the same bit for bit.
template <typename Real, typename Rec, typename Tab, int S, bool PLANNED, bool RUNS = false>
__global__ void __launch_bounds__(64 * kMaxWavesPerBlock)
    tiled_grid_kernel(Geometry G, BinShape B, int pitch, int rows, int wave_lds,
                      const Tab *__restrict__ tab, uint32_t tab_bytes,
                      const Rec *__restrict__ rec, const WorkItem *__restrict__ items,
                      const uint32_t *__restrict__ order,
                      const uint32_t *__restrict__ n_items_ptr, uint32_t *counter,
                      typename Cx<Real>::T *__restrict__ partial,
                      const typename Cx<Real>::T *__restrict__ vis) {
  using C2 = typename Cx<Real>::T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  C2 *acc = reinterpret_cast<C2 *>(smem_raw) + (size_t)wid * wave_lds;
  const uint32_t n_items = *n_items_ptr;
  const int area = rows * pitch;
  const __amdgpu_buffer_rsrc_t tab_rsrc =
      __builtin_amdgcn_make_buffer_rsrc((void *)tab, (short)0, (int)tab_bytes, kBufferWord3);

  for (;;) {
    uint32_t got = 0;
    if (lane == 0) got = atomicAdd(counter, 1u);
    const uint32_t it = (uint32_t)__builtin_amdgcn_readlane((int)got, 0);
    if (it >= n_items) break;
    const uint32_t item = order[it];  // largest items first
    const WorkItem w = items[item];
    for (int i = lane; i < area; i += 64) acc[i] = C2{Real(0), Real(0)};
    const uint32_t n_rec = w.end - w.begin;
    // Records arrive 64 at a time with one coalesced load (lane i holds record i of the
    // batch; the next batch is loaded while this one is processed) and are broadcast to
    // the wavefront with readlane.
    auto load_batch = [&](uint32_t b, Rec &dst) {
      const uint32_t i = b + (uint32_t)lane;
      if (i < n_rec) {
        dst = rec[w.begin + i];
        if constexpr (PLANNED) to_weighted(dst, vis);
      } else {  // padding records carry zero weight
        dst.lds = 0;
        if constexpr (kHasTap<Rec>) dst.tap = 0;
        dst.wr = Real(0);
        dst.wi = Real(0);
      }
    };

    if constexpr (S > 0 && kPairedTab<Tab>) {
      // Paired direct-fetch path (fixed support, FP32 arithmetic): as below, but the taps
      // of records 2i and 2i+1 arrive with one load.
      using P = TapPair<Tab>;
      using Raw = typename P::Raw;
      constexpr int kPasses = (S * S + 63) / 64;
      constexpr int kGroupS = kPasses == 1 ? kGroup : kPasses == 2 ? kGroup / 2 : kGroup / 4;
      constexpr int kPairs = kGroupS / 2;
      constexpr int kGroups = 64 / kGroupS;
      // The table is the pair-ordered copy: in pass q (n_q taps, h_q = ceil(n_q / 2)),
      // entries 2j and 2j+1 hold taps 64q + j and 64q + h_q + j.  Lanes j and 32 + j load
      // entry pair j of records 2i and 2i+1; after the swap, lane j (< 32) holds tap
      // 64q + j and lane 32 + j tap 64q + h_q + j of both records.  In full passes that
      // is tap 64q + lane, whose 64-bit LDS accesses the row pitch keeps free of bank
      // conflicts (pairs of adjacent taps would put each half wavefront on every second
      // column of eight rows, which no uniform pitch spreads over all banks).
      const int half = lane >> 5;
      const int j = lane & 31;
      // all ones in the upper half of the wavefront; opaque to the compiler, which would
      // otherwise turn the AND below back into a per-pair vector select
      uint32_t upper = half ? 0xffffffffu : 0u;
      asm volatile("" : "+v"(upper));
      int p_off[kPasses];
      bool p_on[kPasses];
      uint32_t p_pair[kPasses];  // byte offset of the lane's entry pair inside a sub-kernel
#pragma unroll
      for (int q = 0; q < kPasses; ++q) {
        const int n_q = S * S - 64 * q < 64 ? S * S - 64 * q : 64;
        const int h_q = (n_q + 1) / 2;
        const int t = 64 * q + (half ? h_q : 0) + j;
        p_on[q] = half ? j < n_q - h_q : j < h_q;
        p_off[q] = p_on[q] ? (t / S) * pitch + t % S : 0;
        p_pair[q] = (j < h_q ? (uint32_t)(64 * q + 2 * j) : 0u) * P::kTapBytes;
        // hides the value's range, so that the offset below stays one three-way add
        asm volatile("" : "+v"(p_pair[q]));
      }
      // Byte offset of the lane's entry pair: first record's sub-kernel plus, in the upper
      // half, the (modulo 2^32) distance to the second record's; the scalar unit forms
      // both, so the select costs one vector AND.
      // The records carry their sub-kernel number above the LDS offset (one broadcast
      // for both); a sub-kernel takes kStride entries of the pair-ordered table.
      constexpr int kLast = S * S - 64 * (kPasses - 1);
      constexpr uint32_t kStride = 64 * (kPasses - 1) + 2 * ((kLast + 1) / 2);
      constexpr uint32_t kSubBytes = kStride * P::kTapBytes;
      auto fetch = [&](const Rec &batch, int j, int q) {
        const uint32_t a = (bcast(batch.lds, j) >> kLdsBits) * kSubBytes;
        const uint32_t d = (bcast(batch.lds, j + 1) >> kLdsBits) * kSubBytes - a;
        return P::load(tab_rsrc, a + (upper & d) + p_pair[q]);
      };
      // RUNS: the lane's cells of the current origin (one per pass) and that origin's LDS
      // offset (wave-uniform; -1 before the first record)
      float2 held[kPasses];
      int held_base = -1;
      auto run_record = [&](int base, Real wr, Real wi, const float2 (&t)[kPasses]) {
        if (base != held_base) {  // a new origin: write the held cells back, load the new ones
#pragma unroll
          for (int q = 0; q < kPasses; ++q)
            if (held_base >= 0 && p_on[q]) acc[held_base + p_off[q]] = held[q];
#pragma unroll
          for (int q = 0; q < kPasses; ++q)
            if (p_on[q]) held[q] = acc[base + p_off[q]];
          held_base = base;
        }
#pragma unroll
        for (int q = 0; q < kPasses; ++q) {
          held[q].x = fmadd(wr, t[q].x, held[q].x);
          held[q].x = fmadd(-wi, t[q].y, held[q].x);
          held[q].y = fmadd(wr, t[q].y, held[q].y);
          held[q].y = fmadd(wi, t[q].x, held[q].y);
        }
      };
      Rec cur;
      load_batch(0, cur);
      for (uint32_t b = 0; b < n_rec; b += 64) {
        Rec nxt;
        const bool more = b + 64 < n_rec;
        if (more) load_batch(b + 64, nxt);
        Raw c[2][kPairs][kPasses];
#pragma unroll
        for (int i = 0; i < kPairs; ++i)
#pragma unroll
          for (int q = 0; q < kPasses; ++q) c[0][i][q] = fetch(cur, 2 * i, q);
#pragma unroll
        for (int gI = 0; gI < kGroups; ++gI) {
          if (gI + 1 < kGroups) {
#pragma unroll
            for (int i = 0; i < kPairs; ++i)
#pragma unroll
              for (int q = 0; q < kPasses; ++q)
                c[(gI + 1) & 1][i][q] = fetch(cur, (gI + 1) * kGroupS + 2 * i, q);
          }
#pragma unroll
          for (int i = 0; i < kPairs; ++i) {
            const int j = gI * kGroupS + 2 * i;
            const int base0 = (int)(bcast(cur.lds, j) & kLdsMask);
            const int base1 = (int)(bcast(cur.lds, j + 1) & kLdsMask);
            const Real wr0 = bcast(cur.wr, j), wi0 = bcast(cur.wi, j);
            const Real wr1 = bcast(cur.wr, j + 1), wi1 = bcast(cur.wi, j + 1);
            if constexpr (RUNS) {
              float2 t0[kPasses], t1[kPasses];
#pragma unroll
              for (int q = 0; q < kPasses; ++q) P::split(c[gI & 1][i][q], t0[q], t1[q]);
              run_record(base0, wr0, wi0, t0);
              run_record(base1, wr1, wi1, t1);
            } else {
              // record by record (all passes of record 2i, then of 2i + 1): a cell that both
              // footprints cover through different passes then takes its two updates in
              // record order, as with RUNS
              float2 t0[kPasses], t1[kPasses];
#pragma unroll
              for (int q = 0; q < kPasses; ++q) P::split(c[gI & 1][i][q], t0[q], t1[q]);
#pragma unroll
              for (int q = 0; q < kPasses; ++q)
                if (p_on[q]) accumulate(acc, base0 + p_off[q], wr0, wi0, t0[q]);
#pragma unroll
              for (int q = 0; q < kPasses; ++q)
                if (p_on[q]) accumulate(acc, base1 + p_off[q], wr1, wi1, t1[q]);
            }
          }
        }
        if (more) cur = nxt;
      }
      if constexpr (RUNS) {
#pragma unroll
        for (int q = 0; q < kPasses; ++q)
          if (held_base >= 0 && p_on[q]) acc[held_base + p_off[q]] = held[q];
      }
    } else if constexpr (S > 0) {
      // Direct-fetch path (fixed support, FP64): lane t handles tap t of every record, in
      // kPasses passes of 64 taps when S^2 > 64.  Table taps are loaded one group of
      // kGroupS records ahead of their use; the group shrinks as the passes grow, so the
      // prefetched taps stay within a fixed register budget.  (Staging the batch in LDS
      // and reading each record back as an LDS broadcast measured slower than readlanes.)
      using Tap = decltype(tab_load(tab, 0u));
      constexpr int kPasses = (S * S + 63) / 64;
      constexpr int kGroupS = kPasses == 1 ? kGroup : kPasses == 2 ? kGroup / 2 : kGroup / 4;
      constexpr int kGroups = 64 / kGroupS;
      int p_off[kPasses];
      bool p_on[kPasses];
      uint32_t p_tap[kPasses];
#pragma unroll
      for (int q = 0; q < kPasses; ++q) {
        const int t = q * 64 + lane;
        p_on[q] = t < S * S;
        p_off[q] = (t / S) * pitch + t % S;
        p_tap[q] = p_on[q] ? (uint32_t)t : 0u;
      }
      Rec cur;
      load_batch(0, cur);
      for (uint32_t b = 0; b < n_rec; b += 64) {
        Rec nxt;
        const bool more = b + 64 < n_rec;
        if (more) load_batch(b + 64, nxt);
        Tap c[2][kGroupS][kPasses];
#pragma unroll
        for (int i = 0; i < kGroupS; ++i) {
          const uint32_t tb = (bcast(cur.lds, i) >> kLdsBits) * (uint32_t)(S * S);
#pragma unroll
          for (int q = 0; q < kPasses; ++q) c[0][i][q] = tab_fetch(tab_rsrc, p_tap[q], tb, tab);
        }
#pragma unroll
        for (int gI = 0; gI < kGroups; ++gI) {
          if (gI + 1 < kGroups) {
#pragma unroll
            for (int i = 0; i < kGroupS; ++i) {
              const uint32_t tb = (bcast(cur.lds, (gI + 1) * kGroupS + i) >> kLdsBits) * (uint32_t)(S * S);
#pragma unroll
              for (int q = 0; q < kPasses; ++q) c[(gI + 1) & 1][i][q] = tab_fetch(tab_rsrc, p_tap[q], tb, tab);
            }
          }
#pragma unroll
          for (int i = 0; i < kGroupS; ++i) {
            const int j = gI * kGroupS + i;
            const int base = (int)(bcast(cur.lds, j) & kLdsMask);
            const Real rwr = bcast(cur.wr, j), rwi = bcast(cur.wi, j);
#pragma unroll
            for (int q = 0; q < kPasses; ++q)
              if (p_on[q]) accumulate(acc, base + p_off[q], rwr, rwi, c[gI & 1][i][q]);
          }
        }
        if (more) cur = nxt;
      }
    } else if constexpr (kHasTap<Rec> && std::is_same_v<Real, float>) {
      // Per-record supports with FP32 arithmetic.  Records arrive 64 at a time (one
      // coalesced load, readlane broadcasts).  A record with S <= 8 takes one pass, lane t
      // tap t; its taps load one group of kVarGroup records ahead, at a wave-uniform scalar
      // offset (the table carries 64 zero taps past its end, so lanes t >= S^2 of its last
      // sub-kernel stay inside it).  The lane's cell offset follows the support and is
      // recomputed only when the support changes (a tile's records come plane by plane).
      // Larger supports take their passes as they go.
      using Raw = typename TapRaw<Tab>::T;
      int s_cur = 0, p_off = 0;
      bool p_on = false;
      auto set_support = [&](int Sn) {
        // t / Sn by a float reciprocal: (t + 1/2) / Sn lies at least 1/(2 Sn) from an
        // integer, far beyond the rounding of this product
        const int kv = (int)(((float)lane + 0.5f) * (1.0f / (float)Sn));
        p_on = lane < Sn * Sn;
        p_off = kv * pitch + (lane - kv * Sn);
        s_cur = Sn;
      };
      const uint32_t vlane = (uint32_t)lane * (uint32_t)sizeof(Tab);
      auto fetch_group = [&](const Rec &batch, int g, Raw (&dst)[kVarGroup]) {
#pragma unroll
        for (int i = 0; i < kVarGroup; ++i) {
          const uint32_t tp = bcast(batch.tap, g * kVarGroup + i);
          if ((tp >> kTapBits) < 8u) dst[i] = TapRaw<Tab>::load(tab_rsrc, vlane, (tp & kTapMask) * (uint32_t)sizeof(Tab));
        }
      };
      auto accumulate_group = [&](const Rec &batch, int g, const Raw (&src)[kVarGroup]) {
        bool large = false;
#pragma unroll
        for (int i = 0; i < kVarGroup; ++i) {
          const int j = g * kVarGroup + i;
          const uint32_t tp = bcast(batch.tap, j);
          const int Sr = (int)(tp >> kTapBits) + 1;
          if (Sr <= 8) {
            if (Sr != s_cur) set_support(Sr);
            const int base = (int)(bcast(batch.lds, j) & kLdsMask);
            const Real rwr = bcast(batch.wr, j), rwi = bcast(batch.wi, j);
            if (p_on) accumulate(acc, base + p_off, rwr, rwi, TapRaw<Tab>::value(src[i]));
          } else {
            large = true;
          }
        }
        // records with S > 8 (several passes), their taps loaded as they go
        if (large) {
#pragma unroll 1
          for (int i = 0; i < kVarGroup; ++i) {
            const int j = g * kVarGroup + i;
            const uint32_t tp = bcast(batch.tap, j);
            const int Sr = (int)(tp >> kTapBits) + 1;
            if (Sr <= 8) continue;
            const uint32_t tb = tp & kTapMask;
            const int base = (int)(bcast(batch.lds, j) & kLdsMask);
            const Real rwr = bcast(batch.wr, j), rwi = bcast(batch.wi, j);
            for (int t = lane; t < Sr * Sr; t += 64) {
              const int kv = t / Sr, ku = t - kv * Sr;
              accumulate(acc, base + kv * pitch + ku, rwr, rwi, tab_load(tab, tb + (uint32_t)t));
            }
          }
        }
      };
      Rec cur;
      load_batch(0, cur);
      for (uint32_t b = 0; b < n_rec; b += 64) {
        Rec nxt;
        const bool more = b + 64 < n_rec;
        if (more) load_batch(b + 64, nxt);
        Raw c0[kVarGroup], c1[kVarGroup];
        fetch_group(cur, 0, c0);
        for (int g = 0; g < 64 / kVarGroup; g += 2) {
          fetch_group(cur, g + 1, c1);
          accumulate_group(cur, g, c0);
          if (g + 2 < 64 / kVarGroup) fetch_group(cur, g + 2, c0);
          accumulate_group(cur, g + 1, c1);
        }
        if (more) cur = nxt;
      }
    } else if constexpr (kHasTap<Rec>) {
      // General path (FP64; per-record support up to 32): records by wave-uniform loads,
      // each record's taps in passes of 64 lanes.
      for (uint32_t r = w.begin; r < w.end; ++r) {
        Rec rr = rec[r];
        if constexpr (PLANNED) to_weighted(rr, vis);
        const uint32_t tp = rr.tap;
        const int Sr = S > 0 ? S : (int)(tp >> kTapBits) + 1;
        const uint32_t tb = tp & kTapMask;
        const int base = (int)(rr.lds & kLdsMask);
        for (int t = lane; t < Sr * Sr; t += 64) {
          const int kv = t / Sr, ku = t - kv * Sr;
          accumulate(acc, base + kv * pitch + ku, rr.wr, rr.wi, tab_load(tab, tb + t));
        }
      }
    }

    // flush: the work item's tile (with halo) goes to its own slot of the partial-tile
    // buffer with plain coalesced stores; tile_reduce_kernel adds the slots to the grid
    C2 *dst = partial + (size_t)item * rows * rows;
    for (int i = lane; i < rows * rows; i += 64) {
      const int ry = i / rows, rx = i - ry * rows;
      dst[i] = acc[ry * pitch + rx];
    }
  }
}

// Adds the partial tiles to the grid.  One thread per grid cell (each thread takes two
// cells of a column) sums, in FP64, every work item's partial value for that cell: the items of the cell's own tile and those of
// the tiles to its left/above whose halo reaches it (items of tile t are contiguous in
// the work list: [choff[t], choff[t + 1])).  Each cell has exactly one writer, so the
// grid update needs no atomics and the result does not depend on scheduling.
template <typename Real>
__global__ void __launch_bounds__(256)
    tile_reduce_kernel(Geometry G, BinShape B, int rows, const typename Cx<Real>::T *__restrict__ partial,
                       const uint32_t *__restrict__ choff, Real *grid) {
  using C2 = typename Cx<Real>::T;
  // blockIdx.x * 256 + threadIdx.x is the column; a thread takes rows 2 blockIdx.y and
  // 2 blockIdx.y + 1 (one tile row, since tiles have an even side), whose work items and
  // their offsets it looks up once; blockIdx.z steps through the grids
  const int X = (int)(blockIdx.x * 256 + threadIdx.x), Y = 2 * (int)blockIdx.y;
  if (X >= G.n) return;
  const int64_t cells = (int64_t)G.n * G.n;
  const int T = B.tile;
  const int tx = X >> B.log2_tile, ty = Y >> B.log2_tile, lx = X & (T - 1), ly = Y & (T - 1);
  for (int img = (int)blockIdx.z; img < G.n_grids; img += (int)gridDim.z) {
    double sr0 = 0.0, si0 = 0.0, sr1 = 0.0, si1 = 0.0;
    for (int dy = 0; dy <= ty && ly + dy * T < rows; ++dy) {
      const bool second = ly + 1 + dy * T < rows;  // row Y + 1 is inside this tile's copy too
      for (int dx = 0; dx <= tx && lx + dx * T < rows; ++dx) {
        const int64_t tile = ((int64_t)img * B.nty + (ty - dy)) * B.ntx + (tx - dx);
        const int off = (ly + dy * T) * rows + (lx + dx * T);
        const uint32_t i1 = choff[tile + 1];
        for (uint32_t i = choff[tile]; i < i1; ++i) {
          const C2 *p = partial + (size_t)i * rows * rows + off;
          const C2 v0 = p[0];
          sr0 += (double)v0.x;
          si0 += (double)v0.y;
          if (second) {
            const C2 v1 = p[rows];
            sr1 += (double)v1.x;
            si1 += (double)v1.y;
          }
        }
      }
    }
    C2 *g = reinterpret_cast<C2 *>(grid) + (cells * img + (int64_t)Y * G.n + X);
    if (sr0 != 0.0 || si0 != 0.0) {
      C2 v = g[0];
      v.x = (Real)((double)v.x + sr0);
      v.y = (Real)((double)v.y + si0);
      g[0] = v;
    }
    if (sr1 != 0.0 || si1 != 0.0) {
      C2 v = g[G.n];
      v.x = (Real)((double)v.x + sr1);
      v.y = (Real)((double)v.y + si1);
      g[G.n] = v;
    }
  }
}

template <typename Real, typename Rec, typename Tab, int S, bool PLANNED, bool RUNS = false>
hipError_t launch_one(const wproj_kernels *k, const BinShape &B, const TileShape &ts,
                      const BinWorkspace &W, void *grid, const void *vis, hipStream_t s) {
  auto kern = tiled_grid_kernel<Real, Rec, Tab, S, PLANNED, RUNS>;
  // as many wavefronts per workgroup (up to 4) as their private tiles fit in LDS
  const int wpb = (int)std::max<size_t>(1, std::min<size_t>(kMaxWavesPerBlock, k->max_lds / ts.lds_bytes));
  const size_t lds = ts.lds_bytes * wpb;
  hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * wpb, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  const unsigned blocks = (unsigned)(k->n_cu * per_cu);
  const int wave_lds = (int)(ts.lds_bytes / (2 * sizeof(Real)));
  // the paired fixed-support kernels read the pair-ordered table
  const bool paired = S > 0 && kPairedTab<Tab>;
  if (paired && (!k->d_tab_pair || k->pair_stride != pair_table_stride(S))) return hipErrorInvalidValue;
  const int64_t n_sub = (int64_t)k->params.n_wplanes * k->params.oversample * k->params.oversample;
  const Tab *tab = (const Tab *)(paired ? k->d_tab_pair : k->d_tab);
  const int64_t tab_entries = paired ? n_sub * k->pair_stride : k->n_taps;
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * wpb), lds, s, k->geo, B, ts.pitch,
                     ts.rows, wave_lds, tab, (uint32_t)(tab_entries * sizeof(Tab)),
                     (const Rec *)W.rec, W.items, W.order, W.choff + B.n_tiles, W.counter,
                     (typename Cx<Real>::T *)W.partial, (const typename Cx<Real>::T *)vis);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_reduce(const wproj_kernels *k, const BinShape &B, const TileShape &ts,
                         const BinWorkspace &W, void *grid, hipStream_t s) {
  const dim3 grid3((unsigned)((k->params.n + 255) / 256), (unsigned)(k->params.n / 2),
                   (unsigned)std::min<int64_t>(k->geo.n_grids, 65535));
  hipLaunchKernelGGL(tile_reduce_kernel<Real>, grid3, dim3(256), 0,
                     s, k->geo, B, ts.rows, (const typename Cx<Real>::T *)W.partial, W.choff,
                     (Real *)grid);
  return hipGetLastError();
}

template <typename Real, typename Rec, typename Tab, bool PLANNED, int S>
hipError_t dispatch_fixed(const wproj_kernels *k, const BinShape &B, const TileShape &ts,
                          const BinWorkspace &W, void *grid, const void *vis, hipStream_t s) {
  if constexpr (S > kMaxFixedSupport) {
    if constexpr (!kHasTap<Rec>) return hipErrorInvalidValue;  // packed records need a fixed support
    else return launch_one<Real, Rec, Tab, 0, PLANNED>(k, B, ts, W, grid, vis, s);
  } else {
    if (k->s_max == S) {
      if constexpr (kPairedTab<Tab>)
        if (k->params.accumulate_runs)
          return launch_one<Real, Rec, Tab, S, PLANNED, true>(k, B, ts, W, grid, vis, s);
      return launch_one<Real, Rec, Tab, S, PLANNED>(k, B, ts, W, grid, vis, s);
    }
    return dispatch_fixed<Real, Rec, Tab, PLANNED, S + 1>(k, B, ts, W, grid, vis, s);
  }
}

template <typename Real, typename Rec, typename Tab, bool PLANNED>
hipError_t dispatch_support(const wproj_kernels *k, const BinShape &B, const TileShape &ts,
                            const BinWorkspace &W, void *grid, const void *vis, hipStream_t s) {
  // a fixed support from kMinFixedSupport to kMaxFixedSupport has its own kernel, which
  // takes the sub-kernel from the packed LDS field (pack_sub is set exactly then);
  // per-plane supports take the general path
  if (B.pack_sub)
    return dispatch_fixed<Real, Rec, Tab, PLANNED, kMinFixedSupport>(k, B, ts, W, grid, vis, s);
  return launch_one<Real, Rec, Tab, 0, PLANNED>(k, B, ts, W, grid, vis, s);
}

template <typename Real, typename Rec, typename Tab>
hipError_t dispatch_planned(const wproj_kernels *k, const BinShape &B, const TileShape &ts,
                            const BinWorkspace &W, void *grid, const void *vis, hipStream_t s) {
  if (vis) return dispatch_support<Real, Rec, Tab, true>(k, B, ts, W, grid, vis, s);
  // FP32 W V records of a fixed support are the 12-byte packed form
  if constexpr (std::is_same_v<Rec, RecordF32>)
    if (B.pack_sub)
      return dispatch_fixed<Real, RecordF32P, Tab, false, kMinFixedSupport>(k, B, ts, W, grid, vis, s);
  return dispatch_support<Real, Rec, Tab, false>(k, B, ts, W, grid, vis, s);
}

// Fills the pair-ordered table: one thread per entry.  In pass q of a sub-kernel (n_q
// taps, h = ceil(n_q / 2)), entry 2j is tap 64q + j and entry 2j+1 tap 64q + h + j, or
// zero where n_q is odd and that tap does not exist.
template <typename Tab>
__global__ void __launch_bounds__(256)
    pair_table_kernel(const Tab *__restrict__ src, int64_t n_sub, int s2, int stride, Tab *__restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_sub * stride) return;
  const int64_t sub = i / stride;
  const int e = (int)(i - sub * stride);
  const int q = e / 64, r = e - 64 * q;
  const int n_q = s2 - 64 * q < 64 ? s2 - 64 * q : 64;
  const int h = (n_q + 1) / 2;
  const int jj = r >> 1;
  const bool second = r & 1;
  const int t = 64 * q + (second ? h : 0) + jj;
  Tab v{};
  if (second ? jj < n_q - h : jj < h) v = src[sub * s2 + t];
  dst[i] = v;
}

}  // namespace

int64_t pair_table_stride(int S) {
  const int passes = (S * S + 63) / 64;
  const int last = S * S - 64 * (passes - 1);
  return 64 * (passes - 1) + 2 * ((last + 1) / 2);
}

hipError_t launch_pair_table(const wproj_kernels *k, hipStream_t s) {
  const int S = k->s_max;
  const int64_t n_sub = (int64_t)k->params.n_wplanes * k->params.oversample * k->params.oversample;
  const int64_t total = n_sub * k->pair_stride;
  const unsigned blocks = (unsigned)((total + 255) / 256);
  if (k->params.precision == WPROJ_F32)
    hipLaunchKernelGGL(pair_table_kernel<float2>, dim3(blocks), dim3(256), 0, s, (const float2 *)k->d_tab,
                       n_sub, S * S, (int)k->pair_stride, (float2 *)k->d_tab_pair);
  else
    hipLaunchKernelGGL(pair_table_kernel<half2c>, dim3(blocks), dim3(256), 0, s, (const half2c *)k->d_tab,
                       n_sub, S * S, (int)k->pair_stride, (half2c *)k->d_tab_pair);
  return hipGetLastError();
}

TileShape tile_shape(const wproj_kernels *k, int tile) {
  // One wavefront's private tile: rows = T + S_max - 1 complex cells per side.  The row
  // pitch (in complex cells) is odd-multiple-of-8 so that the 4 rows of 8 taps a half
  // wavefront touches fall on different LDS banks for 64-bit accesses.
  TileShape t;
  t.tile = tile;
  t.rows = tile + k->s_max - 1;
  int pitch = t.rows;
  while ((pitch & 15) != 8) ++pitch;
  t.pitch = pitch;
  const size_t real = k->params.precision == WPROJ_F64 ? 8 : 4;
  t.lds_bytes = 2 * (size_t)t.rows * t.pitch * real;  // per wavefront
  return t;
}

int degrid_pitch(const wproj_kernels *k, int tile) { return (tile + k->s_max - 1) | 1; }

hipError_t launch_tiled_grid(const wproj_kernels *k, const BinShape &B, const BinWorkspace &W,
                             void *grid, hipStream_t s, const void *vis) {
  const TileShape ts = tile_shape(k, B.tile);
  hipError_t e = launch_fill_u32(W.counter, 1, 0u, s);
  if (e != hipSuccess) return e;
  switch (k->params.precision) {
    case WPROJ_F64:
      return dispatch_planned<double, RecordF64, double2>(k, B, ts, W, grid, vis, s);
    case WPROJ_F32:
      return dispatch_planned<float, RecordF32, float2>(k, B, ts, W, grid, vis, s);
    default:
      return dispatch_planned<float, RecordF32, half2c>(k, B, ts, W, grid, vis, s);
  }
}

hipError_t launch_tile_reduce(const wproj_kernels *k, const BinShape &B, const BinWorkspace &W,
                              void *grid, hipStream_t s) {
  const TileShape ts = tile_shape(k, B.tile);
  if (k->params.precision == WPROJ_F64) return launch_reduce<double>(k, B, ts, W, grid, s);
  return launch_reduce<float>(k, B, ts, W, grid, s);
}

}  // namespace wproj
