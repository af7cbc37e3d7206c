// Shapes and buffers of the binned (tiled) gridding path.
#pragma once

#include <type_traits>

#include "wproj_internal.h"

namespace wproj {

// Bits of Record::tap holding the first tap of the visibility's sub-kernel; the top
// bits hold S_p - 1.
constexpr int kTapBits = 26;
constexpr uint32_t kTapMask = (1u << kTapBits) - 1u;

// Bits of Record::lds holding the LDS offset; a tile copy has at most (64 + 31) x 104 =
// 9880 cells.  When BinShape::pack_sub is set, the bits above hold the sub-kernel number
// p O^2 + ov O + ou, so that with a uniform support S the first tap is that number times
// S^2 and the fixed-support gridders read one field instead of two.
constexpr int kLdsBits = 14;
constexpr uint32_t kLdsMask = (1u << kLdsBits) - 1u;
// Fixed supports with gridder kernels of their own.
constexpr int kMinFixedSupport = 3;
constexpr int kMaxFixedSupport = 16;

// Size classes of the largest-first work order (class c: items of more than
// (15 - c) / 16 of a chunk, down to the smallest).
constexpr int kOrderBuckets = 16;

// Partial accumulators per image (weight sums) and per counter, spread by block index.
constexpr int kSlots = 256;

// One binned visibility: the LDS offset of its first cell inside its tile's private
// copy ((y0 - tile y0) pitch + (x0 - tile x0), optionally with the sub-kernel number
// above it), its sub-kernel (first tap | (S-1) << 26) and W V at the path's precision.
struct RecordF32 {
  uint32_t lds;
  uint32_t tap;
  float wr, wi;
};
struct RecordF64 {
  uint32_t lds;
  uint32_t tap;
  double wr, wi;
};
// The FP32 W V record of a fixed support whose sub-kernel number rides in `lds` (packed
// records): the first tap is that number times S^2, so no tap word is stored (12 bytes).
struct RecordF32P {
  uint32_t lds;
  float wr, wi;
};
template <typename Rec> constexpr bool kHasTap = !std::is_same_v<Rec, RecordF32P>;

// Row-carrying records (degridding and planned gridding) hold the visibility's weight in
// `wr` and its row in the low 32 bits of `wi` instead of W V.
__host__ __device__ inline void set_plan(RecordF32 &r, float w, uint32_t j) {
  r.wr = w;
  __builtin_memcpy(&r.wi, &j, 4);
}
__host__ __device__ inline void set_plan(RecordF64 &r, double w, uint32_t j) {
  r.wr = w;
  r.wi = 0.0;
  __builtin_memcpy(&r.wi, &j, 4);
}
__host__ __device__ inline uint32_t get_row(const RecordF32 &r) {
  uint32_t j;
  __builtin_memcpy(&j, &r.wi, 4);
  return j;
}
__host__ __device__ inline uint32_t get_row(const RecordF64 &r) {
  uint32_t j;
  __builtin_memcpy(&j, &r.wi, 4);
  return j;
}

// gfx9 buffer descriptor word 3: 32-bit data format, no swizzle
constexpr int kBufferWord3 = 0x00020000;

// Paired tap fetch (FP32 arithmetic): one load brings two table entries per lane, lanes
// 0-31 for the first record of a pair and lanes 32-63 for the second, so a pair of
// records costs one wide load instead of two narrow ones.  A swap of the upper half of
// the first entries with the lower half of the second entries (v_permlane32_swap, a
// VALU operation) then leaves every lane with the same tap of both records.
template <typename Tab> struct TapPair;
template <> struct TapPair<float2> {
  typedef uint32_t Raw __attribute__((ext_vector_type(4)));
  static constexpr uint32_t kTapBytes = 8;
  __device__ static Raw load(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
    return __builtin_amdgcn_raw_buffer_load_b128(r, byte_off, 0, 0);
  }
  __device__ static void split(const Raw &v, float2 &first, float2 &second) {
    const uint32_t a_re = v[0], a_im = v[1], b_re = v[2], b_im = v[3];
    const auto re = __builtin_amdgcn_permlane32_swap(a_re, b_re, false, false);
    const auto im = __builtin_amdgcn_permlane32_swap(a_im, b_im, false, false);
    const uint32_t f_re = re[0], s_re = re[1], f_im = im[0], s_im = im[1];
    first = make_float2(__uint_as_float(f_re), __uint_as_float(f_im));
    second = make_float2(__uint_as_float(s_re), __uint_as_float(s_im));
  }
};
template <> struct TapPair<half2c> {
  typedef uint32_t Raw __attribute__((ext_vector_type(2)));
  static constexpr uint32_t kTapBytes = 4;
  __device__ static Raw load(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
    return __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0);
  }
  __device__ static void split(const Raw &v, float2 &first, float2 &second) {
    const uint32_t a = v[0], b = v[1];
    const auto x = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    const uint32_t f = x[0], s = x[1];
    half2c hf, hs;
    __builtin_memcpy(&hf, &f, 4);
    __builtin_memcpy(&hs, &s, 4);
    first = make_float2((float)hf.re, (float)hf.im);
    second = make_float2((float)hs.re, (float)hs.im);
  }
};
template <typename Tab> constexpr bool kPairedTab = std::is_same_v<Tab, float2> || std::is_same_v<Tab, half2c>;

// Wave-uniform broadcast of lane j's value (v_readlane).
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

// Binning geometry: tiles of `tile` cells, ntx x nty per image, kw keys per tile
// (n_wplanes when the plane is part of the key, else 1).
struct BinShape {
  int tile;
  int log2_tile;     // tile = 1 << log2_tile
  int pitch;         // LDS row pitch (complex cells) of a tile's private copy
  int ntx, nty;
  int kw;
  int chunk;         // max records per work item
  int pack_sub;      // records carry the sub-kernel number in Record::lds (fixed support)
  int aggregate;     // the key pass aggregates counts per block in LDS (wproj_params::bin_aggregate)
  int stable;        // records keep input order inside a bin (wproj_params::stable_bins)
  int64_t n_tiles;   // n_images * ntx * nty
  int64_t n_keys;    // n_tiles * kw
};

struct WorkItem {
  uint32_t tile;   // img * (ntx * nty) + ty * ntx + tx
  uint32_t begin;  // record range
  uint32_t end;
};

// Workspace carve-up for one call (all device pointers).
struct BinWorkspace {
  uint32_t *slots;     // [3 nvis] (slot, key, record word) when pack_sub, else [4 nvis] (and tap word)
  void *rec;           // [nvis] RecordF32 / RecordF32P / RecordF64
  uint32_t *count;     // [n_keys]
  uint32_t *offset;    // [n_keys + 1]
  uint32_t *nch;       // [n_tiles]
  uint32_t *choff;     // [n_tiles + 1]; choff[n_tiles] = number of work items
  WorkItem *items;     // [max_items]
  uint32_t *scan_tmp;  // scan_temp_words(max(n_keys, n_tiles))
  uint32_t *counter;   // [1] work-queue head
  uint32_t *order;     // [max_items] work-item indices, largest items first
  uint32_t *order_cnt; // [2 * kOrderBuckets] per size class: item count, placement cursor
  int64_t max_items;   // capacity of items, order and partial
  void *partial;       // [max_items][rows][rows] complex: each work item's accumulated tile
  double *wslots;      // [n_images][kSlots] partial weight sums
  unsigned long long *cslots;  // [3][kSlots] partial counters
  // stable binning only (null otherwise): radix-sort buffers
  uint32_t *sort_keys[2];  // [nvis] each: bin keys, ping-pong
  uint32_t *sort_vals[2];  // [nvis] each: visibility indices, ping-pong
  uint32_t *digit_count;   // [radix_digit_slots(nvis)] per-block digit counts, digit-major
  uint32_t *digit_off;     // [radix_digit_slots(nvis) + 1] their exclusive scan
};

// Entries of the per-block digit count array of the stable binning's radix sort.
int64_t radix_digit_slots(int64_t nvis);

int64_t scan_temp_words(int64_t n);
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
hipError_t launch_exclusive_scan(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp,
                                 hipStream_t s);
// Bins visibilities for gridding (records carry W V) or, with vis == nullptr, into
// row-carrying records (weight and row: degridding, with wt == nullptr and weights taken
// as 1, and planned gridding).
hipError_t launch_bin(const wproj_kernels *k, const BinShape &B, int64_t nvis, const double *uvw,
                      const void *vis, const void *wt, const int64_t *img_off, double *wsum,
                      int64_t *counters, const BinWorkspace &W, hipStream_t s);

// rows[i] = row of binned record i (row-carrying records), 0xffffffff past the last.
hipError_t launch_plan_rows(const wproj_kernels *k, const BinShape &B, const BinWorkspace &W, int64_t nvis,
                            uint32_t *rows, hipStream_t s);

// LDS tile geometry of the tiled gridder for a handle.
struct TileShape {
  int tile;   // T
  int rows;   // T + S_max - 1
  int pitch;  // >= rows, padded for conflict-free rows of taps
  size_t lds_bytes;
};
TileShape tile_shape(const wproj_kernels *k, int tile);
// Row pitch (complex cells) of the degridder's tile copy when records are binned for
// degridding only: the smallest odd pitch >= T + S_max - 1.
int degrid_pitch(const wproj_kernels *k, int tile);
// Entries per sub-kernel of the pair-ordered table for support S, and the launch that
// fills k->d_tab_pair from k->d_tab.
int64_t pair_table_stride(int S);
hipError_t launch_pair_table(const wproj_kernels *k, hipStream_t s);
// The tile gridder into the work items' partial tiles, then their sum into the grid.
// With vis != nullptr the records are row-carrying (a plan) and W V is formed from vis.
hipError_t launch_tiled_grid(const wproj_kernels *k, const BinShape &B, const BinWorkspace &W,
                             void *grid, hipStream_t s, const void *vis = nullptr);
hipError_t launch_tile_reduce(const wproj_kernels *k, const BinShape &B, const BinWorkspace &W,
                              void *grid, hipStream_t s);
// Whether launch_tiled_degrid takes the one-tap-per-lane degridder (FP32 arithmetic and
// tables, packed records of a fixed support up to 8, the pair-ordered table); its
// records are binned with the gridder's row pitch.
bool tap_lane_degrid(const wproj_kernels *k, const BinShape &B);
hipError_t launch_tiled_degrid(const wproj_kernels *k, const BinShape &B, const BinWorkspace &W,
                               const void *model_grid, void *vis_out, int64_t nvis, hipStream_t s);

// Rows regrouped by baseline (Eqs. 5 and 6): a stable counting sort over blocks of
// rows_per_block rows, n_keys = n_ant (n_ant + 1) / 2 baseline numbers + 1 for rows with
// an invalid antenna ID.
struct RegroupShape {
  uint32_t n_keys;
  int64_t rows_per_block;
  int64_t n_blocks;
  int64_t n_counts;  // n_keys * n_blocks
};
RegroupShape regroup_shape(int64_t n_rows, int32_t n_ant);
int64_t regroup_workspace_bytes(const RegroupShape &r);
hipError_t launch_regroup(const RegroupShape &r, int64_t n_rows, const int32_t *ant1,
                          const int32_t *ant2, int32_t n_ant, int64_t *perm, int64_t *start,
                          int64_t *counts, void *workspace, hipStream_t s);
hipError_t launch_channel_order(int64_t n_keys, int32_t n_chan, const int64_t *perm,
                                const int64_t *start, const int64_t *counts, int64_t *vis_perm,
                                hipStream_t s);
hipError_t launch_gather_rows(int64_t n_rows, int64_t row_bytes, const int64_t *perm,
                              int64_t n_src_rows, const void *src, void *dst, int64_t *bad,
                              hipStream_t s);

}  // namespace wproj
