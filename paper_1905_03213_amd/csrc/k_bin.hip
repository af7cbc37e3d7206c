// Device binning of visibilities by (image, uv-tile, w-plane): a counting sort.
//
// The paper's GPU path regroups rows before gridding: a key per row (its baseline
// index, Eq. 5), a count array C per key, an exclusive prefix sum of C giving each
// key's first position (Eq. 6), then a reorder.  The same counting-sort pattern is
// used here, re-keyed so that each group is a uv-tile of the grid (and, within it,
// one w-plane) that a workgroup can accumulate in LDS:
//   key pass     classify each visibility, key = ((img * nty + ty) * ntx + tx) * kw + p,
//                count[key] += 1 returning the visibility's slot within its key;
//                also sumW per image and the drop/clamp/bad-weight counters;
//   scan         exclusive prefix sum of count (Eq. 6);
//   scatter      record of visibility j goes to offset[key] + slot;
//   work list    each tile's record range split into chunks of at most `chunk` records.
// Count atomics are aggregated over runs of a wavefront's lanes that share a key, so a
// record's place inside its bin follows the order in which the runs' atomics land (the
// bin's contents are fixed, their order is not).  Stable bins (BinShape::stable) replace
// the scatter by a stable radix sort of the keys and a gather in sorted order, so that a
// bin keeps its visibilities in input order.  The key pass also stores each
// visibility's key and its record's first word (the LDS offset, with the sub-kernel
// number above it for a fixed support) next to its slot, and with per-plane supports the
// record's tap word too, so the scatter reads 12 or 16 bytes instead of the 24-byte uvw
// and never computes a footprint again.
#include <algorithm>
#include <type_traits>

#include "wproj_tiled.h"

namespace wproj {
namespace {

constexpr uint32_t kInvalid = 0xffffffffu;
constexpr uint32_t kFoldBit = 0x80000000u;

// Visibilities per thread of the key pass.  A key-pass thread issues the loads of all its
// visibilities first and then all its count atomics before it waits on any, so a wave
// keeps more loads and atomics in flight than with one visibility per thread.  Two
// measured fastest: with four the key pass is no faster and the scatter after it is
// slower (the order in which slots are handed out changes how its scattered writes
// combine).  The scatter takes two per thread after the per-wavefront-run key pass with
// packed records of a fixed support (cfg2 binning 1.20 ms against 1.24 with one and 1.28
// with four), one otherwise (two measured slower: +0.06 ms after cfg4's aggregated key
// pass, +0.01 ms on cfg3's per-plane supports).
constexpr int kBinBlock = 256;
constexpr int kKeyVpt = 2;

// Runs of consecutive lanes with equal keys (rows of one baseline's channels are adjacent
// and share tiles and planes, so a wavefront holds a few long runs).  The first lane of
// a run adds the run's length to its key's count with one atomic, and each lane's slot
// is the returned base plus its distance from the run's first lane.  Equal keys in
// separate runs take separate atomics, which leaves the counts and the uniqueness of
// slots intact.  Lanes with key == kInvalid take no part.
struct Run {
  int leader;    // first lane of this lane's run
  uint32_t len;  // run length (meaningful in the first lane)
  bool lead;     // this lane adds the run to its key's count
};

__device__ inline Run run_of(uint32_t key) {
  const int lane = threadIdx.x & 63;
  const uint32_t prev = __shfl_up(key, 1, 64);
  const bool start = lane == 0 || key != prev;
  const uint64_t starts = __ballot(start);
  const uint64_t upto = (2ull << lane) - 1ull;  // lanes 0..lane (all 64 bits for lane 63)
  const uint64_t after = starts & ~upto;
  const int next = after ? __ffsll((unsigned long long)after) - 1 : 64;
  Run r;
  r.leader = 63 - __clzll((long long)(starts & upto));
  r.len = (uint32_t)(next - lane);
  r.lead = start && key != kInvalid;
  return r;
}

// Bin key of a gridded visibility of image img (of its grid: the image, or the image's
// w-stacking layer).
__device__ inline uint32_t bin_key(const Geometry &G, const BinShape &B, int img, const Footprint &f) {
  const uint32_t tx = (uint32_t)f.x0 >> B.log2_tile, ty = (uint32_t)f.y0 >> B.log2_tile;
  const uint32_t g = (uint32_t)grid_of(G, img, f);
  const uint32_t tile = (g * (uint32_t)B.nty + ty) * (uint32_t)B.ntx + tx;
  return B.kw > 1 ? tile * (uint32_t)B.kw + (uint32_t)f.p : tile;
}

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// The record's first word: LDS offset of the footprint's first cell in its tile's
// private copy, with the sub-kernel number above it when the records are packed.
__device__ inline uint32_t record_lds(const Geometry &G, const BinShape &B, const Footprint &f) {
  const int lx = f.x0 & (B.tile - 1), ly = f.y0 & (B.tile - 1);
  uint32_t r = (uint32_t)(ly * B.pitch + lx);
  if (B.pack_sub) r |= (uint32_t)((f.p * G.O + f.ov) * G.O + f.ou) << kLdsBits;
  return r;
}

// A record's tap word: its sub-kernel's first tap, with S - 1 above it.
__device__ inline uint32_t tap_word(const Geometry &G, const Footprint &f) {
  const int S = G.supp[f.p];
  return (uint32_t)(G.tab_off[f.p] + (uint32_t)((f.ov * G.O + f.ou) * S * S)) | ((uint32_t)(S - 1) << kTapBits);
}

// Image of every row of the block when one image holds them all (images are contiguous
// row ranges), else -1; first receives the image of the block's first row (-1 when it
// is in none).  The arguments are the same in every lane.
template <int VPT>
__device__ inline int block_image(const int64_t *off, int n_images, int64_t nvis, int &first) {
  const int64_t j_first = (int64_t)blockIdx.x * (kBinBlock * VPT);
  if (j_first >= nvis) {
    first = -1;
    return -1;
  }
  first = image_of(off, n_images, j_first);
  const int last = image_of(off, n_images, min(j_first + (int64_t)(kBinBlock * VPT), nvis) - 1);
  return first >= 0 && first == last ? first : -1;
}

// Visibility j of thread t of block b in pass i: b 256 VPT + 256 i + t, so each pass of
// a wavefront covers 64 consecutive visibilities.
template <int VPT>
__device__ inline int64_t bin_row(int i) {
  return (int64_t)blockIdx.x * (kBinBlock * VPT) + i * kBinBlock + threadIdx.x;
}

// slots holds arrays of nvis words: slot, key (kInvalid when the visibility is not
// gridded; a Hermitian-folded visibility has the key's top bit set, keys stay below
// 2^31), the record's first word and, with TAPWORD (per-plane supports, records that
// carry their first tap), the record's tap word.  A fixed support S_fix packs the
// sub-kernel number into the first word instead.
template <typename Real, bool TAPWORD>
__global__ void __launch_bounds__(kBinBlock)
    key_kernel(Geometry G, BinShape B, int64_t nvis, const double *__restrict__ uvw,
               const Real *__restrict__ wt, const int64_t *__restrict__ img_off,
               int S_fix, uint32_t *__restrict__ slots, uint32_t *count, double *wsum,
               unsigned long long *counters) {
  constexpr int V = kKeyVpt;
  // every load of the thread first
  double c[V][3];
  Real wj[V];
#pragma unroll
  for (int i = 0; i < V; ++i) {
    const int64_t j = bin_row<V>(i);
    c[i][0] = c[i][1] = c[i][2] = 0.0;
    wj[i] = Real(0);
    if (j < nvis) {
      c[i][0] = uvw[3 * j];
      c[i][1] = uvw[3 * j + 1];
      c[i][2] = uvw[3 * j + 2];
      wj[i] = wt ? wt[j] : Real(1);
    }
  }
  int img_b;  // image of the block's first row
  const int img_all = block_image<V>(img_off, G.n_images, nvis, img_b);
  // then every footprint (kernel-table lookups included) ...
  uint32_t key[V], packed[V], tapw[V];
  bool fold[V];
  double w_mine = 0.0;
  unsigned n_drop = 0, n_clamp = 0, n_bad = 0;
#pragma unroll
  for (int i = 0; i < V; ++i) {
    const int64_t j = bin_row<V>(i);
    key[i] = kInvalid;
    packed[i] = 0;
    tapw[i] = 0;
    fold[i] = false;
    int cls = kFlagged;
    bool clamped = false;
    if (j < nvis) {
      const int img = img_all >= 0 ? img_all : image_of(img_off, G.n_images, j);
      if (img >= 0) {
        Footprint f;
        cls = classify(G, c[i], wj[i], f, TAPWORD ? 0 : S_fix);
        if (cls == kGridded) {
          key[i] = bin_key(G, B, img, f);
          fold[i] = f.fold;
          packed[i] = record_lds(G, B, f);
          if constexpr (TAPWORD) tapw[i] = tap_word(G, f);
          clamped = w_clamped(G, c[i][2]);
          // rows of an image other than the block's first row's image (only in blocks
          // that straddle an image boundary) add their weights to their image's slot
          if (img == img_b)
            w_mine += (double)wj[i];
          else if (wsum)
            unsafeAtomicAdd(&wsum[(int64_t)img * kSlots + (blockIdx.x & (kSlots - 1))], (double)wj[i]);
        }
      }
    }
    n_drop += (unsigned)__popcll(__ballot(cls == kDropped));
    n_bad += (unsigned)__popcll(__ballot(cls == kBadWeight));
    n_clamp += (unsigned)__popcll(__ballot(clamped));
  }
  // ... then every count atomic, and only then the slots
  Run run[V];
  uint32_t got[V];
#pragma unroll
  for (int i = 0; i < V; ++i) {
    run[i] = run_of(key[i]);
    uint32_t g = 0;
    if (run[i].lead) g = atomicAdd(&count[key[i]], run[i].len);
    got[i] = g;
  }
#pragma unroll
  for (int i = 0; i < V; ++i) {
    const int64_t j = bin_row<V>(i);
    const uint32_t slot = __shfl(got[i], run[i].leader, 64) + (uint32_t)((threadIdx.x & 63) - run[i].leader);
    if (j < nvis) {
      slots[j] = slot;
      slots[nvis + j] = fold[i] ? (key[i] | kFoldBit) : key[i];
      slots[2 * nvis + j] = packed[i];
      if constexpr (TAPWORD) slots[3 * nvis + j] = tapw[i];
    }
  }
  // Counters and weight sums: reduced over the workgroup in LDS, then one atomic per
  // workgroup into one of kSlots partial accumulators (chosen by block index) so that
  // no address is hit by many workgroups; finalize_kernel adds the slots up.
  __shared__ double s_w[kBinBlock / 64];
  __shared__ unsigned s_c[3][kBinBlock / 64];
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int acc_slot = blockIdx.x & (kSlots - 1);
  const double wv = wave_sum(w_mine);
  if (lane == 0) {
    s_w[wid] = wv;
    s_c[0][wid] = n_drop;
    s_c[1][wid] = n_clamp;
    s_c[2][wid] = n_bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tw = 0.0;
    unsigned c0 = 0, c1 = 0, c2 = 0;
    for (int i = 0; i < kBinBlock / 64; ++i) {
      tw += s_w[i];
      c0 += s_c[0][i];
      c1 += s_c[1][i];
      c2 += s_c[2][i];
    }
    if (wsum && img_b >= 0 && tw != 0.0) unsafeAtomicAdd(&wsum[(int64_t)img_b * kSlots + acc_slot], tw);
    if (counters) {
      if (c0) atomicAdd(&counters[0 * kSlots + acc_slot], (unsigned long long)c0);
      if (c1) atomicAdd(&counters[1 * kSlots + acc_slot], (unsigned long long)c1);
      if (c2) atomicAdd(&counters[2 * kSlots + acc_slot], (unsigned long long)c2);
    }
  }
}

// The key pass with counts aggregated per block in an LDS hash table: a block of
// kAggThreads threads takes kAggSpan consecutive visibilities, the first lane of each
// run of equal keys adds the run to its key's entry (slot within the block's share of
// the key = the returned count), and one global count atomic per distinct key of the
// block then reserves the block's share (its base).  Where the same keys recur within a
// few thousand rows (rows in time order, one channel each: the same baseline every few
// hundred rows, in the same tile and plane for minutes), this replaces most global
// atomics by LDS atomics; where equal keys are adjacent (a row's channels, measurement-
// set order) the wavefront runs already do that and the table only costs time, so the
// choice is the handle's (BinShape::aggregate, which wproj_autotune times).  A run whose
// key finds no entry within kAggProbes probes takes a global atomic of its own.  Same
// outputs as key_kernel.
// Shape measured on cfg4's rows (bin phase): 512 threads x 4 visibilities 1.38 ms, 1024 x 4
// 1.48, 1024 x 2 1.61, 1024 x 8 1.46, 512 x 8 1.39, 256 x 8 1.46; 2048 or 4096 table
// entries alike.
constexpr int kAggThreads = 512;
constexpr int kAggVpt = 4;
constexpr int kAggSpan = kAggThreads * kAggVpt;
constexpr int kAggSlots = 2048;  // a power of two
constexpr int kAggProbes = 16;
constexpr uint32_t kDirect = 0xffffffffu;  // entry index of a run counted globally

__device__ inline uint32_t agg_hash(uint32_t key) { return (key * 2654435761u) >> (32 - 11); }
static_assert(kAggSlots == 1 << 11, "agg_hash yields 11 bits");

template <typename Real, bool TAPWORD>
__global__ void __launch_bounds__(kAggThreads)
    key_agg_kernel(Geometry G, BinShape B, int64_t nvis, const double *__restrict__ uvw,
                   const Real *__restrict__ wt, const int64_t *__restrict__ img_off,
                   int S_fix, uint32_t *__restrict__ slots, uint32_t *count, double *wsum,
                   unsigned long long *counters) {
  constexpr int V = kAggVpt;
  __shared__ uint32_t h_key[kAggSlots], h_cnt[kAggSlots], h_base[kAggSlots];
  for (int i = threadIdx.x; i < kAggSlots; i += kAggThreads) {
    h_key[i] = kInvalid;
    h_cnt[i] = 0;
  }
  const int64_t j_first = (int64_t)blockIdx.x * kAggSpan;
  auto row = [&](int i) { return j_first + i * kAggThreads + threadIdx.x; };
  // every load of the thread first
  double c[V][3];
  Real wj[V];
#pragma unroll
  for (int i = 0; i < V; ++i) {
    const int64_t j = row(i);
    c[i][0] = c[i][1] = c[i][2] = 0.0;
    wj[i] = Real(0);
    if (j < nvis) {
      c[i][0] = uvw[3 * j];
      c[i][1] = uvw[3 * j + 1];
      c[i][2] = uvw[3 * j + 2];
      wj[i] = wt ? wt[j] : Real(1);
    }
  }
  // image of the block's first row, and of all its rows when one image holds them
  int img_b = -1, img_all = -1;
  if (j_first < nvis) {
    img_b = image_of(img_off, G.n_images, j_first);
    const int last = image_of(img_off, G.n_images, min(j_first + (int64_t)kAggSpan, nvis) - 1);
    img_all = img_b >= 0 && img_b == last ? img_b : -1;
  }
  uint32_t key[V], packed[V], tapw[V];
  bool fold[V];
  double w_mine = 0.0;
  unsigned n_drop = 0, n_clamp = 0, n_bad = 0;
#pragma unroll
  for (int i = 0; i < V; ++i) {
    const int64_t j = row(i);
    key[i] = kInvalid;
    packed[i] = 0;
    tapw[i] = 0;
    fold[i] = false;
    int cls = kFlagged;
    bool clamped = false;
    if (j < nvis) {
      const int img = img_all >= 0 ? img_all : image_of(img_off, G.n_images, j);
      if (img >= 0) {
        Footprint f;
        cls = classify(G, c[i], wj[i], f, TAPWORD ? 0 : S_fix);
        if (cls == kGridded) {
          key[i] = bin_key(G, B, img, f);
          fold[i] = f.fold;
          packed[i] = record_lds(G, B, f);
          if constexpr (TAPWORD) tapw[i] = tap_word(G, f);
          clamped = w_clamped(G, c[i][2]);
          if (img == img_b)
            w_mine += (double)wj[i];
          else if (wsum)
            unsafeAtomicAdd(&wsum[(int64_t)img * kSlots + (blockIdx.x & (kSlots - 1))], (double)wj[i]);
        }
      }
    }
    n_drop += (unsigned)__popcll(__ballot(cls == kDropped));
    n_bad += (unsigned)__popcll(__ballot(cls == kBadWeight));
    n_clamp += (unsigned)__popcll(__ballot(clamped));
  }
  __syncthreads();  // the table is cleared
  // runs into the table: entry and rank of each run's first lane
  Run run[V];
  uint32_t where[V], rank[V];
#pragma unroll
  for (int i = 0; i < V; ++i) {
    run[i] = run_of(key[i]);
    uint32_t e = kDirect, r = 0;
    if (run[i].lead) {
      uint32_t h = agg_hash(key[i]);
      for (int probe = 0; probe < kAggProbes; ++probe) {
        const uint32_t old = atomicCAS(&h_key[h], kInvalid, key[i]);
        if (old == kInvalid || old == key[i]) {
          e = h;
          break;
        }
        h = (h + 1u) & (uint32_t)(kAggSlots - 1);
      }
      r = e == kDirect ? atomicAdd(&count[key[i]], run[i].len) : atomicAdd(&h_cnt[e], run[i].len);
    }
    where[i] = e;
    rank[i] = r;
  }
  __syncthreads();  // every run is in the table
  // one global atomic per distinct key of the block
  uint32_t gb[kAggSlots / kAggThreads];
#pragma unroll
  for (int q = 0; q < kAggSlots / kAggThreads; ++q) {
    const int e = threadIdx.x + q * kAggThreads;
    const uint32_t k = h_key[e];
    uint32_t b = 0;
    if (k != kInvalid) b = atomicAdd(&count[k], h_cnt[e]);
    gb[q] = b;
  }
#pragma unroll
  for (int q = 0; q < kAggSlots / kAggThreads; ++q) h_base[threadIdx.x + q * kAggThreads] = gb[q];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < V; ++i) {
    const int64_t j = row(i);
    const uint32_t e = (uint32_t)__shfl((int)where[i], run[i].leader, 64);
    const uint32_t r = (uint32_t)__shfl((int)rank[i], run[i].leader, 64);
    const uint32_t slot = (e == kDirect ? r : h_base[e & (uint32_t)(kAggSlots - 1)] + r) +
                          (uint32_t)((threadIdx.x & 63) - run[i].leader);
    if (j < nvis) {
      slots[j] = slot;
      slots[nvis + j] = fold[i] ? (key[i] | kFoldBit) : key[i];
      slots[2 * nvis + j] = packed[i];
      if constexpr (TAPWORD) slots[3 * nvis + j] = tapw[i];
    }
  }
  // counters and weight sums, as in key_kernel
  __shared__ double s_w[kAggThreads / 64];
  __shared__ unsigned s_c[3][kAggThreads / 64];
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int acc_slot = blockIdx.x & (kSlots - 1);
  const double wv = wave_sum(w_mine);
  if (lane == 0) {
    s_w[wid] = wv;
    s_c[0][wid] = n_drop;
    s_c[1][wid] = n_clamp;
    s_c[2][wid] = n_bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tw = 0.0;
    unsigned c0 = 0, c1 = 0, c2 = 0;
    for (int i = 0; i < kAggThreads / 64; ++i) {
      tw += s_w[i];
      c0 += s_c[0][i];
      c1 += s_c[1][i];
      c2 += s_c[2][i];
    }
    if (wsum && img_b >= 0 && tw != 0.0) unsafeAtomicAdd(&wsum[(int64_t)img_b * kSlots + acc_slot], tw);
    if (counters) {
      if (c0) atomicAdd(&counters[0 * kSlots + acc_slot], (unsigned long long)c0);
      if (c1) atomicAdd(&counters[1 * kSlots + acc_slot], (unsigned long long)c1);
      if (c2) atomicAdd(&counters[2 * kSlots + acc_slot], (unsigned long long)c2);
    }
  }
}

// The record of visibility j and its bin key, from what the key pass stored; false when
// j is not gridded.  The key is loaded first, so that the bin offset it indexes is
// fetched while the rest of the record's inputs arrive; rows that are not gridded load
// nothing more.  TAPWORD: the tap word was stored; otherwise the first tap is the packed
// sub-kernel number times S_fix^2.
template <typename Real, typename Cplx, typename Rec, bool TAPWORD>
__device__ inline bool make_record(int64_t nvis, const Cplx *__restrict__ vis, const Real *__restrict__ wt,
                                   const uint32_t *__restrict__ slots, int S_fix, int64_t j, Rec &r,
                                   uint32_t &key) {
  key = slots[nvis + j];
  if (key == kInvalid) return false;
  const bool fold = (key & kFoldBit) != 0;
  key &= ~kFoldBit;
  r.lds = slots[2 * nvis + j];
  if constexpr (kHasTap<Rec>) {
    if constexpr (TAPWORD)
      r.tap = slots[3 * nvis + j];
    else
      r.tap = (r.lds >> kLdsBits) * (uint32_t)(S_fix * S_fix) | ((uint32_t)(S_fix - 1) << kTapBits);
  }
  const Real w = wt ? wt[j] : Real(1);
  if (vis) {
    // a folded visibility enters conjugated
    const Cplx v = vis[j];
    r.wr = w * v.x;
    r.wi = (fold ? -w : w) * v.y;
  } else if constexpr (kHasTap<Rec>) {
    // row-carrying records mark a folded row by a negative weight
    set_plan(r, fold ? -w : w, (uint32_t)j);
  }
  return true;
}

// Record of visibility j to offset[key] + its slot; V visibilities per thread
// (j = block kBinBlock V + i kBinBlock + thread), every record built before the first is
// stored.
template <typename Real, typename Cplx, typename Rec, bool TAPWORD, int V>
__global__ void __launch_bounds__(kBinBlock)
    scatter_kernel(int64_t nvis, const Cplx *__restrict__ vis, const Real *__restrict__ wt,
                   const uint32_t *__restrict__ slots, const uint32_t *__restrict__ offset, int S_fix,
                   Rec *__restrict__ rec) {
  Rec r[V];
  uint32_t key[V];
  bool ok[V];
  int64_t j[V];
#pragma unroll
  for (int i = 0; i < V; ++i) {
    j[i] = (int64_t)blockIdx.x * (kBinBlock * V) + i * kBinBlock + threadIdx.x;
    ok[i] = j[i] < nvis &&
            make_record<Real, Cplx, Rec, TAPWORD>(nvis, vis, wt, slots, S_fix, j[i], r[i], key[i]);
  }
#pragma unroll
  for (int i = 0; i < V; ++i)
    if (ok[i]) rec[offset[key[i]] + slots[j[i]]] = r[i];
}

// ---- stable binning: least-significant-digit radix sort of the bin keys ----
//
// Each visibility's sort key is its bin key, or n_keys when it is not gridded (so those
// sort last); its value is its index.  A pass sorts by one 8-bit digit and is stable:
// every block counts the digits of its kRadixTile consecutive elements, an exclusive scan
// of the counts laid out digit-major gives each (digit, block) its first output place,
// and within a block the elements keep their order (wavefront w takes the w-th quarter of
// the block's range, 64 elements a step; an element's rank among the equal digits before
// it is the count over earlier steps, kept in LDS per wavefront, plus the equal lanes
// below it in its step, found with one ballot per digit bit).  After the last pass the
// values list the gridded visibilities bin by bin, each bin in input order, and
// gather_kernel writes record p from visibility values[p].
constexpr int kRadixBits = 8;
constexpr int kRadixDigits = 1 << kRadixBits;
constexpr int kRadixThreads = 256;
constexpr int kRadixWaves = kRadixThreads / 64;
constexpr int kRadixSteps = 16;                          // 64-element steps per wavefront
constexpr int kRadixTile = kRadixThreads * kRadixSteps;  // elements per block
static_assert(kRadixThreads == kRadixDigits, "one thread per digit in the block-level steps");

// Lanes of the wavefront whose (valid) digit equals this lane's.
__device__ inline uint64_t same_digit_lanes(uint32_t d, bool valid) {
  uint64_t m = __ballot(valid);
#pragma unroll
  for (int b = 0; b < kRadixBits; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t on = __ballot(bit);
    m &= bit ? on : ~on;
  }
  return m;
}

// Set lanes of m below this lane.
__device__ inline uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Element e of the block's range: wavefront w's quarter, step i, lane.
__device__ inline int64_t radix_elem(int w, int i, int lane) {
  return (int64_t)blockIdx.x * kRadixTile + (int64_t)w * (64 * kRadixSteps) + i * 64 + lane;
}

__global__ void __launch_bounds__(kBinBlock)
    sort_key_kernel(int64_t nvis, uint32_t n_keys, const uint32_t *__restrict__ slots,
                    uint32_t *__restrict__ keys) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nvis) return;
  const uint32_t kw = slots[nvis + j];
  keys[j] = kw != kInvalid ? kw & ~kFoldBit : n_keys;
}

// count[d * n_blocks + block] = elements of the block whose digit is d.
__global__ void __launch_bounds__(kRadixThreads)
    radix_count_kernel(const uint32_t *__restrict__ keys, int64_t n, int shift, int64_t n_blocks,
                       uint32_t *__restrict__ count) {
  __shared__ uint32_t h[kRadixDigits];
  h[threadIdx.x] = 0u;
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t key[kRadixSteps];
#pragma unroll
  for (int i = 0; i < kRadixSteps; ++i) {
    const int64_t e = radix_elem(w, i, lane);
    key[i] = e < n ? keys[e] : 0u;
  }
#pragma unroll
  for (int i = 0; i < kRadixSteps; ++i) {
    const bool valid = radix_elem(w, i, lane) < n;
    const uint32_t d = (key[i] >> shift) & (uint32_t)(kRadixDigits - 1);
    const uint64_t m = same_digit_lanes(d, valid);
    if (valid && lanes_below(m) == 0u) atomicAdd(&h[d], (uint32_t)__popcll(m));
  }
  __syncthreads();
  count[(int64_t)threadIdx.x * n_blocks + blockIdx.x] = h[threadIdx.x];
}

// One stable pass: element e goes to digit_off[d * n_blocks + block] + (elements of digit
// d before it in the block).  vin == nullptr: the values are the element indices;
// kout == nullptr: the keys are not needed after this pass.
__global__ void __launch_bounds__(kRadixThreads)
    radix_place_kernel(const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, int64_t n,
                       int shift, int64_t n_blocks, const uint32_t *__restrict__ digit_off,
                       uint32_t *__restrict__ kout, uint32_t *__restrict__ vout) {
  __shared__ uint32_t cnt[kRadixWaves][kRadixDigits];
  for (int i = threadIdx.x; i < kRadixWaves * kRadixDigits; i += kRadixThreads) cnt[i / kRadixDigits][i % kRadixDigits] = 0u;
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t key[kRadixSteps], val[kRadixSteps], rank[kRadixSteps];
#pragma unroll
  for (int i = 0; i < kRadixSteps; ++i) {
    const int64_t e = radix_elem(w, i, lane);
    key[i] = e < n ? kin[e] : 0u;
    val[i] = e < n ? (vin ? vin[e] : (uint32_t)e) : 0u;
  }
  // rank of each element among the wavefront's earlier elements of its digit; the lanes
  // of a step read the running count before its first lane of each digit adds the step's
  // share (one wavefront's LDS accesses take effect in program order)
#pragma unroll
  for (int i = 0; i < kRadixSteps; ++i) {
    const bool valid = radix_elem(w, i, lane) < n;
    const uint32_t d = (key[i] >> shift) & (uint32_t)(kRadixDigits - 1);
    const uint64_t m = same_digit_lanes(d, valid);
    const uint32_t below = lanes_below(m);
    const uint32_t before = cnt[w][d];
    rank[i] = before + below;
    if (valid && below == 0u) cnt[w][d] = before + (uint32_t)__popcll(m);
  }
  __syncthreads();
  // first output place of wavefront v's elements of digit d (thread d)
  {
    const int d = threadIdx.x;
    uint32_t start = digit_off[(int64_t)d * n_blocks + blockIdx.x];
    for (int v = 0; v < kRadixWaves; ++v) {
      const uint32_t c = cnt[v][d];
      cnt[v][d] = start;
      start += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kRadixSteps; ++i) {
    if (radix_elem(w, i, lane) < n) {
      const uint32_t d = (key[i] >> shift) & (uint32_t)(kRadixDigits - 1);
      const uint32_t pos = cnt[w][d] + rank[i];
      if (kout) kout[pos] = key[i];
      vout[pos] = val[i];
    }
  }
}

// Record p (below the number of gridded visibilities, *total) from visibility order[p].
// (Two records per thread measured slower here: 0.99 against 0.97 ms.)
template <typename Real, typename Cplx, typename Rec, bool TAPWORD>
__global__ void __launch_bounds__(kBinBlock)
    gather_kernel(int64_t nvis, const Cplx *__restrict__ vis, const Real *__restrict__ wt,
                  const uint32_t *__restrict__ slots, const uint32_t *__restrict__ order,
                  const uint32_t *__restrict__ total, int S_fix, Rec *__restrict__ rec) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (int64_t)*total) return;
  Rec r;
  uint32_t key;
  if (make_record<Real, Cplx, Rec, TAPWORD>(nvis, vis, wt, slots, S_fix, (int64_t)order[p], r, key))
    rec[p] = r;
}

// Adds the per-slot partial weight sums and counters into the caller's outputs, in a
// fixed slot order.
__global__ void __launch_bounds__(256)
    finalize_kernel(int n_images, const double *__restrict__ wslots,
                    const unsigned long long *__restrict__ cslots, double *wsum,
                    unsigned long long *counters) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (wsum && t < n_images) {
    double s = 0.0;
    for (int k = 0; k < kSlots; ++k) s += wslots[(int64_t)t * kSlots + k];
    wsum[t] += s;
  }
  if (counters && t < 3) {
    unsigned long long c = 0;
    for (int k = 0; k < kSlots; ++k) c += cslots[t * kSlots + k];
    counters[t] += c;
  }
}

// ---- exclusive scan of uint32 counts (three phases) ----
constexpr int kScanBlock = 1024;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanBlock * kScanItems;

__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *sh, uint32_t &total) {
  // Hillis-Steele over the block in LDS (1024 entries)
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    uint32_t add = t >= off ? sh[t - off] : 0u;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  total = sh[kScanBlock - 1];
  uint32_t incl = sh[t];
  __syncthreads();
  return incl - v;
}

__global__ void __launch_bounds__(kScanBlock)
    scan_tiles_kernel(const uint32_t *__restrict__ in, uint32_t *__restrict__ out, int64_t n,
                      uint32_t *__restrict__ tile_sums) {
  __shared__ uint32_t sh[kScanBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < n ? in[base + i] : 0u;
    s += v[i];
  }
  uint32_t total;
  uint32_t ex = block_exclusive_scan(s, sh, total);
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = ex;
    ex += v[i];
  }
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

// Scans the per-tile sums in place (one block, any count) and writes the grand total.
__global__ void __launch_bounds__(kScanBlock)
    scan_sums_kernel(uint32_t *sums, int64_t n_tiles, uint32_t *total_out) {
  __shared__ uint32_t sh[kScanBlock];
  uint32_t carry = 0;
  for (int64_t b = 0; b < n_tiles; b += kScanBlock) {
    const int64_t i = b + threadIdx.x;
    const uint32_t v = i < n_tiles ? sums[i] : 0u;
    uint32_t total;
    const uint32_t ex = block_exclusive_scan(v, sh, total);
    if (i < n_tiles) sums[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) *total_out = carry;
}

__global__ void __launch_bounds__(256)
    scan_add_kernel(uint32_t *out, int64_t n, const uint32_t *__restrict__ tile_prefix) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += tile_prefix[i / kScanTile];
}

__global__ void __launch_bounds__(256)
    chunk_count_kernel(const uint32_t *__restrict__ offset, int64_t n_tiles, int kw, int chunk,
                       uint32_t *__restrict__ nch) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  const uint32_t b = offset[t * kw], e = offset[(t + 1) * kw];
  nch[t] = (e - b + (uint32_t)chunk - 1) / (uint32_t)chunk;
}

__global__ void __launch_bounds__(256)
    chunk_emit_kernel(const uint32_t *__restrict__ offset, int64_t n_tiles, int kw, int chunk,
                      const uint32_t *__restrict__ choff, WorkItem *__restrict__ items) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  const uint32_t b = offset[t * kw], e = offset[(t + 1) * kw];
  uint32_t o = choff[t];
  for (uint32_t s = b; s < e; s += (uint32_t)chunk, ++o) {
    WorkItem w;
    w.tile = (uint32_t)t;
    w.begin = s;
    w.end = min(e, s + (uint32_t)chunk);
    items[o] = w;
  }
}

// Largest-first work order.  The queue of the gridding and degridding kernels hands
// out work items in this order, so the long items start early and the short ones fill
// the end of the launch instead of one long item running alone (the work list itself
// stays in tile order, which the partial-tile reduce relies on).  Items are counted
// into kOrderBuckets size classes and placed class by class; the order inside a class
// follows the placement atomics, which changes only the schedule, not any result.
__device__ inline int size_class(const WorkItem &w, int chunk) {
  const uint32_t size = w.end - w.begin;  // 1..chunk
  const uint32_t c = (uint32_t)(((uint64_t)((uint32_t)chunk - size) * kOrderBuckets) / (uint32_t)chunk);
  return (int)min(c, (uint32_t)(kOrderBuckets - 1));
}

__global__ void __launch_bounds__(256)
    order_count_kernel(const WorkItem *__restrict__ items, const uint32_t *__restrict__ n_items_ptr,
                       int chunk, uint32_t *class_count) {
  __shared__ uint32_t h[kOrderBuckets];
  if (threadIdx.x < kOrderBuckets) h[threadIdx.x] = 0u;
  __syncthreads();
  const uint32_t n = *n_items_ptr;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&h[size_class(items[i], chunk)], 1u);
  __syncthreads();
  if (threadIdx.x < kOrderBuckets && h[threadIdx.x]) atomicAdd(&class_count[threadIdx.x], h[threadIdx.x]);
}

// order[start of class c + cursor] = item; start of class c = items in classes < c.
__global__ void __launch_bounds__(256)
    order_place_kernel(const WorkItem *__restrict__ items, const uint32_t *__restrict__ n_items_ptr,
                       int chunk, const uint32_t *__restrict__ class_count, uint32_t *cursor,
                       uint32_t *__restrict__ order) {
  __shared__ uint32_t h[kOrderBuckets], base[kOrderBuckets];
  if (threadIdx.x < kOrderBuckets) h[threadIdx.x] = 0u;
  __syncthreads();
  const uint32_t n = *n_items_ptr;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int c = 0;
  uint32_t rank = 0;
  if (i < n) {
    c = size_class(items[i], chunk);
    rank = atomicAdd(&h[c], 1u);
  }
  __syncthreads();
  if (threadIdx.x < kOrderBuckets) {
    uint32_t start = 0;
    for (int k = 0; k < (int)threadIdx.x; ++k) start += class_count[k];
    base[threadIdx.x] = h[threadIdx.x] ? start + atomicAdd(&cursor[threadIdx.x], h[threadIdx.x]) : 0u;
  }
  __syncthreads();
  if (i < n) order[base[c] + rank] = (uint32_t)i;
}

template <typename Rec>
__global__ void __launch_bounds__(256)
    plan_rows_kernel(const Rec *__restrict__ rec, const uint32_t *__restrict__ total, int64_t nvis,
                     uint32_t *__restrict__ rows) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvis) return;
  rows[i] = i < (int64_t)*total ? get_row(rec[i]) : 0xffffffffu;
}

__global__ void fill_u32_kernel(uint32_t *p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Records in bin order: scattered to offset[key] + slot, or, for stable bins, sorted by
// key (radix passes over the key's significant bits) and gathered in sorted order.
template <typename Real, typename Cplx, typename Rec, bool TAPWORD>
hipError_t place_records(const wproj_kernels *k, const BinShape &B, int64_t nvis, const void *vis, const void *wt,
                         const BinWorkspace &W, int S_fix, hipStream_t s) {
  const dim3 grid(nblk(nvis, kBinBlock)), block(kBinBlock);
  if (!B.stable) {
    if (!TAPWORD && !B.aggregate)
      hipLaunchKernelGGL((scatter_kernel<Real, Cplx, Rec, TAPWORD, 2>), dim3(nblk(nvis, 2 * kBinBlock)), block, 0, s,
                         nvis, (const Cplx *)vis, (const Real *)wt, W.slots, W.offset, S_fix, (Rec *)W.rec);
    else
      hipLaunchKernelGGL((scatter_kernel<Real, Cplx, Rec, TAPWORD, 1>), grid, block, 0, s, nvis, (const Cplx *)vis,
                         (const Real *)wt, W.slots, W.offset, S_fix, (Rec *)W.rec);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(sort_key_kernel, grid, block, 0, s, nvis, (uint32_t)B.n_keys, W.slots, W.sort_keys[0]);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // keys run from 0 to n_keys (not gridded)
  int bits = 1;
  while (bits < 32 && (B.n_keys >> bits) != 0) ++bits;
  const int64_t n_blocks = (nvis + kRadixTile - 1) / kRadixTile;
  const int64_t n_counts = n_blocks * kRadixDigits;
  const uint32_t *vals = nullptr;  // element indices in the first pass
  int cur = 0;
  for (int shift = 0; shift < bits; shift += kRadixBits) {
    const bool last = shift + kRadixBits >= bits;
    hipLaunchKernelGGL(radix_count_kernel, dim3((unsigned)n_blocks), dim3(kRadixThreads), 0, s,
                       W.sort_keys[cur], nvis, shift, n_blocks, W.digit_count);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_exclusive_scan(W.digit_count, W.digit_off, n_counts, W.scan_tmp, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(radix_place_kernel, dim3((unsigned)n_blocks), dim3(kRadixThreads), 0, s,
                       W.sort_keys[cur], vals, nvis, shift, n_blocks, W.digit_off,
                       last ? nullptr : W.sort_keys[cur ^ 1], W.sort_vals[cur ^ 1]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    vals = W.sort_vals[cur ^ 1];
    cur ^= 1;
  }
  hipLaunchKernelGGL((gather_kernel<Real, Cplx, Rec, TAPWORD>), grid, block, 0, s, nvis, (const Cplx *)vis,
                     (const Real *)wt, W.slots, vals, W.offset + B.n_keys, S_fix, (Rec *)W.rec);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

int64_t scan_temp_words(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

int64_t radix_digit_slots(int64_t nvis) {
  return std::max<int64_t>(1, (nvis + kRadixTile - 1) / kRadixTile) * kRadixDigits;
}

// out[i] = sum_{k < i} in[i], out[n] = total (out has n + 1 entries).
hipError_t launch_exclusive_scan(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp,
                                 hipStream_t s) {
  const int64_t tiles = (n + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(scan_tiles_kernel, dim3((unsigned)tiles), dim3(kScanBlock), 0, s, in, out, n,
                     tmp);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kScanBlock), 0, s, tmp, tiles, out + n);
  hipLaunchKernelGGL(scan_add_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, out, n, tmp);
  return hipGetLastError();
}

hipError_t launch_plan_rows(const wproj_kernels *k, const BinShape &B, const BinWorkspace &W, int64_t nvis,
                            uint32_t *rows, hipStream_t s) {
  // plans hold row-carrying records: RecordF64 in FP64, RecordF32 otherwise
  const uint32_t *total = W.offset + B.n_keys;
  if (k->params.precision == WPROJ_F64)
    hipLaunchKernelGGL(plan_rows_kernel<RecordF64>, dim3(nblk(nvis, 256)), dim3(256), 0, s,
                       (const RecordF64 *)W.rec, total, nvis, rows);
  else
    hipLaunchKernelGGL(plan_rows_kernel<RecordF32>, dim3(nblk(nvis, 256)), dim3(256), 0, s,
                       (const RecordF32 *)W.rec, total, nvis, rows);
  return hipGetLastError();
}

hipError_t launch_bin(const wproj_kernels *k, const BinShape &B, int64_t nvis, const double *uvw,
                      const void *vis, const void *wt, const int64_t *img_off, double *wsum,
                      int64_t *counters, const BinWorkspace &W, hipStream_t s) {
  const Geometry &G = k->geo;
  hipError_t e = launch_fill_u32(W.count, B.n_keys, 0u, s);
  if (e != hipSuccess) return e;
  // zero the slot accumulators (bit pattern 0 is 0.0 and 0)
  if ((e = launch_fill_u32((uint32_t *)W.wslots, 2 * kSlots * (int64_t)k->params.n_images, 0u, s)) != hipSuccess)
    return e;
  if ((e = launch_fill_u32((uint32_t *)W.cslots, 2 * 3 * kSlots, 0u, s)) != hipSuccess) return e;
  double *wpart = wsum ? W.wslots : nullptr;
  auto *cnt = counters ? W.cslots : nullptr;
  const dim3 key_grid(nblk(nvis, kBinBlock * kKeyVpt)), block(kBinBlock);
  const bool agg = B.aggregate != 0;  // counts aggregated per block in LDS
  const dim3 agg_grid(nblk(nvis, kAggSpan)), agg_block(kAggThreads);
  // per-plane supports: the key pass stores each record's tap word (TAPWORD); a fixed
  // support packs the sub-kernel number into the record's first word instead
  const bool tapword = B.pack_sub == 0;
  const int S_fix = k->s_max;  // the fixed support of packed records
  auto key_pass = [&](auto real_tag, auto tap_tag) {
    using Real = decltype(real_tag);
    constexpr bool TW = decltype(tap_tag)::value;
    if (agg)
      hipLaunchKernelGGL((key_agg_kernel<Real, TW>), agg_grid, agg_block, 0, s, G, B, nvis, uvw, (const Real *)wt,
                         img_off, S_fix, W.slots, W.count, wpart, cnt);
    else
      hipLaunchKernelGGL((key_kernel<Real, TW>), key_grid, block, 0, s, G, B, nvis, uvw, (const Real *)wt, img_off,
                         S_fix, W.slots, W.count, wpart, cnt);
  };
  if (k->params.precision == WPROJ_F64) {
    if (tapword)
      key_pass(double{}, std::true_type{});
    else
      key_pass(double{}, std::false_type{});
  } else {
    if (tapword)
      key_pass(float{}, std::true_type{});
    else
      key_pass(float{}, std::false_type{});
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (wsum || counters) {
    const int ni = k->params.n_images;
    hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)((std::max(ni, 3) + 255) / 256)), dim3(256), 0,
                       s, ni, W.wslots, W.cslots, wsum, reinterpret_cast<unsigned long long *>(counters));
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = launch_exclusive_scan(W.count, W.offset, B.n_keys, W.scan_tmp, s)) != hipSuccess) return e;
  if (k->params.precision == WPROJ_F64)
    e = tapword ? place_records<double, double2, RecordF64, true>(k, B, nvis, vis, wt, W, S_fix, s)
                : place_records<double, double2, RecordF64, false>(k, B, nvis, vis, wt, W, S_fix, s);
  else if (!tapword && vis)  // W V records of a fixed support: no tap word (12 bytes)
    e = place_records<float, float2, RecordF32P, false>(k, B, nvis, vis, wt, W, S_fix, s);
  else
    e = tapword ? place_records<float, float2, RecordF32, true>(k, B, nvis, vis, wt, W, S_fix, s)
                : place_records<float, float2, RecordF32, false>(k, B, nvis, vis, wt, W, S_fix, s);
  if (e != hipSuccess) return e;
  // work list: per tile, ceil(records / chunk) items
  hipLaunchKernelGGL(chunk_count_kernel, dim3(nblk(B.n_tiles, 256)), dim3(256), 0, s, W.offset,
                     B.n_tiles, B.kw, B.chunk, W.nch);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_exclusive_scan(W.nch, W.choff, B.n_tiles, W.scan_tmp, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(chunk_emit_kernel, dim3(nblk(B.n_tiles, 256)), dim3(256), 0, s, W.offset,
                     B.n_tiles, B.kw, B.chunk, W.choff, W.items);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // largest-first order of the work items (their number is choff[n_tiles] <= max_items)
  if ((e = launch_fill_u32(W.order_cnt, 2 * kOrderBuckets, 0u, s)) != hipSuccess) return e;
  const uint32_t *n_items = W.choff + B.n_tiles;
  hipLaunchKernelGGL(order_count_kernel, dim3(nblk(W.max_items, 256)), dim3(256), 0, s, W.items, n_items,
                     B.chunk, W.order_cnt);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(order_place_kernel, dim3(nblk(W.max_items, 256)), dim3(256), 0, s, W.items, n_items,
                     B.chunk, W.order_cnt, W.order_cnt + kOrderBuckets, W.order);
  return hipGetLastError();
}

}  // namespace wproj
