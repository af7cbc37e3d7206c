// C ABI entry points: argument checking, handle construction (kernel tables, grid
// correction, rocFFT plans) and dispatch to the kernel launchers.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <tuple>

#include "wproj_tiled.h"

using namespace wproj;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(WPROJ_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// Prolate spheroidal psi_0 as a Legendre series (host, FP64).
//
// psi_0(c, x) is the eigenfunction with the smallest eigenvalue of
// -d/dx[(1 - x^2) d/dx] + c^2 x^2.  In the normalised Legendre basis
// Pbar_n = sqrt(n + 1/2) P_n the even part is the symmetric tridiagonal matrix
//   d_k = n(n+1) + c^2 (2n(n+1) - 1)/((2n+3)(2n-1)),
//   e_k = c^2 (n+1)(n+2)/((2n+3) sqrt((2n+1)(2n+5))),      n = 2k,
// (Xiao, Rokhlin & Yarvin 2001).  The smallest eigenvalue is found by Sturm-count
// bisection, its eigenvector by inverse iteration with a shift just below it (the
// shifted matrix is then positive definite, so the tridiagonal solve needs no
// pivoting).  Returned: coefficients of P_0, P_2, ... with psi_0(0) > 0.
// ---------------------------------------------------------------------------
std::vector<double> prolate_legendre(double c) {
  const int K = (int)c + 40;
  std::vector<double> d(K), e(K > 1 ? K - 1 : 1, 0.0);
  for (int k = 0; k < K; ++k) {
    const double n = 2.0 * k;
    d[k] = n * (n + 1.0) + c * c * (2.0 * n * (n + 1.0) - 1.0) / ((2.0 * n + 3.0) * (2.0 * n - 1.0));
    if (k + 1 < K)
      e[k] = c * c * (n + 1.0) * (n + 2.0) / ((2.0 * n + 3.0) * sqrt((2.0 * n + 1.0) * (2.0 * n + 5.0)));
  }
  auto below = [&](double x) {  // number of eigenvalues < x
    int cnt = 0;
    double q = d[0] - x;
    if (q < 0) ++cnt;
    for (int k = 1; k < K; ++k) {
      if (q == 0.0) q = 1e-300;
      q = d[k] - x - e[k - 1] * e[k - 1] / q;
      if (q < 0) ++cnt;
    }
    return cnt;
  };
  double lo = d[0], hi = d[0];
  for (int k = 0; k < K; ++k) {
    double r = (k > 0 ? fabs(e[k - 1]) : 0.0) + (k + 1 < K ? fabs(e[k]) : 0.0);
    lo = std::min(lo, d[k] - r);
    hi = std::max(hi, d[k] + r);
  }
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (below(mid) >= 1)
      hi = mid;
    else
      lo = mid;
  }
  const double chi = 0.5 * (lo + hi);
  const double sigma = chi - 1e-9 * std::max(1.0, fabs(chi));
  std::vector<double> x(K, 1.0), y(K), cp(K), dp(K);
  for (int iter = 0; iter < 4; ++iter) {
    // Thomas algorithm on (A - sigma I) y = x
    double b0 = d[0] - sigma;
    cp[0] = (K > 1 ? e[0] : 0.0) / b0;
    dp[0] = x[0] / b0;
    for (int k = 1; k < K; ++k) {
      double den = (d[k] - sigma) - e[k - 1] * cp[k - 1];
      cp[k] = (k + 1 < K ? e[k] : 0.0) / den;
      dp[k] = (x[k] - e[k - 1] * dp[k - 1]) / den;
    }
    y[K - 1] = dp[K - 1];
    for (int k = K - 2; k >= 0; --k) y[k] = dp[k] - cp[k] * y[k + 1];
    double nrm = 0.0;
    for (int k = 0; k < K; ++k) nrm += y[k] * y[k];
    nrm = sqrt(nrm);
    for (int k = 0; k < K; ++k) x[k] = y[k] / nrm;
  }
  std::vector<double> coef(K);
  double at0 = 0.0, p2k0 = 1.0;  // P_{2k}(0) = (-1)^k (2k-1)!!/(2k)!!
  for (int k = 0; k < K; ++k) {
    coef[k] = x[k] * sqrt(2.0 * k + 0.5);
    at0 += coef[k] * p2k0;
    p2k0 *= -(2.0 * k + 1.0) / (2.0 * k + 2.0);
  }
  if (at0 < 0)
    for (double &v : coef) v = -v;
  return coef;
}

int validate(const wproj_params *p, std::vector<int32_t> &supp) {
  if (!p) return fail(WPROJ_EINVAL, "params is NULL");
  const int n = p->n;
  if (n < 2 || n > 32768 || (n & 1)) return fail(WPROJ_EINVAL, "n must be even in [2, 32768]");
  if (!(isfinite(p->cell_rad) && p->cell_rad > 0.0 && (double)n * p->cell_rad < 2.0))
    return fail(WPROJ_EINVAL, "cell_rad must be > 0 with n * cell_rad < 2");
  if (p->n_wplanes < 1 || p->n_wplanes > 4096)
    return fail(WPROJ_EINVAL, "n_wplanes must be in [1, 4096]");
  if (!(isfinite(p->w_max) && p->w_max >= 0.0)) return fail(WPROJ_EINVAL, "w_max must be >= 0");
  if (p->n_wplanes > 1 && !(p->w_max > 0.0))
    return fail(WPROJ_EINVAL, "w_max must be > 0 with more than one w-plane");
  if (p->support < 1 || p->support > 32) return fail(WPROJ_EINVAL, "support must be in [1, 32]");
  if (p->oversample < 1 || p->oversample > 256)
    return fail(WPROJ_EINVAL, "oversample must be in [1, 256]");
  if (p->kernel_image_size < 2 || p->kernel_image_size > 4096 || (p->kernel_image_size & 1))
    return fail(WPROJ_EINVAL, "kernel_image_size must be even in [2, 4096]");
  if (p->precision < WPROJ_F64 || p->precision > WPROJ_F32_F16TABLE)
    return fail(WPROJ_EINVAL, "unknown precision %d", p->precision);
  if (p->n_images < 1) return fail(WPROJ_EINVAL, "n_images must be >= 1");
  if (p->algorithm != WPROJ_ALGO_TILED && p->algorithm != WPROJ_ALGO_PLAIN)
    return fail(WPROJ_EINVAL, "unknown algorithm %d", p->algorithm);
  if (p->tile != 0 && p->tile != 16 && p->tile != 32 && p->tile != 64)
    return fail(WPROJ_EINVAL, "tile must be 0, 16, 32 or 64");
  if (p->chunk != 0 && (p->chunk < 256 || p->chunk > 65536))
    return fail(WPROJ_EINVAL, "chunk must be 0 or in [256, 65536]");
  if (p->w_mode < WPROJ_W_LINEAR || p->w_mode > WPROJ_W_STACK)
    return fail(WPROJ_EINVAL, "unknown w_mode %d", p->w_mode);
  if (p->w_mode == WPROJ_W_STACK) {
    if (p->n_wlayers < 0 || p->n_wlayers > 4096) return fail(WPROJ_EINVAL, "n_wlayers must be in [0, 4096]");
    if (!(p->w_max > 0.0)) return fail(WPROJ_EINVAL, "w-stacking needs w_max > 0");
  } else if (p->n_wlayers != 0 && p->n_wlayers != 1) {
    return fail(WPROJ_EINVAL, "n_wlayers > 1 needs w_mode WPROJ_W_STACK");
  }
  if (p->accumulate_runs != 0 && p->accumulate_runs != 1)
    return fail(WPROJ_EINVAL, "accumulate_runs must be 0 or 1");
  if (p->bin_aggregate != 0 && p->bin_aggregate != 1)
    return fail(WPROJ_EINVAL, "bin_aggregate must be 0 or 1");
  if (p->stable_bins != 0 && p->stable_bins != 1)
    return fail(WPROJ_EINVAL, "stable_bins must be 0 or 1");
  for (int r : p->reserved)
    if (r != 0) return fail(WPROJ_EINVAL, "reserved fields must be zero");
  supp.assign(p->n_wplanes, p->support);
  if (p->support_per_plane)
    for (int i = 0; i < p->n_wplanes; ++i) supp[i] = p->support_per_plane[i];
  for (int s : supp) {
    if (s < 1 || s > 32 || s > n) return fail(WPROJ_EINVAL, "plane support must be in [1, min(32, n)]");
    if (((int64_t)s * p->oversample) & 1) return fail(WPROJ_EINVAL, "S_p * oversample must be even");
  }
  return WPROJ_OK;
}

void destroy(wproj_kernels *k) {
  if (!k) return;
  for (auto &v : k->prof)
    for (auto &pr : v) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  for (hipEvent_t e : k->event_pool) (void)hipEventDestroy(e);
  if (k->fft_fwd) rocfft_plan_destroy(k->fft_fwd);
  if (k->fft_inv) rocfft_plan_destroy(k->fft_inv);
  if (k->fft_c2r) rocfft_plan_destroy(k->fft_c2r);
  (void)hipFree(k->d_supp);
  (void)hipFree(k->d_tab_off);
  (void)hipFree(k->d_tab);
  (void)hipFree(k->d_tab_pair);
  (void)hipFree(k->d_kappa);
  (void)hipFree(k->d_taper);
  delete k;
}

std::once_flag g_fft_once;
rocfft_status g_fft_setup = rocfft_status_success;

struct TempBuffers {
  void *p[4] = {nullptr, nullptr, nullptr, nullptr};
  ~TempBuffers() {
    for (void *q : p) (void)hipFree(q);
  }
};

int check_device(const wproj_kernels *k) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(WPROJ_EHIP, "hipGetDevice failed");
  if (dev != k->device)
    return fail(WPROJ_EINVAL, "handle was built on device %d but device %d is current", k->device, dev);
  return WPROJ_OK;
}

hipEvent_t take_event(wproj_kernels *k) {
  if (!k->event_pool.empty()) {
    hipEvent_t e = k->event_pool.back();
    k->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

constexpr int64_t kAlign = 256;
inline int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

BinShape bin_shape(const wproj_kernels *k) {
  BinShape B;
  B.tile = k->tile;
  B.log2_tile = 0;
  while ((1 << B.log2_tile) < k->tile) ++B.log2_tile;
  B.pitch = tile_shape(k, k->tile).pitch;
  B.ntx = (k->params.n + k->tile - 1) / k->tile;
  B.nty = B.ntx;
  B.kw = k->plane_in_key ? k->params.n_wplanes : 1;
  B.chunk = k->chunk;
  B.aggregate = k->bin_aggregate;
  B.stable = k->stable_bins;
  // a fixed support with a kernel of its own, and sub-kernel numbers that fit above the
  // LDS offset
  const int64_t n_sub = (int64_t)k->params.n_wplanes * k->params.oversample * k->params.oversample;
  B.pack_sub = k->uniform_support && k->s_max >= kMinFixedSupport && k->s_max <= kMaxFixedSupport &&
               n_sub <= (1ll << (32 - kLdsBits));
  B.n_tiles = (int64_t)k->geo.n_grids * B.ntx * B.nty;
  B.n_keys = B.n_tiles * B.kw;
  return B;
}

// Bins the keys can number: the key pass stores the fold flag of fixed-support records in
// the top bit of their 32-bit key word, and the scatter reads it there in every w mode.
int64_t max_keys(const wproj_kernels *) { return (int64_t)0x7fffffffll; }

// Lays the binning buffers out from `base` (nullptr: sizes only); returns total bytes.
int64_t carve(const wproj_kernels *k, int64_t nvis, char *base, BinWorkspace &W) {
  const BinShape B = bin_shape(k);
  const int64_t rec_bytes = k->params.precision == WPROJ_F64 ? sizeof(RecordF64) : sizeof(RecordF32);
  // a tile with r records gives ceil(r / chunk) <= r / chunk + 1 items, and at most
  // min(n_tiles, nvis) tiles hold records
  const int64_t max_items = std::min<int64_t>(B.n_tiles, nvis) + nvis / B.chunk + 1;
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    char *p = base ? base + off : nullptr;
    off += align_up(bytes);
    return p;
  };
  // per visibility: slot, key and the record's first word; with per-plane supports also
  // the record's tap word
  W.slots = (uint32_t *)take(4 * nvis * (B.pack_sub ? 3 : 4));
  W.rec = take(rec_bytes * nvis);
  W.count = (uint32_t *)take(4 * B.n_keys);
  W.offset = (uint32_t *)take(4 * (B.n_keys + 1));
  W.nch = (uint32_t *)take(4 * B.n_tiles);
  W.choff = (uint32_t *)take(4 * (B.n_tiles + 1));
  W.items = (WorkItem *)take((int64_t)sizeof(WorkItem) * max_items);
  const int64_t digit_slots = B.stable ? radix_digit_slots(nvis) : 0;
  W.scan_tmp = (uint32_t *)take(4 * scan_temp_words(std::max({B.n_keys, B.n_tiles, digit_slots})));
  W.counter = (uint32_t *)take(4);
  W.order = (uint32_t *)take(4 * max_items);
  W.order_cnt = (uint32_t *)take(4 * 2 * kOrderBuckets);
  W.max_items = max_items;
  const TileShape ts = tile_shape(k, B.tile);
  const int64_t cplx = k->params.precision == WPROJ_F64 ? 16 : 8;
  W.partial = take(max_items * (int64_t)ts.rows * ts.rows * cplx);
  W.wslots = (double *)take(8 * kSlots * (int64_t)k->params.n_images);
  W.cslots = (unsigned long long *)take(8 * 3 * kSlots);
  for (int i = 0; i < 2; ++i) {
    W.sort_keys[i] = B.stable ? (uint32_t *)take(4 * nvis) : nullptr;
    W.sort_vals[i] = B.stable ? (uint32_t *)take(4 * nvis) : nullptr;
  }
  W.digit_count = B.stable ? (uint32_t *)take(4 * digit_slots) : nullptr;
  W.digit_off = B.stable ? (uint32_t *)take(4 * (digit_slots + 1)) : nullptr;
  return off;
}

// Tile sides the autotuner tries (each only where one wavefront's tile copy fits in a
// workgroup's LDS).  128 is not offered: a 128-cell tile with its halo needs more than
// the 64 KiB a workgroup may hold (146 KB at S = 8 in FP32) and more cells than the
// records' 14-bit LDS offset can address.
constexpr int kTuneTiles[] = {16, 32, 64};
constexpr int kTuneChunks[] = {1024, 2048, 4096, 8192, 16384};

bool plane_in_key_for(const wproj_kernels *k, int tile) {
  const int64_t nt = (k->params.n + tile - 1) / tile;
  return (int64_t)k->geo.n_grids * nt * nt * k->params.n_wplanes <= (1ll << 25);
}

// Workspace for nvis visibilities under any tile/chunk the autotuner may select.
int64_t workspace_bytes_for(const wproj_kernels *k, int64_t nvis) {
  int64_t ws = align_up((int64_t)k->fft_work_bytes);
  if (k->params.algorithm == WPROJ_ALGO_TILED) {
    wproj_kernels tmp;  // geometry only
    tmp.params = k->params;
    tmp.geo = k->geo;
    tmp.s_max = k->s_max;
    tmp.uniform_support = k->uniform_support;
    tmp.stable_bins = k->stable_bins;
    for (int tile : kTuneTiles) {
      if (tile_shape(k, tile).lds_bytes + 256 > k->max_lds) continue;  // never tuned to
      tmp.tile = tile;
      tmp.plane_in_key = plane_in_key_for(k, tile);
      tmp.chunk = kTuneChunks[0];
      BinWorkspace W;
      ws = std::max(ws, carve(&tmp, nvis, nullptr, W));
    }
    BinWorkspace W;
    ws = std::max(ws, carve(k, nvis, nullptr, W));
  }
  return ws;
}

struct TuneKey {
  int n, n_images, n_w, s_max, uniform, O, precision, w_mode, n_layers;
  int log2_nvis;
  bool operator<(const TuneKey &o) const {
    return std::tie(n, n_images, n_w, s_max, uniform, O, precision, w_mode, n_layers, log2_nvis) <
           std::tie(o.n, o.n_images, o.n_w, o.s_max, o.uniform, o.O, o.precision, o.w_mode,
                    o.n_layers, o.log2_nvis);
  }
};
std::mutex g_tune_mu;
struct TuneChoice {
  int tile, chunk, bin_aggregate;
};
std::map<TuneKey, TuneChoice> g_tune_cache;

}  // namespace

namespace wproj {
int set_error(int code, const char *msg) { return fail(code, "%s", msg); }

PhaseTimer::PhaseTimer(const wproj_kernels *kc, int ph, hipStream_t st)
    : k(const_cast<wproj_kernels *>(kc)), phase(ph), s(st) {
  if (!k->profiling) return;
  hipEvent_t start = take_event(k);
  stop = take_event(k);
  if (!start || !stop || hipEventRecord(start, s) != hipSuccess) {
    if (start) k->event_pool.push_back(start);
    if (stop) k->event_pool.push_back(stop);
    stop = nullptr;
    return;
  }
  k->prof[phase].push_back({start, stop});
}
PhaseTimer::~PhaseTimer() {
  if (stop) (void)hipEventRecord(stop, s);
}
}  // namespace wproj

extern "C" {

int wproj_profile(wproj_kernels *k, int enable) {
  g_err.clear();
  if (!k) return fail(WPROJ_EINVAL, "handle is NULL");
  k->profiling = enable != 0;
  return WPROJ_OK;
}

int wproj_profile_read(wproj_kernels *k, double *ms, int64_t *count) {
  g_err.clear();
  if (!k) return fail(WPROJ_EINVAL, "handle is NULL");
  for (int p = 0; p < WPROJ_N_PHASES; ++p) {
    double tot = 0.0;
    for (auto &pr : k->prof[p]) {
      HIP_TRY(hipEventSynchronize(pr.second));
      float t = 0.0f;
      HIP_TRY(hipEventElapsedTime(&t, pr.first, pr.second));
      tot += t;
    }
    if (ms) ms[p] = tot;
    if (count) count[p] = (int64_t)k->prof[p].size();
    for (auto &pr : k->prof[p]) {
      k->event_pool.push_back(pr.first);
      k->event_pool.push_back(pr.second);
    }
    k->prof[p].clear();
  }
  return WPROJ_OK;
}

const char *wproj_last_error(void) { return g_err.c_str(); }

int wproj_version(void) { return 100; }

int wproj_make_kernels(const wproj_params *params, void *stream, wproj_kernels **out) {
  g_err.clear();
  if (!out) return fail(WPROJ_EINVAL, "out is NULL");
  *out = nullptr;
  std::vector<int32_t> supp;
  int rc = validate(params, supp);
  if (rc != WPROJ_OK) return rc;
  hipStream_t s = (hipStream_t)stream;

  wproj_kernels *k = new (std::nothrow) wproj_kernels();
  if (!k) return fail(WPROJ_ENOMEM, "host allocation failed");
  struct Guard {
    wproj_kernels *k;
    ~Guard() { destroy(k); }
  } guard{k};

  k->params = *params;
  k->params.support_per_plane = nullptr;
  if (hipGetDevice(&k->device) != hipSuccess) return fail(WPROJ_EHIP, "hipGetDevice failed");
  const int n = params->n, n_w = params->n_wplanes, O = params->oversample;
  const int m = params->kernel_image_size;
  k->supp_host = supp;
  k->s_max = *std::max_element(supp.begin(), supp.end());
  k->uniform_support = std::all_of(supp.begin(), supp.end(), [&](int v) { return v == supp[0]; });
  k->tab_off_host.assign(n_w + 1, 0);
  for (int p = 0; p < n_w; ++p)
    k->tab_off_host[p + 1] = k->tab_off_host[p] + (int64_t)O * O * supp[p] * supp[p];
  k->n_taps = k->tab_off_host[n_w];
  k->tap_bytes = params->precision == WPROJ_F64 ? 16 : params->precision == WPROJ_F32 ? 8 : 4;
  {
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, k->device));
    k->n_cu = prop.multiProcessorCount;
    k->max_lds = prop.sharedMemPerBlock;
  }
  if (params->tile) {
    k->tile = params->tile;
    if (params->algorithm == WPROJ_ALGO_TILED && tile_shape(k, k->tile).lds_bytes + 256 > k->max_lds)
      return fail(WPROJ_EUNSUPPORTED, "tile %d with support %d needs %zu bytes of LDS per wavefront",
                  k->tile, k->s_max, tile_shape(k, k->tile).lds_bytes);
  } else {
    k->tile = 16;
  }
  if (params->chunk) k->chunk = params->chunk;
  k->bin_aggregate = params->bin_aggregate;
  k->stable_bins = params->stable_bins;

  Geometry &G = k->geo;
  G.n = n;
  G.O = O;
  G.n_w = n_w;
  G.n_images = params->n_images;
  G.log2_O = -1;
  for (int b = 0; b < 9; ++b)
    if ((1 << b) == O) G.log2_O = b;
  G.w_mode = params->w_mode;
  G.n_layers = G.w_mode == WPROJ_W_STACK && params->n_wlayers > 1 ? params->n_wlayers : 1;
  G.n_grids = params->n_images * G.n_layers;
  G.fov = (double)n * params->cell_rad;
  G.cell = params->cell_rad;
  G.w_max = params->w_max;
  G.layer_w = G.w_mode == WPROJ_W_STACK ? (2.0 * params->w_max) / (double)G.n_layers : 0.0;
  G.dw = 0.0;
  if (n_w > 1 && G.w_mode == WPROJ_W_LINEAR) G.dw = (2.0 * params->w_max) / (double)(n_w - 1);
  if (n_w > 1 && G.w_mode == WPROJ_W_FOLD) G.dw = params->w_max / (double)(n_w - 1);
  if (n_w > 1 && G.w_mode == WPROJ_W_STACK) G.dw = G.layer_w / (double)(n_w - 1);
  k->plane_in_key = plane_in_key_for(k, k->tile);  // needs the number of grids

  if (hipMalloc(&k->d_supp, sizeof(int32_t) * n_w) != hipSuccess ||
      hipMalloc(&k->d_tab_off, sizeof(int64_t) * (n_w + 1)) != hipSuccess ||
      hipMalloc(&k->d_tab, (size_t)(k->n_taps + kTabPad) * k->tap_bytes) != hipSuccess ||
      hipMalloc(&k->d_kappa, sizeof(double) * n) != hipSuccess ||
      hipMalloc(&k->d_taper, sizeof(double) * m) != hipSuccess)
    return fail(WPROJ_ENOMEM, "device allocation of kernel tables (%lld taps) failed",
                (long long)k->n_taps);
  // the padding past the last sub-kernel is read (never used) by whole-wavefront tap loads
  HIP_TRY(hipMemsetAsync((char *)k->d_tab + (size_t)k->n_taps * k->tap_bytes, 0,
                         (size_t)kTabPad * k->tap_bytes, s));
  G.supp = k->d_supp;
  G.tab_off = k->d_tab_off;
  HIP_TRY(hipMemcpyAsync(k->d_supp, supp.data(), sizeof(int32_t) * n_w, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(k->d_tab_off, k->tab_off_host.data(), sizeof(int64_t) * (n_w + 1),
                         hipMemcpyHostToDevice, s));

  // taper and correction
  std::vector<double> coef = prolate_legendre(M_PI * params->support / 2.0);
  TempBuffers tmp;
  HIP_TRY(hipMalloc(&tmp.p[0], sizeof(double) * coef.size()));
  HIP_TRY(hipMemcpyAsync(tmp.p[0], coef.data(), sizeof(double) * coef.size(),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(launch_taper((const double *)tmp.p[0], (int)coef.size(), m, n, k->d_taper, k->d_kappa, s));

  // tables, a batch of planes at a time
  const int so_max = k->s_max * O;
  const int64_t per_plane = 16 * ((int64_t)m * m + (int64_t)m * so_max + (int64_t)so_max * so_max);
  int batch = (int)std::max<int64_t>(1, std::min<int64_t>(n_w, (int64_t)(512ll << 20) / per_plane));
  HIP_TRY(hipMalloc(&tmp.p[1], (size_t)batch * m * m * 16));
  HIP_TRY(hipMalloc(&tmp.p[2], (size_t)batch * m * so_max * 16));
  HIP_TRY(hipMalloc(&tmp.p[3], (size_t)batch * so_max * so_max * 16));
  for (int p0 = 0; p0 < n_w; p0 += batch) {
    const int np = std::min(batch, n_w - p0);
    // w-stacking tables are those of the residual planes, linear over [-D/2, D/2]
    if (G.w_mode == WPROJ_W_STACK)
      HIP_TRY(launch_screen(k->d_taper, m, G.fov, G.layer_w / 2.0, G.dw, n_w, WPROJ_W_LINEAR, p0, np,
                            (double2 *)tmp.p[1], s));
    else
      HIP_TRY(launch_screen(k->d_taper, m, G.fov, G.w_max, G.dw, n_w, G.w_mode, p0, np,
                            (double2 *)tmp.p[1], s));
    HIP_TRY(launch_table_dft((const double2 *)tmp.p[1], m, O, k->d_supp, p0, np, so_max,
                             (double2 *)tmp.p[2], (double2 *)tmp.p[3], s));
    HIP_TRY(launch_normalise((const double2 *)tmp.p[3], so_max, O, k->d_supp, k->d_tab_off, p0, np,
                             params->precision, k->d_tab, s));
  }

  // pair-ordered copy for the fixed-support FP32 gridder
  if (params->precision != WPROJ_F64 && k->uniform_support && k->s_max >= kMinFixedSupport &&
      k->s_max <= kMaxFixedSupport) {
    k->pair_stride = pair_table_stride(k->s_max);
    const int64_t n_sub = (int64_t)n_w * O * O;
    if (hipMalloc(&k->d_tab_pair, (size_t)(n_sub * k->pair_stride) * k->tap_bytes) != hipSuccess)
      return fail(WPROJ_ENOMEM, "device allocation of the pair-ordered table failed");
    HIP_TRY(launch_pair_table(k, s));
  }

  // FFT plans (batched over images, in place, unnormalised)
  std::call_once(g_fft_once, [] { g_fft_setup = rocfft_setup(); });
  if (g_fft_setup != rocfft_status_success) return fail(WPROJ_EFFT, "rocfft_setup failed");
  const size_t lengths[2] = {(size_t)n, (size_t)n};
  const rocfft_precision fp =
      params->precision == WPROJ_F64 ? rocfft_precision_double : rocfft_precision_single;
  // one transform per grid: n_images of them, n_images x layers with w-stacking
  if (rocfft_plan_create(&k->fft_inv, rocfft_placement_inplace,
                         rocfft_transform_type_complex_inverse, fp, 2, lengths,
                         (size_t)G.n_grids, nullptr) != rocfft_status_success ||
      rocfft_plan_create(&k->fft_fwd, rocfft_placement_inplace,
                         rocfft_transform_type_complex_forward, fp, 2, lengths,
                         (size_t)G.n_grids, nullptr) != rocfft_status_success)
    return fail(WPROJ_EFFT, "rocfft_plan_create failed for %dx%d x %d", n, n, G.n_grids);
  size_t w1 = 0, w2 = 0;
  rocfft_plan_get_work_buffer_size(k->fft_inv, &w1);
  rocfft_plan_get_work_buffer_size(k->fft_fwd, &w2);
  k->fft_work_bytes = std::max(w1, w2);
  // grid -> image without w-stacking: the image is Re IFFT(G) = IFFT of G's Hermitian part,
  // a complex-to-real transform of the half spectrum (half the work of the complex one).
  // Out of place: the half spectrum in the workspace, the real output over the grid.
  if (params->w_mode != WPROJ_W_STACK) {
    if (rocfft_plan_create(&k->fft_c2r, rocfft_placement_notinplace, rocfft_transform_type_real_inverse, fp, 2,
                           lengths, (size_t)G.n_grids, nullptr) != rocfft_status_success)
      return fail(WPROJ_EFFT, "rocfft_plan_create (complex to real) failed for %dx%d x %d", n, n, G.n_grids);
    const size_t real = params->precision == WPROJ_F64 ? 8 : 4;
    k->herm_bytes = (size_t)G.n_grids * (size_t)n * (size_t)(n / 2 + 1) * 2 * real;
    rocfft_plan_get_work_buffer_size(k->fft_c2r, &k->c2r_work_bytes);
    k->fft_work_bytes = std::max(k->fft_work_bytes, (size_t)align_up((int64_t)k->herm_bytes) + k->c2r_work_bytes);
  }

  HIP_TRY(hipStreamSynchronize(s));
  guard.k = nullptr;
  *out = k;
  return WPROJ_OK;
}

int wproj_free_kernels(wproj_kernels *k) {
  g_err.clear();
  destroy(k);
  return WPROJ_OK;
}

int wproj_export(const wproj_kernels *k, int what, void *dst, int64_t dst_bytes, int64_t *needed,
                 void *stream) {
  g_err.clear();
  if (!k) return fail(WPROJ_EINVAL, "handle is NULL");
  const void *src = nullptr;
  int64_t bytes = 0;
  switch (what) {
    case WPROJ_EXPORT_TABLES:
      src = k->d_tab;
      bytes = k->n_taps * (int64_t)k->tap_bytes;
      break;
    case WPROJ_EXPORT_TABLE_OFFSETS:
      src = k->d_tab_off;
      bytes = 8 * (int64_t)(k->params.n_wplanes + 1);
      break;
    case WPROJ_EXPORT_KAPPA:
      src = k->d_kappa;
      bytes = 8 * (int64_t)k->params.n;
      break;
    case WPROJ_EXPORT_TAPER:
      src = k->d_taper;
      bytes = 8 * (int64_t)k->params.kernel_image_size;
      break;
    case WPROJ_EXPORT_SUPPORTS:
      src = k->d_supp;
      bytes = 4 * (int64_t)k->params.n_wplanes;
      break;
    default:
      return fail(WPROJ_EINVAL, "unknown export %d", what);
  }
  if (needed) *needed = bytes;
  if (!dst) return WPROJ_OK;
  if (dst_bytes < bytes) return fail(WPROJ_EINVAL, "dst holds %lld bytes, %lld needed",
                                     (long long)dst_bytes, (long long)bytes);
  HIP_TRY(hipMemcpyAsync(dst, src, (size_t)bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return WPROJ_OK;
}

int64_t wproj_workspace_size(const wproj_kernels *k, int64_t nvis) {
  g_err.clear();
  if (!k) return fail(WPROJ_EINVAL, "handle is NULL");
  if (nvis < 0) return fail(WPROJ_EINVAL, "nvis < 0");
  return workspace_bytes_for(k, nvis);
}

int wproj_grid(const wproj_kernels *k, int64_t nvis, const double *uvw, const void *vis,
               const void *weight, const int64_t *image_offsets, void *grid, double *weight_sum,
               int64_t *counters, void *workspace, int64_t workspace_bytes, void *stream) {
  g_err.clear();
  if (!k) return fail(WPROJ_EINVAL, "handle is NULL");
  if (nvis < 0) return fail(WPROJ_EINVAL, "nvis < 0");
  if (!grid) return fail(WPROJ_EINVAL, "grid is NULL");
  if (nvis > 0 && (!uvw || !vis || !weight)) return fail(WPROJ_EINVAL, "uvw, vis and weight are required");
  if (k->params.n_images > 1 && !image_offsets)
    return fail(WPROJ_EINVAL, "image_offsets is required when n_images > 1");
  int rc = check_device(k);
  if (rc != WPROJ_OK) return rc;
  const int64_t need = workspace_bytes_for(k, nvis);
  if (workspace_bytes < need || (need > 0 && !workspace))
    return fail(WPROJ_EWORKSPACE, "workspace of %lld bytes given, %lld needed",
                (long long)workspace_bytes, (long long)need);
  if (nvis == 0) return WPROJ_OK;
  hipStream_t s = (hipStream_t)stream;
  if (k->params.algorithm == WPROJ_ALGO_PLAIN) {
    PhaseTimer pt(k, WPROJ_PHASE_PLAIN, s);
    HIP_TRY(launch_plain_grid(k, nvis, uvw, vis, weight, image_offsets, grid, weight_sum, counters, s));
    return WPROJ_OK;
  }
  if (nvis > 0xfffffffell)
    return fail(WPROJ_EINVAL, "the tiled gridder takes at most 2^32 - 2 visibilities per call");
  if (k->n_taps > (int64_t)kTapMask)
    return fail(WPROJ_EUNSUPPORTED, "kernel tables of %lld taps exceed the tiled gridder's 2^26",
                (long long)k->n_taps);
  const BinShape B = bin_shape(k);
  if (B.n_keys >= max_keys(k))
    return fail(WPROJ_EUNSUPPORTED, "%lld bins (images x tiles) exceed the tiled gridder's 31-bit keys",
                (long long)B.n_keys);
  BinWorkspace W;
  carve(k, nvis, (char *)workspace, W);
  {
    PhaseTimer pt(k, WPROJ_PHASE_BIN, s);
    HIP_TRY(launch_bin(k, B, nvis, uvw, vis, weight, image_offsets, weight_sum, counters, W, s));
  }
  {
    PhaseTimer pt(k, WPROJ_PHASE_GRID, s);
    HIP_TRY(launch_tiled_grid(k, B, W, grid, s));
  }
  {
    PhaseTimer pt(k, WPROJ_PHASE_REDUCE, s);
    HIP_TRY(launch_tile_reduce(k, B, W, grid, s));
  }
  return WPROJ_OK;
}

int wproj_tuning(const wproj_kernels *k, int32_t *tile, int32_t *chunk, int32_t *bin_aggregate) {
  g_err.clear();
  if (!k) return fail(WPROJ_EINVAL, "handle is NULL");
  if (tile) *tile = k->tile;
  if (chunk) *chunk = k->chunk;
  if (bin_aggregate) *bin_aggregate = k->bin_aggregate;
  return WPROJ_OK;
}

int wproj_autotune(wproj_kernels *k, int64_t nvis, const double *uvw, const void *vis,
                   const void *weight, const int64_t *image_offsets, void *scratch_grid,
                   void *workspace, int64_t workspace_bytes, void *stream) {
  g_err.clear();
  if (!k) return fail(WPROJ_EINVAL, "handle is NULL");
  if (k->params.algorithm != WPROJ_ALGO_TILED)
    return fail(WPROJ_EUNSUPPORTED, "autotuning applies to the tiled gridder only");
  int lg = 0;
  while (lg < 62 && (1ll << (lg + 1)) <= std::max<int64_t>(nvis, 1)) ++lg;
  const TuneKey key{k->params.n, k->params.n_images, k->params.n_wplanes, k->s_max,
                    k->uniform_support ? 1 : 0, k->params.oversample, k->params.precision,
                    k->params.w_mode, k->geo.n_layers, lg};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      k->tile = it->second.tile;
      k->chunk = it->second.chunk;
      k->bin_aggregate = it->second.bin_aggregate;
      k->plane_in_key = plane_in_key_for(k, k->tile);
      return WPROJ_OK;
    }
  }
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  struct EvGuard {
    hipEvent_t a, b;
    ~EvGuard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } eg{e0, e1};
  const bool was_profiling = k->profiling;
  k->profiling = false;
  const TuneChoice start{k->tile, k->chunk, k->bin_aggregate};
  auto set = [&](const TuneChoice &c) {
    k->tile = c.tile;
    k->chunk = c.chunk;
    k->bin_aggregate = c.bin_aggregate;
    k->plane_in_key = plane_in_key_for(k, c.tile);
  };
  // one warm-up and one timed call of a candidate; on failure the handle is restored
  auto time_one = [&](const TuneChoice &c, float &ms) -> int {
    set(c);
    int rc = wproj_grid(k, nvis, uvw, vis, weight, image_offsets, scratch_grid, nullptr, nullptr,
                        workspace, workspace_bytes, stream);
    if (rc == WPROJ_OK) {
      if (hipEventRecord(e0, s) != hipSuccess) rc = fail(WPROJ_EHIP, "hipEventRecord failed");
      if (rc == WPROJ_OK)
        rc = wproj_grid(k, nvis, uvw, vis, weight, image_offsets, scratch_grid, nullptr, nullptr,
                        workspace, workspace_bytes, stream);
      if (rc == WPROJ_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = fail(WPROJ_EHIP, "event timing failed");
    }
    if (rc != WPROJ_OK) {
      set(start);
      k->profiling = was_profiling;
    }
    return rc;
  };
  // tile and work-item length with per-wavefront counting, then the block-aggregated
  // counting at the best of those
  float best = -1.0f;
  TuneChoice pick = start;
  for (int tile : kTuneTiles) {
    if (tile_shape(k, tile).lds_bytes + 256 > k->max_lds) continue;
    for (int chunk : kTuneChunks) {
      float ms = 0.0f;
      const int rc = time_one({tile, chunk, 0}, ms);
      if (rc != WPROJ_OK) return rc;
      if (best < 0.0f || ms < best) {
        best = ms;
        pick = {tile, chunk, 0};
      }
    }
  }
  {
    float ms = 0.0f;
    const int rc = time_one({pick.tile, pick.chunk, 1}, ms);
    if (rc != WPROJ_OK) return rc;
    if (ms < best) pick.bin_aggregate = 1;
  }
  set(pick);
  k->profiling = was_profiling;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[key] = pick;
  return WPROJ_OK;
}

int wproj_degrid(const wproj_kernels *k, int64_t nvis, const double *uvw, const void *model_grid,
                 const int64_t *image_offsets, void *vis_out, void *workspace,
                 int64_t workspace_bytes, void *stream) {
  g_err.clear();
  if (!k) return fail(WPROJ_EINVAL, "handle is NULL");
  if (nvis < 0) return fail(WPROJ_EINVAL, "nvis < 0");
  if (nvis > 0 && (!uvw || !model_grid || !vis_out))
    return fail(WPROJ_EINVAL, "uvw, model_grid and vis_out are required");
  if (k->params.n_images > 1 && !image_offsets)
    return fail(WPROJ_EINVAL, "image_offsets is required when n_images > 1");
  int rc = check_device(k);
  if (rc != WPROJ_OK) return rc;
  const int64_t need = workspace_bytes_for(k, nvis);
  if (workspace_bytes < need || (need > 0 && !workspace))
    return fail(WPROJ_EWORKSPACE, "workspace of %lld bytes given, %lld needed",
                (long long)workspace_bytes, (long long)need);
  if (nvis == 0) return WPROJ_OK;
  hipStream_t s = (hipStream_t)stream;
  if (k->params.algorithm == WPROJ_ALGO_PLAIN) {
    PhaseTimer pt(k, WPROJ_PHASE_DEGRID, s);
    HIP_TRY(launch_plain_degrid(k, nvis, uvw, model_grid, image_offsets, vis_out, s));
    return WPROJ_OK;
  }
  if (nvis > 0xfffffffell)
    return fail(WPROJ_EINVAL, "the tiled degridder takes at most 2^32 - 2 visibilities per call");
  if (k->n_taps > (int64_t)kTapMask)
    return fail(WPROJ_EUNSUPPORTED, "kernel tables of %lld taps exceed the tiled degridder's 2^26",
                (long long)k->n_taps);
  BinShape B = bin_shape(k);
  if (B.n_keys >= max_keys(k))
    return fail(WPROJ_EUNSUPPORTED, "%lld bins (images x tiles) exceed the tiled degridder's 31-bit keys",
                (long long)B.n_keys);
  BinWorkspace W;
  carve(k, nvis, (char *)workspace, W);
  // records binned for the degridder's own tile layout: the gridder's pitch for the
  // one-tap-per-lane kernel, an odd pitch for the row-per-lane kernel
  if (!tap_lane_degrid(k, B)) B.pitch = degrid_pitch(k, B.tile);
  {
    PhaseTimer pt(k, WPROJ_PHASE_BIN, s);
    HIP_TRY(launch_bin(k, B, nvis, uvw, nullptr, nullptr, image_offsets, nullptr, nullptr, W, s));
  }
  PhaseTimer pt(k, WPROJ_PHASE_DEGRID, s);
  HIP_TRY(launch_tiled_degrid(k, B, W, model_grid, vis_out, nvis, s));
  return WPROJ_OK;
}

int wproj_image(const wproj_kernels *k, int direction, void *grid, void *image,
                const double *weight_sum, void *workspace, int64_t workspace_bytes, void *stream) {
  g_err.clear();
  if (!k) return fail(WPROJ_EINVAL, "handle is NULL");
  if (!grid || !image) return fail(WPROJ_EINVAL, "grid and image are required");
  if (direction == WPROJ_GRID_TO_IMAGE && !weight_sum)
    return fail(WPROJ_EINVAL, "weight_sum is required for GRID_TO_IMAGE");
  if (direction < WPROJ_GRID_TO_IMAGE || direction > WPROJ_GRID_TO_IMAGE_RAW)
    return fail(WPROJ_EINVAL, "unknown direction %d", direction);
  int rc = check_device(k);
  if (rc != WPROJ_OK) return rc;
  if (workspace_bytes < (int64_t)k->fft_work_bytes || (k->fft_work_bytes > 0 && !workspace))
    return fail(WPROJ_EWORKSPACE, "workspace of %lld bytes given, %lld needed",
                (long long)workspace_bytes, (long long)k->fft_work_bytes);
  hipStream_t s = (hipStream_t)stream;
  rocfft_execution_info info = nullptr;
  if (rocfft_execution_info_create(&info) != rocfft_status_success)
    return fail(WPROJ_EFFT, "rocfft_execution_info_create failed");
  struct InfoGuard {
    rocfft_execution_info i;
    ~InfoGuard() { rocfft_execution_info_destroy(i); }
  } ig{info};
  rocfft_execution_info_set_stream(info, s);
  if (k->fft_work_bytes > 0) rocfft_execution_info_set_work_buffer(info, workspace, k->fft_work_bytes);
  void *buf[1] = {grid};
  if (direction == WPROJ_IMAGE_TO_GRID) {
    {
      PhaseTimer pt(k, WPROJ_PHASE_CORRECT, s);
      HIP_TRY(launch_i2g_precorrect(k, image, grid, s));
    }
    PhaseTimer pt(k, WPROJ_PHASE_FFT, s);
    if (rocfft_execute(k->fft_fwd, buf, nullptr, info) != rocfft_status_success)
      return fail(WPROJ_EFFT, "rocfft_execute (forward) failed");
    return WPROJ_OK;
  }
  const double *wsum = direction == WPROJ_GRID_TO_IMAGE ? weight_sum : nullptr;
  if (k->fft_c2r) {
    // twice the Hermitian half spectrum into the workspace, its complex-to-real inverse
    // over the grid, then the correction (with the factor 1/2)
    char *half = (char *)workspace;
    {
      PhaseTimer pt(k, WPROJ_PHASE_FFT, s);
      HIP_TRY(launch_hermitian_half(k, grid, half, s));
      if (k->c2r_work_bytes > 0)
        rocfft_execution_info_set_work_buffer(info, half + align_up((int64_t)k->herm_bytes), k->c2r_work_bytes);
      void *in[1] = {half};
      void *outp[1] = {grid};
      if (rocfft_execute(k->fft_c2r, in, outp, info) != rocfft_status_success)
        return fail(WPROJ_EFFT, "rocfft_execute (complex to real) failed");
    }
    PhaseTimer pt(k, WPROJ_PHASE_CORRECT, s);
    HIP_TRY(launch_g2i_correct_real(k, grid, image, wsum, s));
    return WPROJ_OK;
  }
  {
    PhaseTimer pt(k, WPROJ_PHASE_FFT, s);
    if (rocfft_execute(k->fft_inv, buf, nullptr, info) != rocfft_status_success)
      return fail(WPROJ_EFFT, "rocfft_execute (inverse) failed");
  }
  PhaseTimer pt(k, WPROJ_PHASE_CORRECT, s);
  HIP_TRY(launch_g2i_correct(k, grid, image, wsum, s));
  return WPROJ_OK;
}

int wproj_check_weights(const wproj_kernels *k, const double *weight_sum, void *stream) {
  g_err.clear();
  if (!k) return fail(WPROJ_EINVAL, "handle is NULL");
  if (!weight_sum) return fail(WPROJ_EINVAL, "weight_sum is NULL");
  int rc = check_device(k);
  if (rc != WPROJ_OK) return rc;
  const int ni = k->params.n_images;
  std::vector<double> h(ni);
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  HIP_TRY(hipMemcpy(h.data(), weight_sum, sizeof(double) * ni, hipMemcpyDeviceToHost));
  for (int i = 0; i < ni; ++i)
    if (!(isfinite(h[i]) && h[i] >= 0.0))
      return fail(WPROJ_EINVAL, "weight_sum[%d] = %g is negative or not finite", i, h[i]);
  for (int i = 0; i < ni; ++i)
    if (h[i] == 0.0)
      return fail(WPROJ_EEMPTY, "image %d has no gridded weight (weight_sum 0): its image is all zeros", i);
  return WPROJ_OK;
}

}  // extern "C"

// A binning kept for repeated gridding / degridding of the same rows.
struct wproj_plan {
  const wproj_kernels *k;
  int64_t nvis;
  wproj::BinShape B;
  wproj::BinWorkspace W;
};

int wproj_plan_create(const wproj_kernels *k, int64_t nvis, const double *uvw, const void *weight,
                      const int64_t *image_offsets, double *weight_sum, int64_t *counters,
                      void *workspace, int64_t workspace_bytes, void *stream, wproj_plan **out) {
  g_err.clear();
  if (!out) return fail(WPROJ_EINVAL, "out is NULL");
  *out = nullptr;
  if (!k) return fail(WPROJ_EINVAL, "handle is NULL");
  if (nvis < 0) return fail(WPROJ_EINVAL, "nvis < 0");
  if (nvis > 0 && !uvw) return fail(WPROJ_EINVAL, "uvw is required");
  if (k->params.n_images > 1 && !image_offsets)
    return fail(WPROJ_EINVAL, "image_offsets is required when n_images > 1");
  if (k->params.algorithm != WPROJ_ALGO_TILED)
    return fail(WPROJ_EUNSUPPORTED, "plans are built by the binned (tiled) algorithm only");
  int rc = check_device(k);
  if (rc != WPROJ_OK) return rc;
  const int64_t need = workspace_bytes_for(k, nvis);
  if (workspace_bytes < need || (need > 0 && !workspace))
    return fail(WPROJ_EWORKSPACE, "workspace of %lld bytes given, %lld needed",
                (long long)workspace_bytes, (long long)need);
  if (nvis > 0xfffffffell) return fail(WPROJ_EINVAL, "a plan holds at most 2^32 - 2 visibilities");
  if (k->n_taps > (int64_t)kTapMask)
    return fail(WPROJ_EUNSUPPORTED, "kernel tables of %lld taps exceed the tiled path's 2^26",
                (long long)k->n_taps);
  auto *p = new (std::nothrow) wproj_plan;
  if (!p) return fail(WPROJ_ENOMEM, "plan allocation failed");
  p->k = k;
  p->nvis = nvis;
  p->B = bin_shape(k);
  if (p->B.n_keys >= max_keys(k)) {
    const long long n_keys = (long long)p->B.n_keys;
    delete p;
    return fail(WPROJ_EUNSUPPORTED, "%lld bins exceed the tiled path's 31-bit keys", n_keys);
  }
  carve(k, nvis, (char *)workspace, p->W);
  if (nvis > 0) {
    PhaseTimer pt(k, WPROJ_PHASE_BIN, (hipStream_t)stream);
    const hipError_t e = launch_bin(k, p->B, nvis, uvw, nullptr, weight, image_offsets, weight_sum,
                                    counters, p->W, (hipStream_t)stream);
    if (e != hipSuccess) {
      delete p;
      return fail(WPROJ_EHIP, "binning: %s", hipGetErrorString(e));
    }
  }
  *out = p;
  return WPROJ_OK;
}

int wproj_plan_free(wproj_plan *p) {
  g_err.clear();
  delete p;
  return WPROJ_OK;
}

int wproj_grid_planned(const wproj_plan *p, const void *vis, void *grid, void *stream) {
  g_err.clear();
  if (!p) return fail(WPROJ_EINVAL, "plan is NULL");
  if (!grid) return fail(WPROJ_EINVAL, "grid is NULL");
  if (p->nvis > 0 && !vis) return fail(WPROJ_EINVAL, "vis is required");
  int rc = check_device(p->k);
  if (rc != WPROJ_OK) return rc;
  if (p->nvis == 0) return WPROJ_OK;
  hipStream_t s = (hipStream_t)stream;
  {
    PhaseTimer pt(p->k, WPROJ_PHASE_GRID, s);
    HIP_TRY(launch_tiled_grid(p->k, p->B, p->W, grid, s, vis));
  }
  PhaseTimer pt(p->k, WPROJ_PHASE_REDUCE, s);
  HIP_TRY(launch_tile_reduce(p->k, p->B, p->W, grid, s));
  return WPROJ_OK;
}

int wproj_plan_rows(const wproj_plan *p, uint32_t *rows, void *stream) {
  g_err.clear();
  if (!p) return fail(WPROJ_EINVAL, "plan is NULL");
  if (p->nvis > 0 && !rows) return fail(WPROJ_EINVAL, "rows is NULL");
  int rc = check_device(p->k);
  if (rc != WPROJ_OK) return rc;
  if (p->nvis == 0) return WPROJ_OK;
  HIP_TRY(launch_plan_rows(p->k, p->B, p->W, p->nvis, rows, (hipStream_t)stream));
  return WPROJ_OK;
}

int wproj_degrid_planned(const wproj_plan *p, const void *model_grid, void *vis_out, void *stream) {
  g_err.clear();
  if (!p) return fail(WPROJ_EINVAL, "plan is NULL");
  if (p->nvis > 0 && (!model_grid || !vis_out)) return fail(WPROJ_EINVAL, "model_grid and vis_out are required");
  int rc = check_device(p->k);
  if (rc != WPROJ_OK) return rc;
  if (p->nvis == 0) return WPROJ_OK;
  PhaseTimer pt(p->k, WPROJ_PHASE_DEGRID, (hipStream_t)stream);
  HIP_TRY(launch_tiled_degrid(p->k, p->B, p->W, model_grid, vis_out, p->nvis, (hipStream_t)stream));
  return WPROJ_OK;
}

int wproj_footprints(const wproj_kernels *k, int64_t nvis, const double *uvw, const void *weight,
                     int32_t *out, void *stream) {
  g_err.clear();
  if (!k) return fail(WPROJ_EINVAL, "handle is NULL");
  if (nvis < 0) return fail(WPROJ_EINVAL, "nvis < 0");
  if (nvis > 0 && (!uvw || !out)) return fail(WPROJ_EINVAL, "uvw or out is NULL");
  HIP_TRY(launch_footprints(k, nvis, uvw, weight, out, (hipStream_t)stream));
  return WPROJ_OK;
}

// ---------------------------------------------------------------------------
// Rows regrouped by baseline (Section 2.2, Eqs. 5 and 6) and row gathers.
// ---------------------------------------------------------------------------
namespace {
constexpr int32_t kMaxRegroupAnt = 255;  // n_ant (n_ant + 1)/2 + 1 counters fit in LDS

int check_regroup_args(int64_t n_rows, int32_t n_ant) {
  if (n_rows < 0 || n_rows > 0x7fffffffll) return fail(WPROJ_EINVAL, "n_rows must be in [0, 2^31 - 1]");
  if (n_ant < 1) return fail(WPROJ_EINVAL, "n_ant must be >= 1");
  if (n_ant > kMaxRegroupAnt)
    return fail(WPROJ_EUNSUPPORTED, "n_ant = %d: the regroup keeps one counter per baseline in LDS (n_ant <= %d)",
                n_ant, kMaxRegroupAnt);
  return WPROJ_OK;
}
}  // namespace

int64_t wproj_regroup_workspace_size(int64_t n_rows, int32_t n_ant) {
  g_err.clear();
  const int rc = check_regroup_args(n_rows, n_ant);
  if (rc != WPROJ_OK) return rc;
  return regroup_workspace_bytes(regroup_shape(n_rows, n_ant));
}

int wproj_regroup_rows(int64_t n_rows, const int32_t *ant1, const int32_t *ant2, int32_t n_ant,
                       int64_t *perm, int64_t *start, int64_t *counts, void *workspace,
                       int64_t workspace_bytes, void *stream) {
  g_err.clear();
  const int rc = check_regroup_args(n_rows, n_ant);
  if (rc != WPROJ_OK) return rc;
  if (n_rows > 0 && (!ant1 || !ant2 || !perm)) return fail(WPROJ_EINVAL, "ant1, ant2 or perm is NULL");
  if (!start || !counts) return fail(WPROJ_EINVAL, "start or counts is NULL");
  const RegroupShape r = regroup_shape(n_rows, n_ant);
  const int64_t need = regroup_workspace_bytes(r);
  if (!workspace || workspace_bytes < need)
    return fail(WPROJ_EWORKSPACE, "workspace of %lld bytes given, %lld needed", (long long)workspace_bytes,
                (long long)need);
  HIP_TRY(launch_regroup(r, n_rows, ant1, ant2, n_ant, perm, start, counts, workspace,
                         (hipStream_t)stream));
  return WPROJ_OK;
}

int wproj_regroup_channels(int64_t n_rows, int32_t n_ant, int32_t n_chan, const int64_t *perm,
                           const int64_t *start, const int64_t *counts, int64_t *vis_perm, void *stream) {
  g_err.clear();
  const int rc = check_regroup_args(n_rows, n_ant);
  if (rc != WPROJ_OK) return rc;
  if (n_chan < 1) return fail(WPROJ_EINVAL, "n_chan must be >= 1");
  if (n_rows > 0 && (!perm || !start || !counts || !vis_perm))
    return fail(WPROJ_EINVAL, "perm, start, counts or vis_perm is NULL");
  if (n_rows == 0) return WPROJ_OK;
  const int64_t n_keys = (int64_t)n_ant * (n_ant + 1) / 2 + 1;
  HIP_TRY(launch_channel_order(n_keys, n_chan, perm, start, counts, vis_perm, (hipStream_t)stream));
  return WPROJ_OK;
}

int wproj_gather_rows(int64_t n_rows, int64_t row_bytes, const int64_t *perm, int64_t n_src_rows,
                      const void *src, void *dst, int64_t *bad, void *stream) {
  g_err.clear();
  if (n_rows < 0 || n_src_rows < 0) return fail(WPROJ_EINVAL, "n_rows and n_src_rows must be >= 0");
  if (row_bytes <= 0 || (row_bytes & 3)) return fail(WPROJ_EINVAL, "row_bytes must be a positive multiple of 4");
  if (n_rows > 0 && (!perm || !src || !dst)) return fail(WPROJ_EINVAL, "perm, src or dst is NULL");
  HIP_TRY(launch_gather_rows(n_rows, row_bytes, perm, n_src_rows, src, dst, bad, (hipStream_t)stream));
  return WPROJ_OK;
}

