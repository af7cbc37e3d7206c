// Internal declarations of the gfx950 w-projection library: the handle, the
// per-visibility footprint rule shared by every kernel, and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <rocfft/rocfft.h>
#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

#include "wproj.h"

namespace wproj {

// Kernel tables stored at reduced precision: one FP16 pair per tap.
struct alignas(4) half2c {
  _Float16 re, im;
};

// Geometry every kernel needs, passed by value.
// Zero taps allocated past the end of a kernel table: a wavefront loading one sub-kernel
// of up to 64 taps with lane t at tap t stays inside the allocation for the last one.
constexpr int64_t kTabPad = 64;

struct Geometry {
  int32_t n;        // grid side
  int32_t O;        // oversampling
  int32_t n_w;      // w-planes
  int32_t n_images;
  int32_t log2_O;   // log2(O) when O is a power of two, else -1
  int32_t w_mode;   // wproj_w_mode: linear over [-w_max, w_max], a Hermitian fold, or stacking
  int32_t n_layers; // w-stacking layers L (1 otherwise)
  int32_t n_grids;  // n_images * n_layers
  double fov;       // n * cell_rad
  double w_max;
  double dw;        // plane spacing: 2 w_max / (n_w - 1) (linear), w_max / (n_w - 1) (fold),
                    // layer_w / (n_w - 1) (stacking: residual planes), 0 for a single plane
                    // or the square-root spacing
  double layer_w;   // w-stacking layer width 2 w_max / L (0 otherwise)
  double cell;      // cell_rad (image-plane phase of the stacking layers)
  const int32_t *supp;     // device [n_w] full support per plane
  const int64_t *tab_off;  // device [n_w + 1] first tap of each plane
};

enum VisClass { kGridded = 0, kFlagged = 1, kBadWeight = 2, kDropped = 3 };
// wproj_footprints only: gridded at the Hermitian mirror (-u, -v, -w)
constexpr int kGriddedFolded = 4;

struct Footprint {
  int x0, y0, ou, ov, p;
  bool fold;  // taken at (-u, -v, -w): the visibility enters conjugated
  int layer;  // w-stacking layer (0 otherwise); the row's grid is img * n_layers + layer
};

// floor(a / b) for b > 0
__device__ inline int floor_div32(int a, int b) {
  int q = a / b;
  if (q * b > a) q -= 1;
  return q;
}

// Nearest w-plane, ties rounding up, clamped to [0, n_w - 1].  With a Hermitian fold w
// is the folded coordinate |w|: planes p dw (WPROJ_W_FOLD), or w_max (p / (n_w - 1))^2,
// nearest in sqrt(|w| / w_max) (WPROJ_W_FOLD_SQRT).
__device__ inline int plane_of(const Geometry &G, double w) {
#pragma clang fp contract(off)
  if (G.n_w == 1) return 0;
  double t;
  if (G.w_mode == WPROJ_W_LINEAR)
    t = floor((w + G.w_max) / G.dw + 0.5);
  else if (G.w_mode == WPROJ_W_STACK)  // w is the residual from the layer centre
    t = floor((w + G.layer_w / 2.0) / G.dw + 0.5);
  else if (G.w_mode == WPROJ_W_FOLD)
    t = floor(w / G.dw + 0.5);
  else
    t = floor(sqrt(w / G.w_max) * (double)(G.n_w - 1) + 0.5);
  if (!(t >= 0.0)) return 0;
  if (t > (double)(G.n_w - 1)) return G.n_w - 1;
  return (int)t;
}

// w-stacking: the layer of w, floor((w + w_max) / D) clamped to [0, L - 1], and w's
// residual from that layer's centre -w_max + (layer + 1/2) D, each step rounded in FP64.
__device__ inline int layer_residual(const Geometry &G, double &w) {
#pragma clang fp contract(off)
  double t = floor((w + G.w_max) / G.layer_w);
  int layer = 0;
  if (t >= 0.0) layer = t > (double)(G.n_layers - 1) ? G.n_layers - 1 : (int)t;
  w = w - (-G.w_max + ((double)layer + 0.5) * G.layer_w);
  return layer;
}

// One axis of the footprint: g = coord FoV + n/2 cells, q = floor(g O + 1/2) on the
// 1/O lattice, first cell x0 = floor((q - S O/2)/O) + 1, sub-kernel ou = x0 O - q + S O/2 - 1.
// Each product and sum rounds separately, so the integer outcome is a pure function of
// the float64 inputs.  Returns false when the S cells do not all lie on the grid.
// An on-grid footprint needs q in [S O/2 - O, (n - S) O + S O/2), inside (-O, (n + 1) O];
// q outside that interval is rejected in float64 (NaN included), so the integer steps run
// in 32 bits (n <= 32768 and O <= 256 keep (n + 1) O below 2^24).
__device__ inline bool axis_footprint(const Geometry &G, double coord, int S, int &x0, int &ou) {
#pragma clang fp contract(off)
  double g = coord * G.fov;
  g = g + (double)G.n / 2.0;
  double t = g * (double)G.O;
  double qd = floor(t + 0.5);
  if (!(qd > -(double)G.O && qd <= (double)(G.n + 1) * G.O)) return false;
  const int q = (int)qd;
  const int half = S * G.O / 2;
  // floor((q - half) / O): an arithmetic shift when O is a power of two
  const int d = q - half;
  const int a = (G.log2_O >= 0 ? (d >> G.log2_O) : floor_div32(d, G.O)) + 1;
  if (a < 0 || a + S > G.n) return false;
  x0 = a;
  ou = a * G.O - q + half - 1;
  return true;
}

// S_uniform > 0: every plane has that support (no table lookup).
template <typename WT>
__device__ inline int classify(const Geometry &G, const double *uvw, WT wt, Footprint &f,
                               int S_uniform = 0) {
  if (wt == WT(0)) return kFlagged;
  if (!(isfinite((double)wt) && wt > WT(0))) return kBadWeight;
  double u = uvw[0], v = uvw[1], w = uvw[2];
  if (!(isfinite(u) && isfinite(v) && isfinite(w))) return kDropped;
  // Hermitian fold: V(-u, -v, -w) = conj(V(u, v, w)) for a real sky, so a row with w < 0
  // is gridded as conj(V) at the mirrored point and the planes only cover w >= 0
  f.fold = (G.w_mode == WPROJ_W_FOLD || G.w_mode == WPROJ_W_FOLD_SQRT) && w < 0.0;
  if (f.fold) {
    u = -u;
    v = -v;
    w = -w;
  }
  f.layer = G.w_mode == WPROJ_W_STACK ? layer_residual(G, w) : 0;
  f.p = plane_of(G, w);
  const int S = S_uniform > 0 ? S_uniform : G.supp[f.p];
  if (!axis_footprint(G, u, S, f.x0, f.ou)) return kDropped;
  if (!axis_footprint(G, v, S, f.y0, f.ov)) return kDropped;
  return kGridded;
}

// Grid of a gridded row of image img: one grid per image, or per (image, layer) when
// w-stacking.
__device__ inline int grid_of(const Geometry &G, int img, const Footprint &f) {
  return img * G.n_layers + f.layer;
}

// |w| beyond w_max is clamped to the edge plane (or layer) and counted.
__device__ inline bool w_clamped(const Geometry &G, double w) {
  return (G.n_w > 1 || G.n_layers > 1) && fabs(w) > G.w_max;
}

// Image owning row j: the largest i with off[i] <= j, or -1 outside [off[0], off[n_images]).
__device__ inline int image_of(const int64_t *off, int n_images, int64_t j) {
  if (off == nullptr) return 0;
  if (j < off[0] || j >= off[n_images]) return -1;
  int lo = 0, hi = n_images - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= j)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

}  // namespace wproj

// The opaque handle.
struct wproj_kernels {
  wproj_params params;  // copy; support_per_plane is cleared
  int device = 0;
  wproj::Geometry geo{};
  std::vector<int32_t> supp_host;
  std::vector<int64_t> tab_off_host;
  int s_max = 0;
  bool uniform_support = true;
  int32_t *d_supp = nullptr;
  int64_t *d_tab_off = nullptr;
  void *d_tab = nullptr;  // double2 / float2 / half2c per tap
  int64_t n_taps = 0;
  // With FP32 arithmetic and a fixed support that has its own gridder kernel: the table
  // again, each pass of 64 taps of a sub-kernel stored as pairs (t, t + h), h = half the
  // pass rounded up, for the gridder's two-records-per-load fetch.
  void *d_tab_pair = nullptr;
  int64_t pair_stride = 0;  // entries per sub-kernel (S^2 rounded up to even)
  size_t tap_bytes = 0;
  double *d_kappa = nullptr;
  double *d_taper = nullptr;
  rocfft_plan fft_fwd = nullptr, fft_inv = nullptr;
  // grid -> image without w-stacking: complex-to-real inverse of the grid's Hermitian part
  // (herm_bytes of it at the start of the workspace, the plan's own work buffer after)
  rocfft_plan fft_c2r = nullptr;
  size_t herm_bytes = 0, c2r_work_bytes = 0;
  size_t fft_work_bytes = 0;
  int tile = 16;            // tiled gridder tile side
  bool plane_in_key = true; // bin by (tile, plane) rather than tile alone
  int chunk = 2048;         // max records per gridder work item
  int bin_aggregate = 0;    // binning's count aggregation (wproj_params::bin_aggregate)
  int stable_bins = 0;      // records keep input order inside a bin (wproj_params::stable_bins)
  int n_cu = 256;           // compute units of the device
  size_t max_lds = 65536;   // LDS bytes available to one workgroup
  // phase timing (wproj_profile): recorded (start, stop) event pairs per phase
  bool profiling = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof[WPROJ_N_PHASES];
  std::vector<hipEvent_t> event_pool;
};

namespace wproj {
// RAII marker: records a start event on construction and a stop event on destruction
// when the handle is profiling.
struct PhaseTimer {
  wproj_kernels *k;
  int phase;
  hipStream_t s;
  hipEvent_t stop = nullptr;
  PhaseTimer(const wproj_kernels *kc, int ph, hipStream_t st);
  ~PhaseTimer();
};
}  // namespace wproj

namespace wproj {

// Sets the calling thread's wproj_last_error() message and returns code.
int set_error(int code, const char *msg);

// ---- launchers (each returns hipSuccess or the first launch error) ----

// Table generation (FP64): taper/kappa evaluation from Legendre coefficients of psi_0.
hipError_t launch_taper(const double *d_coef, int n_coef, int m, int n, double *d_taper,
                        double *d_kappa, hipStream_t s);
// Screen for planes [p0, p0 + np): out[p - p0][j][i] complex128.
hipError_t launch_screen(const double *d_taper, int m, double fov, double w_max, double dw,
                         int n_w, int w_mode, int p0, int np, double2 *out, hipStream_t s);
// Row and column DFTs for planes [p0, p0 + np) into C[p - p0][ib][ia], stride so_max.
hipError_t launch_table_dft(const double2 *screen, int m, int O, const int32_t *d_supp, int p0,
                            int np, int so_max, double2 *tmp, double2 *C, hipStream_t s);
// Normalise each sub-kernel and store it in the handle's precision.
hipError_t launch_normalise(const double2 *C, int so_max, int O, const int32_t *d_supp,
                            const int64_t *d_tab_off, int p0, int np, int precision, void *tab,
                            hipStream_t s);

// Plain (no binning) gridder / degridder.
hipError_t launch_plain_grid(const wproj_kernels *k, int64_t nvis, const double *uvw,
                             const void *vis, const void *wt, const int64_t *img_off, void *grid,
                             double *wsum, int64_t *counters, hipStream_t s);
hipError_t launch_plain_degrid(const wproj_kernels *k, int64_t nvis, const double *uvw,
                               const void *grid, const int64_t *img_off, void *vis_out,
                               hipStream_t s);
// Per-visibility footprint and class (wproj_footprints).
hipError_t launch_footprints(const wproj_kernels *k, int64_t nvis, const double *uvw,
                             const void *wt, int32_t *out, hipStream_t s);

// Image-plane kernels around the FFTs.
hipError_t launch_g2i_correct(const wproj_kernels *k, const void *fgrid, void *image,
                              const double *wsum, hipStream_t s);
hipError_t launch_i2g_precorrect(const wproj_kernels *k, const void *image, void *grid,
                                 hipStream_t s);
// H = G + conj(G(-k)) on the half spectrum kx in [0, n/2] (twice the Hermitian part of G,
// whose inverse transform is twice Re IFFT(G)), for the complex-to-real transform.
hipError_t launch_hermitian_half(const wproj_kernels *k, const void *grid, void *half, hipStream_t s);
// The correction applied to the real output R of that transform (R = 2 Re IFFT(G)).
hipError_t launch_g2i_correct_real(const wproj_kernels *k, const void *real, void *image,
                                   const double *wsum, hipStream_t s);

}  // namespace wproj
