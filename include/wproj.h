/*
 * wproj.h -- C ABI of the MI355X (gfx950) w-projection imaging library.
 *
 * W-projection wide-field imaging (the method whose parallel implementation
 * Lao et al. 2019 study; they cite Cornwell, Golap & Bhatnagar 2008 for the
 * mathematics, Sections 1-2): each visibility is convolved onto one uv-grid
 * with an oversampled, w-dependent kernel (a prolate spheroidal taper times
 * the w phase screen, Fourier transformed), the grid is inverse-FFT'd and the
 * taper is divided out of the image.  Degridding is the adjoint.
 *
 * Grids in WPROJ_W_STACK mode: a handle with L = n_wlayers layers has n_images L grids,
 * [n_images][L][n][n]; every "grid" argument below is that array (images are still
 * [n_images][n][n]).
 *
 * Conventions shared by every entry point
 *   - Pointers are DEVICE pointers owned by the caller unless marked (host).
 *     Nothing returned by the library aliases caller memory.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls only enqueue
 *     work on it and return; nothing synchronises except wproj_make_kernels.
 *   - Every entry point returns a wproj_status; on a non-OK status
 *     wproj_last_error() gives a message for the calling thread and no work
 *     has been enqueued.  No C++ exception crosses the ABI.
 *   - Grids are [n_images][n][n] complex, row-major [y][x], interleaved
 *     (re, im): complex128 for WPROJ_F64, complex64 otherwise.  Images are
 *     [n_images][n][n] real (float64 for WPROJ_F64, float32 otherwise).
 *     Cell X of a grid holds u = (X - n/2)/FoV, pixel x holds
 *     l = (x - n/2) cell_rad, FoV = n cell_rad.
 *   - uvw is always float64 [nvis][3], in wavelengths.
 *   - Per visibility: weight 0 = flagged (skipped); a negative or non-finite
 *     weight is skipped and counted; non-finite uvw or a kernel footprint
 *     that leaves the grid drops the visibility (counted); with more than one
 *     w-plane, |w| > w_max is clamped to the edge plane (counted).
 *   - A handle is immutable after wproj_make_kernels and may be used from
 *     several streams at once; the caller's workspace must not be shared by
 *     calls that run concurrently.
 */
#ifndef WPROJ_H
#define WPROJ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  WPROJ_F64 = 0,          /* FP64 tables, FP64 visibilities, FP64 grid */
  WPROJ_F32 = 1,          /* FP32 tables, FP32 visibilities/weights, FP32 grid */
  WPROJ_F32_F16TABLE = 2  /* as WPROJ_F32 but kernel tables stored in FP16 */
} wproj_precision;

typedef enum {
  WPROJ_ALGO_TILED = 0, /* device binning by (image, uv-tile, w-plane) + LDS-tile gridder */
  WPROJ_ALGO_PLAIN = 1  /* one pass, global atomics per tap, no binning (comparison path) */
} wproj_algorithm;

typedef enum {
  WPROJ_W_LINEAR = 0,    /* N_w planes at w_p = -w_max + p 2 w_max/(N_w - 1) */
  WPROJ_W_FOLD = 1,      /* Hermitian fold: a row with w < 0 is gridded as conj(V) at
                            (-u, -v, -w); planes at w_p = p w_max/(N_w - 1) cover [0, w_max] */
  WPROJ_W_FOLD_SQRT = 2, /* Hermitian fold with planes w_p = w_max (p/(N_w - 1))^2, evenly
                            spaced in sqrt(w); nearest plane in sqrt(|w|/w_max) (N_w - 1) */
  WPROJ_W_STACK = 3      /* w-stacking hybrid: n_wlayers layers of width D = 2 w_max/n_wlayers
                            centred at w_l = -w_max + (l + 1/2) D, layer = floor((w + w_max)/D)
                            clamped; each layer has its own grid and a row is gridded with the
                            kernel of its residual w - w_l, N_w planes linear over [-D/2, D/2] */
} wproj_w_mode;

typedef enum {
  WPROJ_OK = 0,
  WPROJ_EINVAL = -1,       /* invalid argument or parameter block */
  WPROJ_ENOMEM = -2,       /* device allocation failed (wproj_make_kernels only) */
  WPROJ_EHIP = -3,         /* a HIP runtime call failed */
  WPROJ_EUNSUPPORTED = -4, /* valid but not supported by this build (message says why) */
  WPROJ_EWORKSPACE = -5,   /* workspace smaller than wproj_workspace_size() */
  WPROJ_EFFT = -6,         /* rocFFT plan creation or execution failed */
  WPROJ_EEMPTY = -7        /* an image has no gridded weight (sum of weights 0): wproj_check_weights */
} wproj_status;

/*
 * Parameter block.  The paper's "primary argument settings" are the image
 * size, cell size, number of w-planes and full support of the convolution
 * kernel (Section 3.1); precision is its single/double comparison
 * (Sections 3.2, 4).  Oversampling, the w range and the kernel-generation
 * sample count are the standard w-projection parameters the paper leaves
 * implicit.
 */
typedef struct {
  int32_t n;                /* grid/image side N: even, 2..32768 */
  int32_t n_wplanes;        /* N_w >= 1: planes as w_mode sets them; one plane = w 0 */
  double cell_rad;          /* image cell (radians) > 0, with n * cell_rad < 2 */
  double w_max;             /* >= 0 (> 0 when N_w > 1), wavelengths */
  int32_t support;          /* S: full support in cells of the w = 0 kernel, 1..32; also sets the
                               taper bandwidth c = pi S / 2 */
  int32_t oversample;       /* O: 1..256; S_p * O must be even */
  const int32_t *support_per_plane; /* (host, nullable) [N_w] full supports S_p, 1..32;
                               NULL = S for every plane.  Read during wproj_make_kernels only. */
  int32_t kernel_image_size; /* m: image-domain samples per axis for kernel generation; even, 2..4096 */
  int32_t precision;        /* wproj_precision */
  int32_t n_images;         /* >= 1: independent images gridded in one call (e.g. channels) */
  int32_t algorithm;        /* wproj_algorithm */
  int32_t tile;             /* tiled gridder tile side: 0 = default (16), else 16, 32 or 64 */
  int32_t chunk;            /* tiled gridder work-item length in records: 0 = default (2048),
                               else 256..65536 */
  int32_t w_mode;           /* wproj_w_mode (0 = linear planes over [-w_max, w_max]).  The fold
                               halves the planes (and tables) needed for a given plane spacing:
                               with a real sky V(-u,-v,-w) = conj(V(u,v,w)), so Re of the image
                               is unchanged.  The paper's own imager uses planes over the full
                               w range (Section 3.1: 23 w-planes); the fold is a variant. */
  int32_t accumulate_runs;  /* 0 or 1.  1: while consecutive binned visibilities of a work item
                               share a footprint origin, each lane of the gridder keeps its grid
                               cell in a register and writes it to the LDS tile only when the
                               origin changes (the paper's CUDA gridder buffers a baseline's
                               successive timestamps in a register the same way, Section 2.2).
                               Same arithmetic in the same order, so the grid is unchanged; it
                               pays when visibilities come baseline by baseline, channel by
                               channel, in time order (wproj_regroup_channels).  Used by the
                               FP32 fixed-support (3..16) gridders, ignored elsewhere. */
  int32_t n_wlayers;        /* WPROJ_W_STACK: layers L, 1..4096 (0 = 1); other modes: 0 or 1.
                               Grids then hold n_images L planes [image][layer][n][n]; the
                               image combines an image's layers (w-stacking, one of the
                               wide-field methods the paper's introduction lists, Section 1). */
  int32_t bin_aggregate;    /* 0 or 1: how binning counts visibilities per bin (the same bins
                               and results either way).  0: the first lane of each run of
                               equal bins in a wavefront adds the run with one global atomic,
                               which suits rows in measurement-set order (a row's channels
                               share bins).  1: blocks of 2048 visibilities first add their
                               counts in an LDS hash table, then take one global atomic per
                               distinct bin, which suits rows whose equal bins lie hundreds of
                               rows apart (one channel per row in time order: the same
                               baseline recurs every few hundred rows, in the same bin for
                               minutes).  wproj_autotune times both. */
  int32_t stable_bins;      /* 0 or 1: the order of records inside a bin (the same bins either
                               way).  0: each visibility's place comes from the count atomics,
                               so it follows their timing and FP32 grids of two runs agree to
                               rounding.  1: a stable counting sort, as the paper's regroup
                               keeps a baseline's rows in time order (Eq. 5 and 6): the bin
                               keys are sorted by a least-significant-digit radix sort (8 bits
                               a pass) and the records gathered in sorted order, so a bin keeps
                               its visibilities in input order and every grid is reproducible
                               bit for bit.  Slower (the sort reads and writes 8 bytes per
                               visibility and pass) and 16 more workspace bytes per
                               visibility.  Tiled algorithm only (ignored by the plain
                               one). */
  int32_t reserved[1];      /* must be zero */
} wproj_params;

typedef struct wproj_kernels wproj_kernels; /* opaque handle */
typedef struct wproj_plan wproj_plan;       /* opaque: a kept binning (see wproj_plan_create) */

/*
 * Build the oversampled w-kernel tables on the device, in FP64, then store
 * them in the handle's precision.  For plane p with support S_p:
 *   screen  s_p(l, m) = psi(l/l_max) psi(m/l_max) exp(+2 pi i w_p (sqrt(1-l^2-m^2) - 1)),
 *           sampled at the m x m cell-centred points nu_i = (2i + 1 - m)/m, l = nu l_max;
 *   table   C_p(a, b) = sum_{i,j} s_p(l_i, m_j) exp(-2 pi i (a l_i + b m_j)/(O FoV)),
 *           its Fourier transform at uv offsets (a/O, b/O) cells, a, b in (-S_p O/2, S_p O/2];
 *   layout  [ov][ou][kv][ku] with tap (kv, ku) of sub-kernel (ov, ou) = C_p(b0 + kv O, a0 + ku O),
 *           a0 = ou + 1 - S_p O/2; each sub-kernel is divided by its complex tap sum.
 * psi is the zeroth-order prolate spheroidal function with c = pi S/2, and
 * the grid correction kappa(x) = 1/psi((x - n/2)/(n/2)) (0 on the edge pixel
 * x = 0) is stored alongside.  Launches on `stream`, synchronises it, and
 * returns the handle in *out (host pointer).  Errors: WPROJ_EINVAL for an
 * invalid block, WPROJ_ENOMEM, WPROJ_EHIP, WPROJ_EFFT.
 */
int wproj_make_kernels(const wproj_params *params, void *stream, wproj_kernels **out);

/* Release a handle (NULL is accepted).  The caller must have finished all work using it. */
int wproj_free_kernels(wproj_kernels *k);

/* What wproj_export copies. */
typedef enum {
  WPROJ_EXPORT_TABLES = 0,      /* tables as stored: c128, c64 or (half re, half im) per tap */
  WPROJ_EXPORT_TABLE_OFFSETS = 1, /* int64 [N_w + 1]: first tap of each plane */
  WPROJ_EXPORT_KAPPA = 2,       /* float64 [n]: grid-correction factors kappa(x) */
  WPROJ_EXPORT_TAPER = 3,       /* float64 [m]: psi(nu_i) at the kernel-generation samples */
  WPROJ_EXPORT_SUPPORTS = 4     /* int32 [N_w]: S_p */
} wproj_export_what;

/*
 * Copy a table held by the handle into device memory dst (bytes available
 * in dst_bytes), enqueued on stream.  With dst == NULL only *needed (host) is
 * written.  Errors: WPROJ_EINVAL (unknown `what`, dst_bytes too small).
 */
int wproj_export(const wproj_kernels *k, int what, void *dst, int64_t dst_bytes, int64_t *needed,
                 void *stream);

/*
 * Bytes of device workspace the grid/degrid/image calls need for nvis
 * visibilities (>= 0), or a negative wproj_status.  The workspace is scratch:
 * its contents on entry are ignored and on return undefined.
 */
int64_t wproj_workspace_size(const wproj_kernels *k, int64_t nvis);

/*
 * Gridding (convolutional resampling onto the uv-grid; the "gridding" step
 * the paper parallelises, Section 2):
 *   grid[i][y0+kv][x0+ku] += W_j V_j T_p[ov][ou][kv][ku]   for every valid visibility j of image i,
 *   weight_sum[i] += W_j                                   over the same visibilities,
 * with p the nearest w-plane (ties round up) and, per axis, g = u FoV + n/2,
 * q = floor(g O + 1/2), x0 = floor((q - S_p O/2)/O) + 1, ou = x0 O - q + S_p O/2 - 1.
 *   uvw           float64 [nvis][3]
 *   vis           [nvis] complex128 (WPROJ_F64) or complex64
 *   weight        [nvis] float64 (WPROJ_F64) or float32
 *   image_offsets int64 [n_images + 1], ascending; rows [off[i], off[i+1]) belong to
 *                 image i, rows outside [off[0], off[n_images]) are ignored.  May be
 *                 NULL when n_images == 1 (all rows belong to image 0).
 *   grid          accumulated into (the caller zeroes it first)
 *   weight_sum    float64 [n_images], accumulated into (nullable)
 *   counters      int64 [3], accumulated into (nullable): dropped (non-finite uvw or
 *                 off-grid), w clamped, bad weight
 * Errors: WPROJ_EINVAL (NULL required pointer, nvis < 0), WPROJ_EWORKSPACE.
 */
int wproj_grid(const wproj_kernels *k, int64_t nvis, const double *uvw, const void *vis,
               const void *weight, const int64_t *image_offsets, void *grid, double *weight_sum,
               int64_t *counters, void *workspace, int64_t workspace_bytes, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): wproj_grid with its workspace taken
 * from a fixed scratch array that the library holds in each GPU's memory
 * (wproj_noalloc_scratch_bytes() = 256 MiB per GPU, from library load until the process
 * ends) instead of from the caller.  Arguments, results, counters and errors are those
 * of wproj_grid; nothing is allocated and no allocating library routine is called.
 * A call whose wproj_workspace_size(k, nvis) exceeds the scratch size is refused with
 * WPROJ_EWORKSPACE before anything is enqueued (roughly: a 2048^2 grid leaves room for
 * a few million visibilities).  All calls on one GPU share that GPU's scratch array and
 * the array keeps the last call's contents (each call clears what it relies on): calls
 * that overlap in time on one GPU, from any stream or thread, race and must not be
 * issued.
 */
int wproj_grid_noalloc(const wproj_kernels *k, int64_t nvis, const double *uvw, const void *vis,
                       const void *weight, const int64_t *image_offsets, void *grid,
                       double *weight_sum, int64_t *counters, void *stream);
/* Bytes of the per-GPU scratch array behind wproj_grid_noalloc. */
int64_t wproj_noalloc_scratch_bytes(void);

/*
 * Degridding, the adjoint of gridding (prediction of model visibilities from a model
 * grid; the paper names gridding and degridding together as the steps earlier GPU and
 * Cell imagers accelerated, Section 2, and its imager's CLEAN cycles predict from the
 * model this way).  With WPROJ_ALGO_TILED the visibilities are binned as for gridding and each tile of the
 * model grid is read once into LDS; WPROJ_ALGO_PLAIN gathers straight from HBM:
 *   vis_out[j] = sum_{kv,ku} conj(T_p[ov][ou][kv][ku]) model_grid[i][y0+kv][x0+ku]
 * with the same footprint rule; rows with non-finite uvw or off-grid footprints, and
 * rows outside every image range, are set to 0.  vis_out is overwritten
 * ([nvis] complex128 for WPROJ_F64, else complex64).  No weights are applied.
 * Errors: WPROJ_EINVAL, WPROJ_EWORKSPACE.
 */
int wproj_degrid(const wproj_kernels *k, int64_t nvis, const double *uvw, const void *model_grid,
                 const int64_t *image_offsets, void *vis_out, void *workspace,
                 int64_t workspace_bytes, void *stream);

typedef enum {
  WPROJ_GRID_TO_IMAGE = 0,     /* image = Re(IDFT(grid)) kappa(x) kappa(y) / weight_sum */
  WPROJ_IMAGE_TO_GRID = 1,     /* grid  = DFT(kappa(x) kappa(y) image) (model prediction) */
  WPROJ_GRID_TO_IMAGE_RAW = 2  /* image = Re(IDFT(grid)) kappa(x) kappa(y) (no weight_sum) */
} wproj_direction;

/*
 * Transforms between grid and image; the DFTs are centred and unnormalised:
 *   IDFT(G)[y][x] = sum_{Y,X} G[Y][X] exp(+2 pi i ((X - n/2)(x - n/2) + (Y - n/2)(y - n/2))/n)
 *   DFT(I)[Y][X]  = sum_{y,x} I[y][x] exp(-2 pi i ((X - n/2)(x - n/2) + (Y - n/2)(y - n/2))/n)
 * (the paper's final IFFT, Sections 2.1-2.2; rocFFT does the 2D transforms).
 * GRID_TO_IMAGE*: grid's contents are destroyed (without w-stacking the image's real
 * transform takes the grid's Hermitian half spectrum, formed in the workspace, and
 * writes its output over the grid; with w-stacking each layer is transformed in place)
 * and image is written.  IMAGE_TO_GRID: image is read and grid is overwritten.
 * weight_sum (float64 [n_images], device) is read only by GRID_TO_IMAGE; an image
 * whose sum is 0 is written as zeros (see wproj_check_weights).
 * Errors: WPROJ_EINVAL, WPROJ_EWORKSPACE, WPROJ_EFFT.
 */
int wproj_image(const wproj_kernels *k, int direction, void *grid, void *image,
                const double *weight_sum, void *workspace, int64_t workspace_bytes, void *stream);

/*
 * The empty-image status.  GRID_TO_IMAGE divides by weight_sum[i] (natural weighting;
 * the paper does not spell out the normalisation of its images, Section 3.1 compares
 * them by noise and peak flux).  An image that received no gridded visibility has
 * weight_sum[i] == 0; wproj_image cannot report that, because it only enqueues work
 * and the sums live on the device, so it writes that image as all zeros (0 instead of
 * a division by 0) and returns WPROJ_OK.  wproj_check_weights waits for `stream`,
 * reads the n_images sums (device, float64) and returns WPROJ_EEMPTY, naming the first
 * such image in wproj_last_error(), if any sum is 0, WPROJ_EINVAL if any is negative
 * or not finite, else WPROJ_OK.  Synchronises `stream`.  Errors: WPROJ_EINVAL, WPROJ_EHIP.
 */
int wproj_check_weights(const wproj_kernels *k, const double *weight_sum, void *stream);

/*
 * Choose the tiled gridder's tile side (16, 32 or 64 cells, each where one wavefront's
 * tile copy with its halo fits in a workgroup's LDS) and work-item length (1024 ..
 * 16384 binned records) for this handle by timing each candidate on the caller's data
 * (one warm-up and one timed wproj_grid per candidate, HIP events on `stream`), then, at
 * the fastest of those, binning with counts aggregated per block (bin_aggregate = 1)
 * against per-wavefront runs (0), and keep the fastest configuration in the handle.  The choice is also cached per problem shape (grid size,
 * images, planes, supports, oversampling, precision, visibility count rounded to a
 * power of two) for the life of the process, and later calls on a handle of the same
 * shape reuse it without timing.  Arguments are those of wproj_grid; scratch_grid
 * ([n_images][n][n], device) is written with garbage.  Synchronises `stream`.  Mutates
 * the handle: no other call may use it concurrently.  The paper attributes the
 * flattening of its scaling curves to workload imbalance between threads and nodes
 * (Sections 3.2, 4); the work-item length is the knob that trades that imbalance
 * against per-item overhead (work items are handed out largest first, so the imbalance
 * left is mostly that of the last, smallest items).  Errors: as wproj_grid; WPROJ_EUNSUPPORTED for a handle
 * built with WPROJ_ALGO_PLAIN.
 */
int wproj_autotune(wproj_kernels *k, int64_t nvis, const double *uvw, const void *vis,
                   const void *weight, const int64_t *image_offsets, void *scratch_grid,
                   void *workspace, int64_t workspace_bytes, void *stream);

/* The tiled gridder configuration in use: *tile (cells), *chunk (records) and
 * *bin_aggregate (wproj_params::bin_aggregate); host pointers, each nullable. */
int wproj_tuning(const wproj_kernels *k, int32_t *tile, int32_t *chunk, int32_t *bin_aggregate);

/* Phases timed by wproj_profile. */
typedef enum {
  WPROJ_PHASE_BIN = 0,      /* key/count, scan, scatter, work list (tiled gridding) */
  WPROJ_PHASE_GRID = 1,     /* the LDS-tile gridder kernel (work-queue reset + gridder) */
  WPROJ_PHASE_PLAIN = 2,    /* the plain gridder kernel */
  WPROJ_PHASE_FFT = 3,      /* rocFFT execution inside wproj_image */
  WPROJ_PHASE_CORRECT = 4,  /* grid-correction / pre-correction kernel of wproj_image */
  WPROJ_PHASE_DEGRID = 5,   /* the degridder kernel */
  WPROJ_PHASE_REDUCE = 6,   /* adding the tile gridder's partial tiles into the grid */
  WPROJ_N_PHASES = 7
} wproj_phase;

/*
 * Per-phase timing with HIP events (the paper times its phases, e.g. "gridding" and
 * "data loading", as averaged wall-clock, Section 3.2).  enable != 0 starts recording an
 * event pair around every phase the handle's calls enqueue, on the call's stream;
 * enable == 0 stops.  wproj_profile_read waits for the recorded events, writes the
 * summed milliseconds and the number of recorded intervals of each phase into
 * ms[WPROJ_N_PHASES] and count[WPROJ_N_PHASES] (host, either nullable), and clears the
 * record.  Profiling mutates the handle: do not use it while other threads use the
 * same handle.  Errors: WPROJ_EINVAL, WPROJ_EHIP.
 */
int wproj_profile(wproj_kernels *k, int enable);
int wproj_profile_read(wproj_kernels *k, double *ms, int64_t *count);

/*
 * Plans: the binning of one set of rows, kept for repeated gridding and degridding of
 * those rows (e.g. the major cycles of an imaging loop, where uvw and weights stay fixed
 * and the visibilities change).  wproj_plan_create bins nvis rows as wproj_grid does
 * (same footprints, same drops and counters; weight_sum and counters are accumulated
 * into here, nullable) and keeps, for every gridded row, its footprint, sub-kernel,
 * weight and row index in the caller's workspace.  Then
 *   wproj_grid_planned(plan, vis, grid)       == wproj_grid with the plan's uvw, weights
 *                                                and image offsets, accumulated into grid
 *                                                (no weight_sum or counters);
 *   wproj_degrid_planned(plan, model, vis_out) == wproj_degrid of the rows the plan grids;
 *                                                rows it does not grid (flagged, bad weight,
 *                                                dropped) get 0.
 * The workspace (at least wproj_workspace_size(k, nvis) bytes) belongs to the plan until
 * wproj_plan_free: it must stay allocated and must not be passed to other calls.  Calls
 * on one plan must not run concurrently (they share the workspace's scratch part); the
 * handle must outlive the plan, and its tuning at creation time is kept by the plan.
 * vis / vis_out: [nvis] complex of the handle's precision; grids as for wproj_grid.
 * Only the binned (tiled) algorithm builds plans (WPROJ_EUNSUPPORTED otherwise).
 * Errors: WPROJ_EINVAL, WPROJ_EUNSUPPORTED, WPROJ_EWORKSPACE, WPROJ_ENOMEM, WPROJ_EHIP.
 */
int wproj_plan_create(const wproj_kernels *k, int64_t nvis, const double *uvw, const void *weight,
                      const int64_t *image_offsets, double *weight_sum, int64_t *counters,
                      void *workspace, int64_t workspace_bytes, void *stream, wproj_plan **out);
int wproj_plan_free(wproj_plan *plan);
int wproj_grid_planned(const wproj_plan *plan, const void *vis, void *grid, void *stream);
int wproj_degrid_planned(const wproj_plan *plan, const void *model_grid, void *vis_out, void *stream);

/*
 * The binned order a plan keeps (the counting sort that Eq. 5 and 6 describe for the
 * paper's baseline regroup, keyed here by bin): rows[i] (uint32, device, nvis entries) =
 * the row whose record is i-th in bin order, for i below the number of rows the plan
 * grids; the remaining entries are set to 0xffffffff.  Bins run in key order (image,
 * tile row, tile column, then w-plane when planes are binned apart), each bin's rows
 * contiguous; with stable_bins a bin's rows are in increasing order, otherwise in the
 * order the count atomics handed out.  Errors: WPROJ_EINVAL, WPROJ_EHIP.
 */
int wproj_plan_rows(const wproj_plan *plan, uint32_t *rows, void *stream);

/*
 * The loss of the differentiable forward model (model image -> predicted visibilities by
 * wproj_image(IMAGE_TO_GRID) then wproj_degrid) and its gradient, in one pass.  The paper
 * defines no loss (its imager grids and images); this is the weighted least-squares
 * misfit of the visibilities:
 *   chi2[0] = sum_j w_j |o_j - p_j|^2                (FP64; overwritten, not accumulated)
 *   grad_j  = -2 w_j (o_j - p_j)                    (= d chi2/d Re p_j + i d chi2/d Im p_j)
 * precision: wproj_precision of the arrays (WPROJ_F64: complex double and double weights;
 * otherwise complex float and float weights).  vis_obs o, pred p: [nvis] complex,
 * device; weight w: [nvis] real, device, nullable (all 1); chi2: one double, device;
 * grad: [nvis] complex, device, nullable (not written).  The sum runs in a fixed order,
 * so chi2 is reproducible bit for bit.  workspace: device, at least
 * wproj_chi2_workspace_size() bytes (per-block partial sums); calls that share a
 * workspace must not overlap.  Errors: WPROJ_EINVAL, WPROJ_EWORKSPACE, WPROJ_EHIP.
 */
int64_t wproj_chi2_workspace_size(void);
int wproj_chi2(int precision, int64_t nvis, const void *vis_obs, const void *pred, const void *weight,
               double *chi2, void *grad, void *workspace, int64_t workspace_bytes, void *stream);

/*
 * Per-visibility footprint: the uvw -> grid step every gridding and degridding call
 * takes, exported.  For visibility j, out[6 j .. 6 j + 5] (int32, device) =
 * {x0, y0, ou, ov, p, class}: first footprint cell (x0, y0), sub-kernel (ou, ov), w-plane
 * p, and class 0 = gridded, 1 = flagged (weight 0), 2 = weight negative or non-finite,
 * 3 = dropped (non-finite uvw or footprint off the grid), 4 = gridded at the Hermitian
 * mirror (-u, -v, -w) with conj(V) (w < 0 under a folding w_mode; the footprint given is
 * that of the mirrored point).  With
 *   g = u FoV + n/2, q = floor(g O + 1/2), x0 = floor((q - S O/2)/O) + 1,
 *   ou = x0 O - q + S O/2 - 1  (the same for v, y0, ov),
 *   p = nearest plane of w, ties up, clamped to [0, n_wplanes - 1]  (S = S_p; see w_mode),
 * every product and sum rounded separately in float64.  Rows of class != 0 carry -1
 * for x0 .. p.  weight: float64 for WPROJ_F64, float32 otherwise, nullable (all 1).
 * Errors: WPROJ_EINVAL, WPROJ_EHIP.
 */
int wproj_footprints(const wproj_kernels *k, int64_t nvis, const double *uvw, const void *weight,
                     int32_t *out, void *stream);

/*
 * Rows regrouped by baseline (Section 2.2, Eqs. 5 and 6): the preprocessing of the
 * paper's GPU imager, which groups the rows of a measurement set (one timestamp of one
 * baseline, all channels; stored in time order) by baseline, keeping time order inside
 * each baseline.  For rows j = 0 .. n_rows - 1 with 0-based antenna IDs ant1[j], ant2[j]:
 *   I_B(j)    = (-S^2 + 2 S n_ant + S)/2 + |ant1[j] - ant2[j]|, S = min(ant1[j], ant2[j])
 *               (Eq. 5), which numbers every antenna pair, autocorrelations included,
 *               0 .. n_b - 1 with n_b = n_ant (n_ant + 1)/2; a row with an ID outside
 *               [0, n_ant) gets I_B = n_b and goes last;
 *   counts[b] = number of rows with I_B = b (the array C), b = 0 .. n_b;
 *   start[b]  = sum of counts[b'] over b' < b (Eq. 6), b = 0 .. n_b;
 *   perm[k]   = the row placed at position k: rows in increasing I_B, each baseline's
 *               rows in their original order (a stable counting sort).
 * ant1, ant2: int32 [n_rows]; perm: int64 [n_rows]; start, counts: int64 [n_b + 1] (all
 * device).  n_rows in [0, 2^31 - 1]; n_ant in [1, 255] (WPROJ_EUNSUPPORTED above: one
 * counter per baseline is kept in LDS).  The workspace (device, caller-owned, scratch)
 * must hold wproj_regroup_workspace_size(n_rows, n_ant) bytes.
 * Errors: WPROJ_EINVAL, WPROJ_EUNSUPPORTED, WPROJ_EWORKSPACE, WPROJ_EHIP.
 */
int64_t wproj_regroup_workspace_size(int64_t n_rows, int32_t n_ant);
int wproj_regroup_rows(int64_t n_rows, const int32_t *ant1, const int32_t *ant2, int32_t n_ant,
                       int64_t *perm, int64_t *start, int64_t *counts, void *workspace,
                       int64_t workspace_bytes, void *stream);

/*
 * Visibility order for rows regrouped by baseline, channel by channel (the order in which
 * the paper's CUDA gridder walks a baseline's samples, successive timestamps of one
 * baseline and channel one after another, Section 2.2).  Inputs are the outputs of
 * wproj_regroup_rows for n_rows rows of n_chan channels each (source visibility index
 * row n_chan + c).  Baseline b's count_b rows become n_chan runs of count_b visibilities,
 * one run per channel, each in time order:
 *   vis_perm[start[b] n_chan + c counts[b] + t] = perm[start[b] + t] n_chan + c,
 * t = 0 .. counts[b] - 1, c = 0 .. n_chan - 1.  vis_perm: int64 [n_rows n_chan] (device);
 * apply it with wproj_gather_rows to per-visibility arrays (uvw rows of 24 bytes,
 * visibilities, weights).  n_rows and n_ant as for wproj_regroup_rows; n_chan >= 1.
 * Errors: WPROJ_EINVAL, WPROJ_EUNSUPPORTED, WPROJ_EHIP.
 */
int wproj_regroup_channels(int64_t n_rows, int32_t n_ant, int32_t n_chan, const int64_t *perm,
                           const int64_t *start, const int64_t *counts, int64_t *vis_perm,
                           void *stream);

/*
 * Row gather, e.g. to apply a regroup permutation to the rows of uvw, visibilities or
 * weights: dst row k = src row perm[k], k = 0 .. n_rows - 1, rows of row_bytes bytes (a
 * positive multiple of 4; src and dst 4-byte aligned and not overlapping).  perm: int64
 * [n_rows] (device).  An entry outside [0, n_src_rows) leaves its destination row
 * unchanged and adds 1 to *bad (device int64, nullable, accumulated into).
 * Errors: WPROJ_EINVAL, WPROJ_EHIP.
 */
int wproj_gather_rows(int64_t n_rows, int64_t row_bytes, const int64_t *perm, int64_t n_src_rows,
                      const void *src, void *dst, int64_t *bad, void *stream);

/*
 * Measurement aid, not part of imaging: the device's LDS data rate for the access
 * shape of the tile gridder's private tiles (each lane its own 8-byte word, 64
 * consecutive words per instruction, 8 independent accesses in flight per lane, every
 * CU filled with workgroups).  mode 0 = 64-bit reads, 1 = 64-bit writes, 2 = 64-bit
 * read, add and write of the same word.  Runs the streaming kernel once untimed and
 * once between HIP events on `stream`, waits, and writes the aggregate bytes per
 * second (and, if ms is not NULL, the kernel time in ms) to host memory.  rounds
 * (1..2^20) sets the work: each lane moves rounds x 64 bytes (x 2 in mode 2).
 * Allocates and frees a small output buffer.  Errors: WPROJ_EINVAL, WPROJ_ENOMEM,
 * WPROJ_EHIP.
 */
int wproj_measure_lds(int mode, int32_t rounds, double *bytes_per_second, double *ms, void *stream);

/*
 * Measures the rate at which the vector-memory path returns data from L1 to the
 * registers, for buffer loads of `width` bytes per lane (4, 8 or 16: the tap fetches of
 * the gridder and degridder load 8 or 16 bytes per lane).  Every CU runs resident
 * workgroups of 256 lanes that stream loads with 8 in flight per lane from a 16 KiB
 * window that stays in L1; the kernel is timed with HIP events on `stream` after one
 * warm-up launch (synchronous: the call waits for the timing).  bytes_per_second
 * receives bytes delivered to registers / elapsed time (all CUs together); ms (nullable)
 * the launch time.  rounds in [1, 2^20] sets the length of the launch.  Allocates and
 * frees a 16 KiB window (zeroed) and a small output buffer.  Errors: WPROJ_EINVAL,
 * WPROJ_ENOMEM, WPROJ_EHIP.
 */
int wproj_measure_vmem(int width, int32_t rounds, double *bytes_per_second, double *ms, void *stream);

/* Message describing the last non-OK status returned on the calling thread ("" if none). */
const char *wproj_last_error(void);

/* Library version: major * 10000 + minor * 100 + patch. */
int wproj_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WPROJ_H */
