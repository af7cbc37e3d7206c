/*
 * Plain FP64 w-projection gridding and degridding in C -- TEST INFRASTRUCTURE ONLY.
 *
 * Part of the oracle: the tests use it for full-size parity (the numpy oracle
 * would take minutes there) and the benchmark times it as the CPU baseline.
 * It is checked against the numpy oracle (oracle/wproj_ref.py) by the CPU
 * tests.  The product library never links or calls it.
 *
 * Per visibility (the standard w-projection gridding step the paper applies,
 * Sections 1-2; the paper parallelises exactly this loop with OpenMP threads
 * over rows, each thread gridding into its own sub-grid that is summed at the
 * end, Section 2.1):
 *   plane     p  = clamp(floor((w + w_max)/dw + 1/2)), dw = 2 w_max/(N_w - 1)
 *   per axis  g  = u FoV + N/2, q = floor(g O + 1/2),
 *             x0 = floor((q - S_p O/2)/O) + 1, ou = x0 O - q + S_p O/2 - 1
 *   drop      if a coordinate is non-finite or x0 < 0 or x0 + S_p > N
 *   grid[y0+kv][x0+ku] += W V T_p[ov][ou][kv][ku]
 * With a Hermitian fold (w_mode 1: planes p dw, dw = w_max/(N_w - 1); w_mode 2: planes
 * w_max (p/(N_w - 1))^2, nearest in sqrt|w|) a row with w < 0 is taken at (-u, -v, -w)
 * with conj(V), and degridding returns the conjugate for it.  With w-stacking (w_mode 3,
 * n_layers layers of width D = 2 w_max/n_layers centred at w_l = -w_max + (l + 1/2) D,
 * layer = clamp(floor((w + w_max)/D))) a row goes to its layer's grid (grid index
 * image n_layers + layer) with the plane of its residual w - w_l, planes linear over
 * [-D/2, D/2] (dw = D/(N_w - 1)).
 * Kernel tables come in as built by the numpy oracle: complex128 interleaved,
 * plane p at tap offset tab_off[p], laid out [ov][ou][kv][ku].
 *
 * Built with -ffp-contract=off so each multiply and add rounds on its own,
 * matching numpy's evaluation of the same expressions.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int n, n_w, O, w_mode, n_layers;
  double fov, w_max, dw, layer_w;
  const int32_t *supp;
} plan_t;

static int64_t floor_div(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b) != 0 && ((a < 0) != (b < 0))) q -= 1;
  return q;
}

/* w is the folded (non-negative) coordinate when w_mode != 0 */
static int plane_of(const plan_t *P, double w) {
  if (P->n_w == 1) return 0;
  double t;
  if (P->w_mode == 0)
    t = floor((w + P->w_max) / P->dw + 0.5);
  else if (P->w_mode == 3) /* w is the residual from the layer centre */
    t = floor((w + P->layer_w / 2.0) / P->dw + 0.5);
  else if (P->w_mode == 1)
    t = floor(w / P->dw + 0.5);
  else
    t = floor(sqrt(w / P->w_max) * (double)(P->n_w - 1) + 0.5);
  if (!(t >= 0.0)) return 0; /* also catches NaN */
  if (t > (double)(P->n_w - 1)) return P->n_w - 1;
  return (int)t;
}

/* 1 when the S-cell footprint along this axis is on the grid. */
static int axis_fp(const plan_t *P, double coord, int S, int *x0, int *ou) {
  double g = coord * P->fov;
  g = g + (double)P->n / 2.0;
  double t = g * (double)P->O;
  double qd = floor(t + 0.5);
  if (!isfinite(qd) || fabs(qd) >= 1e15) return 0;
  int64_t q = (int64_t)qd;
  int64_t half = (int64_t)S * P->O / 2;
  int64_t a = floor_div(q - half, P->O) + 1;
  int64_t o = a * P->O - q + half - 1;
  if (a < 0 || a + S > P->n) return 0;
  *x0 = (int)a;
  *ou = (int)o;
  return 1;
}

/* w-stacking layer of w, clamped to [0, n_layers - 1] */
static int layer_of(const plan_t *P, double w) {
  if (P->n_layers == 1) return 0;
  double t = floor((w + P->w_max) / P->layer_w);
  if (!(t >= 0.0)) return 0;
  if (t > (double)(P->n_layers - 1)) return P->n_layers - 1;
  return (int)t;
}

/* 0: gridded; 1: flagged (W == 0); 2: bad weight; 3: dropped.  *fold = 1 when the row
   is taken at (-u, -v, -w); *layer = its w-stacking layer (0 otherwise). */
static int classify(const plan_t *P, const double *uvw, double wt, int *p, int *x0, int *y0,
                    int *ou, int *ov, int *fold, int *layer) {
  *fold = 0;
  *layer = 0;
  if (wt == 0.0) return 1;
  if (!(isfinite(wt) && wt > 0.0)) return 2;
  if (!(isfinite(uvw[0]) && isfinite(uvw[1]) && isfinite(uvw[2]))) return 3;
  double u = uvw[0], v = uvw[1], w = uvw[2];
  if ((P->w_mode == 1 || P->w_mode == 2) && w < 0.0) {
    u = -u;
    v = -v;
    w = -w;
    *fold = 1;
  }
  if (P->w_mode == 3) {
    *layer = layer_of(P, w);
    w = w - (-P->w_max + ((double)*layer + 0.5) * P->layer_w);
  }
  *p = plane_of(P, w);
  int S = P->supp[*p];
  if (!axis_fp(P, u, S, x0, ou)) return 3;
  if (!axis_fp(P, v, S, y0, ov)) return 3;
  return 0;
}

static void init_plan(plan_t *P, int n, double cell, int n_w, double w_max, int w_mode,
                      int n_layers, const int32_t *supp, int O) {
  P->n = n;
  P->n_w = n_w;
  P->O = O;
  P->w_mode = w_mode;
  P->n_layers = w_mode == 3 ? n_layers : 1;
  P->fov = (double)n * cell;
  P->w_max = w_max;
  P->layer_w = w_mode == 3 ? (2.0 * w_max) / (double)P->n_layers : 0.0;
  if (n_w == 1)
    P->dw = 0.0;
  else if (w_mode == 0)
    P->dw = (2.0 * w_max) / (double)(n_w - 1);
  else if (w_mode == 3)
    P->dw = P->layer_w / (double)(n_w - 1);
  else
    P->dw = w_max / (double)(n_w - 1);
  P->supp = supp;
}

/* Rows [s, e) into the image's grids G (n_layers of them, layer fastest).  Only rows whose
   layer is congruent to rem modulo mod are gridded and counted (mod = 1: all rows). */
static void grid_range(const plan_t *P, const double *tab, const int64_t *tab_off, int64_t s,
                       int64_t e, const double *uvw, const double *vis, const double *wt,
                       double *G0, double *sumw, int64_t *cnt, int mod, int rem) {
  const int n = P->n, O = P->O;
  for (int64_t j = s; j < e; ++j) {
    int p, x0, y0, ou, ov, fold, layer;
    int c = classify(P, uvw + 3 * j, wt[j], &p, &x0, &y0, &ou, &ov, &fold, &layer);
    if (layer % mod != rem) continue;
    if (c == 2) cnt[2] += 1;
    if (c == 3) cnt[0] += 1;
    if (c != 0) continue;
    if ((P->n_w > 1 || P->n_layers > 1) && fabs(uvw[3 * j + 2]) > P->w_max) cnt[1] += 1;
    double *G = G0 + 2 * (int64_t)layer * n * n;
    const int S = P->supp[p];
    const double ar = wt[j] * vis[2 * j];
    const double ai = wt[j] * (fold ? -vis[2 * j + 1] : vis[2 * j + 1]);
    const double *T = tab + 2 * (tab_off[p] + ((int64_t)ov * O + ou) * S * S);
    for (int kv = 0; kv < S; ++kv) {
      double *row = G + 2 * ((int64_t)(y0 + kv) * n + x0);
      for (int ku = 0; ku < S; ++ku) {
        const double tr = T[2 * (kv * S + ku)], ti = T[2 * (kv * S + ku) + 1];
        row[2 * ku] += ar * tr - ai * ti;
        row[2 * ku + 1] += ar * ti + ai * tr;
      }
    }
    *sumw += wt[j];
  }
}

/*
 * Grid nvis visibilities into grid (accumulated into, [n_images][n][n] complex128
 * interleaved).  sumw[n_images] and counters[3] (dropped, w clamped, bad weight)
 * are accumulated into.  img_off is the CSR split of rows over images (NULL for one
 * image).  nthreads > 1 uses OpenMP: one image -> private per-thread grids over
 * contiguous row ranges, summed in thread order; several images -> one image per task.
 */
int wref_grid(int n, double cell, int n_w, double w_max, int w_mode, int n_layers,
              const int32_t *supp, int O, const double *tab, const int64_t *tab_off, int64_t nvis,
              const double *uvw, const double *vis, const double *wt, int n_images,
              const int64_t *img_off, double *grid, double *sumw, int64_t *counters, int nthreads) {
  plan_t P;
  init_plan(&P, n, cell, n_w, w_max, w_mode, n_layers, supp, O);
  const int64_t cells = (int64_t)n * n;
  const int L = P.n_layers;
  if (nthreads < 1) nthreads = 1;
  if (L > 1) {
    /* w-stacking: each thread grids the rows of the layers congruent to its number, over
       every image, in row order (no private grids) */
    int64_t cnt_all[3] = {0, 0, 0};
    double *sw_all = (double *)calloc((size_t)nthreads * n_images, sizeof(double));
    if (!sw_all) return -2;
#pragma omp parallel num_threads(nthreads)
    {
      int t = 0, nt = 1;
#ifdef _OPENMP
      t = omp_get_thread_num();
      nt = omp_get_num_threads();
#endif
      int64_t cnt[3] = {0, 0, 0};
      for (int im = 0; im < n_images; ++im) {
        int64_t s = img_off ? img_off[im] : 0, e = img_off ? img_off[im + 1] : nvis;
        grid_range(&P, tab, tab_off, s, e, uvw, vis, wt, grid + 2 * cells * L * im,
                   sw_all + (int64_t)t * n_images + im, cnt, nt, t);
      }
#pragma omp critical
      {
        cnt_all[0] += cnt[0];
        cnt_all[1] += cnt[1];
        cnt_all[2] += cnt[2];
      }
    }
    /* rows with no layer (flagged, bad weight or dropped) are counted by thread 0 only:
       classify gives them layer 0 */
    for (int im = 0; im < n_images; ++im)
      for (int t = 0; t < nthreads; ++t) sumw[im] += sw_all[(int64_t)t * n_images + im];
    for (int k = 0; k < 3; ++k) counters[k] += cnt_all[k];
    free(sw_all);
    return 0;
  }
  if (n_images > 1 || nthreads == 1) {
    int64_t cnt_all[3] = {0, 0, 0};
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) if (nthreads > 1)
    for (int im = 0; im < n_images; ++im) {
      int64_t s = img_off ? img_off[im] : 0, e = img_off ? img_off[im + 1] : nvis;
      int64_t cnt[3] = {0, 0, 0};
      double sw = 0.0;
      grid_range(&P, tab, tab_off, s, e, uvw, vis, wt, grid + 2 * cells * im, &sw, cnt, 1, 0);
      sumw[im] += sw;
#pragma omp critical
      {
        cnt_all[0] += cnt[0];
        cnt_all[1] += cnt[1];
        cnt_all[2] += cnt[2];
      }
    }
    for (int k = 0; k < 3; ++k) counters[k] += cnt_all[k];
    return 0;
  }
  double *priv = (double *)calloc((size_t)nthreads * 2 * cells, sizeof(double));
  double *sw = (double *)calloc((size_t)nthreads, sizeof(double));
  int64_t *cnt = (int64_t *)calloc((size_t)nthreads * 3, sizeof(int64_t));
  if (!priv || !sw || !cnt) {
    free(priv);
    free(sw);
    free(cnt);
    return -2;
  }
#pragma omp parallel num_threads(nthreads)
  {
    int t = 0, nt = 1;
#ifdef _OPENMP
    t = omp_get_thread_num();
    nt = omp_get_num_threads();
#endif
    int64_t s = nvis * t / nt, e = nvis * (t + 1) / nt;
    grid_range(&P, tab, tab_off, s, e, uvw, vis, wt, priv + 2 * cells * t, sw + t, cnt + 3 * t, 1, 0);
  }
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int64_t c = 0; c < 2 * cells; ++c) {
    double acc = grid[c];
    for (int t = 0; t < nthreads; ++t) acc += priv[2 * cells * t + c];
    grid[c] = acc;
  }
  for (int t = 0; t < nthreads; ++t) {
    sumw[0] += sw[t];
    for (int k = 0; k < 3; ++k) counters[k] += cnt[3 * t + k];
  }
  free(priv);
  free(sw);
  free(cnt);
  return 0;
}

/*
 * Degrid: V_j = sum_taps conj(T_p[ov][ou][kv][ku]) M[y0+kv][x0+ku] (complex128
 * interleaved, overwritten); rows with non-finite uvw or off-grid footprints get 0.
 */
int wref_degrid(int n, double cell, int n_w, double w_max, int w_mode, int n_layers,
                const int32_t *supp, int O, const double *tab, const int64_t *tab_off, int64_t nvis,
                const double *uvw, int n_images, const int64_t *img_off, const double *M,
                double *vis_out, int nthreads) {
  plan_t P;
  init_plan(&P, n, cell, n_w, w_max, w_mode, n_layers, supp, O);
  const int64_t cells = (int64_t)n * n;
  if (nthreads < 1) nthreads = 1;
  for (int im = 0; im < n_images; ++im) {
    int64_t s = img_off ? img_off[im] : 0, e = img_off ? img_off[im + 1] : nvis;
#pragma omp parallel for schedule(static) num_threads(nthreads) if (nthreads > 1)
    for (int64_t j = s; j < e; ++j) {
      int p, x0, y0, ou, ov, fold = 0, layer = 0;
      double vr = 0.0, vi = 0.0;
      if (classify(&P, uvw + 3 * j, 1.0, &p, &x0, &y0, &ou, &ov, &fold, &layer) == 0) {
        const double *Mi = M + 2 * cells * ((int64_t)im * P.n_layers + layer);
        const int S = P.supp[p];
        const double *T = tab + 2 * (tab_off[p] + ((int64_t)ov * O + ou) * S * S);
        for (int kv = 0; kv < S; ++kv) {
          const double *row = Mi + 2 * ((int64_t)(y0 + kv) * n + x0);
          for (int ku = 0; ku < S; ++ku) {
            const double tr = T[2 * (kv * S + ku)], ti = T[2 * (kv * S + ku) + 1];
            const double mr = row[2 * ku], mi = row[2 * ku + 1];
            vr += tr * mr + ti * mi;
            vi += tr * mi - ti * mr;
          }
        }
      }
      vis_out[2 * j] = vr;
      vis_out[2 * j + 1] = fold ? -vi : vi;
    }
  }
  return 0;
}
