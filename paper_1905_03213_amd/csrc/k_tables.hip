// Kernel-table generation in FP64 on the device.
//
// For plane p (support S_p, oversampling O, m image samples per axis):
//   taper    psi(nu) = psi_0(c, nu)/psi_0(c, 0), evaluated from its Legendre series;
//   screen   s_p[j][i] = psi(nu_i) psi(nu_j) exp(+2 pi i w_p (sqrt(1 - l_i^2 - m_j^2) - 1)),
//            nu_i = (2i + 1 - m)/m, l_i = nu_i FoV/2, zero where l^2 + m^2 >= 1;
//   DFT      C_p[ib][ia] = sum_j E[ib][j] sum_i s_p[j][i] E[ia][i],
//            E[r][i] = exp(-2 pi i a (i + 1/2 - m/2)/(O m)), a = r + 1 - S_p O/2,
//            the Fourier transform of the screen at uv offsets a/O cells;
//   tables   sub-kernel (ov, ou), tap (kv, ku) = C_p[ov + kv O][ou + ku O] divided by the
//            sub-kernel's complex tap sum, stored [ov][ou][kv][ku].
// This is the standard w-projection kernel construction (the method the paper applies,
// Sections 1-2); the two DFTs are small dense products done once per handle.
#include "wproj_internal.h"

namespace wproj {
namespace {

__device__ double legendre_even_series(const double *coef, int n_coef, double x) {
  // coef[k] multiplies P_{2k}(x); P_n by the three-term recurrence.
  double p_prev = 1.0, p_cur = x;
  double s = coef[0];
  for (int n = 1; n < 2 * n_coef - 1; ++n) {
    double p_next = ((2.0 * n + 1.0) * x * p_cur - n * p_prev) / (n + 1.0);
    p_prev = p_cur;
    p_cur = p_next;
    if (((n + 1) & 1) == 0) s += coef[(n + 1) >> 1] * p_cur;
  }
  return s;
}

__global__ void taper_kernel(const double *coef, int n_coef, int m, int n, double *taper,
                             double *kappa) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m + n) return;
  const double s0 = legendre_even_series(coef, n_coef, 0.0);
  if (t < m) {
    double nu = (2.0 * t + 1.0 - m) / (double)m;
    taper[t] = legendre_even_series(coef, n_coef, nu) / s0;
  } else {
    int x = t - m;
    double nu = ((double)x - n / 2.0) / (n / 2.0);
    double k = 0.0;
    if (fabs(nu) < 1.0) {
      double psi = legendre_even_series(coef, n_coef, nu) / s0;
      k = 1.0 / psi;
    }
    kappa[x] = k;
  }
}

__global__ void screen_kernel(const double *taper, int m, double fov, double w_max, double dw,
                              int n_w, int w_mode, int p0, int np, double2 *out) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = (int64_t)np * m * m;
  if (t >= total) return;
  int i = (int)(t % m);
  int j = (int)((t / m) % m);
  int p = p0 + (int)(t / ((int64_t)m * m));
  // plane values: linear over [-w_max, w_max], or over [0, w_max] with a Hermitian fold
  // (evenly spaced in w, or in sqrt(w))
  double wp = 0.0;
  if (n_w > 1) {
    if (w_mode == WPROJ_W_LINEAR) {
      wp = -w_max + p * dw;
    } else if (w_mode == WPROJ_W_FOLD) {
      wp = p * dw;
    } else {
      const double f = (double)p / (double)(n_w - 1);
      wp = w_max * (f * f);
    }
  }
  double lmax = fov / 2.0;
  double li = (2.0 * i + 1.0 - m) / (double)m * lmax;
  double mj = (2.0 * j + 1.0 - m) / (double)m * lmax;
  double r2 = li * li + mj * mj;
  double2 v = make_double2(0.0, 0.0);
  if (r2 < 1.0) {
    double amp = taper[i] * taper[j];
    double sn, cs;
    sincospi(2.0 * wp * (sqrt(1.0 - r2) - 1.0), &sn, &cs);
    v = make_double2(amp * cs, amp * sn);
  }
  out[t] = v;
}

// E[r][i] for plane support S: exp(-2 pi i a (2i + 1 - m)/(2 O m)), a = r + 1 - S O/2.
__device__ inline double2 dft_coef(int r, int i, int S, int O, int m) {
  int64_t a = (int64_t)r + 1 - (int64_t)S * O / 2;
  double arg = -(double)(a * (2 * i + 1 - m)) / (double)((int64_t)O * m);
  double sn, cs;
  sincospi(arg, &sn, &cs);
  return make_double2(cs, sn);
}

// tmp[p][j][ia] = sum_i screen[p][j][i] E[ia][i]
__global__ void dft_rows_kernel(const double2 *screen, int m, int O, const int32_t *supp, int p0,
                                int np, int so_max, double2 *tmp) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = (int64_t)np * m * so_max;
  if (t >= total) return;
  int ia = (int)(t % so_max);
  int j = (int)((t / so_max) % m);
  int pl = (int)(t / ((int64_t)so_max * m));
  int S = supp[p0 + pl];
  double2 acc = make_double2(0.0, 0.0);
  if (ia < S * O) {
    const double2 *row = screen + ((int64_t)pl * m + j) * m;
    for (int i = 0; i < m; ++i) {
      double2 e = dft_coef(ia, i, S, O, m);
      double2 s = row[i];
      acc.x += s.x * e.x - s.y * e.y;
      acc.y += s.x * e.y + s.y * e.x;
    }
  }
  tmp[t] = acc;
}

// C[p][ib][ia] = sum_j E[ib][j] tmp[p][j][ia]
__global__ void dft_cols_kernel(const double2 *tmp, int m, int O, const int32_t *supp, int p0,
                                int np, int so_max, double2 *C) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = (int64_t)np * so_max * so_max;
  if (t >= total) return;
  int ia = (int)(t % so_max);
  int ib = (int)((t / so_max) % so_max);
  int pl = (int)(t / ((int64_t)so_max * so_max));
  int S = supp[p0 + pl];
  double2 acc = make_double2(0.0, 0.0);
  if (ia < S * O && ib < S * O) {
    const double2 *col = tmp + (int64_t)pl * m * so_max + ia;
    for (int j = 0; j < m; ++j) {
      double2 e = dft_coef(ib, j, S, O, m);
      double2 s = col[(int64_t)j * so_max];
      acc.x += s.x * e.x - s.y * e.y;
      acc.y += s.x * e.y + s.y * e.x;
    }
  }
  C[t] = acc;
}

template <typename T>
__device__ inline void store_tap(T *tab, int64_t idx, double re, double im);
template <>
__device__ inline void store_tap<double2>(double2 *tab, int64_t idx, double re, double im) {
  tab[idx] = make_double2(re, im);
}
template <>
__device__ inline void store_tap<float2>(float2 *tab, int64_t idx, double re, double im) {
  tab[idx] = make_float2((float)re, (float)im);
}
template <>
__device__ inline void store_tap<half2c>(half2c *tab, int64_t idx, double re, double im) {
  half2c h;
  h.re = (_Float16)re;  // one rounding, to nearest even, straight from float64
  h.im = (_Float16)im;
  tab[idx] = h;
}

// One block of 256 threads per (plane, ov, ou) sub-kernel.
template <typename T>
__global__ void __launch_bounds__(256) normalise_kernel(const double2 *C, int so_max, int O,
                                                        const int32_t *supp,
                                                        const int64_t *tab_off, int p0, T *tab) {
  __shared__ double sre[256], sim[256];
  const int sub = blockIdx.x;  // ov * O + ou
  const int pl = blockIdx.y;
  const int p = p0 + pl;
  const int S = supp[p];
  const int ov = sub / O, ou = sub % O;
  const double2 *Cp = C + (int64_t)pl * so_max * so_max;
  double re = 0.0, im = 0.0;
  for (int k = threadIdx.x; k < S * S; k += blockDim.x) {
    int kv = k / S, ku = k % S;
    double2 c = Cp[(int64_t)(ov + kv * O) * so_max + (ou + ku * O)];
    re += c.x;
    im += c.y;
  }
  sre[threadIdx.x] = re;
  sim[threadIdx.x] = im;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      sre[threadIdx.x] += sre[threadIdx.x + w];
      sim[threadIdx.x] += sim[threadIdx.x + w];
    }
    __syncthreads();
  }
  const double sr = sre[0], si = sim[0];
  const double den = sr * sr + si * si;
  const int64_t base = tab_off[p] + (int64_t)sub * S * S;
  for (int k = threadIdx.x; k < S * S; k += blockDim.x) {
    int kv = k / S, ku = k % S;
    double2 c = Cp[(int64_t)(ov + kv * O) * so_max + (ou + ku * O)];
    // c / (sr + i si)
    double qr = (c.x * sr + c.y * si) / den;
    double qi = (c.y * sr - c.x * si) / den;
    store_tap<T>(tab, base + k, qr, qi);
  }
}

inline unsigned blocks_for(int64_t total, int bs) { return (unsigned)((total + bs - 1) / bs); }

}  // namespace

hipError_t launch_taper(const double *d_coef, int n_coef, int m, int n, double *d_taper,
                        double *d_kappa, hipStream_t s) {
  hipLaunchKernelGGL(taper_kernel, dim3(blocks_for(m + n, 256)), dim3(256), 0, s, d_coef, n_coef,
                     m, n, d_taper, d_kappa);
  return hipGetLastError();
}

hipError_t launch_screen(const double *d_taper, int m, double fov, double w_max, double dw,
                         int n_w, int w_mode, int p0, int np, double2 *out, hipStream_t s) {
  int64_t total = (int64_t)np * m * m;
  hipLaunchKernelGGL(screen_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, s, d_taper, m,
                     fov, w_max, dw, n_w, w_mode, p0, np, out);
  return hipGetLastError();
}

hipError_t launch_table_dft(const double2 *screen, int m, int O, const int32_t *d_supp, int p0,
                            int np, int so_max, double2 *tmp, double2 *C, hipStream_t s) {
  int64_t t1 = (int64_t)np * m * so_max;
  hipLaunchKernelGGL(dft_rows_kernel, dim3(blocks_for(t1, 256)), dim3(256), 0, s, screen, m, O,
                     d_supp, p0, np, so_max, tmp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int64_t t2 = (int64_t)np * so_max * so_max;
  hipLaunchKernelGGL(dft_cols_kernel, dim3(blocks_for(t2, 256)), dim3(256), 0, s, tmp, m, O,
                     d_supp, p0, np, so_max, C);
  return hipGetLastError();
}

hipError_t launch_normalise(const double2 *C, int so_max, int O, const int32_t *d_supp,
                            const int64_t *d_tab_off, int p0, int np, int precision, void *tab,
                            hipStream_t s) {
  dim3 grid((unsigned)(O * O), (unsigned)np);
  switch (precision) {
    case WPROJ_F64:
      hipLaunchKernelGGL(normalise_kernel<double2>, grid, dim3(256), 0, s, C, so_max, O, d_supp,
                         d_tab_off, p0, (double2 *)tab);
      break;
    case WPROJ_F32:
      hipLaunchKernelGGL(normalise_kernel<float2>, grid, dim3(256), 0, s, C, so_max, O, d_supp,
                         d_tab_off, p0, (float2 *)tab);
      break;
    default:
      hipLaunchKernelGGL(normalise_kernel<half2c>, grid, dim3(256), 0, s, C, so_max, O, d_supp,
                         d_tab_off, p0, (half2c *)tab);
      break;
  }
  return hipGetLastError();
}

}  // namespace wproj
