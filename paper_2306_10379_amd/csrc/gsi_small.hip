// Single-workgroup float64 solves on the p x p projected problem: the stop test and
// Polak-Ribiere coefficient, the eigendecomposition of P^T P (parallel cyclic Jacobi in
// LDS, warm-started from the previous iteration's eigenvectors), the line-search diagonals,
// the exact line search (bracket from the branch roots, Brent's method on phi'), the
// retraction factor M, Cholesky QR and Rayleigh-Ritz.
//
// The p x p matrices live in the small buffer as PP x PP row-major arrays (PP = 16, 32, 64 or
// 128, the smallest that holds p) whose padding is zero; dense products among them use f64
// MFMA. Working matrices sit in LDS up to PP = 64 and in the small buffer's work area above.
#include <math.h>

#include "gsi_kernels.h"
#include "gsi_small_dev.h"

namespace gsi {

// ---------------------------------------------------------------- kernels

__global__ __launch_bounds__(WG) void k_after_grad(int PP, const double* __restrict__ red, double* __restrict__ small,
                                                   Scalars* __restrict__ sc, double* __restrict__ hist, int cond) {
  if (sc->done) return;
  if (cond == GRAD_PENDING && sc->grad_ready) return;
  if (cond == GRAD_AFTER_FUSED && (sc->null_step || sc->refresh || sc->grad_ready)) return;
  __shared__ double sbeta, sphi;
  // the scalars and the trace of C are read by all threads at once (one round trip) and the
  // sequential decisions below work on the LDS copy: dependent global reads one after the
  // other cost a memory latency each
  __shared__ Scalars ls;
  for (int i = threadIdx.x; i < (int)(sizeof(Scalars) / 4); i += blockDim.x)
    reinterpret_cast<int32_t*>(&ls)[i] = reinterpret_cast<const int32_t*>(sc)[i];
  if (threadIdx.x < 64) {
    double d = 0.0;
    for (int i = threadIdx.x; i < PP; i += 64) d += small[S_C * PP * PP + i * PP + i];
    d = wave_sum(d);
    if (threadIdx.x == 0) sphi = -0.5 * d;
  }
  __syncthreads();
  const double* K = red;
  if (threadIdx.x == 0) {
    Scalars* lsc = &ls;
    const double gg = red[PP * PP], gdot = red[PP * PP + 1], ginf = red[PP * PP + 2];
    const int k = lsc->k;
    sc->gg = gg;
    sc->gdot = gdot;
    sc->ginf = ginf;
    const double rho = sqrt(gg) / (lsc->sqrt_p * lsc->nA);
    const double phi = sphi;
    sc->rho = rho;
    sc->phi = phi;
    if (k == 0) {
      lsc->ginf0 = ginf;
      sc->ginf0 = ginf;
    }
    if (k < lsc->hist_cap) {
      double* h = hist + (int64_t)k * H_FIELDS;
      h[H_RHO] = rho;
      h[H_PHI] = phi;
      h[H_MU] = 0.0;
      h[H_BETA] = 0.0;
      h[H_GINF] = lsc->ginf0 > 0.0 ? ginf / lsc->ginf0 : 0.0;
      if (k + 1 > lsc->hist_len) sc->hist_len = k + 1;
    }
    double beta = 0.0;
    if (k == 0 || rho <= 0.5 * lsc->rho_best) {
      lsc->rho_best = rho;
      lsc->k_best = k;
      sc->rho_best = rho;
      sc->k_best = k;
    }
    if (!isfinite(gg)) {
      ls.done = sc->done = 3;
    } else if (rho <= lsc->tol) {
      ls.done = sc->done = 1;
    } else if (k >= lsc->max_iter) {
      ls.done = sc->done = 2;
    } else if (lsc->stall_window > 0 && k - lsc->k_best > lsc->stall_window) {
      ls.done = sc->done = 4;  // stagnation: the block precision cannot resolve further progress
    } else {
      const bool restart = lsc->method == 1 || k == 0 || lsc->restart_next ||
                           (lsc->k_restart > 0 && k % lsc->k_restart == 0) || !(lsc->gg_old > 0.0);
      beta = restart ? 0.0 : (gg - gdot) / lsc->gg_old;
      sc->restart = restart ? 1 : 0;
      sc->restart_next = 0;
      sc->null_step = 0;
      sc->beta_pr = beta;
      if (k < lsc->hist_cap) hist[(int64_t)k * H_FIELDS + H_BETA] = beta;
    }
    sbeta = beta;
    sc->grad_ready = 1;
  }
  __syncthreads();
  if (ls.done) return;
  const double beta = sbeta;
  double* Kd = small + S_KD * PP * PP;
  double* Ks = small + S_K * PP * PP;
  const double* W = small + S_W * PP * PP;
  for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) {
    Ks[e] = K[e];
    Kd[e] = K[e] + (beta != 0.0 ? beta * W[e] : 0.0);
  }
}

__global__ __launch_bounds__(WG) void k_after_dir(int PP, const double* __restrict__ red, double* __restrict__ small,
                                                  Scalars* __restrict__ sc) {
  if (sc->done) return;
  double* S = small + S_S * PP * PP;
  // lane j of each wave, rows dealt to the waves (no division by the runtime PP)
  for (int i = threadIdx.x >> 6; i < PP; i += blockDim.x >> 6)
    for (int j = threadIdx.x & 63; j < PP; j += 64) S[i * PP + j] = 0.5 * (red[i * PP + j] + red[j * PP + i]);
  if (threadIdx.x == 0) {
    const double gp = red[PP * PP];
    sc->gp = gp;
    if (!(gp > 0.0)) {
      if (sc->restart) {
        sc->done = 3;  // the projected gradient is not a descent direction: G = 0 to rounding
      } else {
        sc->null_step = 1;
        sc->restart_next = 1;
        sc->n_null += 1;
        sc->grad_ready = 0;  // the next iteration forms the gradient again (and restarts)
      }
    }
  }
}

// Eigendecomposition of P^T P (see eig_dev), one workgroup.
template <int PP>
__global__ __launch_bounds__(WG) void k_eig(double* __restrict__ small, Scalars* __restrict__ sc) {
  if (sc->done || sc->null_step) return;
  // this single workgroup shares its CU with the SpMM running concurrently: raise its
  // waves' issue priority so the latency-bound rotation rounds are not starved
  __builtin_amdgcn_s_setprio(3);
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ double cs[2 * MAXP];
  __shared__ int uv[MAXP];
  __shared__ int nrot, anyr;
  const int sweeps = eig_dev<PP>(small, sc->p, sc->v_valid != 0, reinterpret_cast<double*>(lds_raw), cs, uv, &nrot,
                                 &anyr);
  if (threadIdx.x == 0) {
    sc->v_valid = 1;
    sc->sweeps = sweeps;
    sc->n_sweeps += sweeps;
  }
}

// Line search and retraction factor (see linesearch_dev), one workgroup; red holds the
// reduced Grams P^T A P, P^T A X of the SpMM.
template <int PP>
__global__ __launch_bounds__(WG) void k_linesearch(const double* __restrict__ red, double* __restrict__ small,
                                                   Scalars* __restrict__ sc, double* __restrict__ hist,
                                                   int recompute_ax, int want_mc) {
  if (sc->done || sc->null_step) return;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ Terms terms;
  __shared__ double smu, sbmax;
  __shared__ int sok, sevals;
  // the scalars read by the sequential tail, loaded by all threads at once
  __shared__ Scalars ls;
  for (int i = threadIdx.x; i < (int)(sizeof(Scalars) / 4); i += blockDim.x)
    reinterpret_cast<int32_t*>(&ls)[i] = reinterpret_cast<const int32_t*>(sc)[i];
  __syncthreads();
  const int p = ls.p;
  double* work = PP > PP_LDS_MAX ? small + small_work_offset(PP) + 4 * PP * (PP + 1)
                                 : reinterpret_cast<double*>(lds_raw);
  linesearch_dev<PP>(red, red + PP * PP, small, p, work, terms, &smu, &sok, &sevals, &sbmax, want_mc != 0);
  if (threadIdx.x == 0) {
    sc->brent_evals = sevals;
    sc->grad_ready = 0;  // X changes (or the step is void and the next iteration restarts)
    if (!sok) {
      if (ls.restart) {
        sc->done = 3;
      } else {
        sc->null_step = 1;
        sc->restart_next = 1;
        sc->n_null = ls.n_null + 1;
      }
    } else {
      const int k = ls.k;
      const double mu = smu;
      const int refresh = (recompute_ax || mu * sqrt(sbmax) <= 1e3 * EPS) ? 1 : 0;
      sc->mu = mu;
      sc->refresh = refresh;
      if (k < ls.hist_cap) hist[(int64_t)k * H_FIELDS + H_MU] = mu;
      sc->n_restart = ls.n_restart + ls.restart;
      sc->n_refresh = ls.n_refresh + refresh;
      sc->n_spmm = ls.n_spmm + 1 + refresh;
      sc->gg_old = ls.gg;
      sc->k = k + 1;
    }
  }
}

__global__ __launch_bounds__(WG) void k_after_update_grams(int PP, const double* __restrict__ red,
                                                           double* __restrict__ small, Scalars* __restrict__ sc) {
  if (sc->done || sc->null_step) return;
  double* C = small + S_C * PP * PP;
  double* W = small + S_W * PP * PP;
  for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) {
    const int i = e / PP, j = e % PP;
    if (!sc->refresh) C[e] = 0.5 * (red[i * PP + j] + red[j * PP + i]);
    W[e] = red[PP * PP + e];
  }
}

__global__ __launch_bounds__(WG) void k_after_refresh(int PP, const double* __restrict__ red,
                                                      double* __restrict__ small, Scalars* __restrict__ sc) {
  if (sc->done || sc->null_step || !sc->refresh) return;
  double* C = small + S_C * PP * PP;
  for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) {
    const int i = e / PP, j = e % PP;
    C[e] = 0.5 * (red[i * PP + j] + red[j * PP + i]);
  }
}

// Cholesky G = L L^T of the leading p x p block of red, then M = L^{-T} (so X M has
// orthonormal columns when G = X^T X). flag = 1 on a non-positive or tiny pivot.
__global__ __launch_bounds__(WG) void k_chol_inv(int PP, int p, const double* __restrict__ red,
                                                 double* __restrict__ small, int* __restrict__ flag) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  // p up to 64 in LDS; above, in the work area of the small buffer
  const bool wide = PP > PP_LDS_MAX;
  double* L = wide ? small + small_work_offset(PP) + 4 * PP * (PP + 1) : reinterpret_cast<double*>(lds_raw);
  double* Li = L + (wide ? PP * PP : MAXP * MAXP);
  __shared__ int bad;
  __shared__ double dmax;
  for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
    const int i = e / p, j = e % p;
    L[e] = 0.5 * (red[i * PP + j] + red[j * PP + i]);
  }
  if (threadIdx.x == 0) {
    bad = 0;
    double m = 0.0;
    for (int i = 0; i < p; ++i) m = fmax(m, red[i * PP + i]);
    dmax = m;
  }
  __syncthreads();
  for (int j = 0; j < p; ++j) {
    if (threadIdx.x == 0) {
      const double piv = L[j * p + j];
      if (!(piv > 1e-13 * dmax) || !isfinite(piv)) bad = 1;
      L[j * p + j] = sqrt(fabs(piv) > 0.0 ? fabs(piv) : 1.0);
    }
    __syncthreads();
    const double ljj = L[j * p + j];
    for (int i = j + 1 + threadIdx.x; i < p; i += blockDim.x) L[i * p + j] /= ljj;
    __syncthreads();
    for (int e = threadIdx.x; e < (p - j - 1) * (p - j - 1); e += blockDim.x) {
      const int i = j + 1 + e / (p - j - 1), k = j + 1 + e % (p - j - 1);
      if (k <= i) L[i * p + k] -= L[i * p + j] * L[k * p + j];
    }
    __syncthreads();
  }
  // Li = L^{-1} (lower), one column per thread
  for (int c = threadIdx.x; c < p; c += blockDim.x) {
    for (int i = 0; i < p; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) s -= L[i * p + k] * Li[k * p + c];
      Li[i * p + c] = i < c ? 0.0 : s / L[i * p + i];
    }
  }
  __syncthreads();
  double* M = small + S_M * PP * PP;
  for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) {
    const int i = e / PP, j = e % PP;
    M[e] = (i < p && j < p) ? Li[j * p + i] : 0.0;  // M = L^{-T}
  }
  if (threadIdx.x == 0 && bad) *flag = 1;
}

// After a Cholesky QR pass X <- X M (M = R^{-1} in small[S_M]): C <- M^T C M, W <- M^T W.
// If the factorization was flagged as failed, M is reset to the identity instead.
template <int PP>
__global__ __launch_bounds__(WG) void k_transform_cw(double* __restrict__ small, int* __restrict__ flag) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double* T1 = PP > PP_LDS_MAX ? small + small_work_offset(PP) + 4 * PP * (PP + 1) : reinterpret_cast<double*>(lds_raw);
  double* T2 = T1 + PP * PP;
  double* M = small + S_M * PP * PP;
  double* C = small + S_C * PP * PP;
  double* W = small + S_W * PP * PP;
  if (*flag) {
    for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) M[e] = (e / PP) == (e % PP) ? 1.0 : 0.0;
    __syncthreads();
    if (threadIdx.x == 0) *flag = 0;
    return;
  }
  wg_mm<PP>(C, false, M, false, T1);  // C M
  wg_mm<PP>(M, true, W, false, T2);   // M^T W
  __syncthreads();
  wg_mm<PP>(M, true, T1, false, C);   // M^T C M
  for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) W[e] = T2[e];
  __syncthreads();
  for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) {
    const int i = e / PP, j = e % PP;
    if (i < j) {
      const double v = 0.5 * (C[i * PP + j] + C[j * PP + i]);
      C[i * PP + j] = v;
      C[j * PP + i] = v;
    }
  }
}

// Rayleigh-Ritz: eig of sym(red) (p x p): eigenvalues descending into vals[0..p),
// eigenvectors as the columns of small[S_M] (stride PP, padding zero).
__global__ __launch_bounds__(WG) void k_ritz(int PP, int p, const double* __restrict__ red, double* __restrict__ small,
                                             double* __restrict__ vals) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  // p up to 64 in LDS; above, in the work area of the small buffer
  const bool wide = PP > PP_LDS_MAX;
  double* A = wide ? small + small_work_offset(PP) + 4 * PP * (PP + 1) : reinterpret_cast<double*>(lds_raw);
  double* V = A + (wide ? PP * (PP + 1) : MAXP * (MAXP + 1));
  __shared__ double cs[2 * MAXP];  // at most 64 rotations per round (p <= 128)
  __shared__ int uv[MAXP];
  __shared__ int nrot, anyr;
  __shared__ int order[TMAXP];
  const int ld = p | 1;  // odd stride: no LDS bank conflicts in the column sweeps
  for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
    const int i = e / p, j = e % p;
    A[i * ld + j] = 0.5 * (red[i * PP + j] + red[j * PP + i]);
    V[i * ld + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  jacobi(p, ld, A, V, cs, uv, &nrot, &anyr);
  if (threadIdx.x == 0) {
    for (int i = 0; i < p; ++i) order[i] = i;
    for (int i = 1; i < p; ++i) {  // insertion sort, descending
      const int o = order[i];
      const double v = A[o * ld + o];
      int j = i - 1;
      while (j >= 0 && A[order[j] * ld + order[j]] < v) { order[j + 1] = order[j]; --j; }
      order[j + 1] = o;
    }
    for (int i = 0; i < p; ++i) vals[i] = A[order[i] * ld + order[i]];
  }
  __syncthreads();
  double* M = small + S_M * PP * PP;
  for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) {
    const int i = e / PP, j = e % PP;
    M[e] = (i < p && j < p) ? V[i * ld + order[j]] : 0.0;
  }
}

// ---------------------------------------------------------------- launchers

static constexpr int RITZ_LDS = 2 * MAXP * (MAXP + 1) * (int)sizeof(double);

template <int PP>
static hipError_t init_pp() {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_eig<PP>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 3 * PP * (PP + 1) * 8);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_linesearch<PP>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 4 * PP * PP * 8);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_transform_cw<PP>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 2 * PP * PP * 8);
  return e;
}

hipError_t Small::init() {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_ritz), hipFuncAttributeMaxDynamicSharedMemorySize,
                                     RITZ_LDS);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_chol_inv), hipFuncAttributeMaxDynamicSharedMemorySize,
                            RITZ_LDS);
  if (e == hipSuccess) e = init_pp<16>();
  if (e == hipSuccess) e = init_pp<32>();
  if (e == hipSuccess) e = init_pp<64>();
  // p up to 128: the Jacobi's matrix in LDS (the other p x p kernels use the work area)
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_eig<128>), hipFuncAttributeMaxDynamicSharedMemorySize,
                            128 * 129 * 8);
  return e;
}
void Small::after_grad(hipStream_t st, int PP, const double* red, double* small, Scalars* sc, double* hist, int cond) {
  hipLaunchKernelGGL(k_after_grad, dim3(1), dim3(WG), 0, st, PP, red, small, sc, hist, cond);
}
void Small::after_dir(hipStream_t st, int PP, const double* red, double* small, Scalars* sc) {
  hipLaunchKernelGGL(k_after_dir, dim3(1), dim3(WG), 0, st, PP, red, small, sc);
}
void Small::eig(hipStream_t st, int PP, double* small, Scalars* sc) {
  switch (PP) {
    case 16: k_eig<16><<<1, WG, 3 * 16 * 17 * 8, st>>>(small, sc); break;
    case 32: k_eig<32><<<1, WG, 3 * 32 * 33 * 8, st>>>(small, sc); break;
    case 64: k_eig<64><<<1, WG, 3 * 64 * 65 * 8, st>>>(small, sc); break;
    case 128: k_eig<128><<<1, WG, 128 * 129 * 8, st>>>(small, sc); break;
  }
}
void Small::linesearch(hipStream_t st, int PP, const double* red, double* small, Scalars* sc, double* hist,
                       int recompute_ax, bool want_mc) {
  const int mc = want_mc ? 1 : 0;
  switch (PP) {
    case 16: k_linesearch<16><<<1, WG, 4 * 16 * 16 * 8, st>>>(red, small, sc, hist, recompute_ax, mc); break;
    case 32: k_linesearch<32><<<1, WG, 4 * 32 * 32 * 8, st>>>(red, small, sc, hist, recompute_ax, mc); break;
    case 64: k_linesearch<64><<<1, WG, 4 * 64 * 64 * 8, st>>>(red, small, sc, hist, recompute_ax, mc); break;
    case 128: k_linesearch<128><<<1, WG, 0, st>>>(red, small, sc, hist, recompute_ax, mc); break;
  }
}
void Small::after_update_grams(hipStream_t st, int PP, const double* red, double* small, Scalars* sc) {
  hipLaunchKernelGGL(k_after_update_grams, dim3(1), dim3(WG), 0, st, PP, red, small, sc);
}
void Small::after_refresh(hipStream_t st, int PP, const double* red, double* small, Scalars* sc) {
  hipLaunchKernelGGL(k_after_refresh, dim3(1), dim3(WG), 0, st, PP, red, small, sc);
}
void Small::chol_inv(hipStream_t st, int PP, int p, const double* red, double* small, int* flag) {
  hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(WG), PP > PP_LDS_MAX ? 0 : RITZ_LDS, st, PP, p, red, small, flag);
}
void Small::transform_cw(hipStream_t st, int PP, double* small, int* flag) {
  switch (PP) {
    case 16: k_transform_cw<16><<<1, WG, 2 * 16 * 16 * 8, st>>>(small, flag); break;
    case 32: k_transform_cw<32><<<1, WG, 2 * 32 * 32 * 8, st>>>(small, flag); break;
    case 64: k_transform_cw<64><<<1, WG, 2 * 64 * 64 * 8, st>>>(small, flag); break;
    case 128: k_transform_cw<128><<<1, WG, 0, st>>>(small, flag); break;
  }
}
void Small::ritz(hipStream_t st, int PP, int p, const double* red, double* small, double* out_vals) {
  hipLaunchKernelGGL(k_ritz, dim3(1), dim3(WG), PP > PP_LDS_MAX ? 0 : RITZ_LDS, st, PP, p, red, small, out_vals);
}

}  // namespace gsi
