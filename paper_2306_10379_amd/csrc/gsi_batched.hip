// Batched solve: many independent eigenproblems of different n and p in one persistent
// launch. Every workgroup pulls problem indices from an atomic queue (largest problems
// first) and runs the whole Riemannian CG iteration for one problem with workgroup barriers
// only: gradient, direction, eigendecomposition of P^T P, SpMM, Grams, line search and
// retraction (the same steps and readings as the single-problem path, see gsi_kernels.hip
// and gsi_small.hip). Blocks are float32 or float64; the p x p state is float64.
//
// Passes within a workgroup read rows that other waves of the same workgroup wrote in the
// previous pass; an agent-scope fence (L1 invalidation) plus a barrier separates passes.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <utility>
#include <new>
#include <string>
#include <vector>

#include "../../include/gsi.h"
#include "gsi_kernels.h"
#include "gsi_small_dev.h"

namespace gsi {

struct BatchProblem {
  int64_t n;
  int32_t p, PP;
  const int32_t* rowptr;
  const int32_t* colind;
  const void* vals;  // block precision, negated when the smallest eigenvalues are wanted
  void *X, *Y, *G0, *G1, *P0, *P1, *Z;  // whole 64-row tiles, PP columns
  double* small;                        // S_COUNT * PP * PP
  double nA;                            // ||A||_inf
  double* ritz;                         // p outputs (Ritz values of the operator solved)
  int32_t iters, status, restarts, null_steps;
  double rho;
};

struct BatchCtl {
  int32_t next;  // queue head
  int32_t count;
  int32_t method, k_restart, max_iter, stall_window, recompute_ax, pad;
  double tol;
  const int32_t* order;  // queue order (problem indices)
};

__device__ __forceinline__ void pass_barrier() {
  __threadfence();
  __syncthreads();
}

// ---------------------------------------------------------------- streaming passes (one workgroup)

template <typename T, int PP>
__device__ void b_load_matrix(T* __restrict__ s, const double* __restrict__ M) {
  for (int i = threadIdx.x; i < PP * PP; i += blockDim.x) s[i] = (T)M[i];
}

// G = X C - Y; sums of G^2 and G_old G, max absolute row sum.
template <typename T, int PP>
__device__ __noinline__ void b_grad(int64_t n, const T* X, const T* Y, const T* Gold, T* G, const T* sC, bool have_old,
                       double& gg, double& gdot, double& ginf) {
  const int w = threadIdx.x >> 6;
  const int64_t ntiles = (n + TR - 1) / TR;
  for (int64_t t = 0; t < ntiles; ++t) {
    const int64_t row0 = t * TR + 16 * w;
    T a[PP / 4];
    load_al<T, PP>(X, row0, n, a);
    typename Vec4<T>::type acc[PP / 16];
    zero_acc<T, PP>(acc);
    product<T, PP>(a, sC, acc);
    T y[PP / 16][4], g[PP / 16][4];
    load_rl<T, PP>(Y, row0, n, y);
#pragma unroll
    for (int cb = 0; cb < PP / 16; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) g[cb][r] = acc[cb][r] - y[cb][r];
    store_rl<T, PP>(G, row0, n, g);
    double rs[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int cb = 0; cb < PP / 16; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double gv = (double)g[cb][r];
        gg += gv * gv;
        rs[r] += fabs(gv);
      }
    if (have_old) {
      T go[PP / 16][4];
      load_rl<T, PP>(Gold, row0, n, go);
#pragma unroll
      for (int cb = 0; cb < PP / 16; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) gdot += (double)go[cb][r] * (double)g[cb][r];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) ginf = fmax(ginf, group16_sum(rs[r]));
  }
}

// P = G + beta P_old - X KD; sum of G P.
template <typename T, int PP>
__device__ __noinline__ void b_dir(int64_t n, const T* X, const T* G, const T* Pold, T* P, const T* sK, T beta, bool use_old,
                      double& gp) {
  const int w = threadIdx.x >> 6;
  const int64_t ntiles = (n + TR - 1) / TR;
  for (int64_t t = 0; t < ntiles; ++t) {
    const int64_t row0 = t * TR + 16 * w;
    T a[PP / 4];
    load_al<T, PP>(X, row0, n, a);
    typename Vec4<T>::type acc[PP / 16];
    zero_acc<T, PP>(acc);
    product<T, PP>(a, sK, acc);
    T g[PP / 16][4], p[PP / 16][4];
    load_rl<T, PP>(G, row0, n, g);
    if (use_old) load_rl<T, PP>(Pold, row0, n, p);
#pragma unroll
    for (int cb = 0; cb < PP / 16; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) p[cb][r] = g[cb][r] + (use_old ? beta * p[cb][r] : T(0)) - acc[cb][r];
    store_rl<T, PP>(P, row0, n, p);
#pragma unroll
    for (int cb = 0; cb < PP / 16; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) gp += (double)g[cb][r] * (double)p[cb][r];
  }
}

// X <- (X - mu P) M, Y <- (Y - mu Z) M (Y skipped when upd_y is false).
template <typename T, int PP>
__device__ __noinline__ void b_update(int64_t n, T* X, T* Y, const T* P, const T* Z, const T* sM, T mu, bool upd_y) {
  const int w = threadIdx.x >> 6;
  const int64_t ntiles = (n + TR - 1) / TR;
  for (int64_t t = 0; t < ntiles; ++t) {
    const int64_t row0 = t * TR + 16 * w;
    T a1[PP / 4], a2[PP / 4], b[PP / 4];
    load_al<T, PP>(X, row0, n, a1);
    load_al<T, PP>(P, row0, n, b);
#pragma unroll
    for (int s = 0; s < PP / 4; ++s) a1[s] = a1[s] - mu * b[s];
    typename Vec4<T>::type xacc[PP / 16], yacc[PP / 16];
    zero_acc<T, PP>(xacc);
    zero_acc<T, PP>(yacc);
    if (upd_y) {
      load_al<T, PP>(Y, row0, n, a2);
      load_al<T, PP>(Z, row0, n, b);
#pragma unroll
      for (int s = 0; s < PP / 4; ++s) a2[s] = a2[s] - mu * b[s];
      product2<T, PP>(a1, a2, sM, xacc, yacc);
    } else {
      product<T, PP>(a1, sM, xacc);
    }
    T xo[PP / 16][4], yo[PP / 16][4];
#pragma unroll
    for (int cb = 0; cb < PP / 16; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        xo[cb][r] = xacc[cb][r];
        yo[cb][r] = yacc[cb][r];
      }
    // every wave reads and writes only its own rows, so in-place is safe
    store_rl<T, PP>(X, row0, n, xo);
    if (upd_y) store_rl<T, PP>(Y, row0, n, yo);
  }
}

// OUT = IN M in place.
template <typename T, int PP>
__device__ __noinline__ void b_product(int64_t n, T* IN, const T* sM) {
  const int w = threadIdx.x >> 6;
  const int64_t ntiles = (n + TR - 1) / TR;
  for (int64_t t = 0; t < ntiles; ++t) {
    const int64_t row0 = t * TR + 16 * w;
    T a[PP / 4];
    load_al<T, PP>(IN, row0, n, a);
    typename Vec4<T>::type acc[PP / 16];
    zero_acc<T, PP>(acc);
    product<T, PP>(a, sM, acc);
    T o[PP / 16][4];
#pragma unroll
    for (int cb = 0; cb < PP / 16; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) o[cb][r] = acc[cb][r];
    store_rl<T, PP>(IN, row0, n, o);
  }
}

// Z = A W over all rows.
template <typename T, int PP>
__device__ __noinline__ void b_spmm(int64_t n, const int32_t* rowptr, const int32_t* colind, const T* vals, const T* W, T* Z) {
  constexpr int EPL = 4, LPR = PP / EPL, RPB = WG / LPR;
  const int sub = threadIdx.x / LPR, lane = threadIdx.x % LPR;
  for (int64_t row = sub; row < n; row += RPB) {
    T acc[EPL] = {T(0), T(0), T(0), T(0)};
    const int32_t j0 = rowptr[row], j1 = rowptr[row + 1];
    for (int32_t j = j0; j < j1; ++j) {
      const T v = vals[j];
      const T* src = W + (int64_t)colind[j] * PP + EPL * lane;
#pragma unroll
      for (int e = 0; e < EPL; ++e) acc[e] += v * src[e];
    }
    T* zr = Z + row * PP + EPL * lane;
#pragma unroll
    for (int e = 0; e < EPL; ++e) zr[e] = acc[e];
  }
}

// out1 = A^T B1, out2 = A^T B2 (B2 may be null): PP x PP float64, same lane scheme as k_gram.
template <typename T, int PP>
__device__ __noinline__ void b_gram(int64_t n, const T* A, const T* B1, const T* B2, double* out1, double* out2) {
  constexpr int V = PP / 16;
  constexpr int MAXU = (2 * V + 3) / 4;
  const int ng = B2 ? 2 : 1;
  const int units = ng * V;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, c = l & 15;
  const int gsel = w % ng;
  const T* B = gsel ? B2 : B1;
  const int nu = (units > w) ? (units - w + 3) / 4 : 0;
  const int64_t ntiles = (n + TR - 1) / TR;
  typename Vec4<T>::type acc[MAXU][V];
#pragma unroll
  for (int q = 0; q < MAXU; ++q)
#pragma unroll
    for (int jb = 0; jb < V; ++jb) acc[q][jb] = typename Vec4<T>::type{0, 0, 0, 0};
  if (nu > 0) {
    for (int64_t t = 0; t < ntiles; ++t) {
      for (int s = 0; s < TR / 4; ++s) {
        const int64_t row = t * TR + 4 * s + g;
        T a[V], b[V];
#pragma unroll
        for (int e = 0; e < V; ++e) {
          a[e] = row < n ? A[row * PP + V * c + e] : T(0);
          b[e] = row < n ? B[row * PP + V * c + e] : T(0);
        }
#pragma unroll
        for (int q = 0; q < MAXU; ++q) {
          if (q < nu) {
            const int ib = (w + 4 * q) / ng;
#pragma unroll
            for (int jb = 0; jb < V; ++jb) acc[q][jb] = mfma(a[ib], b[jb], acc[q][jb]);
          }
        }
      }
    }
  }
  double* o = gsel ? out2 : out1;
#pragma unroll
  for (int q = 0; q < MAXU; ++q) {
    if (q < nu) {
      const int ib = (w + 4 * q) / ng;
#pragma unroll
      for (int jb = 0; jb < V; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r) o[(rowof<T>(g, r) * V + ib) * PP + c * V + jb] = (double)acc[q][jb][r];
    }
  }
}

// ---------------------------------------------------------------- small helpers (one workgroup)

// Workgroup sums (and a max) of thread values; result in every thread.
__device__ void b_reduce3(double& a, double& b, double& m, double* red /* 12 */) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  double sa = wave_sum(a), sb = wave_sum(b), sm = wave_max(m);
  __syncthreads();
  if (l == 0) { red[3 * w] = sa; red[3 * w + 1] = sb; red[3 * w + 2] = sm; }
  __syncthreads();
  a = red[0] + red[3] + red[6] + red[9];
  b = red[1] + red[4] + red[7] + red[10];
  m = fmax(fmax(red[2], red[5]), fmax(red[8], red[11]));
  __syncthreads();
}

// Cholesky of sym(G) (p x p block of a PP x PP matrix), M = L^{-T} into Mout (PP x PP,
// padding zero). Returns false on a non-positive or tiny pivot. lds: 2 PP^2 doubles.
template <int PP>
__device__ __noinline__ bool b_chol_inv(const double* G, double* Mout, int p, double* lds, int* bad) {
  double* L = lds;
  double* Li = lds + PP * PP;
  for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
    const int i = e / p, j = e % p;
    L[e] = 0.5 * (G[i * PP + j] + G[j * PP + i]);
  }
  if (threadIdx.x == 0) *bad = 0;
  __syncthreads();
  double dmax = 0.0;
  for (int i = 0; i < p; ++i) dmax = fmax(dmax, L[i * p + i]);
  for (int j = 0; j < p; ++j) {
    __syncthreads();
    if (threadIdx.x == 0) {
      const double piv = L[j * p + j];
      if (!(piv > 1e-13 * dmax) || !isfinite(piv)) *bad = 1;
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
  }
  __syncthreads();
  for (int c = threadIdx.x; c < p; c += blockDim.x) {
    for (int i = 0; i < p; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) s -= L[i * p + k] * Li[k * p + c];
      Li[i * p + c] = i < c ? 0.0 : s / L[i * p + i];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) {
    const int i = e / PP, j = e % PP;
    Mout[e] = (i < p && j < p) ? Li[j * p + i] : 0.0;
  }
  __syncthreads();
  return *bad == 0;
}

// Out-of-line wrappers: the solver below calls every pass as a function, so each keeps its
// own register allocation instead of the sum over one giant inlined body.
template <int PP>
__device__ __noinline__ int b_eig(double* small, int p, bool warm, double* lds, double* cs, int* uv, int* nrot,
                                  int* anyr) {
  return eig_dev<PP>(small, p, warm, lds, cs, uv, nrot, anyr);
}
template <int PP>
__device__ __noinline__ void b_linesearch(const double* PZr, const double* PYr, double* small, int p, double* lds,
                                          Terms& terms, double* smu, int* sok, int* sevals, double* sbmax) {
  linesearch_dev<PP>(PZr, PYr, small, p, lds, terms, smu, sok, sevals, sbmax);
}

// ---------------------------------------------------------------- one problem

struct BatchShared {
  Terms terms;
  double cs[2 * MAXP];
  double red[12];
  double smu, sbmax, beta;
  int uv[MAXP];
  int nrot, anyr, sok, sevals, bad, stop, restart, restart_next, refresh, null_step;
};

template <typename T, int PP>
__device__ __noinline__ void solve_problem(BatchProblem& pr, const BatchCtl& ctl, unsigned char* lds, BatchShared& sh) {
  const int64_t n = pr.n;
  const int p = pr.p;
  T* X = (T*)pr.X;
  T* Y = (T*)pr.Y;
  T* Gb[2] = {(T*)pr.G0, (T*)pr.G1};
  T* Pb[2] = {(T*)pr.P0, (T*)pr.P1};
  T* Z = (T*)pr.Z;
  const T* vals = (const T*)pr.vals;
  double* small = pr.small;
  T* sMat = reinterpret_cast<T*>(lds);
  double* dl = reinterpret_cast<double*>(lds + PP * PP * sizeof(T) + 64);
  double* C = small + S_C * PP * PP;
  double* K = small + S_K * PP * PP;
  double* KD = small + S_KD * PP * PP;
  double* W = small + S_W * PP * PP;
  double* S = small + S_S * PP * PP;
  double* PZ = small + S_PZ * PP * PP;
  double* PY = small + S_PY * PP * PP;
  double* M = small + S_M * PP * PP;
  double* G2 = small + S_T1 * PP * PP;
  const double sqrt_p = sqrt((double)p);
  for (int e = threadIdx.x; e < S_COUNT * PP * PP; e += blockDim.x) small[e] = 0.0;
  pass_barrier();
  // orthonormalize X0: two Cholesky QR passes
  bool ok = true;
  for (int pass = 0; pass < 2 && ok; ++pass) {
    b_gram<T, PP>(n, X, X, nullptr, G2, nullptr);
    pass_barrier();
    ok = b_chol_inv<PP>(G2, M, p, dl, &sh.bad);
    b_load_matrix<T, PP>(sMat, M);
    __syncthreads();
    if (ok) b_product<T, PP>(n, X, sMat);
    pass_barrier();
  }
  if (!ok) {
    if (threadIdx.x == 0) { pr.status = 3; pr.iters = 0; pr.rho = NAN; }
    return;
  }
  // Y = A X, C = sym(X^T Y)
  b_spmm<T, PP>(n, pr.rowptr, pr.colind, vals, X, Y);
  pass_barrier();
  b_gram<T, PP>(n, X, Y, nullptr, G2, nullptr);
  pass_barrier();
  for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) C[e] = 0.5 * (G2[e] + G2[(e % PP) * PP + e / PP]);
  pass_barrier();
  int k = 0, restarts = 0, nulls = 0, k_best = 0;
  double gg_old = 0.0, rho = 0.0, rho_best = 0.0;
  bool v_valid = false;
  if (threadIdx.x == 0) { sh.restart_next = 0; sh.stop = 0; }
  __syncthreads();
  for (;;) {
    const int par = k & 1;
    // gradient pass
    b_load_matrix<T, PP>(sMat, C);
    __syncthreads();
    double gg = 0.0, gdot = 0.0, ginf = 0.0;
    b_grad<T, PP>(n, X, Y, Gb[par ^ 1], Gb[par], sMat, k > 0, gg, gdot, ginf);
    b_reduce3(gg, gdot, ginf, sh.red);
    pass_barrier();
    b_gram<T, PP>(n, X, Gb[par], nullptr, K, nullptr);  // K = X^T G
    pass_barrier();
    rho = sqrt(gg) / (sqrt_p * pr.nA);
    if (k == 0 || rho <= 0.5 * rho_best) { rho_best = rho; k_best = k; }
    int stop = 0;
    if (!isfinite(gg)) stop = 3;
    else if (rho <= ctl.tol) stop = 1;
    else if (k >= ctl.max_iter) stop = 2;
    else if (ctl.stall_window > 0 && k - k_best > ctl.stall_window) stop = 4;
    if (stop) {
      if (threadIdx.x == 0) { pr.status = stop; pr.iters = k; pr.rho = rho; }
      break;
    }
    const bool restart = ctl.method == GSI_RSD || k == 0 || sh.restart_next ||
                         (ctl.k_restart > 0 && k % ctl.k_restart == 0) || !(gg_old > 0.0);
    const double beta = restart ? 0.0 : (gg - gdot) / gg_old;
    for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) KD[e] = K[e] + (restart ? 0.0 : beta * W[e]);
    pass_barrier();
    // direction pass
    b_load_matrix<T, PP>(sMat, KD);
    __syncthreads();
    double gp = 0.0, dz1 = 0.0, dz2 = 0.0;
    b_dir<T, PP>(n, X, Gb[par], Pb[par ^ 1], Pb[par], sMat, (T)beta, !restart, gp);
    b_reduce3(gp, dz1, dz2, sh.red);
    pass_barrier();
    if (!(gp > 0.0)) {
      if (restart) {
        if (threadIdx.x == 0) { pr.status = 3; pr.iters = k; pr.rho = rho; }
        break;
      }
      ++nulls;
      if (threadIdx.x == 0) sh.restart_next = 1;
      __syncthreads();
      continue;
    }
    b_gram<T, PP>(n, Pb[par], Pb[par], nullptr, G2, nullptr);  // S = P^T P
    pass_barrier();
    for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) S[e] = 0.5 * (G2[e] + G2[(e % PP) * PP + e / PP]);
    pass_barrier();
    b_eig<PP>(small, p, v_valid, dl, sh.cs, sh.uv, &sh.nrot, &sh.anyr);
    v_valid = true;
    // SpMM and the line-search Grams
    b_spmm<T, PP>(n, pr.rowptr, pr.colind, vals, Pb[par], Z);
    pass_barrier();
    b_gram<T, PP>(n, Pb[par], Z, Y, PZ, PY);
    pass_barrier();
    b_linesearch<PP>(PZ, PY, small, p, dl, sh.terms, &sh.smu, &sh.sok, &sh.sevals, &sh.sbmax);
    if (!sh.sok) {
      if (restart) {
        if (threadIdx.x == 0) { pr.status = 3; pr.iters = k; pr.rho = rho; }
        break;
      }
      ++nulls;
      if (threadIdx.x == 0) sh.restart_next = 1;
      __syncthreads();
      continue;
    }
    const double mu = sh.smu;
    const bool refresh = ctl.recompute_ax || mu * sqrt(sh.sbmax) <= 1e3 * 2.220446049250313e-16;
    restarts += restart ? 1 : 0;
    // retraction
    b_load_matrix<T, PP>(sMat, M);
    __syncthreads();
    b_update<T, PP>(n, X, Y, Pb[par], Z, sMat, (T)mu, !refresh);
    pass_barrier();
    if (refresh) {
      b_spmm<T, PP>(n, pr.rowptr, pr.colind, vals, X, Y);
      pass_barrier();
      b_gram<T, PP>(n, X, Y, nullptr, G2, nullptr);
      pass_barrier();
      for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) C[e] = 0.5 * (G2[e] + G2[(e % PP) * PP + e / PP]);
      pass_barrier();
    }
    gg_old = gg;
    if (threadIdx.x == 0) sh.restart_next = 0;
    __syncthreads();
    ++k;
  }
  // Rayleigh-Ritz values of the final C (eigenvalues of the operator solved, descending)
  pass_barrier();
  for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) S[e] = C[e];
  pass_barrier();
  b_eig<PP>(small, p, false, dl, sh.cs, sh.uv, &sh.nrot, &sh.anyr);
  if (threadIdx.x == 0) {
    pr.restarts = restarts;
    pr.null_steps = nulls;
  }
  // eig_dev clamps negative eigenvalues at zero (it is written for P^T P): take the Ritz
  // values as diag(V^T C V) with the eigenvectors it returned, sorted descending
  double* V = small + S_V * PP * PP;
  double* T1 = dl;
  wg_mm<PP>(C, false, V, false, T1);
  __syncthreads();
  double* th = T1 + PP * PP;  // LDS scratch for the p Ritz values
  for (int i = threadIdx.x; i < p; i += blockDim.x) {
    double s = 0.0;
    for (int q = 0; q < PP; ++q) s += V[q * PP + i] * T1[q * PP + i];
    th[i] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < p; ++i) {
      const double v = th[i];
      int j = i - 1;
      while (j >= 0 && th[j] < v) { th[j + 1] = th[j]; --j; }
      th[j + 1] = v;
    }
    for (int i = 0; i < p; ++i) pr.ritz[i] = th[i];
  }
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(WG) void k_batched(BatchProblem* __restrict__ probs, BatchCtl* __restrict__ ctl) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ BatchShared sh;
  __shared__ int sidx;
  for (;;) {
    if (threadIdx.x == 0) {
      const int q = atomicAdd(&ctl->next, 1);
      sidx = q < ctl->count ? ctl->order[q] : -1;
    }
    __syncthreads();
    const int idx = sidx;
    __syncthreads();
    if (idx < 0) return;
    BatchProblem pr = probs[idx];
    if (pr.PP == 16)
      solve_problem<T, 16>(pr, *ctl, lds_raw, sh);
    else
      solve_problem<T, 32>(pr, *ctl, lds_raw, sh);
    if (threadIdx.x == 0) {
      probs[idx].iters = pr.iters;
      probs[idx].status = pr.status;
      probs[idx].rho = pr.rho;
      probs[idx].restarts = pr.restarts;
      probs[idx].null_steps = pr.null_steps;
    }
    __syncthreads();
  }
}

__global__ void k_batched_reset(BatchCtl* ctl) {
  if (threadIdx.x == 0) ctl->next = 0;
}

// dynamic LDS: product matrix (PP^2 T) + 64 bytes + 4 PP (PP+1) doubles (Jacobi / line search)
template <typename T>
constexpr int batched_lds() {
  return 32 * 32 * (int)sizeof(T) + 64 + 4 * 32 * 33 * 8;
}

}  // namespace gsi

using namespace gsi;

struct gsi_batch {
  hipStream_t st = nullptr;
  bool own_stream = false;
  int count = 0;
  int fp32 = 1;
  std::vector<void*> allocs;
  BatchProblem* dprobs = nullptr;
  BatchCtl* dctl = nullptr;
  std::vector<BatchProblem> hprobs;
  double* ritz = nullptr;
  std::vector<int64_t> ritz_off;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int grid = 0;
  std::string err;
};

namespace {
template <typename U>
U* balloc(gsi_batch* b, size_t count, hipError_t& e) {
  void* p = nullptr;
  if (e != hipSuccess) return nullptr;
  e = hipMalloc(&p, count * sizeof(U) + 256);
  if (e != hipSuccess) return nullptr;
  b->allocs.push_back(p);
  return reinterpret_cast<U*>(p);
}
}  // namespace

extern "C" {

gsi_status gsi_create_batched(gsi_batch_handle* out, int32_t count, const gsi_csr* A, const int32_t* p,
                              const gsi_options* opt, const double* const* X0, void* stream) {
  if (!out || !A || !p || !opt || !X0 || count < 1) return GSI_EINVAL;
  *out = nullptr;
  gsi_batch* b = new (std::nothrow) gsi_batch();
  if (!b) return GSI_ENOMEM;
  *out = b;
  b->count = count;
  b->fp32 = opt->precision == GSI_MIXED_FP32;
  b->st = reinterpret_cast<hipStream_t>(stream);
  if (!b->st) {
    if (hipStreamCreate(&b->st) != hipSuccess) { b->err = "stream creation failed"; return GSI_EDEVICE; }
    b->own_stream = true;
  }
  if (opt->which != 1 && opt->which != -1) { b->err = "which must be +1 or -1"; return GSI_EINVAL; }
  for (int i = 0; i < count; ++i) {
    if (p[i] < 1 || p[i] > 32 || p[i] >= A[i].n || !A[i].rowptr || !A[i].colind || !A[i].vals || !X0[i]) {
      b->err = "problem " + std::to_string(i) + ": need 1 <= p <= 32, p < n and device arrays";
      return GSI_EINVAL;
    }
    if (A[i].n > INT32_MAX || A[i].nnz > INT32_MAX) { b->err = "n or nnz >= 2^31"; return GSI_EUNSUPPORTED; }
  }
  hipError_t e = hipSuccess;
  const size_t es = b->fp32 ? sizeof(float) : sizeof(double);
  b->hprobs.resize(count);
  int64_t rtot = 0;
  for (int i = 0; i < count; ++i) { b->ritz_off.push_back(rtot); rtot += p[i]; }
  b->ritz = balloc<double>(b, rtot, e);
  int* flags = balloc<int>(b, 4, e);
  double* pmax = balloc<double>(b, 256, e);
  if (e != hipSuccess) { b->err = "allocation failed"; return GSI_ENOMEM; }
  const double sign = opt->which > 0 ? 1.0 : -1.0;
  for (int i = 0; i < count; ++i) {
    BatchProblem& pr = b->hprobs[i];
    memset(&pr, 0, sizeof(pr));
    const int64_t n = A[i].n, nnz = A[i].nnz;
    const int PP = p[i] <= 16 ? 16 : 32;
    const size_t blk = (size_t)((n + TR - 1) / TR * TR) * PP;
    pr.n = n;
    pr.p = p[i];
    pr.PP = PP;
    int32_t* rp = balloc<int32_t>(b, n + 1, e);
    int32_t* ci = balloc<int32_t>(b, nnz, e);
    void* vv = balloc<unsigned char>(b, nnz * es, e);
    void* blocks[7];
    for (int q = 0; q < 7; ++q) blocks[q] = balloc<unsigned char>(b, blk * es, e);
    pr.small = balloc<double>(b, (size_t)S_COUNT * PP * PP, e);
    if (e != hipSuccess) { b->err = "allocation failed"; return GSI_ENOMEM; }
    for (int q = 0; q < 7; ++q) e = e == hipSuccess ? hipMemsetAsync(blocks[q], 0, blk * es, b->st) : e;
    if (e == hipSuccess) e = hipMemcpyAsync(rp, A[i].rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToDevice, b->st);
    if (e == hipSuccess) e = hipMemcpyAsync(ci, A[i].colind, sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice, b->st);
    if (e != hipSuccess) { b->err = std::string("copy: ") + hipGetErrorString(e); return GSI_EDEVICE; }
    // validate and take ||A||_inf
    (void)hipMemsetAsync(flags, 0, 4 * sizeof(int), b->st);
    launch_csr_check(b->st, 256, n, nnz, A[i].rowptr, A[i].colind, A[i].vals, pmax, flags);
    std::vector<double> pm(256);
    int fl = 0;
    (void)hipMemcpyAsync(pm.data(), pmax, 256 * sizeof(double), hipMemcpyDeviceToHost, b->st);
    (void)hipMemcpyAsync(&fl, flags, sizeof(int), hipMemcpyDeviceToHost, b->st);
    e = hipStreamSynchronize(b->st);
    if (e != hipSuccess) { b->err = std::string("validate: ") + hipGetErrorString(e); return GSI_EDEVICE; }
    if (fl) { b->err = "problem " + std::to_string(i) + ": invalid CSR or non-finite values"; return GSI_EINVAL; }
    double nA = 0.0;
    for (double v : pm) nA = v > nA ? v : nA;
    pr.nA = nA;
    if (b->fp32) {
      launch_convert<double, float>(b->st, nnz, A[i].vals, (float*)vv, sign);
      launch_pack<float>(b->st, n, p[i], PP, X0[i], (float*)blocks[0], 1.0);
    } else {
      launch_convert<double, double>(b->st, nnz, A[i].vals, (double*)vv, sign);
      launch_pack<double>(b->st, n, p[i], PP, X0[i], (double*)blocks[0], 1.0);
    }
    pr.rowptr = rp;
    pr.colind = ci;
    pr.vals = vv;
    pr.X = blocks[0]; pr.Y = blocks[1]; pr.G0 = blocks[2]; pr.G1 = blocks[3];
    pr.P0 = blocks[4]; pr.P1 = blocks[5]; pr.Z = blocks[6];
    pr.ritz = b->ritz + b->ritz_off[i];
    pr.status = -1;
  }
  // queue: largest n * p first (longest-processing-time order)
  std::vector<int32_t> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
    return b->hprobs[a].n * b->hprobs[a].p > b->hprobs[c].n * b->hprobs[c].p;
  });
  int32_t* dorder = balloc<int32_t>(b, count, e);
  b->dprobs = balloc<BatchProblem>(b, count, e);
  b->dctl = balloc<BatchCtl>(b, 1, e);
  if (e != hipSuccess) { b->err = "allocation failed"; return GSI_ENOMEM; }
  BatchCtl ctl;
  memset(&ctl, 0, sizeof(ctl));
  ctl.count = count;
  ctl.method = opt->method;
  ctl.k_restart = opt->k_restart;
  ctl.max_iter = opt->max_iter;
  ctl.stall_window = b->fp32 ? 200 : 0;
  ctl.recompute_ax = opt->recompute_ax;
  ctl.tol = opt->tol;
  ctl.order = dorder;
  e = hipMemcpyAsync(dorder, order.data(), sizeof(int32_t) * count, hipMemcpyHostToDevice, b->st);
  if (e == hipSuccess) e = hipMemcpyAsync(b->dctl, &ctl, sizeof(ctl), hipMemcpyHostToDevice, b->st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->dprobs, b->hprobs.data(), sizeof(BatchProblem) * count, hipMemcpyHostToDevice, b->st);
  if (e == hipSuccess) e = hipStreamSynchronize(b->st);
  if (e != hipSuccess) { b->err = std::string("upload: ") + hipGetErrorString(e); return GSI_EDEVICE; }
  // persistent grid: enough workgroups to fill the device, never more than the problems
  const int lds = b->fp32 ? batched_lds<float>() : batched_lds<double>();
  const void* kern = b->fp32 ? reinterpret_cast<const void*>(k_batched<float>)
                             : reinterpret_cast<const void*>(k_batched<double>);
  e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  int per_cu = 1;
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, WG, lds);
  int dev = 0, ncu = 256;
  hipDeviceProp_t prop;
  (void)hipGetDevice(&dev);
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0) ncu = prop.multiProcessorCount;
  if (e != hipSuccess) { b->err = std::string("kernel attributes: ") + hipGetErrorString(e); return GSI_EDEVICE; }
  b->grid = std::max(1, std::min(count, ncu * std::max(per_cu, 1)));
  return GSI_OK;
}

gsi_status gsi_solve_batched(gsi_batch_handle b, int32_t* iters, int32_t* status) {
  if (!b) return GSI_EINVAL;
  hipError_t e = hipSuccess;
  if (!b->gexec) {
    // one graph: reset the queue head (a kernel, not a memset), then the persistent solve
    e = hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      k_batched_reset<<<1, 64, 0, b->st>>>(b->dctl);
      const int lds = b->fp32 ? batched_lds<float>() : batched_lds<double>();
      if (b->fp32)
        k_batched<float><<<b->grid, WG, lds, b->st>>>(b->dprobs, b->dctl);
      else
        k_batched<double><<<b->grid, WG, lds, b->st>>>(b->dprobs, b->dctl);
      e = hipStreamEndCapture(b->st, &b->graph);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) { b->err = std::string("graph: ") + hipGetErrorString(e); return GSI_EDEVICE; }
  }
  e = hipGraphLaunch(b->gexec, b->st);
  if (e == hipSuccess) e = hipStreamSynchronize(b->st);
  if (e != hipSuccess) { b->err = std::string("solve: ") + hipGetErrorString(e); return GSI_EDEVICE; }
  std::vector<BatchProblem> res(b->count);
  e = hipMemcpy(res.data(), b->dprobs, sizeof(BatchProblem) * b->count, hipMemcpyDeviceToHost);
  if (e != hipSuccess) { b->err = std::string("results: ") + hipGetErrorString(e); return GSI_EDEVICE; }
  gsi_status s = GSI_OK;
  for (int i = 0; i < b->count; ++i) {
    if (iters) iters[i] = res[i].iters;
    if (status) status[i] = res[i].status;
    if (res[i].status == 2 && s == GSI_OK) s = GSI_NOT_CONVERGED;
    if (res[i].status == 3) s = GSI_BREAKDOWN;
  }
  return s;
}

gsi_status gsi_batched_results(gsi_batch_handle b, int32_t i, double* ritz, double* rho, int32_t* restarts) {
  if (!b || i < 0 || i >= b->count) return GSI_EINVAL;
  BatchProblem pr;
  hipError_t e = hipMemcpy(&pr, b->dprobs + i, sizeof(pr), hipMemcpyDeviceToHost);
  if (e == hipSuccess && ritz) e = hipMemcpy(ritz, pr.ritz, sizeof(double) * pr.p, hipMemcpyDeviceToHost);
  if (e != hipSuccess) { b->err = std::string("results: ") + hipGetErrorString(e); return GSI_EDEVICE; }
  if (rho) *rho = pr.rho;
  if (restarts) *restarts = pr.restarts;
  return GSI_OK;
}

gsi_status gsi_batched_get_x(gsi_batch_handle b, int32_t i, double* X_out) {
  if (!b || !X_out || i < 0 || i >= b->count) return GSI_EINVAL;
  const BatchProblem& pr = b->hprobs[i];
  if (b->fp32)
    launch_unpack<float>(b->st, pr.n, pr.p, pr.PP, (const float*)pr.X, X_out);
  else
    launch_unpack<double>(b->st, pr.n, pr.p, pr.PP, (const double*)pr.X, X_out);
  hipError_t e = hipStreamSynchronize(b->st);
  if (e != hipSuccess) { b->err = std::string("get_x: ") + hipGetErrorString(e); return GSI_EDEVICE; }
  return GSI_OK;
}

const char* gsi_batched_last_error(gsi_batch_handle b) { return b ? b->err.c_str() : "null handle"; }

void gsi_destroy_batched(gsi_batch_handle b) {
  if (!b) return;
  if (b->st) (void)hipStreamSynchronize(b->st);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (void* p : b->allocs) (void)hipFree(p);
  if (b->own_stream) (void)hipStreamDestroy(b->st);
  delete b;
}

}  // extern "C"
