// Streaming kernels over the tall n x p blocks: the fused gradient, direction and
// retraction passes, the block SpMM with its Gram epilogue, generic Gram / product
// passes and the fixed-order reduction of per-workgroup partial sums.
//
// Every multi-workgroup kernel writes per-workgroup partial sums (Gram matrices and
// scalars) to partials[blockIdx.x * nv + ...]; k_reduce sums them in a fixed order, so
// results are bitwise reproducible run to run.
#include "gsi_kernels.h"

namespace gsi {

template <typename T, int PP>
__device__ __forceinline__ void load_matrix_lds(T* __restrict__ sM, const double* __restrict__ M) {
  for (int i = threadIdx.x; i < PP * PP; i += WG) sM[i] = (T)M[i];
}

// ---------------------------------------------------------------- gradient pass
// G = -(Y - X C) (Sec. 3.1, eq. gradPhi) with C = X^T A X, fused with
//   <G, G>, <G_old, G>, ||G||_inf (max absolute row sum) and the Gram K = X^T G
// (the tangent-space defect of G, removed from the direction in the next pass).
// Partials: K (PP*PP), <G,G>, <G_old,G>, ||G||_inf.
template <typename T, int PP>
__global__ __launch_bounds__(WG) void k_grad(int64_t n, const T* __restrict__ X, const T* __restrict__ Y,
                                             T* __restrict__ G0, T* __restrict__ G1,
                                             const double* __restrict__ small, const Scalars* __restrict__ sc,
                                             double* __restrict__ partials) {
  if (sc->done) return;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* sC = reinterpret_cast<T*>(lds_raw);
  T* sX = sC + PP * PP;
  T* sG = sX + TR * PP;
  __shared__ double red[4 * 3];
  const int par = sc->k & 1;
  T* G = par ? G1 : G0;
  const T* Gold = par ? G0 : G1;
  const bool have_old = sc->k > 0;
  load_matrix_lds<T, PP>(sC, small + S_C * PP * PP);
  __syncthreads();
  const int w = threadIdx.x >> 6;
  const int64_t ntiles = (n + TR - 1) / TR;
  int64_t t0, t1;
  tile_range(ntiles, t0, t1);
  typename Vec4<T>::type kacc[GramSplit<PP>::PER_WAVE];
  gram_zero<T, PP>(kacc);
  double gg = 0.0, gdot = 0.0, ginf = 0.0;
  for (int64_t t = t0; t < t1; ++t) {
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
    T x[PP / 16][4];
    load_rl<T, PP>(X, row0, n, x);
    rl_to_lds<T, PP>(sX, x);
    rl_to_lds<T, PP>(sG, g);
    __syncthreads();
    gram_tile<T, PP>(sX, sG, kacc);
    __syncthreads();
  }
  const int64_t nv = PP * PP + 3;
  double* out = partials + (int64_t)blockIdx.x * nv;
  gram_store<T, PP>(out, kacc);
  // scalars: sums for gg, gdot; max for ginf
  {
    const int l = threadIdx.x & 63;
    double s0 = wave_sum(gg), s1 = wave_sum(gdot), s2 = wave_max(ginf);
    if (l == 0) { red[w * 3 + 0] = s0; red[w * 3 + 1] = s1; red[w * 3 + 2] = s2; }
    __syncthreads();
    if (threadIdx.x == 0) {
      out[PP * PP + 0] = red[0] + red[3] + red[6] + red[9];
      out[PP * PP + 1] = red[1] + red[4] + red[7] + red[10];
      out[PP * PP + 2] = fmax(fmax(red[2], red[5]), fmax(red[8], red[11]));
    }
  }
}

// ---------------------------------------------------------------- direction pass
// P = (I - X X^T)(G + beta P_old) = G + beta P_old - X (K + beta W)   (Sec. 5.1, eq. Pnew,
// projected onto the tangent space as in Algorithm 4), fused with <G, P> and S = P^T P.
// Partials: S (PP*PP), <G,P>.
template <typename T, int PP>
__global__ __launch_bounds__(WG) void k_dir(int64_t n, const T* __restrict__ X, const T* __restrict__ G0,
                                            const T* __restrict__ G1, T* __restrict__ P0, T* __restrict__ P1,
                                            const double* __restrict__ small, const Scalars* __restrict__ sc,
                                            double* __restrict__ partials) {
  if (sc->done) return;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* sK = reinterpret_cast<T*>(lds_raw);
  T* sP = sK + PP * PP;
  __shared__ double red[4];
  const int par = sc->k & 1;
  const T* G = par ? G1 : G0;
  T* P = par ? P1 : P0;
  const T* Pold = par ? P0 : P1;
  const T beta = (T)sc->beta_pr;
  const bool use_old = sc->beta_pr != 0.0;
  load_matrix_lds<T, PP>(sK, small + S_KD * PP * PP);
  __syncthreads();
  const int w = threadIdx.x >> 6;
  const int64_t ntiles = (n + TR - 1) / TR;
  int64_t t0, t1;
  tile_range(ntiles, t0, t1);
  typename Vec4<T>::type sacc[GramSplit<PP>::PER_WAVE];
  gram_zero<T, PP>(sacc);
  double gp = 0.0;
  for (int64_t t = t0; t < t1; ++t) {
    const int64_t row0 = t * TR + 16 * w;
    T a[PP / 4];
    load_al<T, PP>(X, row0, n, a);
    typename Vec4<T>::type acc[PP / 16];
    zero_acc<T, PP>(acc);
    product<T, PP>(a, sK, acc);
    T g[PP / 16][4], p[PP / 16][4];
    load_rl<T, PP>(G, row0, n, g);
    if (use_old) {
      load_rl<T, PP>(Pold, row0, n, p);
#pragma unroll
      for (int cb = 0; cb < PP / 16; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) p[cb][r] = g[cb][r] + beta * p[cb][r] - acc[cb][r];
    } else {
#pragma unroll
      for (int cb = 0; cb < PP / 16; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) p[cb][r] = g[cb][r] - acc[cb][r];
    }
    store_rl<T, PP>(P, row0, n, p);
#pragma unroll
    for (int cb = 0; cb < PP / 16; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) gp += (double)g[cb][r] * (double)p[cb][r];
    rl_to_lds<T, PP>(sP, p);
    __syncthreads();
    gram_tile<T, PP>(sP, sP, sacc);
    __syncthreads();
  }
  const int64_t nv = PP * PP + 1;
  double* out = partials + (int64_t)blockIdx.x * nv;
  gram_store<T, PP>(out, sacc);
  const int l = threadIdx.x & 63;
  double s = wave_sum(gp);
  if (l == 0) red[w] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[PP * PP] = red[0] + red[1] + red[2] + red[3];
}

// ---------------------------------------------------------------- retraction pass
// X <- (X - mu P) M and Y <- (Y - mu Z) M with M = V D_mu^{-1} V^T (Sec. 5.2, eq. Xnew_P;
// Sec. 6.1, eq. save_matvec). In place. When the state asks for an explicit A X the Y
// update is skipped (Y is formed by the SpMM that follows). With GRAMS the pass also
// accumulates X^T Y and X^T P of the new X (partials: 2 PP*PP).
template <typename T, int PP, bool GRAMS>
__global__ __launch_bounds__(WG) void k_update(int64_t n, T* __restrict__ X, T* __restrict__ Y,
                                               const T* __restrict__ P0, const T* __restrict__ P1,
                                               const T* __restrict__ Z, const double* __restrict__ small,
                                               const Scalars* __restrict__ sc, double* __restrict__ partials) {
  if (sc->done || sc->null_step) return;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* sM = reinterpret_cast<T*>(lds_raw);
  T* sX = sM + PP * PP;
  T* sY = sX + TR * PP;
  T* sP = sY + TR * PP;
  const int par = (sc->k - 1) & 1;  // the step was accepted: k already counts it
  const T* P = par ? P1 : P0;
  const T mu = (T)sc->mu;
  const bool upd_y = !sc->refresh;
  load_matrix_lds<T, PP>(sM, small + S_M * PP * PP);
  __syncthreads();
  const int w = threadIdx.x >> 6;
  const int64_t ntiles = (n + TR - 1) / TR;
  int64_t t0, t1;
  tile_range(ntiles, t0, t1);
  typename Vec4<T>::type cacc[GRAMS ? GramSplit<PP>::PER_WAVE : 1], wacc[GRAMS ? GramSplit<PP>::PER_WAVE : 1];
  if constexpr (GRAMS) {
    gram_zero<T, PP>(cacc);
    gram_zero<T, PP>(wacc);
  }
  for (int64_t t = t0; t < t1; ++t) {
    const int64_t row0 = t * TR + 16 * w;
    T a1[PP / 4], a2[PP / 4], b[PP / 4];
    load_al<T, PP>(X, row0, n, a1);
    load_al<T, PP>(P, row0, n, b);
#pragma unroll
    for (int s = 0; s < PP / 4; ++s) a1[s] = a1[s] - mu * b[s];
    typename Vec4<T>::type xacc[PP / 16], yacc[PP / 16];
    zero_acc<T, PP>(xacc);
    if (upd_y) {
      load_al<T, PP>(Y, row0, n, a2);
      load_al<T, PP>(Z, row0, n, b);
#pragma unroll
      for (int s = 0; s < PP / 4; ++s) a2[s] = a2[s] - mu * b[s];
      zero_acc<T, PP>(yacc);
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
        yo[cb][r] = upd_y ? yacc[cb][r] : T(0);
      }
    store_rl<T, PP>(X, row0, n, xo);
    if (upd_y) store_rl<T, PP>(Y, row0, n, yo);
    if constexpr (GRAMS) {
      T pv[PP / 16][4];
      load_rl<T, PP>(P, row0, n, pv);
      rl_to_lds<T, PP>(sX, xo);
      rl_to_lds<T, PP>(sY, yo);
      rl_to_lds<T, PP>(sP, pv);
      __syncthreads();
      gram_tile<T, PP>(sX, sY, cacc);
      gram_tile<T, PP>(sX, sP, wacc);
      __syncthreads();
    }
  }
  if constexpr (GRAMS) {
    double* out = partials + (int64_t)blockIdx.x * (2 * PP * PP);
    gram_store<T, PP>(out, cacc);
    gram_store<T, PP>(out + PP * PP, wacc);
  }
}

// ---------------------------------------------------------------- block SpMM
// Z = A_op W for a full symmetric CSR, W and Z row-major n x PP. A row is handled by
// LPR = PP / 4 lanes, each owning 4 consecutive columns. Optional Gram epilogue over the
// workgroup's TR rows: W^T Z and (if Y3 != nullptr) W^T Y3. Partials: 1 or 2 PP*PP.
// sel: which buffers to use: 0 = fixed (W, Z as given), 1 = W is P of the current
// iteration (picked by parity from W/W1), for the iteration's SpMM.
template <typename T, int PP, bool GRAMS>
__global__ __launch_bounds__(WG) void k_spmm(int64_t n, const int32_t* __restrict__ rowptr,
                                             const int32_t* __restrict__ colind, const T* __restrict__ vals,
                                             const T* __restrict__ W0, const T* __restrict__ W1, T* __restrict__ Z,
                                             const T* __restrict__ Y3, const Scalars* __restrict__ sc, int mode,
                                             double* __restrict__ partials) {
  // mode 0: always run, W = W0. mode 1: iteration SpMM (skip when done / null step),
  // W = P of the current iteration. mode 2: refresh A X (run only when sc->refresh).
  if (mode == 1 && (sc->done || sc->null_step)) return;
  if (mode == 2 && (sc->done || sc->null_step || !sc->refresh)) return;
  const T* W = W0;
  if (mode == 1) W = ((sc->k & 1) ? W1 : W0);
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* sW = reinterpret_cast<T*>(lds_raw);
  T* sZ = sW + TR * PP;
  T* sY = sZ + TR * PP;
  constexpr int EPL = 4;
  constexpr int LPR = PP / EPL;       // lanes per row
  constexpr int RPW = 64 / LPR;       // rows per wave pass
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int sub = l / LPR, lane = l % LPR;
  const int64_t ntiles = (n + TR - 1) / TR;
  int64_t t0, t1;
  tile_range(ntiles, t0, t1);
  typename Vec4<T>::type zacc[GRAMS ? GramSplit<PP>::PER_WAVE : 1], yacc[GRAMS ? GramSplit<PP>::PER_WAVE : 1];
  if constexpr (GRAMS) {
    gram_zero<T, PP>(zacc);
    gram_zero<T, PP>(yacc);
  }
  for (int64_t t = t0; t < t1; ++t) {
#pragma unroll
    for (int pass = 0; pass < 16 / RPW; ++pass) {
      const int lrow = 16 * w + pass * RPW + sub;
      const int64_t row = t * TR + lrow;
      T acc[EPL] = {T(0), T(0), T(0), T(0)};
      if (row < n) {
        const int32_t j0 = rowptr[row], j1 = rowptr[row + 1];
        int32_t j = j0;
        for (; j + 1 < j1; j += 2) {
          const int32_t ca = colind[j], cbb = colind[j + 1];
          const T va = vals[j], vb = vals[j + 1];
          const T* pa = W + (int64_t)ca * PP + EPL * lane;
          const T* pb = W + (int64_t)cbb * PP + EPL * lane;
#pragma unroll
          for (int e = 0; e < EPL; ++e) acc[e] += va * pa[e];
#pragma unroll
          for (int e = 0; e < EPL; ++e) acc[e] += vb * pb[e];
        }
        if (j < j1) {
          const int32_t ca = colind[j];
          const T va = vals[j];
          const T* pa = W + (int64_t)ca * PP + EPL * lane;
#pragma unroll
          for (int e = 0; e < EPL; ++e) acc[e] += va * pa[e];
        }
        T* zr = Z + row * PP + EPL * lane;
#pragma unroll
        for (int e = 0; e < EPL; ++e) zr[e] = acc[e];
      }
      if constexpr (GRAMS) {
#pragma unroll
        for (int e = 0; e < EPL; ++e) sZ[lrow * PP + EPL * lane + e] = acc[e];
      }
    }
    if constexpr (GRAMS) {
      // own rows of W (and Y3) into LDS
      for (int i = threadIdx.x; i < TR * PP; i += WG) {
        const int64_t row = t * TR + i / PP;
        sW[i] = row < n ? W[row * PP + (i % PP)] : T(0);
        if (Y3) sY[i] = row < n ? Y3[row * PP + (i % PP)] : T(0);
      }
      __syncthreads();
      gram_tile<T, PP>(sW, sZ, zacc);
      if (Y3) gram_tile<T, PP>(sW, sY, yacc);
      __syncthreads();
    }
  }
  if constexpr (GRAMS) {
    const int64_t nv = (Y3 ? 2 : 1) * PP * PP;
    double* out = partials + (int64_t)blockIdx.x * nv;
    gram_store<T, PP>(out, zacc);
    if (Y3) gram_store<T, PP>(out + PP * PP, yacc);
  }
}

// ---------------------------------------------------------------- generic passes
// Partials of A^T B (PP*PP per workgroup).
template <typename T, int PP>
__global__ __launch_bounds__(WG) void k_gram(int64_t n, const T* __restrict__ A, const T* __restrict__ B,
                                             double* __restrict__ partials) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* sA = reinterpret_cast<T*>(lds_raw);
  T* sB = sA + TR * PP;
  const int w = threadIdx.x >> 6;
  const int64_t ntiles = (n + TR - 1) / TR;
  int64_t t0, t1;
  tile_range(ntiles, t0, t1);
  typename Vec4<T>::type acc[GramSplit<PP>::PER_WAVE];
  gram_zero<T, PP>(acc);
  for (int64_t t = t0; t < t1; ++t) {
    const int64_t row0 = t * TR + 16 * w;
    T a[PP / 16][4], b[PP / 16][4];
    load_rl<T, PP>(A, row0, n, a);
    load_rl<T, PP>(B, row0, n, b);
    rl_to_lds<T, PP>(sA, a);
    rl_to_lds<T, PP>(sB, b);
    __syncthreads();
    gram_tile<T, PP>(sA, sB, acc);
    __syncthreads();
  }
  gram_store<T, PP>(partials + (int64_t)blockIdx.x * PP * PP, acc);
}

// OUT = IN M (M from the small buffer, PP x PP). IN and OUT may alias.
template <typename T, int PP>
__global__ __launch_bounds__(WG) void k_product(int64_t n, const T* IN, T* OUT, const double* __restrict__ M) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* sM = reinterpret_cast<T*>(lds_raw);
  load_matrix_lds<T, PP>(sM, M);
  __syncthreads();
  const int w = threadIdx.x >> 6;
  const int64_t ntiles = (n + TR - 1) / TR;
  int64_t t0, t1;
  tile_range(ntiles, t0, t1);
  for (int64_t t = t0; t < t1; ++t) {
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
    store_rl<T, PP>(OUT, row0, n, o);
  }
}

// Column sums of squares of R = Y - X diag(theta): per-workgroup partials (PP).
template <typename T, int PP>
__global__ __launch_bounds__(WG) void k_colres(int64_t n, const T* __restrict__ X, const T* __restrict__ Y,
                                               const double* __restrict__ theta, double* __restrict__ partials) {
  __shared__ double red[WG];
  const int col = threadIdx.x % PP;
  const int rows_per = WG / PP;
  const int64_t ntiles = (n + TR - 1) / TR;
  int64_t t0, t1;
  tile_range(ntiles, t0, t1);
  double s = 0.0;
  const double th = theta[col];
  for (int64_t row = t0 * TR + threadIdx.x / PP; row < t1 * TR && row < n; row += rows_per) {
    const double r = (double)Y[row * PP + col] - th * (double)X[row * PP + col];
    s += r * r;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < PP) {
    double tot = 0.0;
    for (int k = threadIdx.x; k < WG; k += PP) tot += red[k];
    partials[(int64_t)blockIdx.x * PP + threadIdx.x] = tot;
  }
}

// ---------------------------------------------------------------- reduction
// out[v] = sum_b partials[b * nv + v] (fixed order) for v < max_from, max over b otherwise.
// cond: 0 always; 1 skip when the solve is done or the step is null; 2 run only when an
// explicit A X refresh was requested; 3 skip when the solve is done.
__global__ __launch_bounds__(WG) void k_reduce(const double* __restrict__ partials, int nb, int64_t nv,
                                               int64_t max_from, double* __restrict__ out,
                                               const Scalars* __restrict__ sc, int cond) {
  if (cond == 1 && (sc->done || sc->null_step)) return;
  if (cond == 2 && (sc->done || sc->null_step || !sc->refresh)) return;
  if (cond == 3 && sc->done) return;
  const int64_t v = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (v >= nv) return;
  double s = 0.0;
  if (v < max_from) {
    for (int b = 0; b < nb; ++b) s += partials[(int64_t)b * nv + v];
  } else {
    for (int b = 0; b < nb; ++b) s = fmax(s, partials[(int64_t)b * nv + v]);
  }
  out[v] = s;
}

// ---------------------------------------------------------------- packing and checks
// dst (n x PP, T) <- scale * src (n x p, double); padding columns zero.
template <typename T>
__global__ void k_pack(int64_t n, int p, int PP, const double* __restrict__ src, T* __restrict__ dst, double scale) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * PP) return;
  const int64_t row = i / PP;
  const int col = (int)(i % PP);
  dst[i] = col < p ? (T)(scale * src[row * p + col]) : T(0);
}

template <typename T>
__global__ void k_unpack(int64_t n, int p, int PP, const T* __restrict__ src, double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * p) return;
  dst[i] = (double)src[(i / p) * PP + (i % p)];
}

template <typename TS, typename TD>
__global__ void k_convert(int64_t count, const TS* __restrict__ src, TD* __restrict__ dst, double scale) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = (TD)(scale * (double)src[i]);
}

// CSR checks and ||A||_inf: partial max of absolute row sums per workgroup, error flags:
// bit 0 rowptr not monotone / out of range, bit 1 column index out of range, bit 2
// non-finite value, bit 3 columns not sorted within a row.
__global__ void k_csr_check(int64_t n, int64_t nnz, const int32_t* __restrict__ rowptr,
                            const int32_t* __restrict__ colind, const double* __restrict__ vals,
                            double* __restrict__ partial_max, int* __restrict__ flags) {
  __shared__ double red[WG];
  double m = 0.0;
  int f = 0;
  for (int64_t row = (int64_t)blockIdx.x * WG + threadIdx.x; row < n; row += (int64_t)gridDim.x * WG) {
    const int64_t j0 = rowptr[row], j1 = rowptr[row + 1];
    if (j1 < j0 || j0 < 0 || j1 > nnz) { f |= 1; continue; }
    double s = 0.0;
    int32_t prev = -1;
    for (int64_t j = j0; j < j1; ++j) {
      const int32_t c = colind[j];
      if (c < 0 || c >= n) f |= 2;
      if (c <= prev) f |= 8;
      prev = c;
      const double v = vals[j];
      if (!isfinite(v)) f |= 4;
      s += fabs(v);
    }
    m = fmax(m, s);
  }
  if (f) atomicOr(flags, f);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = WG / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial_max[blockIdx.x] = red[0];
}

// Non-finite check of a dense block: sets flags bit 0.
__global__ void k_finite(int64_t count, const double* __restrict__ x, int* __restrict__ flags) {
  int f = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(x[i])) f = 1;
  if (f) atomicOr(flags, 1);
}

// ---------------------------------------------------------------- launchers

template <typename T, int PP>
int lds_bytes(Pass pass) {
  const int m = PP * PP * (int)sizeof(T), tile = TR * PP * (int)sizeof(T);
  switch (pass) {
    case Pass::Grad: return m + 2 * tile;
    case Pass::Dir: return m + tile;
    case Pass::Update: return m;
    case Pass::UpdateGrams: return m + 3 * tile;
    case Pass::Spmm: return 3 * tile;
    case Pass::SpmmPlain: return 0;
    case Pass::Gram: return 2 * tile;
    case Pass::Product: return m;
  }
  return 0;
}

template <typename T, int PP>
hipError_t set_lds_limits() {
  hipError_t e = hipSuccess;
#define GSI_SET(kern, pass)                                                                                       \
  if (e == hipSuccess)                                                                                            \
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, \
                            lds_bytes<T, PP>(pass));
  GSI_SET((k_grad<T, PP>), Pass::Grad)
  GSI_SET((k_dir<T, PP>), Pass::Dir)
  GSI_SET((k_update<T, PP, false>), Pass::Update)
  GSI_SET((k_update<T, PP, true>), Pass::UpdateGrams)
  GSI_SET((k_spmm<T, PP, true>), Pass::Spmm)
  GSI_SET((k_gram<T, PP>), Pass::Gram)
  GSI_SET((k_product<T, PP>), Pass::Product)
#undef GSI_SET
  return e;
}

template <typename T, int PP>
void Kernels<T, PP>::grad(hipStream_t st, int nb, int64_t n, const T* X, const T* Y, T* G0, T* G1,
                          const double* small, const Scalars* sc, double* partials) {
  k_grad<T, PP><<<nb, WG, lds_bytes<T, PP>(Pass::Grad), st>>>(n, X, Y, G0, G1, small, sc, partials);
}
template <typename T, int PP>
void Kernels<T, PP>::dir(hipStream_t st, int nb, int64_t n, const T* X, const T* G0, const T* G1, T* P0, T* P1,
                         const double* small, const Scalars* sc, double* partials) {
  k_dir<T, PP><<<nb, WG, lds_bytes<T, PP>(Pass::Dir), st>>>(n, X, G0, G1, P0, P1, small, sc, partials);
}
template <typename T, int PP>
void Kernels<T, PP>::update(hipStream_t st, int nb, int64_t n, T* X, T* Y, const T* P0, const T* P1, const T* Z,
                            const double* small, const Scalars* sc, double* partials, bool grams) {
  if (grams)
    k_update<T, PP, true><<<nb, WG, lds_bytes<T, PP>(Pass::UpdateGrams), st>>>(n, X, Y, P0, P1, Z, small, sc, partials);
  else
    k_update<T, PP, false><<<nb, WG, lds_bytes<T, PP>(Pass::Update), st>>>(n, X, Y, P0, P1, Z, small, sc, partials);
}
template <typename T, int PP>
void Kernels<T, PP>::spmm(hipStream_t st, int nb, int64_t n, const int32_t* rowptr, const int32_t* colind,
                          const T* vals, const T* W0, const T* W1, T* Z, const T* Y3, const Scalars* sc, int mode,
                          bool grams, double* partials) {
  if (grams)
    k_spmm<T, PP, true><<<nb, WG, lds_bytes<T, PP>(Pass::Spmm), st>>>(n, rowptr, colind, vals, W0, W1, Z, Y3, sc, mode, partials);
  else
    k_spmm<T, PP, false><<<nb, WG, 0, st>>>(n, rowptr, colind, vals, W0, W1, Z, Y3, sc, mode, partials);
}
template <typename T, int PP>
void Kernels<T, PP>::gram(hipStream_t st, int nb, int64_t n, const T* A, const T* B, double* partials) {
  k_gram<T, PP><<<nb, WG, lds_bytes<T, PP>(Pass::Gram), st>>>(n, A, B, partials);
}
template <typename T, int PP>
void Kernels<T, PP>::product(hipStream_t st, int nb, int64_t n, const T* IN, T* OUT, const double* M) {
  k_product<T, PP><<<nb, WG, lds_bytes<T, PP>(Pass::Product), st>>>(n, IN, OUT, M);
}
template <typename T, int PP>
void Kernels<T, PP>::colres(hipStream_t st, int nb, int64_t n, const T* X, const T* Y, const double* theta,
                            double* partials) {
  k_colres<T, PP><<<nb, WG, 0, st>>>(n, X, Y, theta, partials);
}
template <typename T, int PP>
hipError_t Kernels<T, PP>::init() {
  return set_lds_limits<T, PP>();
}

void launch_reduce(hipStream_t st, const double* partials, int nb, int64_t nv, int64_t max_from, double* out,
                   const Scalars* sc, int cond) {
  const int blocks = (int)((nv + WG - 1) / WG);
  hipLaunchKernelGGL(k_reduce, dim3(blocks), dim3(WG), 0, st, partials, nb, nv, max_from, out, sc, cond);
}

// small[slot] = sym(red) (PP x PP), the projected matrix after an explicit Gram.
__global__ void k_set_sym(int PP, const double* __restrict__ red, double* __restrict__ dst) {
  for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) {
    const int i = e / PP, j = e % PP;
    dst[e] = 0.5 * (red[i * PP + j] + red[j * PP + i]);
  }
}
void launch_set_sym(hipStream_t st, int PP, const double* red, double* dst) {
  hipLaunchKernelGGL(k_set_sym, dim3(1), dim3(WG), 0, st, PP, red, dst);
}

template <typename T>
void launch_pack(hipStream_t st, int64_t n, int p, int PP, const double* src, T* dst, double scale) {
  const int64_t total = n * PP;
  hipLaunchKernelGGL((k_pack<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, n, p, PP, src, dst, scale);
}
template <typename T>
void launch_unpack(hipStream_t st, int64_t n, int p, int PP, const T* src, double* dst) {
  const int64_t total = n * p;
  hipLaunchKernelGGL((k_unpack<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, n, p, PP, src, dst);
}
template <typename TS, typename TD>
void launch_convert(hipStream_t st, int64_t count, const TS* src, TD* dst, double scale) {
  hipLaunchKernelGGL((k_convert<TS, TD>), dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count, src, dst,
                     scale);
}
void launch_csr_check(hipStream_t st, int nb, int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colind,
                      const double* vals, double* partial_max, int* flags) {
  hipLaunchKernelGGL(k_csr_check, dim3(nb), dim3(WG), 0, st, n, nnz, rowptr, colind, vals, partial_max, flags);
}
void launch_finite(hipStream_t st, int64_t count, const double* x, int* flags) {
  hipLaunchKernelGGL(k_finite, dim3(1024), dim3(256), 0, st, count, x, flags);
}

template struct Kernels<double, 16>;
template struct Kernels<double, 32>;
template struct Kernels<double, 64>;
template struct Kernels<float, 16>;
template struct Kernels<float, 32>;
template struct Kernels<float, 64>;
template void launch_pack<double>(hipStream_t, int64_t, int, int, const double*, double*, double);
template void launch_pack<float>(hipStream_t, int64_t, int, int, const double*, float*, double);
template void launch_unpack<double>(hipStream_t, int64_t, int, int, const double*, double*);
template void launch_unpack<float>(hipStream_t, int64_t, int, int, const float*, double*);
template void launch_convert<float, double>(hipStream_t, int64_t, const float*, double*, double);
template void launch_convert<double, float>(hipStream_t, int64_t, const double*, float*, double);
template void launch_convert<double, double>(hipStream_t, int64_t, const double*, double*, double);

}  // namespace gsi
