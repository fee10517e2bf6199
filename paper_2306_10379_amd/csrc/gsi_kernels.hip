// Streaming kernels over the tall n x p blocks: the fused gradient, direction and
// retraction passes, the block SpMM (CSR in float64, float32 or bfloat16, the filter step
// of subspace iteration, the matrix-free stencil), the Gram and product passes and the
// fixed-order reduction of per-workgroup partial sums.
//
// Every multi-workgroup kernel writes per-workgroup partial sums (Gram matrices and
// scalars) to partials[blockIdx.x * nv + ...]; k_reduce sums them in a fixed order, so
// results are bitwise reproducible run to run.
#include <type_traits>

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
// Partials: K (PP*PP), <G,G>, <G_old,G>, ||G||_inf. The tall blocks hold a whole number of
// TR-row tiles (rows n .. are zero), so the Gram may read the last tile in full.
template <typename T, int PP>
__global__ __launch_bounds__(WG) void k_grad(int64_t n, const T* __restrict__ X, const T* __restrict__ Y,
                                             T* __restrict__ G0, T* __restrict__ G1,
                                             const double* __restrict__ small, const Scalars* __restrict__ sc,
                                             double* __restrict__ partials, int cond) {
  if (sc->done) return;
  if (cond == GRAD_PENDING && sc->grad_ready) return;
  // the p x p factor in LDS (a wider one runs k_grad_wide)
  static_assert(!factor_wide<T, PP>(), "k_grad_wide takes this width");
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* sC = reinterpret_cast<T*>(lds_raw);
  T* sG = sC + PP * PP;
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
  // at PP = 64 each wave owns column block w of X in the Gram: its 64 x 16 slice of the
  // tile is loaded at the top of the tile, so the loads overlap the product (K^T blocks
  // (q, w) = G^T X are accumulated and stored transposed)
  constexpr bool XCOL = (PP == 64);
  const int lg = (threadIdx.x & 63) >> 4, lc = threadIdx.x & 15;
  for (int64_t t = t0; t < t1; ++t) {
    const int64_t row0 = t * TR + 16 * w;
    T xcol[XCOL ? TR / 4 : 1];
    if constexpr (XCOL) {
#pragma unroll
      for (int s = 0; s < TR / 4; ++s) xcol[s] = gld(X + (t * TR + 4 * s + lg) * PP + 16 * w + lc);
    }
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
    // K += X^T G over the tile: X straight from memory (its rows were just read, and the
    // tall blocks are allocated with whole tiles of zero rows), G through LDS
    rl_to_lds<T, PP>(sG, g);
    __syncthreads();
    if constexpr (XCOL) {
#pragma unroll
      for (int s = 0; s < TR / 4; ++s)
#pragma unroll
        for (int q = 0; q < 4; ++q) kacc[q] = mfma(sG[(4 * s + lg) * PP + 16 * q + lc], xcol[s], kacc[q]);
    } else {
      gram_tile<T, PP>(X + t * TR * PP, sG, kacc);
    }
    __syncthreads();
  }
  const int64_t nv = PP * PP + 3;
  double* out = partials + (int64_t)blockIdx.x * nv;
  if constexpr (XCOL) {
    // kacc[q] holds block (q, w) of K^T: element (i, j) -> K[16 w + j][16 q + i]
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) out[(16 * w + lc) * PP + 16 * q + rowof<T>(lg, r)] = (double)kacc[q][r];
  } else {
    gram_store<T, PP>(out, kacc);
  }
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
// projected onto the tangent space as in Algorithm 4), fused with <G, P> and S = P^T P (its
// upper blocks formed, the lower ones mirrored).
// Partials: S (PP*PP), <G,P>.
template <typename T, int PP>
__global__ __launch_bounds__(WG) void k_dir(int64_t n, const T* __restrict__ X, const T* __restrict__ G0,
                                            const T* __restrict__ G1, T* __restrict__ P0, T* __restrict__ P1,
                                            const double* __restrict__ small, const Scalars* __restrict__ sc,
                                            double* __restrict__ partials, uint16_t* __restrict__ P16,
                                            float* __restrict__ P32) {
  if (sc->done) return;
  // the p x p factor in LDS (a wider one runs k_dir_wide)
  static_assert(!factor_wide<T, PP>(), "k_dir_wide takes this width");
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
  typename Vec4<T>::type sacc[SymSplit<PP>::PER_WAVE];
#pragma unroll
  for (int q = 0; q < SymSplit<PP>::PER_WAVE; ++q) sacc[q] = typename Vec4<T>::type{0, 0, 0, 0};
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
    if (P16) {
      // bfloat16 copy of P for the SpMM of the bfloat16 mode
      const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = row0 + rowof<T>(g, r);
        if (row < n)
#pragma unroll
          for (int cb = 0; cb < PP / 16; ++cb) gst(P16 + row * PP + 16 * cb + c, bf16_round((float)p[cb][r]));
      }
    }
    if (P32) {
      // float32 copy of P for the float32-input SpMM of a mixed solve's float64 phase
      const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = row0 + rowof<T>(g, r);
        if (row < n)
#pragma unroll
          for (int cb = 0; cb < PP / 16; ++cb) gst(P32 + row * PP + 16 * cb + c, (float)p[cb][r]);
      }
    }
#pragma unroll
    for (int cb = 0; cb < PP / 16; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) gp += (double)g[cb][r] * (double)p[cb][r];
    rl_to_lds<T, PP>(sP, p);
    __syncthreads();
    gram_tile_sym<T, PP>(sP, sacc);
    __syncthreads();
  }
  const int64_t nv = PP * PP + 1;
  double* out = partials + (int64_t)blockIdx.x * nv;
  gram_store_sym<T, PP>(out, sacc);
  const int l = threadIdx.x & 63;
  double s = wave_sum(gp);
  if (l == 0) red[w] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[PP * PP] = red[0] + red[1] + red[2] + red[3];
}

// ---------------------------------------------------------------- wide blocks (float64, PP = 128)
// At PP = 128 the float64 factor (128 KB) does not fit LDS beside a tile, and a wave that holds
// 16 rows of every operand across 128 columns runs out of registers. The gradient and direction
// passes there use workgroups of 8 waves over the same 64-row tiles: the tile of X is staged in
// LDS, wave w forms column block w (16 columns) of the product for all 64 rows, reading the
// factor's column block through the caches, and in the Gram that column block, still in the
// wave's registers in the D layout, is the right operand of the blocks (ib, w). An LDS tile
// keeps its rows 144 elements apart, with the 16-byte granules of a row permuted by row
// (wide_at), so that both the product's reads (16 rows, one granule each) and the Gram's (4
// consecutive rows, 16 columns each) fall on distinct banks.
constexpr int WGW = 2 * WG;  // threads per workgroup of the wide passes
constexpr int WPP = 128;     // their padded width
constexpr int WLD = 144;     // LDS row stride: odd rows start half a bank period (128 B) on

// LDS element of (row, col): 16-byte granule k of the row within its group of 8 is stored at
// k ^ ((row / 2) mod 8). The permutation depends on row mod 16 and moves elements within
// aligned groups of 16 columns, so wide_at(row + 16 a, col + 16 b) = wide_at(row, col) +
// 16 a WLD + 16 b: the accesses below take a lane base from wide_at and constant offsets.
__device__ __forceinline__ int wide_at(int row, int col) { return row * WLD + (col ^ (2 * ((row >> 1) & 7))); }
constexpr int WTILE = TR * WLD;  // elements of an LDS tile

// Global load / store at a wave-uniform base plus a per-lane element offset of 32 bits, the
// offset made opaque where it is formed: each access takes one offset register at its point
// of use, where 64-bit addresses formed ahead for a whole tile would hold many.
template <typename V>
__device__ __forceinline__ V wld(const V* base, int off) {
  asm volatile("" : "+v"(off));
  return *(const __attribute__((address_space(1))) V*)(reinterpret_cast<const char*>(base) +
                                                       (uint32_t)(off * (int)sizeof(V)));
}
template <typename V>
__device__ __forceinline__ void wst(V* base, int off, V v) {
  asm volatile("" : "+v"(off));
  *(__attribute__((address_space(1))) V*)(reinterpret_cast<char*>(base) + (uint32_t)(off * (int)sizeof(V))) = v;
}

// The whole tile t of a tall block (its rows past n are zero rows of the allocation), 16 bytes
// per lane, and its store into an LDS tile (a wave writes one row per step).
// Parts [m0, m0 + M) of the 8 granules per lane (the first half, the second half or all).
template <int M = 8>
__device__ __forceinline__ void wide_load(int tid, const double* __restrict__ A, int64_t t, d2 (&v)[M], int m0 = 0) {
  const d2* src = reinterpret_cast<const d2*>(A + t * TR * WPP);
#pragma unroll
  for (int m = 0; m < M; ++m) v[m] = wld(src, tid + WGW * (m0 + m));
}
template <int M = 8>
__device__ __forceinline__ void wide_store(int tid, double* __restrict__ s, const d2 (&v)[M], int m0 = 0) {
  // granule m of the lane: row tid / 64 + 8 m, column 2 (tid mod 64)
  const int b0 = wide_at(tid >> 6, 2 * (tid & 63)), b1 = wide_at((tid >> 6) + 8, 2 * (tid & 63));
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int mm = m0 + m;
    *reinterpret_cast<d2*>(s + ((mm & 1) ? b1 : b0) + 16 * (mm >> 1) * WLD) = v[m];
  }
}

// The wave's column block of the tile's 64 rows in the D layout: v[rg][r] is element
// (row0 + 16 rg + rowof(g, r), 16 w + c). Loads read whole tiles (rows past n are zero rows of
// the allocation); stores skip rows past n.
__device__ __forceinline__ void wide_load_cols(int tid, const double* __restrict__ B, int64_t row0, double (&v)[4][4]) {
  const int w = tid >> 6, l = tid & 63, g = l >> 4, c = l & 15;
  const double* b = B + row0 * WPP;
  const int o = rowof<double>(g, 0) * WPP + 16 * w + c;
#pragma unroll
  for (int rg = 0; rg < 4; ++rg)
#pragma unroll
    for (int r = 0; r < 4; ++r) v[rg][r] = wld(b, o + (16 * rg + 4 * r) * WPP);
}
__device__ __forceinline__ void wide_store_cols(int tid, double* __restrict__ B, int64_t row0, int64_t n,
                                                const double (&v)[4][4]) {
  const int w = tid >> 6, l = tid & 63, g = l >> 4, c = l & 15;
  double* b = B + row0 * WPP;
  const int o = rowof<double>(g, 0) * WPP + 16 * w + c;
  const int64_t left = n - row0 - rowof<double>(g, 0);  // rows of this lane group below n
#pragma unroll
  for (int rg = 0; rg < 4; ++rg)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (16 * rg + 4 * r < left) wst(b, o + (16 * rg + 4 * r) * WPP, v[rg][r]);
}

// acc[rg] += (LDS tile) * M, the wave's column block: k-steps in pairs, lane group g taking
// contraction indices 8 j + 2 g and 8 j + 2 g + 1 of pair j (one 16-byte LDS read per row
// group), the factor's elements loaded two pairs ahead.
__device__ __forceinline__ void wide_product(int tid, const double* __restrict__ s, const double* __restrict__ M,
                                             d4 (&acc)[4]) {
  const int w = tid >> 6, l = tid & 63, g = l >> 4, c = l & 15;
  const int mc = 16 * w + c + 2 * g * WPP;
  // element (16 rg + c, 8 j + 2 g) of the tile: la0 / la1 (j even / odd) + 16 rg WLD + 16 (j / 2)
  const int la0 = wide_at(c, 2 * g), la1 = wide_at(c, 8 + 2 * g);
  double bq[3][2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    bq[j][0] = wld(M, mc + 8 * j * WPP);
    bq[j][1] = wld(M, mc + (8 * j + 1) * WPP);
  }
#pragma unroll
  for (int j = 0; j < WPP / 8; ++j) {
    if (j + 2 < WPP / 8) {
      bq[(j + 2) % 3][0] = wld(M, mc + 8 * (j + 2) * WPP);
      bq[(j + 2) % 3][1] = wld(M, mc + (8 * (j + 2) + 1) * WPP);
    }
    d2 a[4];
#pragma unroll
    for (int rg = 0; rg < 4; ++rg)
      a[rg] = *reinterpret_cast<const d2*>(s + ((j & 1) ? la1 : la0) + 16 * rg * WLD + 16 * (j >> 1));
#pragma unroll
    for (int rg = 0; rg < 4; ++rg) acc[rg] = mfma(a[rg].x, bq[j % 3][0], acc[rg]);
#pragma unroll
    for (int rg = 0; rg < 4; ++rg) acc[rg] = mfma(a[rg].y, bq[j % 3][1], acc[rg]);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Lane bases of the Gram's A operand: element (16 rg + rowof(g, r), 16 ib + c) of an LDS tile
// is at lb[r] + 16 rg WLD + 16 ib.
__device__ __forceinline__ void wide_gram_bases(int tid, int (&lb)[4]) {
  const int l = tid & 63, g = l >> 4, c = l & 15;
#pragma unroll
  for (int r = 0; r < 4; ++r) lb[r] = wide_at(rowof<double>(g, r), c);
}
// One step (rows 16 rg + 4 r + 0..3) of a Gram block (ib, w): A = the LDS tile's columns
// 16 ib .., B = the wave's column block b (D layout).
__device__ __forceinline__ d4 wide_gram_step(const int (&lb)[4], const double* __restrict__ s, int rg, int r, int ib,
                                             double b, d4 acc) {
  return mfma(s[lb[r] + 16 * rg * WLD + 16 * ib], b, acc);
}

// Gradient pass at PP = 128 (as k_grad): G, <G, G>, <G_old, G>, ||G||_inf and K = X^T G, the
// wave's blocks (ib, w) of K. The X tiles are double-buffered in LDS (the next one is loaded
// during the current one), so one barrier per tile; the row sums of |G| of the 8 column blocks
// meet in LDS and wave 0 takes their maximum one tile later.
template <typename T, int PP>
__global__ __launch_bounds__(WGW) void k_grad_wide(int64_t n, const T* __restrict__ X, const T* __restrict__ Y,
                                                  T* __restrict__ G0, T* __restrict__ G1,
                                                  const double* __restrict__ small, const Scalars* __restrict__ sc,
                                                  double* __restrict__ partials, int cond) {
  static_assert(std::is_same<T, double>::value && PP == WPP, "the wide passes are float64 at PP = 128");
  if (sc->done) return;
  if (cond == GRAD_PENDING && sc->grad_ready) return;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double* sX = reinterpret_cast<double*>(lds_raw);  // two tiles
  double* rsum = sX + 2 * WTILE;                    // [2][8][TR]
  __shared__ double red[8 * 3];
  const double* Cm = small + S_C * PP * PP;
  const int par = sc->k & 1;
  double* G = par ? G1 : G0;
  const double* Gold = par ? G0 : G1;
  const bool have_old = sc->k > 0;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, c = l & 15;
  const int64_t ntiles = (n + TR - 1) / TR;
  int64_t t0, t1;
  tile_range(ntiles, t0, t1);
  d4 kacc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) kacc[q] = d4{0, 0, 0, 0};
  double gg = 0.0, gdot = 0.0, ginf = 0.0;
  d2 xn[8];
  if (t0 < t1) {
    wide_load(threadIdx.x, X, t0, xn);
    wide_store(threadIdx.x, sX, xn);
  }
  for (int64_t t = t0; t < t1; ++t) {
    // the lane's offsets are formed anew in every tile (held across the loop they would take
    // the registers the tile needs)
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int buf = (int)((t - t0) & 1);
    const double* sx = sX + buf * WTILE;
    // tile t is in sx; every wave is past the previous tile (its Gram's reads of the other
    // buffer, its row sums)
    __syncthreads();
    if (w == 0 && t > t0) {
      const double* rs = rsum + (buf ^ 1) * 8 * TR;
      double v = 0.0;
#pragma unroll
      for (int ww = 0; ww < 8; ++ww) v += rs[ww * TR + l];
      ginf = fmax(ginf, v);
    }
    const int64_t row0 = t * TR;
    double y[4][4], go[4][4];
    wide_load_cols(tid, Y, row0, y);
    if (have_old) wide_load_cols(tid, Gold, row0, go);
    d4 acc[4];
#pragma unroll
    for (int rg = 0; rg < 4; ++rg) acc[rg] = d4{0, 0, 0, 0};
    wide_product(tid, sx, Cm, acc);
    // G = X C - Y in place of y
    double* rs = rsum + buf * 8 * TR + w * TR;
#pragma unroll
    for (int rg = 0; rg < 4; ++rg)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double gv = acc[rg][r] - y[rg][r];
        y[rg][r] = gv;
        gg += gv * gv;
        if (have_old) gdot += go[rg][r] * gv;
        const double a = group16_sum(fabs(gv));
        if (c == 0) rs[16 * rg + rowof<double>(g, r)] = a;
      }
    wide_store_cols(tid, G, row0, n, y);
    if (t + 1 < t1) wide_load(tid, X, t + 1, xn);
    // K += X^T G over the tile
    int lb[4];
    wide_gram_bases(tid, lb);
#pragma unroll
    for (int rg = 0; rg < 4; ++rg)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
#pragma unroll
        for (int ib = 0; ib < 8; ++ib) kacc[ib] = wide_gram_step(lb, sx, rg, r, ib, y[rg][r], kacc[ib]);
        __builtin_amdgcn_sched_barrier(0);
      }
    if (t + 1 < t1) wide_store(tid, sX + (buf ^ 1) * WTILE, xn);
  }
  __syncthreads();
  if (w == 0 && t1 > t0) {
    const double* rs = rsum + (int)((t1 - 1 - t0) & 1) * 8 * TR;
    double v = 0.0;
#pragma unroll
    for (int ww = 0; ww < 8; ++ww) v += rs[ww * TR + l];
    ginf = fmax(ginf, v);
  }
  const int64_t nv = PP * PP + 3;
  double* out = partials + (int64_t)blockIdx.x * nv;
#pragma unroll
  for (int ib = 0; ib < 8; ++ib)
#pragma unroll
    for (int r = 0; r < 4; ++r) out[(16 * ib + rowof<double>(g, r)) * PP + 16 * w + c] = kacc[ib][r];
  const double s0 = wave_sum(gg), s1 = wave_sum(gdot), s2 = wave_max(ginf);
  if (l == 0) {
    red[w * 3 + 0] = s0;
    red[w * 3 + 1] = s1;
    red[w * 3 + 2] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0, m = 0.0;
    for (int ww = 0; ww < 8; ++ww) {
      a += red[ww * 3 + 0];
      b += red[ww * 3 + 1];
      m = fmax(m, red[ww * 3 + 2]);
    }
    out[PP * PP + 0] = a;
    out[PP * PP + 1] = b;
    out[PP * PP + 2] = m;
  }
}

// Direction pass at PP = 128 (as k_dir): P, <G, P> and S = P^T P. The blocks of S are shared
// out by pairs of column blocks {i, i + d mod 8}: wave w forms (w + d mod 8, w) for d = 0 .. 3
// and, when w < 4, d = 4 (4 or 5 blocks each, 36 in all), and writes the mirror of each
// off-diagonal one.
template <typename T, int PP>
__global__ __launch_bounds__(WGW) void k_dir_wide(int64_t n, const T* __restrict__ X, const T* __restrict__ G0,
                                                 const T* __restrict__ G1, T* __restrict__ P0, T* __restrict__ P1,
                                                 const double* __restrict__ small, const Scalars* __restrict__ sc,
                                                 double* __restrict__ partials, uint16_t* __restrict__ P16,
                                                 float* __restrict__ P32) {
  static_assert(std::is_same<T, double>::value && PP == WPP, "the wide passes are float64 at PP = 128");
  if (sc->done) return;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double* sX = reinterpret_cast<double*>(lds_raw);
  double* sP = sX + WTILE;
  __shared__ double red[8];
  const double* Km = small + S_KD * PP * PP;
  const int par = sc->k & 1;
  const double* G = par ? G1 : G0;
  double* P = par ? P1 : P0;
  const double* Pold = par ? P0 : P1;
  const double beta = sc->beta_pr;
  const bool use_old = beta != 0.0;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, c = l & 15;
  const int nd = w < 4 ? 5 : 4;
  const int64_t ntiles = (n + TR - 1) / TR;
  int64_t t0, t1;
  tile_range(ntiles, t0, t1);
  d4 sacc[5];
#pragma unroll
  for (int d = 0; d < 5; ++d) sacc[d] = d4{0, 0, 0, 0};
  double gp = 0.0;
  d2 xn[8];
  if (t0 < t1) wide_load(threadIdx.x, X, t0, xn);
  for (int64_t t = t0; t < t1; ++t) {
    int tid = threadIdx.x;  // offsets formed anew in every tile (as in k_grad_wide)
    asm volatile("" : "+v"(tid));
    // every wave is past the previous tile's reads of sX and sP
    __syncthreads();
    wide_store(tid, sX, xn);
    const int64_t row0 = t * TR;
    double gv[4][4], p[4][4];
    wide_load_cols(tid, G, row0, gv);
    if (use_old) wide_load_cols(tid, Pold, row0, p);
    __syncthreads();
    d4 acc[4];
#pragma unroll
    for (int rg = 0; rg < 4; ++rg) acc[rg] = d4{0, 0, 0, 0};
    wide_product(tid, sX, Km, acc);
    int lb[4];
    wide_gram_bases(tid, lb);
#pragma unroll
    for (int rg = 0; rg < 4; ++rg)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double pv = use_old ? gv[rg][r] + beta * p[rg][r] - acc[rg][r] : gv[rg][r] - acc[rg][r];
        p[rg][r] = pv;
        gp += gv[rg][r] * pv;
        sP[lb[r] + 16 * rg * WLD + 16 * w] = pv;
      }
    wide_store_cols(tid, P, row0, n, p);
    if (P16 || P32) {
      // bfloat16 / float32 copies of P for the SpMM of the mixed modes
#pragma unroll
      for (int rg = 0; rg < 4; ++rg)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = row0 + 16 * rg + rowof<double>(g, r);
          if (row < n) {
            if (P16) gst(P16 + row * PP + 16 * w + c, bf16_round((float)p[rg][r]));
            if (P32) gst(P32 + row * PP + 16 * w + c, (float)p[rg][r]);
          }
        }
    }
    if (t + 1 < t1) wide_load(tid, X, t + 1, xn);
    __syncthreads();
#pragma unroll
    for (int d = 0; d < 5; ++d)
      if (d < nd) {
        const int ib = (w + d) & 7;
#pragma unroll
        for (int rg = 0; rg < 4; ++rg)
#pragma unroll
          for (int r = 0; r < 4; ++r) sacc[d] = wide_gram_step(lb, sP, rg, r, ib, p[rg][r], sacc[d]);
        __builtin_amdgcn_sched_barrier(0);
      }
  }
  const int64_t nv = PP * PP + 1;
  double* out = partials + (int64_t)blockIdx.x * nv;
#pragma unroll
  for (int d = 0; d < 5; ++d)
    if (d < nd) {
      const int ib = (w + d) & 7;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * ib + rowof<double>(g, r), j = 16 * w + c;
        out[i * PP + j] = sacc[d][r];
        if (d) out[j * PP + i] = sacc[d][r];
      }
    }
  const double s = wave_sum(gp);
  if (l == 0) red[w] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0;
    for (int ww = 0; ww < 8; ++ww) a += red[ww];
    out[PP * PP] = a;
  }
}

// ---------------------------------------------------------------- retraction pass
// X <- (X - mu P) M and Y <- (Y - mu Z) M with M = V diag((1 + mu^2 b)^-1/2) V^T, the
// inverse square root of I + mu^2 P^T P (Sec. 5.2, eq. Xnew_P; Sec. 6.1, eq. save_matvec). In place. When the state asks for an explicit A X the Y
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

// The retraction pass fused with the next iteration's gradient pass. With a1 = X - mu P and
// a2 = Y - mu Z (rows in the A-operand layout):
//   X <- a1 M,  Y <- a2 M,  G <- X_new C_next - Y_new = a1 (M C_next) - a2 M,
// where C_next is the line search's p x p recursion for X_new^T A X_new and M C_next is formed
// there (small[S_MC]); and the gradient pass's partial sums of G: K = X_new^T G, <G, G>,
// <G_old, G>, ||G||_inf (Sec. 3.1 eq. gradPhi; Sec. 5.2 eq. Xnew_P; Sec. 6.1 eq. save_matvec).
// X_new and G are both in the D layout, where the four rows of register r of the 16 x 16
// blocks are the contraction index of one MFMA step, so K accumulates without LDS: every wave
// keeps all (PP/16)^2 blocks of its rows' K and the four waves' blocks are added in wave order
// in LDS at the end. When the step asks for an explicit A X (refresh) only X is updated and the
// gradient pass runs after the product; a void step or a finished solve returns at once. X and
// Y come out bit for bit as from k_update; G differs from the separate pass's X_new C - Y_new
// by rounding only (the product with C is taken before the rounding of X_new).
template <typename T, int PP>
__global__ __launch_bounds__(WG) void k_update_grad(int64_t n, T* __restrict__ X, T* __restrict__ Y,
                                                    const T* __restrict__ P0, const T* __restrict__ P1,
                                                    const T* __restrict__ Z, T* __restrict__ G0, T* __restrict__ G1,
                                                    const double* __restrict__ small, const Scalars* __restrict__ sc,
                                                    double* __restrict__ partials) {
  if (sc->done || sc->null_step) return;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* sM = reinterpret_cast<T*>(lds_raw);
  T* sMC = sM + PP * PP;
  __shared__ double red[4 * 3];
  const int par = (sc->k - 1) & 1;  // the step was accepted: k already counts it
  const T* P = par ? P1 : P0;
  const int gpar = sc->k & 1;       // G_k, in the gradient pass's buffer convention
  T* G = gpar ? G1 : G0;
  const T* Gold = gpar ? G0 : G1;
  const T mu = (T)sc->mu;
  const bool full = !sc->refresh;
  load_matrix_lds<T, PP>(sM, small + S_M * PP * PP);
  if (full) load_matrix_lds<T, PP>(sMC, small + S_MC * PP * PP);
  __syncthreads();
  const int w = threadIdx.x >> 6;
  const int64_t ntiles = (n + TR - 1) / TR;
  int64_t t0, t1;
  tile_range(ntiles, t0, t1);
  constexpr int NB = PP / 16;
  typedef typename Vec4<T>::type V4;
  V4 kacc[NB * NB];
#pragma unroll
  for (int q = 0; q < NB * NB; ++q) kacc[q] = V4{0, 0, 0, 0};
  double gg = 0.0, gdot = 0.0, ginf = 0.0;
  for (int64_t t = t0; t < t1; ++t) {
    const int64_t row0 = t * TR + 16 * w;
    T a1[PP / 4], a2[PP / 4], b[PP / 4];
    load_al<T, PP>(X, row0, n, a1);
    load_al<T, PP>(P, row0, n, b);
#pragma unroll
    for (int s = 0; s < PP / 4; ++s) a1[s] = a1[s] - mu * b[s];
    V4 xacc[NB];
    zero_acc<T, PP>(xacc);
    if (full) {
      // G_old with the other operands: one wait per tile (a load issued after the stores
      // would wait for them too)
      T go[NB][4];
      load_rl<T, PP>(Gold, row0, n, go);
      load_al<T, PP>(Y, row0, n, a2);
      load_al<T, PP>(Z, row0, n, b);
#pragma unroll
      for (int s = 0; s < PP / 4; ++s) a2[s] = a2[s] - mu * b[s];
      V4 yacc[NB], gacc[NB];
      zero_acc<T, PP>(yacc);
      zero_acc<T, PP>(gacc);
      product2<T, PP>(a1, a2, sM, xacc, yacc);
      product<T, PP>(a1, sMC, gacc);
      T xo[NB][4], yo[NB][4], g[NB][4];
#pragma unroll
      for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          xo[cb][r] = xacc[cb][r];
          yo[cb][r] = yacc[cb][r];
          g[cb][r] = gacc[cb][r] - yacc[cb][r];
        }
      store_rl<T, PP>(X, row0, n, xo);
      store_rl<T, PP>(Y, row0, n, yo);
      store_rl<T, PP>(G, row0, n, g);
      double rs[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double gv = (double)g[cb][r];
          gg += gv * gv;
          rs[r] += fabs(gv);
          gdot += (double)go[cb][r] * gv;
        }
#pragma unroll
      for (int r = 0; r < 4; ++r) ginf = fmax(ginf, group16_sum(rs[r]));
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
#pragma unroll
          for (int cb2 = 0; cb2 < NB; ++cb2) kacc[cb * NB + cb2] = mfma(xo[cb][r], g[cb2][r], kacc[cb * NB + cb2]);
    } else {
      product<T, PP>(a1, sM, xacc);
      T xo[NB][4];
#pragma unroll
      for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) xo[cb][r] = xacc[cb][r];
      store_rl<T, PP>(X, row0, n, xo);
    }
  }
  if (!full) return;
  // the waves' K blocks added in wave order in LDS (the factors are no longer needed; the
  // dynamic LDS holds 2 PP^2 elements of T, at least PP^2 doubles)
  double* sK = reinterpret_cast<double*>(lds_raw);
  const int l = threadIdx.x & 63, lg = l >> 4, lc = l & 15;
  __syncthreads();
  for (int ww = 0; ww < 4; ++ww) {
    if (w == ww) {
#pragma unroll
      for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int cb2 = 0; cb2 < NB; ++cb2)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int e = (16 * cb + rowof<T>(lg, r)) * PP + 16 * cb2 + lc;
            sK[e] = (ww ? sK[e] : 0.0) + (double)kacc[cb * NB + cb2][r];
          }
    }
    __syncthreads();
  }
  const int64_t nv = PP * PP + 3;
  double* out = partials + (int64_t)blockIdx.x * nv;
  for (int e = threadIdx.x; e < PP * PP; e += WG) out[e] = sK[e];
  {
    const double s0 = wave_sum(gg), s1 = wave_sum(gdot), s2 = wave_max(ginf);
    if (l == 0) {
      red[w * 3 + 0] = s0;
      red[w * 3 + 1] = s1;
      red[w * 3 + 2] = s2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      out[PP * PP + 0] = red[0] + red[3] + red[6] + red[9];
      out[PP * PP + 1] = red[1] + red[4] + red[7] + red[10];
      out[PP * PP + 2] = fmax(fmax(red[2], red[5]), fmax(red[8], red[11]));
    }
  }
}

// ---------------------------------------------------------------- block SpMM
// Z = A_op W for a full symmetric CSR, W and Z row-major n x PP. One workgroup per TR-row
// tile; spmm_tile deals the tiles to the XCDs (blockIdx.x mod 8) so that the rows a tile's
// gathers reach stay in that XCD's L2: one contiguous slab per XCD, or, for a banded matrix,
// one chunk of every plane of rows after the other. The tile's CSR structure is staged in
// LDS first (csr_stage). A row is handled by LPR lanes, each owning the 16 bytes of
// consecutive columns that one load moves (2 in float64, 4 in float32): a row of W is one
// gather instruction's worth of lanes, and at 16 bytes per lane the kernel needs fewer
// registers (more waves in flight) than with two loads per lane (777 -> 701 us at 128^3,
// p = 64, float64). The column indices and values of a batch of U nonzeros are read before
// its U gathers are issued, so each lane has up to U independent loads in flight. U is 8, or 7
// when no row holds more than 7 nonzeros (a 7-point stencil: 644 -> 627 us at 128^3, p = 64,
// where a batch of 8 spends one gather of the 8 on padding; same bits).
// mode 0: always run, W = W0. mode 1: the iteration's SpMM (skipped when the solve is done
// or the step is null), W = P of the current iteration (W0/W1 by parity). mode 2: explicit
// A X (runs only when requested).
__device__ __forceinline__ bool spmm_skip(const Scalars* sc, int mode) {
  if (mode == 1) return sc->done || sc->null_step;
  if (mode == 2) return sc->done || sc->null_step || !sc->refresh;
  return false;
}

__device__ __forceinline__ int64_t xcd_tile(int64_t ntiles) {
  const int64_t per = (ntiles + 7) / 8;
  return (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

// Tile of this workgroup (ntiles or more: none). plane_tiles == 0: the XCDs (blockIdx mod 8)
// each sweep one contiguous slab (xcd_tile). plane_tiles > 0 (a banded matrix whose rows
// reach about plane_tiles tiles away, e.g. the neighbouring planes of a 3D grid): the rows
// are cut into planes of plane_tiles tiles, each plane is dealt to the 8 XCDs as 8 chunks
// and every XCD sweeps its chunk of one plane after the other, so that the rows its current
// chunk reaches in the previous and next plane are still in that XCD's L2.
__device__ __forceinline__ int64_t spmm_tile(int64_t ntiles, int64_t plane_tiles) {
  if (plane_tiles <= 0) return xcd_tile(ntiles);
  const int64_t chunk = (plane_tiles + 7) / 8;
  const int64_t x = blockIdx.x & 7, i = blockIdx.x >> 3;
  const int64_t local = x * chunk + i % chunk;
  if (local >= plane_tiles) return ntiles;
  return (i / chunk) * plane_tiles + local;
}

// Workgroups of an SpMM launch (8 per XCD round; see spmm_tile).
inline int64_t spmm_grid(int64_t ntiles, int64_t plane_tiles) {
  if (plane_tiles <= 0) return 8 * ((ntiles + 7) / 8);
  const int64_t chunk = (plane_tiles + 7) / 8, planes = (ntiles + plane_tiles - 1) / plane_tiles;
  return 8 * chunk * planes;
}

// The row pointers of a workgroup's tile and, when they fit (at most CSR_CAP nonzeros), its
// column indices and values, read into LDS with coalesced loads before any gather: a gather
// then waits on one LDS read instead of two dependent global loads. Returns whether the
// indices and values were staged (the same answer in every thread of the workgroup).
constexpr int CSR_CAP = 2048;
template <typename V>
__device__ __forceinline__ bool csr_stage(int32_t* s_rp, int32_t* s_col, V* s_val, const int32_t* __restrict__ rowptr,
                                          const int32_t* __restrict__ colind, const V* __restrict__ vals, int64_t r0,
                                          int nrows) {
  if ((int)threadIdx.x <= nrows) s_rp[threadIdx.x] = rowptr[r0 + threadIdx.x];
  __syncthreads();
  const int32_t base = s_rp[0], cnt = s_rp[nrows] - base;
  const bool staged = cnt <= CSR_CAP;
  if (staged)
    for (int i = threadIdx.x; i < cnt; i += WG) {
      s_col[i] = colind[base + i];
      s_val[i] = vals[base + i];
    }
  __syncthreads();
  return staged;
}

template <typename T, int PP, int U>
__global__ __launch_bounds__(WG) void k_spmm(int64_t n, const int32_t* __restrict__ rowptr,
                                             const int32_t* __restrict__ colind, const T* __restrict__ vals,
                                             const T* __restrict__ W0, const T* __restrict__ W1, T* __restrict__ Z,
                                             const Scalars* __restrict__ sc, int mode, int64_t plane_tiles) {
  if (spmm_skip(sc, mode)) return;
  const T* W = (mode == 1 && (sc->k & 1)) ? W1 : W0;
  constexpr int EPL = 16 / (int)sizeof(T);  // columns per lane: one 16-byte gather per nonzero
  constexpr int LPR = PP / EPL;             // lanes per row
  constexpr int RPB = WG / LPR;             // rows per block pass
  const int64_t ntiles = (n + TR - 1) / TR;
  const int64_t t = spmm_tile(ntiles, plane_tiles);
  if (t >= ntiles) return;
  __shared__ int32_t s_rp[TR + 1];
  __shared__ int32_t s_col[CSR_CAP];
  __shared__ T s_val[CSR_CAP];
  const int64_t r0 = t * TR;
  const int nrows = (int)((n - r0) < TR ? (n - r0) : TR);
  const bool staged = csr_stage(s_rp, s_col, s_val, rowptr, colind, vals, r0, nrows);
  const int32_t base = s_rp[0];
  const int sub = threadIdx.x / LPR, lane = threadIdx.x % LPR;
  for (int pass = 0; pass < TR / RPB; ++pass) {
    const int lr = pass * RPB + sub;
    if (lr >= nrows) continue;
    const int64_t row = r0 + lr;
    typedef typename std::conditional<sizeof(T) == 8, d2, f4>::type V16;
    V16 acc = {};
    const int32_t j0 = s_rp[lr], j1 = s_rp[lr + 1];
    for (int32_t j = j0; j < j1; j += U) {
      int32_t col[U];
      T v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool ok = j + u < j1;
        if (staged) {
          col[u] = ok ? s_col[j + u - base] : 0;
          v[u] = ok ? s_val[j + u - base] : T(0);
        } else {
          col[u] = ok ? colind[j + u] : 0;
          v[u] = ok ? vals[j + u] : T(0);
        }
      }
      V16 x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = gld(reinterpret_cast<const V16*>(W + (int64_t)col[u] * PP + EPL * lane));
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int e = 0; e < EPL; ++e) acc[e] += v[u] * x[u][e];
    }
    // non-temporal: Z is not read again by this launch, and keeping it out of the caches
    // leaves them to the rows of W that neighbouring tiles gather (669 against 704 us in a
    // probe at 128^3, p = 64)
    __builtin_nontemporal_store(acc, reinterpret_cast<V16*>(Z + row * PP + EPL * lane));
  }
}

// Z (float32) = A W with bfloat16 values and a bfloat16 W, float32 accumulation (the
// products of two bfloat16 numbers are exact in float32). Same tiling and modes as k_spmm;
// a lane owns 8 consecutive columns (one 16-byte gather per nonzero).
template <int PP, int U>
__global__ __launch_bounds__(WG) void k_spmm16(int64_t n, const int32_t* __restrict__ rowptr,
                                               const int32_t* __restrict__ colind, const uint16_t* __restrict__ vals,
                                               const uint16_t* __restrict__ W, float* __restrict__ Z,
                                               const Scalars* __restrict__ sc, int mode, int64_t plane_tiles) {
  if (spmm_skip(sc, mode)) return;
  constexpr int EPL = 8;
  constexpr int LPR = PP / EPL;  // lanes per row
  constexpr int RPB = WG / LPR;  // rows per block pass
  const int64_t ntiles = (n + TR - 1) / TR;
  const int64_t t = spmm_tile(ntiles, plane_tiles);
  if (t >= ntiles) return;
  constexpr int PASSES = (TR + RPB - 1) / RPB;  // at PP = 16 a pass spans 128 rows: half the lanes idle
  __shared__ int32_t s_rp[TR + 1];
  __shared__ int32_t s_col[CSR_CAP];
  __shared__ uint16_t s_val[CSR_CAP];
  const int64_t r0 = t * TR;
  const int nrows = (int)((n - r0) < TR ? (n - r0) : TR);
  const bool staged = csr_stage(s_rp, s_col, s_val, rowptr, colind, vals, r0, nrows);
  const int32_t base = s_rp[0];
  const int sub = threadIdx.x / LPR, lane = threadIdx.x % LPR;
#pragma unroll
  for (int pass = 0; pass < PASSES; ++pass) {
    const int lr = pass * RPB + sub;
    if (lr >= nrows) continue;
    const int64_t row = r0 + lr;
    float acc[EPL];
#pragma unroll
    for (int e = 0; e < EPL; ++e) acc[e] = 0.f;
    const int32_t j0 = s_rp[lr], j1 = s_rp[lr + 1];
    for (int32_t j = j0; j < j1; j += U) {
      int32_t col[U];
      float v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool ok = j + u < j1;
        if (staged) {
          col[u] = ok ? s_col[j + u - base] : 0;
          v[u] = ok ? bf16_widen(s_val[j + u - base]) : 0.f;
        } else {
          col[u] = ok ? colind[j + u] : 0;
          v[u] = ok ? bf16_widen(vals[j + u]) : 0.f;
        }
      }
      u4 x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = gld(reinterpret_cast<const u4*>(W + (int64_t)col[u] * PP + EPL * lane));
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t w4[4] = {x[u][0], x[u][1], x[u][2], x[u][3]};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          acc[2 * q] += v[u] * bf16_widen(w4[q] & 0xffffu);
          acc[2 * q + 1] += v[u] * bf16_widen(w4[q] >> 16);
        }
      }
    }
    float* zr = Z + row * PP + EPL * lane;
    *reinterpret_cast<float4*>(zr) = make_float4(acc[0], acc[1], acc[2], acc[3]);
    *reinterpret_cast<float4*>(zr + 4) = make_float4(acc[4], acc[5], acc[6], acc[7]);
  }
}

// Z (float64) = A W from float32 values and a float32 W: each product of two float32 numbers
// is exact in float64 and the sum is float64, so the only error is the rounding of A and W
// to float32 (half the gather bytes of float64). Same tiling and modes as k_spmm.
template <int PP, int U>
__global__ __launch_bounds__(WG) void k_spmm_fin(int64_t n, const int32_t* __restrict__ rowptr,
                                                 const int32_t* __restrict__ colind, const float* __restrict__ vals,
                                                 const float* __restrict__ W, double* __restrict__ Z,
                                                 const Scalars* __restrict__ sc, int mode, int64_t plane_tiles) {
  if (spmm_skip(sc, mode)) return;
  constexpr int EPL = 4;
  constexpr int LPR = PP / EPL;  // lanes per row
  constexpr int RPB = WG / LPR;  // rows per block pass
  const int64_t ntiles = (n + TR - 1) / TR;
  const int64_t t = spmm_tile(ntiles, plane_tiles);
  if (t >= ntiles) return;
  __shared__ int32_t s_rp[TR + 1];
  __shared__ int32_t s_col[CSR_CAP];
  __shared__ float s_val[CSR_CAP];
  const int64_t r0 = t * TR;
  const int nrows = (int)((n - r0) < TR ? (n - r0) : TR);
  const bool staged = csr_stage(s_rp, s_col, s_val, rowptr, colind, vals, r0, nrows);
  const int32_t base = s_rp[0];
  const int sub = threadIdx.x / LPR, lane = threadIdx.x % LPR;
#pragma unroll
  for (int pass = 0; pass < TR / RPB; ++pass) {
    const int lr = pass * RPB + sub;
    if (lr >= nrows) continue;
    const int64_t row = r0 + lr;
    double acc[EPL] = {0.0, 0.0, 0.0, 0.0};
    const int32_t j0 = s_rp[lr], j1 = s_rp[lr + 1];
    for (int32_t j = j0; j < j1; j += U) {
      int32_t col[U];
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool ok = j + u < j1;
        if (staged) {
          col[u] = ok ? s_col[j + u - base] : 0;
          v[u] = ok ? (double)s_val[j + u - base] : 0.0;
        } else {
          col[u] = ok ? colind[j + u] : 0;
          v[u] = ok ? (double)vals[j + u] : 0.0;
        }
      }
      f4 x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = gld(reinterpret_cast<const f4*>(W + (int64_t)col[u] * PP + EPL * lane));
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int e = 0; e < EPL; ++e) acc[e] += v[u] * (double)x[u][e];
    }
    double* zr = Z + row * PP + EPL * lane;
    *reinterpret_cast<double2*>(zr) = make_double2(acc[0], acc[1]);
    *reinterpret_cast<double2*>(zr + 2) = make_double2(acc[2], acc[3]);
  }
}

// Z = alpha (A W) + beta W + gamma V (V nullable): one step of a polynomial filter's
// three-term recurrence fused into the SpMM (the row of W and of V a lane needs for the
// epilogue is its own output row). Always runs (mode 0), same tiling as k_spmm.
template <typename T, int PP, int U>
__global__ __launch_bounds__(WG) void k_spmm_axpy(int64_t n, const int32_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ colind, const T* __restrict__ vals,
                                                  const T* __restrict__ W, const T* __restrict__ V, T* __restrict__ Z,
                                                  double alpha, double beta, double gamma, int64_t plane_tiles) {
  typedef typename std::conditional<sizeof(T) == 8, d2, f4>::type V16;
  constexpr int EPL = 16 / (int)sizeof(T);  // one 16-byte gather per nonzero per lane
  constexpr int LPR = PP / EPL;
  constexpr int RPB = WG / LPR;
  const int64_t ntiles = (n + TR - 1) / TR;
  const int64_t t = spmm_tile(ntiles, plane_tiles);
  if (t >= ntiles) return;
  __shared__ int32_t s_rp[TR + 1];
  __shared__ int32_t s_col[CSR_CAP];
  __shared__ T s_val[CSR_CAP];
  const int64_t r0 = t * TR;
  const int nrows = (int)((n - r0) < TR ? (n - r0) : TR);
  const bool staged = csr_stage(s_rp, s_col, s_val, rowptr, colind, vals, r0, nrows);
  const int32_t base = s_rp[0];
  const int sub = threadIdx.x / LPR, lane = threadIdx.x % LPR;
  for (int pass = 0; pass < TR / RPB; ++pass) {
    const int lr = pass * RPB + sub;
    if (lr >= nrows) continue;
    const int64_t row = r0 + lr;
    V16 acc = {};
    const int32_t j0 = s_rp[lr], j1 = s_rp[lr + 1];
    for (int32_t j = j0; j < j1; j += U) {
      int32_t col[U];
      T v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool ok = j + u < j1;
        if (staged) {
          col[u] = ok ? s_col[j + u - base] : 0;
          v[u] = ok ? s_val[j + u - base] : T(0);
        } else {
          col[u] = ok ? colind[j + u] : 0;
          v[u] = ok ? vals[j + u] : T(0);
        }
      }
      V16 x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = gld(reinterpret_cast<const V16*>(W + (int64_t)col[u] * PP + EPL * lane));
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int e = 0; e < EPL; ++e) acc[e] += v[u] * x[u][e];
    }
    const int64_t o = row * PP + EPL * lane;
    const V16 wo = gld(reinterpret_cast<const V16*>(W + o));
    V16 vo = {};
    if (V) vo = gld(reinterpret_cast<const V16*>(V + o));
    V16 zo;
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      double z = alpha * (double)acc[e] + beta * (double)wo[e];
      if (V) z += gamma * (double)vo[e];
      zo[e] = (T)z;
    }
    gst(reinterpret_cast<V16*>(Z + o), zo);
  }
}

// ---------------------------------------------------------------- matrix-free stencil SpMM
// Z = A W for a 5- or 7-point stencil on an nx x ny x nz grid (lexicographic order, x
// fastest): row r holds diag[r] on the diagonal and `off` at each neighbour inside the grid
// (r -+ nx ny, r -+ nx, r -+ 1). No index or value arrays are read: W once (neighbours from
// the caches), diag once, Z written once. The seven terms are summed in increasing column
// order with zero weights for neighbours outside the grid, the order and arithmetic of the
// CSR kernel, so both give identical results for the same matrix. AXPY: Z = alpha (A W) +
// beta W + gamma V (V nullable) for the Chebyshev recurrence; such a launch always runs.
template <typename T, int PP, bool AXPY>
__global__ __launch_bounds__(WG) void k_spmm_stencil(int64_t n, int32_t nx, int32_t ny, int32_t nz,
                                                     const T* __restrict__ diag, T off, const T* __restrict__ W0,
                                                     const T* __restrict__ W1, T* __restrict__ Z,
                                                     const Scalars* __restrict__ sc, int mode, int64_t plane_tiles,
                                                     const T* __restrict__ V, double alpha, double beta,
                                                     double gamma) {
  if (!AXPY && spmm_skip(sc, mode)) return;
  const T* W = (!AXPY && mode == 1 && (sc->k & 1)) ? W1 : W0;
  constexpr int EPL = 4;
  constexpr int LPR = PP / EPL;
  constexpr int RPB = WG / LPR;
  constexpr int PASSES = TR / RPB > 0 ? TR / RPB : 1;
  const int64_t ntiles = (n + TR - 1) / TR;
  const int64_t t = spmm_tile(ntiles, plane_tiles);
  if (t >= ntiles) return;
  const int sub = threadIdx.x / LPR, lane = threadIdx.x % LPR;
  const int64_t plane = (int64_t)nx * ny;
#pragma unroll
  for (int pass = 0; pass < PASSES; ++pass) {
    if (pass * RPB + sub >= TR) continue;
    const int64_t row = t * TR + pass * RPB + sub;
    if (row >= n) continue;
    const uint32_t r32 = (uint32_t)row;
    const uint32_t i = r32 % (uint32_t)nx, jk = r32 / (uint32_t)nx;
    const uint32_t j = jk % (uint32_t)ny, k = jk / (uint32_t)ny;
    int64_t col[7];
    T v[7];
    col[0] = k > 0 ? row - plane : row;                v[0] = k > 0 ? off : T(0);
    col[1] = j > 0 ? row - nx : row;                   v[1] = j > 0 ? off : T(0);
    col[2] = i > 0 ? row - 1 : row;                    v[2] = i > 0 ? off : T(0);
    col[3] = row;                                      v[3] = diag[row];
    col[4] = i + 1 < (uint32_t)nx ? row + 1 : row;     v[4] = i + 1 < (uint32_t)nx ? off : T(0);
    col[5] = j + 1 < (uint32_t)ny ? row + nx : row;    v[5] = j + 1 < (uint32_t)ny ? off : T(0);
    col[6] = k + 1 < (uint32_t)nz ? row + plane : row; v[6] = k + 1 < (uint32_t)nz ? off : T(0);
    T x[7][EPL];
#pragma unroll
    for (int u = 0; u < 7; ++u)
#pragma unroll
      for (int e = 0; e < EPL; ++e) x[u][e] = gld(W + col[u] * PP + EPL * lane + e);
    T acc[EPL] = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int u = 0; u < 7; ++u)
#pragma unroll
      for (int e = 0; e < EPL; ++e) acc[e] += v[u] * x[u][e];
    const int64_t o = row * PP + EPL * lane;
    if constexpr (AXPY) {
#pragma unroll
      for (int e = 0; e < EPL; ++e) {
        double z = alpha * (double)acc[e] + beta * (double)x[3][e];
        if (V) z += gamma * (double)gld(V + o + e);
        gst(Z + o + e, (T)z);
      }
    } else {
#pragma unroll
      for (int e = 0; e < EPL; ++e) gst(Z + o + e, acc[e]);
    }
  }
}

// The same product for grids with at least SY rows in y (2D and 3D), with each row of W
// read from memory about once instead of once per neighbour. A workgroup owns a tile of
// SX x SY grid points in x and y, a chunk of SCC columns and a run of up to SZC planes, and
// marches through its planes in z: the current plane of the tile with a one-point halo in x
// and y sits in LDS (the x and y neighbours and the centre are read from there), the previous
// plane's centres stay in registers, and the next plane's tile and halo are loaded into
// registers while the current plane is computed, then written to LDS. Thread t owns the
// 16-byte piece q = t mod TPP of the chunk at the points t / TPP + PPS s of the tile (point
// = y SX + x). The seven terms are those of k_spmm_stencil in the same order with the same
// zero weights outside the grid, so both kernels return the same bits. Grid: (PP / SCC)
// chunks fastest, then x tiles, y tiles, runs of planes.
constexpr int SX = 32, SY = 8, SCC = 16, SZC = 32;
constexpr int SHX = SX + 2, SHY = SY + 2, SNH = 2 * SX + 2 * SY;  // halo points: no corners

// Halo point h of a tile -> its tile coordinates (-1 or SX / SY on the border).
__device__ __forceinline__ void march_halo_xy(int h, int& lx, int& ly) {
  if (h < SX) { lx = h; ly = -1; }
  else if (h < 2 * SX) { lx = h - SX; ly = SY; }
  else if (h < 2 * SX + SY) { lx = -1; ly = h - 2 * SX; }
  else { lx = SX; ly = h - 2 * SX - SY; }
}

inline int64_t march_grid(int PP, const int32_t* dims) {
  return (int64_t)(PP / SCC) * ((dims[0] + SX - 1) / SX) * ((dims[1] + SY - 1) / SY) * ((dims[2] + SZC - 1) / SZC);
}

template <typename T, int PP, bool AXPY>
__global__ __launch_bounds__(WG) void k_spmm_march(int32_t nx, int32_t ny, int32_t nz, const T* __restrict__ diag,
                                                   T off, const T* __restrict__ W0, const T* __restrict__ W1,
                                                   T* __restrict__ Z, const Scalars* __restrict__ sc, int mode,
                                                   const T* __restrict__ V, double alpha, double beta, double gamma) {
  if (!AXPY && spmm_skip(sc, mode)) return;
  const T* W = (!AXPY && mode == 1 && (sc->k & 1)) ? W1 : W0;
  typedef typename std::conditional<sizeof(T) == 8, d2, f4>::type V16;
  constexpr int E = 16 / (int)sizeof(T);         // elements per piece
  constexpr int TPP = SCC / E;                   // pieces of a point's chunk
  constexpr int PPS = WG / TPP;                  // points per pass of the workgroup
  constexpr int NS = SX * SY / PPS;              // points per thread
  constexpr int NCC = PP / SCC;
  constexpr int HQ = (SNH * TPP + WG - 1) / WG;  // halo pieces per thread
  static_assert(PP % SCC == 0 && (SX * SY) % PPS == 0, "tile shape");
  __shared__ V16 L[SHX * SHY * TPP];
  const int tx = (nx + SX - 1) / SX, ty = (ny + SY - 1) / SY;
  int b = blockIdx.x;
  const int cc = b % NCC;
  b /= NCC;
  const int bx = b % tx;
  b /= tx;
  const int by = b % ty;
  const int z0 = (b / ty) * SZC;
  if (z0 >= nz) return;  // the whole workgroup, before any barrier
  const int z1 = z0 + SZC < nz ? z0 + SZC : nz;
  const int x0 = bx * SX, y0 = by * SY, c0 = cc * SCC;
  const int q = threadIdx.x % TPP, p0 = threadIdx.x / TPP;
  const int64_t plane = (int64_t)nx * ny;
  const V16 zero = {};
  auto piece = [&](const T* base, int gx, int gy, int z, int qq) -> const V16* {
    return reinterpret_cast<const V16*>(base + ((int64_t)z * plane + (int64_t)gy * nx + gx) * PP + c0) + qq;
  };
  auto load_centres = [&](int z, V16* ctr) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int pt = p0 + PPS * s, gx = x0 + pt % SX, gy = y0 + pt / SX;
      ctr[s] = (gx < nx && gy < ny) ? gld(piece(W, gx, gy, z, q)) : zero;
    }
  };
  auto load_halo = [&](int z, V16* hl) {
#pragma unroll
    for (int hh = 0; hh < HQ; ++hh) {
      const int idx = threadIdx.x + WG * hh;
      hl[hh] = zero;
      if (idx < SNH * TPP) {
        int lx, ly;
        march_halo_xy(idx / TPP, lx, ly);
        const int gx = x0 + lx, gy = y0 + ly;
        if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) hl[hh] = gld(piece(W, gx, gy, z, idx % TPP));
      }
    }
  };
  auto store_lds = [&](const V16* ctr, const V16* hl) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int pt = p0 + PPS * s;
      L[((pt / SX + 1) * SHX + pt % SX + 1) * TPP + q] = ctr[s];
    }
#pragma unroll
    for (int hh = 0; hh < HQ; ++hh) {
      const int idx = threadIdx.x + WG * hh;
      if (idx < SNH * TPP) {
        int lx, ly;
        march_halo_xy(idx / TPP, lx, ly);
        L[((ly + 1) * SHX + lx + 1) * TPP + idx % TPP] = hl[hh];
      }
    }
  };
  V16 prv[NS], nxt[NS], hal[HQ];
  if (z0 > 0) load_centres(z0 - 1, prv);
  else {
#pragma unroll
    for (int s = 0; s < NS; ++s) prv[s] = zero;
  }
  load_centres(z0, nxt);
  load_halo(z0, hal);
  store_lds(nxt, hal);
  __syncthreads();
  for (int z = z0; z < z1; ++z) {
    // the next plane: its centres (the z + 1 terms) and, inside the run, its halo
    if (z + 1 < nz) load_centres(z + 1, nxt);
    else {
#pragma unroll
      for (int s = 0; s < NS; ++s) nxt[s] = zero;
    }
    if (z + 1 < z1) load_halo(z + 1, hal);
    const T vzm = z > 0 ? off : T(0), vzp = z + 1 < nz ? off : T(0);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int pt = p0 + PPS * s, lx = pt % SX, ly = pt / SX, gx = x0 + lx, gy = y0 + ly;
      if (gx >= nx || gy >= ny) continue;
      const int c = ((ly + 1) * SHX + lx + 1) * TPP + q;
      const V16 wym = L[c - SHX * TPP], wxm = L[c - TPP], wc = L[c], wxp = L[c + TPP], wyp = L[c + SHX * TPP];
      const T vym = gy > 0 ? off : T(0), vxm = gx > 0 ? off : T(0);
      const T vxp = gx + 1 < nx ? off : T(0), vyp = gy + 1 < ny ? off : T(0);
      const int64_t row = (int64_t)z * plane + (int64_t)gy * nx + gx;
      const T dg = diag[row];
      V16 acc;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        T a = T(0);
        a += vzm * prv[s][e];
        a += vym * wym[e];
        a += vxm * wxm[e];
        a += dg * wc[e];
        a += vxp * wxp[e];
        a += vyp * wyp[e];
        a += vzp * nxt[s][e];
        acc[e] = a;
      }
      const int64_t o = row * PP + c0 + E * q;
      if constexpr (AXPY) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          double zz = alpha * (double)acc[e] + beta * (double)wc[e];
          if (V) zz += gamma * (double)gld(V + o + e);
          acc[e] = (T)zz;
        }
      }
      __builtin_nontemporal_store(acc, reinterpret_cast<V16*>(Z + o));  // not read again here
      prv[s] = wc;
    }
    __syncthreads();  // every thread is done with plane z in LDS
    if (z + 1 < z1) {
      store_lds(nxt, hal);
      __syncthreads();
    }
  }
}

// Diagonal of a stencil operator, scaled: out[r] = scale (d + (dv ? dv[r] : 0)).
template <typename T>
__global__ void k_stencil_diag(int64_t n, double d, const double* __restrict__ dv, double scale, T* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) out[r] = (T)(scale * (d + (dv ? dv[r] : 0.0)));
}

// Per-block maxima of the absolute row sums |d + dv[r]| + |off| (number of grid neighbours)
// and the finiteness flag (4) of dv.
__global__ void k_stencil_check(int64_t n, int32_t nx, int32_t ny, int32_t nz, double d, double off,
                                const double* __restrict__ dv, double* __restrict__ partial_max,
                                int* __restrict__ flags) {
  __shared__ double red[WG];
  double m = 0.0;
  int f = 0;
  for (int64_t row = (int64_t)blockIdx.x * WG + threadIdx.x; row < n; row += (int64_t)gridDim.x * WG) {
    const uint32_t r32 = (uint32_t)row;
    const uint32_t i = r32 % (uint32_t)nx, jk = r32 / (uint32_t)nx;
    const uint32_t j = jk % (uint32_t)ny, k = jk / (uint32_t)ny;
    const int deg = (i > 0) + (i + 1 < (uint32_t)nx) + (j > 0) + (j + 1 < (uint32_t)ny) + (k > 0) +
                    (k + 1 < (uint32_t)nz);
    const double dr = d + (dv ? dv[row] : 0.0);
    if (!isfinite(dr)) f |= 4;
    m = fmax(m, fabs(dr) + fabs(off) * deg);
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

// Z = a Y + b X over count elements.
template <typename T>
__global__ void k_axpby(int64_t count, const T* __restrict__ Y, const T* __restrict__ X, T* __restrict__ Z, double a,
                        double b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) Z[i] = (T)(a * (double)Y[i] + b * (double)X[i]);
}

// ---------------------------------------------------------------- Gram pass
// Partials of A^T B1 and (when B2 != nullptr) A^T B2 over the workgroup's rows, without LDS.
// At k-step s a lane (g = l/16, c = l%16) reads row 4s+g, columns c*V .. c*V+V-1 of each
// operand (V = PP/16 contiguous values, one or two 16-byte loads), so every row is read
// once per operand, fully coalesced. "Virtual block" vb of a lane's V values holds the
// columns {c*V + vb}; MFMA unit (gram, ib) accumulates the 16 x 16 blocks (ib, jb) for all
// jb, i.e. Gram entries (i*V + ib, j*V + jb). Units are dealt to the 4 waves so that a
// wave works on one Gram only. With mode 1 / 2 the pass follows the SpMM of the same
// mode (skip rules; A = P by parity for mode 1).
template <typename T, int PP>
struct GramUnits {
  static constexpr int V = PP / 16;
  static constexpr int MAXU = (2 * V + 3) / 4;  // units per wave with two Grams
};

template <typename T, int V>
__device__ __forceinline__ void load_row_v(const T* __restrict__ B, int64_t row, int64_t n, int c, T (&v)[V]) {
  const bool ok = row < n;
  const T* p = B + (ok ? row : 0) * (16 * V) + V * c;
  if constexpr (sizeof(T) * V == 32) {
    if constexpr (sizeof(T) == 8) {
      const double2 q0 = ok ? *reinterpret_cast<const double2*>(p) : make_double2(0.0, 0.0);
      const double2 q1 = ok ? *reinterpret_cast<const double2*>(p + 2) : make_double2(0.0, 0.0);
      v[0] = q0.x; v[1] = q0.y; v[2] = q1.x; v[3] = q1.y;
    } else {
      const float4 q0 = ok ? *reinterpret_cast<const float4*>(p) : make_float4(0.f, 0.f, 0.f, 0.f);
      const float4 q1 = ok ? *reinterpret_cast<const float4*>(p + 4) : make_float4(0.f, 0.f, 0.f, 0.f);
      v[0] = q0.x; v[1] = q0.y; v[2] = q0.z; v[3] = q0.w;
      v[4] = q1.x; v[5] = q1.y; v[6] = q1.z; v[7] = q1.w;
    }
  } else {
#pragma unroll
    for (int e = 0; e < V; ++e) v[e] = ok ? p[e] : T(0);
  }
}

template <typename T, int PP>
__global__ __launch_bounds__(WG) void k_gram(int64_t n, const T* __restrict__ A0, const T* __restrict__ A1,
                                             const T* __restrict__ B1, const T* __restrict__ B2,
                                             const Scalars* __restrict__ sc, int mode,
                                             double* __restrict__ partials) {
  if (spmm_skip(sc, mode)) return;
  constexpr int V = GramUnits<T, PP>::V;
  constexpr int MAXU = GramUnits<T, PP>::MAXU;
  const T* A = (mode == 1 && (sc->k & 1)) ? A1 : A0;
  const int ng = B2 ? 2 : 1;
  const int units = ng * V;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, c = l & 15;
  // unit u = w + 4q: gram = u % ng, ib = u / ng
  const int gsel = w % ng;
  const T* B = gsel ? B2 : B1;
  const int nu = (units > w) ? (units - w + 3) / 4 : 0;
  const int64_t ntiles = (n + TR - 1) / TR;
  int64_t t0, t1;
  tile_range(ntiles, t0, t1);
  typename Vec4<T>::type acc[MAXU][V];
#pragma unroll
  for (int q = 0; q < MAXU; ++q)
#pragma unroll
    for (int jb = 0; jb < V; ++jb) acc[q][jb] = typename Vec4<T>::type{0, 0, 0, 0};
  if (nu > 0) {
    for (int64_t t = t0; t < t1; ++t) {
#pragma unroll 2
      for (int s = 0; s < TR / 4; ++s) {
        const int64_t row = t * TR + 4 * s + g;
        T a[V], b[V];
        load_row_v<T, V>(A, row, n, c, a);
        load_row_v<T, V>(B, row, n, c, b);
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
  double* out = partials + (int64_t)blockIdx.x * ng * PP * PP;
#pragma unroll
  for (int q = 0; q < MAXU; ++q) {
    if (q < nu) {
      const int ib = (w + 4 * q) / ng;
      double* o = out + gsel * PP * PP;
#pragma unroll
      for (int jb = 0; jb < V; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = rowof<T>(g, r);
          o[(i * V + ib) * PP + c * V + jb] = (double)acc[q][jb][r];
        }
    }
  }
}

// A^T B1 and (TWO) A^T B2 at PP = 128 in float64, with the workgroups of the wide passes: the
// A tiles double-buffered in LDS as in k_grad_wide, wave w holding column block w of B1 and B2
// in the D layout and forming the blocks (ib, w) of both Grams. The B values of a row group
// are replaced by the next tile's as soon as its MFMAs have issued (the last tile reloads
// itself, unused), and the next A tile goes to the other buffer in two halves during the
// current one, so one barrier per tile and no load waits on the next tile's start.
template <typename T, int PP, bool TWO>
__global__ __launch_bounds__(WGW) void k_gram_wide(int64_t n, const T* __restrict__ A0, const T* __restrict__ A1,
                                                  const T* __restrict__ B1, const T* __restrict__ B2,
                                                  const Scalars* __restrict__ sc, int mode,
                                                  double* __restrict__ partials) {
  static_assert(std::is_same<T, double>::value && PP == WPP, "the wide passes are float64 at PP = 128");
  if (spmm_skip(sc, mode)) return;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double* sA = reinterpret_cast<double*>(lds_raw);  // two tiles
  const double* A = (mode == 1 && (sc->k & 1)) ? A1 : A0;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, c = l & 15;
  const int64_t ntiles = (n + TR - 1) / TR;
  int64_t t0, t1;
  tile_range(ntiles, t0, t1);
  d4 acc1[8], acc2[TWO ? 8 : 1];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc1[q] = d4{0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < (TWO ? 8 : 1); ++q) acc2[q] = d4{0, 0, 0, 0};
  double b1[4][4], b2[TWO ? 4 : 1][4];
  if (t0 < t1) {
    d2 x0[8];
    wide_load(threadIdx.x, A, t0, x0);
    wide_store(threadIdx.x, sA, x0);
    wide_load_cols(threadIdx.x, B1, t0 * TR, b1);
    if constexpr (TWO) wide_load_cols(threadIdx.x, B2, t0 * TR, b2);
  }
  for (int64_t t = t0; t < t1; ++t) {
    int tid = threadIdx.x;  // offsets formed anew in every tile (as in k_grad_wide)
    asm volatile("" : "+v"(tid));
    const int buf = (int)((t - t0) & 1);
    const double* sa = sA + buf * WTILE;
    const int64_t tn = t + 1 < t1 ? t + 1 : t;
    double* sn = sA + (buf ^ 1) * WTILE;
    __syncthreads();  // tile t is in sa; every wave is past the previous tile's reads
    d2 xn[4];
    int lb[4];
    wide_gram_bases(tid, lb);
    const int o = rowof<double>(g, 0) * PP + 16 * w + c;
    const double* n1 = B1 + tn * TR * PP;
    const double* n2 = TWO ? B2 + tn * TR * PP : nullptr;
#pragma unroll
    for (int rg = 0; rg < 4; ++rg)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
#pragma unroll
        for (int ib = 0; ib < 8; ++ib) {
          const double a = sa[lb[r] + 16 * rg * WLD + 16 * ib];
          acc1[ib] = mfma(a, b1[rg][r], acc1[ib]);
          if constexpr (TWO) acc2[ib] = mfma(a, b2[rg][r], acc2[ib]);
        }
        b1[rg][r] = wld(n1, o + (16 * rg + 4 * r) * PP);
        if constexpr (TWO) b2[rg][r] = wld(n2, o + (16 * rg + 4 * r) * PP);
        if (r == 3 && rg < 3) {
          // the next A tile: first half loaded after row group 0, stored after row group 1
          // (when the second half is loaded), second half stored after row group 2
          if (rg > 0) wide_store<4>(tid, sn, xn, 4 * (rg - 1));
          if (rg < 2) wide_load<4>(tid, A, tn, xn, 4 * rg);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
  }
  double* out = partials + (int64_t)blockIdx.x * (TWO ? 2 : 1) * PP * PP;
#pragma unroll
  for (int ib = 0; ib < 8; ++ib)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = (16 * ib + rowof<double>(g, r)) * PP + 16 * w + c;
      out[e] = acc1[ib][r];
      if constexpr (TWO) out[PP * PP + e] = acc2[ib][r];
    }
  (void)l;
}

// A^T B1 and (TWO) A^T B2 at PP = 64 (the iteration's P^T Z and P^T Y): wave w owns the 16 columns
// 16w .. 16w+15 of P (loaded at the top of each tile, so the loads overlap the staging) and
// the eight 16 x 16 output blocks (w, q) of both Grams; each wave stages its 16 rows of Z
// and Y in LDS, from where all four waves read them. Every row of P, Z and Y is read from
// memory once per workgroup. Rows of a tile past n are the zero padding of the blocks.
template <typename T, int PP, bool TWO>
__global__ __launch_bounds__(WG) void k_gram2(int64_t n, const T* __restrict__ A0, const T* __restrict__ A1,
                                              const T* __restrict__ B1, const T* __restrict__ B2,
                                              const Scalars* __restrict__ sc, int mode,
                                              double* __restrict__ partials) {
  static_assert(PP == 64, "k_gram2 is written for 64 columns");
  if (spmm_skip(sc, mode)) return;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* sZ = reinterpret_cast<T*>(lds_raw);
  T* sY = sZ + TR * PP;
  const T* A = (mode == 1 && (sc->k & 1)) ? A1 : A0;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, c = l & 15;
  const int64_t ntiles = (n + TR - 1) / TR;
  int64_t t0, t1;
  tile_range(ntiles, t0, t1);
  typename Vec4<T>::type accZ[4], accY[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    accZ[q] = typename Vec4<T>::type{0, 0, 0, 0};
    accY[q] = typename Vec4<T>::type{0, 0, 0, 0};
  }
  // staging: wave w copies rows 16w .. 16w+15 of the tile, 4 rows per step, a lane 4 values
  constexpr int EPL = 4, LPR = PP / EPL, RPS = 64 / LPR;
  const int sr = l / LPR, sc4 = (l % LPR) * EPL;
  for (int64_t t = t0; t < t1; ++t) {
    const int64_t base = t * TR;
    T pcol[TR / 4];
#pragma unroll
    for (int s = 0; s < TR / 4; ++s) pcol[s] = gld(A + (base + 4 * s + g) * PP + 16 * w + c);
    // 16-byte pieces: two per lane and row for float64, one for float32
    typedef typename std::conditional<sizeof(T) == 8, d2, f4>::type V16;
    constexpr int NV = EPL * (int)sizeof(T) / 16;
    V16 z[16 / RPS][NV], y[16 / RPS][NV];
#pragma unroll
    for (int k = 0; k < 16 / RPS; ++k) {
      const int r = 16 * w + k * RPS + sr;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        z[k][v] = gld(reinterpret_cast<const V16*>(B1 + (base + r) * PP + sc4) + v);
        if constexpr (TWO) y[k][v] = gld(reinterpret_cast<const V16*>(B2 + (base + r) * PP + sc4) + v);
      }
    }
#pragma unroll
    for (int k = 0; k < 16 / RPS; ++k) {
      const int r = 16 * w + k * RPS + sr;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        reinterpret_cast<V16*>(to_lds(sZ + r * PP + sc4))[v] = z[k][v];
        if constexpr (TWO) reinterpret_cast<V16*>(to_lds(sY + r * PP + sc4))[v] = y[k][v];
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < TR / 4; ++s)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int idx = (4 * s + g) * PP + 16 * q + c;
        accZ[q] = mfma(pcol[s], sZ[idx], accZ[q]);
        if constexpr (TWO) accY[q] = mfma(pcol[s], sY[idx], accY[q]);
      }
    __syncthreads();
  }
  double* out = partials + (int64_t)blockIdx.x * (TWO ? 2 : 1) * PP * PP;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t o = (16 * w + rowof<T>(g, r)) * PP + 16 * q + c;
      out[o] = (double)accZ[q][r];
      if constexpr (TWO) out[PP * PP + o] = (double)accY[q][r];
    }
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
// out[v] = sum_b partials[b * nv + v] for v < max_from, max over b otherwise. A workgroup
// covers 64 consecutive values with 4 slices of the nb partials each (b = q, q+4, ...);
// the slices are combined in a fixed order, so the result is deterministic.
// cond: 0 always; 1 skip when the solve is done or the step is null; 2 run only when an
// explicit A X refresh was requested; 3 skip when the solve is done.
__global__ __launch_bounds__(WG) void k_reduce(const double* __restrict__ partials, int nb, int64_t nv,
                                               int64_t max_from, double* __restrict__ out,
                                               const Scalars* __restrict__ sc, int cond) {
  if (cond == 1 && (sc->done || sc->null_step)) return;
  if (cond == 2 && (sc->done || sc->null_step || !sc->refresh)) return;
  if (cond == 3 && sc->done) return;
  if (cond == GRAD_PENDING && (sc->done || sc->grad_ready)) return;
  if (cond == GRAD_AFTER_FUSED && (sc->done || sc->null_step || sc->refresh || sc->grad_ready)) return;
  __shared__ double part[4][64];
  const int q = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t v = (int64_t)blockIdx.x * 64 + l;
  const bool use_max = v >= max_from;
  double s = 0.0;
  if (v < nv) {
    int b = q;
    for (; b + 28 < nb; b += 32) {
      double x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = partials[(int64_t)(b + 4 * u) * nv + v];
#pragma unroll
      for (int u = 0; u < 8; ++u) s = use_max ? fmax(s, x[u]) : s + x[u];
    }
    for (; b < nb; b += 4) {
      const double x = partials[(int64_t)b * nv + v];
      s = use_max ? fmax(s, x) : s + x;
    }
  }
  part[q][l] = s;
  __syncthreads();
  if (q == 0 && v < nv) {
    out[v] = use_max ? fmax(fmax(part[0][l], part[1][l]), fmax(part[2][l], part[3][l]))
                     : (part[0][l] + part[1][l]) + (part[2][l] + part[3][l]);
  }
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

// Complex basis from the real embedding of a Hermitian problem: column j of the n x pc
// complex output (interleaved re, im) is column 2j of the 2n x 2pc real block X (padded
// width PP) read as top half + i bottom half.
__global__ void k_complex_extract(int64_t n, int pc, int PP, const double* __restrict__ X, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * pc) return;
  const int64_t r = i / pc;
  const int j = (int)(i % pc);
  out[2 * i] = X[r * PP + 2 * j];
  out[2 * i + 1] = X[(n + r) * PP + 2 * j];
}

template <typename TS, typename TD>
__global__ void k_convert(int64_t count, const TS* __restrict__ src, TD* __restrict__ dst, double scale) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = (TD)(scale * (double)src[i]);
}

// dst = bfloat16(float32(scale * src)) (round to nearest even at each narrowing).
__global__ void k_to_bf16(int64_t count, const double* __restrict__ src, uint16_t* __restrict__ dst, double scale) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = bf16_round((float)(scale * src[i]));
}

// CSR checks and ||A||_inf: partial max of absolute row sums per workgroup, error flags:
// bit 0 rowptr not monotone / out of range, bit 1 column index out of range, bit 2
// non-finite value, bit 3 columns not sorted within a row.
__global__ void k_csr_check(int64_t n, int64_t nnz, const int32_t* __restrict__ rowptr,
                            const int32_t* __restrict__ colind, const double* __restrict__ vals,
                            double* __restrict__ partial_max, int* __restrict__ flags,
                            double* __restrict__ partial_band) {
  __shared__ double red[WG];
  __shared__ int64_t redb[WG];
  double m = 0.0;
  int64_t band = 0;
  int f = 0;
  for (int64_t row = (int64_t)blockIdx.x * WG + threadIdx.x; row < n; row += (int64_t)gridDim.x * WG) {
    const int64_t j0 = rowptr[row], j1 = rowptr[row + 1];
    if (j1 < j0 || j0 < 0 || j1 > nnz) { f |= 1; continue; }
    if (j1 - j0 > 7) f |= 32;  // not an error: the SpMM's batch of gathers stays at 8
    double s = 0.0;
    int32_t prev = -1;
    for (int64_t j = j0; j < j1; ++j) {
      const int32_t c = colind[j];
      if (c < 0 || c >= n) f |= 2;
      if (c <= prev) f |= 8;
      prev = c;
      const int64_t d = (int64_t)c - row;
      band = (d < 0 ? -d : d) > band ? (d < 0 ? -d : d) : band;
      const double v = vals[j];
      if (!isfinite(v)) f |= 4;
      s += fabs(v);
    }
    m = fmax(m, s);
  }
  if (f) atomicOr(flags, f);
  red[threadIdx.x] = m;
  redb[threadIdx.x] = band;
  __syncthreads();
  for (int o = WG / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
      redb[threadIdx.x] = redb[threadIdx.x] > redb[threadIdx.x + o] ? redb[threadIdx.x] : redb[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial_max[blockIdx.x] = red[0];
    if (partial_band) partial_band[blockIdx.x] = (double)redb[0];
  }
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
    // the wide passes: two tiles (and the row sums [2][8][TR] of the gradient pass)
    case Pass::Grad: return factor_wide<T, PP>() ? (2 * WTILE + 16 * TR) * (int)sizeof(double) : m + tile;
    case Pass::Dir: return factor_wide<T, PP>() ? 2 * WTILE * (int)sizeof(double) : m + tile;
    case Pass::Update: return m;
    case Pass::UpdateGrams: return m + 3 * tile;
    case Pass::UpdateGrad: return 2 * m;
    case Pass::Spmm: return 0;
    case Pass::SpmmPlain: return 0;
    case Pass::Gram: return 0;
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
  if constexpr (factor_wide<T, PP>()) {
    GSI_SET((k_grad_wide<T, PP>), Pass::Grad)
    GSI_SET((k_dir_wide<T, PP>), Pass::Dir)
    for (const void* k : {reinterpret_cast<const void*>(k_gram_wide<T, PP, true>),
                          reinterpret_cast<const void*>(k_gram_wide<T, PP, false>)})
      if (e == hipSuccess)
        e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 2 * WTILE * (int)sizeof(double));
  } else {
    GSI_SET((k_grad<T, PP>), Pass::Grad)
    GSI_SET((k_dir<T, PP>), Pass::Dir)
  }
  GSI_SET((k_update<T, PP, false>), Pass::Update)
  // the retraction with Gram epilogue and the fused retraction-gradient pass are not used above
  // PP = 64 (their LDS would exceed a CU's)
  if constexpr (PP <= PP_LDS_MAX) {
    GSI_SET((k_update<T, PP, true>), Pass::UpdateGrams)
    GSI_SET((k_update_grad<T, PP>), Pass::UpdateGrad)
  }
  GSI_SET((k_product<T, PP>), Pass::Product)
  if constexpr (PP == 64) {
    if (e == hipSuccess)
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_gram2<T, PP, true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 2 * TR * PP * (int)sizeof(T));
  }
#undef GSI_SET
  return e;
}

template <typename T, int PP>
void Kernels<T, PP>::grad(hipStream_t st, int nb, int64_t n, const T* X, const T* Y, T* G0, T* G1,
                          const double* small, const Scalars* sc, double* partials, int cond) {
  if constexpr (factor_wide<T, PP>())
    k_grad_wide<T, PP><<<nb, WGW, lds_bytes<T, PP>(Pass::Grad), st>>>(n, X, Y, G0, G1, small, sc, partials, cond);
  else
    k_grad<T, PP><<<nb, WG, lds_bytes<T, PP>(Pass::Grad), st>>>(n, X, Y, G0, G1, small, sc, partials, cond);
}
template <typename T, int PP>
void Kernels<T, PP>::update_grad(hipStream_t st, int nb, int64_t n, T* X, T* Y, const T* P0, const T* P1,
                                 const T* Z, T* G0, T* G1, const double* small, const Scalars* sc,
                                 double* partials) {
  if constexpr (PP <= PP_LDS_MAX)  // not used above (the host keeps the separate passes there)
    k_update_grad<T, PP><<<nb, WG, lds_bytes<T, PP>(Pass::UpdateGrad), st>>>(n, X, Y, P0, P1, Z, G0, G1, small, sc,
                                                                            partials);
}
template <typename T, int PP>
void Kernels<T, PP>::dir(hipStream_t st, int nb, int64_t n, const T* X, const T* G0, const T* G1, T* P0, T* P1,
                         const double* small, const Scalars* sc, double* partials, uint16_t* P16, float* P32) {
  if constexpr (factor_wide<T, PP>())
    k_dir_wide<T, PP><<<nb, WGW, lds_bytes<T, PP>(Pass::Dir), st>>>(n, X, G0, G1, P0, P1, small, sc, partials, P16,
                                                                    P32);
  else
    k_dir<T, PP><<<nb, WG, lds_bytes<T, PP>(Pass::Dir), st>>>(n, X, G0, G1, P0, P1, small, sc, partials, P16, P32);
}
template <typename T, int PP>
void Kernels<T, PP>::spmm_axpy(hipStream_t st, int64_t n, const int32_t* rowptr, const int32_t* colind, const T* vals,
                               const T* W, const T* V, T* Z, double alpha, double beta, double gamma,
                               int64_t plane_tiles, int batch) {
  const int64_t grid = spmm_grid((n + TR - 1) / TR, plane_tiles);
  if (batch == 7)
    k_spmm_axpy<T, PP, 7><<<dim3((unsigned)grid), dim3(WG), 0, st>>>(n, rowptr, colind, vals, W, V, Z, alpha, beta,
                                                                    gamma, plane_tiles);
  else
    k_spmm_axpy<T, PP, 8><<<dim3((unsigned)grid), dim3(WG), 0, st>>>(n, rowptr, colind, vals, W, V, Z, alpha, beta,
                                                                    gamma, plane_tiles);
}
// Grids with at least SY rows in y march through their planes (k_spmm_march); lines use
// the row-tile kernel.
template <typename T, int PP>
void Kernels<T, PP>::spmm_stencil(hipStream_t st, int64_t n, const int32_t* dims, const T* diag, double off,
                                  const T* W0, const T* W1, T* Z, const Scalars* sc, int mode, int64_t plane_tiles) {
  if (dims[1] >= SY) {
    k_spmm_march<T, PP, false><<<dim3((unsigned)march_grid(PP, dims)), dim3(WG), 0, st>>>(
        dims[0], dims[1], dims[2], diag, (T)off, W0, W1, Z, sc, mode, nullptr, 1.0, 0.0, 0.0);
    return;
  }
  const int64_t grid = spmm_grid((n + TR - 1) / TR, plane_tiles);
  k_spmm_stencil<T, PP, false><<<dim3((unsigned)grid), dim3(WG), 0, st>>>(
      n, dims[0], dims[1], dims[2], diag, (T)off, W0, W1, Z, sc, mode, plane_tiles, nullptr, 1.0, 0.0, 0.0);
}
template <typename T, int PP>
void Kernels<T, PP>::spmm_stencil_axpy(hipStream_t st, int64_t n, const int32_t* dims, const T* diag, double off,
                                       const T* W, const T* V, T* Z, double alpha, double beta, double gamma,
                                       int64_t plane_tiles) {
  if (dims[1] >= SY) {
    k_spmm_march<T, PP, true><<<dim3((unsigned)march_grid(PP, dims)), dim3(WG), 0, st>>>(
        dims[0], dims[1], dims[2], diag, (T)off, W, W, Z, nullptr, 0, V, alpha, beta, gamma);
    return;
  }
  const int64_t grid = spmm_grid((n + TR - 1) / TR, plane_tiles);
  k_spmm_stencil<T, PP, true><<<dim3((unsigned)grid), dim3(WG), 0, st>>>(
      n, dims[0], dims[1], dims[2], diag, (T)off, W, W, Z, nullptr, 0, plane_tiles, V, alpha, beta, gamma);
}
template <typename T, int PP>
void Kernels<T, PP>::spmm_fin(hipStream_t st, int64_t n, const int32_t* rowptr, const int32_t* colind,
                              const float* vals, const float* W, double* Z, const Scalars* sc, int mode,
                              int64_t plane_tiles, int batch) {
  const int64_t grid = spmm_grid((n + TR - 1) / TR, plane_tiles);
  if (batch == 7)
    k_spmm_fin<PP, 7><<<dim3((unsigned)grid), dim3(WG), 0, st>>>(n, rowptr, colind, vals, W, Z, sc, mode, plane_tiles);
  else
    k_spmm_fin<PP, 8><<<dim3((unsigned)grid), dim3(WG), 0, st>>>(n, rowptr, colind, vals, W, Z, sc, mode, plane_tiles);
}
template <typename T, int PP>
void Kernels<T, PP>::spmm16(hipStream_t st, int64_t n, const int32_t* rowptr, const int32_t* colind,
                            const uint16_t* vals, const uint16_t* W, float* Z, const Scalars* sc, int mode,
                            int64_t plane_tiles, int batch) {
  const int64_t grid = spmm_grid((n + TR - 1) / TR, plane_tiles);
  if (batch == 7)
    k_spmm16<PP, 7><<<dim3((unsigned)grid), dim3(WG), 0, st>>>(n, rowptr, colind, vals, W, Z, sc, mode, plane_tiles);
  else
    k_spmm16<PP, 8><<<dim3((unsigned)grid), dim3(WG), 0, st>>>(n, rowptr, colind, vals, W, Z, sc, mode, plane_tiles);
}
template <typename T, int PP>
void Kernels<T, PP>::update(hipStream_t st, int nb, int64_t n, T* X, T* Y, const T* P0, const T* P1, const T* Z,
                            const double* small, const Scalars* sc, double* partials, bool grams) {
  // the Gram epilogue exists up to PP = 64 (the host refuses explicit_c above)
  if constexpr (PP <= PP_LDS_MAX) {
    if (grams) {
      k_update<T, PP, true><<<nb, WG, lds_bytes<T, PP>(Pass::UpdateGrams), st>>>(n, X, Y, P0, P1, Z, small, sc,
                                                                               partials);
      return;
    }
  }
  k_update<T, PP, false><<<nb, WG, lds_bytes<T, PP>(Pass::Update), st>>>(n, X, Y, P0, P1, Z, small, sc, partials);
}
template <typename T, int PP>
void Kernels<T, PP>::spmm(hipStream_t st, int64_t n, const int32_t* rowptr, const int32_t* colind, const T* vals,
                          const T* W0, const T* W1, T* Z, const Scalars* sc, int mode, int64_t plane_tiles,
                          int batch) {
  const int64_t grid = spmm_grid((n + TR - 1) / TR, plane_tiles);
  if (batch == 7)
    k_spmm<T, PP, 7><<<dim3((unsigned)grid), dim3(WG), 0, st>>>(n, rowptr, colind, vals, W0, W1, Z, sc, mode,
                                                               plane_tiles);
  else
    k_spmm<T, PP, 8><<<dim3((unsigned)grid), dim3(WG), 0, st>>>(n, rowptr, colind, vals, W0, W1, Z, sc, mode,
                                                               plane_tiles);
}
template <typename T, int PP>
void Kernels<T, PP>::gram(hipStream_t st, int nb, int64_t n, const T* A0, const T* A1, const T* B1, const T* B2,
                          const Scalars* sc, int mode, double* partials) {
  if constexpr (PP == 64) {
    // the staged pass; with one Gram (B2 == nullptr: X^T X of the orthonormalization,
    // X^T A X of the Rayleigh-Ritz step) only B1 is staged
    if (B2)
      k_gram2<T, PP, true><<<nb, WG, 2 * TR * PP * sizeof(T), st>>>(n, A0, A1, B1, B2, sc, mode, partials);
    else
      k_gram2<T, PP, false><<<nb, WG, TR * PP * sizeof(T), st>>>(n, A0, A1, B1, B2, sc, mode, partials);
    return;
  }
  if constexpr (factor_wide<T, PP>()) {
    if (B2)
      k_gram_wide<T, PP, true><<<nb, WGW, 2 * WTILE * sizeof(double), st>>>(n, A0, A1, B1, B2, sc, mode, partials);
    else
      k_gram_wide<T, PP, false><<<nb, WGW, 2 * WTILE * sizeof(double), st>>>(n, A0, A1, B1, B2, sc, mode, partials);
    return;
  }
  k_gram<T, PP><<<nb, WG, 0, st>>>(n, A0, A1, B1, B2, sc, mode, partials);
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
  const int blocks = (int)((nv + 63) / 64);
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
template <typename T>
void launch_axpby(hipStream_t st, int64_t count, const T* Y, const T* X, T* Z, double a, double b) {
  hipLaunchKernelGGL((k_axpby<T>), dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count, Y, X, Z, a, b);
}
template void launch_axpby<double>(hipStream_t, int64_t, const double*, const double*, double*, double, double);
void launch_to_bf16(hipStream_t st, int64_t count, const double* src, uint16_t* dst, double scale) {
  hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count, src, dst, scale);
}
void launch_csr_check(hipStream_t st, int nb, int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colind,
                      const double* vals, double* partial_max, int* flags, double* partial_band) {
  hipLaunchKernelGGL(k_csr_check, dim3(nb), dim3(WG), 0, st, n, nnz, rowptr, colind, vals, partial_max, flags,
                     partial_band);
}
template <typename T>
void launch_stencil_diag(hipStream_t st, int64_t n, double d, const double* dv, double scale, T* out) {
  hipLaunchKernelGGL(k_stencil_diag<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, d, dv, scale, out);
}
template void launch_stencil_diag<double>(hipStream_t, int64_t, double, const double*, double, double*);
template void launch_stencil_diag<float>(hipStream_t, int64_t, double, const double*, double, float*);
void launch_stencil_check(hipStream_t st, int nb, int64_t n, const int32_t* dims, double d, double off,
                          const double* dv, double* partial_max, int* flags) {
  hipLaunchKernelGGL(k_stencil_check, dim3(nb), dim3(WG), 0, st, n, dims[0], dims[1], dims[2], d, off, dv,
                     partial_max, flags);
}
void launch_complex_extract(hipStream_t st, int64_t n, int pc, int PP, const double* X, double* out) {
  const int64_t count = n * pc;
  if (count > 0)
    hipLaunchKernelGGL(k_complex_extract, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, n, pc, PP, X, out);
}
void launch_finite(hipStream_t st, int64_t count, const double* x, int* flags) {
  hipLaunchKernelGGL(k_finite, dim3(1024), dim3(256), 0, st, count, x, flags);
}

template struct Kernels<double, 16>;
template struct Kernels<double, 32>;
template struct Kernels<double, 64>;
template struct Kernels<double, 128>;
template struct Kernels<float, 128>;
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
