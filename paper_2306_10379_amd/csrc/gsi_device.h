// Device-side building blocks shared by the gsi kernels (gfx950, wave64).
//
// Tall n x p blocks are row-major with leading dimension PP = 16, 32 or 64, the smallest
// that holds p (padding columns are kept at zero). A workgroup has 4 waves; a wave owns 16-row
// tiles. Dense contractions use MFMA 16x16x4 (f64 or f32):
//   A operand (16 x 4):  lane l holds A[l % 16][l / 16]
//   B operand (4 x 16):  lane l holds B[l / 16][l % 16]
//   D (16 x 16):         f64: lane l, reg r holds D[l/16 + 4r][l % 16]
//                        f32: lane l, reg r holds D[4(l/16) + r][l % 16]
// "RL" is the D layout of a 16 x PP tile: slot [cb][r] of lane (g = l/16, c = l%16) is
// element (rowof(g, r), 16 cb + c). "AL" is the A-operand layout of a 16 x PP tile with a
// permuted contraction index kappa(s, g); see load_al.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gsi {

constexpr int WG = 256;      // threads per workgroup
constexpr int TR = 64;       // rows per workgroup tile (4 waves x 16 rows)

// Whether a PP x PP factor of element type T is too wide for LDS beside a tile (above 64 KB:
// float64 at PP = 128); such passes read it through the caches.
template <typename T, int PP>
constexpr bool factor_wide() { return (size_t)PP * PP * sizeof(T) > 65536; }

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

template <typename T> struct Vec4;
template <> struct Vec4<double> { typedef d4 type; };
template <> struct Vec4<float> { typedef f4 type; };

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Row (within a 16-row tile) of D-layout register r for lane group g.
template <typename T> __device__ __forceinline__ int rowof(int g, int r);
template <> __device__ __forceinline__ int rowof<double>(int g, int r) { return g + 4 * r; }
template <> __device__ __forceinline__ int rowof<float>(int g, int r) { return 4 * g + r; }

// Contraction-index permutation for AL loads: each lane reads E = 16/sizeof(T)
// consecutive elements (16 bytes) per load; k-step s of lane group g uses column
// kappa(s, g) = 4E * (s / E) + E * g + (s % E).
template <typename T> struct AL {
  static constexpr int E = 16 / (int)sizeof(T);
  __device__ __forceinline__ static int kappa(int s, int g) { return 4 * E * (s / E) + E * g + (s % E); }
};

// Global-memory accesses through pointers the compiler cannot trace to a kernel argument
// (loaded from memory, or parameters of out-of-line functions) compile to flat_*
// instructions, which count on the LDS counter too, so that every wait for an LDS read
// drains all loads in flight. gld / gst access through a global-address-space pointer
// (global_* instructions); to_lds does the same for LDS pointers.
template <typename T>
__device__ __forceinline__ T gld(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ void gst(T* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}
template <typename T>
__device__ __forceinline__ T* to_lds(T* p) {
  return (T*)((__attribute__((address_space(3))) T*)p);
}

// bfloat16 (the upper 16 bits of a float32): rounding to nearest, ties to even, and
// widening. NaN stays NaN (quiet bit forced).
__device__ __forceinline__ uint16_t bf16_round(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x0040u);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_widen(uint32_t b) { return __uint_as_float(b << 16); }

// ---------------------------------------------------------------- tile I/O (per wave)

template <typename T, int PP>
__device__ __forceinline__ void zero_rl(T (&v)[PP / 16][4]) {
#pragma unroll
  for (int cb = 0; cb < PP / 16; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) v[cb][r] = T(0);
}

template <typename T, int PP>
__device__ __forceinline__ void load_rl(const T* __restrict__ B, int64_t row0, int64_t n, T (&v)[PP / 16][4]) {
  const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t row = row0 + rowof<T>(g, r);
    const bool ok = row < n;
    const T* p = B + (ok ? row : 0) * PP + c;
#pragma unroll
    for (int cb = 0; cb < PP / 16; ++cb) v[cb][r] = ok ? gld(p + 16 * cb) : T(0);
  }
}

template <typename T, int PP>
__device__ __forceinline__ void store_rl(T* __restrict__ B, int64_t row0, int64_t n, const T (&v)[PP / 16][4]) {
  const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t row = row0 + rowof<T>(g, r);
    if (row < n) {
      T* p = B + row * PP + c;
#pragma unroll
      for (int cb = 0; cb < PP / 16; ++cb) gst(p + 16 * cb, v[cb][r]);
    }
  }
}

// A-operand layout: lane (g, c) holds row c; k-step s holds column kappa(s, g).
template <typename T, int PP>
__device__ __forceinline__ void load_al(const T* __restrict__ B, int64_t row0, int64_t n, T (&a)[PP / 4]) {
  constexpr int E = AL<T>::E;
  const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
  const int64_t row = row0 + c;
  const bool ok = row < n;
  const T* p = B + (ok ? row : 0) * PP + E * g;
#pragma unroll
  for (int t = 0; t < PP / (4 * E); ++t) {
    if constexpr (E == 2) {
      const d2 q = ok ? gld(reinterpret_cast<const d2*>(p + 4 * E * t)) : d2{0.0, 0.0};
      a[E * t + 0] = q.x;
      a[E * t + 1] = q.y;
    } else {
      const f4 q = ok ? gld(reinterpret_cast<const f4*>(p + 4 * E * t)) : f4{0.f, 0.f, 0.f, 0.f};
      a[E * t + 0] = q.x;
      a[E * t + 1] = q.y;
      a[E * t + 2] = q.z;
      a[E * t + 3] = q.w;
    }
  }
}

// acc[ncb] (RL, 16 x PP) += A (AL, 16 x PP) * M (PP x PP, row-major in LDS).
template <typename T, int PP>
__device__ __forceinline__ void product(const T (&a)[PP / 4], const T* __restrict__ M,
                                        typename Vec4<T>::type (&acc)[PP / 16]) {
  const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
#pragma unroll
  for (int s = 0; s < PP / 4; ++s) {
    const T* mrow = M + AL<T>::kappa(s, g) * PP + c;
#pragma unroll
    for (int ncb = 0; ncb < PP / 16; ++ncb) acc[ncb] = mfma(a[s], mrow[16 * ncb], acc[ncb]);
    // at PP = 128 the unrolled loop holds 256 operand loads, which the scheduler would issue
    // all at once (spilling); one k-step at a time keeps 8 in flight
    if constexpr (PP > 64) __builtin_amdgcn_sched_barrier(0);
  }
}

// Two products with the same right factor: acc1 += A1 * M, acc2 += A2 * M.
template <typename T, int PP>
__device__ __forceinline__ void product2(const T (&a1)[PP / 4], const T (&a2)[PP / 4], const T* __restrict__ M,
                                         typename Vec4<T>::type (&acc1)[PP / 16],
                                         typename Vec4<T>::type (&acc2)[PP / 16]) {
  const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
#pragma unroll
  for (int s = 0; s < PP / 4; ++s) {
    const T* mrow = M + AL<T>::kappa(s, g) * PP + c;
#pragma unroll
    for (int ncb = 0; ncb < PP / 16; ++ncb) {
      const T b = mrow[16 * ncb];
      acc1[ncb] = mfma(a1[s], b, acc1[ncb]);
      acc2[ncb] = mfma(a2[s], b, acc2[ncb]);
    }
    if constexpr (PP > 64) __builtin_amdgcn_sched_barrier(0);  // as in product
  }
}

template <typename T, int PP>
__device__ __forceinline__ void zero_acc(typename Vec4<T>::type (&acc)[PP / 16]) {
#pragma unroll
  for (int cb = 0; cb < PP / 16; ++cb) acc[cb] = typename Vec4<T>::type{0, 0, 0, 0};
}

// ---------------------------------------------------------------- Gram phase (per workgroup)
//
// The workgroup's TR x PP tiles of A and B sit row-major in LDS (A may also be a tile in
// global memory with the same layout). Output blocks
// (ib, jb) of A^T B (16 x 16 each, NBK = PP/16 per side) are dealt round-robin to the
// 4 waves; a wave keeps its blocks in registers across all tiles it processes.
template <int PP>
struct GramSplit {
  static constexpr int NBK = PP / 16;
  static constexpr int NBLK = NBK * NBK;
  static constexpr int PER_WAVE = (NBLK + 3) / 4;
};

template <typename T, int PP>
__device__ __forceinline__ void gram_zero(typename Vec4<T>::type (&acc)[GramSplit<PP>::PER_WAVE]) {
#pragma unroll
  for (int q = 0; q < GramSplit<PP>::PER_WAVE; ++q) acc[q] = typename Vec4<T>::type{0, 0, 0, 0};
}

template <typename T, int PP>
__device__ __forceinline__ void gram_tile(const T* __restrict__ sA, const T* __restrict__ sB,
                                          typename Vec4<T>::type (&acc)[GramSplit<PP>::PER_WAVE]) {
  using GS = GramSplit<PP>;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, c = l & 15;
#pragma unroll
  for (int q = 0; q < GS::PER_WAVE; ++q) {
    const int blk = w + 4 * q;
    if (blk < GS::NBLK) {
      const int ib = blk / GS::NBK, jb = blk % GS::NBK;
#pragma unroll 4
      for (int s = 0; s < TR / 4; ++s) {
        const int row = 4 * s + g;
        acc[q] = mfma(sA[row * PP + 16 * ib + c], sB[row * PP + 16 * jb + c], acc[q]);
      }
    }
    // at PP = 128 (16 blocks per wave) one block's loads at a time (as in product)
    if constexpr (PP > 64) __builtin_amdgcn_sched_barrier(0);
  }
}

// Write a wave's Gram blocks (as double) into a PP x PP row-major output.
template <typename T, int PP>
__device__ __forceinline__ void gram_store(double* __restrict__ out,
                                           const typename Vec4<T>::type (&acc)[GramSplit<PP>::PER_WAVE]) {
  using GS = GramSplit<PP>;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, c = l & 15;
#pragma unroll
  for (int q = 0; q < GS::PER_WAVE; ++q) {
    const int blk = w + 4 * q;
    if (blk < GS::NBLK) {
      const int ib = blk / GS::NBK, jb = blk % GS::NBK;
#pragma unroll
      for (int r = 0; r < 4; ++r) out[(16 * ib + rowof<T>(g, r)) * PP + 16 * jb + c] = (double)acc[q][r];
    }
  }
}

// Symmetric Gram A^T A of the workgroup's LDS tile: only the blocks (ib, jb) with ib <= jb are
// formed, dealt round-robin to the 4 waves (at PP = 64: 10 blocks, at most 3 per wave instead of
// 4). A block and its mirror multiply the same pairs of elements in the same order, so writing
// the mirror gives bit for bit what the full product gives.
template <int PP>
struct SymSplit {
  static constexpr int NBK = PP / 16;
  static constexpr int NBLK = NBK * (NBK + 1) / 2;
  static constexpr int PER_WAVE = (NBLK + 3) / 4;
};

// Block (ib, jb), ib <= jb, of upper-triangle index blk (row by row).
template <int PP>
__device__ __forceinline__ void sym_block(int blk, int& ib, int& jb) {
  ib = 0;
#pragma unroll
  for (int i = 0; i < PP / 16; ++i) {
    const int cnt = PP / 16 - i;
    if (blk >= cnt && ib == i) {
      blk -= cnt;
      ib = i + 1;
    }
  }
  jb = ib + blk;
}

template <typename T, int PP>
__device__ __forceinline__ void gram_tile_sym(const T* __restrict__ sA,
                                              typename Vec4<T>::type (&acc)[SymSplit<PP>::PER_WAVE]) {
  using SS = SymSplit<PP>;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, c = l & 15;
#pragma unroll
  for (int q = 0; q < SS::PER_WAVE; ++q) {
    const int blk = w + 4 * q;
    if (blk < SS::NBLK) {
      int ib, jb;
      sym_block<PP>(blk, ib, jb);
#pragma unroll 4
      for (int s = 0; s < TR / 4; ++s) {
        const int row = 4 * s + g;
        acc[q] = mfma(sA[row * PP + 16 * ib + c], sA[row * PP + 16 * jb + c], acc[q]);
      }
    }
    if constexpr (PP > 64) __builtin_amdgcn_sched_barrier(0);  // as in gram_tile
  }
}

// Write a wave's blocks of a symmetric Gram and the mirrors of its off-diagonal blocks.
template <typename T, int PP>
__device__ __forceinline__ void gram_store_sym(double* __restrict__ out,
                                               const typename Vec4<T>::type (&acc)[SymSplit<PP>::PER_WAVE]) {
  using SS = SymSplit<PP>;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, c = l & 15;
#pragma unroll
  for (int q = 0; q < SS::PER_WAVE; ++q) {
    const int blk = w + 4 * q;
    if (blk < SS::NBLK) {
      int ib, jb;
      sym_block<PP>(blk, ib, jb);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * ib + rowof<T>(g, r), j = 16 * jb + c;
        out[i * PP + j] = (double)acc[q][r];
        if (ib != jb) out[j * PP + i] = (double)acc[q][r];
      }
    }
  }
}

// Store a wave's RL tile into the workgroup LDS tile (rows 16*wave ...).
template <typename T, int PP>
__device__ __forceinline__ void rl_to_lds(T* __restrict__ s, const T (&v)[PP / 16][4]) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, c = l & 15;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int cb = 0; cb < PP / 16; ++cb) s[(16 * w + rowof<T>(g, r)) * PP + 16 * cb + c] = v[cb][r];
}

// ---------------------------------------------------------------- reductions

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
// Sum over the 16 lanes of a lane group (lanes with equal l / 16).
__device__ __forceinline__ double group16_sum(double v) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Workgroup reduction of NV values per thread; result valid in thread 0.
template <int NV>
__device__ __forceinline__ void wg_sum(double (&v)[NV], double* __restrict__ scratch /* 4*NV */) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = wave_sum(v[i]);
    if (l == 0) scratch[w * NV + i] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = scratch[i] + scratch[NV + i] + scratch[2 * NV + i] + scratch[3 * NV + i];
  }
  __syncthreads();
}

// XCD-aware tile range: workgroups are dealt round-robin to the 8 XCDs; give the
// workgroups of one XCD adjacent chunks of rows so its L2 sees a contiguous slab.
__device__ __forceinline__ void tile_range(int64_t ntiles, int64_t& t0, int64_t& t1) {
  const int nb = gridDim.x, b = blockIdx.x;
  int logical = b;
  if ((nb & 7) == 0) logical = (b & 7) * (nb >> 3) + (b >> 3);
  const int64_t per = (ntiles + nb - 1) / nb;
  t0 = (int64_t)logical * per;
  t1 = t0 + per < ntiles ? t0 + per : ntiles;
  if (t0 > ntiles) t0 = ntiles;
}

}  // namespace gsi
