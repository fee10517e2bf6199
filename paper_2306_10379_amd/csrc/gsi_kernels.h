// Host-side launchers of the device kernels (internal to libgsi).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gsi_device.h"
#include "gsi_state.h"

namespace gsi {

enum class Pass { Grad, Dir, Update, UpdateGrams, UpdateGrad, Spmm, SpmmPlain, Gram, Product };

// When a gradient pass, its reduction and its bookkeeping (after_grad) run. ALWAYS: every
// iteration (the unfused sequence). PENDING: at the top of an iteration of the fused sequence,
// only when the gradient is not current (the solve's first iteration, after an explicit A X, a
// void step or a host-side change of the state). AFTER_FUSED: at the end of an iteration of the
// fused sequence, when its retraction pass formed the gradient (a step was taken and A X was
// carried by the recursion).
enum GradCond { GRAD_ALWAYS = 0, GRAD_PENDING = 4, GRAD_AFTER_FUSED = 5 };

template <typename T, int PP>
int lds_bytes(Pass pass);

// Streaming passes for block element type T and padded width PP.
template <typename T, int PP>
struct Kernels {
  static hipError_t init();
  static void grad(hipStream_t st, int nb, int64_t n, const T* X, const T* Y, T* G0, T* G1, const double* small,
                   const Scalars* sc, double* partials, int cond = GRAD_ALWAYS);
  // P16 / P32 (nullable): bfloat16 / float32 copy of P written beside it
  static void dir(hipStream_t st, int nb, int64_t n, const T* X, const T* G0, const T* G1, T* P0, T* P1,
                  const double* small, const Scalars* sc, double* partials, uint16_t* P16 = nullptr,
                  float* P32 = nullptr);
  static void update(hipStream_t st, int nb, int64_t n, T* X, T* Y, const T* P0, const T* P1, const T* Z,
                     const double* small, const Scalars* sc, double* partials, bool grams);
  // the retraction fused with the next gradient (k_update_grad); partials as for grad
  static void update_grad(hipStream_t st, int nb, int64_t n, T* X, T* Y, const T* P0, const T* P1, const T* Z,
                          T* G0, T* G1, const double* small, const Scalars* sc, double* partials);
  // plane_tiles > 0: banded tile order (see spmm_tile in gsi_kernels.hip); 0: one slab per XCD
  static void spmm(hipStream_t st, int64_t n, const int32_t* rowptr, const int32_t* colind, const T* vals,
                   const T* W0, const T* W1, T* Z, const Scalars* sc, int mode, int64_t plane_tiles = 0,
                   int batch = 8);
  // A^T B1 (and A^T B2 when B2 != nullptr); mode as for spmm (mode 1 picks A0/A1 by parity)
  static void gram(hipStream_t st, int nb, int64_t n, const T* A0, const T* A1, const T* B1, const T* B2,
                   const Scalars* sc, int mode, double* partials);
  static void product(hipStream_t st, int nb, int64_t n, const T* IN, T* OUT, const double* M);
  // Z = A W with bfloat16 values and W, float32 accumulation and output
  static void spmm16(hipStream_t st, int64_t n, const int32_t* rowptr, const int32_t* colind, const uint16_t* vals,
                     const uint16_t* W, float* Z, const Scalars* sc, int mode, int64_t plane_tiles = 0,
                     int batch = 8);
  // Z = alpha (A W) + beta W + gamma V (V nullable), always runs
  static void spmm_axpy(hipStream_t st, int64_t n, const int32_t* rowptr, const int32_t* colind, const T* vals,
                        const T* W, const T* V, T* Z, double alpha, double beta, double gamma,
                        int64_t plane_tiles = 0, int batch = 8);
  // Z (float64) = A W from float32 values and W, float64 products and accumulation
  static void spmm_fin(hipStream_t st, int64_t n, const int32_t* rowptr, const int32_t* colind, const float* vals,
                       const float* W, double* Z, const Scalars* sc, int mode, int64_t plane_tiles = 0,
                       int batch = 8);
  static void colres(hipStream_t st, int nb, int64_t n, const T* X, const T* Y, const double* theta,
                     double* partials);
  // matrix-free stencil operator on the grid dims[0] x dims[1] x dims[2] (host array):
  // diagonal diag[r], `off` at each neighbour; mode as for spmm
  static void spmm_stencil(hipStream_t st, int64_t n, const int32_t* dims, const T* diag, double off, const T* W0,
                           const T* W1, T* Z, const Scalars* sc, int mode, int64_t plane_tiles = 0);
  // Z = alpha (A W) + beta W + gamma V for the stencil operator, always runs
  static void spmm_stencil_axpy(hipStream_t st, int64_t n, const int32_t* dims, const T* diag, double off,
                                const T* W, const T* V, T* Z, double alpha, double beta, double gamma,
                                int64_t plane_tiles = 0);
};

void launch_reduce(hipStream_t st, const double* partials, int nb, int64_t nv, int64_t max_from, double* out,
                   const Scalars* sc, int cond);
void launch_set_sym(hipStream_t st, int PP, const double* red, double* dst);
void launch_to_bf16(hipStream_t st, int64_t count, const double* src, uint16_t* dst, double scale);
template <typename T>
void launch_axpby(hipStream_t st, int64_t count, const T* Y, const T* X, T* Z, double a, double b);
template <typename T>
void launch_pack(hipStream_t st, int64_t n, int p, int PP, const double* src, T* dst, double scale);
template <typename T>
void launch_unpack(hipStream_t st, int64_t n, int p, int PP, const T* src, double* dst);
template <typename TS, typename TD>
void launch_convert(hipStream_t st, int64_t count, const TS* src, TD* dst, double scale);
void launch_csr_check(hipStream_t st, int nb, int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colind,
                      const double* vals, double* partial_max, int* flags,
                      double* partial_band = nullptr);
void launch_finite(hipStream_t st, int64_t count, const double* x, int* flags);
void launch_complex_extract(hipStream_t st, int64_t n, int pc, int PP, const double* X, double* out);
template <typename T>
void launch_stencil_diag(hipStream_t st, int64_t n, double d, const double* dv, double scale, T* out);
void launch_stencil_check(hipStream_t st, int nb, int64_t n, const int32_t* dims, double d, double off,
                          const double* dv, double* partial_max, int* flags);

// Single-workgroup p x p solves (gsi_small.hip). All read/write the small buffer and the
// scalars; `red` is the reduced partial-sum vector of the preceding pass.
struct Small {
  static hipError_t init();
  // after the gradient pass: rho, history, stop test, Polak-Ribiere beta, K + beta W; marks the
  // gradient current (grad_ready). cond (GradCond): when it runs
  static void after_grad(hipStream_t st, int PP, const double* red, double* small, Scalars* sc, double* hist,
                         int cond = 0);
  // after the direction pass: S = P^T P, descent test
  static void after_dir(hipStream_t st, int PP, const double* red, double* small, Scalars* sc);
  // eigendecomposition of P^T P (warm-started); independent of the SpMM
  static void eig(hipStream_t st, int PP, double* small, Scalars* sc);
  // after the SpMM: line-search diagonals, Get_Mu, M, next C and W (and M C_next for the fused
  // retraction-gradient pass); marks the gradient stale (the step changes X, or is void)
  static void linesearch(hipStream_t st, int PP, const double* red, double* small, Scalars* sc, double* hist,
                         int recompute_ax, bool want_mc = false);
  // after an update with Gram epilogue: C = sym(X^T Y), W = X^T P (explicit)
  static void after_update_grams(hipStream_t st, int PP, const double* red, double* small, Scalars* sc);
  // after an explicit A X: C = sym(X^T Y) (runs only when sc->refresh)
  static void after_refresh(hipStream_t st, int PP, const double* red, double* small, Scalars* sc);
  // Cholesky factor of the reduced Gram (PP x PP): writes R^{-1} into small[S_M]; flag on failure
  static void chol_inv(hipStream_t st, int PP, int p, const double* red, double* small, int* flag);
  // after a Cholesky QR pass with R^{-1} in small[S_M]: C <- R^{-T} C R^{-1}, W <- R^{-T} W;
  // when *flag is set (the factorization failed) M is reset to I and C, W are kept
  static void transform_cw(hipStream_t st, int PP, double* small, int* flag);
  // eigendecomposition of sym(red) (p x p): theta (descending) into out_vals, U into small[S_M]
  static void ritz(hipStream_t st, int PP, int p, const double* red, double* small, double* out_vals);
};

}  // namespace gsi
