/* Learned warm start for the subspace iteration: a sine-basis neural operator that maps a
 * potential V on an N x N grid to a start block of p columns for H = -Laplacian + V, with
 * its forward pass, training gradient and Adam step as hand-written gfx950 kernels.
 *
 * Why: the convergence bounds of Sec. 4 run from the angle between the start block and the
 * wanted invariant subspace, so a start block closer to it (the random start of Sec. 6 is
 * the fallback) needs fewer iterations to the same residual; the solver still runs to the
 * tolerance, so the network can only cost iterations, never accuracy.
 *
 * Network (widths w, sine modes m, L hidden layers, p outputs), float32 activations with
 * float32 accumulation (the p x p loss algebra in float64); the weights are float32, or,
 * with bf16_weights set, a bfloat16 working copy of a float32 master (below):
 *   In  = [V / 20, x, y]                       x = (col + 1)/(N + 1), y = (row + 1)/(N + 1)
 *   U_0 = W_lift In + b_lift                   pointwise 3 -> w
 *   U_{l+1} = gelu(K_l(U_l) + W_l U_l + b_l)   l = 0 .. L-1, gelu(t) = t Phi_n(t), Phi_n the normal CDF
 *   Y   = Phi + K_out(U_L) + W_out U_L + b_out w -> p, no activation
 *   K(U)[o] = S^T (sum_c R[o][c] .* (S U[c] S^T)) S, S[k][i] = sqrt(2/(N+1)) sin(pi (k+1)(i+1)/(N+1)), k < m
 *   Phi: fixed prior, column a = sqrt(n) times the a-th lowest Dirichlet mode of the grid
 *   Laplacian s_l(row) s_k(col), s_k(i) = sqrt(2/(N+1)) sin(pi k (i+1)/(N+1)), ordered by
 *   k^2 + l^2, then k: the exact eigenvectors for V = 0, so the network learns the correction
 *   the potential makes (a zero output layer returns the free modes).
 * Loss per sample with Y read as n x p (n = N^2, column a = channel a) and target X*
 * (orthonormal n x p): p - Tr((Y^T Y)^-1 (X*^T Y)^T (X*^T Y)), the sum of squared sines of the
 * principal angles between span(Y) and span(X*); a batch loss is the mean.
 *
 * Flat parameter vector (float32, this order): W_lift (w x 3, [c][a]), b_lift (w); per hidden
 * layer R (w x w x m x m, [o][c][k1][k2]), W (w x w, [o][c]), b (w); R_out (p x w x m x m),
 * W_out (p x w), b_out (p). The gradient uses the same layout.
 *
 * bfloat16 weights (bf16_weights = 1): every parameter the forward and backward passes read
 * comes from a bfloat16 copy of the float32 parameter vector, each entry rounded to nearest
 * (ties to even) when the vector is set (creation, fno_set_params) and after every Adam step;
 * the products with those weights widen them to float32 and accumulate in float32. The
 * gradient is the float32 gradient of the loss at the rounded weights, and Adam updates the
 * float32 master (fno_get_params returns the master), so steps smaller than a bfloat16 ulp
 * still accumulate.
 *
 * Limits: N a multiple of 16, N <= 1024; 1 <= m <= 32, m <= N; 1 <= w <= 32; 1 <= p <= 32;
 * L >= 0; batch 1 .. max_batch; bf16_weights 0 or 1. All pointers to data are device pointers owned by the
 * caller; calls are ordered on the stream given at creation; no call allocates after
 * fno_create. Errors: GSI_EINVAL for sizes or null pointers, GSI_ENOMEM, GSI_EDEVICE
 * (HIP error, or a singular Gram Y^T Y in the loss: message in fno_last_error). */
#ifndef FNO_H
#define FNO_H
#include <stdint.h>

#include "gsi.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fno_net* fno_handle;

typedef struct {
  int32_t N;          /* grid side */
  int32_t modes;      /* m */
  int32_t width;      /* w */
  int32_t layers;     /* L */
  int32_t p;          /* output columns */
  int32_t max_batch;  /* largest batch of any call */
  int32_t bf16_weights; /* 0: float32 weights; 1: bfloat16 working copy of a float32 master */
} fno_config;

/* Number of parameters of cfg (also the gradient length); -1 for an invalid cfg. */
int64_t fno_param_count(const fno_config* cfg);

/* Creates the network with parameters drawn from a seeded normal distribution (b = 0; W_lift
 * std 1/sqrt(3); hidden R, W std 1/sqrt(w); the output layer R_out, W_out, b_out zero, so
 * that the untrained network returns the prior) and Adam moments at zero. *h is set even
 * on failure (for the message) and must be destroyed. */
gsi_status fno_create(fno_handle* h, const fno_config* cfg, uint64_t seed, void* hip_stream);

/* Copy parameters in from / out to a device array of fno_param_count floats. */
gsi_status fno_set_params(fno_handle h, const float* params);
gsi_status fno_get_params(fno_handle h, float* params);

/* Forward pass for B potentials V (device, B x N^2 float32, row-major grid). Writes Y as B
 * blocks of n x p row-major: float32 into Y32 and/or float64 into Y64 (each nullable). */
gsi_status fno_forward(fno_handle h, const float* V, int32_t B, float* Y32, double* Y64);

/* Forward pass, loss and gradient for B potentials V and targets Xs (device, B blocks of
 * n x p row-major float32 with orthonormal columns). loss: host array of B per-sample
 * losses (nullable); grad: device array of fno_param_count floats receiving the gradient of
 * the mean loss (nullable; the gradient is also kept for fno_adam). Syncs. */
gsi_status fno_loss_grad(fno_handle h, const float* V, const float* Xs, int32_t B, double* loss, float* grad);

/* One Adam step (Kingma and Ba) on the gradient of the last fno_loss_grad, with bias
 * correction by the handle's own step count. */
gsi_status fno_adam(fno_handle h, float lr, float beta1, float beta2, float eps);

const char* fno_last_error(fno_handle h);
void fno_destroy(fno_handle h);

#ifdef __cplusplus
}
#endif
#endif /* FNO_H */
