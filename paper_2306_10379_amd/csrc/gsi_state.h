// Per-solve device state shared by the kernels and the host driver.
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace gsi {

// History fields per recorded iterate.
enum { H_RHO = 0, H_PHI, H_MU, H_BETA, H_GINF, H_FIELDS };

// Scalars, flags and counters; one instance in device memory per solve.
struct Scalars {
  double gg;        // <G, G>
  double gdot;      // <G_old, G>
  double ginf;      // ||G||_inf (max absolute row sum)
  double gp;        // <G, P>
  double gg_old;    // <G_old, G_old>
  double rho, phi, ginf0;
  double mu, beta_pr;
  double nA;        // ||A||_inf
  double tol;
  double sqrt_p;
  int32_t k;            // accepted iterations
  int32_t done;         // 0 running, 1 converged, 2 max_iter, 3 breakdown
  int32_t restart_next; // next direction is the projected gradient
  int32_t null_step;    // current iteration takes no step
  int32_t restart;      // current direction is a restart
  int32_t refresh;      // A X is formed explicitly after this update
  int32_t brent_evals;
  int32_t max_iter, k_restart, method, p;
  int32_t n_restart, n_refresh, n_null, n_spmm;
  int32_t hist_len, hist_cap;
  int32_t v_valid;      // small[S_V] holds the previous eigenvectors of P^T P (warm start)
  int32_t sweeps;       // Jacobi sweeps of the last eigendecomposition
  int32_t n_sweeps;     // Jacobi sweeps, summed over the solve
  int32_t stall_window; // > 0: stop (done = 4) when rho has not halved for this many iterations
  double rho_best;      // smallest rho so far (halving checkpoints)
  int32_t k_best;
  int32_t grad_ready;    // G, its sums and the stop test are current for X (set by the gradient's
                         // bookkeeping, cleared when X is about to change or a step is void)
};

// Offsets (in doubles) of the p x p matrices (stored PP x PP, row-major) in the small buffer.
enum {
  S_C = 0,   // C = sym(X^T A X)
  S_K,       // X^T G
  S_KD,      // K + beta W: right factor of the direction pass
  S_W,       // X^T P_old
  S_S,       // P^T P
  S_PZ,      // P^T A P
  S_PY,      // P^T A X
  S_V,       // eigenvectors of P^T P (also kept as the next warm start)
  S_M,       // retraction factor V diag((1 + mu^2 b)^-1/2) V^T
  S_MC,      // M C_next: the right factor of the next gradient in the fused retraction pass
  S_T1,      // temporaries
  S_T2,
  S_VEC,     // vectors of length PP: b (eigenvalues of P^T P), then scratch
  S_COUNT
};

// Block widths above 64 (p up to 128, float64): a PP x PP float64 matrix is 128 KB, so the
// single-workgroup p x p kernels keep their working matrices in a work area after the slots
// and vectors instead of LDS: [0, 3 PP (PP + 1)) for the eigendecomposition of P^T P, which
// runs beside the SpMM on a second stream, [4 PP (PP + 1), 8 PP (PP + 1)) for the others.
constexpr int PP_LDS_MAX = 64;
constexpr size_t small_work_offset(int PP) { return (size_t)S_COUNT * PP * PP + 8 * (size_t)PP; }
constexpr size_t small_work_doubles(int PP) { return PP > PP_LDS_MAX ? (size_t)8 * PP * (PP + 1) : 0; }
constexpr size_t small_doubles(int PP) { return small_work_offset(PP) + small_work_doubles(PP); }

}  // namespace gsi
