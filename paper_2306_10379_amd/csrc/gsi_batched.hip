// Batched solve: many independent eigenproblems of different n and p in one persistent
// launch. Every workgroup pulls problem indices from an atomic queue (largest problems
// first) and runs the whole Riemannian CG iteration for one problem with workgroup barriers
// (once the queue has drained, a running problem may recruit idle workgroups into a team
// that splits its rows; see k_batched): gradient, direction, eigendecomposition of P^T P, SpMM, Grams, line search and
// retraction (the same steps and readings as the single-problem path, see gsi_kernels.hip
// and gsi_small.hip). The p x p state is float64. Blocks are float64, or float32 first and
// float64 after: the float32 phase runs until rho <= switch_tol (or rho stops improving),
// then the iterate, the previous gradient and the previous direction are widened and the
// iteration continues in float64 to tol without a restart.
//
// One workgroup owns a problem, so it must keep many loads in flight by itself: the
// streaming passes issue the loads of 2-4 tiles before using any of them, every wave takes
// part in each Gram (partial sums combined across waves in a fixed order), and the SpMM
// gathers the nonzeros of a row in batches of 8.
//
// Passes read rows that other waves of the same workgroup wrote in the previous pass; an
// agent-scope fence (L1 invalidation) plus a barrier separates passes.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <utility>
#include <new>
#include <string>
#include <vector>

#include <type_traits>

#include "../../include/gsi.h"
#include "gsi_kernels.h"
#include "gsi_small_dev.h"

namespace gsi {

constexpr int NBLK = 7;      // X, Y, G0, G1, P0, P1, Z
constexpr int TMAX = 16;     // largest team of workgroups on one problem
constexpr int TPM_MIN = 4;   // fewest 64-row tiles per team member that storage is sized for
// default team policy (gsi_batched_set_tuning changes it): fewest tiles per member,
// workgroups recruited at one check, iterations between checks
constexpr int TPM_DEF = 16, GROW_DEF = 4, ESC_DEF = 32;

struct BatchProblem {
  int64_t n;
  int32_t p, PP;
  const int32_t* rowptr;
  const int32_t* colind;
  const void* vals[2];      // [0] float32, [1] float64 values (negated for the smallest), null if unused
  void* blk[2][NBLK];       // float32 / float64 blocks: whole 64-row tiles, PP columns, null if unused
  const double* X0;         // packed start block (float64, PP columns)
  double* small;            // tmax x S_COUNT x PP x PP: p x p state of each team member
  double* xch;              // 2 x TMAX x (2 PP^2 + 8) exchange slots (tmax > 1 only)
  double nA;                // ||A||_inf
  double* ritz;             // p outputs (Ritz values of the operator solved)
  int32_t tmax, team;       // largest team allowed this solve / team size reached
  int32_t tcap, tiles;      // member storage allocated; row tiles
  int32_t iters, iters_low, status, restarts, null_steps;
  int32_t shape;            // tile shape of the passes (see Shape); 0 = the defaults of Unroll
  double rho;
  int64_t t_begin, t_switch, t_end;  // device wall clock
  int64_t ticks[GSI_NPASS];          // wall-clock ticks per pass (first member)
};

// Loop state handed by a problem's first member to the workgroups that join it.
struct LoopState {
  int32_t k, k_best, restart_next, v_valid, phase, team, base, xc;
  double gg_old, rho_best;
};

struct QEntry {
  int32_t prob, rank;
};

struct BatchCtl {
  int32_t headA;  // queue of problems to start (stage 1)
  int32_t count;
  int32_t headB, tailB;  // queue of team-member entries
  int32_t idle;          // workgroups waiting for work, minus entries reserved for them
  int32_t active;        // problems not finished
  int32_t abort;         // set on a team wait timeout: every workgroup leaves
  int32_t method, k_restart, max_iter, stall_window, recompute_ax, mixed, pad;
  int32_t tpm, grow_step, esc_every, pad2;  // team policy
  double tol, switch_tol;
  int64_t timeout_ticks;  // longest wait at a team barrier (wall-clock ticks)
  const int32_t* order;   // stage-1 queue order (problem indices)
  QEntry* qB;             // count x (TMAX - 1) entries
  int32_t* readyB;        // entry published flags
  int32_t* bars;          // per-problem team barrier counters
  int32_t* grow;          // per-problem number of workgroups recruited at the last check
  LoopState* ls;          // per-problem loop state at the last recruitment
};

// State handed from the float32 phase to the float64 phase.
struct Resume {
  int k;          // iteration reached
  double gg_old;  // <G_{k-1}, G_{k-1}>
  int carry;      // G_{k-1} and P_{k-1} sit in the buffers of parity (k-1) & 1
};

// One workgroup's part in a problem: rank among t members, its tiles [ta, tb) and rows
// [r0, r1), the barrier counter value when the team took its present size (base), the
// barriers passed since (gen) and the exchange counter (all equal in all members).
struct Team {
  int rank, t, gen, xc, base;
  int64_t ta, tb, r0, r1;
  __device__ void set(int rk, int tt, int64_t n) {
    rank = rk;
    t = tt;
    const int64_t nt = (n + TR - 1) / TR;
    ta = nt * rk / tt;
    tb = nt * (rk + 1) / tt;
    r0 = ta * TR;
    r1 = tb * TR < n ? tb * TR : n;
  }
};

__device__ __forceinline__ int ld_acq(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void pass_barrier() {
  __threadfence();
  __syncthreads();
}

// Tiles whose loads are issued together in the streaming passes (the defaults, sized so that
// no pass spills registers): U for the passes reading three blocks, UU for the retraction
// (four blocks), UG for the Grams; CH nonzeros gathered per batch in the SpMM.
template <typename T, int PP>
struct Unroll {
  static constexpr int U = sizeof(T) * PP >= 256 ? 2 : 4;
  static constexpr int UU = sizeof(T) * PP >= 256 ? 1 : 2;
  static constexpr int UG = PP == 16 ? 4 : (sizeof(T) == 8 ? 1 : 2);
  static constexpr int CH = 8;
};

// Per-problem tile shape (BatchProblem::shape, set by gsi_batched_set_shapes from the tuner's
// table): 4-bit fields u (bits 0-3), uu (4-7), ug (8-11), ch (12-15), each 0 for the default
// of Unroll or one of the built values: u, ug in {1, 2, 4}, uu in {1, 2}, ch in {4, 8, 16}
// (16 coded as 15).
struct Shape {
  int u, uu, ug, ch;
  template <typename T, int PP>
  __device__ static Shape of(int32_t code) {
    Shape s;
    const int cu = code & 15, cuu = (code >> 4) & 15, cug = (code >> 8) & 15, cch = (code >> 12) & 15;
    s.u = cu ? cu : Unroll<T, PP>::U;
    s.uu = cuu ? cuu : Unroll<T, PP>::UU;
    s.ug = cug ? cug : Unroll<T, PP>::UG;
    s.ch = cch == 15 ? 16 : (cch ? cch : Unroll<T, PP>::CH);
    return s;
  }
};

// f(integral_constant<int, v>) for v in {1, 2, 4} (2 for anything else) / {4, 8, 16} (8).
template <typename F>
__device__ __forceinline__ void with_124(int v, F&& f) {
  if (v == 1) f(std::integral_constant<int, 1>());
  else if (v == 4) f(std::integral_constant<int, 4>());
  else f(std::integral_constant<int, 2>());
}
template <typename F>
__device__ __forceinline__ void with_12(int v, F&& f) {
  if (v == 1) f(std::integral_constant<int, 1>());
  else f(std::integral_constant<int, 2>());
}
template <typename F>
__device__ __forceinline__ void with_48_16(int v, F&& f) {
  if (v == 4) f(std::integral_constant<int, 4>());
  else if (v == 16) f(std::integral_constant<int, 16>());
  else f(std::integral_constant<int, 8>());
}

// ---------------------------------------------------------------- streaming passes (one workgroup)

template <typename T, int PP>
__device__ void b_load_matrix(T* __restrict__ s, const double* __restrict__ M) {
  for (int i = threadIdx.x; i < PP * PP; i += blockDim.x) s[i] = (T)gld(M + i);
}

// G = X C - Y over tiles [ta, tb); sums of G^2 and G_old G, max absolute row sum.
template <typename T, int PP, int U>
__device__ __noinline__ void b_grad(int64_t n, int64_t ta, int64_t tb, const T* X, const T* Y, const T* Gold, T* G,
                                    const T* sC, bool have_old, double* sums) {
  const int w = threadIdx.x >> 6;
  sC = to_lds(sC);
  double gg = 0.0, gdot = 0.0, ginf = 0.0;
  for (int64_t t = ta; t < tb; t += U) {
    T a[U][PP / 4], y[U][PP / 16][4], go[U][PP / 16][4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t row0 = (t + u) * TR + 16 * w, nv = t + u < tb ? n : 0;
      load_al<T, PP>(X, row0, nv, a[u]);
      load_rl<T, PP>(Y, row0, nv, y[u]);
      if (have_old) load_rl<T, PP>(Gold, row0, nv, go[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t row0 = (t + u) * TR + 16 * w, nv = t + u < tb ? n : 0;
      typename Vec4<T>::type acc[PP / 16];
      zero_acc<T, PP>(acc);
      product<T, PP>(a[u], sC, acc);
      T g[PP / 16][4];
#pragma unroll
      for (int cb = 0; cb < PP / 16; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) g[cb][r] = acc[cb][r] - y[u][cb][r];
      store_rl<T, PP>(G, row0, nv, g);
      double rs[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int cb = 0; cb < PP / 16; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double gv = (double)g[cb][r];
          gg += gv * gv;
          rs[r] += fabs(gv);
          if (have_old) gdot += (double)go[u][cb][r] * gv;
        }
#pragma unroll
      for (int r = 0; r < 4; ++r) ginf = fmax(ginf, group16_sum(rs[r]));
    }
  }
  sums[0] = gg;
  sums[1] = gdot;
  sums[2] = ginf;
}

// P = G + beta P_old - X KD over tiles [ta, tb); sum of G P.
template <typename T, int PP, int U>
__device__ __noinline__ void b_dir(int64_t n, int64_t ta, int64_t tb, const T* X, const T* G, const T* Pold, T* P,
                                   const T* sK, T beta, bool use_old, double* sums) {
  const int w = threadIdx.x >> 6;
  sK = to_lds(sK);
  double gp = 0.0;
  for (int64_t t = ta; t < tb; t += U) {
    T a[U][PP / 4], g[U][PP / 16][4], po[U][PP / 16][4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t row0 = (t + u) * TR + 16 * w, nv = t + u < tb ? n : 0;
      load_al<T, PP>(X, row0, nv, a[u]);
      load_rl<T, PP>(G, row0, nv, g[u]);
      if (use_old) load_rl<T, PP>(Pold, row0, nv, po[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t row0 = (t + u) * TR + 16 * w, nv = t + u < tb ? n : 0;
      typename Vec4<T>::type acc[PP / 16];
      zero_acc<T, PP>(acc);
      product<T, PP>(a[u], sK, acc);
      T pn[PP / 16][4];
#pragma unroll
      for (int cb = 0; cb < PP / 16; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          pn[cb][r] = g[u][cb][r] + (use_old ? beta * po[u][cb][r] : T(0)) - acc[cb][r];
          gp += (double)g[u][cb][r] * (double)pn[cb][r];
        }
      store_rl<T, PP>(P, row0, nv, pn);
    }
  }
  sums[0] = gp;
}

// X <- (X - mu P) M, Y <- (Y - mu Z) M over tiles [ta, tb) (Y skipped when upd_y is false).
template <typename T, int PP, int U>
__device__ __noinline__ void b_update(int64_t n, int64_t ta, int64_t tb, T* X, T* Y, const T* P, const T* Z,
                                      const T* sM, T mu, bool upd_y) {
  const int w = threadIdx.x >> 6;
  sM = to_lds(sM);
  for (int64_t t = ta; t < tb; t += U) {
    T a1[U][PP / 4], b1[U][PP / 4], a2[U][PP / 4], b2[U][PP / 4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t row0 = (t + u) * TR + 16 * w, nv = t + u < tb ? n : 0;
      load_al<T, PP>(X, row0, nv, a1[u]);
      load_al<T, PP>(P, row0, nv, b1[u]);
      if (upd_y) {
        load_al<T, PP>(Y, row0, nv, a2[u]);
        load_al<T, PP>(Z, row0, nv, b2[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t row0 = (t + u) * TR + 16 * w, nv = t + u < tb ? n : 0;
#pragma unroll
      for (int s = 0; s < PP / 4; ++s) a1[u][s] = a1[u][s] - mu * b1[u][s];
      typename Vec4<T>::type xacc[PP / 16], yacc[PP / 16];
      zero_acc<T, PP>(xacc);
      zero_acc<T, PP>(yacc);
      if (upd_y) {
#pragma unroll
        for (int s = 0; s < PP / 4; ++s) a2[u][s] = a2[u][s] - mu * b2[u][s];
        product2<T, PP>(a1[u], a2[u], sM, xacc, yacc);
      } else {
        product<T, PP>(a1[u], sM, xacc);
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
      store_rl<T, PP>(X, row0, nv, xo);
      if (upd_y) store_rl<T, PP>(Y, row0, nv, yo);
    }
  }
}

// IN <- IN M in place over tiles [ta, tb).
template <typename T, int PP, int U>
__device__ __noinline__ void b_product(int64_t n, int64_t ta, int64_t tb, T* IN, const T* sM) {
  const int w = threadIdx.x >> 6;
  sM = to_lds(sM);
  for (int64_t t = ta; t < tb; t += U) {
    T a[U][PP / 4];
#pragma unroll
    for (int u = 0; u < U; ++u) load_al<T, PP>(IN, (t + u) * TR + 16 * w, t + u < tb ? n : 0, a[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      typename Vec4<T>::type acc[PP / 16];
      zero_acc<T, PP>(acc);
      product<T, PP>(a[u], sM, acc);
      T o[PP / 16][4];
#pragma unroll
      for (int cb = 0; cb < PP / 16; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) o[cb][r] = acc[cb][r];
      store_rl<T, PP>(IN, (t + u) * TR + 16 * w, t + u < tb ? n : 0, o);
    }
  }
}

// E consecutive elements at p (E * sizeof(T) bytes, naturally aligned), zeros when !ok.
template <typename T, int E>
__device__ __forceinline__ void load_run(const T* __restrict__ p, bool ok, T (&d)[E]) {
  if constexpr (E * sizeof(T) == 32) {
    const d2* q = reinterpret_cast<const d2*>(p);
    const d2 u = ok ? gld(q) : d2{0.0, 0.0}, v = ok ? gld(q + 1) : d2{0.0, 0.0};
    d[0] = u.x; d[1] = u.y; d[2] = v.x; d[3] = v.y;
  } else if constexpr (E * sizeof(T) == 16 && sizeof(T) == 8) {
    const d2 u = ok ? gld(reinterpret_cast<const d2*>(p)) : d2{0.0, 0.0};
    d[0] = u.x; d[1] = u.y;
  } else if constexpr (E * sizeof(T) == 16) {
    const f4 u = ok ? gld(reinterpret_cast<const f4*>(p)) : f4{0.f, 0.f, 0.f, 0.f};
    d[0] = u.x; d[1] = u.y; d[2] = u.z; d[3] = u.w;
  } else if constexpr (E == 2 && sizeof(T) == 4) {
    const f2 u = ok ? gld(reinterpret_cast<const f2*>(p)) : f2{0.f, 0.f};
    d[0] = u.x; d[1] = u.y;
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) d[e] = ok ? gld(p + e) : T(0);
  }
}

// Z = A W over rows [r0, r1): LPR lanes per row, 4 columns per lane, nonzeros of a row
// gathered in batches of CH so that the index loads and the gathers of a batch overlap.
template <typename T, int PP, int CH>
__device__ __noinline__ void b_spmm(int64_t r0, int64_t r1, const int32_t* rowptr, const int32_t* colind,
                                    const T* vals, const T* W, T* Z) {
  constexpr int EPL = 4, LPR = PP / EPL, RPB = WG / LPR;
  const int sub = threadIdx.x / LPR, lane = threadIdx.x % LPR;
  for (int64_t row = r0 + sub; row < r1; row += RPB) {
    T acc[EPL] = {T(0), T(0), T(0), T(0)};
    const int32_t j0 = gld(rowptr + row), j1 = gld(rowptr + row + 1);
    for (int32_t jb = j0; jb < j1; jb += CH) {
      int32_t col[CH];
      T v[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const bool ok = jb + u < j1;
        col[u] = ok ? gld(colind + jb + u) : -1;
        v[u] = ok ? gld(vals + jb + u) : T(0);
      }
      T src[CH][EPL];
#pragma unroll
      for (int u = 0; u < CH; ++u)
        load_run<T, EPL>(W + (int64_t)(col[u] < 0 ? 0 : col[u]) * PP + EPL * lane, col[u] >= 0, src[u]);
#pragma unroll
      for (int u = 0; u < CH; ++u)
#pragma unroll
        for (int e = 0; e < EPL; ++e) acc[e] += v[u] * src[u][e];
    }
    T* zr = Z + row * PP + EPL * lane;
#pragma unroll
    for (int e = 0; e < EPL; ++e) gst(zr + e, acc[e]);
  }
}

// out1 = A^T B1, out2 = A^T B2 (B2 may be null) over tiles [ta, tb): PP x PP float64.
// Lane (g, c) of every wave owns columns V c .. V c + V - 1 (V = PP / 16) of the rows
// 16 w + 4 s + g of each tile and keeps all (16 V)^2 products of its column runs in MFMA
// accumulators; the waves' partial sums are then added in wave order through red (LDS,
// 2 PP^2 doubles). Output (V i + ib, V j + jb) comes from accumulator [ib][jb], D row i,
// column j. Blocks span whole tiles with zero padding rows, so only the tile index is
// checked.
template <typename T, int PP, int U>
__device__ __noinline__ void b_gram(int64_t ta, int64_t tb, const T* A, const T* B1, const T* B2, double* out1,
                                    double* out2, double* red) {
  constexpr int V = PP / 16;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, c = l & 15;
  const bool two = B2 != nullptr;
  red = to_lds(red);
  typename Vec4<T>::type acc1[V][V], acc2[V][V];
#pragma unroll
  for (int ib = 0; ib < V; ++ib)
#pragma unroll
    for (int jb = 0; jb < V; ++jb) {
      acc1[ib][jb] = typename Vec4<T>::type{0, 0, 0, 0};
      acc2[ib][jb] = typename Vec4<T>::type{0, 0, 0, 0};
    }
  for (int64_t t = ta; t < tb; t += U) {
    T a[U][4][V], b1[U][4][V], b2[U][4][V];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool ok = t + u < tb;
      const int64_t off = ((ok ? t + u : ta) * TR + 16 * w + g) * PP + V * c;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        load_run<T, V>(A + off + 4 * s * PP, ok, a[u][s]);
        load_run<T, V>(B1 + off + 4 * s * PP, ok, b1[u][s]);
        if (two) load_run<T, V>(B2 + off + 4 * s * PP, ok, b2[u][s]);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int ib = 0; ib < V; ++ib)
#pragma unroll
          for (int jb = 0; jb < V; ++jb) {
            acc1[ib][jb] = mfma(a[u][s][ib], b1[u][s][jb], acc1[ib][jb]);
            if (two) acc2[ib][jb] = mfma(a[u][s][ib], b2[u][s][jb], acc2[ib][jb]);
          }
  }
  for (int ww = 0; ww < 4; ++ww) {
    if (w == ww) {
#pragma unroll
      for (int ib = 0; ib < V; ++ib)
#pragma unroll
        for (int jb = 0; jb < V; ++jb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int e = (rowof<T>(g, r) * V + ib) * PP + c * V + jb;
            red[e] = (ww ? red[e] : 0.0) + (double)acc1[ib][jb][r];
            if (two) red[PP * PP + e] = (ww ? red[PP * PP + e] : 0.0) + (double)acc2[ib][jb][r];
          }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) {
    gst(out1 + e, red[e]);
    if (two) gst(out2 + e, red[PP * PP + e]);
  }
}

// dst (float64) <- src (T) over n_el elements.
template <typename T>
__device__ void b_widen(int64_t n_el, const T* __restrict__ src, double* __restrict__ dst) {
  for (int64_t i = threadIdx.x; i < n_el; i += blockDim.x) gst(dst + i, (double)gld(src + i));
}

// dst (T) <- src (float64) over n_el elements.
template <typename T>
__device__ void b_narrow(int64_t n_el, const double* __restrict__ src, T* __restrict__ dst) {
  for (int64_t i = threadIdx.x; i < n_el; i += blockDim.x) gst(dst + i, (T)gld(src + i));
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
  double xv[8];
  double smu, sbmax;
  int uv[MAXP];
  int nrot, anyr, sok, sevals, bad, restart_next, flag, want, job, rank;
};

// Wall-clock ticks spent per pass (indices of the GSI_PASS_* enumeration).
struct PassClock {
  int64_t last;
  int64_t* tk;
  __device__ void mark(int slot) {
    const int64_t now = wall_clock64();
    tk[slot] += now - last;
    last = now;
  }
};

// Barrier over the t workgroups of a team: every member's global writes before it are
// visible to every member after it. Returns false (in all threads) when the wait exceeds
// the time limit or another workgroup has aborted the launch.
__device__ bool team_sync(Team& tm, BatchCtl* ctl, int32_t* bar, BatchShared& sh) {
  ++tm.gen;
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    __threadfence();
    atomicAdd(bar, 1);
    const int target = tm.base + tm.gen * tm.t;
    const int64_t t0 = wall_clock64();
    while (ld_acq(bar) < target) {
      if (ld_acq(&ctl->abort)) { ok = 0; break; }
      if (wall_clock64() - t0 > ctl->timeout_ticks) {
        st_rel(&ctl->abort, 1);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __threadfence();
    sh.flag = ok;
  }
  __syncthreads();
  return sh.flag != 0;
}

template <int PP>
__device__ __forceinline__ double* xslot(const BatchProblem& pr, int set, int m) {
  return pr.xch + ((int64_t)set * TMAX + m) * (2 * PP * PP + 8);
}

// Partial results of this member: nmat PP x PP matrices already in its slot of the current
// set (written by b_gram), ns sums and nx maxima in v. Afterwards d1 (and d2) hold the
// team sums of the matrices and v the team sums / maxima, added in member order so that
// every member holds the same values.
template <int PP>
__device__ bool exchange(Team& tm, BatchCtl* ctl, BatchProblem& pr, int32_t* bar, BatchShared& sh, int nmat,
                         double* d1, double* d2, double* v, int ns, int nx) {
  const int set = tm.xc & 1;
  ++tm.xc;
  if (threadIdx.x == 0)
    for (int j = 0; j < ns + nx; ++j) gst(xslot<PP>(pr, set, tm.rank) + 2 * PP * PP + j, v[j]);
  if (!team_sync(tm, ctl, bar, sh)) return false;
  const double* s0 = xslot<PP>(pr, set, 0);
  constexpr int XW = 2 * PP * PP + 8;
  for (int e = threadIdx.x; e < nmat * PP * PP; e += blockDim.x) {
    double acc = 0.0;
    for (int m = 0; m < tm.t; ++m) acc += gld(s0 + (int64_t)m * XW + e);
    if (e < PP * PP)
      gst(d1 + e, acc);
    else
      gst(d2 + e - PP * PP, acc);
  }
  if (threadIdx.x < ns + nx) {
    const int j = threadIdx.x;
    double acc = j < ns ? 0.0 : -INFINITY;
    for (int m = 0; m < tm.t; ++m) {
      const double x = gld(s0 + (int64_t)m * XW + 2 * PP * PP + j);
      acc = j < ns ? acc + x : fmax(acc, x);
    }
    sh.xv[j] = acc;
  }
  __syncthreads();
  for (int j = 0; j < ns + nx; ++j) v[j] = sh.xv[j];
  __syncthreads();
  return true;
}

// Gram of this member's tiles into dst (one workgroup) or into its exchange slot (team).
template <typename T, int PP>
__device__ void gram_part(const Team& tm, BatchProblem& pr, const T* A, const T* B1, const T* B2, double* d1,
                          double* d2, double* dl) {
  const int ug = Shape::of<T, PP>(pr.shape).ug;
  with_124(ug, [&](auto U) {
    if (tm.t == 1) {
      b_gram<T, PP, decltype(U)::value>(tm.ta, tm.tb, A, B1, B2, d1, d2, dl);
    } else {
      double* slot = xslot<PP>(pr, tm.xc & 1, tm.rank);
      b_gram<T, PP, decltype(U)::value>(tm.ta, tm.tb, A, B1, B2, slot, B2 ? slot + PP * PP : nullptr, dl);
    }
  });
}

// Gram plus scalars over the team (a plain barrier for a lone workgroup).
template <typename T, int PP>
__device__ bool team_gram(Team& tm, BatchCtl* ctl, BatchProblem& pr, int32_t* bar, BatchShared& sh, const T* A,
                          const T* B1, const T* B2, double* d1, double* d2, double* dl, double* v, int ns, int nx) {
  gram_part<T, PP>(tm, pr, A, B1, B2, d1, d2, dl);
  if (tm.t == 1) {
    pass_barrier();
    return true;
  }
  return exchange<PP>(tm, ctl, pr, bar, sh, B2 ? 2 : 1, d1, d2, v, ns, nx);
}

// One phase of the iteration for one problem, blocks of type T. A fresh phase starts from
// the X in the T block set (orthonormalized here by two Cholesky QR passes); with rs.carry
// it resumes at rs.k with the previous gradient and direction already in the buffers of
// parity (rs.k - 1) & 1 (widened from the float32 phase), so the first direction is not a
// restart. A workgroup joining a running problem (join != null) enters the loop with the
// state published by the first member. Stops at rho <= tol (1), max_iter (2), breakdown (3),
// with stall_window > 0 when rho has not halved for stall_window iterations (4), or on an
// aborted team wait (5). On return rs describes the state reached.
template <typename T, int PP>
__device__ __noinline__ int solve_phase(BatchProblem& pr, BatchCtl* ctl, int idx, unsigned char* lds,
                                        BatchShared& sh, Resume& rs, double tol, int stall_window, PassClock& clk,
                                        Team& tm, const LoopState* join) {
  constexpr int SI = sizeof(T) == 4 ? 0 : 1;
  const int64_t n = pr.n;
  const int p = pr.p;
  int32_t* bar = ctl->bars + idx;
  T* X = (T*)pr.blk[SI][0];
  T* Y = (T*)pr.blk[SI][1];
  T* Gb[2] = {(T*)pr.blk[SI][2], (T*)pr.blk[SI][3]};
  T* Pb[2] = {(T*)pr.blk[SI][4], (T*)pr.blk[SI][5]};
  T* Z = (T*)pr.blk[SI][6];
  const T* vals = (const T*)pr.vals[SI];
  double* small = pr.small + (int64_t)tm.rank * S_COUNT * PP * PP;
  T* sMat = reinterpret_cast<T*>(lds);
  double* dl = reinterpret_cast<double*>(lds + PP * PP * sizeof(double) + 64);
  double* C = small + S_C * PP * PP;
  double* K = small + S_K * PP * PP;
  double* KD = small + S_KD * PP * PP;
  double* W = small + S_W * PP * PP;
  double* S = small + S_S * PP * PP;
  double* PZ = small + S_PZ * PP * PP;
  double* PY = small + S_PY * PP * PP;
  double* M = small + S_M * PP * PP;
  double* G2 = small + S_T1 * PP * PP;
  double* G3 = small + S_T2 * PP * PP;
  const double sqrt_p = sqrt((double)p);
  const bool carry = rs.carry && rs.k > 0;
  const Shape shp = Shape::of<T, PP>(pr.shape);
  int k, k_best, restarts = 0, nulls = 0, stop = 0;
  double gg_old, rho = 0.0, rho_best;
  bool v_valid;
  double v[4];
  if (join) {
    k = join->k;
    k_best = join->k_best;
    gg_old = join->gg_old;
    rho_best = join->rho_best;
    v_valid = join->v_valid != 0;
    if (threadIdx.x == 0) sh.restart_next = join->restart_next;
    __syncthreads();
  } else {
    for (int e = threadIdx.x; e < S_COUNT * PP * PP; e += blockDim.x) small[e] = 0.0;
    pass_barrier();
    // orthonormalize X: two Cholesky QR passes
    bool ok = true;
    for (int pass = 0; pass < 2 && ok; ++pass) {
      if (!team_gram<T, PP>(tm, ctl, pr, bar, sh, X, X, nullptr, G2, nullptr, dl, v, 0, 0)) { stop = 5; break; }
      ok = b_chol_inv<PP>(G2, M, p, dl, &sh.bad);
      b_load_matrix<T, PP>(sMat, M);
      __syncthreads();
      if (ok) with_124(shp.u, [&](auto U) { b_product<T, PP, decltype(U)::value>(n, tm.ta, tm.tb, X, sMat); });
      pass_barrier();
    }
    if (stop == 0 && tm.t > 1 && !team_sync(tm, ctl, bar, sh)) stop = 5;
    clk.mark(GSI_PASS_REFRESH);
    if (stop == 0 && !ok) stop = 3;
    if (stop) {
      rs.carry = 0;
      if (threadIdx.x == 0 && tm.rank == 0) { pr.status = stop; pr.iters = rs.k; pr.rho = NAN; }
      __syncthreads();
      return stop;
    }
    // Y = A X, C = sym(X^T Y); with a carried direction also W = X^T P_old
    with_48_16(shp.ch, [&](auto C) { b_spmm<T, PP, decltype(C)::value>(tm.r0, tm.r1, pr.rowptr, pr.colind, vals, X, Y); });
    pass_barrier();
    if (!team_gram<T, PP>(tm, ctl, pr, bar, sh, X, Y, carry ? Pb[(rs.k - 1) & 1] : nullptr, G2, carry ? W : nullptr,
                          dl, v, 0, 0)) {
      rs.carry = 0;
      if (threadIdx.x == 0 && tm.rank == 0) { pr.status = 5; pr.iters = rs.k; pr.rho = NAN; }
      __syncthreads();
      return 5;
    }
    for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) C[e] = 0.5 * (G2[e] + G2[(e % PP) * PP + e / PP]);
    pass_barrier();
    clk.mark(GSI_PASS_REFRESH);
    k = carry ? rs.k : 0;
    k_best = k;
    gg_old = carry ? rs.gg_old : 0.0;
    rho_best = 0.0;
    v_valid = false;
    if (threadIdx.x == 0) sh.restart_next = 0;
    __syncthreads();
  }
  const int k_first = join ? -1 : k;
  int k_check = join ? k : -1;
  for (;;) {
    // every esc_every iterations, once the stage-1 queue has drained, the first member
    // recruits idle workgroups; a team meets at a barrier to learn the outcome, then the
    // enlarged team meets the recruits, which copy the first member's p x p state
    if (k % ctl->esc_every == 0 && k != k_check && tm.t < pr.tmax) {
      k_check = k;
      if (threadIdx.x == 0 && tm.rank == 0) {
        int want = 0;
        if (ld_acq(&ctl->headA) >= ctl->count && !ld_acq(&ctl->abort)) {
          const int room = pr.tmax - tm.t < ctl->grow_step ? pr.tmax - tm.t : ctl->grow_step;
          int cur = ld_acq(&ctl->idle);
          while (cur > 0) {
            const int w = cur < room ? cur : room;
            const int old = atomicCAS(&ctl->idle, cur, cur - w);
            if (old == cur) { want = w; break; }
            cur = old;
          }
        }
        if (want > 0) {
          LoopState* ls = ctl->ls + idx;
          ls->k = k;
          ls->k_best = k_best;
          ls->restart_next = sh.restart_next;
          ls->v_valid = v_valid ? 1 : 0;
          ls->phase = SI;
          ls->team = tm.t + want;
          ls->base = tm.base + (tm.t > 1 ? (tm.gen + 1) * tm.t : 0);
          ls->xc = tm.xc;
          ls->gg_old = gg_old;
          ls->rho_best = rho_best;
          __threadfence();
          const int slot0 = atomicAdd(&ctl->tailB, want);
          for (int j = 0; j < want; ++j) {
            ctl->qB[slot0 + j].prob = idx;
            ctl->qB[slot0 + j].rank = tm.t + j;
          }
          __threadfence();
          for (int j = 0; j < want; ++j) st_rel(ctl->readyB + slot0 + j, 1);
        }
        if (tm.t > 1) st_rel(ctl->grow + idx, want);
        sh.want = want;
      }
      if (tm.t > 1) {
        if (!team_sync(tm, ctl, bar, sh)) { stop = 5; break; }
        if (threadIdx.x == 0) sh.want = ld_acq(ctl->grow + idx);
      }
      __syncthreads();
      const int want = sh.want;
      __syncthreads();
      if (want > 0) {
        tm.base += tm.gen * tm.t;
        tm.gen = 0;
        tm.set(tm.rank, tm.t + want, n);
        if (!team_sync(tm, ctl, bar, sh)) { stop = 5; break; }
      }
    }
    const int par = k & 1;
    // gradient pass and K = X^T G
    b_load_matrix<T, PP>(sMat, C);
    __syncthreads();
    double sums[3];
    with_124(shp.u, [&](auto U) { b_grad<T, PP, decltype(U)::value>(n, tm.ta, tm.tb, X, Y, Gb[par ^ 1], Gb[par], sMat, k > 0, sums); });
    double gg = sums[0], gdot = sums[1], ginf = sums[2];
    b_reduce3(gg, gdot, ginf, sh.red);
    clk.mark(GSI_PASS_GRAD);
    v[0] = gg;
    v[1] = gdot;
    v[2] = ginf;
    if (!team_gram<T, PP>(tm, ctl, pr, bar, sh, X, Gb[par], nullptr, K, nullptr, dl, v, 2, 1)) { stop = 5; break; }
    gg = v[0];
    gdot = v[1];
    clk.mark(GSI_PASS_GRAM);
    rho = sqrt(gg) / (sqrt_p * pr.nA);
    if (k == k_first || rho <= 0.5 * rho_best) { rho_best = rho; k_best = k; }
    if (!isfinite(gg)) stop = 3;
    else if (rho <= tol) stop = 1;
    else if (k >= ctl->max_iter) stop = 2;
    else if (stall_window > 0 && k - k_best > stall_window) stop = 4;
    if (stop) break;
    const bool restart = ctl->method == GSI_RSD || k == 0 || sh.restart_next ||
                         (ctl->k_restart > 0 && k % ctl->k_restart == 0) || !(gg_old > 0.0);
    const double beta = restart ? 0.0 : (gg - gdot) / gg_old;
    for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) KD[e] = K[e] + (restart ? 0.0 : beta * W[e]);
    pass_barrier();
    // direction pass and S = P^T P
    b_load_matrix<T, PP>(sMat, KD);
    __syncthreads();
    clk.mark(GSI_PASS_SMALL);
    with_124(shp.u, [&](auto U) { b_dir<T, PP, decltype(U)::value>(n, tm.ta, tm.tb, X, Gb[par], Pb[par ^ 1], Pb[par], sMat, (T)beta, !restart, sums); });
    double gp = sums[0], dz1 = 0.0, dz2 = 0.0;
    b_reduce3(gp, dz1, dz2, sh.red);
    clk.mark(GSI_PASS_DIR);
    v[0] = gp;
    if (!team_gram<T, PP>(tm, ctl, pr, bar, sh, Pb[par], Pb[par], nullptr, G2, nullptr, dl, v, 1, 0)) {
      stop = 5;
      break;
    }
    gp = v[0];
    if (!(gp > 0.0)) {
      if (restart) { stop = 3; break; }
      ++nulls;
      if (threadIdx.x == 0) sh.restart_next = 1;
      __syncthreads();
      continue;
    }
    for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) S[e] = 0.5 * (G2[e] + G2[(e % PP) * PP + e / PP]);
    pass_barrier();
    clk.mark(GSI_PASS_GRAM);
    b_eig<PP>(small, p, v_valid, dl, sh.cs, sh.uv, &sh.nrot, &sh.anyr);
    v_valid = true;
    clk.mark(GSI_PASS_EIG);
    // SpMM of this member's rows (every row of P is final after the exchange above) and
    // the line-search Grams
    with_48_16(shp.ch, [&](auto C) { b_spmm<T, PP, decltype(C)::value>(tm.r0, tm.r1, pr.rowptr, pr.colind, vals, Pb[par], Z); });
    pass_barrier();
    clk.mark(GSI_PASS_SPMM);
    if (!team_gram<T, PP>(tm, ctl, pr, bar, sh, Pb[par], Z, Y, PZ, PY, dl, v, 0, 0)) { stop = 5; break; }
    clk.mark(GSI_PASS_GRAM);
    b_linesearch<PP>(PZ, PY, small, p, dl, sh.terms, &sh.smu, &sh.sok, &sh.sevals, &sh.sbmax);
    clk.mark(GSI_PASS_LINESEARCH);
    if (!sh.sok) {
      if (restart) { stop = 3; break; }
      ++nulls;
      if (threadIdx.x == 0) sh.restart_next = 1;
      __syncthreads();
      continue;
    }
    const double mu = sh.smu;
    const bool refresh = ctl->recompute_ax || mu * sqrt(sh.sbmax) <= 1e3 * EPS;
    restarts += restart ? 1 : 0;
    // retraction
    b_load_matrix<T, PP>(sMat, M);
    __syncthreads();
    with_12(shp.uu, [&](auto U) { b_update<T, PP, decltype(U)::value>(n, tm.ta, tm.tb, X, Y, Pb[par], Z, sMat, (T)mu, !refresh); });
    pass_barrier();
    clk.mark(GSI_PASS_UPDATE);
    if (refresh) {
      if (tm.t > 1 && !team_sync(tm, ctl, bar, sh)) { stop = 5; break; }
      with_48_16(shp.ch, [&](auto C) { b_spmm<T, PP, decltype(C)::value>(tm.r0, tm.r1, pr.rowptr, pr.colind, vals, X, Y); });
      pass_barrier();
      if (!team_gram<T, PP>(tm, ctl, pr, bar, sh, X, Y, nullptr, G3, nullptr, dl, v, 0, 0)) { stop = 5; break; }
      for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) C[e] = 0.5 * (G3[e] + G3[(e % PP) * PP + e / PP]);
      pass_barrier();
      clk.mark(GSI_PASS_REFRESH);
    }
    gg_old = gg;
    if (threadIdx.x == 0) sh.restart_next = 0;
    __syncthreads();
    ++k;
  }
  // the previous gradient and direction are those of iteration k - 1 unless this step
  // just restarted them
  rs.carry = (stop == 1 || stop == 2 || stop == 4) && k > 0 && gg_old > 0.0 && !sh.restart_next;
  rs.k = k;
  rs.gg_old = gg_old;
  if (threadIdx.x == 0 && tm.rank == 0) {
    pr.status = stop;
    pr.iters = k;
    pr.rho = rho;
    pr.restarts += restarts;
    pr.null_steps += nulls;
  }
  __syncthreads();
  return stop;
}

// Ritz values of the final C (eigenvalues of the operator solved, descending).
template <int PP>
__device__ __noinline__ void final_ritz(BatchProblem& pr, unsigned char* lds, BatchShared& sh) {
  double* small = pr.small;
  const int p = pr.p;
  double* dl = reinterpret_cast<double*>(lds + PP * PP * sizeof(double) + 64);
  double* C = small + S_C * PP * PP;
  double* S = small + S_S * PP * PP;
  pass_barrier();
  for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) S[e] = C[e];
  pass_barrier();
  b_eig<PP>(small, p, false, dl, sh.cs, sh.uv, &sh.nrot, &sh.anyr);
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

// Rows [ta, tb) tiles of src widened into dst.
template <int PP>
__device__ void widen_tiles(const Team& tm, const void* src, void* dst) {
  const int64_t e0 = tm.ta * TR * PP, e1 = tm.tb * TR * PP;
  b_widen<float>(e1 - e0, (const float*)src + e0, (double*)dst + e0);
}

// One workgroup's part in problem pr: the whole solve (rank 0, join == null) or, for a
// workgroup recruited into a running problem, from the published loop state to the end.
template <int PP>
__device__ __noinline__ void solve_problem(BatchProblem& pr, BatchCtl* ctl, int idx, unsigned char* lds,
                                           BatchShared& sh, int64_t* tk, int rank, const LoopState* join) {
  PassClock clk{wall_clock64(), tk};
  Resume rs{0, 0.0, 0};
  Team tm;
  tm.gen = 0;
  tm.xc = join ? join->xc : 0;
  tm.base = join ? join->base : 0;
  if (join) {
    tm.set(rank, join->team, pr.n);
    // copy the first member's p x p state, then meet the team
    const double* s0 = pr.small;
    double* sr = pr.small + (int64_t)rank * S_COUNT * PP * PP;
    for (int e = threadIdx.x; e < S_COUNT * PP * PP; e += blockDim.x) gst(sr + e, gld(s0 + e));
    if (!team_sync(tm, ctl, ctl->bars + idx, sh)) return;
  } else {
    tm.set(0, 1, pr.n);
    if (threadIdx.x == 0) { pr.restarts = 0; pr.null_steps = 0; pr.iters_low = 0; pr.team = 1; }
  }
  const int64_t nel = (pr.n + TR - 1) / TR * TR * PP;
  int phase = join ? join->phase : (ctl->mixed ? 0 : 1);
  if (phase == 0) {
    if (!join) {
      b_narrow<float>(nel, pr.X0, (float*)pr.blk[0][0]);
      pass_barrier();
    }
    const int st = solve_phase<float, PP>(pr, ctl, idx, lds, sh, rs, fmax(ctl->switch_tol, ctl->tol),
                                          ctl->stall_window, clk, tm, join);
    if (st == 5) return;
    join = nullptr;
    widen_tiles<PP>(tm, pr.blk[0][0], pr.blk[1][0]);
    if (rs.carry) {
      const int q = (rs.k - 1) & 1;
      widen_tiles<PP>(tm, pr.blk[0][2 + q], pr.blk[1][2 + q]);
      widen_tiles<PP>(tm, pr.blk[0][4 + q], pr.blk[1][4 + q]);
    }
    pass_barrier();
    if (threadIdx.x == 0 && tm.rank == 0) { pr.iters_low = rs.k; pr.t_switch = wall_clock64(); }
    clk.mark(GSI_PASS_SMALL);
  } else if (!join) {
    b_narrow<double>(nel, pr.X0, (double*)pr.blk[1][0]);
    pass_barrier();
  }
  const int st = solve_phase<double, PP>(pr, ctl, idx, lds, sh, rs, ctl->tol, 0, clk, tm, join);
  if (threadIdx.x == 0 && tm.rank == 0) pr.team = tm.t;
  if (st != 5 && tm.rank == 0) final_ritz<PP>(pr, lds, sh);
  clk.mark(GSI_PASS_SMALL);
}

// Persistent scheduler. A workgroup takes, in order of preference: a problem from the
// stage-1 queue (alone); a member entry of a team being formed; otherwise it waits as an
// idle workgroup (counted in ctl->idle, which problems reserve before posting entries, so
// that every posted entry has a waiting workgroup to take it) until no problem is left.
__global__ __launch_bounds__(WG) void k_batched(BatchProblem* __restrict__ probs, BatchCtl* __restrict__ ctl) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ BatchShared sh;
  int counted = 0;  // thread 0: this workgroup is counted in ctl->idle
  for (;;) {
    if (threadIdx.x == 0) {
      int job = -1, rank = 0;
      if (ld_acq(&ctl->headA) < ctl->count) {
        const int q = atomicAdd(&ctl->headA, 1);
        if (q < ctl->count) job = ctl->order[q];
      }
      if (job >= 0 && counted) {
        atomicSub(&ctl->idle, 1);
        counted = 0;
      }
      if (job < 0) {
        if (!counted) {
          atomicAdd(&ctl->idle, 1);
          counted = 1;
        }
        for (;;) {
          if (ld_acq(&ctl->abort)) break;
          const int h = ld_acq(&ctl->headB);
          if (h < ld_acq(&ctl->tailB)) {
            if (atomicCAS(&ctl->headB, h, h + 1) != h) continue;
            const int64_t t0 = wall_clock64();
            bool ok = true;
            while (!ld_acq(ctl->readyB + h)) {
              if (wall_clock64() - t0 > ctl->timeout_ticks) { st_rel(&ctl->abort, 1); ok = false; break; }
              __builtin_amdgcn_s_sleep(1);
            }
            __threadfence();
            if (ok) {
              job = ctl->qB[h].prob;
              rank = ctl->qB[h].rank;
              counted = 0;  // the reservation that posted the entry consumed the count
            }
            break;
          }
          if (ld_acq(&ctl->active) == 0) break;
          __builtin_amdgcn_s_sleep(127);
        }
      }
      sh.job = job;
      sh.rank = rank;
    }
    __syncthreads();
    const int idx = sh.job, rank = sh.rank;
    __syncthreads();
    if (idx < 0) return;
    BatchProblem pr = probs[idx];
    {
      const int cap = pr.tiles / ctl->tpm;
      pr.tmax = cap < 1 ? 1 : (cap < pr.tcap ? cap : pr.tcap);
    }
    int64_t tk[GSI_NPASS];
    for (int i = 0; i < GSI_NPASS; ++i) tk[i] = 0;
    if (rank > 0) {
      const LoopState st = ctl->ls[idx];
      if (pr.PP == 16)
        solve_problem<16>(pr, ctl, idx, lds_raw, sh, tk, rank, &st);
      else
        solve_problem<32>(pr, ctl, idx, lds_raw, sh, tk, rank, &st);
      continue;
    }
    const int64_t t_begin = wall_clock64();
    if (pr.PP == 16)
      solve_problem<16>(pr, ctl, idx, lds_raw, sh, tk, 0, nullptr);
    else
      solve_problem<32>(pr, ctl, idx, lds_raw, sh, tk, 0, nullptr);
    if (threadIdx.x == 0) {
      BatchProblem& o = probs[idx];
      o.iters = pr.iters;
      o.iters_low = pr.iters_low;
      o.status = pr.status;
      o.rho = pr.rho;
      o.restarts = pr.restarts;
      o.null_steps = pr.null_steps;
      o.team = pr.team;
      o.t_begin = t_begin;
      o.t_switch = ctl->mixed ? pr.t_switch : t_begin;
      o.t_end = wall_clock64();
      for (int i = 0; i < GSI_NPASS; ++i) o.ticks[i] = tk[i];
      __threadfence();
      atomicSub(&ctl->active, 1);
    }
    __syncthreads();
  }
}

// Per-solve reset of the queues, counters and team barriers (a kernel, so that the graph
// holds no memset node).
__global__ void k_batched_reset(BatchCtl* ctl) {
  const int count = ctl->count;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count * (TMAX - 1); i += gridDim.x * blockDim.x)
    ctl->readyB[i] = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) ctl->bars[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->headA = 0;
    ctl->headB = 0;
    ctl->tailB = 0;
    ctl->idle = 0;
    ctl->active = count;
    ctl->abort = 0;
  }
}

// dynamic LDS: product matrix (PP^2 doubles at most) + 64 bytes + 4 PP (PP+1) doubles
// (Jacobi, line search, Gram reduction)
constexpr int batched_lds() { return 32 * 32 * 8 + 64 + 4 * 32 * 33 * 8; }

}  // namespace gsi

using namespace gsi;

struct gsi_batch {
  hipStream_t st = nullptr;
  bool own_stream = false;
  int count = 0;
  int mixed = 0;
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

gsi_status fetch(gsi_batch* b, std::vector<BatchProblem>& res) {
  res.resize(b->count);
  hipError_t e = hipMemcpy(res.data(), b->dprobs, sizeof(BatchProblem) * b->count, hipMemcpyDeviceToHost);
  if (e != hipSuccess) { b->err = std::string("results: ") + hipGetErrorString(e); return GSI_EDEVICE; }
  return GSI_OK;
}

double tick_us() {
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
      khz <= 0)
    return 0.0;
  return 1e3 / (double)khz;
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
  b->mixed = opt->precision == GSI_MIXED_FP32;
  b->st = reinterpret_cast<hipStream_t>(stream);
  if (!b->st) {
    if (hipStreamCreate(&b->st) != hipSuccess) { b->err = "stream creation failed"; return GSI_EDEVICE; }
    b->own_stream = true;
  }
  if (opt->which != 1 && opt->which != -1) { b->err = "which must be +1 or -1"; return GSI_EINVAL; }
  if (opt->precision != GSI_FP64 && opt->precision != GSI_MIXED_FP32) { b->err = "unknown precision"; return GSI_EINVAL; }
  if (opt->method != GSI_RSD && opt->method != GSI_RCG) { b->err = "batched solves run RSD or RCG"; return GSI_EINVAL; }
  if (opt->recompute_ax != 0 && opt->recompute_ax != 1) { b->err = "recompute_ax must be 0 or 1"; return GSI_EINVAL; }
  for (int i = 0; i < count; ++i) {
    if (p[i] < 1 || p[i] > 32 || p[i] >= A[i].n || !A[i].rowptr || !A[i].colind || !A[i].vals || !X0[i]) {
      b->err = "problem " + std::to_string(i) + ": need 1 <= p <= 32, p < n and device arrays";
      return GSI_EINVAL;
    }
    if (A[i].n > INT32_MAX || A[i].nnz > INT32_MAX) { b->err = "n or nnz >= 2^31"; return GSI_EUNSUPPORTED; }
  }
  hipError_t e = hipSuccess;
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
    double* x0 = balloc<double>(b, blk, e);
    for (int si = b->mixed ? 0 : 1; si < 2; ++si) {
      const size_t es = si ? sizeof(double) : sizeof(float);
      pr.vals[si] = balloc<unsigned char>(b, nnz * es, e);
      for (int q = 0; q < NBLK; ++q) {
        pr.blk[si][q] = balloc<unsigned char>(b, blk * es, e);
        if (e == hipSuccess) e = hipMemsetAsync(pr.blk[si][q], 0, blk * es, b->st);
      }
    }
    const int64_t nt = (n + TR - 1) / TR;
    pr.tiles = (int32_t)nt;
    pr.tcap = (int)std::max<int64_t>(1, std::min<int64_t>(TMAX, nt / TPM_MIN));
    pr.small = balloc<double>(b, (size_t)pr.tcap * S_COUNT * PP * PP, e);
    if (pr.tcap > 1) pr.xch = balloc<double>(b, (size_t)2 * TMAX * (2 * PP * PP + 8), e);
    if (e != hipSuccess) { b->err = "allocation failed"; return GSI_ENOMEM; }
    if (e == hipSuccess) e = hipMemsetAsync(x0, 0, blk * sizeof(double), b->st);
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
    if (b->mixed) launch_convert<double, float>(b->st, nnz, A[i].vals, (float*)pr.vals[0], sign);
    launch_convert<double, double>(b->st, nnz, A[i].vals, (double*)pr.vals[1], sign);
    launch_pack<double>(b->st, n, p[i], PP, X0[i], x0, 1.0);
    pr.rowptr = rp;
    pr.colind = ci;
    pr.X0 = x0;
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
  QEntry* qB = balloc<QEntry>(b, (size_t)count * (TMAX - 1), e);
  int32_t* readyB = balloc<int32_t>(b, (size_t)count * (TMAX - 1), e);
  int32_t* bars = balloc<int32_t>(b, count, e);
  int32_t* grow = balloc<int32_t>(b, count, e);
  LoopState* ls = balloc<LoopState>(b, count, e);
  if (e != hipSuccess) { b->err = "allocation failed"; return GSI_ENOMEM; }
  BatchCtl ctl;
  memset(&ctl, 0, sizeof(ctl));
  ctl.count = count;
  ctl.method = opt->method;
  ctl.k_restart = opt->k_restart;
  ctl.max_iter = opt->max_iter;
  ctl.stall_window = opt->stall_window > 0 ? opt->stall_window : 60;
  ctl.recompute_ax = opt->recompute_ax;
  ctl.mixed = b->mixed;
  ctl.tol = opt->tol;
  ctl.switch_tol = opt->switch_tol;
  ctl.tpm = TPM_DEF;
  ctl.grow_step = GROW_DEF;
  ctl.esc_every = ESC_DEF;
  ctl.order = dorder;
  ctl.qB = qB;
  ctl.readyB = readyB;
  ctl.bars = bars;
  ctl.grow = grow;
  ctl.ls = ls;
  {
    // a team barrier waits at most 30 s (members step together; a healthy wait is
    // one pass of one iteration)
    int dev = 0, khz = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) khz = 100000;
    ctl.timeout_ticks = (int64_t)khz * 1000 * 30;
  }
  e = hipMemcpyAsync(dorder, order.data(), sizeof(int32_t) * count, hipMemcpyHostToDevice, b->st);
  if (e == hipSuccess) e = hipMemcpyAsync(b->dctl, &ctl, sizeof(ctl), hipMemcpyHostToDevice, b->st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->dprobs, b->hprobs.data(), sizeof(BatchProblem) * count, hipMemcpyHostToDevice, b->st);
  if (e == hipSuccess) e = hipStreamSynchronize(b->st);
  if (e != hipSuccess) { b->err = std::string("upload: ") + hipGetErrorString(e); return GSI_EDEVICE; }
  // persistent grid: enough workgroups to fill the device, never more than the problems
  const int lds = batched_lds();
  const void* kern = reinterpret_cast<const void*>(k_batched);
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
      k_batched_reset<<<std::max(1, std::min(1024, b->count * (TMAX - 1) / 256 + 1)), 256, 0, b->st>>>(b->dctl);
      k_batched<<<b->grid, WG, batched_lds(), b->st>>>(b->dprobs, b->dctl);
      e = hipStreamEndCapture(b->st, &b->graph);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) { b->err = std::string("graph: ") + hipGetErrorString(e); return GSI_EDEVICE; }
  }
  e = hipGraphLaunch(b->gexec, b->st);
  if (e == hipSuccess) e = hipStreamSynchronize(b->st);
  if (e != hipSuccess) { b->err = std::string("solve: ") + hipGetErrorString(e); return GSI_EDEVICE; }
  std::vector<BatchProblem> res;
  gsi_status s = fetch(b, res);
  if (s != GSI_OK) return s;
  for (int i = 0; i < b->count; ++i) {
    if (iters) iters[i] = res[i].iters;
    if (status) status[i] = res[i].status;
    if (res[i].status == 2 && s == GSI_OK) s = GSI_NOT_CONVERGED;
    if (res[i].status == 3 && s != GSI_EDEVICE) s = GSI_BREAKDOWN;
    if (res[i].status == 5 || res[i].status < 0) {
      s = GSI_EDEVICE;
      b->err = "problem " + std::to_string(i) + ": team wait timed out or the launch was aborted";
    }
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
  launch_unpack<double>(b->st, pr.n, pr.p, pr.PP, (const double*)pr.blk[1][0], X_out);
  hipError_t e = hipStreamSynchronize(b->st);
  if (e != hipSuccess) { b->err = std::string("get_x: ") + hipGetErrorString(e); return GSI_EDEVICE; }
  return GSI_OK;
}

gsi_status gsi_batched_set_tuning(gsi_batch_handle b, int32_t tiles_per_member, int32_t recruit_step,
                                  int32_t check_every) {
  if (!b || tiles_per_member < TPM_MIN || recruit_step < 1 || recruit_step > TMAX - 1 || check_every < 1) {
    if (b) b->err = "tuning: tiles_per_member >= 4, 1 <= recruit_step <= 15, check_every >= 1";
    return GSI_EINVAL;
  }
  BatchCtl ctl;
  hipError_t e = hipMemcpy(&ctl, b->dctl, sizeof(ctl), hipMemcpyDeviceToHost);
  ctl.tpm = tiles_per_member;
  ctl.grow_step = recruit_step;
  ctl.esc_every = check_every;
  if (e == hipSuccess) e = hipMemcpy(b->dctl, &ctl, sizeof(ctl), hipMemcpyHostToDevice);
  if (e != hipSuccess) { b->err = std::string("tuning: ") + hipGetErrorString(e); return GSI_EDEVICE; }
  return GSI_OK;
}

gsi_status gsi_batched_set_shapes(gsi_batch_handle b, const int32_t* shapes) {
  if (!b) return GSI_EINVAL;
  if (!shapes) { b->err = "shapes: null array"; return GSI_EINVAL; }
  for (int i = 0; i < b->count; ++i) {
    const int32_t c = shapes[i];
    const int u = c & 15, uu = (c >> 4) & 15, ug = (c >> 8) & 15, ch = (c >> 12) & 15;
    const bool ok = (c >> 16) == 0 && (u == 0 || u == 1 || u == 2 || u == 4) && (uu == 0 || uu == 1 || uu == 2) &&
                    (ug == 0 || ug == 1 || ug == 2 || ug == 4) && (ch == 0 || ch == 4 || ch == 8);
    // ch is a 4-bit field: 16 nonzeros per batch are coded as 0xf
    const bool ok16 = (c >> 16) == 0 && ch == 15;
    if (!ok && !(ok16 && (u == 0 || u == 1 || u == 2 || u == 4) && (uu == 0 || uu == 1 || uu == 2) &&
                 (ug == 0 || ug == 1 || ug == 2 || ug == 4))) {
      b->err = "shapes: problem " + std::to_string(i) + " has an unknown shape code";
      return GSI_EINVAL;
    }
  }
  std::vector<BatchProblem> cur(b->count);
  hipError_t e = hipMemcpy(cur.data(), b->dprobs, sizeof(BatchProblem) * b->count, hipMemcpyDeviceToHost);
  for (int i = 0; i < b->count; ++i) {
    cur[i].shape = shapes[i];
    b->hprobs[i].shape = shapes[i];
  }
  if (e == hipSuccess) e = hipMemcpy(b->dprobs, cur.data(), sizeof(BatchProblem) * b->count, hipMemcpyHostToDevice);
  if (e != hipSuccess) { b->err = std::string("shapes: ") + hipGetErrorString(e); return GSI_EDEVICE; }
  return GSI_OK;
}

gsi_status gsi_batched_set_wait_limit(gsi_batch_handle b, double seconds) {
  if (!b || !(seconds > 0.0) || seconds > 3600.0) {
    if (b) b->err = "wait limit: 0 < seconds <= 3600";
    return GSI_EINVAL;
  }
  const double us = tick_us();
  if (!(us > 0.0)) { b->err = "wait limit: wall clock rate unavailable"; return GSI_EDEVICE; }
  BatchCtl ctl;
  hipError_t e = hipMemcpy(&ctl, b->dctl, sizeof(ctl), hipMemcpyDeviceToHost);
  ctl.timeout_ticks = (int64_t)(seconds * 1e6 / us) > 0 ? (int64_t)(seconds * 1e6 / us) : 1;
  if (e == hipSuccess) e = hipMemcpy(b->dctl, &ctl, sizeof(ctl), hipMemcpyHostToDevice);
  if (e != hipSuccess) { b->err = std::string("wait limit: ") + hipGetErrorString(e); return GSI_EDEVICE; }
  return GSI_OK;
}

gsi_status gsi_batched_timeline(gsi_batch_handle b, double* begin_us, double* switch_us, double* end_us,
                                int32_t* iters_low, int32_t* team) {
  if (!b) return GSI_EINVAL;
  std::vector<BatchProblem> res;
  gsi_status s = fetch(b, res);
  if (s != GSI_OK) return s;
  const double us = tick_us();
  if (us <= 0.0) { b->err = "timeline: wall clock rate unavailable"; return GSI_EDEVICE; }
  int64_t t0 = INT64_MAX;
  for (const BatchProblem& r : res) t0 = std::min(t0, r.t_begin);
  for (int i = 0; i < b->count; ++i) {
    if (begin_us) begin_us[i] = (double)(res[i].t_begin - t0) * us;
    if (switch_us) switch_us[i] = (double)(res[i].t_switch - t0) * us;
    if (end_us) end_us[i] = (double)(res[i].t_end - t0) * us;
    if (iters_low) iters_low[i] = res[i].iters_low;
    if (team) team[i] = res[i].team;
  }
  return GSI_OK;
}

gsi_status gsi_batched_pass_times(gsi_batch_handle b, double* us) {
  if (!b || !us) return GSI_EINVAL;
  std::vector<BatchProblem> res;
  gsi_status s = fetch(b, res);
  if (s != GSI_OK) return s;
  const double t = tick_us();
  if (t <= 0.0) { b->err = "pass times: wall clock rate unavailable"; return GSI_EDEVICE; }
  for (int i = 0; i < b->count; ++i)
    for (int q = 0; q < GSI_NPASS; ++q) us[(int64_t)i * GSI_NPASS + q] = (double)res[i].ticks[q] * t;
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
