// Host driver and C ABI of libgsi (see include/gsi.h).
//
// One handle owns device copies of the operator (a CSR matrix or a stencil's diagonal) and
// X0, the tall blocks, the p x p small state and the scalars. An iteration is a fixed launch
// sequence (gradient pass, direction pass, eigendecomposition of P^T P on a second stream,
// SpMM, its Gram pass, line search, retraction, optional explicit A X); subspace iteration
// has its own sequence (si_iterate). Every kernel reads the control flags from device
// memory, so the sequence is identical for all iterations, needs no host round trip and is
// captured once in a HIP graph. The host only polls the convergence flag every check_every
// iterations.
#include <hip/hip_runtime.h>

#include <type_traits>
#include <cmath>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

#include "../../include/gsi.h"
#include "gsi_kernels.h"

using namespace gsi;

namespace {

constexpr int MAXP = 64;    // widest block of the SI, stencil and explicit-C paths
constexpr int MAXP_F64 = 128;  // widest block of RCG / RSD on a CSR matrix (float64 or mixed)

// Padded block width: the kernels are built for 16, 32 and 64 columns; the padding
// columns stay zero.
int padded_width(int p) { return p <= 16 ? 16 : (p <= 32 ? 32 : (p <= 64 ? 64 : 128)); }

// The seeded start block of gsi_create with X0 == NULL (the generator is stated in gsi.h):
// SplitMix64 as a counter-based generator (output k is the mixing function of
// seed + (k + 1) golden-ratio increments; Steele, Lea and Flood 2014) and the first
// Box-Muller normal of each pair of its outputs.
__device__ __forceinline__ uint64_t splitmix_out(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void k_seed_block(int64_t count, uint64_t seed, double* __restrict__ X) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
    const double u1 = ((double)(splitmix_out(seed, 2 * (uint64_t)e) >> 11) + 0.5) * 0x1.0p-53;
    const double u2 = ((double)(splitmix_out(seed, 2 * (uint64_t)e + 1) >> 11) + 0.5) * 0x1.0p-53;
    X[e] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925 * u2);
  }
}

struct Dev {
  std::vector<void*> ptrs;
  hipError_t err = hipSuccess;
  template <typename U>
  U* alloc(size_t count) {
    if (err != hipSuccess) return nullptr;
    void* p = nullptr;
    err = hipMalloc(&p, count * sizeof(U) + 256);
    if (err != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return reinterpret_cast<U*>(p);
  }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
};

// Tall blocks, matrix values and per-solve state for one block precision.
template <typename T>
struct Engine {
  int64_t n = 0;
  int p = 0, PP = 0, nb = 0;
  T *X = nullptr, *Y = nullptr, *G0 = nullptr, *G1 = nullptr, *P0 = nullptr, *P1 = nullptr, *Z = nullptr;
  T* vals = nullptr;
  uint16_t* vals16 = nullptr;  // bfloat16 values and bfloat16 copy of P (bfloat16 mode only)
  uint16_t* P16 = nullptr;
  // float64 engine of a mixed solve: float32 values and a float32 copy of P for the SpMM
  const float* vals32 = nullptr;
  float* P32 = nullptr;
  double* small = nullptr;
  Scalars* sc = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool explicit_grams = false;
  // the retraction pass also forms the next gradient (k_update_grad): the float64 engine of the
  // gradient-type methods with C and W carried by the recursion
  bool fused = false;

  bool alloc(Dev& d, int64_t n_, int p_, int nb_, int64_t nnz, bool bf16 = false) {
    n = n_; p = p_; PP = padded_width(p_); nb = nb_;
    // whole TR-row tiles; the rows past n stay zero (cleared once here, never written)
    const size_t blk = (size_t)((n + TR - 1) / TR * TR) * PP;
    X = d.alloc<T>(blk); Y = d.alloc<T>(blk); G0 = d.alloc<T>(blk); G1 = d.alloc<T>(blk);
    P0 = d.alloc<T>(blk); P1 = d.alloc<T>(blk); Z = d.alloc<T>(blk);
    vals = d.alloc<T>((size_t)nnz);
    if (bf16) {
      vals16 = d.alloc<uint16_t>((size_t)nnz);
      P16 = d.alloc<uint16_t>(blk);
    }
    small = d.alloc<double>(small_doubles(PP));
    sc = d.alloc<Scalars>(1);
    if (d.err != hipSuccess) return false;
    for (T* b : {X, Y, G0, G1, P0, P1, Z})
      if (hipMemset(b, 0, blk * sizeof(T)) != hipSuccess) return false;
    if (P16 && hipMemset(P16, 0, blk * sizeof(uint16_t)) != hipSuccess) return false;
    return true;
  }
  void destroy_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr; graph = nullptr;
  }
};

}  // namespace

struct gsi_ctx {
  gsi_options opt;
  hipStream_t st = nullptr;
  int64_t n = 0, nnz = 0;
  int p = 0, PP = 0, nb = 0;
  Dev dev;
  int32_t *rowptr = nullptr, *colind = nullptr;
  int nb_gram = 0;              // workgroups of the iteration's two-Gram pass
  double* partials = nullptr;  // max(nb, nb_gram) * (2 PP^2 + 8)
  double* red = nullptr;       // 2 PP^2 + 8
  double* hist = nullptr;      // (hist_cap) * H_FIELDS
  double* dvec = nullptr;      // device vector scratch (Ritz values etc.)
  int* flags = nullptr;
  int hist_cap = 0;
  double nA = 0.0;
  int64_t plane_tiles = 0;  // banded SpMM tile order (0: one slab per XCD)
  int spmm_batch = 8;       // gathers per batch of the CSR SpMM: 7 when no row holds more than 7
  // matrix-free stencil operator (gsi_create_stencil): grid, neighbour weight (times the
  // sign of which); the engines' vals hold the n diagonal entries
  // RCG or RCG(+) (A X by the recursion or formed every iteration): recompute_ax = -1 lets
  // the first iterations of each solve time both and keep the faster
  int rax = 0;
  bool rax_pending = false;
  double rax_ms[2] = {0.0, 0.0};
  int hermitian_p = 0;  // > 0: a Hermitian problem of this many complex columns, held as its real embedding
  bool stencil = false;
  int32_t sdims[3] = {1, 1, 1};
  double sdiag = 0.0, soff = 0.0;
  Engine<double> e64;
  Engine<float> e32;
  bool mixed = false;
  bool bf16 = false;      // mixed phase with bfloat16 SpMM values and inputs
  // subspace iteration (GSI_SI): outer iterations, products with A, rho history
  int si_k = 0, si_spmm = 0, si_done = 0;
  std::vector<double> si_rho;
  int phase = 0;          // 0: float64 engine active; 1: float32 engine active (mixed mode)
  int low_iters = 0;      // accepted iterations of the float32 phase
  int low_spmm = 0, low_restarts = 0, low_refresh = 0, low_null = 0, low_sweeps = 0;
  int hist_off = 0;       // history offset of the float64 phase
  bool own_stream = false;
  hipStream_t st2 = nullptr;  // second stream: the eigendecomposition overlaps the SpMM
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // optional per-pass event timing (gsi_pass_times)
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
  size_t ev_next = 0;
  double pass_ms[GSI_NPASS] = {0};
  int32_t pass_count[GSI_NPASS] = {0};
  std::string err;
};

namespace {

// Symmetry check of a CSR matrix: for every stored a_ij, row j must store a_ji with the same
// value (binary search, column indices sorted within rows). Sets flag 16 otherwise.
__global__ void k_sym_check(int64_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                            const double* __restrict__ vals, int* __restrict__ flags) {
  int bad = 0;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    for (int32_t k = rowptr[r]; k < rowptr[r + 1]; ++k) {
      const int32_t c = colind[k];
      int32_t lo = rowptr[c], hi = rowptr[c + 1] - 1;
      bool found = false;
      while (lo <= hi) {
        const int32_t mid = lo + (hi - lo) / 2;
        const int32_t m = colind[mid];
        if (m == (int32_t)r) {
          found = vals[mid] == vals[k];
          break;
        }
        if (m < (int32_t)r) lo = mid + 1; else hi = mid - 1;
      }
      if (!found) bad = 1;
    }
  }
  if (bad) atomicOr(flags, 16);
}

gsi_status fail(gsi_ctx* h, gsi_status s, const std::string& msg) {
  if (h) h->err = msg;
  return s;
}

// Z = A_op W through the handle's operator: the CSR kernel or the matrix-free stencil.
template <typename T, int PP>
void spmm_op(gsi_ctx* h, Engine<T>& e, const T* W0, const T* W1, T* Z, int mode) {
  if (h->stencil)
    Kernels<T, PP>::spmm_stencil(h->st, e.n, h->sdims, e.vals, h->soff, W0, W1, Z, e.sc, mode, h->plane_tiles);
  else
    Kernels<T, PP>::spmm(h->st, e.n, h->rowptr, h->colind, e.vals, W0, W1, Z, e.sc, mode, h->plane_tiles,
                         h->spmm_batch);
}

gsi_status hip_check(gsi_ctx* h, hipError_t e, const char* what) {
  if (e == hipSuccess) return GSI_OK;
  return fail(h, GSI_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define GSI_TRY(expr)                       \
  do {                                      \
    gsi_status _s = (expr);                 \
    if (_s != GSI_OK) return _s;            \
  } while (0)

template <typename T, typename F>
void dispatch_pp(int PP, F&& f) {
  switch (PP) {
    case 16: f(std::integral_constant<int, 16>()); break;
    case 32: f(std::integral_constant<int, 32>()); break;
    case 64: f(std::integral_constant<int, 64>()); break;
    case 128: f(std::integral_constant<int, 128>()); break;  // p above 64: RCG / RSD on a CSR matrix
    default: break;
  }
}

// Event timing of one launch (only when the handle's timing mode is on).
struct PassTimer {
  gsi_ctx* h;
  int pass;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  hipEvent_t get() {
    if (h->ev_next >= h->ev_pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      h->ev_pool.push_back(e);
    }
    return h->ev_pool[h->ev_next++];
  }
  PassTimer(gsi_ctx* h_, int pass_, hipStream_t st_ = nullptr) : h(h_), pass(pass_), st(st_ ? st_ : h_->st) {
    if (!h->timing) return;
    a = get();
    b = get();
    if (a && b) (void)hipEventRecord(a, st);
  }
  ~PassTimer() {
    if (!h->timing || !a || !b) return;
    (void)hipEventRecord(b, st);
    h->ev_pending.push_back({pass, {a, b}});
  }
};

// Fold completed event pairs into the per-pass totals (the stream has been synchronized).
void collect_times(gsi_ctx* h) {
  for (auto& pe : h->ev_pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pe.second.first, pe.second.second) == hipSuccess) {
      h->pass_ms[pe.first] += ms;
      h->pass_count[pe.first] += 1;
    }
  }
  h->ev_pending.clear();
  h->ev_next = 0;
}

// reduce partials of nv values (sum below max_from, max above)
void reduce(gsi_ctx* h, int nb, int64_t nv, int64_t max_from, const Scalars* sc, int cond) {
  PassTimer t(h, GSI_PASS_REDUCE);
  launch_reduce(h->st, h->partials, nb, nv, max_from, h->red, sc, cond);
}

// Orthonormalize the engine's X in place by two passes of Cholesky QR.
template <typename T>
gsi_status cholqr2(gsi_ctx* h, Engine<T>& e) {
  for (int pass = 0; pass < 2; ++pass) {
    dispatch_pp<T>(e.PP, [&](auto PPc) {
      constexpr int PP = decltype(PPc)::value;
      Kernels<T, PP>::gram(h->st, e.nb, e.n, e.X, e.X, e.X, nullptr, e.sc, 0, h->partials);
      reduce(h, e.nb, (int64_t)PP * PP, (int64_t)PP * PP, e.sc, 0);
      Small::chol_inv(h->st, PP, e.p, h->red, e.small, h->flags);
      Kernels<T, PP>::product(h->st, e.nb, e.n, e.X, e.X, e.small + S_M * PP * PP);
    });
  }
  int flag = 0;
  GSI_TRY(hip_check(h, hipMemcpyAsync(&flag, h->flags, sizeof(int), hipMemcpyDeviceToHost, h->st), "copy flag"));
  GSI_TRY(hip_check(h, hipStreamSynchronize(h->st), "cholqr2"));
  if (flag) {
    (void)hipMemsetAsync(h->flags, 0, sizeof(int), h->st);
    return fail(h, GSI_BREAKDOWN, "Cholesky QR: the block is rank deficient or not finite");
  }
  return GSI_OK;
}

// Y = A X explicitly with C = sym(X^T Y); reset the iteration state. `cont` (nullable)
// carries the counter, Polak-Ribiere denominator and history length of an earlier phase.
template <typename T>
gsi_status init_state(gsi_ctx* h, Engine<T>& e, double tol, int max_iter, int hist_off,
                      const Scalars* cont = nullptr, int stall_window = 0) {
  Scalars s;
  memset(&s, 0, sizeof(s));
  s.stall_window = stall_window;
  if (cont) {
    s.k = cont->k;
    s.gg_old = cont->gg_old;
    s.hist_len = cont->hist_len;
    s.ginf0 = cont->ginf0;
    s.restart_next = cont->restart_next;
    // the stall window of a continued solve counts from here
    s.k_best = cont->k;
    s.rho_best = 1e300;
  }
  s.nA = h->nA;
  s.tol = tol;
  s.sqrt_p = sqrt((double)e.p);
  s.max_iter = max_iter;
  s.k_restart = h->opt.k_restart;
  s.method = h->opt.method;
  s.p = e.p;
  s.hist_cap = h->hist_cap - hist_off;
  GSI_TRY(hip_check(h, hipMemcpyAsync(e.sc, &s, sizeof(s), hipMemcpyHostToDevice, h->st), "state upload"));
  GSI_TRY(hip_check(h, hipMemsetAsync(e.small, 0, sizeof(double) * small_doubles(e.PP), h->st),
                    "small reset"));
  dispatch_pp<T>(e.PP, [&](auto PPc) {
    constexpr int PP = decltype(PPc)::value;
    spmm_op<T, PP>(h, e, e.X, e.X, e.Y, 0);
    Kernels<T, PP>::gram(h->st, e.nb, e.n, e.X, e.X, e.Y, nullptr, e.sc, 0, h->partials);
    reduce(h, e.nb, (int64_t)PP * PP, (int64_t)PP * PP, e.sc, 0);
    launch_set_sym(h->st, PP, h->red, e.small + S_C * PP * PP);
  });
  return hip_check(h, hipGetLastError(), "init_state launch");
}

// One iteration's launch sequence. Unfused: gradient pass and its bookkeeping, direction
// pass, eigendecomposition of P^T P (second stream) beside the SpMM and its Gram pass, line
// search, retraction, explicit A X when asked for. Fused (e.fused): the gradient pass at the
// top runs only when the gradient is not current (the first iteration, after an explicit A X, a
// void step or a host-side change of the state); the retraction pass forms the next gradient
// and its partial sums, whose bookkeeping runs at the end of the iteration.
template <typename T>
void launch_iteration(gsi_ctx* h, Engine<T>& e, double* hist) {
  const int recompute = h->rax;
  const bool fused = e.fused;
  const int gcond = fused ? GRAD_PENDING : GRAD_ALWAYS;
  dispatch_pp<T>(e.PP, [&](auto PPc) {
    constexpr int PP = decltype(PPc)::value;
    const int64_t P2 = (int64_t)PP * PP;
    {
      PassTimer t(h, GSI_PASS_GRAD);
      Kernels<T, PP>::grad(h->st, e.nb, e.n, e.X, e.Y, e.G0, e.G1, e.small, e.sc, h->partials, gcond);
    }
    reduce(h, e.nb, P2 + 3, P2 + 2, e.sc, fused ? GRAD_PENDING : 3);
    {
      PassTimer t(h, GSI_PASS_SMALL);
      Small::after_grad(h->st, PP, h->red, e.small, e.sc, hist, gcond);
    }
    {
      PassTimer t(h, GSI_PASS_DIR);
      Kernels<T, PP>::dir(h->st, e.nb, e.n, e.X, e.G0, e.G1, e.P0, e.P1, e.small, e.sc, h->partials, e.P16, e.P32);
    }
    reduce(h, e.nb, P2 + 1, P2 + 1, e.sc, 1);
    {
      PassTimer t(h, GSI_PASS_SMALL);
      Small::after_dir(h->st, PP, h->red, e.small, e.sc);
    }
    // the eigendecomposition of P^T P needs only S: run it on the second stream while the
    // SpMM and its Gram pass run on the first
    // (in timing mode it runs alone on the first stream, so that its duration is its own)
    hipStream_t est = h->timing ? h->st : h->st2;
    if (!h->timing) {
      (void)hipEventRecord(h->ev_fork, h->st);
      (void)hipStreamWaitEvent(h->st2, h->ev_fork, 0);
    }
    {
      PassTimer t(h, GSI_PASS_EIG, est);
      Small::eig(est, PP, e.small, e.sc);
    }
    if (!h->timing) (void)hipEventRecord(h->ev_join, h->st2);
    {
      PassTimer t(h, GSI_PASS_SPMM);
      if constexpr (std::is_same<T, float>::value) {
        if (e.P16)
          Kernels<T, PP>::spmm16(h->st, e.n, h->rowptr, h->colind, e.vals16, e.P16, e.Z, e.sc, 1, h->plane_tiles,
                                 h->spmm_batch);
        else
          spmm_op<T, PP>(h, e, e.P0, e.P1, e.Z, 1);
      } else {
        if (e.P32)
          Kernels<T, PP>::spmm_fin(h->st, e.n, h->rowptr, h->colind, e.vals32, e.P32, e.Z, e.sc, 1, h->plane_tiles,
                                   h->spmm_batch);
        else
          spmm_op<T, PP>(h, e, e.P0, e.P1, e.Z, 1);
      }
    }
    {
      PassTimer t(h, GSI_PASS_GRAM);
      Kernels<T, PP>::gram(h->st, h->nb_gram, e.n, e.P0, e.P1, e.Z, e.Y, e.sc, 1, h->partials);
    }
    reduce(h, h->nb_gram, 2 * P2, 2 * P2, e.sc, 1);
    if (!h->timing) (void)hipStreamWaitEvent(h->st, h->ev_join, 0);
    {
      PassTimer t(h, GSI_PASS_LINESEARCH);
      Small::linesearch(h->st, PP, h->red, e.small, e.sc, hist, recompute, fused);
    }
    {
      PassTimer t(h, GSI_PASS_UPDATE);
      if (fused)
        Kernels<T, PP>::update_grad(h->st, e.nb, e.n, e.X, e.Y, e.P0, e.P1, e.Z, e.G0, e.G1, e.small, e.sc,
                                    h->partials);
      else
        Kernels<T, PP>::update(h->st, e.nb, e.n, e.X, e.Y, e.P0, e.P1, e.Z, e.small, e.sc, h->partials,
                               e.explicit_grams);
    }
    if (fused) {
      // the new gradient's bookkeeping, when the retraction formed it (the partials of the
      // explicit A X below go to other entries of the reduced vector: red is reused only
      // after this reduction has been consumed)
      reduce(h, e.nb, P2 + 3, P2 + 2, e.sc, GRAD_AFTER_FUSED);
      PassTimer t(h, GSI_PASS_SMALL);
      Small::after_grad(h->st, PP, h->red, e.small, e.sc, hist, GRAD_AFTER_FUSED);
    }
    if (e.explicit_grams) {
      reduce(h, e.nb, 2 * P2, 2 * P2, e.sc, 1);
      PassTimer t(h, GSI_PASS_SMALL);
      Small::after_update_grams(h->st, PP, h->red, e.small, e.sc);
    }
    {
      PassTimer t(h, GSI_PASS_REFRESH);
      spmm_op<T, PP>(h, e, e.X, e.X, e.Y, 2);
      Kernels<T, PP>::gram(h->st, e.nb, e.n, e.X, e.X, e.Y, nullptr, e.sc, 2, h->partials);
    }
    reduce(h, e.nb, P2, P2, e.sc, 2);
    {
      PassTimer t(h, GSI_PASS_SMALL);
      Small::after_refresh(h->st, PP, h->red, e.small, e.sc);
    }
  });
}

template <typename T>
gsi_status enqueue_iterations(gsi_ctx* h, Engine<T>& e, double* hist, int count) {
  if (h->opt.use_graph && !h->timing) {
    if (!e.gexec) {
      GSI_TRY(hip_check(h, hipStreamBeginCapture(h->st, hipStreamCaptureModeThreadLocal), "begin capture"));
      launch_iteration(h, e, hist);
      hipError_t ce = hipStreamEndCapture(h->st, &e.graph);
      GSI_TRY(hip_check(h, ce, "end capture"));
      GSI_TRY(hip_check(h, hipGraphInstantiate(&e.gexec, e.graph, nullptr, nullptr, 0), "graph instantiate"));
    }
    for (int i = 0; i < count; ++i)
      GSI_TRY(hip_check(h, hipGraphLaunch(e.gexec, h->st), "graph launch"));
  } else {
    for (int i = 0; i < count; ++i) launch_iteration(h, e, hist);
  }
  return hip_check(h, hipGetLastError(), "iteration launch");
}

// One Cholesky QR pass on X between iterations: X <- X R^{-1}, Y <- Y R^{-1} (Y = A X keeps
// holding), C <- R^{-T} C R^{-1}, W <- R^{-T} W. Used in the float32 phase, where the
// rounding of the retraction lets X^T X - I grow like sqrt(k) eps_32 and would floor the
// attainable residual.
template <typename T>
void reorthonormalize(gsi_ctx* h, Engine<T>& e) {
  dispatch_pp<T>(e.PP, [&](auto PPc) {
    constexpr int PP = decltype(PPc)::value;
    Kernels<T, PP>::gram(h->st, e.nb, e.n, e.X, e.X, e.X, nullptr, e.sc, 0, h->partials);
    reduce(h, e.nb, (int64_t)PP * PP, (int64_t)PP * PP, e.sc, 0);
    Small::chol_inv(h->st, PP, e.p, h->red, e.small, h->flags + 2);
    Small::transform_cw(h->st, PP, e.small, h->flags + 2);
    Kernels<T, PP>::product(h->st, e.nb, e.n, e.X, e.X, e.small + S_M * PP * PP);
    Kernels<T, PP>::product(h->st, e.nb, e.n, e.Y, e.Y, e.small + S_M * PP * PP);
  });
}

// Automatic choice between the A X recursion and RCG(+): one iteration to warm up, then
// `trial` iterations of each variant timed with events on the solver's stream (launched
// directly, the same way for both); the faster is kept for the rest of the solve. All
// these iterations are iterations of the solve.
template <typename T>
gsi_status choose_recompute(gsi_ctx* h, Engine<T>& e, double* hist) {
  const int trial = 3;
  hipEvent_t ev[3];
  for (auto& x : ev)
    if (hipEventCreate(&x) != hipSuccess) return fail(h, GSI_EDEVICE, "event creation failed");
  e.destroy_graph();
  h->rax = 0;
  launch_iteration(h, e, hist);
  (void)hipEventRecord(ev[0], h->st);
  for (int i = 0; i < trial; ++i) launch_iteration(h, e, hist);
  (void)hipEventRecord(ev[1], h->st);
  h->rax = 1;
  for (int i = 0; i < trial; ++i) launch_iteration(h, e, hist);
  (void)hipEventRecord(ev[2], h->st);
  gsi_status s = hip_check(h, hipEventSynchronize(ev[2]), "recompute trial");
  float a = 0.f, b = 0.f;
  if (s == GSI_OK) {
    (void)hipEventElapsedTime(&a, ev[0], ev[1]);
    (void)hipEventElapsedTime(&b, ev[1], ev[2]);
    h->rax_ms[0] = a / trial;
    h->rax_ms[1] = b / trial;
    h->rax = b < a ? 1 : 0;
  }
  for (auto& x : ev) (void)hipEventDestroy(x);
  h->rax_pending = false;
  e.destroy_graph();
  return s;
}

template <typename T>
gsi_status run_until_done(gsi_ctx* h, Engine<T>& e, double* hist, Scalars* out, bool reorth = false,
                          bool verify = false) {
  if (h->rax_pending && !h->timing) GSI_TRY(choose_recompute(h, e, hist));
  // in timing mode poll every iteration so that no launch after convergence is timed
  const int every = h->timing ? 1 : (h->opt.check_every > 0 ? h->opt.check_every : 25);
  for (;;) {
    GSI_TRY(enqueue_iterations(h, e, hist, every));
    GSI_TRY(hip_check(h, hipMemcpyAsync(out, e.sc, sizeof(Scalars), hipMemcpyDeviceToHost, h->st), "poll"));
    GSI_TRY(hip_check(h, hipStreamSynchronize(h->st), "iterate"));
    if (h->timing) collect_times(h);
    if (out->done == 4 && e.P32) {
      // the float32 copies of A and P set the attainable residual of this phase (their
      // rounding enters the A X recursion and the line-search Grams): continue with the
      // float64 SpMM from an explicit A X and C, without a stall window
      e.P32 = nullptr;
      e.vals32 = nullptr;
      e.destroy_graph();
      dispatch_pp<T>(e.PP, [&](auto PPc) {
        constexpr int PP = decltype(PPc)::value;
        spmm_op<T, PP>(h, e, e.X, e.X, e.Y, 0);
        Kernels<T, PP>::gram(h->st, e.nb, e.n, e.X, e.X, e.Y, nullptr, e.sc, 0, h->partials);
        reduce(h, e.nb, (int64_t)PP * PP, (int64_t)PP * PP, e.sc, 0);
        launch_set_sym(h->st, PP, h->red, e.small + S_C * PP * PP);
      });
      out->done = 0;
      out->stall_window = 0;
      out->restart_next = 1;
      out->grad_ready = 0;  // the gradient of the new A X is formed at the top of the next iteration
      GSI_TRY(hip_check(h, hipMemcpyAsync(e.sc, out, sizeof(Scalars), hipMemcpyHostToDevice, h->st), "resume"));
      continue;
    }
    if (out->done == 1 && verify) {
      // the AX recursion used float32-input SpMMs: confirm with A X and C in float64 and
      // let the next gradient pass test rho again (once; max_iter or a breakdown end at once)
      verify = false;
      dispatch_pp<T>(e.PP, [&](auto PPc) {
        constexpr int PP = decltype(PPc)::value;
        spmm_op<T, PP>(h, e, e.X, e.X, e.Y, 0);
        Kernels<T, PP>::gram(h->st, e.nb, e.n, e.X, e.X, e.Y, nullptr, e.sc, 0, h->partials);
        reduce(h, e.nb, (int64_t)PP * PP, (int64_t)PP * PP, e.sc, 0);
        launch_set_sym(h->st, PP, h->red, e.small + S_C * PP * PP);
      });
      out->done = 0;
      out->grad_ready = 0;
      GSI_TRY(hip_check(h, hipMemcpyAsync(e.sc, out, sizeof(Scalars), hipMemcpyHostToDevice, h->st), "resume"));
      continue;
    }
    if (out->done) return GSI_OK;
    if (reorth) reorthonormalize(h, e);
  }
}

gsi_status read_scalars(gsi_ctx* h, const Scalars* dsc, Scalars* out) {
  GSI_TRY(hip_check(h, hipMemcpyAsync(out, dsc, sizeof(Scalars), hipMemcpyDeviceToHost, h->st), "scalars"));
  return hip_check(h, hipStreamSynchronize(h->st), "scalars sync");
}

// Switch a mixed-precision solve to the float64 phase: X64 <- X32, Cholesky QR in
// float64, explicit A X and C. When the float32 phase stopped at its tolerance, the
// conjugate-gradient recursion continues: iteration k is redone in float64 with the float32
// G_{k-1}, P_{k-1} as the previous gradient and direction (W = X^T P_{k-1} formed
// explicitly for the new X). After a float32 breakdown the float64 phase restarts with
// the projected gradient.
gsi_status switch_to_fp64(gsi_ctx* h) {
  Scalars s32;
  GSI_TRY(read_scalars(h, h->e32.sc, &s32));
  const int k = s32.k;
  h->low_iters = k;
  h->low_spmm = s32.n_spmm + 1;
  h->low_restarts = s32.n_restart;
  h->low_refresh = s32.n_refresh;
  h->low_null = s32.n_null;
  h->low_sweeps = s32.n_sweeps;
  const bool carry = (s32.done == 1 || s32.done == 4) && k >= 1 && !s32.restart_next && s32.gg_old > 0.0;
  const int64_t rows = (h->n + TR - 1) / TR * TR;
  launch_convert<float, double>(h->st, rows * h->PP, h->e32.X, h->e64.X, 1.0);
  GSI_TRY(cholqr2(h, h->e64));
  Scalars cont = s32;
  cont.restart_next = carry ? 0 : 1;
  if (cont.hist_len > k + 1) cont.hist_len = k + 1;
  h->hist_off = 0;
  // with the float32-input SpMM the float64 phase watches for a stall as well (a wide
  // window: plain float64 progress can be slow); a stall there drops to the float64 SpMM
  const int sw = h->opt.stall_window > 0 ? h->opt.stall_window : 60;
  GSI_TRY(init_state(h, h->e64, h->opt.tol, h->opt.max_iter, 0, &cont, h->stencil ? 0 : 16 * sw));
  if (carry) {
    const int po = (k - 1) & 1;
    Engine<float>& a = h->e32;
    Engine<double>& b = h->e64;
    launch_convert<float, double>(h->st, rows * h->PP, po ? a.G1 : a.G0, po ? b.G1 : b.G0, 1.0);
    launch_convert<float, double>(h->st, rows * h->PP, po ? a.P1 : a.P0, po ? b.P1 : b.P0, 1.0);
    const double* Pold = po ? b.P1 : b.P0;
    dispatch_pp<double>(b.PP, [&](auto PPc) {
      constexpr int PP = decltype(PPc)::value;
      Kernels<double, PP>::gram(h->st, b.nb, b.n, b.X, b.X, Pold, nullptr, b.sc, 0, h->partials);
      reduce(h, b.nb, (int64_t)PP * PP, (int64_t)PP * PP, b.sc, 0);
    });
    GSI_TRY(hip_check(h, hipMemcpyAsync(b.small + S_W * b.PP * b.PP, h->red, sizeof(double) * b.PP * b.PP,
                                        hipMemcpyDeviceToDevice, h->st),
                      "carry W"));
  }
  // the float64 phase's SpMM reads float32 copies of A and P (the float32 blocks are free now)
  if (!h->stencil) {
    h->e64.vals32 = h->e32.vals;
    h->e64.P32 = h->e32.Z;
  }
  h->e64.destroy_graph();
  h->phase = 0;
  return hip_check(h, hipStreamSynchronize(h->st), "switch");
}

// Two Cholesky QR passes on an arbitrary block of the float64 engine.
gsi_status cholqr2_buf(gsi_ctx* h, Engine<double>& e, double* B) {
  for (int pass = 0; pass < 2; ++pass) {
    dispatch_pp<double>(e.PP, [&](auto PPc) {
      constexpr int PP = decltype(PPc)::value;
      Kernels<double, PP>::gram(h->st, e.nb, e.n, B, B, B, nullptr, e.sc, 0, h->partials);
      reduce(h, e.nb, (int64_t)PP * PP, (int64_t)PP * PP, e.sc, 0);
      Small::chol_inv(h->st, PP, e.p, h->red, e.small, h->flags);
      Kernels<double, PP>::product(h->st, e.nb, e.n, B, B, e.small + S_M * PP * PP);
    });
  }
  int flag = 0;
  GSI_TRY(hip_check(h, hipMemcpyAsync(&flag, h->flags, sizeof(int), hipMemcpyDeviceToHost, h->st), "copy flag"));
  GSI_TRY(hip_check(h, hipStreamSynchronize(h->st), "cholqr2"));
  if (flag) {
    (void)hipMemsetAsync(h->flags, 0, sizeof(int), h->st);
    return fail(h, GSI_BREAKDOWN, "Cholesky QR of the filtered block: rank deficient or not finite");
  }
  return GSI_OK;
}

// Rayleigh-Ritz of (Q, AQ) into X = Q U, Y = (A Q) U with Ritz values in dvec, then the
// residual rho = ||Y - X diag(theta)||_F / (sqrt(p) ||A||_inf) (Algorithm 1 steps 2, 6-7).
gsi_status si_ritz(gsi_ctx* h, const double* Q, double* AQ, double* rho) {
  Engine<double>& e = h->e64;
  double* theta = h->dvec;
  dispatch_pp<double>(e.PP, [&](auto PPc) {
    constexpr int PP = decltype(PPc)::value;
    Kernels<double, PP>::gram(h->st, e.nb, e.n, Q, Q, AQ, nullptr, e.sc, 0, h->partials);
    reduce(h, e.nb, (int64_t)PP * PP, (int64_t)PP * PP, e.sc, 0);
    Small::ritz(h->st, PP, e.p, h->red, e.small, theta);
    Kernels<double, PP>::product(h->st, e.nb, e.n, Q, e.X, e.small + S_M * PP * PP);
    Kernels<double, PP>::product(h->st, e.nb, e.n, AQ, e.Y, e.small + S_M * PP * PP);
    Kernels<double, PP>::colres(h->st, e.nb, e.n, e.X, e.Y, theta, h->partials);
    reduce(h, e.nb, PP, PP, e.sc, 0);
  });
  std::vector<double> cr(h->PP);
  GSI_TRY(hip_check(h, hipMemcpyAsync(cr.data(), h->red, sizeof(double) * h->PP, hipMemcpyDeviceToHost, h->st),
                    "si residual"));
  GSI_TRY(hip_check(h, hipStreamSynchronize(h->st), "si ritz"));
  double sq = 0.0;
  for (int i = 0; i < h->p; ++i) sq += cr[i];
  *rho = sqrt(sq > 0.0 ? sq : 0.0) / (sqrt((double)h->p) * h->nA);
  return GSI_OK;
}

// Up to `count` outer iterations of subspace iteration with a polynomial filter (Algorithm 1)
// from the current X (orthonormal), Y = A X. The Chebyshev filter runs the three-term
// recurrence of C_d((t - c)/h) normalized at cheb_top (Zhou and Saad 2007) with each step
// fused into an SpMM; the first step reuses Y = A X.
gsi_status si_iterate(gsi_ctx* h, int count) {
  Engine<double>& e = h->e64;
  const int64_t rows = (h->n + TR - 1) / TR * TR;
  const int64_t nel = rows * h->PP;
  const int d = h->opt.cheb_degree;
  if (h->si_rho.empty()) {
    // Rayleigh-Ritz of the start block: rho_0 (A X formed when the handle was started)
    double r0;
    GSI_TRY(hip_check(h, hipMemcpyAsync(e.G0, e.X, nel * sizeof(double), hipMemcpyDeviceToDevice, h->st), "si"));
    GSI_TRY(hip_check(h, hipMemcpyAsync(e.Z, e.Y, nel * sizeof(double), hipMemcpyDeviceToDevice, h->st), "si"));
    GSI_TRY(si_ritz(h, e.G0, e.Z, &r0));
    h->si_rho.push_back(r0);
    h->si_spmm = 1;
    if (r0 <= h->opt.tol) h->si_done = 1;
  }
  for (int it = 0; it < count && !h->si_done; ++it) {
    if (h->si_k >= h->opt.max_iter) {
      h->si_done = 2;
      break;
    }
    double* Xh = e.G0;
    if (d <= 0) {
      GSI_TRY(hip_check(h, hipMemcpyAsync(Xh, e.Y, nel * sizeof(double), hipMemcpyDeviceToDevice, h->st), "si"));
    } else {
      const double c = 0.5 * (h->opt.cheb_lo + h->opt.cheb_hi), hw = 0.5 * (h->opt.cheb_hi - h->opt.cheb_lo);
      const double sigma1 = hw / (h->opt.cheb_top - c);
      double sigma = sigma1;
      // three rotating blocks; the first step reads X and Y = A X
      double* pool[3] = {e.G0, e.G1, e.P0};
      double* prev = e.X;
      double* cur = e.G0;
      launch_axpby<double>(h->st, nel, e.Y, e.X, cur, sigma1 / hw, -c * sigma1 / hw);
      for (int j = 2; j <= d; ++j) {
        const double sigma_new = 1.0 / (2.0 / sigma1 - sigma);
        double* nxt = pool[0];
        for (double* b : pool)
          if (b != cur && b != prev) { nxt = b; break; }
        const double a = 2.0 * sigma_new / hw;
        dispatch_pp<double>(e.PP, [&](auto PPc) {
          constexpr int PP = decltype(PPc)::value;
          if (h->stencil)
            Kernels<double, PP>::spmm_stencil_axpy(h->st, e.n, h->sdims, e.vals, h->soff, cur, prev, nxt, a,
                                                   -c * a, -sigma * sigma_new, h->plane_tiles);
          else
            Kernels<double, PP>::spmm_axpy(h->st, e.n, h->rowptr, h->colind, e.vals, cur, prev, nxt, a, -c * a,
                                           -sigma * sigma_new, h->plane_tiles, h->spmm_batch);
        });
        prev = cur;
        cur = nxt;
        sigma = sigma_new;
      }
      Xh = cur;
      h->si_spmm += d - 1;
    }
    GSI_TRY(cholqr2_buf(h, e, Xh));
    dispatch_pp<double>(e.PP, [&](auto PPc) {
      constexpr int PP = decltype(PPc)::value;
      spmm_op<double, PP>(h, e, Xh, Xh, e.Z, 0);
    });
    h->si_spmm += 1;
    double r;
    GSI_TRY(si_ritz(h, Xh, e.Z, &r));
    h->si_rho.push_back(r);
    ++h->si_k;
    if (!(r == r)) { h->si_done = 3; break; }
    if (r <= h->opt.tol) h->si_done = 1;
  }
  return GSI_OK;
}

gsi_status start(gsi_ctx* h, const double* X0) {
  // pack X0 into the active engine, orthonormalize, form A X and reset the state
  h->e64.destroy_graph();
  h->e32.destroy_graph();
  h->e64.vals32 = nullptr;
  h->e64.P32 = nullptr;
  h->si_k = h->si_spmm = h->si_done = 0;
  h->si_rho.clear();
  h->rax = h->opt.recompute_ax > 0 ? 1 : 0;
  h->rax_pending = h->opt.recompute_ax < 0;
  h->low_iters = h->low_spmm = h->low_restarts = h->low_refresh = h->low_null = h->low_sweeps = 0;
  h->hist_off = 0;
  if (h->mixed) {
    launch_pack<float>(h->st, h->n, h->p, h->PP, X0, h->e32.X, 1.0);
    GSI_TRY(cholqr2(h, h->e32));
    // the low-precision phase also ends when rho has not halved for stall_window iterations
    // (its rounding floor); the float64 phase then continues
    GSI_TRY(init_state(h, h->e32, h->opt.switch_tol > h->opt.tol ? h->opt.switch_tol : h->opt.tol,
                       h->opt.max_iter, 0, nullptr, h->opt.stall_window > 0 ? h->opt.stall_window : 60));
    h->phase = 1;
  } else {
    launch_pack<double>(h->st, h->n, h->p, h->PP, X0, h->e64.X, 1.0);
    GSI_TRY(cholqr2(h, h->e64));
    GSI_TRY(init_state(h, h->e64, h->opt.tol, h->opt.max_iter, 0));
    h->phase = 0;
  }
  return hip_check(h, hipStreamSynchronize(h->st), "start");
}

}  // namespace

extern "C" {

void gsi_options_default(gsi_options* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->p = 8;
  o->which = 1;
  o->method = GSI_RCG;
  o->precision = GSI_FP64;
  o->recompute_ax = 0;
  o->k_restart = 0;
  o->max_iter = 10000;
  o->tol = 1e-8;
  o->switch_tol = 1e-5;
  o->check_every = 25;
  o->use_graph = 1;
  o->stall_window = 60;
}

const char* gsi_status_str(gsi_status s) {
  switch (s) {
    case GSI_OK: return "ok";
    case GSI_EINVAL: return "invalid argument";
    case GSI_ENOMEM: return "out of device memory";
    case GSI_EDEVICE: return "device error";
    case GSI_NOT_CONVERGED: return "not converged";
    case GSI_BREAKDOWN: return "breakdown";
    case GSI_EUNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* gsi_last_error(gsi_handle h) { return h ? h->err.c_str() : "null handle"; }

}  // extern "C"

namespace {

// Shared by gsi_create (A != nullptr) and gsi_create_stencil (S != nullptr).
gsi_status create_impl(gsi_handle* out, const gsi_csr* A, const gsi_stencil* S, const gsi_options* opt,
                       const double* X0, void* stream) {
  if (!out || (!A && !S) || !opt) return GSI_EINVAL;
  *out = nullptr;
  gsi_ctx* h = new (std::nothrow) gsi_ctx();
  if (!h) return GSI_ENOMEM;
  h->opt = *opt;
  h->st = reinterpret_cast<hipStream_t>(stream);
  if (!h->st) {
    // graphs cannot be captured on the null stream: use an owned blocking stream, which
    // is ordered with the null stream
    const hipError_t se = hipStreamCreate(&h->st);
    if (se != hipSuccess) {
      h->st = nullptr;
      h->err = std::string("stream creation failed: ") + hipGetErrorString(se);
      *out = h;
      return GSI_EDEVICE;
    }
    h->own_stream = true;
  }
  {
    hipError_t se = hipStreamCreate(&h->st2);
    if (se == hipSuccess) se = hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming);
    if (se == hipSuccess) se = hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming);
    if (se != hipSuccess) {
      h->err = std::string("stream or event creation failed: ") + hipGetErrorString(se);
      *out = h;
      return GSI_EDEVICE;
    }
  }
  auto bail = [&](gsi_status s, const std::string& m) {
    // keep the handle so the caller can read the error text
    h->err = m;
    *out = h;
    return s;
  };
  int64_t n_op = 0;
  if (A) {
    if (A->n < 2 || A->nnz < 1 || !A->rowptr || !A->colind || !A->vals) return bail(GSI_EINVAL, "bad CSR arguments");
    if (A->n > (int64_t)INT32_MAX || A->nnz > (int64_t)INT32_MAX) return bail(GSI_EUNSUPPORTED, "n or nnz >= 2^31");
    n_op = A->n;
  } else {
    if (S->nx < 1 || S->ny < 1 || S->nz < 1 || !std::isfinite(S->diag) || !std::isfinite(S->off))
      return bail(GSI_EINVAL, "bad stencil arguments");
    if (S->nx > INT32_MAX || S->ny > INT32_MAX || S->nz > INT32_MAX ||
        (double)S->nx * (double)S->ny * (double)S->nz > (double)INT32_MAX)
      return bail(GSI_EUNSUPPORTED, "n >= 2^31");
    n_op = S->nx * S->ny * S->nz;
    if (n_op < 2) return bail(GSI_EINVAL, "bad stencil arguments");
    if (opt->precision == GSI_MIXED_BF16) return bail(GSI_EUNSUPPORTED, "bfloat16 mode needs a CSR matrix");
  }
  if (opt->p < 1 || opt->p >= n_op) return bail(GSI_EINVAL, "need 1 <= p < n");
  if (opt->p > MAXP_F64) return bail(GSI_EUNSUPPORTED, "p above 128 is not built");
  if (opt->p > MAXP && (S || opt->method == GSI_SI || opt->explicit_c))
    return bail(GSI_EUNSUPPORTED, "p above 64 is built for RCG / RSD on a CSR matrix without explicit_c");
  if (opt->which != 1 && opt->which != -1) return bail(GSI_EINVAL, "which must be +1 or -1");
  if (opt->method != GSI_RSD && opt->method != GSI_RCG && opt->method != GSI_SI)
    return bail(GSI_EINVAL, "unknown method");
  if (opt->method == GSI_SI && opt->precision != GSI_FP64)
    return bail(GSI_EUNSUPPORTED, "subspace iteration runs in float64 only");
  if (opt->method == GSI_SI && opt->cheb_degree > 0 &&
      !(opt->cheb_hi > opt->cheb_lo && opt->cheb_top > opt->cheb_hi))
    return bail(GSI_EINVAL, "Chebyshev filter needs cheb_lo < cheb_hi < cheb_top");
  if (opt->precision != GSI_FP64 && opt->precision != GSI_MIXED_FP32 && opt->precision != GSI_MIXED_BF16)
    return bail(GSI_EINVAL, "unknown precision");
  if (!(opt->tol >= 0.0) || opt->max_iter < 0) return bail(GSI_EINVAL, "bad tol or max_iter");
  h->n = n_op;
  h->nnz = A ? A->nnz : n_op;  // values held: the nonzeros, or the stencil's diagonal
  if (S) {
    h->stencil = true;
    h->sdims[0] = (int32_t)S->nx;
    h->sdims[1] = (int32_t)S->ny;
    h->sdims[2] = (int32_t)S->nz;
    h->sdiag = S->diag;
    h->soff = (opt->which > 0 ? 1.0 : -1.0) * S->off;
  }
  h->p = opt->p;
  h->PP = padded_width(opt->p);
  h->mixed = opt->precision == GSI_MIXED_FP32 || opt->precision == GSI_MIXED_BF16;
  h->bf16 = opt->precision == GSI_MIXED_BF16;
  const int64_t ntiles = (h->n + TR - 1) / TR;
  int dev = 0;
  hipDeviceProp_t prop;
  (void)hipGetDevice(&dev);
  int ncu = 256;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0) ncu = prop.multiProcessorCount;
  // two workgroups per CU for the streaming passes (the register-limited residency of the
  // float64 passes at p = 64): more workgroups did not move the passes and only enlarge the
  // per-workgroup partial sums the reductions read (measured at n = 128^3, p = 64)
  h->nb = (int)(ntiles < 2 * (int64_t)ncu ? ntiles : 2 * (int64_t)ncu);
  // the iteration's P^T A P / P^T A X pass on four workgroups per CU: alone it ran 835 -> 730 us
  // (128^3, p = 64); inside the solve the pass itself stays near 0.70 ms but the retraction pass
  // after it runs 1.78 -> 1.72 ms (solve 12.47 -> 12.34 s, two builds on one GPU, two solves each)
  h->nb_gram = (int)(ntiles < 4 * (int64_t)ncu ? ntiles : 4 * (int64_t)ncu);
  h->hist_cap = opt->max_iter + 2;
  Dev& d = h->dev;
  if (A) {
    h->rowptr = d.alloc<int32_t>(h->n + 1);
    h->colind = d.alloc<int32_t>(h->nnz);
  }
  h->partials = d.alloc<double>((size_t)(h->nb > h->nb_gram ? h->nb : h->nb_gram) * (2 * h->PP * h->PP + 8) + 4096);
  h->red = d.alloc<double>(2 * h->PP * h->PP + 8);
  h->hist = d.alloc<double>((size_t)h->hist_cap * H_FIELDS);
  h->dvec = d.alloc<double>(4 * MAXP_F64 + 4096);
  h->flags = d.alloc<int>(4);
  if (d.err != hipSuccess) { d.release(); return bail(GSI_ENOMEM, "device allocation failed"); }
  if (!h->e64.alloc(d, h->n, h->p, h->nb, h->nnz)) { d.release(); return bail(GSI_ENOMEM, "device allocation failed"); }
  if (h->mixed && !h->e32.alloc(d, h->n, h->p, h->nb, h->nnz, h->bf16)) {
    d.release();
    return bail(GSI_ENOMEM, "device allocation failed");
  }
  // kernel attributes
  hipError_t ke = Small::init();
  dispatch_pp<double>(h->PP, [&](auto PPc) {
    constexpr int PP = decltype(PPc)::value;
    if (ke == hipSuccess) ke = Kernels<double, PP>::init();
    if (ke == hipSuccess) ke = Kernels<float, PP>::init();
  });
  if (ke != hipSuccess) return bail(GSI_EDEVICE, std::string("kernel attributes: ") + hipGetErrorString(ke));
  hipStream_t st = h->st;
  gsi_status s = GSI_OK;
  if (A)
    s = hip_check(h, hipMemcpyAsync(h->rowptr, A->rowptr, sizeof(int32_t) * (h->n + 1), hipMemcpyDeviceToDevice, st),
                  "copy rowptr");
  if (s == GSI_OK && A)
    s = hip_check(h, hipMemcpyAsync(h->colind, A->colind, sizeof(int32_t) * h->nnz, hipMemcpyDeviceToDevice, st),
                  "copy colind");
  if (s == GSI_OK) s = hip_check(h, hipMemsetAsync(h->flags, 0, 4 * sizeof(int), st), "flags");
  if (s != GSI_OK) return bail(s, h->err);
  // validate the CSR and compute ||A||_inf
  const int cb = 256;
  if (A) {
    launch_csr_check(st, cb, h->n, h->nnz, A->rowptr, A->colind, A->vals, h->dvec, h->flags, h->dvec + cb);
  } else {
    launch_stencil_check(st, cb, h->n, h->sdims, S->diag, S->off, S->diag_vec, h->dvec, h->flags);
    (void)hipMemsetAsync(h->dvec + cb, 0, sizeof(double) * cb, st);
  }
  // X0 == NULL: the seeded start block, drawn into a buffer released after the start
  double* x0_drawn = nullptr;
  if (!X0) {
    if (hipMalloc(&x0_drawn, sizeof(double) * (size_t)h->n * h->p) != hipSuccess)
      return bail(GSI_ENOMEM, "out of device memory for the start block");
    hipLaunchKernelGGL(k_seed_block, dim3(2048), dim3(256), 0, st, h->n * (int64_t)h->p, (uint64_t)opt->x0_seed,
                       x0_drawn);
    X0 = x0_drawn;
  }
  struct FreeOnExit {
    double* p;
    hipStream_t s;
    ~FreeOnExit() {
      if (p) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(p);
      }
    }
  } x0_guard{x0_drawn, st};
  launch_finite(st, h->n * (int64_t)h->p, X0, h->flags + 1);
  std::vector<double> pm(2 * cb);
  int fl[2] = {0, 0};
  s = hip_check(h, hipMemcpyAsync(pm.data(), h->dvec, sizeof(double) * 2 * cb, hipMemcpyDeviceToHost, st), "norm");
  if (s == GSI_OK) s = hip_check(h, hipMemcpyAsync(fl, h->flags, 2 * sizeof(int), hipMemcpyDeviceToHost, st), "flags");
  if (s == GSI_OK) s = hip_check(h, hipStreamSynchronize(st), "validate");
  if (s != GSI_OK) return bail(s, h->err);
  if (fl[0] & 1) return bail(GSI_EINVAL, "rowptr is not monotone or out of range");
  if (fl[0] & 2) return bail(GSI_EINVAL, "column index out of range");
  if (fl[0] & 8) return bail(GSI_EINVAL, "column indices not sorted within a row");
  if (fl[0] & 4) return bail(GSI_BREAKDOWN, "non-finite matrix value");
  h->spmm_batch = (A && !(fl[0] & 32)) ? 7 : 8;
  if (fl[1]) return bail(GSI_BREAKDOWN, "non-finite value in X0");
  if (A && opt->check_symmetric) {
    // the structure is valid (checked above), so the searches stay inside the arrays
    hipLaunchKernelGGL(k_sym_check, dim3(1024), dim3(256), 0, st, h->n, A->rowptr, A->colind, A->vals, h->flags);
    int fs = 0;
    s = hip_check(h, hipMemcpyAsync(&fs, h->flags, sizeof(int), hipMemcpyDeviceToHost, st), "flags");
    if (s == GSI_OK) s = hip_check(h, hipStreamSynchronize(st), "symmetry check");
    if (s != GSI_OK) return bail(s, h->err);
    if (fs & 16) return bail(GSI_EINVAL, "matrix is not symmetric");
  }
  (void)hipMemsetAsync(h->flags, 0, 4 * sizeof(int), st);
  double nA = 0.0, band = 0.0;
  for (int i = 0; i < cb; ++i) {
    nA = pm[i] > nA ? pm[i] : nA;
    band = pm[cb + i] > band ? pm[cb + i] : band;
  }
  // band of a stencil: its farthest neighbour (a plane, a grid line or the next node)
  if (S) band = S->nz > 1 ? (double)(S->nx * S->ny) : (S->ny > 1 ? (double)S->nx : 1.0);
  if (!(nA > 0.0)) return bail(GSI_EINVAL, "zero matrix");
  h->nA = nA;
  // banded SpMM tile order when the rows reach at least 64 tiles away and the matrix spans
  // at least 4 such planes (3D grids); otherwise one contiguous slab per XCD
  {
    const int64_t pt = ((int64_t)band + TR - 1) / TR, ntiles = (h->n + TR - 1) / TR;
    h->plane_tiles = (pt >= 64 && 4 * pt <= ntiles) ? pt : 0;
  }
  const double sign = opt->which > 0 ? 1.0 : -1.0;
  if (A) {
    launch_convert<double, double>(st, h->nnz, A->vals, h->e64.vals, sign);
    if (h->mixed) launch_convert<double, float>(st, h->nnz, A->vals, h->e32.vals, sign);
    if (h->bf16) launch_to_bf16(st, h->nnz, A->vals, h->e32.vals16, sign);
  } else {
    launch_stencil_diag<double>(st, h->n, S->diag, S->diag_vec, sign, h->e64.vals);
    if (h->mixed) launch_stencil_diag<float>(st, h->n, S->diag, S->diag_vec, sign, h->e32.vals);
  }
  h->e64.explicit_grams = opt->explicit_c != 0;
  h->e32.explicit_grams = opt->explicit_c != 0;
  // the fused pass keeps M and M C in LDS: up to PP = 64
  h->e64.fused = !h->e64.explicit_grams && (opt->method == GSI_RCG || opt->method == GSI_RSD) && h->PP <= MAXP;
  s = start(h, X0);
  if (s != GSI_OK) return bail(s, h->err);
  *out = h;
  return GSI_OK;
}

}  // namespace

extern "C" {

gsi_status gsi_create(gsi_handle* out, const gsi_csr* A, const gsi_options* opt, const double* X0, void* stream) {
  if (!A) return GSI_EINVAL;
  return create_impl(out, A, nullptr, opt, X0, stream);
}

gsi_status gsi_create_stencil(gsi_handle* out, const gsi_stencil* S, const gsi_options* opt, const double* X0,
                              void* stream) {
  if (!S) return GSI_EINVAL;
  return create_impl(out, nullptr, S, opt, X0, stream);
}

gsi_status gsi_create_hermitian(gsi_handle* out, const gsi_zcsr* A, const gsi_options* opt, const double* X0,
                                void* stream) {
  if (!out || !A || !opt || !X0) return GSI_EINVAL;
  *out = nullptr;
  if (A->n < 1 || A->nnz < 1 || !A->rowptr || !A->colind || !A->vals) return GSI_EINVAL;
  if (opt->p < 1 || 2 * opt->p > MAXP) return GSI_EUNSUPPORTED;
  if (A->n >= (int64_t)INT32_MAX / 2 || 4 * A->nnz >= (int64_t)INT32_MAX) return GSI_EUNSUPPORTED;
  const int64_t n = A->n, nnz = A->nnz;
  const int p = opt->p;
  // the real embedding [[Re A, -Im A], [Im A, Re A]] and [[Re X0, -Im X0], [Im X0, Re X0]],
  // built on the host from copies of the device arrays (rows stay sorted: the left block's
  // columns precede the right block's; imaginary parts that are zero are not stored)
  std::vector<int32_t> rp(n + 1), ci(nnz);
  std::vector<double> va(2 * nnz), x0(2 * n * p);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (hipStreamSynchronize(st) != hipSuccess ||
      hipMemcpy(rp.data(), A->rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(ci.data(), A->colind, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(va.data(), A->vals, sizeof(double) * 2 * nnz, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(x0.data(), X0, sizeof(double) * 2 * n * p, hipMemcpyDeviceToHost) != hipSuccess)
    return GSI_EDEVICE;
  if (rp[0] != 0 || rp[n] != nnz) return GSI_EINVAL;
  for (int64_t r = 0; r < n; ++r)
    if (rp[r + 1] < rp[r]) return GSI_EINVAL;
  // a column index outside [0, n) would land in the other block of the embedding, where the
  // check of the embedded matrix cannot see it
  for (int64_t j = 0; j < nnz; ++j)
    if (ci[j] < 0 || ci[j] >= n) return GSI_EINVAL;
  std::vector<int32_t> erp(2 * n + 1), eci;
  std::vector<double> eva;
  eci.reserve(4 * nnz);
  eva.reserve(4 * nnz);
  erp[0] = 0;
  for (int half = 0; half < 2; ++half)
    for (int64_t r = 0; r < n; ++r) {
      // left block: Re A (top) / Im A (bottom); right block: -Im A (top) / Re A (bottom)
      for (int blk = 0; blk < 2; ++blk)
        for (int32_t j = rp[r]; j < rp[r + 1]; ++j) {
          const double re = va[2 * j], im = va[2 * j + 1];
          const double v = half == 0 ? (blk == 0 ? re : -im) : (blk == 0 ? im : re);
          const bool real_part = (half == 0) == (blk == 0);
          if (!real_part && v == 0.0) continue;
          eci.push_back((int32_t)(blk * n + ci[j]));
          eva.push_back(v);
        }
      erp[half * n + r + 1] = (int32_t)eci.size();
    }
  std::vector<double> ex((size_t)2 * n * 2 * p);
  for (int64_t r = 0; r < n; ++r)
    for (int j = 0; j < p; ++j) {
      const double re = x0[2 * (r * p + j)], im = x0[2 * (r * p + j) + 1];
      ex[r * 2 * p + j] = re;
      ex[r * 2 * p + p + j] = -im;
      ex[(n + r) * 2 * p + j] = im;
      ex[(n + r) * 2 * p + p + j] = re;
    }
  int32_t *drp = nullptr, *dci = nullptr;
  double *dva = nullptr, *dx = nullptr;
  gsi_status s = GSI_OK;
  if (hipMalloc(&drp, sizeof(int32_t) * erp.size()) != hipSuccess ||
      hipMalloc(&dci, sizeof(int32_t) * eci.size()) != hipSuccess ||
      hipMalloc(&dva, sizeof(double) * eva.size()) != hipSuccess ||
      hipMalloc(&dx, sizeof(double) * ex.size()) != hipSuccess)
    s = GSI_ENOMEM;
  if (s == GSI_OK &&
      (hipMemcpy(drp, erp.data(), sizeof(int32_t) * erp.size(), hipMemcpyHostToDevice) != hipSuccess ||
       hipMemcpy(dci, eci.data(), sizeof(int32_t) * eci.size(), hipMemcpyHostToDevice) != hipSuccess ||
       hipMemcpy(dva, eva.data(), sizeof(double) * eva.size(), hipMemcpyHostToDevice) != hipSuccess ||
       hipMemcpy(dx, ex.data(), sizeof(double) * ex.size(), hipMemcpyHostToDevice) != hipSuccess))
    s = GSI_EDEVICE;
  if (s == GSI_OK) {
    gsi_csr E;
    E.n = 2 * n;
    E.nnz = (int64_t)eci.size();
    E.rowptr = drp;
    E.colind = dci;
    E.vals = dva;
    gsi_options o2 = *opt;
    o2.p = 2 * p;
    s = create_impl(out, &E, nullptr, &o2, dx, stream);
    if (*out) {
      (*out)->hermitian_p = p;
      (void)hipStreamSynchronize((*out)->st);
    }
  }
  (void)hipDeviceSynchronize();
  for (void* q : {(void*)drp, (void*)dci, (void*)dva, (void*)dx})
    if (q) (void)hipFree(q);
  return s;
}

gsi_status gsi_hermitian_results(gsi_handle h, double* ritz, double* Xc, double* rho) {
  if (!h) return GSI_EINVAL;
  if (h->hermitian_p <= 0) return fail(h, GSI_EUNSUPPORTED, "not a Hermitian handle");
  const int pc = h->hermitian_p;
  std::vector<double> r2(2 * pc);
  GSI_TRY(gsi_residuals(h, r2.data(), nullptr, rho, nullptr));
  // every eigenvalue of the embedding appears twice; the Ritz pairs are adjacent
  if (ritz)
    for (int j = 0; j < pc; ++j) ritz[j] = r2[2 * j];
  if (Xc) {
    launch_complex_extract(h->st, h->n / 2, pc, h->PP, h->e64.X, Xc);
    GSI_TRY(hip_check(h, hipStreamSynchronize(h->st), "complex basis"));
  }
  return GSI_OK;
}

gsi_status gsi_step(gsi_handle h, int32_t n_iter) {
  if (!h || n_iter < 0) return GSI_EINVAL;
  if (h->opt.method == GSI_SI) return si_iterate(h, n_iter);
  if (h->phase == 1) return enqueue_iterations(h, h->e32, h->hist, n_iter);
  return enqueue_iterations(h, h->e64, h->hist + (size_t)h->hist_off * H_FIELDS, n_iter);
}

gsi_status gsi_solve(gsi_handle h, int32_t* iters_out) {
  if (!h) return GSI_EINVAL;
  if (h->opt.method == GSI_SI) {
    GSI_TRY(si_iterate(h, INT32_MAX));
    if (iters_out) *iters_out = h->si_k;
    if (h->si_done == 1) return GSI_OK;
    if (h->si_done == 2) return fail(h, GSI_NOT_CONVERGED, "max_iter reached");
    return fail(h, GSI_BREAKDOWN, "subspace iteration: non-finite residual");
  }
  Scalars s;
  if (h->phase == 1) {
    // a float32 breakdown means float32 resolution is exhausted: refine in float64
    GSI_TRY(run_until_done(h, h->e32, h->hist, &s, true));
    GSI_TRY(switch_to_fp64(h));
  }
  GSI_TRY(run_until_done(h, h->e64, h->hist + (size_t)h->hist_off * H_FIELDS, &s, false, h->e64.P32 != nullptr));
  if (iters_out) *iters_out = s.k;
  if (s.done == 1) return GSI_OK;
  if (s.done == 2) return fail(h, GSI_NOT_CONVERGED, "max_iter reached");
  return fail(h, GSI_BREAKDOWN, "breakdown: non-finite values or no descent step");
}

gsi_status gsi_residuals(gsi_handle h, double* ritz, double* col_res, double* rho, double* phi) {
  if (!h) return GSI_EINVAL;
  if (h->phase == 1) GSI_TRY(switch_to_fp64(h));
  Engine<double>& e = h->e64;
  const int p = h->p;
  double* theta = h->dvec;
  dispatch_pp<double>(e.PP, [&](auto PPc) {
    constexpr int PP = decltype(PPc)::value;
    spmm_op<double, PP>(h, e, e.X, e.X, e.Y, 0);
    Kernels<double, PP>::gram(h->st, e.nb, e.n, e.X, e.X, e.Y, nullptr, e.sc, 0, h->partials);
    reduce(h, e.nb, (int64_t)PP * PP, (int64_t)PP * PP, e.sc, 0);
    Small::ritz(h->st, PP, p, h->red, e.small, theta);
    Kernels<double, PP>::product(h->st, e.nb, e.n, e.X, e.X, e.small + S_M * PP * PP);
    Kernels<double, PP>::product(h->st, e.nb, e.n, e.Y, e.Y, e.small + S_M * PP * PP);
    Kernels<double, PP>::colres(h->st, e.nb, e.n, e.X, e.Y, theta, h->partials);
    reduce(h, e.nb, PP, PP, e.sc, 0);
  });
  std::vector<double> th(p), cr(h->PP);
  GSI_TRY(hip_check(h, hipMemcpyAsync(th.data(), theta, sizeof(double) * p, hipMemcpyDeviceToHost, h->st), "ritz"));
  GSI_TRY(hip_check(h, hipMemcpyAsync(cr.data(), h->red, sizeof(double) * h->PP, hipMemcpyDeviceToHost, h->st),
                    "colres"));
  GSI_TRY(hip_check(h, hipStreamSynchronize(h->st), "residuals"));
  // restart the iteration from the rotated basis
  e.destroy_graph();
  {
    Scalars s;
    GSI_TRY(read_scalars(h, e.sc, &s));
    int done = 0, one = 1;
    GSI_TRY(hip_check(h, hipMemcpyAsync(&e.sc->done, &done, sizeof(int), hipMemcpyHostToDevice, h->st), "reset"));
    GSI_TRY(hip_check(h, hipMemcpyAsync(&e.sc->restart_next, &one, sizeof(int), hipMemcpyHostToDevice, h->st),
                      "reset"));
    // the rotated basis has its own gradient, formed at the top of the next iteration
    GSI_TRY(hip_check(h, hipMemcpyAsync(&e.sc->grad_ready, &done, sizeof(int), hipMemcpyHostToDevice, h->st),
                      "reset"));
    dispatch_pp<double>(e.PP, [&](auto PPc) {
      constexpr int PP = decltype(PPc)::value;
      Kernels<double, PP>::gram(h->st, e.nb, e.n, e.X, e.X, e.Y, nullptr, e.sc, 0, h->partials);
      reduce(h, e.nb, (int64_t)PP * PP, (int64_t)PP * PP, e.sc, 0);
      launch_set_sym(h->st, PP, h->red, e.small + S_C * PP * PP);
    });
    GSI_TRY(hip_check(h, hipStreamSynchronize(h->st), "restart"));
  }
  double sq = 0.0, ph = 0.0;
  const double sign = h->opt.which > 0 ? 1.0 : -1.0;
  for (int i = 0; i < p; ++i) {
    sq += cr[i];
    ph += th[i];
    if (ritz) ritz[i] = sign * th[i];
    if (col_res) col_res[i] = sqrt(cr[i] > 0.0 ? cr[i] : 0.0);
  }
  if (rho) *rho = sqrt(sq) / (sqrt((double)p) * h->nA);
  if (phi) *phi = -0.5 * ph;
  return GSI_OK;
}

gsi_status gsi_get_x(gsi_handle h, double* X_out) {
  if (!h || !X_out) return GSI_EINVAL;
  if (h->phase == 1)
    launch_unpack<float>(h->st, h->n, h->p, h->PP, h->e32.X, X_out);
  else
    launch_unpack<double>(h->st, h->n, h->p, h->PP, h->e64.X, X_out);
  return hip_check(h, hipStreamSynchronize(h->st), "get_x");
}

gsi_status gsi_set_x0(gsi_handle h, const double* X0) {
  if (!h || !X0) return GSI_EINVAL;
  return start(h, X0);
}

gsi_status gsi_set_values(gsi_handle h, const double* vals) {
  if (!h || !vals) return GSI_EINVAL;
  hipStream_t st = h->st;
  const int cb = 256;
  GSI_TRY(hip_check(h, hipMemsetAsync(h->flags, 0, 4 * sizeof(int), st), "flags"));
  if (h->stencil)
    launch_stencil_check(st, cb, h->n, h->sdims, h->sdiag, h->soff, vals, h->dvec, h->flags);
  else
    launch_csr_check(st, cb, h->n, h->nnz, h->rowptr, h->colind, vals, h->dvec, h->flags, nullptr);
  std::vector<double> pm(cb);
  int fl = 0;
  GSI_TRY(hip_check(h, hipMemcpyAsync(pm.data(), h->dvec, sizeof(double) * cb, hipMemcpyDeviceToHost, st), "norm"));
  GSI_TRY(hip_check(h, hipMemcpyAsync(&fl, h->flags, sizeof(int), hipMemcpyDeviceToHost, st), "flags"));
  GSI_TRY(hip_check(h, hipStreamSynchronize(st), "set_values"));
  (void)hipMemsetAsync(h->flags, 0, 4 * sizeof(int), st);
  if (fl & 4) return fail(h, GSI_BREAKDOWN, "non-finite matrix value");
  double nA = 0.0;
  for (int i = 0; i < cb; ++i) nA = pm[i] > nA ? pm[i] : nA;
  if (!(nA > 0.0)) return fail(h, GSI_EINVAL, "zero matrix");
  h->nA = nA;
  // the current basis, unpacked into a float64 block (the engine's G0 holds >= n*p doubles;
  // the restart below resets the state that used it)
  if (h->phase == 1)
    launch_unpack<float>(st, h->n, h->p, h->PP, h->e32.X, h->e64.G0);
  else
    launch_unpack<double>(st, h->n, h->p, h->PP, h->e64.X, h->e64.G0);
  const double sign = h->opt.which > 0 ? 1.0 : -1.0;
  if (h->stencil) {
    launch_stencil_diag<double>(st, h->n, h->sdiag, vals, sign, h->e64.vals);
    if (h->mixed) launch_stencil_diag<float>(st, h->n, h->sdiag, vals, sign, h->e32.vals);
  } else {
    launch_convert<double, double>(st, h->nnz, vals, h->e64.vals, sign);
    if (h->mixed) launch_convert<double, float>(st, h->nnz, vals, h->e32.vals, sign);
    if (h->bf16) launch_to_bf16(st, h->nnz, vals, h->e32.vals16, sign);
  }
  return start(h, h->e64.G0);
}

gsi_status gsi_recompute_choice(gsi_handle h, int32_t* recompute_ax, double* ms_recursion, double* ms_recompute) {
  if (!h) return GSI_EINVAL;
  if (recompute_ax) *recompute_ax = h->rax;
  if (ms_recursion) *ms_recursion = h->rax_ms[0];
  if (ms_recompute) *ms_recompute = h->rax_ms[1];
  return GSI_OK;
}

}  // extern "C"

namespace {
// A product staged through an engine's G0 between steps: the gradient of the next step is
// formed again and its direction restarts (G0 may have held the current or the previous
// gradient).
template <typename T>
void invalidate_gradient(gsi_ctx* h, Engine<T>& e) {
  if (!e.sc) return;
  static const int zero = 0, one = 1;
  (void)hipMemcpyAsync(&e.sc->grad_ready, &zero, sizeof(int), hipMemcpyHostToDevice, h->st);
  (void)hipMemcpyAsync(&e.sc->restart_next, &one, sizeof(int), hipMemcpyHostToDevice, h->st);
}
}  // namespace

extern "C" {

gsi_status gsi_spmm(gsi_handle h, const double* W, double* Z) {
  if (!h || !W || !Z) return GSI_EINVAL;
  Engine<double>& e = h->e64;
  invalidate_gradient(h, e);
  // stage through the engine's Z / G0 buffers (padded layout)
  launch_pack<double>(h->st, h->n, h->p, h->PP, W, e.G0, 1.0);
  dispatch_pp<double>(e.PP, [&](auto PPc) {
    constexpr int PP = decltype(PPc)::value;
    spmm_op<double, PP>(h, e, e.G0, e.G0, e.Z, 0);
  });
  launch_unpack<double>(h->st, h->n, h->p, h->PP, e.Z, Z);
  return hip_check(h, hipGetLastError(), "spmm");
}

gsi_status gsi_spmm_lowp(gsi_handle h, const double* W, double* Z) {
  if (!h || !W || !Z) return GSI_EINVAL;
  if (!h->mixed) {
    h->err = "gsi_spmm_lowp needs a mixed-precision handle";
    return GSI_EUNSUPPORTED;
  }
  Engine<float>& e = h->e32;
  invalidate_gradient(h, e);
  invalidate_gradient(h, h->e64);
  const int64_t rows = (h->n + TR - 1) / TR * TR;
  dispatch_pp<float>(e.PP, [&](auto PPc) {
    constexpr int PP = decltype(PPc)::value;
    if (h->bf16) {
      launch_pack<double>(h->st, h->n, h->p, h->PP, W, h->e64.G0, 1.0);
      launch_to_bf16(h->st, rows * PP, h->e64.G0, e.P16, 1.0);
      Kernels<float, PP>::spmm16(h->st, e.n, h->rowptr, h->colind, e.vals16, e.P16, e.Z, e.sc, 0, h->plane_tiles,
                                 h->spmm_batch);
    } else {
      launch_pack<float>(h->st, h->n, h->p, h->PP, W, e.G0, 1.0);
      spmm_op<float, PP>(h, e, e.G0, e.G0, e.Z, 0);
    }
  });
  launch_unpack<float>(h->st, h->n, h->p, h->PP, e.Z, Z);
  return hip_check(h, hipGetLastError(), "spmm_lowp");
}

gsi_status gsi_history(gsi_handle h, int32_t* count, double* rho, double* phi, double* mu, double* beta_pr,
                       double* ginf_rel) {
  if (!h || !count) return GSI_EINVAL;
  if (h->opt.method == GSI_SI) {
    const int m = (int)h->si_rho.size() < *count ? (int)h->si_rho.size() : *count;
    for (int i = 0; i < m; ++i) {
      if (rho) rho[i] = h->si_rho[i];
      if (phi) phi[i] = 0.0;
      if (mu) mu[i] = 0.0;
      if (beta_pr) beta_pr[i] = 0.0;
      if (ginf_rel) ginf_rel[i] = 0.0;
    }
    *count = m;
    return GSI_OK;
  }
  Scalars s;
  GSI_TRY(read_scalars(h, h->phase == 1 ? h->e32.sc : h->e64.sc, &s));
  const int len = (h->phase == 1 ? 0 : h->hist_off) + s.hist_len;
  const int m = len < *count ? len : *count;
  std::vector<double> buf((size_t)(m > 0 ? m : 1) * H_FIELDS);
  if (m > 0)
    GSI_TRY(hip_check(h, hipMemcpy(buf.data(), h->hist, sizeof(double) * m * H_FIELDS, hipMemcpyDeviceToHost),
                      "history"));
  for (int i = 0; i < m; ++i) {
    const double* r = &buf[(size_t)i * H_FIELDS];
    if (rho) rho[i] = r[H_RHO];
    if (phi) phi[i] = r[H_PHI];
    if (mu) mu[i] = r[H_MU];
    if (beta_pr) beta_pr[i] = r[H_BETA];
    if (ginf_rel) ginf_rel[i] = r[H_GINF];
  }
  *count = m;
  return GSI_OK;
}

gsi_status gsi_counters(gsi_handle h, int32_t* iters, int32_t* spmm, int32_t* restarts, int32_t* refreshes,
                        int32_t* null_steps, int32_t* low_iters, int32_t* eig_sweeps) {
  if (!h) return GSI_EINVAL;
  if (h->opt.method == GSI_SI) {
    if (iters) *iters = h->si_k;
    if (spmm) *spmm = h->si_spmm;
    for (int32_t* q : {restarts, refreshes, null_steps, low_iters, eig_sweeps})
      if (q) *q = 0;
    return GSI_OK;
  }
  Scalars s;
  GSI_TRY(read_scalars(h, h->phase == 1 ? h->e32.sc : h->e64.sc, &s));
  const bool lowonly = h->phase == 1;
  if (iters) *iters = s.k;  // the float64 phase continues the float32 phase's count
  if (spmm) *spmm = s.n_spmm + 1 + (lowonly ? 0 : h->low_spmm);
  if (restarts) *restarts = s.n_restart + (lowonly ? 0 : h->low_restarts);
  if (refreshes) *refreshes = s.n_refresh + (lowonly ? 0 : h->low_refresh);
  if (null_steps) *null_steps = s.n_null + (lowonly ? 0 : h->low_null);
  if (low_iters) *low_iters = lowonly ? s.k : h->low_iters;
  if (eig_sweeps) *eig_sweeps = s.n_sweeps + (lowonly ? 0 : h->low_sweeps);
  return GSI_OK;
}

gsi_status gsi_pass_times(gsi_handle h, int32_t enable, double* ms, int32_t* counts) {
  if (!h) return GSI_EINVAL;
  GSI_TRY(hip_check(h, hipStreamSynchronize(h->st), "pass times"));
  collect_times(h);
  for (int i = 0; i < GSI_NPASS; ++i) {
    if (ms) ms[i] = h->pass_ms[i];
    if (counts) counts[i] = h->pass_count[i];
  }
  if (enable >= 0) {
    h->timing = enable != 0;
    for (int i = 0; i < GSI_NPASS; ++i) {
      h->pass_ms[i] = 0.0;
      h->pass_count[i] = 0;
    }
  }
  return GSI_OK;
}

void gsi_destroy(gsi_handle h) {
  if (!h) return;
  if (h->st) (void)hipStreamSynchronize(h->st);
  h->e64.destroy_graph();
  h->e32.destroy_graph();
  if (h->st2) (void)hipStreamSynchronize(h->st2);
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  if (h->ev_join) (void)hipEventDestroy(h->ev_join);
  if (h->st2) (void)hipStreamDestroy(h->st2);
  h->dev.release();
  if (h->own_stream) (void)hipStreamDestroy(h->st);
  delete h;
}

}  // extern "C"
