// Single-workgroup float64 building blocks for the p x p projected problem, shared by the
// per-iteration kernels (gsi_small.hip) and the batched persistent solver (gsi_batched.hip):
// f64 MFMA products of PP x PP matrices, parallel cyclic Jacobi, and Get_Mu with Brent's
// method on phi'.
#pragma once
#include <math.h>

#include "gsi_device.h"
#include "gsi_state.h"

namespace gsi {

constexpr double EPS = 2.220446049250313e-16;
constexpr int MAXP = 64;

// Order LDS traffic among the lanes of one wavefront (used where only wave 0 runs).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------- dense PP x PP products

// Cout = alpha * op(A) op(B) for PP x PP row-major operands (any memory space), f64 MFMA,
// 16 x 16 output blocks dealt to the 4 waves. No barrier inside. The operands of a block
// are all loaded before its products: from global memory the block then waits for one
// round of loads instead of one per group of K steps (these single-workgroup kernels have
// no other waves to hide the latency).
template <int PP>
__device__ inline void wg_mm(const double* A, bool ta, const double* B, bool tb, double* Cout, double alpha = 1.0) {
  constexpr int NBK = PP / 16;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, c = l & 15;
  for (int blk = w; blk < NBK * NBK; blk += 4) {
    const int ib = blk / NBK, jb = blk % NBK;
    double a[PP / 4], b[PP / 4];
#pragma unroll
    for (int s = 0; s < PP / 4; ++s) {
      const int k = 4 * s + g;
      a[s] = ta ? A[k * PP + 16 * ib + c] : A[(16 * ib + c) * PP + k];
      b[s] = tb ? B[(16 * jb + c) * PP + k] : B[k * PP + 16 * jb + c];
    }
    d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < PP / 4; ++s) acc = mfma(a[s], b[s], acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) Cout[(16 * ib + g + 4 * r) * PP + 16 * jb + c] = alpha * acc[r];
  }
}

// out[i] = sign * sum_k V[k][i] T[k][i]  (the diagonal of V^T T), i < PP.
template <int PP>
__device__ inline void col_dots(const double* V, const double* T, double* out, double sign) {
  for (int i = threadIdx.x; i < PP; i += blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < PP; ++k) s += V[k * PP + i] * T[k * PP + i];
    out[i] = sign * s;
  }
}

// ---------------------------------------------------------------- Jacobi

// Parallel cyclic Jacobi (round-robin pairs) on the leading p x p block of the symmetric
// matrix A (LDS, stride ld). On return the diagonal of A holds the eigenvalues and V
// (LDS, stride ld) has been multiplied by all rotations. A rotation is skipped when its
// pivot is below eps * ||A||_F or eps * sqrt(|a_uu a_vv|); the sweeps stop when a whole
// sweep skips every rotation. Returns the number of sweeps.
__device__ inline int jacobi(int p, int ld, double* A, double* V, double* cs /* 2*MAXP */, int* uv /* MAXP */,
                      int* nrot_s, int* any_s) {
  const int m = p + (p & 1);
  const int half = m / 2;
  __shared__ double fro;
  if (threadIdx.x < 64) {
    double s = 0.0;
    for (int e = threadIdx.x; e < p * p; e += 64) {
      const double v = A[(e / p) * ld + e % p];
      s += v * v;
    }
    s = wave_sum(s);
    if (threadIdx.x == 0) fro = sqrt(s);
  }
  __syncthreads();
  const double athr = EPS * fro;
  int sweep = 0;
  for (; sweep < 40; ++sweep) {
    if (threadIdx.x == 0) *any_s = 0;
    for (int round = 0; round < m - 1; ++round) {
      if (threadIdx.x < 64) {  // wave 0: rotation parameters, compacted to the rotating pairs
        const int i = threadIdx.x;
        bool rot = false;
        double c = 1.0, s = 0.0;
        int code = 0;
        if (i < half) {
          auto player = [&](int pos) { return pos == 0 ? 0 : ((pos - 1 + round) % (m - 1)) + 1; };
          int u = player(i), v = player(m - 1 - i);
          if (u > v) { const int t = u; u = v; v = t; }
          if (v < p) {
            const double auu = A[u * ld + u], avv = A[v * ld + v], auv = A[u * ld + v];
            if (fabs(auv) > athr && fabs(auv) > EPS * sqrt(fabs(auu * avv)) && fabs(auv) > 1e-300) {
              const double tau = (avv - auu) / (2.0 * auv);
              const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
              c = 1.0 / sqrt(1.0 + t * t);
              s = t * c;
              code = u * MAXP + v;
              rot = true;
            }
          }
        }
        const uint64_t mask = __ballot(rot);
        if (rot) {
          const int idx = __popcll(mask & ((1ull << i) - 1ull));
          cs[2 * idx] = c;
          cs[2 * idx + 1] = s;
          uv[idx] = code;
        }
        if (i == 0) {
          *nrot_s = __popcll(mask);
          if (mask) *any_s = 1;
        }
      }
      __syncthreads();
      const int nrot = *nrot_s;
      if (nrot == 0) continue;  // uniform: every thread read the same value after the barrier
      // rows: A <- J^T A. Lane k of every wave takes column k (p <= 64), the waves take the
      // rotations in turn: no integer division by the runtime p
      const int k = threadIdx.x & 63, w0 = threadIdx.x >> 6, nw = blockDim.x >> 6;
      if (k < p)
        for (int i = w0; i < nrot; i += nw) {
          const int u = uv[i] / MAXP, v = uv[i] % MAXP;
          const double c = cs[2 * i], s = cs[2 * i + 1];
          const double au = A[u * ld + k], av = A[v * ld + k];
          A[u * ld + k] = c * au - s * av;
          A[v * ld + k] = s * au + c * av;
        }
      __syncthreads();
      // columns: A <- A J, V <- V J (row k)
      if (k < p)
        for (int i = w0; i < nrot; i += nw) {
          const int u = uv[i] / MAXP, v = uv[i] % MAXP;
          const double c = cs[2 * i], s = cs[2 * i + 1];
          const double au = A[k * ld + u], av = A[k * ld + v];
          A[k * ld + u] = c * au - s * av;
          A[k * ld + v] = s * au + c * av;
          const double vu = V[k * ld + u], vv = V[k * ld + v];
          V[k * ld + u] = c * vu - s * vv;
          V[k * ld + v] = s * vu + c * vv;
        }
      __syncthreads();
    }
    __syncthreads();
    if (*any_s == 0) break;
    __syncthreads();
  }
  __syncthreads();
  return sweep + 1;
}

// ---------------------------------------------------------------- line search (wave 0)

struct Terms {
  double a[MAXP], b[MAXP], g[MAXP], z[MAXP];
  int act[MAXP];
};

// phi'(mu) = - sum over active terms of (z + d mu - b z mu^2) / (1 + b mu^2)^2 (Sec. 5.2,
// eq. deriv_P), evaluated by wave 0 (lane i holds term i).
__device__ inline double dphi(const Terms& T, int p, double mu) {
  const int l = threadIdx.x & 63;
  double v = 0.0;
  if (l < p && T.act[l]) {
    const double b = T.b[l], z = T.z[l], d = T.g[l] - T.a[l] * b;
    const double den = 1.0 + b * mu * mu;
    v = (z + d * mu - b * z * mu * mu) / (den * den);
  }
  return -wave_sum(v);
}

// Get_Mu (Algorithm 3, Sec. 5.2, Sec. 6.1): returns mu > 0 or -1 when no usable bracket.
// Called by wave 0 only; p terms (padding terms have b = 0), preal the block size for the
// activity threshold; *evals counts phi' evaluations.
__device__ inline double get_mu(Terms& T, int p, int preal, int* evals) {
  const int l = threadIdx.x & 63;
  const double bl = l < p ? T.b[l] : 0.0;
  const double bmax = wave_max(bl);
  int ev = 0;
  if (!(bmax > 0.0)) { *evals = 0; return -1.0; }
  const bool act = l < p && bl > preal * EPS * bmax;
  if (l < p) T.act[l] = act ? 1 : 0;
  wave_sync();
  const bool conv = act && T.z[l] > 0.0;
  if (__ballot(conv) == 0) { *evals = 0; return -1.0; }
  // f(0) = -sum of active zeta
  const double f0 = dphi(T, p, 0.0);
  ++ev;
  if (!(f0 < 0.0)) { *evals = ev; return -1.0; }
  // branch roots of the convex branches, without cancellation (Sec. 6.1, eqs. derv1/derv2)
  double xi = INFINITY;
  if (conv) {
    const double b = T.b[l], z = T.z[l], d = T.g[l] - T.a[l] * b;
    const double s = sqrt(d * d + 4.0 * b * z * z);
    xi = d < 0.0 ? 2.0 * z / (fabs(d) + s) : (d + s) / (2.0 * b * z);
  }
  // phi' at every candidate root, each lane evaluating its own candidate
  double fxi = -1.0;
  if (conv) {
    double acc = 0.0;
    for (int i = 0; i < p; ++i) {
      if (!T.act[i]) continue;
      const double b = T.b[i], z = T.z[i], d = T.g[i] - T.a[i] * b;
      const double den = 1.0 + b * xi * xi;
      acc += (z + d * xi - b * z * xi * xi) / (den * den);
    }
    fxi = -acc;
  }
  ev += 1;
  // hi: smallest root with phi' >= 0; lo: largest root below hi (or 0)
  double hi = (conv && fxi >= 0.0) ? xi : INFINITY;
  for (int o = 32; o > 0; o >>= 1) hi = fmin(hi, __shfl_xor(hi, o, 64));
  double lo = (conv && xi < hi) ? xi : 0.0;
  for (int o = 32; o > 0; o >>= 1) lo = fmax(lo, __shfl_xor(lo, o, 64));
  double fhi;
  if (hi == INFINITY) {
    int widen = 0;
    hi = 2.0 * (lo > 0.0 ? lo : 1.0);
    fhi = dphi(T, p, hi);
    ++ev;
    while (fhi < 0.0 && widen < 60) {
      lo = hi;
      hi *= 2.0;
      fhi = dphi(T, p, hi);
      ++ev;
      ++widen;
    }
    if (fhi < 0.0) { *evals = ev; return -1.0; }
  } else {
    fhi = dphi(T, p, hi);
    ++ev;
  }
  if (fhi == 0.0) { *evals = ev; return hi; }
  double flo = dphi(T, p, lo);
  ++ev;
  if (flo == 0.0) { *evals = ev; return lo; }
  // Brent's method (Brent 1973, ch. 4): inverse quadratic interpolation / secant steps
  // safeguarded by bisection, on phi' over [lo, hi] with flo < 0 < fhi.
  double a = lo, b = hi, c = lo, fa = flo, fb = fhi, fc = flo;
  double d = b - a, e = d;
  for (int it = 0; it < 200; ++it) {
    if ((fb > 0.0 && fc > 0.0) || (fb < 0.0 && fc < 0.0)) {
      c = a; fc = fa; d = b - a; e = d;
    }
    if (fabs(fc) < fabs(fb)) {
      a = b; b = c; c = a;
      fa = fb; fb = fc; fc = fa;
    }
    const double tol1 = 2.0 * EPS * fabs(b) + 1e-300;
    const double xm = 0.5 * (c - b);
    if (fabs(xm) <= tol1 || fb == 0.0) break;
    if (fabs(e) >= tol1 && fabs(fa) > fabs(fb)) {
      double pp, q, r;
      const double s = fb / fa;
      if (a == c) {
        pp = 2.0 * xm * s;
        q = 1.0 - s;
      } else {
        q = fa / fc;
        r = fb / fc;
        pp = s * (2.0 * xm * q * (q - r) - (b - a) * (r - 1.0));
        q = (q - 1.0) * (r - 1.0) * (s - 1.0);
      }
      if (pp > 0.0) q = -q; else pp = -pp;
      if (2.0 * pp < fmin(3.0 * xm * q - fabs(tol1 * q), fabs(e * q))) {
        e = d;
        d = pp / q;
      } else {
        d = xm;
        e = d;
      }
    } else {
      d = xm;
      e = d;
    }
    a = b;
    fa = fb;
    b += fabs(d) > tol1 ? d : (xm > 0.0 ? tol1 : -tol1);
    fb = dphi(T, p, b);
    ++ev;
  }
  *evals = ev;
  return b;
}


// ---------------------------------------------------------------- eigendecomposition of P^T P

// P^T P = V diag(b) V^T (Sec. 5.2) for S = small[S_S]: writes V (small[S_V]) and b
// (small[S_VEC ...]); returns the Jacobi sweep count. Warm start (warm = true): the previous
// V, made orthonormal again by one Newton-Schulz step V <- V (3 I - V^T V) / 2, turns S
// into a nearly diagonal V^T S V when the directions change little from step to step.
// lds: 3 PP (PP + 1) doubles. The products use stride PP, the rotations stride PP + 1 (an
// odd stride in doubles keeps the column sweeps of the rotations free of LDS bank
// conflicts). Whole workgroup.
template <int PP>
__device__ inline int eig_dev(double* small, int p, bool warm, double* lds, double* cs, int* uv, int* nrot,
                              int* anyr) {
  constexpr int LP = PP + 1;
  double* A = lds;
  double* V = A + PP * LP;
  double* T = V + PP * LP;
  const double* S = small + S_S * PP * PP;
  double* Vg = small + S_V * PP * PP;
  if (warm) {
    wg_mm<PP>(Vg, true, Vg, false, T);  // T = V^T V
    __syncthreads();
    for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) T[e] = 0.5 * (((e / PP) == (e % PP) ? 3.0 : 0.0) - T[e]);
    __syncthreads();
    wg_mm<PP>(Vg, false, T, false, V);  // V = V (3I - V^T V) / 2
  } else {
    for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) V[e] = (e / PP) == (e % PP) ? 1.0 : 0.0;
  }
  __syncthreads();
  wg_mm<PP>(S, false, V, false, T);  // T = S V
  __syncthreads();
  wg_mm<PP>(V, true, T, false, A);  // A = V^T S V
  __syncthreads();
  // re-lay A (into T) and V (into A) with stride LP for the rotations
  for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) T[(e / PP) * LP + e % PP] = A[e];
  __syncthreads();
  for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) A[(e / PP) * LP + e % PP] = V[e];
  __syncthreads();
  double* Ap = T;
  double* Vp = A;
  const int sweeps = jacobi(p, LP, Ap, Vp, cs, uv, nrot, anyr);
  double* b = small + S_VEC * PP * PP;
  for (int i = threadIdx.x; i < PP; i += blockDim.x) b[i] = i < p ? fmax(Ap[i * LP + i], 0.0) : 0.0;
  for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) Vg[e] = Vp[(e / PP) * LP + e % PP];
  __syncthreads();
  return sweeps;
}

// ---------------------------------------------------------------- line search and retraction factor

// Exact line search (Sec. 5.2, Algorithm 3, Sec. 6.1) from V, b (eig_dev), C = small[S_C],
// S = small[S_S] and the Grams P^T A P (PZr) and P^T A X (PYr). On success (*sok = 1) it
// writes mu (*smu), M = small[S_M], the next C and W (small[S_C], small[S_W]) and the largest
// b (*sbmax). lds: 4 PP^2 doubles; terms, smu, sok, sevals, sbmax in shared memory. Whole
// workgroup.
template <int PP>
__device__ inline void linesearch_dev(const double* PZr, const double* PYr, double* small, int p, double* lds,
                                      Terms& terms, double* smu, int* sok, int* sevals, double* sbmax) {
  double* V = lds;
  double* Mc = V + PP * PP;
  double* T1 = Mc + PP * PP;
  double* T2 = T1 + PP * PP;
  const double* S = small + S_S * PP * PP;
  double* C = small + S_C * PP * PP;
  const double* bvec = small + S_VEC * PP * PP;
  for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) V[e] = small[S_V * PP * PP + e];
  for (int i = threadIdx.x; i < MAXP; i += blockDim.x) terms.b[i] = i < PP ? bvec[i] : 0.0;
  __syncthreads();
  // line-search diagonals (Sec. 5.2, eq. CG_linesearch_D) in the basis V; the diagonal of
  // V^T B V only needs the symmetric part of B, so the raw Grams are used
  wg_mm<PP>(C, false, V, false, T1);
  wg_mm<PP>(PZr, false, V, false, T2);
  __syncthreads();
  col_dots<PP>(V, T1, terms.a, 1.0);
  col_dots<PP>(V, T2, terms.g, 1.0);
  wg_mm<PP>(PYr, false, V, false, Mc);
  __syncthreads();
  col_dots<PP>(V, Mc, terms.z, -1.0);
  __syncthreads();
  if (threadIdx.x < 64) {
    int evals = 0;
    const double mu = get_mu(terms, PP, p, &evals);
    if (threadIdx.x == 0) {
      *smu = mu;
      *sok = mu > 0.0 && isfinite(mu);
      *sevals = evals;
      double bmax = 0.0;
      for (int i = 0; i < p; ++i) bmax = fmax(bmax, terms.b[i]);
      *sbmax = bmax;
    }
  }
  __syncthreads();
  if (!*sok) return;
  const double mu = *smu;
  // M = V diag((1 + mu^2 b)^{-1/2}) V^T (Sec. 5.2, eq. Xnew_P). V is orthogonal only to
  // about (number of rotations) * eps, which would let X(mu) drift from orthonormality
  // step after step; one Newton step for the inverse square root of B = I + mu^2 S,
  // M <- M (3 I - M B M) / 2, restores M B M = I to second order.
  // (terms.a is free after Get_Mu: it holds the PP column factors (1 + mu^2 b)^{-1/2})
  for (int i = threadIdx.x; i < PP; i += blockDim.x) terms.a[i] = 1.0 / sqrt(1.0 + mu * mu * terms.b[i]);
  __syncthreads();
  for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) T1[e] = V[e] * terms.a[e % PP];
  __syncthreads();
  wg_mm<PP>(T1, false, V, true, Mc);  // Mc = V D V^T
  __syncthreads();
  wg_mm<PP>(S, false, Mc, false, T1);  // T1 = S M
  __syncthreads();
  for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) T1[e] = Mc[e] + mu * mu * T1[e];  // B M
  __syncthreads();
  wg_mm<PP>(Mc, false, T1, false, T2);  // M B M
  __syncthreads();
  for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) T2[e] = ((e / PP) == (e % PP) ? 3.0 : 0.0) - T2[e];
  __syncthreads();
  wg_mm<PP>(Mc, false, T2, false, T1);  // M (3I - M B M)
  __syncthreads();
  double* M = small + S_M * PP * PP;
  for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) {
    const int i = e / PP, j = e % PP;
    const double v = 0.25 * (T1[i * PP + j] + T1[j * PP + i]);
    Mc[e] = v;
    M[e] = v;
  }
  __syncthreads();
  // next C = M (C - mu (P^T Y + Y^T P) + mu^2 P^T Z) M and next W = X_new^T P = -mu M S
  // (X^T P = 0 for the tangent direction; A X recursion of Sec. 6.1, eq. save_matvec)
  for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) {
    const int i = e / PP, j = e % PP;
    T2[e] = C[e] - mu * (PYr[e] + PYr[j * PP + i]) + 0.5 * mu * mu * (PZr[e] + PZr[j * PP + i]);
  }
  __syncthreads();
  wg_mm<PP>(Mc, false, T2, false, T1);
  __syncthreads();
  wg_mm<PP>(T1, false, Mc, false, T2);
  double* W = small + S_W * PP * PP;
  wg_mm<PP>(Mc, false, S, false, W, -mu);
  __syncthreads();
  for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) {
    const int i = e / PP, j = e % PP;
    C[e] = 0.5 * (T2[e] + T2[j * PP + i]);
  }
  __syncthreads();
}

}  // namespace gsi
