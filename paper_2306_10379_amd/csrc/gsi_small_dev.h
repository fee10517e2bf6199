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
constexpr int MAXP = 64;    // block width of the batched solve and of the one-wave routines below
constexpr int TMAXP = 128;  // block width of the single-problem float64 path (two terms per lane)
constexpr int JCODE = 256;  // pair code u * JCODE + v of the Jacobi rotations (u, v < TMAXP)

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
              code = u * JCODE + v;
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
      // rows: A <- J^T A. Lane k of every wave takes columns k, k + 64 (p <= 128), the waves
      // take the rotations in turn: no integer division by the runtime p
      const int w0 = threadIdx.x >> 6, nw = blockDim.x >> 6;
      for (int k = threadIdx.x & 63; k < p; k += 64)
        for (int i = w0; i < nrot; i += nw) {
          const int u = uv[i] / JCODE, v = uv[i] % JCODE;
          const double c = cs[2 * i], s = cs[2 * i + 1];
          const double au = A[u * ld + k], av = A[v * ld + k];
          A[u * ld + k] = c * au - s * av;
          A[v * ld + k] = s * au + c * av;
        }
      __syncthreads();
      // columns: A <- A J, V <- V J (row k)
      for (int k = threadIdx.x & 63; k < p; k += 64)
        for (int i = w0; i < nrot; i += nw) {
          const int u = uv[i] / JCODE, v = uv[i] % JCODE;
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

// Reciprocal, reciprocal square root and square root in float64 from the hardware
// approximations refined by two Newton steps each (the quadratic convergence takes the
// approximation to the last bits); for positive normal arguments.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-x * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-x * y, y, 1.0);
  return fma(0.5 * y, e, y);
}

// Parallel cyclic Jacobi, register-resident (used by the eigendecomposition of P^T P).
//
// The players 0..m-1 (m = p rounded up to even; an odd p gets one zero padding row) meet in
// the round-robin order of the cyclic-by-rows parallel ordering: in round r, position 0
// holds player 0 and position i >= 1 player ((i - 1 + r) mod (m - 1)) + 1, and positions
// i and m-1-i form pair i. The matrix is held in "slot" order, slot 2i for position i and
// slot 2i+1 for position m-1-i, so that every pair is a diagonal 2 x 2 block. Thread t < R h
// (h = m / 2 pairs, R = 256 / h) owns pair J = t mod h: the 2 x 2 blocks (I, J) for
// I = t / h + R q in registers, and the entries of V's columns u_J, v_J (the players of
// pair J) in rows t / h + R q, V in LDS in player order. A round: every wave's lanes 0..h-1
// read the diagonal blocks and form the pair rotations into the wave's own LDS table; each
// thread rotates its blocks (two-sided) and its entries of V (one-sided, in place) and writes
// its blocks to the other LDS buffer at the slots their rows and columns move to for the
// next round (a fixed permutation: every player moves one position, position 1 wraps to
// m-1, position 0 stays); one barrier; each thread reads its blocks back. After m - 1 rounds
// the slots are back in their first order. A rotation is skipped when its pivot is not
// above eps ||A||_F and eps sqrt(|a_pp a_qq|); the sweeps stop at the start of a sweep in
// which no rotation would be made (the whole matrix is tested before the sweep, so no
// confirming sweep is run). Returns the number of sweeps made.
//
// Input: A0 (player order, stride lda, LDS, p x p). Output: eigenvalues into d[0..p),
// V (LDS, stride LV, PP rows) multiplied by all rotations. Abuf: 2 PP^2 doubles of LDS
// (may overlap A0: A0 is read before the first write). Whole workgroup (256 threads).
// FULL: m = PP (p >= PP - 1) and PP >= 32: the pair count and thread layout are compile-time
// constants and the 256 threads own exactly the (PP/2)^2 blocks and the PP rows of V, so the
// validity tests of the general case vanish.
template <int PP, bool FULL>
__device__ inline int jacobi_regs(int p, const double* A0, int lda, double* Abuf, double* V, int LV, double* d) {
  constexpr int NBQ = PP * PP / 1024 > 0 ? PP * PP / 1024 : 1;  // blocks per thread
  constexpr int NVQ = PP * PP / 512 > 0 ? PP * PP / 512 : 1;    // rows of V per thread
  constexpr int H = PP / 2;
  static_assert(!FULL || (H * H == WG * NBQ && PP * H == WG * NVQ), "FULL layout needs PP >= 32");
  struct alignas(16) Rot { double c, s, t, app, aqq; int u, v; };
  __shared__ Rot rtab[WG / 64][H];
  __shared__ double fro_part[WG / 64];
  const int m = FULL ? PP : p + (p & 1), h = FULL ? H : m / 2, R = WG / h;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const bool owner = FULL || tid < R * h;
  const int J = owner ? tid % h : 0, I0 = owner ? tid / h : 0;
  auto pos_of_slot = [&](int s) { return (s & 1) ? m - 1 - (s >> 1) : (s >> 1); };
  auto slot_of_pos = [&](int q) { return q < h ? 2 * q : 2 * (m - 1 - q) + 1; };
  // slot a row/column moves to for the next round
  auto next_slot = [&](int s) {
    const int q = pos_of_slot(s);
    return slot_of_pos(q == 0 ? 0 : (q == 1 ? m - 1 : q - 1));
  };
  auto addr = [&](int i, int j) { return ((i >> 1) * h + (j >> 1)) * 4 + (i & 1) * 2 + (j & 1); };
  double B[NBQ][4];
  int bI[NBQ], dst[NBQ][4];
  double fro2 = 0.0;
#pragma unroll
  for (int q = 0; q < NBQ; ++q) {
    const int I = I0 + R * q;
    bI[q] = (FULL || (owner && I < h)) ? I : -1;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      B[q][e] = 0.0;
      dst[q][e] = 0;
    }
    if (bI[q] >= 0) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int si = 2 * I + (e >> 1), sj = 2 * J + (e & 1);
        const int xi = pos_of_slot(si), xj = pos_of_slot(sj);  // round 0: player x sits at position x
        const double v = (xi < p && xj < p) ? A0[xi * lda + xj] : 0.0;
        B[q][e] = v;
        fro2 += v * v;
        dst[q][e] = addr(next_slot(si), next_slot(sj));
      }
    }
  }
  int vr[NVQ];
#pragma unroll
  for (int q = 0; q < NVQ; ++q) {
    const int r = I0 + R * q;
    vr[q] = (FULL || (owner && r < m)) ? r : -1;
  }
  fro2 = wave_sum(fro2);
  if (lane == 0) fro_part[w] = fro2;
  __syncthreads();  // also: every read of A0 is done before Abuf (which may overlap it) is written
  double fsum = 0.0;
  for (int k = 0; k < WG / 64; ++k) fsum += fro_part[k];
  const double athr2 = EPS * EPS * fsum;  // (eps ||A||_F)^2
  int cur = 0;
#pragma unroll
  for (int q = 0; q < NBQ; ++q)
    if (FULL || bI[q] >= 0)
#pragma unroll
      for (int e = 0; e < 4; ++e) Abuf[addr(2 * bI[q] + (e >> 1), 2 * J + (e & 1))] = B[q][e];
  __syncthreads();
  // pair k = lane of every wave (k < h): its players u (position k), v (position m-1-k)
  int pu = lane, pv = m - 1 - lane;
  Rot* tab = rtab[w];
  int sweep = 0;
  for (; sweep < 40; ++sweep) {
    bool stop = false;
    for (int round = 0; round < m - 1; ++round) {
      const double* Ac = Abuf + cur * PP * PP;
      double* An = Abuf + (cur ^ 1) * PP * PP;
      if (lane < h) {
        const double* blk = Ac + (lane * h + lane) * 4;
        const double app = blk[0], apq = blk[1], aqq = blk[3];
        const double apq2 = apq * apq;
        double c = 1.0, s = 0.0, t = 0.0;
        if (apq2 > athr2 && apq2 > EPS * EPS * fabs(app * aqq) && fabs(apq) > 1e-300) {
          // t = tan of the angle that zeroes a_pq: sgn(tau) / (|tau| + sqrt(1 + tau^2)),
          // tau = (a_qq - a_pp) / (2 a_pq); |tau| <= 1/eps here, so 1 + tau^2 cannot overflow
          const double tau = (aqq - app) * rcp_nr(2.0 * apq);
          const double q1 = 1.0 + tau * tau;
          const double root = q1 * rsq_nr(q1);
          const double ta = rcp_nr(fabs(tau) + root);
          t = tau >= 0.0 ? ta : -ta;
          c = rsq_nr(1.0 + t * t);
          s = t * c;
        }
        Rot rr;
        rr.c = c; rr.s = s; rr.t = t; rr.app = app; rr.aqq = aqq; rr.u = pu; rr.v = pv;
        tab[lane] = rr;
      }
      wave_sync();
      if (round == 0) {
        // would this sweep rotate anything? (the whole matrix against the skip rule)
        int big = 0;
        const double dJ0 = tab[J].app, dJ1 = tab[J].aqq;
#pragma unroll
        for (int q = 0; q < NBQ; ++q) {
          if (!FULL && bI[q] < 0) continue;
          const double dI0 = tab[bI[q]].app, dI1 = tab[bI[q]].aqq;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int a = e >> 1, c = e & 1;
            if (bI[q] == J && a == c) continue;
            const double x2 = B[q][e] * B[q][e];
            const double di = a ? dI1 : dI0, dj = c ? dJ1 : dJ0;
            if (x2 > athr2 && x2 > EPS * EPS * fabs(di * dj) && fabs(B[q][e]) > 1e-300) big = 1;
          }
        }
        if (!__syncthreads_or(big)) {
          stop = true;
          break;
        }
      }
      if (owner) {
        const Rot rJ = tab[J];
        // blocks: B <- R_I^T B R_J; the diagonal block gets the rotated diagonal and an
        // exact zero off the diagonal
#pragma unroll
        for (int q = 0; q < NBQ; ++q) {
          if (!FULL && bI[q] < 0) continue;
          const double cI = tab[bI[q]].c, sI = tab[bI[q]].s;
          double* x = B[q];
          const double r0 = cI * x[0] - sI * x[2], r1 = cI * x[1] - sI * x[3];
          const double r2 = sI * x[0] + cI * x[2], r3 = sI * x[1] + cI * x[3];
          double y0 = rJ.c * r0 - rJ.s * r1, y1 = rJ.s * r0 + rJ.c * r1;
          double y2 = rJ.c * r2 - rJ.s * r3, y3 = rJ.s * r2 + rJ.c * r3;
          const bool dg = bI[q] == J && rJ.s != 0.0;
          const double off = x[1];
          x[0] = dg ? x[0] - rJ.t * off : y0;
          x[3] = dg ? x[3] + rJ.t * off : y3;
          x[1] = dg ? 0.0 : y1;
          x[2] = dg ? 0.0 : y2;
        }
        // V <- V R_J on the columns of pair J's players, in place
        if (rJ.s != 0.0) {
          double xu[NVQ], xv[NVQ];
#pragma unroll
          for (int q = 0; q < NVQ; ++q) {
            xu[q] = 0.0;
            xv[q] = 0.0;
            if (FULL || vr[q] >= 0) {
              xu[q] = V[vr[q] * LV + rJ.u];
              xv[q] = V[vr[q] * LV + rJ.v];
            }
          }
#pragma unroll
          for (int q = 0; q < NVQ; ++q)
            if (FULL || vr[q] >= 0) {
              V[vr[q] * LV + rJ.u] = rJ.c * xu[q] - rJ.s * xv[q];
              V[vr[q] * LV + rJ.v] = rJ.s * xu[q] + rJ.c * xv[q];
            }
        }
#pragma unroll
        for (int q = 0; q < NBQ; ++q)
          if (FULL || bI[q] >= 0)
#pragma unroll
            for (int e = 0; e < 4; ++e) An[dst[q][e]] = B[q][e];
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < NBQ; ++q)
        if (FULL || bI[q] >= 0) {
          const double* blk = An + (bI[q] * h + J) * 4;
#pragma unroll
          for (int e = 0; e < 4; ++e) B[q][e] = blk[e];
        }
      cur ^= 1;
      // next round: every player except player 0 moves on (m - 1 wraps to 1)
      if (lane != 0) pu = pu == m - 1 ? 1 : pu + 1;
      pv = pv == m - 1 ? 1 : pv + 1;
    }
    if (stop) break;
  }
  // eigenvalue of player x: the diagonal entry at its slot (the slots are in their first order)
  const double* Ac = Abuf + cur * PP * PP;
  for (int x = tid; x < p; x += WG) {
    const int sx = slot_of_pos(x);
    d[x] = Ac[addr(sx, sx)];
  }
  __syncthreads();
  return sweep;
}

// ---------------------------------------------------------------- line search (wave 0)

struct Terms {
  double a[TMAXP], b[TMAXP], g[TMAXP], z[TMAXP];
  int act[TMAXP];
};

// phi'(mu) = - sum over active terms of (z + d mu - b z mu^2) / (1 + b mu^2)^2 (Sec. 5.2,
// eq. deriv_P), evaluated by wave 0 (lane i holds terms i and i + 64).
__device__ inline double dphi_term(const Terms& T, int i, double mu) {
  const double b = T.b[i], z = T.z[i], d = T.g[i] - T.a[i] * b;
  const double den = 1.0 + b * mu * mu;
  return (z + d * mu - b * z * mu * mu) / (den * den);
}
__device__ inline double dphi(const Terms& T, int p, double mu) {
  const int l = threadIdx.x & 63;
  double v = 0.0;
  if (l < p && T.act[l]) v = dphi_term(T, l, mu);
  if (l + 64 < p && T.act[l + 64]) v += dphi_term(T, l + 64, mu);
  return -wave_sum(v);
}

// Get_Mu (Algorithm 3, Sec. 5.2, Sec. 6.1): returns mu > 0 or -1 when no usable bracket.
// Called by wave 0 only; p terms (padding terms have b = 0), preal the block size for the
// activity threshold; *evals counts phi' evaluations.
__device__ inline double get_mu(Terms& T, int p, int preal, int* evals) {
  // lane l holds terms l and l + 64 (the second only for p > 64)
  const int l = threadIdx.x & 63, l2 = l + 64;
  const double bl = l < p ? T.b[l] : 0.0;
  const double bl2 = l2 < p ? T.b[l2] : 0.0;
  const double bmax = wave_max(l2 < p ? fmax(bl, bl2) : bl);
  int ev = 0;
  if (!(bmax > 0.0)) { *evals = 0; return -1.0; }
  const bool act = l < p && bl > preal * EPS * bmax;
  const bool act2 = l2 < p && bl2 > preal * EPS * bmax;
  if (l < p) T.act[l] = act ? 1 : 0;
  if (l2 < p) T.act[l2] = act2 ? 1 : 0;
  wave_sync();
  const bool conv = act && T.z[l] > 0.0;
  const bool conv2 = act2 && T.z[l2] > 0.0;
  if (__ballot(conv || conv2) == 0) { *evals = 0; return -1.0; }
  // f(0) = -sum of active zeta
  const double f0 = dphi(T, p, 0.0);
  ++ev;
  if (!(f0 < 0.0)) { *evals = ev; return -1.0; }
  // branch roots of the convex branches, without cancellation (Sec. 6.1, eqs. derv1/derv2)
  auto root = [&](int i) {
    const double b = T.b[i], z = T.z[i], d = T.g[i] - T.a[i] * b;
    const double s = sqrt(d * d + 4.0 * b * z * z);
    return d < 0.0 ? 2.0 * z / (fabs(d) + s) : (d + s) / (2.0 * b * z);
  };
  // phi' at a candidate root: the sum over every active term
  auto dphi_all = [&](double x) {
    double acc = 0.0;
    for (int i = 0; i < p; ++i) {
      if (!T.act[i]) continue;
      const double b = T.b[i], z = T.z[i], d = T.g[i] - T.a[i] * b;
      const double den = 1.0 + b * x * x;
      acc += (z + d * x - b * z * x * x) / (den * den);
    }
    return -acc;
  };
  // every lane evaluates its own candidates
  const double xi = conv ? root(l) : INFINITY;
  const double xi2 = conv2 ? root(l2) : INFINITY;
  const double fxi = conv ? dphi_all(xi) : -1.0;
  const double fxi2 = conv2 ? dphi_all(xi2) : -1.0;
  ev += 1;
  // hi: smallest root with phi' >= 0; lo: largest root below hi (or 0)
  double hi = (conv && fxi >= 0.0) ? xi : INFINITY;
  if (conv2 && fxi2 >= 0.0) hi = fmin(hi, xi2);
  for (int o = 32; o > 0; o >>= 1) hi = fmin(hi, __shfl_xor(hi, o, 64));
  double lo = (conv && xi < hi) ? xi : 0.0;
  if (conv2 && xi2 < hi) lo = fmax(lo, xi2);
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
// lds: 3 PP (PP + 1) doubles: V with the odd stride PP + 1 (the in-place column updates of
// the rotations are then free of bank conflicts) and the two block buffers of jacobi_regs,
// which also hold the temporaries of the products (stride PP). Whole workgroup. The
// arguments cs, uv, nrot, anyr are unused (kept for the callers' shared-memory layout).
template <int PP>
__device__ inline int eig_dev(double* small, int p, bool warm, double* lds, double* cs, int* uv, int* nrot,
                              int* anyr) {
  if constexpr (PP > PP_LDS_MAX) {
    // p up to 128: the parallel cyclic Jacobi (jacobi) with A = V^T S V in LDS (PP x (PP + 1),
    // 132 KB) and the eigenvectors and the products' temporaries in the work area of the small
    // buffer
    constexpr int LD = PP + 1;
    double* A = lds;
    double* work = small + small_work_offset(PP);
    double* Vw = work;                 // PP x LD
    double* T0 = work + PP * LD;       // PP x PP
    double* T1 = work + 2 * PP * LD;   // PP x PP
    const double* S = small + S_S * PP * PP;
    double* Vg = small + S_V * PP * PP;
    if (warm) {
      wg_mm<PP>(Vg, true, Vg, false, T0);  // T0 = V^T V
      __syncthreads();
      for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) T0[e] = 0.5 * (((e / PP) == (e % PP) ? 3.0 : 0.0) - T0[e]);
      __syncthreads();
      wg_mm<PP>(Vg, false, T0, false, T1);  // T1 = V (3I - V^T V) / 2
    } else {
      for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) T1[e] = (e / PP) == (e % PP) ? 1.0 : 0.0;
    }
    __syncthreads();
    wg_mm<PP>(S, false, T1, false, T0);  // T0 = S V
    __syncthreads();
    wg_mm<PP>(T1, true, T0, false, Vw);  // V^T S V (Vw as a stride-PP temporary)
    __syncthreads();
    // symmetric to the last bit before the rotations (they read both triangles)
    for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) {
      const int i = e / PP, j = e % PP;
      A[i * LD + j] = 0.5 * (Vw[i * PP + j] + Vw[j * PP + i]);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) Vw[(e / PP) * LD + e % PP] = T1[e];
    __syncthreads();
    const int sweeps = jacobi(p, LD, A, Vw, cs, uv, nrot, anyr);
    double* b = small + S_VEC * PP * PP;
    for (int i = threadIdx.x; i < PP; i += blockDim.x) b[i] = i < p ? fmax(A[i * LD + i], 0.0) : 0.0;
    for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) Vg[e] = Vw[(e / PP) * LD + e % PP];
    __syncthreads();
    return sweeps;
  } else {
  constexpr int LV = PP + 1;
  double* Vv = lds;             // PP x LV
  double* Ab = lds + PP * LV;   // 2 PP^2: jacobi_regs buffers
  double* T0 = Ab;              // temporaries, stride PP
  double* V1 = Ab + PP * PP;
  const double* S = small + S_S * PP * PP;
  double* Vg = small + S_V * PP * PP;
  if (warm) {
    wg_mm<PP>(Vg, true, Vg, false, T0);  // T0 = V^T V
    __syncthreads();
    for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) T0[e] = 0.5 * (((e / PP) == (e % PP) ? 3.0 : 0.0) - T0[e]);
    __syncthreads();
    wg_mm<PP>(Vg, false, T0, false, V1);  // V1 = V (3I - V^T V) / 2
  } else {
    for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) V1[e] = (e / PP) == (e % PP) ? 1.0 : 0.0;
  }
  __syncthreads();
  wg_mm<PP>(S, false, V1, false, Vv);  // Vv (as a stride-PP temporary) = S V
  __syncthreads();
  wg_mm<PP>(V1, true, Vv, false, T0);  // T0 = V^T S V
  __syncthreads();
  for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) Vv[(e / PP) * LV + e % PP] = V1[e];
  __syncthreads();
  double* b = small + S_VEC * PP * PP;
  // the compile-time layout needs every thread to own blocks: PP >= 32 (H^2 = 256 NBQ)
  const int sweeps = (PP >= 32 && p >= PP - 1) ? jacobi_regs<PP, PP >= 32>(p, T0, PP, Ab, Vv, LV, b)
                                               : jacobi_regs<PP, false>(p, T0, PP, Ab, Vv, LV, b);
  for (int i = threadIdx.x; i < PP; i += blockDim.x) b[i] = i < p ? fmax(b[i], 0.0) : 0.0;
  for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) Vg[e] = Vv[(e / PP) * LV + e % PP];
  __syncthreads();
  return sweeps;
  }
}

// ---------------------------------------------------------------- line search and retraction factor

// Exact line search (Sec. 5.2, Algorithm 3, Sec. 6.1) from V, b (eig_dev), C = small[S_C],
// S = small[S_S] and the Grams P^T A P (PZr) and P^T A X (PYr). On success (*sok = 1) it
// writes mu (*smu), M = small[S_M], the next C and W (small[S_C], small[S_W]) and the largest
// b (*sbmax), and with want_mc also M C_next = small[S_MC] (the right factor of the next
// gradient, G = (X - mu P) M C_next - (Y - mu Z) M, for the fused retraction pass). lds: 4 PP^2
// doubles; terms, smu, sok, sevals, sbmax in shared memory. Whole workgroup.
template <int PP>
__device__ inline void linesearch_dev(const double* PZr, const double* PYr, double* small, int p, double* lds,
                                      Terms& terms, double* smu, int* sok, int* sevals, double* sbmax,
                                      bool want_mc = false) {
  double* V = lds;
  double* Mc = V + PP * PP;
  double* T1 = Mc + PP * PP;
  double* T2 = T1 + PP * PP;
  const double* S = small + S_S * PP * PP;
  double* C = small + S_C * PP * PP;
  const double* bvec = small + S_VEC * PP * PP;
  for (int e = threadIdx.x; e < PP * PP; e += blockDim.x) V[e] = small[S_V * PP * PP + e];
  for (int i = threadIdx.x; i < TMAXP; i += blockDim.x) terms.b[i] = i < PP ? bvec[i] : 0.0;
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
  if (want_mc) {
    wg_mm<PP>(Mc, false, C, false, small + S_MC * PP * PP);
    __syncthreads();
  }
}

}  // namespace gsi
