// Sine-basis neural operator for warm starts (see include/fno.h): forward pass, subspace
// loss, gradient and Adam, all as gfx950 kernels on float32 data, with the weights read as
// float32 or from a bfloat16 working copy (Wp).
//
// Data layout: activations channel-major, [sample][channel][N x N grid, row-major], so a
// channel of a sample is one contiguous n = N^2 vector. The sine transform of a channel,
// S U S^T, is two contractions over contiguous indices (rows, then the transposed result),
// the inverse S^T V S likewise through the transposed sine matrix St = S^T; all four are
// C = P Q^T products done by one MFMA kernel (k_pqt) with a strided output. Gram-like
// reductions over the whole grid (weight gradients, the p x p Grams of the loss) split the
// grid over workgroups and add the partial results in a fixed order (k_pqt_small,
// k_sum_parts). Pointwise channel mixing, GELU and the mode-wise channel mixing are plain
// coalesced kernels. The p x p loss algebra (Cholesky of Y^T Y) runs in float64, one
// workgroup per sample.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/fno.h"
#include "gsi_device.h"

namespace fno {

using gsi::f4;
using gsi::gld;
using gsi::gst;
using gsi::mfma;
constexpr int WG = 256;

__device__ __forceinline__ f4 ld4(const float* p) { return gld(reinterpret_cast<const f4*>(p)); }

// A run of weights: the float32 master, or (h set) its bfloat16 working copy, widened on
// reading. The choice is the same for every thread of a launch.
struct Wp {
  const float* f;
  const uint16_t* h;
  __device__ __forceinline__ float operator[](int64_t i) const {
    return h ? gsi::bf16_widen(gld(h + i)) : gld(f + i);
  }
};

// ---------------------------------------------------------------- C = alpha P Q^T + beta C

struct PQt {
  const float* P;
  int64_t ldp, sPb;  // row stride, batch stride
  const float* Q;
  int64_t ldq, sQb;
  float* C;
  int64_t so_r, so_c, sCb;  // output element (r, c) of batch b at C + b sCb + r so_r + c so_c
  int R, Cc, K;             // K a multiple of 16, ldp and ldq multiples of 4
  float alpha, beta;
};

// Workgroup: rows 64 bx .. + 63, columns 32 by .. + 31 of batch entry bz. Wave w owns 16 rows
// and two 16-column MFMA blocks. Lane (g, c) = (l / 16, l % 16) loads 16 bytes at k0 + 4g of
// P row (row0 + c) and of Q rows (col0 + c), (col0 + 16 + c); MFMA step q contracts index
// k0 + 4g + q over g (A lane layout A[c][g], B lane layout B[g][c]), so the four steps cover
// k0 .. k0 + 15. D: register r of lane (g, c) is row 4g + r, column c.
__global__ __launch_bounds__(WG) void k_pqt(PQt a) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, c = l & 15;
  const int64_t b = blockIdx.z;
  const int row0 = blockIdx.x * 64 + 16 * w, col0 = blockIdx.y * 32;
  if (row0 >= a.R) return;  // whole wave outside; the kernel has no barrier
  const float* P = a.P + b * a.sPb;
  const float* Q = a.Q + b * a.sQb;
  const int pr = row0 + c, qr0 = col0 + c, qr1 = col0 + 16 + c;
  const bool pok = pr < a.R, ok0 = qr0 < a.Cc, ok1 = qr1 < a.Cc;
  const float* pp = P + (int64_t)(pok ? pr : 0) * a.ldp + 4 * g;
  const float* qp0 = Q + (int64_t)(ok0 ? qr0 : 0) * a.ldq + 4 * g;
  const float* qp1 = Q + (int64_t)(ok1 ? qr1 : 0) * a.ldq + 4 * g;
  const f4 z = {0.f, 0.f, 0.f, 0.f};
  f4 acc0 = z, acc1 = z;
#pragma unroll 2
  for (int k0 = 0; k0 < a.K; k0 += 16) {
    const f4 pv = pok ? ld4(pp + k0) : z;
    const f4 v0 = ok0 ? ld4(qp0 + k0) : z;
    const f4 v1 = ok1 ? ld4(qp1 + k0) : z;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      acc0 = mfma(pv[q], v0[q], acc0);
      acc1 = mfma(pv[q], v1[q], acc1);
    }
  }
  float* Cb = a.C + b * a.sCb;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = row0 + 4 * g + r;
    if (row >= a.R) continue;
    if (ok0) {
      float* o = Cb + row * a.so_r + qr0 * a.so_c;
      gst(o, a.alpha * acc0[r] + (a.beta != 0.f ? a.beta * gld(o) : 0.f));
    }
    if (ok1) {
      float* o = Cb + row * a.so_r + qr1 * a.so_c;
      gst(o, a.alpha * acc1[r] + (a.beta != 0.f ? a.beta * gld(o) : 0.f));
    }
  }
}

// ---------------------------------------------------------------- small outputs, long K

struct PQtSmall {
  const float* P;
  int64_t ldp, sPb;
  const float* Q;
  int64_t ldq, sQb;
  int R, Cc;  // both <= 32
  int64_t K;  // multiple of 16
  int splits;
  float* part;  // [batch][split][32 x 32]
};

// Partial P_b Q_b^T over the split's share of K: grid (splits, batch). Every wave takes every
// fourth 16-wide step of the share and keeps all four 16 x 16 blocks; the waves' sums are
// added in wave order in LDS.
__global__ __launch_bounds__(WG) void k_pqt_small(PQtSmall a) {
  __shared__ float red[32 * 32];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, c = l & 15;
  const int s = blockIdx.x, b = blockIdx.y;
  const int64_t nk = a.K / 16;
  const int64_t k_lo = nk * s / a.splits, k_hi = nk * (s + 1) / a.splits;
  const float* P = a.P + (int64_t)b * a.sPb;
  const float* Q = a.Q + (int64_t)b * a.sQb;
  const bool pok0 = c < a.R, pok1 = 16 + c < a.R, qok0 = c < a.Cc, qok1 = 16 + c < a.Cc;
  const float* p0 = P + (pok0 ? c : 0) * a.ldp + 4 * g;
  const float* p1 = P + (pok1 ? 16 + c : 0) * a.ldp + 4 * g;
  const float* q0 = Q + (qok0 ? c : 0) * a.ldq + 4 * g;
  const float* q1 = Q + (qok1 ? 16 + c : 0) * a.ldq + 4 * g;
  const f4 z = {0.f, 0.f, 0.f, 0.f};
  f4 acc[2][2] = {{z, z}, {z, z}};
  for (int64_t kk = k_lo + w; kk < k_hi; kk += 4) {
    const int64_t k0 = kk * 16;
    const f4 a0 = pok0 ? ld4(p0 + k0) : z, a1 = pok1 ? ld4(p1 + k0) : z;
    const f4 b0 = qok0 ? ld4(q0 + k0) : z, b1 = qok1 ? ld4(q1 + k0) : z;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      acc[0][0] = mfma(a0[q], b0[q], acc[0][0]);
      acc[0][1] = mfma(a0[q], b1[q], acc[0][1]);
      acc[1][0] = mfma(a1[q], b0[q], acc[1][0]);
      acc[1][1] = mfma(a1[q], b1[q], acc[1][1]);
    }
  }
  for (int ww = 0; ww < 4; ++ww) {
    if (w == ww) {
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int e = (16 * rb + 4 * g + r) * 32 + 16 * cb + c;
            red[e] = (ww ? red[e] : 0.f) + acc[rb][cb][r];
          }
    }
    __syncthreads();
  }
  float* out = a.part + ((int64_t)b * a.splits + s) * 1024;
  for (int e = threadIdx.x; e < 1024; e += WG) gst(out + e, red[e]);
}

// out[gr][r][c] (at gr so_g + r ldo + c) = alpha * sum of the group's partials in order.
template <typename TO>
__global__ void k_sum_parts(const float* part, int per_group, int groups, int R, int Cc, TO* out, int64_t so_g,
                            int ldo, float alpha) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int gr = blockIdx.y;
  if (e >= R * Cc || gr >= groups) return;
  const int r = e / Cc, c = e % Cc;
  double acc = 0.0;
  for (int j = 0; j < per_group; ++j) acc += (double)gld(part + ((int64_t)gr * per_group + j) * 1024 + r * 32 + c);
  gst(out + gr * so_g + r * ldo + c, (TO)(alpha * acc));
}

// ---------------------------------------------------------------- pointwise kernels

__device__ __forceinline__ float gelu(float t) { return 0.5f * t * (1.0f + erff(t * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float t) {
  return 0.5f * (1.0f + erff(t * 0.70710678118654752f)) + t * 0.39894228040143268f * expf(-0.5f * t * t);
}

// In[b] = [V / 20, x, y]; U0[b][c] = W_lift In + b_lift. Thread per (sample, node).
__global__ void k_lift(const float* V, int N, int w, Wp W, Wp bias, float* In, float* U0, int B) {
  const int64_t n = (int64_t)N * N;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)B * n) return;
  const int64_t b = id / n, j = id % n;
  const float h = 1.0f / (float)(N + 1);
  const float f0 = gld(V + id) * 0.05f, f1 = (float)(j % N + 1) * h, f2 = (float)(j / N + 1) * h;
  gst(In + (b * 3 + 0) * n + j, f0);
  gst(In + (b * 3 + 1) * n + j, f1);
  gst(In + (b * 3 + 2) * n + j, f2);
  for (int c = 0; c < w; ++c)
    gst(U0 + (b * w + c) * n + j, bias[c] + W[3 * c] * f0 + W[3 * c + 1] * f1 + W[3 * c + 2] * f2);
}

// s = Vs[b][o] + sum_c W[o][c] U[b][c] + bias[o] (+ add[o], the same for every sample);
// Pre = s (if given); Out = act ? gelu(s) : s.
__global__ __launch_bounds__(WG) void k_point_fwd(const float* Vs, const float* U, Wp W, Wp bias, const float* add,
                                                  float* Pre, float* Out, int O, int C, int64_t n, int B, int act) {
  __shared__ float sW[32 * 32 + 32];
  for (int e = threadIdx.x; e < O * C; e += WG) sW[e] = W[e];
  for (int e = threadIdx.x; e < O; e += WG) sW[1024 + e] = bias[e];
  __syncthreads();
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)B * n) return;
  const int64_t b = id / n, j = id % n;
  float u[32];
#pragma unroll
  for (int c = 0; c < 32; ++c) u[c] = c < C ? gld(U + (b * C + c) * n + j) : 0.f;
  for (int o = 0; o < O; ++o) {
    float s = gld(Vs + (b * O + o) * n + j) + sW[1024 + o] + (add ? gld(add + o * n + j) : 0.f);
#pragma unroll
    for (int c = 0; c < 32; ++c)
      if (c < C) s += sW[o * C + c] * u[c];
    if (Pre) gst(Pre + (b * O + o) * n + j, s);
    gst(Out + (b * O + o) * n + j, act ? gelu(s) : s);
  }
}

// dPre = act ? dOut * gelu'(Pre) : dOut (stored when dPre is given); dU[b][c] = sum_o W[o][c] dPre[b][o].
__global__ __launch_bounds__(WG) void k_point_bwd(const float* dOut, const float* Pre, Wp W, float* dPre, float* dU,
                                                  int O, int C, int64_t n, int B, int act) {
  __shared__ float sW[32 * 32];
  for (int e = threadIdx.x; e < O * C; e += WG) sW[e] = W[e];
  __syncthreads();
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)B * n) return;
  const int64_t b = id / n, j = id % n;
  float du[32];
#pragma unroll
  for (int c = 0; c < 32; ++c) du[c] = 0.f;
  for (int o = 0; o < O; ++o) {
    float d = gld(dOut + (b * O + o) * n + j);
    if (act) d *= gelu_d(gld(Pre + (b * O + o) * n + j));
    if (dPre) gst(dPre + (b * O + o) * n + j, d);
#pragma unroll
    for (int c = 0; c < 32; ++c)
      if (c < C) du[c] += sW[o * C + c] * d;
  }
#pragma unroll
  for (int c = 0; c < 32; ++c)
    if (c < C) gst(dU + (b * C + c) * n + j, du[c]);
}

// ---------------------------------------------------------------- mode-wise channel mixing

// Vh[b][o][k] = sum_c R[o][c][k] Uh[b][c][k] on the m x m modes (zero on the padding of MP).
__global__ void k_mix_fwd(Wp R, const float* Uh, float* Vh, int B, int O, int C, int m, int MP) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)MP * MP;
  if (id >= (int64_t)B * O * per) return;
  const int64_t bo = id / per, k = id % per;
  const int k1 = (int)(k / MP), k2 = (int)(k % MP);
  const int64_t b = bo / O, o = bo % O;
  float s = 0.f;
  if (k1 < m && k2 < m)
    for (int c = 0; c < C; ++c)
      s += R[((o * C + c) * m + k1) * m + k2] * gld(Uh + (b * C + c) * per + k);
  gst(Vh + id, s);
}

// dUh[b][c][k] = sum_o R[o][c][k] dVh[b][o][k].
__global__ void k_mix_bwd(Wp R, const float* dVh, float* dUh, int B, int O, int C, int m, int MP) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)MP * MP;
  if (id >= (int64_t)B * C * per) return;
  const int64_t bc = id / per, k = id % per;
  const int k1 = (int)(k / MP), k2 = (int)(k % MP);
  const int64_t b = bc / C, c = bc % C;
  float s = 0.f;
  if (k1 < m && k2 < m)
    for (int o = 0; o < O; ++o)
      s += R[((o * C + c) * m + k1) * m + k2] * gld(dVh + (b * O + o) * per + k);
  gst(dUh + id, s);
}

// dR[o][c][k1][k2] = sum_b dVh[b][o][k] Uh[b][c][k].
__global__ void k_mix_wgrad(const float* dVh, const float* Uh, float* dR, int B, int O, int C, int m, int MP) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)O * C * m * m) return;
  const int64_t oc = id / (m * m), k = id % (m * m);
  const int k1 = (int)(k / m), k2 = (int)(k % m);
  const int64_t o = oc / C, c = oc % C;
  const int64_t per = (int64_t)MP * MP, kp = (int64_t)k1 * MP + k2;
  float s = 0.f;
  for (int b = 0; b < B; ++b) s += gld(dVh + ((int64_t)b * O + o) * per + kp) * gld(Uh + ((int64_t)b * C + c) * per + kp);
  gst(dR + id, s);
}

// ---------------------------------------------------------------- loss

// One workgroup per sample: G = Y^T Y, Bm = X*^T Y (float64, rows of 32). Cholesky of G,
// Gi = G^-1, M = Bm^T Bm, loss = p - Tr(Gi M), and the coefficients of the gradient
// dLoss/dY = scale (Y Kc - X* Ec) with Kc = Gi M Gi, Ec = Bm Gi, scale = 2 / batch.
__global__ __launch_bounds__(WG) void k_loss_small(const double* G, const double* Bm, int p, double scale,
                                                   double* loss, float* Kc, float* Ec, int* bad) {
  __shared__ double L[32 * 33], Li[32 * 33], Gi[32 * 33], Ms[32 * 33], T[32 * 33], Bs[32 * 33];
  __shared__ int sbad;
  const int b = blockIdx.x, t = threadIdx.x;
  const double* Gb = G + (int64_t)b * 1024;
  const double* Bb = Bm + (int64_t)b * 1024;
  for (int e = t; e < p * p; e += WG) {
    const int i = e / p, j = e % p;
    L[i * 33 + j] = 0.5 * (Gb[i * 32 + j] + Gb[j * 32 + i]);
    Bs[i * 33 + j] = Bb[i * 32 + j];
    Li[i * 33 + j] = 0.0;
  }
  if (t == 0) sbad = 0;
  __syncthreads();
  if (t == 0) {
    // Cholesky (lower) and the inverse of L, serially: p <= 32
    for (int j = 0; j < p && !sbad; ++j) {
      double d = L[j * 33 + j];
      for (int k = 0; k < j; ++k) d -= L[j * 33 + k] * L[j * 33 + k];
      if (!(d > 0.0) || !isfinite(d)) { sbad = 1; break; }
      const double ljj = sqrt(d);
      L[j * 33 + j] = ljj;
      for (int i = j + 1; i < p; ++i) {
        double s = L[i * 33 + j];
        for (int k = 0; k < j; ++k) s -= L[i * 33 + k] * L[j * 33 + k];
        L[i * 33 + j] = s / ljj;
      }
    }
    if (!sbad)
      for (int cidx = 0; cidx < p; ++cidx)
        for (int i = cidx; i < p; ++i) {
          double s = (i == cidx) ? 1.0 : 0.0;
          for (int k = cidx; k < i; ++k) s -= L[i * 33 + k] * Li[k * 33 + cidx];
          Li[i * 33 + cidx] = s / L[i * 33 + i];
        }
  }
  __syncthreads();
  if (sbad) {
    if (t == 0) { loss[b] = NAN; atomicExch(bad, 1); }
    for (int e = t; e < 1024; e += WG) { Kc[(int64_t)b * 1024 + e] = 0.f; Ec[(int64_t)b * 1024 + e] = 0.f; }
    return;
  }
  // Gi = Li^T Li ; M = Bm^T Bm
  for (int e = t; e < p * p; e += WG) {
    const int i = e / p, j = e % p;
    double s = 0.0, m = 0.0;
    for (int k = (i > j ? i : j); k < p; ++k) s += Li[k * 33 + i] * Li[k * 33 + j];
    for (int k = 0; k < p; ++k) m += Bs[k * 33 + i] * Bs[k * 33 + j];
    Gi[i * 33 + j] = s;
    Ms[i * 33 + j] = m;
  }
  __syncthreads();
  // T = Gi M
  for (int e = t; e < p * p; e += WG) {
    const int i = e / p, j = e % p;
    double s = 0.0;
    for (int k = 0; k < p; ++k) s += Gi[i * 33 + k] * Ms[k * 33 + j];
    T[i * 33 + j] = s;
  }
  __syncthreads();
  if (t == 0) {
    double tr = 0.0;
    for (int i = 0; i < p; ++i) tr += T[i * 33 + i];
    loss[b] = (double)p - tr;
  }
  // Kc = T Gi, Ec = Bm Gi (row index a' of the sum, column a of dY)
  for (int e = t; e < 1024; e += WG) {
    const int i = e / 32, j = e % 32;
    double kv = 0.0, ev = 0.0;
    if (i < p && j < p)
      for (int k = 0; k < p; ++k) {
        kv += T[i * 33 + k] * Gi[k * 33 + j];
        ev += Bs[i * 33 + k] * Gi[k * 33 + j];
      }
    Kc[(int64_t)b * 1024 + e] = (float)(scale * kv);
    Ec[(int64_t)b * 1024 + e] = (float)(scale * ev);
  }
}

// dY[b][a][i] = sum_a' Kc[a'][a] Y[b][a'][i] - Ec[a'][a] X[b][a'][i]. Thread per (sample, node).
__global__ __launch_bounds__(WG) void k_loss_dy(const float* Y, const float* X, const float* Kc, const float* Ec,
                                                float* dY, int p, int64_t n, int B) {
  __shared__ float sK[1024], sE[1024];
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // every sample of a workgroup's range: n is a multiple of 256, so one sample per block
  const int64_t b = ((int64_t)blockIdx.x * blockDim.x) / n;
  for (int e = threadIdx.x; e < 1024; e += WG) {
    sK[e] = b < B ? gld(Kc + b * 1024 + e) : 0.f;
    sE[e] = b < B ? gld(Ec + b * 1024 + e) : 0.f;
  }
  __syncthreads();
  if (id >= (int64_t)B * n) return;
  const int64_t j = id % n;
  float y[32], x[32];
#pragma unroll
  for (int a = 0; a < 32; ++a) {
    y[a] = a < p ? gld(Y + (b * p + a) * n + j) : 0.f;
    x[a] = a < p ? gld(X + (b * p + a) * n + j) : 0.f;
  }
  for (int a = 0; a < p; ++a) {
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < 32; ++q)
      if (q < p) s += sK[q * 32 + a] * y[q] - sE[q * 32 + a] * x[q];
    gst(dY + (b * p + a) * n + j, s);
  }
}

// ---------------------------------------------------------------- layout, Adam

// dst[b][a][i] = src[b][i][a] (B blocks n x p row-major -> channel-major).
__global__ void k_to_channels(const float* src, float* dst, int p, int64_t n, int B) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)B * n * p) return;
  const int64_t b = id / (n * p), r = id % (n * p), a = r / n, i = r % n;
  gst(dst + id, gld(src + (b * n + i) * p + a));
}

// Y32 / Y64 [b][i][a] = Y[b][a][i].
__global__ void k_from_channels(const float* Y, float* Y32, double* Y64, int p, int64_t n, int B) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)B * n * p) return;
  const int64_t b = id / (n * p), r = id % (n * p), i = r / p, a = r % p;
  const float v = gld(Y + (b * p + a) * n + i);
  if (Y32) gst(Y32 + id, v);
  if (Y64) gst(Y64 + id, (double)v);
}

// Adam on the float32 master w; wbf (nullable) receives the updated weights rounded to bfloat16.
__global__ void k_adam(float* w, uint16_t* wbf, const float* g, float* m1, float* m2, int64_t count, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = gld(g + i);
  const float m = b1 * gld(m1 + i) + (1.f - b1) * gi;
  const float v = b2 * gld(m2 + i) + (1.f - b2) * gi * gi;
  gst(m1 + i, m);
  gst(m2 + i, v);
  const float nw = gld(w + i) - lr * (m / c1) / (sqrtf(v / c2) + eps);
  gst(w + i, nw);
  if (wbf) gst(wbf + i, gsi::bf16_round(nw));
}

__global__ void k_round_bf16(const float* w, uint16_t* wbf, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) gst(wbf + i, gsi::bf16_round(gld(w + i)));
}

// splitmix64 (Steele, Lea, Flood 2014) and Box-Muller for the seeded initial weights.
struct Rng {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
  double normal() { return sqrt(-2.0 * log(uniform())) * cos(6.283185307179586 * uniform()); }
};

}  // namespace fno

using namespace fno;

struct fno_net {
  fno_config cfg{};
  int MP = 0;
  int64_t n = 0, count = 0;
  hipStream_t st = nullptr;
  bool own_stream = false;
  std::string err;
  std::vector<void*> allocs;
  // parameter offsets: lift, per hidden layer (R, W, b), output layer (R, W, b)
  int64_t oWl = 0, obl = 0;
  std::vector<int64_t> oR, oW, ob;  // L + 1 entries, the last is the output layer
  float *params = nullptr, *grad = nullptr, *m1 = nullptr, *m2 = nullptr;
  uint16_t* wbf = nullptr;  // bfloat16 working copy of params (bf16_weights), else null
  int64_t step = 0;
  float *S = nullptr, *St = nullptr, *ones = nullptr, *prior = nullptr;
  float *In = nullptr, *Y = nullptr, *Xc = nullptr, *dY = nullptr, *dPre = nullptr, *dUa = nullptr, *dUb = nullptr;
  float *Wt = nullptr, *Vh = nullptr, *dUh = nullptr, *Zt = nullptr, *Vs = nullptr, *part = nullptr;
  std::vector<float*> act, pre, uh;
  double *G = nullptr, *Bm = nullptr, *lossd = nullptr;
  float *Kc = nullptr, *Ec = nullptr;
  int* bad = nullptr;
  int splits = 1;
};

namespace {

bool valid(const fno_config* c) {
  return c && c->N >= 16 && c->N <= 1024 && c->N % 16 == 0 && c->modes >= 1 && c->modes <= 32 && c->modes <= c->N &&
         c->width >= 1 && c->width <= 32 && c->p >= 1 && c->p <= 32 && c->layers >= 0 && c->max_batch >= 1 &&
         (c->bf16_weights == 0 || c->bf16_weights == 1);
}

// The weights at parameter offset off, in the format the passes read.
Wp wp(const fno_net* h, int64_t off) { return Wp{h->params + off, h->wbf ? h->wbf + off : nullptr}; }

int64_t count_params(const fno_config* c) {
  const int64_t w = c->width, m = c->modes, p = c->p;
  return 3 * w + w + c->layers * (w * w * m * m + w * w + w) + p * w * m * m + p * w + p;
}

template <typename U>
U* nalloc(fno_net* h, size_t count, hipError_t& e) {
  void* ptr = nullptr;
  if (e != hipSuccess) return nullptr;
  e = hipMalloc(&ptr, std::max<size_t>(count, 1) * sizeof(U) + 256);
  if (e != hipSuccess) return nullptr;
  h->allocs.push_back(ptr);
  return reinterpret_cast<U*>(ptr);
}

inline unsigned blocks(int64_t work, int per = WG) { return (unsigned)((work + per - 1) / per); }

// C = alpha P Q^T + beta C with the grid for R x Cc outputs per batch entry
void pqt(fno_net* h, const PQt& a, int batch) {
  dim3 grid((unsigned)((a.R + 63) / 64), (unsigned)((a.Cc + 31) / 32), (unsigned)batch);
  k_pqt<<<grid, WG, 0, h->st>>>(a);
}

// Uh[bc] = S U[bc] S^T for BC channels (MP x MP each, zero beyond m)
void fwd_transform(fno_net* h, const float* U, int BC, float* Uh) {
  const int N = h->cfg.N, MP = h->MP;
  pqt(h, PQt{U, N, h->n, h->S, N, 0, h->Wt, 1, N, (int64_t)MP * N, N, MP, N, 1.f, 0.f}, BC);
  pqt(h, PQt{h->S, N, 0, h->Wt, N, (int64_t)MP * N, Uh, MP, 1, (int64_t)MP * MP, MP, MP, N, 1.f, 0.f}, BC);
}

// Out[bo] = S^T Vh[bo] S + beta Out[bo] for BO channels
void inv_transform(fno_net* h, const float* Vh, int BO, float* Out, float beta) {
  const int N = h->cfg.N, MP = h->MP;
  pqt(h, PQt{Vh, MP, (int64_t)MP * MP, h->St, MP, 0, h->Zt, 1, MP, (int64_t)N * MP, MP, N, MP, 1.f, 0.f}, BO);
  pqt(h, PQt{h->St, MP, 0, h->Zt, MP, (int64_t)N * MP, Out, N, 1, h->n, N, N, MP, 1.f, beta}, BO);
}

// out (groups of R x Cc, element (r, c) at gr so_g + r ldo + c) = alpha * sum over the
// batch entries of each group of P_b Q_b^T, with P_b: R x n, Q_b: Cc x n.
template <typename TO>
void gram_small(fno_net* h, const float* P, int64_t sPb, const float* Q, int64_t sQb, int R, int Cc, int B,
                bool per_sample, TO* out, int64_t so_g, int ldo, float alpha) {
  PQtSmall a{P, h->n, sPb, Q, h->n, sQb, R, Cc, h->n, h->splits, h->part};
  k_pqt_small<<<dim3((unsigned)h->splits, (unsigned)B), WG, 0, h->st>>>(a);
  const int groups = per_sample ? B : 1;
  const int per_group = per_sample ? h->splits : B * h->splits;
  k_sum_parts<TO><<<dim3(blocks(R * Cc), (unsigned)groups), WG, 0, h->st>>>(h->part, per_group, groups, R, Cc, out,
                                                                            so_g, ldo, alpha);
}

void forward(fno_net* h, const float* V, int B) {
  const fno_config& c = h->cfg;
  const int w = c.width, p = c.p, L = c.layers, m = c.modes, MP = h->MP;
  const int64_t n = h->n;
  k_lift<<<blocks(B * n), WG, 0, h->st>>>(V, c.N, w, wp(h, h->oWl), wp(h, h->obl), h->In, h->act[0], B);
  for (int l = 0; l <= L; ++l) {
    const int O = l < L ? w : p;
    fwd_transform(h, h->act[l], B * w, h->uh[l]);
    k_mix_fwd<<<blocks((int64_t)B * O * MP * MP), WG, 0, h->st>>>(wp(h, h->oR[l]), h->uh[l], h->Vh, B, O, w, m, MP);
    inv_transform(h, h->Vh, B * O, h->Vs, 0.f);
    k_point_fwd<<<blocks(B * n), WG, 0, h->st>>>(h->Vs, h->act[l], wp(h, h->oW[l]), wp(h, h->ob[l]),
                                                 l < L ? nullptr : h->prior, l < L ? h->pre[l] : nullptr, l < L ? h->act[l + 1] : h->Y, O, w, n,
                                                 B, l < L ? 1 : 0);
  }
}

// Backward from dY (channel-major, the gradient of the mean loss) into h->grad.
void backward(fno_net* h, int B) {
  const fno_config& c = h->cfg;
  const int w = c.width, p = c.p, L = c.layers, m = c.modes, MP = h->MP;
  const int64_t n = h->n;
  float* cur = h->dUa;
  float* nxt = h->dUb;
  for (int l = L; l >= 0; --l) {
    const int O = l < L ? w : p;
    const float* dOut = l < L ? cur : h->dY;
    float* dU = l < L ? nxt : cur;
    // dPre (= dY for the output layer) and the local part of dU
    k_point_bwd<<<blocks(B * n), WG, 0, h->st>>>(dOut, l < L ? h->pre[l] : nullptr, wp(h, h->oW[l]),
                                                 l < L ? h->dPre : nullptr, dU, O, w, n, B, l < L ? 1 : 0);
    const float* dP = l < L ? h->dPre : h->dY;
    // W and b gradients: sums over samples and nodes
    gram_small<float>(h, dP, (int64_t)O * n, h->act[l], (int64_t)w * n, O, w, B, false, h->grad + h->oW[l], 0, w, 1.f);
    gram_small<float>(h, dP, (int64_t)O * n, h->ones, 0, O, 1, B, false, h->grad + h->ob[l], 0, 1, 1.f);
    // spectral part: dVh = S dPre S^T, dR, dUh, dU += S^T dUh S
    fwd_transform(h, dP, B * O, h->Vh);
    k_mix_wgrad<<<blocks((int64_t)O * w * m * m), WG, 0, h->st>>>(h->Vh, h->uh[l], h->grad + h->oR[l], B, O, w, m, MP);
    k_mix_bwd<<<blocks((int64_t)B * w * MP * MP), WG, 0, h->st>>>(wp(h, h->oR[l]), h->Vh, h->dUh, B, O, w, m, MP);
    inv_transform(h, h->dUh, B * w, dU, 1.f);
    if (l < L) std::swap(cur, nxt);
  }
  // lift: cur holds dU_0
  gram_small<float>(h, cur, (int64_t)w * n, h->In, 3 * n, w, 3, B, false, h->grad + h->oWl, 0, 3, 1.f);
  gram_small<float>(h, cur, (int64_t)w * n, h->ones, 0, w, 1, B, false, h->grad + h->obl, 0, 1, 1.f);
}

gsi_status hip_status(fno_net* h, hipError_t e, const char* what) {
  if (e == hipSuccess) return GSI_OK;
  h->err = std::string(what) + ": " + hipGetErrorString(e);
  return GSI_EDEVICE;
}

}  // namespace

extern "C" {

int64_t fno_param_count(const fno_config* cfg) { return valid(cfg) ? count_params(cfg) : -1; }

gsi_status fno_create(fno_handle* out, const fno_config* cfg, uint64_t seed, void* stream) {
  if (!out) return GSI_EINVAL;
  *out = nullptr;
  fno_net* h = new (std::nothrow) fno_net();
  if (!h) return GSI_ENOMEM;
  *out = h;
  if (!valid(cfg)) {
    h->err = "invalid configuration (N a multiple of 16 in 16..1024, 1 <= modes <= 32, width, p <= 32, bf16_weights 0 or 1)";
    return GSI_EINVAL;
  }
  h->cfg = *cfg;
  const fno_config& c = h->cfg;
  h->MP = (c.modes + 15) / 16 * 16;
  h->n = (int64_t)c.N * c.N;
  h->count = count_params(cfg);
  h->splits = (int)std::max<int64_t>(1, std::min<int64_t>(32, h->n / 16 / 16));
  h->st = reinterpret_cast<hipStream_t>(stream);
  if (!h->st) {
    if (hipStreamCreate(&h->st) != hipSuccess) { h->err = "stream creation failed"; return GSI_EDEVICE; }
    h->own_stream = true;
  }
  const int w = c.width, p = c.p, L = c.layers, m = c.modes, N = c.N, MP = h->MP;
  const int64_t n = h->n, B = c.max_batch, mx = std::max(w, p);
  // parameter offsets in the documented order
  int64_t off = 0;
  h->oWl = off; off += 3 * w;
  h->obl = off; off += w;
  for (int l = 0; l <= L; ++l) {
    const int64_t O = l < L ? w : p;
    h->oR.push_back(off); off += O * w * m * m;
    h->oW.push_back(off); off += O * w;
    h->ob.push_back(off); off += O;
  }
  hipError_t e = hipSuccess;
  h->params = nalloc<float>(h, h->count, e);
  h->grad = nalloc<float>(h, h->count, e);
  if (c.bf16_weights) h->wbf = nalloc<uint16_t>(h, h->count, e);
  h->m1 = nalloc<float>(h, h->count, e);
  h->m2 = nalloc<float>(h, h->count, e);
  h->S = nalloc<float>(h, (size_t)MP * N, e);
  h->St = nalloc<float>(h, (size_t)N * MP, e);
  h->ones = nalloc<float>(h, n, e);
  h->prior = nalloc<float>(h, (size_t)p * n, e);
  h->In = nalloc<float>(h, B * 3 * n, e);
  for (int l = 0; l <= L; ++l) h->act.push_back(nalloc<float>(h, B * w * n, e));
  for (int l = 0; l < L; ++l) h->pre.push_back(nalloc<float>(h, B * w * n, e));
  for (int l = 0; l <= L; ++l) h->uh.push_back(nalloc<float>(h, B * w * MP * MP, e));
  h->Y = nalloc<float>(h, B * p * n, e);
  h->Xc = nalloc<float>(h, B * p * n, e);
  h->dY = nalloc<float>(h, B * p * n, e);
  h->dPre = nalloc<float>(h, B * mx * n, e);
  h->dUa = nalloc<float>(h, B * w * n, e);
  h->dUb = nalloc<float>(h, B * w * n, e);
  h->Vs = nalloc<float>(h, B * mx * n, e);
  h->Wt = nalloc<float>(h, B * mx * MP * N, e);
  h->Zt = nalloc<float>(h, B * mx * N * MP, e);
  h->Vh = nalloc<float>(h, B * mx * MP * MP, e);
  h->dUh = nalloc<float>(h, B * w * MP * MP, e);
  h->part = nalloc<float>(h, (size_t)B * h->splits * 1024, e);
  h->G = nalloc<double>(h, B * 1024, e);
  h->Bm = nalloc<double>(h, B * 1024, e);
  h->lossd = nalloc<double>(h, B, e);
  h->Kc = nalloc<float>(h, B * 1024, e);
  h->Ec = nalloc<float>(h, B * 1024, e);
  h->bad = nalloc<int>(h, 1, e);
  if (e != hipSuccess) { h->err = "out of device memory"; return GSI_ENOMEM; }
  // host-side constants: sine matrices (zero beyond m), ones, seeded parameters
  std::vector<float> S((size_t)MP * N, 0.f), St((size_t)N * MP, 0.f), ones(n, 1.f), prm(h->count, 0.f);
  const double sc = sqrt(2.0 / (N + 1));
  for (int k = 0; k < m; ++k)
    for (int i = 0; i < N; ++i) {
      const double v = sc * sin(M_PI * (double)(k + 1) * (double)(i + 1) / (double)(N + 1));
      S[(size_t)k * N + i] = (float)v;
      St[(size_t)i * MP + k] = (float)v;
    }
  // prior: sqrt(n) times the p lowest Dirichlet modes s_l(row) s_k(col), by k^2 + l^2, then k
  std::vector<float> prior((size_t)p * n);
  {
    std::vector<std::pair<int, int>> modes;
    const int K = (int)ceil(sqrt(2.0 * p)) + 2;
    for (int k = 1; k <= K; ++k)
      for (int l = 1; l <= K; ++l) modes.push_back({k, l});
    std::stable_sort(modes.begin(), modes.end(), [](const std::pair<int, int>& x, const std::pair<int, int>& y) {
      const int ex = x.first * x.first + x.second * x.second, ey = y.first * y.first + y.second * y.second;
      return ex != ey ? ex < ey : x.first < y.first;
    });
    for (int a = 0; a < p; ++a) {
      const int k = modes[a].first, l = modes[a].second;
      for (int r = 0; r < N; ++r)
        for (int c2 = 0; c2 < N; ++c2)
          prior[(size_t)a * n + (size_t)r * N + c2] =
              (float)((double)N * sc * sin(M_PI * l * (r + 1.0) / (N + 1.0)) * sc * sin(M_PI * k * (c2 + 1.0) / (N + 1.0)));
    }
  }
  Rng rng{seed};
  auto fill = [&](int64_t o, int64_t cnt, double sd) {
    for (int64_t i = 0; i < cnt; ++i) prm[o + i] = (float)(sd * rng.normal());
  };
  fill(h->oWl, 3 * w, 1.0 / sqrt(3.0));
  for (int l = 0; l < L; ++l) {  // the output layer starts at zero: the network starts at the prior
    fill(h->oR[l], (int64_t)w * w * m * m, 1.0 / sqrt((double)w));
    fill(h->oW[l], (int64_t)w * w, 1.0 / sqrt((double)w));
  }
  e = hipMemcpyAsync(h->S, S.data(), S.size() * 4, hipMemcpyHostToDevice, h->st);
  if (e == hipSuccess) e = hipMemcpyAsync(h->St, St.data(), St.size() * 4, hipMemcpyHostToDevice, h->st);
  if (e == hipSuccess) e = hipMemcpyAsync(h->ones, ones.data(), ones.size() * 4, hipMemcpyHostToDevice, h->st);
  if (e == hipSuccess) e = hipMemcpyAsync(h->params, prm.data(), prm.size() * 4, hipMemcpyHostToDevice, h->st);
  if (e == hipSuccess) e = hipMemcpyAsync(h->prior, prior.data(), prior.size() * 4, hipMemcpyHostToDevice, h->st);
  if (e == hipSuccess) e = hipMemsetAsync(h->m1, 0, h->count * 4, h->st);
  if (e == hipSuccess) e = hipMemsetAsync(h->m2, 0, h->count * 4, h->st);
  if (e == hipSuccess) e = hipMemsetAsync(h->grad, 0, h->count * 4, h->st);
  if (e == hipSuccess && h->wbf) {
    k_round_bf16<<<blocks(h->count), WG, 0, h->st>>>(h->params, h->wbf, h->count);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(h->st);
  return hip_status(h, e, "create");
}

gsi_status fno_set_params(fno_handle h, const float* params) {
  if (!h || !params) return GSI_EINVAL;
  hipError_t e = hipMemcpyAsync(h->params, params, h->count * 4, hipMemcpyDeviceToDevice, h->st);
  if (e == hipSuccess && h->wbf) {
    k_round_bf16<<<blocks(h->count), WG, 0, h->st>>>(h->params, h->wbf, h->count);
    e = hipGetLastError();
  }
  return hip_status(h, e, "set_params");
}

gsi_status fno_get_params(fno_handle h, float* params) {
  if (!h || !params) return GSI_EINVAL;
  hipError_t e = hipMemcpyAsync(params, h->params, h->count * 4, hipMemcpyDeviceToDevice, h->st);
  if (e == hipSuccess) e = hipStreamSynchronize(h->st);
  return hip_status(h, e, "get_params");
}

gsi_status fno_forward(fno_handle h, const float* V, int32_t B, float* Y32, double* Y64) {
  if (!h || !V || B < 1 || B > h->cfg.max_batch) return GSI_EINVAL;
  forward(h, V, B);
  if (Y32 || Y64)
    k_from_channels<<<blocks((int64_t)B * h->n * h->cfg.p), WG, 0, h->st>>>(h->Y, Y32, Y64, h->cfg.p, h->n, B);
  return hip_status(h, hipGetLastError(), "forward");
}

gsi_status fno_loss_grad(fno_handle h, const float* V, const float* Xs, int32_t B, double* loss, float* grad) {
  if (!h || !V || !Xs || B < 1 || B > h->cfg.max_batch) return GSI_EINVAL;
  const int p = h->cfg.p;
  const int64_t n = h->n;
  forward(h, V, B);
  k_to_channels<<<blocks((int64_t)B * n * p), WG, 0, h->st>>>(Xs, h->Xc, p, n, B);
  hipError_t e = hipMemsetAsync(h->bad, 0, sizeof(int), h->st);
  gram_small<double>(h, h->Y, (int64_t)p * n, h->Y, (int64_t)p * n, p, p, B, true, h->G, 1024, 32, 1.f);
  gram_small<double>(h, h->Xc, (int64_t)p * n, h->Y, (int64_t)p * n, p, p, B, true, h->Bm, 1024, 32, 1.f);
  k_loss_small<<<B, WG, 0, h->st>>>(h->G, h->Bm, p, 2.0 / B, h->lossd, h->Kc, h->Ec, h->bad);
  k_loss_dy<<<blocks((int64_t)B * n), WG, 0, h->st>>>(h->Y, h->Xc, h->Kc, h->Ec, h->dY, p, n, B);
  backward(h, B);
  if (e == hipSuccess && grad) e = hipMemcpyAsync(grad, h->grad, h->count * 4, hipMemcpyDeviceToDevice, h->st);
  std::vector<double> lh(B);
  int bad = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(lh.data(), h->lossd, B * sizeof(double), hipMemcpyDeviceToHost, h->st);
  if (e == hipSuccess) e = hipMemcpyAsync(&bad, h->bad, sizeof(int), hipMemcpyDeviceToHost, h->st);
  if (e == hipSuccess) e = hipStreamSynchronize(h->st);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return hip_status(h, e, "loss_grad");
  if (loss)
    for (int i = 0; i < B; ++i) loss[i] = lh[i];
  if (bad) { h->err = "singular Gram Y^T Y in the loss"; return GSI_EDEVICE; }
  return GSI_OK;
}

gsi_status fno_adam(fno_handle h, float lr, float beta1, float beta2, float eps) {
  if (!h) return GSI_EINVAL;
  ++h->step;
  const float c1 = 1.f - powf(beta1, (float)h->step), c2 = 1.f - powf(beta2, (float)h->step);
  k_adam<<<blocks(h->count), WG, 0, h->st>>>(h->params, h->wbf, h->grad, h->m1, h->m2, h->count, lr, beta1, beta2, eps,
                                              c1, c2);
  return hip_status(h, hipGetLastError(), "adam");
}

const char* fno_last_error(fno_handle h) { return h ? h->err.c_str() : "null handle"; }

void fno_destroy(fno_handle h) {
  if (!h) return;
  if (h->st) (void)hipStreamSynchronize(h->st);
  for (void* ptr : h->allocs) (void)hipFree(ptr);
  if (h->own_stream) (void)hipStreamDestroy(h->st);
  delete h;
}

}  // extern "C"
