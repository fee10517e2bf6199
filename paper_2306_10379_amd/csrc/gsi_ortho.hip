// Standalone orthonormalization of a tall block by two passes of Cholesky QR: X <- X R^{-1}
// with R^T R = X^T X, twice. It is the re-orthonormalization step of the iteration (the
// start block, a warm start, a precision switch) offered on a caller's block, row-major with
// leading dimension p (no padding), float64, in place.
//
// One pass: k_ortho_gram writes per-workgroup partial sums of the upper triangle of X^T X;
// k_ortho_chol adds them in a fixed order (the result repeats bit for bit), factors the sum
// (right-looking Cholesky in LDS) and inverts the factor; k_ortho_apply multiplies X by
// R^{-1} tile by tile. A failed factorization (a non-positive or tiny pivot: X is rank
// deficient or not finite) sets a flag that makes the later kernels of the call return
// without touching X.
//
// Scratch (per call): the partial sums, R^{-1} and two flags. gsi_orthonormalize allocates
// it for the call; gsi_orthonormalize_noalloc uses a file-scope device array instead, so
// that callers that cannot allocate device memory can call it.
#include <hip/hip_runtime.h>

#include <mutex>
#include <stdint.h>

#include "../../include/gsi.h"

namespace {

constexpr int OWG = 256;        // threads per workgroup
constexpr int OMAXP = 64;       // largest block width
constexpr int OMAXWG = 256;     // workgroups of the Gram pass (the partial sums they write)
constexpr int OMAXP2 = OMAXP * (OMAXP + 1) / 2;
constexpr int OTILE = 32;       // rows per tile of the product pass
// scratch layout in doubles: partials [OMAXWG * OMAXP2], R^{-1} [OMAXP * OMAXP], flags
constexpr size_t OFF_RINV = (size_t)OMAXWG * OMAXP2;
constexpr size_t OFF_FLAGS = OFF_RINV + (size_t)OMAXP * OMAXP;
constexpr size_t SCRATCH_DOUBLES = OFF_FLAGS + 64;

// Scratch of gsi_orthonormalize_noalloc: 4.3 MB on every device the library runs on, held
// until the process ends. Host code must not pass this name to a kernel (it is a host-side
// stand-in there): it uses the device address from hipGetSymbolAddress.
__device__ __align__(256) double scratch[SCRATCH_DOUBLES];

int gram_blocks(int64_t n) {
  const int64_t t = (n + 63) / 64;
  return (int)(t < OMAXWG ? t : OMAXWG);
}

// Upper triangle of X^T X over the 64-row tiles of this workgroup (tile loop strided by the
// grid), entry e = (i, j), i <= j, in row-major order of the upper triangle. Partials:
// partials[blockIdx.x * p (p + 1) / 2 + e].
__global__ __launch_bounds__(OWG) void k_ortho_gram(int64_t n, int p, const double* __restrict__ X,
                                                    double* __restrict__ partials, const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double sX[64 * OMAXP];
  const int P2 = p * (p + 1) / 2;
  constexpr int PER = (OMAXP2 + OWG - 1) / OWG;
  int ei[PER], ej[PER];
  double acc[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    int e = threadIdx.x + OWG * k, i = 0;
    ei[k] = -1;
    ej[k] = 0;
    acc[k] = 0.0;
    if (e < P2) {
      while (e >= p - i) { e -= p - i; ++i; }
      ei[k] = i;
      ej[k] = i + e;
    }
  }
  const int64_t ntiles = (n + 63) / 64;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t r0 = t * 64;
    const int64_t cnt = (n - r0 < 64 ? n - r0 : 64) * p;
    const double* src = X + r0 * p;
    for (int e = threadIdx.x; e < 64 * p; e += OWG) sX[e] = e < cnt ? src[e] : 0.0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      if (ei[k] >= 0) {
        double s = acc[k];
        for (int r = 0; r < 64; ++r) s += sX[r * p + ei[k]] * sX[r * p + ej[k]];
        acc[k] = s;
      }
    }
    __syncthreads();
  }
  double* out = partials + (int64_t)blockIdx.x * P2;
#pragma unroll
  for (int k = 0; k < PER; ++k)
    if (ei[k] >= 0) out[threadIdx.x + OWG * k] = acc[k];
}

// One workgroup: G = sum of the nb partials (fixed order), G = L L^T, rinv = L^{-T} (upper
// triangular, p x p row-major, zero below the diagonal). flag_out = 1 when a pivot is not
// above 1e-13 max_i G_ii (or not finite), or when flag_in (nullable) is already set.
__global__ __launch_bounds__(OWG) void k_ortho_chol(int p, int nb, const double* __restrict__ partials,
                                                    double* __restrict__ rinv, const int* __restrict__ flag_in,
                                                    int* __restrict__ flag_out) {
  // lower triangle: L (strictly below the diagonal); upper triangle with the diagonal: R^{-1}
  __shared__ double A[OMAXP * OMAXP];
  __shared__ double dL[OMAXP];
  __shared__ int bad;
  __shared__ double dmax;
  if (flag_in && *flag_in) {
    if (threadIdx.x == 0) *flag_out = 1;
    return;
  }
  const int P2 = p * (p + 1) / 2;
  for (int e = threadIdx.x; e < P2; e += OWG) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partials[(int64_t)b * P2 + e];
    int i = 0, r = e;
    while (r >= p - i) { r -= p - i; ++i; }
    const int j = i + r;
    A[i * OMAXP + j] = s;
    A[j * OMAXP + i] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    bad = 0;
    double m = 0.0;
    for (int i = 0; i < p; ++i) m = fmax(m, A[i * OMAXP + i]);
    dmax = m;
  }
  __syncthreads();
  // right-looking Cholesky on the lower triangle
  for (int j = 0; j < p; ++j) {
    if (threadIdx.x == 0) {
      const double piv = A[j * OMAXP + j];
      if (!(piv > 1e-13 * dmax) || !isfinite(piv)) bad = 1;
      dL[j] = sqrt(fabs(piv) > 0.0 && isfinite(piv) ? fabs(piv) : 1.0);
    }
    __syncthreads();
    const double ljj = dL[j];
    for (int i = j + 1 + threadIdx.x; i < p; i += OWG) A[i * OMAXP + j] /= ljj;
    __syncthreads();
    const int m = p - j - 1;
    for (int e = threadIdx.x; e < m * m; e += OWG) {
      const int i = j + 1 + e / m, k = j + 1 + e % m;
      if (k <= i) A[i * OMAXP + k] -= A[i * OMAXP + j] * A[k * OMAXP + j];
    }
    __syncthreads();
  }
  // row c of R^{-1} = column c of L^{-1}: thread c, forward substitution
  for (int c = threadIdx.x; c < p; c += OWG) {
    A[c * OMAXP + c] = 1.0 / dL[c];
    for (int i = c + 1; i < p; ++i) {
      double s = 0.0;
      for (int k = c; k < i; ++k) s -= A[i * OMAXP + k] * A[c * OMAXP + k];
      A[c * OMAXP + i] = s / dL[i];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < p * p; e += OWG) {
    const int i = e / p, j = e % p;
    rinv[e] = j >= i ? A[i * OMAXP + j] : 0.0;
  }
  if (threadIdx.x == 0) *flag_out = bad;
}

// X <- X R^{-1} in place, OTILE rows at a time (the tile is read into LDS before any of
// its rows is written). Returns at once when the factorization failed.
__global__ __launch_bounds__(OWG) void k_ortho_apply(int64_t n, int p, double* __restrict__ X,
                                                     const double* __restrict__ rinv, const int* __restrict__ flag) {
  if (*flag) return;
  __shared__ double sR[OMAXP * OMAXP];
  __shared__ double sX[OTILE * OMAXP];
  for (int e = threadIdx.x; e < p * p; e += OWG) sR[e] = rinv[e];
  const int64_t ntiles = (n + OTILE - 1) / OTILE;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t r0 = t * OTILE;
    const int64_t cnt = (n - r0 < OTILE ? n - r0 : OTILE) * p;
    double* dst = X + r0 * p;
    __syncthreads();
    for (int e = threadIdx.x; e < cnt; e += OWG) sX[e] = dst[e];
    __syncthreads();
    for (int e = threadIdx.x; e < cnt; e += OWG) {
      const int r = e / p, j = e % p;
      double s = 0.0;
      for (int i = 0; i <= j; ++i) s += sX[r * p + i] * sR[i * p + j];
      dst[e] = s;
    }
  }
}

// The two passes on the stream; scratch is a device pointer of SCRATCH_DOUBLES doubles.
// Returns the flag of the second pass (read back after a synchronization).
gsi_status run_cholqr2(int64_t n, int p, double* X, double* scr, hipStream_t st) {
  const int nb = gram_blocks(n);
  double* partials = scr;
  double* rinv = scr + OFF_RINV;
  int* flags = reinterpret_cast<int*>(scr + OFF_FLAGS);
  for (int pass = 0; pass < 2; ++pass) {
    const int* fin = pass ? flags : nullptr;
    int* fout = flags + pass;
    hipLaunchKernelGGL(k_ortho_gram, dim3(nb), dim3(OWG), 0, st, n, p, X, partials, fin);
    hipLaunchKernelGGL(k_ortho_chol, dim3(1), dim3(OWG), 0, st, p, nb, partials, rinv, fin, fout);
    hipLaunchKernelGGL(k_ortho_apply, dim3(nb), dim3(OWG), 0, st, n, p, X, rinv, fout);
  }
  if (hipGetLastError() != hipSuccess) return GSI_EDEVICE;
  int flag = 0;
  if (hipMemcpyAsync(&flag, flags + 1, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) return GSI_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return GSI_EDEVICE;
  return flag ? GSI_BREAKDOWN : GSI_OK;
}

gsi_status check_args(const double* X, int64_t n, int32_t p) {
  if (!X || p < 1 || n < p) return GSI_EINVAL;
  if (p > OMAXP) return GSI_EUNSUPPORTED;
  return GSI_OK;
}

// Device address of `scratch` on each device, looked up once per device with that device
// current (each device holds its own copy of the array at its own address).
constexpr int MAXDEV = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAXDEV] = {nullptr};

gsi_status scratch_for_current_device(double** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAXDEV) return GSI_EDEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return GSI_EDEVICE;
    g_scratch_ptr[dev] = reinterpret_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return GSI_OK;
}

}  // namespace

extern "C" {

gsi_status gsi_orthonormalize(double* X, int64_t n, int32_t p, void* hip_stream) {
  gsi_status s = check_args(X, n, p);
  if (s != GSI_OK) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  void* scr = nullptr;
  if (hipMalloc(&scr, SCRATCH_DOUBLES * sizeof(double)) != hipSuccess) return GSI_ENOMEM;
  s = run_cholqr2(n, p, X, reinterpret_cast<double*>(scr), st);
  if (s == GSI_EDEVICE) (void)hipStreamSynchronize(st);
  (void)hipFree(scr);
  return s;
}

gsi_status gsi_orthonormalize_noalloc(double* X, int64_t n, int32_t p, void* hip_stream) {
  gsi_status s = check_args(X, n, p);
  if (s != GSI_OK) return s;
  double* scr = nullptr;
  s = scratch_for_current_device(&scr);
  if (s != GSI_OK) return s;
  return run_cholqr2(n, p, X, scr, reinterpret_cast<hipStream_t>(hip_stream));
}

}  // extern "C"
