// Streaming reference kernels: the rates at which this GPU copies, reads and writes a
// large buffer with the access pattern of the solver's streaming passes (16 bytes per lane,
// grid-stride over contiguous memory). They fix the achievable ceiling that the solver's
// kernels are compared with, next to the published HBM peak.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gsi.h"
#include "gsi_device.h"

namespace gsi {
namespace {

// Grids as measured fastest for each kind on the 256-CU device: 16384 workgroups of 256
// threads for the copy and the write (non-temporal stores, as in the kernels whose outputs
// are not read again by the same launch), 2048 for the read-only pass
constexpr int SWG = 256;
constexpr int SGRID = 16384;
constexpr int SGRID_READ = 2048;

__global__ __launch_bounds__(SWG) void k_stream_copy(int64_t count, const d2* __restrict__ src, d2* __restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * SWG + threadIdx.x; i < count; i += (int64_t)SGRID * SWG)
    __builtin_nontemporal_store(gld(src + i), dst + i);
}

// The sum is stored only in the impossible case that it is NaN-free and equals a sentinel,
// which keeps the loads without a write per thread.
__global__ __launch_bounds__(SWG) void k_stream_read(int64_t count, const d2* __restrict__ src, double* __restrict__ sink) {
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * SWG + threadIdx.x; i < count; i += (int64_t)SGRID_READ * SWG) {
    const d2 v = gld(src + i);
    s += v.x + v.y;
  }
  if (s == 1.2345678901234567e300) gst(sink, s);
}

__global__ __launch_bounds__(SWG) void k_stream_write(int64_t count, d2* __restrict__ dst, double value) {
  const d2 v = {value, value};
  for (int64_t i = (int64_t)blockIdx.x * SWG + threadIdx.x; i < count; i += (int64_t)SGRID * SWG)
    __builtin_nontemporal_store(v, dst + i);
}

}  // namespace
}  // namespace gsi

using namespace gsi;

extern "C" gsi_status gsi_stream_rates(void* a, void* b, int64_t bytes, int32_t reps, double* us, void* stream) {
  if (!a || !b || !us || bytes < 16 || (bytes & 15) || reps < 1) return GSI_EINVAL;
  if ((reinterpret_cast<uintptr_t>(a) & 15) || (reinterpret_cast<uintptr_t>(b) & 15)) return GSI_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int64_t count = bytes / 16;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  // write first, then the copy (so that b ends equal to a), then the read
  const int order[3] = {2, 0, 1};
  for (int o = 0; o < 3 && e == hipSuccess; ++o) {
    const int kind = order[o];
    auto launch = [&] {
      if (kind == 0)
        k_stream_copy<<<SGRID, SWG, 0, st>>>(count, reinterpret_cast<const d2*>(a), reinterpret_cast<d2*>(b));
      else if (kind == 1)
        k_stream_read<<<SGRID_READ, SWG, 0, st>>>(count, reinterpret_cast<const d2*>(a), reinterpret_cast<double*>(b));
      else
        k_stream_write<<<SGRID, SWG, 0, st>>>(count, reinterpret_cast<d2*>(b), 1.0);
    };
    launch();  // untimed first launch
    e = hipEventRecord(e0, st);
    for (int r = 0; r < reps && e == hipSuccess; ++r) launch();
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess) us[kind] = 1e3 * (double)ms / reps;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return e == hipSuccess ? GSI_OK : GSI_EDEVICE;
}
