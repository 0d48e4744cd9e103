// lbm_probe.hip -- measurement aid of the library: a plain device copy.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lbm_kernels.h"

namespace lbm {

// ------------------------------------------------------------ copy probe
//
// A plain device-to-device copy of 16-byte vectors, one per thread per
// iteration of a grid-stride loop, on a grid of 1024-lane workgroups large
// enough to keep every CU's memory pipeline full: the HBM rate a pure stream
// reaches on this GPU, the practical ceiling next to the published peak.
typedef float __attribute__((ext_vector_type(4))) f32x4;

__global__ void __launch_bounds__(1024) k_copy(const f32x4 *__restrict__ a, f32x4 *__restrict__ b,
                                               int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(&a[i]), &b[i]);
}

hipError_t copy_rate(size_t bytes, int reps, double *gbs) {
  *gbs = 0;
  const int64_t n = (int64_t)(bytes / sizeof(f32x4));
  if (n <= 0 || reps <= 0) return hipErrorInvalidValue;
  f32x4 *a = nullptr, *b = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&a, (size_t)n * sizeof(f32x4));
  if (e == hipSuccess) e = hipMalloc(&b, (size_t)n * sizeof(f32x4));
  if (e == hipSuccess) e = hipMemset(a, 0, (size_t)n * sizeof(f32x4));
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const int64_t blocks = std::min<int64_t>((n + 1023) / 1024, 65536);
  for (int r = 0; r < 3 && e == hipSuccess; r++) {
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(1024), 0, nullptr, a, b, n);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
  for (int r = 0; r < reps && e == hipSuccess; r++) {
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(1024), 0, nullptr, a, b, n);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e == hipSuccess && ms > 0) *gbs = 2.0 * (double)n * sizeof(f32x4) * reps / (ms * 1e-3) / 1e9;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (a) (void)hipFree(a);
  if (b) (void)hipFree(b);
  return e;
}

}  // namespace lbm
