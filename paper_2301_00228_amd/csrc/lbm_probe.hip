// lbm_probe.hip -- measurement aids of the library: plain device copies.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/lbm.h"
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

// ------------------------------------------------------ layout copy probe
//
// A plain copy with the array structure of one storage's state: each state
// array (2 fields x the storage's population slots, and the four arrays of u
// and du/dt, at their storage widths) copied to an array of its own, by
// 256-lane workgroups that each march 256 columns x 16 rows of 8192-node
// rows, loading row r + 1 before storing row r -- the interior march's
// access pattern without its arithmetic, halo or LDS exchange.  A copy of
// many arrays at once reaches less than a single-stream copy, so this rate,
// not k_copy's, is the ceiling that the layout sets for one pass over the
// state.
constexpr int kLcRow = 8192, kLcRows = 16, kLcLanes = 256;
constexpr int kLcMaxArrays = 14;
struct LcPtrs {
  const void *in[kLcMaxArrays];
  void *out[kLcMaxArrays];
};

template <class TP, int NP, class TU>
__global__ void __launch_bounds__(kLcLanes) k_layout_copy(LcPtrs p) {
  constexpr int strips = kLcRow / kLcLanes;
  const int tx = (int)blockIdx.x % strips, ty = (int)blockIdx.x / strips;
  const int64_t k0 = (int64_t)ty * kLcRows * kLcRow + tx * kLcLanes + (int)threadIdx.x;
  TP a[NP], na[NP];
  TU b[4], nb[4];
#pragma unroll
  for (int q = 0; q < NP; q++) a[q] = static_cast<const TP *>(p.in[q])[k0];
#pragma unroll
  for (int q = 0; q < 4; q++) b[q] = static_cast<const TU *>(p.in[NP + q])[k0];
  for (int r = 0; r < kLcRows; r++) {
    const int64_t k = k0 + (int64_t)r * kLcRow;
    if (r + 1 < kLcRows) {
#pragma unroll
      for (int q = 0; q < NP; q++) na[q] = static_cast<const TP *>(p.in[q])[k + kLcRow];
#pragma unroll
      for (int q = 0; q < 4; q++) nb[q] = static_cast<const TU *>(p.in[NP + q])[k + kLcRow];
    }
#pragma unroll
    for (int q = 0; q < NP; q++) static_cast<TP *>(p.out[q])[k] = a[q];
#pragma unroll
    for (int q = 0; q < 4; q++) static_cast<TU *>(p.out[NP + q])[k] = b[q];
#pragma unroll
    for (int q = 0; q < NP; q++) a[q] = na[q];
#pragma unroll
    for (int q = 0; q < 4; q++) b[q] = nb[q];
  }
}

template <class TP, int NP, class TU>
static hipError_t layout_copy_t(int64_t nodes, int reps, double *gbs) {
  constexpr int64_t block_nodes = (int64_t)kLcRow * kLcRows;
  const int64_t n = (nodes + block_nodes - 1) / block_nodes * block_nodes;
  const size_t bp = (size_t)n * sizeof(TP), bu = (size_t)n * sizeof(TU);
  LcPtrs p{};
  hipError_t e = hipSuccess;
  for (int q = 0; q < NP + 4 && e == hipSuccess; q++) {
    const size_t bytes = q < NP ? bp : bu;
    void *a = nullptr, *b = nullptr;
    e = hipMalloc(&a, bytes);
    p.in[q] = a;
    if (e == hipSuccess) e = hipMalloc(&b, bytes);
    p.out[q] = b;
    if (e == hipSuccess) e = hipMemset(a, 0, bytes);
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const dim3 grid((unsigned)(n / (kLcLanes * kLcRows)));
  for (int r = 0; r < 2 && e == hipSuccess; r++) {
    hipLaunchKernelGGL((k_layout_copy<TP, NP, TU>), grid, dim3(kLcLanes), 0, nullptr, p);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
  for (int r = 0; r < reps && e == hipSuccess; r++) {
    hipLaunchKernelGGL((k_layout_copy<TP, NP, TU>), grid, dim3(kLcLanes), 0, nullptr, p);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e == hipSuccess && ms > 0)
    *gbs = 2.0 * (double)(NP * bp + 4 * bu) * reps / (ms * 1e-3) / 1e9;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  for (int q = 0; q < kLcMaxArrays; q++) {
    if (p.in[q]) (void)hipFree(const_cast<void *>(p.in[q]));
    if (p.out[q]) (void)hipFree(p.out[q]);
  }
  return e;
}

hipError_t layout_copy_rate(int storage, int64_t nodes, int reps, double *gbs) {
  *gbs = 0;
  if (nodes <= 0 || reps <= 0) return hipErrorInvalidValue;
  switch (storage) {
    case LBM_STORE_F64: return layout_copy_t<double, 10, double>(nodes, reps, gbs);
    case LBM_STORE_F32: return layout_copy_t<float, 10, float>(nodes, reps, gbs);
    case LBM_STORE_F32DEV: return layout_copy_t<float, 10, double>(nodes, reps, gbs);
    case LBM_STORE_F16DEV:
    case LBM_STORE_BF16DEV: return layout_copy_t<uint32_t, 8, double>(nodes, reps, gbs);
  }
  return hipErrorInvalidValue;
}

}  // namespace lbm
