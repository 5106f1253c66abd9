// Roofline denominators measured on the device itself: a streaming copy
// (HBM bandwidth) and register-only matrix-instruction loops (int8 and FP64
// matrix throughput).  They carry none of the method's arithmetic; the
// benchmark divides each kernel's achieved rate by these and by the
// published figures.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/sadmm.h"

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

typedef unsigned int u4v __attribute__((ext_vector_type(4)));

// 16-byte grid-stride copy with non-temporal loads and stores (the data is
// streamed once); n16 = number of 16-byte words.
__global__ __launch_bounds__(256) void copy16_kernel(const u4v* __restrict__ src, u4v* __restrict__ dst,
                                                     int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n16; i += 4 * stride) {
    u4v v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
    for (int u = 0; u < 4; ++u) __builtin_nontemporal_store(v[u], dst + i + u * stride);
  }
  for (; i < n16; i += stride) dst[i] = src[i];
}

// 16-byte grid-stride read (XOR of the words, one result per thread).
__global__ __launch_bounds__(256) void read16_kernel(const u4v* __restrict__ src, unsigned* __restrict__ out,
                                                     int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned acc = 0u;
  for (; i + 3 * stride < n16; i += 4 * stride) {
    u4v v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = src[i + u * stride];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  for (; i < n16; i += stride) acc ^= src[i].x;
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

// Each wave issues iters x CH products of the given instruction on operands
// held in registers; one value per lane is stored so nothing is elided.
template <int CH>
__global__ __launch_bounds__(256) void mfma_i8_probe_kernel(int iters, int* __restrict__ sink) {
  const int t = threadIdx.x;
  const v4i a = {t, t * 3 + 1, t ^ 5, t + 7};
  const v4i b = {t * 5, t + 11, t ^ 9, 3 - t};
  v4i acc[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) acc[c] = v4i{c, 0, 0, 0};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < CH; ++c) acc[c] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, acc[c], 0, 0, 0);
  }
  int s = 0;
#pragma unroll
  for (int c = 0; c < CH; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  sink[(int64_t)blockIdx.x * blockDim.x + t] = s;
}

typedef int v16i __attribute__((ext_vector_type(16)));
template <int CH>
__global__ __launch_bounds__(256) void mfma_i8_32_probe_kernel(int iters, int* __restrict__ sink) {
  const int t = threadIdx.x;
  const v4i a = {t, t * 3 + 1, t ^ 5, t + 7};
  const v4i b = {t * 5, t + 11, t ^ 9, 3 - t};
  v16i acc[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) {
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[c][e] = e == 0 ? c : 0;
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < CH; ++c) acc[c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc[c], 0, 0, 0);
  }
  int s = 0;
#pragma unroll
  for (int c = 0; c < CH; ++c)
#pragma unroll
    for (int e = 0; e < 16; ++e) s += acc[c][e];
  sink[(int64_t)blockIdx.x * blockDim.x + t] = s;
}

template <int CH>
__global__ __launch_bounds__(256) void mfma_f64_probe_kernel(int iters, double* __restrict__ sink) {
  const int t = threadIdx.x;
  const double a = 1.0 + 1e-3 * t, b = 1.0 - 1e-3 * t;
  v4d acc[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) acc[c] = v4d{(double)c, 0.0, 0.0, 0.0};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < CH; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < CH; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  sink[(int64_t)blockIdx.x * blockDim.x + t] = s;
}

}  // namespace

extern "C" {

int sadmm_probe_bandwidth(int32_t kind, const void* src, void* dst, int64_t bytes, int32_t reps,
                          void* stream, double* ms) {
  if ((kind != 0 && kind != 1) || !src || !ms || bytes <= 0 || (bytes & 15) || reps < 1) return SADMM_E_ARG;
  if (kind == 0 && !dst) return SADMM_E_ARG;
  if ((reinterpret_cast<uintptr_t>(src) & 15) || (reinterpret_cast<uintptr_t>(dst) & 15)) return SADMM_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t n16 = bytes / 16;
  const int grid = 256 * 32;
  unsigned* sink = nullptr;
  if (kind == 1 && hipMalloc(&sink, sizeof(unsigned) * grid * 256) != hipSuccess) return SADMM_E_NOMEM;
  auto launch = [&]() {
    if (kind == 0)
      copy16_kernel<<<grid, 256, 0, s>>>(static_cast<const u4v*>(src), static_cast<u4v*>(dst), n16);
    else
      read16_kernel<<<grid, 256, 0, s>>>(static_cast<const u4v*>(src), sink, n16);
  };
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  launch();                                     // warm
  hipEventRecord(e0, s);
  for (int r = 0; r < reps; ++r) launch();
  hipEventRecord(e1, s);
  int rc = SADMM_OK;
  float f = 0.f;
  if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
      hipEventElapsedTime(&f, e0, e1) != hipSuccess)
    rc = SADMM_E_HIP;
  *ms = (double)f / reps;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (sink) hipFree(sink);
  return rc;
}

int sadmm_probe_mfma(int32_t kind, int32_t iters, void* stream, double* ops_per_s) {
  if (!ops_per_s || kind < 0 || kind > 2 || iters < 1) return SADMM_E_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return SADMM_E_HIP;
  // work-groups of 4 waves: 8 waves per SIMD for the 16 x 16 shapes, 4 for 32 x 32
  const int grid = ncu * (kind == 2 ? 4 : 8);
  constexpr int CH16 = 4, CH32 = 2;
  void* sink = nullptr;
  if (hipMalloc(&sink, (size_t)grid * 256 * 8) != hipSuccess) return SADMM_E_NOMEM;
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  auto launch = [&]() {
    if (kind == 0)
      mfma_i8_probe_kernel<CH16><<<grid, 256, 0, s>>>(iters, static_cast<int*>(sink));
    else if (kind == 1)
      mfma_f64_probe_kernel<CH16><<<grid, 256, 0, s>>>(iters, static_cast<double*>(sink));
    else
      mfma_i8_32_probe_kernel<CH32><<<grid, 256, 0, s>>>(iters, static_cast<int*>(sink));
  };
  launch();                                      // warm
  hipEventRecord(e0, s);
  launch();
  hipEventRecord(e1, s);
  int rc = SADMM_OK;
  float f = 0.f;
  if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
      hipEventElapsedTime(&f, e0, e1) != hipSuccess || f <= 0.f)
    rc = SADMM_E_HIP;
  // operations per instruction (multiply and add): int8 16x16x64 and 32x32x32 =
  // 32768 and 65536; FP64 16x16x4 = 2048
  const double per = kind == 0 ? 32768.0 : (kind == 1 ? 2048.0 : 65536.0);
  const double n_inst = (double)grid * 4 * iters * (kind == 2 ? CH32 : CH16);
  *ops_per_s = rc == SADMM_OK ? n_inst * per / (f * 1e-3) : 0.0;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipFree(sink);
  return rc;
}

}  // extern "C"
