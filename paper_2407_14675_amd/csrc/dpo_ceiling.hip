// Machine ceilings measured on the device the library runs on: the
// denominators of the sweeps' rooflines next to the published peaks.
//   * a streaming copy and a streaming read of float4 rows (the HBM rate a
//     plain kernel reaches; four 16-byte loads in flight per thread);
//   * a plain FP32 FMA loop: eight independent chains of v_fma_f32 per lane
//     (packed FP32 forms are disabled in every build of this library), the
//     VALU issue rate of the ordinary instructions the sweeps are made of.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dpo_kernels.h"

namespace dpo {

namespace {

constexpr int kCeilBlock = 256;
constexpr int kCeilUnroll = 4;
constexpr int kFmaChains = 8;

__global__ __launch_bounds__(kCeilBlock) void k_ceil_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                                          int64_t n4) {
  const int64_t base = (int64_t)blockIdx.x * (kCeilBlock * kCeilUnroll) + threadIdx.x;
  float4 v[kCeilUnroll];
#pragma unroll
  for (int k = 0; k < kCeilUnroll; k++) {
    const int64_t i = base + (int64_t)k * kCeilBlock;
    if (i < n4) v[k] = src[i];
  }
#pragma unroll
  for (int k = 0; k < kCeilUnroll; k++) {
    const int64_t i = base + (int64_t)k * kCeilBlock;
    if (i < n4) dst[i] = v[k];
  }
}

__global__ __launch_bounds__(kCeilBlock) void k_ceil_read(const float4* __restrict__ src, int64_t n4,
                                                          float* __restrict__ sink) {
  const int64_t base = (int64_t)blockIdx.x * (kCeilBlock * kCeilUnroll) + threadIdx.x;
  float4 v[kCeilUnroll];
#pragma unroll
  for (int k = 0; k < kCeilUnroll; k++) {
    const int64_t i = base + (int64_t)k * kCeilBlock;
    v[k] = i < n4 ? src[i] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  float acc = 0.0f;
#pragma unroll
  for (int k = 0; k < kCeilUnroll; k++) acc += (v[k].x + v[k].y) + (v[k].z + v[k].w);
  // never true for the finite data the caller passes; keeps the loads live
  if (acc == -1.0e38f) sink[0] = acc;
}

__global__ __launch_bounds__(kCeilBlock) void k_ceil_fma(int iters, float a, float b, float* __restrict__ sink) {
  float x[kFmaChains];
#pragma unroll
  for (int k = 0; k < kFmaChains; k++) x[k] = (float)(threadIdx.x + k) * 1e-3f;
  for (int it = 0; it < iters; it++) {
#pragma unroll
    for (int k = 0; k < kFmaChains; k++) x[k] = fmaf(x[k], a, b);
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < kFmaChains; k++) s += x[k];
  if (s == -1.0e38f) sink[0] = s;
}

}  // namespace

hipError_t launch_ceil_copy(const float* src, float* dst, int64_t n, hipStream_t s) {
  const int64_t n4 = n / 4;
  const int64_t blocks = (n4 + kCeilBlock * kCeilUnroll - 1) / (kCeilBlock * kCeilUnroll);
  hipLaunchKernelGGL(k_ceil_copy, dim3((unsigned)blocks), dim3(kCeilBlock), 0, s,
                     reinterpret_cast<const float4*>(src), reinterpret_cast<float4*>(dst), n4);
  return hipGetLastError();
}

hipError_t launch_ceil_read(const float* src, int64_t n, float* sink, hipStream_t s) {
  const int64_t n4 = n / 4;
  const int64_t blocks = (n4 + kCeilBlock * kCeilUnroll - 1) / (kCeilBlock * kCeilUnroll);
  hipLaunchKernelGGL(k_ceil_read, dim3((unsigned)blocks), dim3(kCeilBlock), 0, s,
                     reinterpret_cast<const float4*>(src), n4, sink);
  return hipGetLastError();
}

hipError_t launch_ceil_fma(int blocks, int iters, float* sink, hipStream_t s) {
  hipLaunchKernelGGL(k_ceil_fma, dim3(blocks), dim3(kCeilBlock), 0, s, iters, 0.999999f, 1e-7f, sink);
  return hipGetLastError();
}

}  // namespace dpo
