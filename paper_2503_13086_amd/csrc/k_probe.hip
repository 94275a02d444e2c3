// Measurement probes for gfx950: the achievable rates the rooflines divide by.
//
// k_probe_copy streams 16-byte vectors from one buffer to another with non-temporal
// loads and stores, one vector per thread in 256-thread workgroups: its bytes read +
// written per second is the HBM rate a streaming kernel reaches on this chip.  (Of
// the shapes measured on a 1 GiB copy, 64-1024 threads with 1-16 vectors each,
// with and without non-temporal hints, this one was fastest: 6.8-6.9 TB/s, against
// 4.5 TB/s for 512 threads with 8 vectors each and 5.3 TB/s for torch's copy.)  k_probe_fma runs eight independent chains of fp32 fused
// multiply-adds per thread with the build's code generation (packed fp32 off), so
// its rate is the fp32 FMA issue rate the raster kernels can reach.
#include "gs_internal.h"

namespace gsk {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int kCopyThreads = 256;
constexpr int kCopyVecsPerThread = 1;

__global__ __launch_bounds__(kCopyThreads) void k_probe_copy(const f4* __restrict__ src, f4* __restrict__ dst,
                                                              size_t n_vec) {
  const size_t base = (size_t)blockIdx.x * kCopyThreads * kCopyVecsPerThread + threadIdx.x;
  f4 v[kCopyVecsPerThread];
#pragma unroll
  for (int k = 0; k < kCopyVecsPerThread; ++k) {
    const size_t i = base + (size_t)k * kCopyThreads;
    if (i < n_vec) v[k] = __builtin_nontemporal_load(src + i);
  }
#pragma unroll
  for (int k = 0; k < kCopyVecsPerThread; ++k) {
    const size_t i = base + (size_t)k * kCopyThreads;
    if (i < n_vec) __builtin_nontemporal_store(v[k], dst + i);
  }
}

constexpr int kFmaChains = 8;

__global__ __launch_bounds__(256) void k_probe_fma(float* __restrict__ out, int iters, float a, float b) {
  float x[kFmaChains];
#pragma unroll
  for (int k = 0; k < kFmaChains; ++k) x[k] = (float)(threadIdx.x + k);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kFmaChains; ++k) x[k] = __fmaf_rn(x[k], a, b);
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < kFmaChains; ++k) s += x[k];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

hipError_t launch_probe_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
  const size_t n_vec = bytes / 16;
  if (n_vec == 0) return hipSuccess;
  const size_t per_block = (size_t)kCopyThreads * kCopyVecsPerThread;
  const size_t blocks = (n_vec + per_block - 1) / per_block;
  hipLaunchKernelGGL(k_probe_copy, dim3((unsigned)blocks), dim3(kCopyThreads), 0, s,
                     reinterpret_cast<const f4*>(src), reinterpret_cast<f4*>(dst), n_vec);
  return hipGetLastError();
}

hipError_t launch_probe_fma(float* out, int blocks, int iters, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  // a and b keep every chain finite: x -> 0.999 x + 0.001 stays in [0, max(x0, 1)]
  hipLaunchKernelGGL(k_probe_fma, dim3((unsigned)blocks), dim3(256), 0, s, out, iters, 0.999f, 0.001f);
  return hipGetLastError();
}

int64_t probe_fma_flops(int blocks, int iters) { return (int64_t)blocks * 256 * iters * kFmaChains * 2; }

}  // namespace gsk
