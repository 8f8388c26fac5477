// peaks.hip -- microbenchmarks of the arithmetic rates the roofline figures
// of bench.py are set against: FMA chains on the vector ALUs (FP64, FP32)
// and chains of matrix-core instructions (FP64 16x16x4, FP32 16x16x4, BF16
// 16x16x32 with FP32 accumulation).  Measurement support only: no part of the
// method runs here, and the library (libaenet_probe.so) is separate from the
// one behind include/aenet_gpu.h.
//
// Every function enqueues one launch of `blocks` blocks of 256 threads on
// `stream` (a hipStream_t, NULL = default) and returns 0, or the HIP error
// code of the launch.  `out` is a device buffer of at least blocks * 256
// elements of the function's type; it is written only in a branch whose
// condition the arithmetic never meets, which keeps the chains from being
// removed.  The flop count of one launch is returned through `flops`.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kThreads = 256;
constexpr int kChains = 8;  // independent accumulation chains per lane

template <typename T>
__global__ __launch_bounds__(kThreads) void k_fma(int64_t iters, T a, T b, T* out) {
  T x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = T(threadIdx.x + c) * T(1e-3);
  for (int64_t k = 0; k < iters; ++k) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = fma(x[c], a, b);
  }
  T s = T(0);
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  if (s == T(-7.25)) out[(size_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kAcc = 8;  // independent accumulators per wavefront

__global__ __launch_bounds__(kThreads) void k_mfma_f64(int64_t iters, double a, double* out) {
  v4d acc[kAcc];
#pragma unroll
  for (int c = 0; c < kAcc; ++c) acc[c] = v4d{0, 0, 0, 0};
  const double b = a * (double)(threadIdx.x & 7);
  for (int64_t k = 0; k < iters; ++k) {
#pragma unroll
    for (int c = 0; c < kAcc; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  }
  double s = 0;
#pragma unroll
  for (int c = 0; c < kAcc; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  if (s == -7.25) out[(size_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_mfma_f32(int64_t iters, float a, float* out) {
  v4f acc[kAcc];
#pragma unroll
  for (int c = 0; c < kAcc; ++c) acc[c] = v4f{0, 0, 0, 0};
  const float b = a * (float)(threadIdx.x & 7);
  for (int64_t k = 0; k < iters; ++k) {
#pragma unroll
    for (int c = 0; c < kAcc; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
  }
  float s = 0;
#pragma unroll
  for (int c = 0; c < kAcc; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  if (s == -7.25f) out[(size_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_mfma_bf16(int64_t iters, float a, float* out) {
  v4f acc[kAcc];
#pragma unroll
  for (int c = 0; c < kAcc; ++c) acc[c] = v4f{0, 0, 0, 0};
  v8bf x, y;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    x[t] = (__bf16)(a * (float)(t + 1));
    y[t] = (__bf16)(a * (float)((threadIdx.x + t) & 7));
  }
  for (int64_t k = 0; k < iters; ++k) {
#pragma unroll
    for (int c = 0; c < kAcc; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, acc[c], 0, 0, 0);
  }
  float s = 0;
#pragma unroll
  for (int c = 0; c < kAcc; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  if (s == -7.25f) out[(size_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

int done() {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : (int)e;
}

}  // namespace

extern "C" {

// FP64 / FP32 fused multiply-adds: 2 flops each, kChains per lane per iteration
int probe_fma_f64(int64_t iters, int blocks, double* out, double* flops, void* stream) {
  hipLaunchKernelGGL(k_fma<double>, dim3(blocks), dim3(kThreads), 0, (hipStream_t)stream, iters, 0.999999,
                     1e-6, out);
  *flops = 2.0 * kChains * (double)iters * blocks * kThreads;
  return done();
}

int probe_fma_f32(int64_t iters, int blocks, float* out, double* flops, void* stream) {
  hipLaunchKernelGGL(k_fma<float>, dim3(blocks), dim3(kThreads), 0, (hipStream_t)stream, iters, 0.999999f,
                     1e-6f, out);
  *flops = 2.0 * kChains * (double)iters * blocks * kThreads;
  return done();
}

// matrix-core chains: per wavefront and instruction 2 * 16 * 16 * K flops
// (K = 4 for FP64 and FP32, 32 for BF16), kAcc instructions per iteration
int probe_mfma_f64(int64_t iters, int blocks, double* out, double* flops, void* stream) {
  hipLaunchKernelGGL(k_mfma_f64, dim3(blocks), dim3(kThreads), 0, (hipStream_t)stream, iters, 1e-3, out);
  *flops = 2.0 * 16 * 16 * 4 * kAcc * (double)iters * blocks * (kThreads / 64);
  return done();
}

int probe_mfma_f32(int64_t iters, int blocks, float* out, double* flops, void* stream) {
  hipLaunchKernelGGL(k_mfma_f32, dim3(blocks), dim3(kThreads), 0, (hipStream_t)stream, iters, 1e-3f, out);
  *flops = 2.0 * 16 * 16 * 4 * kAcc * (double)iters * blocks * (kThreads / 64);
  return done();
}

int probe_mfma_bf16(int64_t iters, int blocks, float* out, double* flops, void* stream) {
  hipLaunchKernelGGL(k_mfma_bf16, dim3(blocks), dim3(kThreads), 0, (hipStream_t)stream, iters, 1e-3f, out);
  *flops = 2.0 * 16 * 16 * 32 * kAcc * (double)iters * blocks * (kThreads / 64);
  return done();
}

}  // extern "C"
