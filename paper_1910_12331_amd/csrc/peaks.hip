// Measured peaks of one MI355X for the roofline figures: HBM bandwidth of a streaming copy and
// the dense matrix-core rates of the MFMA instructions the kernels use. Not a step of the method;
// built into its own library (libcppeaks.so) and called only by the benchmark.
//
//   cpk_copy_gbs        a grid-stride 16-byte copy of n bytes (read n, write n): bytes moved
//                       per second, the usual stream-copy figure (2 n / t).
//   cpk_mfma_tflops     a register-only loop of one MFMA kind on every SIMD: 32 (FP64: 16)
//                       independent accumulators per wavefront, no memory traffic inside the
//                       loop. kind 0: 16x16x4 FP32, 1: 16x16x4 FP64,
//                       2: 16x16x32 bf16 (FP32 accumulation).
// Both time `reps` launches with HIP events on the default stream and return the rate of the
// mean launch; they return a negative value on a HIP error.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// U 16-byte loads in flight per thread per round, then U stores.
template <int U, bool NT>
__global__ __launch_bounds__(256) void k_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                              int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n16; i += U * stride) {
    u32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i + u * stride < n16)
        v[u] = NT ? __builtin_nontemporal_load(src + i + u * stride) : src[i + u * stride];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i + u * stride < n16) {
        if (NT) __builtin_nontemporal_store(v[u], dst + i + u * stride);
        else dst[i + u * stride] = v[u];
      }
  }
}

typedef float fv4 __attribute__((ext_vector_type(4)));
typedef double dv4 __attribute__((ext_vector_type(4)));
typedef __bf16 bv8 __attribute__((ext_vector_type(8)));

constexpr int KACC = 32;      // FP32 and bf16 accumulators per wavefront (128 registers)
constexpr int KACC64 = 16;    // FP64 accumulators (also 128 registers)

// Every wavefront runs `iters` rounds of KACC independent MFMAs; the accumulators are written
// out (by one lane) only so that the loop is not removed.
__global__ __launch_bounds__(256) void k_mfma_f32(float* out, int iters) {
  fv4 acc[KACC];
  const float a = 1.0f + threadIdx.x * 1e-7f, b = 1.0f - threadIdx.x * 1e-7f;
#pragma unroll
  for (int k = 0; k < KACC; ++k) acc[k] = fv4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int i = 0; i < iters; ++i)
#pragma unroll
    for (int k = 0; k < KACC; ++k) acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[k], 0, 0, 0);
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < KACC; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_mfma_f64(double* out, int iters) {
  dv4 acc[KACC64];
  const double a = 1.0 + threadIdx.x * 1e-12, b = 1.0 - threadIdx.x * 1e-12;
#pragma unroll
  for (int k = 0; k < KACC64; ++k) acc[k] = dv4{0.0, 0.0, 0.0, 0.0};
  for (int i = 0; i < iters; ++i)
#pragma unroll
    for (int k = 0; k < KACC64; ++k) acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[k], 0, 0, 0);
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < KACC64; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_mfma_bf16(float* out, int iters) {
  fv4 acc[KACC];
  bv8 a, b;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    a[j] = (__bf16)(1.0f + (threadIdx.x + j) * 1e-3f);
    b[j] = (__bf16)(1.0f - (threadIdx.x + j) * 1e-3f);
  }
#pragma unroll
  for (int k = 0; k < KACC; ++k) acc[k] = fv4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int i = 0; i < iters; ++i)
#pragma unroll
    for (int k = 0; k < KACC; ++k)
      acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[k], 0, 0, 0);
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < KACC; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

template <typename F>
double time_launches(F launch, int reps) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.0;
  launch();   // warm-up
  if (hipDeviceSynchronize() != hipSuccess) return -1.0;
  (void)hipEventRecord(e0, 0);
  for (int r = 0; r < reps; ++r) launch();
  (void)hipEventRecord(e1, 0);
  if (hipEventSynchronize(e1) != hipSuccess) return -1.0;
  float ms = 0.0f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (hipGetLastError() != hipSuccess) return -1.0;
  return ms * 1e-3 / reps;
}

}  // namespace

extern "C" {

// src, dst: device buffers of n bytes (n a multiple of 16, both 16-byte aligned). blocks:
// workgroups of 256 threads; variant: 0 = one load per thread and round, 1 = four, 2 = four
// with non-temporal loads and stores.
double cpk_copy_gbs(const void* src, void* dst, int64_t n, int reps, int blocks, int variant) {
  if (!src || !dst || n <= 0 || n % 16 || reps < 1 || blocks < 1) return -1.0;
  const int64_t n16 = n / 16;
  const u32x4* s = (const u32x4*)src;
  u32x4* d = (u32x4*)dst;
  const double t = time_launches([&] {
    if (variant == 0) hipLaunchKernelGGL((k_copy<1, false>), dim3(blocks), dim3(256), 0, 0, s, d, n16);
    else if (variant == 1) hipLaunchKernelGGL((k_copy<4, false>), dim3(blocks), dim3(256), 0, 0, s, d, n16);
    else hipLaunchKernelGGL((k_copy<4, true>), dim3(blocks), dim3(256), 0, 0, s, d, n16);
  }, reps);
  return t > 0.0 ? 2.0 * (double)n / t / 1e9 : -1.0;
}

// out: device buffer of at least `blocks` doubles. blocks: workgroups of `threads` threads (a
// multiple of 64, at most 256).
double cpk_mfma_tflops(int kind, void* out, int blocks, int threads, int iters, int reps) {
  if (!out || blocks < 1 || threads < 64 || threads > 256 || threads % 64 || iters < 1 || reps < 1)
    return -1.0;
  double flops_per_mfma;
  double t;
  switch (kind) {
    case 0:
      flops_per_mfma = 2.0 * 16 * 16 * 4;
      t = time_launches([&] {
        hipLaunchKernelGGL(k_mfma_f32, dim3(blocks), dim3(threads), 0, 0, (float*)out, iters);
      }, reps);
      break;
    case 1:
      flops_per_mfma = 2.0 * 16 * 16 * 4;
      t = time_launches([&] {
        hipLaunchKernelGGL(k_mfma_f64, dim3(blocks), dim3(threads), 0, 0, (double*)out, iters);
      }, reps);
      break;
    case 2:
      flops_per_mfma = 2.0 * 16 * 16 * 32;
      t = time_launches([&] {
        hipLaunchKernelGGL(k_mfma_bf16, dim3(blocks), dim3(threads), 0, 0, (float*)out, iters);
      }, reps);
      break;
    default:
      return -1.0;
  }
  if (t <= 0.0) return -1.0;
  const double mfmas = (double)blocks * (threads / 64) * iters * (kind == 1 ? KACC64 : KACC);
  return mfmas * flops_per_mfma / t / 1e12;
}

}  // extern "C"
