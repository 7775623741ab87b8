// Matrix-core peak microbenchmark for gfx950 (measurement only; not part of
// the (T) library).  Every wave issues long chains of independent MFMAs on
// register operands (no memory traffic inside the timed loop), so the
// measured rate is the matrix cores' issue limit at the clock the GPU holds
// under that load.  The (T) kernels' achieved rates are reported against
// both this measured peak and the published one.
//
//   kind 0: v_mfma_f64_16x16x4_f64      2 * 16 * 16 * 4  =  2048 flops
//   kind 1: v_mfma_f32_16x16x32_bf16    2 * 16 * 16 * 32 = 16384 flops
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kAcc = 8;   // independent accumulators per wave (hides the MFMA latency)

// Both kernels carry an occupancy bound of two work-groups a CU: without it
// the compiler kept the loop-carried accumulators in ordinary registers and
// copied all of them to and from the accumulation registers around every
// trip's MFMAs (128 copies and a wait per 8 MFMAs), which measured about 64%
// of the real float64 rate.  With the bound the loop is the MFMAs alone
// (checked in the generated assembly).

__global__ __launch_bounds__(256, 2) void k_peak_f64(double* out, int iters) {
  d4 acc[kAcc];
#pragma unroll
  for (int n = 0; n < kAcc; ++n) acc[n] = d4{0.0, 0.0, 0.0, 0.0};
  const double a = 1e-3 * double(threadIdx.x & 63);
  const double b = 1.0 + 1e-9 * double(blockIdx.x);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int n = 0; n < kAcc; ++n)
      acc[n] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[n], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int n = 0; n < kAcc; ++n) s += acc[n][0] + acc[n][1] + acc[n][2] + acc[n][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256, 2) void k_peak_bf16(float* out, int iters) {
  f4 acc[kAcc];
#pragma unroll
  for (int n = 0; n < kAcc; ++n) acc[n] = f4{0.f, 0.f, 0.f, 0.f};
  bf16x8 a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = __bf16(1e-3f * float((threadIdx.x + e) & 63));
    b[e] = __bf16(1.0f + 1e-2f * float(e));
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int n = 0; n < kAcc; ++n)
      acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[n], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int n = 0; n < kAcc; ++n) s += acc[n][0] + acc[n][1] + acc[n][2] + acc[n][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

extern "C" {

// Runs `kind` on the current device with `blocks` work-groups of 256 threads
// and `iters` loop trips (kAcc MFMAs each per wave), on a stream of its own,
// and writes the achieved TFLOP/s to *tflops.  The scratch output buffer
// (blocks * 256 values) is allocated and freed here.  Returns 0, or -1 for bad
// arguments, or the HIP error code.
int sie_mfma_peak(int kind, int iters, int blocks, double* tflops) {
  if (!tflops || iters < 1 || blocks < 1 || (kind != 0 && kind != 1)) return -1;
  void* out = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t err = hipMalloc(&out, size_t(blocks) * 256 * sizeof(double));
  if (err == hipSuccess) err = hipStreamCreate(&s);
  if (err == hipSuccess) err = hipEventCreate(&e0);
  if (err == hipSuccess) err = hipEventCreate(&e1);
  auto launch = [&](int it) {
    if (kind == 0)
      hipLaunchKernelGGL(k_peak_f64, dim3(blocks), dim3(256), 0, s, static_cast<double*>(out), it);
    else
      hipLaunchKernelGGL(k_peak_bf16, dim3(blocks), dim3(256), 0, s, static_cast<float*>(out), it);
  };
  if (err == hipSuccess) {
    // warm-up of the same length as the timed launch: the clocks take tens
    // of milliseconds of sustained load to settle (a short warm-up measured
    // 42 TFLOP/s float64 where a long one gives 50)
    launch(iters);
    err = hipGetLastError();
  }
  if (err == hipSuccess) err = hipEventRecord(e0, s);
  if (err == hipSuccess) {
    launch(iters);
    err = hipGetLastError();
  }
  if (err == hipSuccess) err = hipEventRecord(e1, s);
  if (err == hipSuccess) err = hipEventSynchronize(e1);
  float ms = 0.f;
  if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
  if (err == hipSuccess) {
    const double per = kind == 0 ? 2048.0 : 16384.0;
    const double flops = per * kAcc * double(iters) * 4.0 * double(blocks);   // 4 waves a group
    *tflops = flops / (double(ms) * 1e-3) / 1e12;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  if (out) (void)hipFree(out);
  return err == hipSuccess ? 0 : int(err);
}

}  // extern "C"
