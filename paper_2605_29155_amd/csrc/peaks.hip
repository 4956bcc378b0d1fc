// peaks.hip -- measured vector-FMA and copy rates of the GPU, the ceilings the
// roofline fractions of the layer's kernels are read against.
//
// fma32 / fma64: every lane runs `iters` rounds of eight independent FMA
// chains (a = a * b + c), enough independent work per wave that issue, not
// latency, sets the rate.  Packed FP32 is disabled in this build, so the FP32
// figure is the rate of single (unpacked) FP32 FMAs.
// copy: float4 loads and stores of n4 16-byte elements, bytes moved = 32 x n4.
#include <hip/hip_runtime.h>

#include <cstddef>

namespace {

template <class R>
__global__ __launch_bounds__(256) void k_fma(int iters, R* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  R a0 = (R)i * (R)1e-9, a1 = a0 + (R)1, a2 = a0 + (R)2, a3 = a0 + (R)3, a4 = a0 + (R)4, a5 = a0 + (R)5,
    a6 = a0 + (R)6, a7 = a0 + (R)7;
  const R b = (R)0.999999, c = (R)1e-7;
  for (int k = 0; k < iters; ++k) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a0 = a0 * b + c; a1 = a1 * b + c; a2 = a2 * b + c; a3 = a3 * b + c;
      a4 = a4 * b + c; a5 = a5 * b + c; a6 = a6 * b + c; a7 = a7 * b + c;
    }
  }
  out[i] = ((a0 + a1) + (a2 + a3)) + ((a4 + a5) + (a6 + a7));
}

__global__ __launch_bounds__(256) void k_copy(const float4* __restrict__ src, float4* __restrict__ dst, size_t n4) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" {

// FLOP per launch: 2 * 8 * 8 * iters * blocks * threads (the inner loop is unrolled eight times)
int peak_fma32(int blocks, int threads, int iters, float* out, void* stream) {
  if (threads < 1 || threads > 256) return -1;
  k_fma<float><<<blocks, threads, 0, (hipStream_t)stream>>>(iters, out);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int peak_fma64(int blocks, int threads, int iters, double* out, void* stream) {
  if (threads < 1 || threads > 256) return -1;
  k_fma<double><<<blocks, threads, 0, (hipStream_t)stream>>>(iters, out);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int peak_copy(const void* src, void* dst, size_t n4, int blocks, void* stream) {
  k_copy<<<blocks, 256, 0, (hipStream_t)stream>>>((const float4*)src, (float4*)dst, n4);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // extern "C"
