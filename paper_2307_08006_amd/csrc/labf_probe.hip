// labf_probe.hip -- achievable-peak probes of the chip for roofline reporting:
// chains of FP32 and FP64 FMAs, a chain of FP32 reciprocal square roots, and a
// streaming triad.  Each compute probe runs 8 independent dependency chains
// per lane so that issue, not latency, bounds it; packed FP32 is disabled for
// the whole library, so the FP32 figure is the non-packed issue rate.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace labf {

constexpr int PROBE_CHAINS = 8;

template <typename F>
__global__ __launch_bounds__(256) void k_probe_fma(F *out, int iters, F a, F b) {
  F c[PROBE_CHAINS];
#pragma unroll
  for (int k = 0; k < PROBE_CHAINS; ++k) c[k] = (F)(threadIdx.x + k);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < PROBE_CHAINS; ++k) c[k] = fma(c[k], a, b);
  }
  F s = (F)0;
#pragma unroll
  for (int k = 0; k < PROBE_CHAINS; ++k) s += c[k];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_probe_rsq(float *out, int iters) {
  float c[PROBE_CHAINS];
#pragma unroll
  for (int k = 0; k < PROBE_CHAINS; ++k) c[k] = 1.0f + (float)(threadIdx.x + k);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < PROBE_CHAINS; ++k) c[k] = __builtin_amdgcn_rsqf(c[k]);  // stays in (0, inf)
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < PROBE_CHAINS; ++k) s += c[k];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_probe_triad(float4 *a, const float4 *b, const float4 *c, float s,
                                                     int64_t n4) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x) {
    const float4 x = b[i], y = c[i];
    a[i] = make_float4(x.x + s * y.x, x.y + s * y.y, x.z + s * y.z, x.w + s * y.w);
  }
}

hipError_t launch_probe(int kind, int64_t n, void *buf0, void *buf1, void *buf2, unsigned blocks,
                        hipStream_t s) {
  if (kind == 0) k_probe_fma<float><<<blocks, 256, 0, s>>>((float *)buf0, (int)n, 0.999999f, 1e-7f);
  else if (kind == 1) k_probe_fma<double><<<blocks, 256, 0, s>>>((double *)buf0, (int)n, 0.999999, 1e-7);
  else if (kind == 2) k_probe_rsq<<<blocks, 256, 0, s>>>((float *)buf0, (int)n);
  else k_probe_triad<<<blocks, 256, 0, s>>>((float4 *)buf0, (const float4 *)buf1, (const float4 *)buf2, 0.5f, n / 4);
  return hipGetLastError();
}

}  // namespace labf
