// Rate the FP64 vector pipes sustain at the running clock: every lane runs
// independent chains of fused multiply-adds, enough of them per wave to cover
// the FMA latency, so the launch is bound by FP64 issue alone.  The roofline
// of the flux kernels is quoted against the published peak; this measured
// rate is reported beside it.
#include <hip/hip_runtime.h>

#include "../../include/acat.h"

namespace {

constexpr int FMA_THREADS = 256;
constexpr int FMA_CHAINS = 16;

__global__ __launch_bounds__(FMA_THREADS) void k_fma_chains(double* out, int32_t iters, double b, double c) {
  double a[FMA_CHAINS];
#pragma unroll
  for (int k = 0; k < FMA_CHAINS; ++k) a[k] = 1.0 + 1e-3 * k + 1e-9 * threadIdx.x;
  for (int32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < FMA_CHAINS; ++k) a[k] = fma(a[k], b, c);
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < FMA_CHAINS; ++k) s += a[k];
  out[(int64_t)blockIdx.x * FMA_THREADS + threadIdx.x] = s;
}

}  // namespace

extern "C" acat_status acat_fp64_fma_rate(int32_t blocks, int32_t iters, double* out, int64_t out_len,
                                          void* stream) {
  if (!out) return ACAT_ERR_NULL;
  if (blocks < 1 || blocks > (1 << 20) || iters < 1 || out_len < (int64_t)blocks * FMA_THREADS)
    return ACAT_ERR_ARG;
  k_fma_chains<<<blocks, FMA_THREADS, 0, static_cast<hipStream_t>(stream)>>>(out, iters, 0.999999, 1e-7);
  return hipGetLastError() == hipSuccess ? ACAT_OK : ACAT_ERR_DEVICE;
}
