// FP64 fused multiply-add loop: the measured ceiling of the vector FP64 units
// (declared in gvof_probe.h).
#include <hip/hip_runtime.h>

#include "gvof_probe.h"

namespace {

constexpr int kProbeThreads = 256;

// Eight independent chains per thread, so a wavefront always has an FMA ready
// to issue; a and b arrive at run time, so nothing folds.
__global__ __launch_bounds__(kProbeThreads) void k_probe_fma(double* __restrict__ out, int iters, double a,
                                                             double b) {
  const int t = blockIdx.x * kProbeThreads + threadIdx.x;
  const double s = (double)(t % 7);
  double x0 = s, x1 = s + 1.0, x2 = s + 2.0, x3 = s + 3.0, x4 = s + 4.0, x5 = s + 5.0, x6 = s + 6.0, x7 = s + 7.0;
#pragma unroll 4
  for (int i = 0; i < iters; ++i) {
    x0 = fma(x0, a, b);
    x1 = fma(x1, a, b);
    x2 = fma(x2, a, b);
    x3 = fma(x3, a, b);
    x4 = fma(x4, a, b);
    x5 = fma(x5, a, b);
    x6 = fma(x6, a, b);
    x7 = fma(x7, a, b);
  }
  out[t] = ((x0 + x1) + (x2 + x3)) + ((x4 + x5) + (x6 + x7));
}

}  // namespace

extern "C" int gvof_probe_fp64_fma(double* out, int32_t blocks, int32_t iters, double a, double b, void* stream) {
  if (!out || blocks < 1 || iters < 0) return -1;
  k_probe_fma<<<blocks, kProbeThreads, 0, (hipStream_t)stream>>>(out, iters, a, b);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}
