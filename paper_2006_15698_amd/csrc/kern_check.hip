// Accuracy check of the reciprocal and square root that the FP64 flux
// kernels use (stage_fp64.h): the same device functions applied to an array,
// so that a test can compare them with the correctly rounded operations.

#include "dg_internal.h"
#include "stage_fp64.h"

namespace {

__global__ void __launch_bounds__(256)
k_recip_root(const double* __restrict__ x, double* __restrict__ r, double* __restrict__ s, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double v = x[i];
    r[i] = dgdev::recip(v);
    s[i] = dgdev::root(v);
  }
}

}  // namespace

int dg_launch_recip_root(hipStream_t stream, const double* x, double* r, double* s, int64_t n) {
  const int64_t blocks64 = (n + 255) / 256;
  const unsigned grid = (unsigned)(blocks64 < 65536 ? (blocks64 > 0 ? blocks64 : 1) : 65536);
  hipLaunchKernelGGL(k_recip_root, dim3(grid), dim3(256), 0, stream, x, r, s, n);
  return (int)hipGetLastError();
}
