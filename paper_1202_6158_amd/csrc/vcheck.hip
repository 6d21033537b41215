// Validation of a personalisation vector held in device memory: the checks a
// host vector gets (every entry finite and non-negative, sum within 1e-9 of
// one, so that V is a distribution as Section 2.1 requires), made by one
// reduction on the caller's stream into scratch of the caller's workspace and
// a read-back of two numbers (no allocation, no device-wide synchronisation).
#include <algorithm>
#include <cmath>
#include <string>

#include "internal.h"
#include "kernels.h"

namespace di {

namespace {

__global__ void k_vcheck_zero(double* out) {
  if (threadIdx.x < 2) out[threadIdx.x] = 0.0;
}

// out[0] += sum of the valid entries, out[1] += count of the invalid ones.
__global__ __launch_bounds__(kBlock) void k_vcheck(const double* __restrict__ v, int64_t n,
                                                   double* __restrict__ out) {
  __shared__ double s_red[kBlock / 64];
  double sum = 0.0, bad = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    const double x = v[i];
    if (isfinite(x) && x >= 0.0) sum += x;
    else bad += 1.0;
  }
  sum = block_sum(sum, s_red);
  bad = block_sum(bad, s_red);
  if (threadIdx.x == 0) {
    atomicAdd(&out[0], sum);
    atomicAdd(&out[1], bad);
  }
}

}  // namespace

void validate_device_vector(const double* v, int64_t n, const char* what, double* dscratch,
                            double* hscratch, hipStream_t s) {
  k_vcheck_zero<<<1, 64, 0, s>>>(dscratch);
  DI_HIP(hipGetLastError());
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, 1024));
  k_vcheck<<<grid, kBlock, 0, s>>>(v, n, dscratch);
  DI_HIP(hipGetLastError());
  DI_HIP(hipMemcpyAsync(hscratch, dscratch, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  DI_HIP(hipStreamSynchronize(s));
  const double h[2] = {hscratch[0], hscratch[1]};
  DI_REQUIRE(h[1] == 0.0, std::string(what) + " has a negative or non-finite entry");
  DI_REQUIRE(std::fabs(h[0] - 1.0) <= 1e-9, std::string(what) + " does not sum to 1");
}

}  // namespace di
