// Validation of a personalisation vector held in device memory: the checks a
// host vector gets (every entry finite and non-negative, sum within 1e-9 of
// one, so that V is a distribution as Section 2.1 requires), made by two
// small reductions on the caller's stream into scratch of the caller's
// workspace and a read-back of two numbers (no allocation, no atomics, no
// device-wide synchronisation).
#include <algorithm>
#include <cmath>
#include <string>

#include "internal.h"
#include "kernels.h"

namespace di {

namespace {

constexpr int kCheckBlocks = 256;  // partial-sum slots; the grid never exceeds it

// Block b writes (sum of the valid entries, count of the invalid ones) of its
// grid-stride share to part[2b], part[2b+1]; four independent loads per step.
__global__ __launch_bounds__(kBlock) void k_vcheck(const double* __restrict__ v, int64_t n,
                                                   double* __restrict__ part) {
  __shared__ double s_red[kBlock / 64];
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  double sum = 0.0, bad = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += 4 * stride) {
    double x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = i + u * stride < n ? v[i + u * stride] : 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (isfinite(x[u]) && x[u] >= 0.0) sum += x[u];
      else bad += 1.0;
    }
  }
  sum = block_sum(sum, s_red);
  bad = block_sum(bad, s_red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sum;
    part[2 * blockIdx.x + 1] = bad;
  }
}

// One block: out[0..1] = the sums of the nblk partial pairs (fixed order).
__global__ __launch_bounds__(kBlock) void k_vcheck_final(const double* __restrict__ part,
                                                         int nblk, double* __restrict__ out) {
  __shared__ double s_red[kBlock / 64];
  const int t = threadIdx.x;
  const double sum = block_sum(t < nblk ? part[2 * t] : 0.0, s_red);
  const double bad = block_sum(t < nblk ? part[2 * t + 1] : 0.0, s_red);
  if (t == 0) {
    out[0] = sum;
    out[1] = bad;
  }
}

}  // namespace

void validate_device_vector(const double* v, int64_t n, const char* what, double* dscratch,
                            double* hscratch, hipStream_t s) {
  static_assert(kCheckBlocks <= kBlock, "the final reduction takes one pair per thread");
  static_assert(2 * kCheckBlocks + 2 <= kFlushAcc, "a solve lends its flush scratch");
  const int grid = (int)std::max<int64_t>(
      1, std::min<int64_t>((n + 4 * kBlock - 1) / (4 * kBlock), kCheckBlocks));
  double* const out = dscratch + 2 * kCheckBlocks;
  k_vcheck<<<grid, kBlock, 0, s>>>(v, n, dscratch);
  DI_HIP(hipGetLastError());
  k_vcheck_final<<<1, kBlock, 0, s>>>(dscratch, grid, out);
  DI_HIP(hipGetLastError());
  DI_HIP(hipMemcpyAsync(hscratch, out, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  DI_HIP(hipStreamSynchronize(s));
  const double h[2] = {hscratch[0], hscratch[1]};
  DI_REQUIRE(h[1] == 0.0, std::string(what) + " has a negative or non-finite entry");
  DI_REQUIRE(std::fabs(h[0] - 1.0) <= 1e-9, std::string(what) + " does not sum to 1");
}

}  // namespace di
