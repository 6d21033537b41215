// Graph update: the fluid injection of the updating equation (Section 3.3).
//
// When P changes to P' after some rounds, the state (F, H) of the old solve
// becomes a state of the new one by adding d (P' - P) H to the fluid: then
// H + F = F_0 + d P' H holds again (Theorem 1 for P'), and continuing the
// D-iteration with P' from there converges to the solution of X = dP'X + F_0
// (Theorem 4), usually with far fewer diffusions than a fresh solve when the
// change is small.  The injected fluid mixes signs; the round kernel takes
// nodes on |F_i|.
#include <algorithm>
#include <cmath>

#include "internal.h"
#include "kernels.h"

namespace di {

namespace {

// delta += (P' - P) H restricted to the rows that differ: a node whose
// out-links (and weights) are the same in both graphs contributes nothing, so
// only the changed rows push, +H_i p'(j,i) to the new children and
// -H_i p(j,i) to the old ones (fp64 atomics; a change touches few rows).
__global__ __launch_bounds__(kBlock) void k_inject_rows(
    int64_t n, const int64_t* __restrict__ rp0, const int32_t* __restrict__ c0,
    const double* __restrict__ w0, const int64_t* __restrict__ rp1,
    const int32_t* __restrict__ c1, const double* __restrict__ w1,
    const double* __restrict__ H, double* __restrict__ delta) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const double h = H[i];
    if (h == 0.0) continue;
    const int64_t a0 = rp0[i], b0 = rp0[i + 1], a1 = rp1[i], b1 = rp1[i + 1];
    bool same = b0 - a0 == b1 - a1 && (w0 == nullptr) == (w1 == nullptr);
    for (int64_t k = 0; same && k < b0 - a0; ++k)
      same = c0[a0 + k] == c1[a1 + k] && (!w0 || w0[a0 + k] == w1[a1 + k]);
    if (same) continue;
    for (int64_t e = a1; e < b1; ++e)
      atomicAdd(&delta[c1[e]], h * (w1 ? w1[e] : 1.0 / (double)(b1 - a1)));
    for (int64_t e = a0; e < b0; ++e)
      atomicAdd(&delta[c0[e]], -h * (w0 ? w0[e] : 1.0 / (double)(b0 - a0)));
  }
}

// F_j += d delta_j, one rounding into the fluid type.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_inject_apply(int64_t n, double d,
                                                         const double* __restrict__ delta,
                                                         T* __restrict__ F) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += stride)
    if (delta[j] != 0.0) F[j] = (T)((double)F[j] + d * delta[j]);
}

template <typename T>
void inject(const Graph* g0, const Graph* g1, double d, T* F, const double* H, hipStream_t s) {
  const int64_t n = g1->n;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, 8192));
  // stream-ordered scratch: no device-wide synchronisation per update
  double* delta = nullptr;
  DI_HIP(hipMallocAsync(reinterpret_cast<void**>(&delta), n * 8, s));
  DI_HIP(hipMemsetAsync(delta, 0, n * 8, s));
  k_inject_rows<<<grid, kBlock, 0, s>>>(
      n, g0->row_ptr.as<int64_t>(), g0->col.as<int32_t>(),
      g0->weighted ? g0->w.as<double>() : nullptr, g1->row_ptr.as<int64_t>(),
      g1->col.as<int32_t>(), g1->weighted ? g1->w.as<double>() : nullptr, H, delta);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    k_inject_apply<T><<<grid, kBlock, 0, s>>>(n, d, delta, F);
    e = hipGetLastError();
  }
  (void)hipFreeAsync(delta, s);
  DI_HIP(e);
  // F is a device output: ready in stream order, no host wait
}

}  // namespace

}  // namespace di

using namespace di;

extern "C" di_status di_inject_update(const di_graph* g_old, const di_graph* g_new,
                                      int32_t precision, double d, void* F, const double* H,
                                      void* stream) {
  return guarded([&] {
    DI_REQUIRE(g_old != nullptr && g_new != nullptr, "graph is NULL");
    DI_REQUIRE(g_old->n == g_new->n, "the two graphs must have the same number of nodes");
    DI_REQUIRE(std::isfinite(d) && d >= 0.0 && d < 1.0, "d must satisfy 0 <= d < 1");
    DI_REQUIRE(F != nullptr && H != nullptr, "F and H must be device pointers");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (precision == DI_FP64)
      inject<double>(g_old, g_new, d, static_cast<double*>(F), H, s);
    else if (precision == DI_FP32_FLUID)
      inject<float>(g_old, g_new, d, static_cast<float*>(F), H, s);
    else
      DI_REQUIRE(false, "unknown precision");
  });
}
