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

#include "kernels.h"

namespace di {

namespace {

// F_j += d (sum over in-links i of j in P' of H_i p'(j,i) - the same in P),
// one thread per node, both sums in fp64 over the in-link lists (sorted by
// source, so an unchanged row cancels exactly), one rounding into F.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_inject(
    int64_t n, double d, const int64_t* __restrict__ ip1, const int32_t* __restrict__ is1,
    const double* __restrict__ iw1, const int32_t* __restrict__ deg1,
    const int64_t* __restrict__ ip0, const int32_t* __restrict__ is0,
    const double* __restrict__ iw0, const int32_t* __restrict__ deg0,
    const double* __restrict__ H, T* __restrict__ F) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += stride) {
    double s1 = 0.0, s0 = 0.0;
    for (int64_t e = ip1[j]; e < ip1[j + 1]; ++e) {
      const int32_t i = is1[e];
      s1 += H[i] * (iw1 ? iw1[e] : 1.0 / (double)deg1[i]);
    }
    for (int64_t e = ip0[j]; e < ip0[j + 1]; ++e) {
      const int32_t i = is0[e];
      s0 += H[i] * (iw0 ? iw0[e] : 1.0 / (double)deg0[i]);
    }
    if (s1 != s0) F[j] = (T)((double)F[j] + d * (s1 - s0));
  }
}

template <typename T>
void inject(const Graph* g0, const Graph* g1, double d, T* F, const double* H, hipStream_t s) {
  const int64_t n = g1->n;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, 8192));
  k_inject<T><<<grid, kBlock, 0, s>>>(
      n, d, g1->in_ptr.as<int64_t>(), g1->in_src.as<int32_t>(),
      g1->weighted ? g1->in_w.as<double>() : nullptr, g1->deg.as<int32_t>(),
      g0->in_ptr.as<int64_t>(), g0->in_src.as<int32_t>(),
      g0->weighted ? g0->in_w.as<double>() : nullptr, g0->deg.as<int32_t>(), H, F);
  DI_HIP(hipGetLastError());
  DI_HIP(hipStreamSynchronize(s));
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
