// Graph update: the fluid injection of the updating equation (Section 3.2).
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
// Each block takes kBlock consecutive rows and compares the links of those
// with equal degree as one concatenated range (consecutive threads read
// consecutive links), flagging in LDS the rows where a link or weight differs;
// the pushes of the flagged rows are then spread over the block the same way,
// so a changed hub row does not serialise on one thread.
__global__ __launch_bounds__(kBlock) void k_inject_rows(
    int64_t n, const int64_t* __restrict__ rp0, const int32_t* __restrict__ c0,
    const double* __restrict__ w0, const int64_t* __restrict__ rp1,
    const int32_t* __restrict__ c1, const double* __restrict__ w1,
    const double* __restrict__ H, double* __restrict__ delta) {
  __shared__ long long s_off[kBlock];  // exclusive prefix of the links each row compares
  __shared__ long long s_a0[kBlock], s_a1[kBlock];
  __shared__ int s_diff[kBlock];
  __shared__ double s_h[kBlock];
  __shared__ long long s_n1[kBlock];  // new out-degree of a flagged row
  __shared__ long long s_scr[kBlock / 64];
  const int t = threadIdx.x;
  const bool same_kind = (w0 == nullptr) == (w1 == nullptr);
  for (int64_t r0 = (int64_t)blockIdx.x * kBlock; r0 < n; r0 += (int64_t)gridDim.x * kBlock) {
    const int64_t r = r0 + t;
    double h = 0.0;
    int64_t a0 = 0, b0 = 0, a1 = 0, b1 = 0;
    int diff = 0;
    long long len = 0;
    if (r < n) {
      h = H[r];
      a0 = rp0[r];
      b0 = rp0[r + 1];
      a1 = rp1[r];
      b1 = rp1[r + 1];
      if (h != 0.0) {  // a row with no history pushes nothing either way
        if (b0 - a0 != b1 - a1 || !same_kind) diff = 1;
        else len = b0 - a0;
      }
    }
    long long total = 0;
    const long long off = block_exscan<kBlock>(len, s_scr, &total);
    s_off[t] = off;
    s_a0[t] = a0;
    s_a1[t] = a1;
    s_diff[t] = diff;
    __syncthreads();
    for (long long q = t; q < total; q += kBlock) {
      // the row of comparison q: the last j with s_off[j] <= q (it has links)
      int lo = 0, hi = kBlock - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_off[mid] <= q) lo = mid;
        else hi = mid - 1;
      }
      const long long k = q - s_off[lo];
      const int64_t e0 = s_a0[lo] + k, e1 = s_a1[lo] + k;
      if (c0[e0] != c1[e1] || (w0 && w0[e0] != w1[e1])) s_diff[lo] = 1;
    }
    __syncthreads();
    // pushes of the flagged rows: new links first (+), then old links (-)
    const long long plen = (r < n && h != 0.0 && s_diff[t]) ? (b1 - a1) + (b0 - a0) : 0;
    long long ptotal = 0;
    const long long poff = block_exscan<kBlock>(plen, s_scr, &ptotal);
    s_off[t] = poff;
    s_h[t] = h;
    s_n1[t] = b1 - a1;
    s_a0[t] = a0;
    s_a1[t] = a1;
    s_diff[t] = (int)(b0 - a0);  // now: old out-degree
    __syncthreads();
    for (long long q = t; q < ptotal; q += kBlock) {
      int lo = 0, hi = kBlock - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_off[mid] <= q) lo = mid;
        else hi = mid - 1;
      }
      const long long k = q - s_off[lo], n1 = s_n1[lo];
      if (k < n1) {
        const int64_t e = s_a1[lo] + k;
        unsafeAtomicAdd(&delta[c1[e]], s_h[lo] * (w1 ? w1[e] : 1.0 / (double)n1));
      } else {
        const int64_t e = s_a0[lo] + (k - n1);
        unsafeAtomicAdd(&delta[c0[e]], -s_h[lo] * (w0 ? w0[e] : 1.0 / (double)s_diff[lo]));
      }
    }
    __syncthreads();  // the LDS arrays are reused by the next rows
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
