// Power-iteration comparator (MAT-ITER, Sections 2.1 and 4) on gfx950.
//
//   X_{n+1} = d P X_n + (1-d) V,  X_0 = 0,  stop when ||X_n - X_{n-1}||_1 < tol,
//
// without dangling completion; the result is normalised at the end (the
// renormalisation that replaces completion, Section 4.2).  Each product is a
// pull over in-links: row blocks of up to kPullRows rows / kPullNnz links stage
// the gathered source values in LDS (coalesced index reads), one thread then
// sums each row; a row with more in-links than a block holds is reduced by
// the whole workgroup.  The iterate is stored twice, as X and as X/outdeg (the
// value every out-link carries), so a link costs one gather.
//
// precision DI_FP64: fp64 iterate.  DI_FP32_FLUID: the delta form
//   F_0 = (1-d)V, F_{n+1} = d P F_n (fp32 gather), X_{n+1} = X_n + F_{n+1} (fp64),
// whose increments are the Jacobi fluid of the D-iteration.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>

#include <hip/hip_ext.h>

#include "kernels.h"

namespace di {

struct PowCtl {
  int done_at;   // -1 while running; else k: X_k met the stop rule
  int reason;    // 1 converged, 2 non-finite, 3 max iterations
  double res;    // ||X_k - X_{k-1}||_1 at the stop
  double sum;    // flush sum
  double pad[5];
  double acc[3][256];  // residual partials of products k (slot k % 3), spread over 256 slots
};

template <typename G>  // G: gathered type (double, or float for the delta form)
struct PowArgs {
  int64_t n;
  const int64_t* in_ptr;
  const int32_t* in_src;
  const double* in_w;
  const int32_t* deg;
  const int32_t* blk;
  const double* v;
  double d, tol;
  int64_t max_iter;
  double* x[2];  // iterate (fp64); the delta form accumulates into x[0]
  G* xs[2];      // value carried by each out-link
  PowCtl* ctl;
  int delta;
};

template <typename G>
__global__ __launch_bounds__(kBlock) void k_pow_init(PowArgs<G> a) {
  const double u = 1.0 / (double)a.n;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * kBlock) {
    if (a.delta) {
      // F_0 = (1-d)V is the first increment: X_1 = F_0.
      const double f = (1.0 - a.d) * (a.v ? a.v[i] : u);
      const int dg = a.deg[i];
      a.x[0][i] = f;
      a.xs[0][i] = (G)(dg > 0 ? (a.in_w ? f : f / dg) : 0.0);
    } else {
      a.x[0][i] = 0.0;
      a.xs[0][i] = (G)0;
    }
  }
  if (blockIdx.x == 0) {
    for (int k = threadIdx.x; k < 3 * 256; k += kBlock) (&a.ctl->acc[0][0])[k] = 0.0;
    if (threadIdx.x == 0) {
      a.ctl->done_at = -1;
      a.ctl->reason = 0;
      a.ctl->res = 0.0;
      a.ctl->sum = 0.0;
    }
  }
}

// Product k: X_{k+1} = d P X_k + (1-d) V (delta form: F_{k+1} = d P F_k,
// X += F_{k+1}).  Every workgroup first reduces the residual of product k-1
// from its 256 slots (same order everywhere, so all agree on the stop).
template <typename G, bool kWeighted>
__global__ __launch_bounds__(kBlock) void k_pull(PowArgs<G> a, int k) {
  PowCtl* ctl = a.ctl;
  if (__hip_atomic_load(&ctl->done_at, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= 0) return;
  __shared__ double s_val[kPullNnz];
  __shared__ double s_red[kBlock / 64];
  __shared__ int s_long[kPullRows];  // rows of this block summed by a wave
  __shared__ int s_nlong;
  if (k >= 1) {
    const double res = block_sum(ctl->acc[(k - 1) % 3][threadIdx.x], s_red);
    int reason = 0;
    if (!isfinite(res)) reason = 2;
    else if (res < a.tol) reason = 1;
    else if ((int64_t)k >= a.max_iter) reason = 3;
    if (reason) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->res = res;
        ctl->reason = reason;
        ctl->done_at = k;
      }
      return;
    }
  }
  if (blockIdx.x == 0) ctl->acc[(k + 1) % 3][threadIdx.x] = 0.0;  // for product k+1
  const int cur = k & 1, nxt = cur ^ 1;
  const G* __restrict__ xs = a.xs[cur];
  G* __restrict__ ys = a.xs[nxt];
  // Blocks are listed longest first so that hub rows start early.
  const int r0 = a.blk[2 * blockIdx.x], r1 = a.blk[2 * blockIdx.x + 1];
  const int64_t e0 = a.in_ptr[r0], e1 = a.in_ptr[r1];
  const double u = 1.0 / (double)a.n;
  double diff = 0.0;
  auto finish_row = [&](int r, double gathered) {
    const double base = a.delta ? 0.0 : (1.0 - a.d) * (a.v ? a.v[r] : u);
    const double y = base + a.d * gathered;  // X_{k+1} (or F_{k+1} in delta form)
    const int dg = a.deg[r];
    const double carry = dg > 0 ? (kWeighted ? y : y / dg) : 0.0;
    if (a.delta) {
      diff += fabs(y);
      a.x[0][r] += y;
    } else {
      diff += fabs(y - a.x[cur][r]);
      a.x[nxt][r] = y;
    }
    ys[r] = (G)carry;
  };
  // Gathers in groups of kGU independent loads per thread.
  auto gather = [&](int64_t e) {
    double t = (double)xs[a.in_src[e]];
    if (kWeighted) t *= a.in_w[e];
    return t;
  };
  constexpr int kGU = 4;
  constexpr int kGB = 8;         // gathers in flight per thread (row blocks)
  constexpr int kShortRow = 32;  // rows longer than this are summed by a wave
  if (r1 - r0 == 1 && e1 - e0 > kPullNnz) {
    double acc = 0.0;
    for (int64_t e00 = e0 + threadIdx.x; e00 < e1; e00 += kGU * kBlock) {
      int32_t src[kGU];
#pragma unroll
      for (int q = 0; q < kGU; ++q) {
        const int64_t e = e00 + (int64_t)q * kBlock;
        src[q] = e < e1 ? a.in_src[e] : -1;
      }
      // unconditional gathers (a slot past the end reads entry 0), so that
      // none waits for another: a load in a branch gets a wait of its own
      G g[kGU];
#pragma unroll
      for (int q = 0; q < kGU; ++q) g[q] = xs[max(src[q], 0)];
      double t[kGU];
#pragma unroll
      for (int q = 0; q < kGU; ++q) t[q] = src[q] >= 0 ? (double)g[q] : 0.0;
#pragma unroll
      for (int q = 0; q < kGU; ++q) {
        const int64_t e = e00 + (int64_t)q * kBlock;
        if (kWeighted && src[q] >= 0) t[q] *= a.in_w[e];
        acc += t[q];
      }
    }
    acc = block_sum(acc, s_red);
    if (threadIdx.x == 0) finish_row(r0, acc);
  } else {
    // this thread's row's in-link range, loaded beside the gathers
    const int r = r0 + threadIdx.x;
    int64_t rb = 0, rc = 0;
    if (r < r1) {
      rb = a.in_ptr[r] - e0;
      rc = a.in_ptr[r + 1] - e0;
    }
    for (int64_t e00 = e0 + threadIdx.x; e00 < e1; e00 += kGB * kBlock) {
      int32_t src[kGB];
#pragma unroll
      for (int q = 0; q < kGB; ++q) {
        const int64_t e = e00 + (int64_t)q * kBlock;
        src[q] = e < e1 ? a.in_src[e] : -1;
      }
      G g[kGB];  // unconditional gathers, as above
#pragma unroll
      for (int q = 0; q < kGB; ++q) g[q] = xs[max(src[q], 0)];
      double t[kGB];
#pragma unroll
      for (int q = 0; q < kGB; ++q) t[q] = src[q] >= 0 ? (double)g[q] : 0.0;
#pragma unroll
      for (int q = 0; q < kGB; ++q) {
        const int64_t e = e00 + (int64_t)q * kBlock;
        if (src[q] >= 0) s_val[e - e0] = kWeighted ? t[q] * a.in_w[e] : t[q];
      }
    }
    if (threadIdx.x == 0) s_nlong = 0;
    __syncthreads();
    // Short rows: summed by their own thread.  Longer ones are listed and
    // each summed by a whole wave, so that no thread walks a hub row alone.
    if (r < r1) {
      if (rc - rb <= kShortRow) {
        double acc = 0.0;
        for (int64_t q = rb; q < rc; ++q) acc += s_val[q];
        finish_row(r, acc);
      } else {
        s_long[atomicAdd(&s_nlong, 1)] = r;
      }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int k = wid; k < s_nlong; k += kBlock / 64) {
      const int rr = s_long[k];
      const int64_t b = a.in_ptr[rr] - e0, c = a.in_ptr[rr + 1] - e0;
      double acc = 0.0;
      for (int64_t q = b + lane; q < c; q += 64) acc += s_val[q];
      acc = wave_sum(acc);
      if (lane == 0) finish_row(rr, acc);
    }
  }
  (void)gather;
  diff = block_sum(diff, s_red);
  if (threadIdx.x == 0 && diff != 0.0) unsafeAtomicAdd(&ctl->acc[k % 3][blockIdx.x & 255], diff);
}

static_assert(kBlock == 256, "one residual slot per thread");

__global__ __launch_bounds__(kBlock) void k_pow_zero(double* __restrict__ slots) {
  slots[threadIdx.x] = 0.0;
}

__global__ __launch_bounds__(kBlock) void k_pow_sum(int64_t n, const double* __restrict__ x,
                                                    double* __restrict__ slots) {
  __shared__ double s_red[kBlock / 64];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    s += x[i];
  s = block_sum(s, s_red);
  if (threadIdx.x == 0) unsafeAtomicAdd(&slots[blockIdx.x & 255], s);
}

__global__ __launch_bounds__(kBlock) void k_pow_sum_reduce(double* __restrict__ slots, PowCtl* ctl) {
  __shared__ double s_red[kBlock / 64];
  const double s = block_sum(slots[threadIdx.x], s_red);
  if (threadIdx.x == 0) ctl->sum = s;
}

__global__ __launch_bounds__(kBlock) void k_pow_write(int64_t n, const double* __restrict__ x,
                                                      const PowCtl* ctl, int normalize,
                                                      double* __restrict__ out) {
  const double s = normalize ? ctl->sum : 1.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    out[i] = x[i] / s;
}

struct PowWorkspace {
  DevBuf x0, x1, xs0, xs1, v, out, ctl;
  PinnedBuf hctl;
};

// Device buffers of one power solve: the two iterates, the two per-link
// values, the control block; and a host copy of the control block.
struct PowBufs {
  double* x0;
  double* x1;
  void* xs0;
  void* xs1;
  PowCtl* ctl;
  PowCtl* hctl;
};

// Bytes a power solve of n nodes needs from its buffers (gathered type G).
template <typename G>
static int64_t pow_bytes(int64_t n) {
  auto up = [](int64_t b) { return (b + 255) / 256 * 256; };
  return 2 * up(n * 8) + 2 * up(n * (int64_t)sizeof(G)) + up((int64_t)sizeof(PowCtl));
}

// The product loop and the flush on the given buffers.  vdev: device V or
// NULL (uniform); out: device x or NULL.  timed: the solve's own time from
// HIP events (else from the host clock around the stream's completion) and,
// with DI_TIMING, per-launch events.
template <typename G>
static di_status power_run(Graph* g, const double* vdev, const di_opts* o, double* out,
                           di_stats* st, hipStream_t s, const PowBufs& b, bool timed) {
  const bool delta = std::is_same<G, float>::value;
  const int64_t n = g->n;
  const int64_t max_iter = o->max_rounds > 0 ? o->max_rounds : 1000000;
  PowArgs<G> a;
  memset(&a, 0, sizeof(a));
  a.n = n;
  a.in_ptr = g->in_ptr.as<int64_t>();
  a.in_src = g->in_src.as<int32_t>();
  a.in_w = g->weighted ? g->in_w.as<double>() : nullptr;
  a.deg = g->deg.as<int32_t>();
  a.blk = g->pull_blk.as<int32_t>();
  a.v = vdev;
  a.d = o->d;
  a.tol = o->tol;
  a.max_iter = max_iter;
  a.x[0] = b.x0;
  a.x[1] = b.x1;
  a.xs[0] = static_cast<G*>(b.xs0);
  a.xs[1] = static_cast<G*>(b.xs1);
  a.ctl = b.ctl;
  a.delta = delta ? 1 : 0;
  const int grid_n = (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, 2048));
  std::unique_ptr<EventTimer> timer;
  const auto t0 = std::chrono::steady_clock::now();
  if (timed) timer.reset(new EventTimer(s));
  k_pow_init<G><<<grid_n, kBlock, 0, s>>>(a);
  DI_HIP(hipGetLastError());
  PowCtl* h = b.hctl;
  LaunchTimer lt(s, timed && (o->flags & DI_TIMING) != 0);
  int k = 0;
  int chunk = 16;
  for (;;) {
    for (int i = 0; i < chunk; ++i, ++k) {
      if (lt.on) {
        hipEvent_t e0, e1;
        lt.next(&e0, &e1);
        if (g->weighted)
          hipExtLaunchKernelGGL(k_pull<G, true>, dim3((int)g->npull), dim3(kBlock), 0, s, e0, e1,
                                0, a, k);
        else
          hipExtLaunchKernelGGL(k_pull<G, false>, dim3((int)g->npull), dim3(kBlock), 0, s, e0,
                                e1, 0, a, k);
      } else if (g->weighted) {
        k_pull<G, true><<<(int)g->npull, kBlock, 0, s>>>(a, k);
      } else {
        k_pull<G, false><<<(int)g->npull, kBlock, 0, s>>>(a, k);
      }
      DI_HIP(hipGetLastError());
    }
    DI_HIP(hipMemcpyAsync(h, b.ctl, sizeof(PowCtl), hipMemcpyDeviceToHost, s));
    DI_HIP(hipStreamSynchronize(s));
    if (h->done_at >= 0) break;
    // ||X_k - X_{k-1}||_1 decays by about d per product: plan the rest.
    chunk = 16;
    if (o->d > 0 && o->d < 1) {
      double res = 0;
      for (int q = 0; q < 256; ++q) res += h->acc[(k - 1) % 3][q];
      if (res > 0 && res > o->tol)
        chunk = std::max(2, std::min(64, (int)std::ceil(std::log(o->tol / res) / std::log(o->d)) + 1));
    }
  }
  const int K = h->done_at;  // X_K is the answer
  const double* xr = delta ? a.x[0] : a.x[K & 1];
  double* slots = &a.ctl->acc[0][0];
  k_pow_zero<<<1, kBlock, 0, s>>>(slots);
  DI_HIP(hipGetLastError());
  k_pow_sum<<<grid_n, kBlock, 0, s>>>(n, xr, slots);
  DI_HIP(hipGetLastError());
  k_pow_sum_reduce<<<1, kBlock, 0, s>>>(slots, a.ctl);
  DI_HIP(hipGetLastError());
  if (out) {
    k_pow_write<<<grid_n, kBlock, 0, s>>>(n, xr, a.ctl, o->normalize, out);
    DI_HIP(hipGetLastError());
  }
  double secs;
  if (timer) {
    secs = timer->stop();
  } else {
    DI_HIP(hipStreamSynchronize(s));
    secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  DI_HIP(hipMemcpyAsync(h, b.ctl, sizeof(PowCtl), hipMemcpyDeviceToHost, s));
  DI_HIP(hipStreamSynchronize(s));
  if (st) {
    const double d = o->d, r = h->res, S = h->sum;
    st->residual_l1 = r;
    st->err_bound_l1 = o->normalize ? (S > 0 ? 2.0 * d * r / ((1.0 - d) * S) : 0.0) : d * r / (1.0 - d);
    st->mass_drift = 0.0;
    st->seconds = secs;
    st->rounds = K + (delta ? 1 : 0);
    st->nodes_diffused = (int64_t)K * n;
    st->edges_diffused = (int64_t)K * g->m;
    // launches 0..K-1 compute products; launch K only detects the stop.
    st->kernel_seconds = lt.on ? lt.total((size_t)K) : 0.0;
    st->kernel_launches = lt.on ? (int64_t)K : 0;
  }
  if (h->reason == 2) {
    set_error("non-finite residual");
    return DI_EDEVICE;
  }
  if (h->reason == 3) {
    set_error("max_rounds reached before ||X_n - X_n-1||_1 < tol");
    return DI_ENOTCONV;
  }
  return DI_OK;
}

template <typename G>
static di_status power_impl(Graph* g, const double* v, const di_opts* o, double* x,
                            di_stats* st, hipStream_t s) {
  const bool dev = (o->flags & DI_DEVICE_PTRS) != 0;
  const int64_t n = g->n;
  if (v && !dev) validate_vector(v, n, "v");
  PowWorkspace ws;
  ws.x0.alloc(n * 8);
  ws.x1.alloc(n * 8);
  ws.xs0.alloc(n * sizeof(G));
  ws.xs1.alloc(n * sizeof(G));
  ws.ctl.alloc(sizeof(PowCtl));
  ws.hctl.alloc(sizeof(PowCtl));
  // a device v: checked with the residual partials of the control block,
  // which k_pow_init clears afterwards
  if (v && dev)
    validate_device_vector(v, n, "v", &ws.ctl.as<PowCtl>()->acc[0][0],
                           &ws.hctl.as<PowCtl>()->acc[0][0], s);
  const double* vdev = nullptr;
  if (v) {
    if (dev) vdev = v;
    else {
      ws.v.alloc(n * 8);
      DI_HIP(hipMemcpyAsync(ws.v.p, v, n * 8, hipMemcpyHostToDevice, s));
      vdev = ws.v.as<double>();
    }
  }
  double* out = dev ? x : nullptr;
  if (x && !dev) {
    ws.out.alloc(n * 8);
    out = ws.out.as<double>();
  }
  const PowBufs b{ws.x0.as<double>(), ws.x1.as<double>(), ws.xs0.p, ws.xs1.p,
                  ws.ctl.as<PowCtl>(), ws.hctl.as<PowCtl>()};
  const di_status rc = power_run<G>(g, vdev, o, out, st, s, b, true);
  if (x && !dev) {
    DI_HIP(hipMemcpyAsync(x, out, n * 8, hipMemcpyDeviceToHost, s));
    DI_HIP(hipStreamSynchronize(s));
  }
  return rc;
}

// ------------------------------------------------ allocation-free variant

// Fixed scratch of di_power_solve_noalloc: each device that runs it holds one
// copy for the life of the process.  Host code never passes this name to a
// kernel or a copy (on the host it only stands for the symbol); it uses the
// device address that hipGetSymbolAddress returns for the current device.
__device__ __align__(256) unsigned char scratch[DI_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the scratch array on the current device (looked up once
// per device, with that device current).
static unsigned char* scratch_ptr() {
  int dev = 0;
  DI_HIP(hipGetDevice(&dev));
  DI_REQUIRE(dev >= 0 && dev < kMaxDevices, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    DI_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    DI_REQUIRE(p != nullptr, "scratch symbol has no device address");
    g_scratch_ptr[dev] = p;
  }
  return static_cast<unsigned char*>(g_scratch_ptr[dev]);
}

template <typename G>
static di_status power_noalloc_impl(Graph* g, const double* v, const di_opts* o, double* x,
                                    di_stats* st, hipStream_t s) {
  DI_REQUIRE((o->flags & DI_DEVICE_PTRS) != 0,
             "di_power_solve_noalloc takes device vectors only (set DI_DEVICE_PTRS)");
  DI_REQUIRE((o->flags & DI_TIMING) == 0, "di_power_solve_noalloc does not take DI_TIMING");
  int dev = 0;
  DI_HIP(hipGetDevice(&dev));
  DI_REQUIRE(dev == g->device, "the graph lives on another device than the current one");
  const int64_t n = g->n;
  DI_REQUIRE(pow_bytes<G>(n) <= (int64_t)DI_NOALLOC_SCRATCH_BYTES,
             "graph too large for the fixed scratch of di_power_solve_noalloc");
  unsigned char* p = scratch_ptr();
  auto up = [](int64_t b) { return (b + 255) / 256 * 256; };
  PowBufs b;
  b.x0 = reinterpret_cast<double*>(p);
  p += up(n * 8);
  b.x1 = reinterpret_cast<double*>(p);
  p += up(n * 8);
  b.xs0 = p;
  p += up(n * (int64_t)sizeof(G));
  b.xs1 = p;
  p += up(n * (int64_t)sizeof(G));
  b.ctl = reinterpret_cast<PowCtl*>(p);
  PowCtl hctl;  // host copy of the control block: on this thread's stack
  b.hctl = &hctl;
  if (v) validate_device_vector(v, n, "v", &b.ctl->acc[0][0], &hctl.acc[0][0], s);
  return power_run<G>(g, v, o, x, st, s, b, false);
}

}  // namespace di

using namespace di;

extern "C" di_status di_power_solve(const di_graph* gc, const double* v, const di_opts* opts,
                                    double* x, di_stats* stats, void* stream) {
  di_status rc = DI_OK;
  di_status g = guarded([&] {
    DI_REQUIRE(gc != nullptr, "graph is NULL");
    validate_d_tol(opts);
    Graph* g = const_cast<di_graph*>(gc);
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = opts->precision == DI_FP64 ? power_impl<double>(g, v, opts, x, stats, s)
                                    : power_impl<float>(g, v, opts, x, stats, s);
  });
  return g != DI_OK ? g : rc;
}

extern "C" di_status di_power_solve_noalloc(const di_graph* gc, const double* v,
                                            const di_opts* opts, double* x, di_stats* stats,
                                            void* stream) {
  di_status rc = DI_OK;
  di_status g = guarded([&] {
    DI_REQUIRE(gc != nullptr, "graph is NULL");
    validate_d_tol(opts);
    Graph* g = const_cast<di_graph*>(gc);
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = opts->precision == DI_FP64 ? power_noalloc_impl<double>(g, v, opts, x, stats, s)
                                    : power_noalloc_impl<float>(g, v, opts, x, stats, s);
  });
  return g != DI_OK ? g : rc;
}
