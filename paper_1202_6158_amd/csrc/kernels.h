// Device-side building blocks shared by the D-iteration kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace di {

// Scatter record: a push of `val` to node (window base + loc).
template <typename T>
struct PairT;
template <>
struct alignas(8) PairT<float> {
  uint32_t loc;
  float val;
};
template <>
struct alignas(16) PairT<double> {
  uint32_t loc;
  uint32_t pad;
  double val;
};

// Round sums, accumulated by the windows' workgroups into kSlots slots
// (window b adds into slot b % kSlots, so each address sees few atomics) and
// reduced by every workgroup of the next round.  Fields: fluid held before
// the take (the stopping residual), fluid taken from non-dangling nodes,
// fluid taken from dangling nodes, score sum over nodes holding fluid, nodes
// holding fluid, nodes taken, out-links pushed; and the largest untaken score
// (bits of a non-negative double, combined with an unsigned max).
constexpr int kSlots = 64;
constexpr int kSums = 7;
struct alignas(64) Slot {
  double sum[kSums];
  unsigned long long mrem;
};

constexpr int kFlushSums = 5;       // sums the flush takes per vector
constexpr int kFlushSlots = 256;    // partial-sum slots per flush sum
constexpr int kFlushAcc = kFlushSums * kFlushSlots;

// Control block in device memory.  Each field but bar is written by
// workgroup 0 of one launch (one round) and read only by later ones.
struct Ctl {
  int stop_round;  // -1 while running; else the last round whose set was taken
  int reason;      // 1 converged, 2 non-finite residual, 3 max rounds
  int err;         // capacity / range violation (never set on valid input); 4: barrier time-out
  unsigned bar;    // grid barrier arrivals of the one-launch solve
  double nf;       // ||F||_1 seen by the stopping round, before its take
  double theta;    // threshold of the latest round
  long long nodes_total, edges_total;  // diffusions and out-links used
  long long last_taken, last_edges;    // of the latest round
  // flush sums: sum(H+F), sum(H), sum|F|, sum over dangling of H, sum(F)
  double fl[kFlushSums];
};

// Workgroup barrier.  L (LDS only): orders the LDS accesses of the
// workgroup without waiting for the waves' outstanding global stores, for
// barriers that publish nothing through global memory inside the workgroup.
template <bool L = false>
__device__ __forceinline__ void wg_barrier() {
  if constexpr (L) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  } else {
    __syncthreads();
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Block-wide sum / max over NT threads (fixed order: deterministic); every
// thread gets the result.  scratch holds NT/64 entries.
template <int NT = kBlock>
__device__ __forceinline__ double block_sum(double v, double* scratch) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) t += scratch[i];
  return t;
}
template <int NT = kBlock>
__device__ __forceinline__ double block_max(double v, double* scratch) {
  v = wave_max(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double t = scratch[0];
#pragma unroll
  for (int i = 1; i < NT / 64; ++i) t = fmax(t, scratch[i]);
  return t;
}

// Sums K values (and one max) across the block in one LDS round trip;
// scratch holds (K+1) * NT/64 doubles.  Fixed order: deterministic.
template <int NT, int K>
constexpr int block_reduce_k_scratch() { return (K + 1) * (NT / 64 + 1); }

// Block sums of K doubles and the block max of one more, returned to every
// thread in a fixed order (deterministic).  Up to 512 threads every thread
// adds the per-wave partials itself; larger blocks let wave 0 reduce them
// (one partial per lane), so the registers used do not grow with the block.
// scratch: block_reduce_k_scratch<NT, K>() doubles.
template <int NT, int K, bool L = false>
__device__ __forceinline__ void block_reduce_k(double (&v)[K], double& mx, double* scratch) {
  constexpr int NW = NT / 64;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  mx = wave_max(mx);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  wg_barrier<L>();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) scratch[k * NW + wid] = v[k];
    scratch[K * NW + wid] = mx;
  }
  wg_barrier<L>();
  if constexpr (NW <= 8) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double t = 0.0;
#pragma unroll
      for (int i = 0; i < NW; ++i) t += scratch[k * NW + i];
      v[k] = t;
    }
    double m = scratch[K * NW];
#pragma unroll
    for (int i = 1; i < NW; ++i) m = fmax(m, scratch[K * NW + i]);
    mx = m;
  } else {
    double* out = scratch + (K + 1) * NW;
    if (wid == 0) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const double t = wave_sum(lane < NW ? scratch[k * NW + lane] : 0.0);
        if (lane == 0) out[k] = t;
      }
      const double m = wave_max(lane < NW ? scratch[K * NW + lane] : -INFINITY);
      if (lane == 0) out[K] = m;
    }
    wg_barrier<L>();
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = out[k];
    mx = out[K];
  }
  wg_barrier<L>();
}

// Exclusive block scan of one non-negative value per thread; returns the
// thread's prefix and writes the block total to *total.
template <int NT = kBlock, bool L = false>
__device__ __forceinline__ long long block_exscan(long long v, long long* scratch /* NT/64 */,
                                                  long long* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  long long incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const long long t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  wg_barrier<L>();
  if (lane == 63) scratch[wid] = incl;
  wg_barrier<L>();
  long long base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) {
    if (i < wid) base += scratch[i];
    tot += scratch[i];
  }
  *total = tot;
  return base + incl - v;
}

// Two exclusive scans (a, b) in one LDS round trip.
template <int NT, bool L = false>
__device__ __forceinline__ void block_exscan2(long long a, long long b, long long* scratch /* 2*NT/64 */,
                                              long long* pa, long long* pb, long long* ta,
                                              long long* tb) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  long long ia = a, ib = b;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const long long t1 = __shfl_up(ia, o, 64);
    const long long t2 = __shfl_up(ib, o, 64);
    if (lane >= o) {
      ia += t1;
      ib += t2;
    }
  }
  wg_barrier<L>();
  if (lane == 63) {
    scratch[wid] = ia;
    scratch[NT / 64 + wid] = ib;
  }
  wg_barrier<L>();
  long long ba = 0, bb = 0, sa = 0, sb = 0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) {
    const long long x = scratch[i], y = scratch[NT / 64 + i];
    if (i < wid) {
      ba += x;
      bb += y;
    }
    sa += x;
    sb += y;
  }
  *pa = ba + ia - a;
  *pb = bb + ib - b;
  *ta = sa;
  *tb = sb;
}

}  // namespace di
