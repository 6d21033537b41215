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

// Partial sums of one window in one round (written by the window's
// workgroup, reduced by every workgroup of the next round).
struct alignas(64) Part {
  double nf;    // fluid held before the take (the stopping residual)
  double snd;   // fluid taken from non-dangling nodes (pushed on)
  double sd;    // fluid taken from dangling nodes (leaves the system)
  double ssc;   // sum of the schedule's score over nodes holding fluid
  double mrem;  // largest untaken score
  unsigned long long nnz, taken, edges;  // nodes holding fluid, taken, out-links pushed
};

// Control block in device memory.  Each field is written by workgroup 0 of
// one launch and read only by later launches.
struct Ctl {
  int stop_round;  // -1 while running; else the last round whose set was taken
  int reason;      // 1 converged, 2 non-finite residual, 3 max rounds
  int err;         // capacity / range violation (never set on valid input)
  int pad;
  double nf;       // ||F||_1 seen by the stopping round, before its take
  double theta;    // threshold of the latest round
  long long nodes_total, edges_total;  // diffusions and out-links used
  long long last_taken, last_edges;    // of the latest round
  double fl[4];    // flush sums: sum(H+F), sum(H), sum(F), sum over dangling of H
};

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

// Block-wide sum / max over kBlock threads (fixed order: deterministic);
// every thread gets the result.
__device__ __forceinline__ double block_sum(double v, double* scratch /* kBlock/64 */) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < kBlock / 64; ++i) t += scratch[i];
  return t;
}
__device__ __forceinline__ double block_max(double v, double* scratch /* kBlock/64 */) {
  v = wave_max(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double t = scratch[0];
#pragma unroll
  for (int i = 1; i < kBlock / 64; ++i) t = fmax(t, scratch[i]);
  return t;
}

// Exclusive block scan of one non-negative value per thread; returns the
// thread's prefix and writes the block total to *total.
__device__ __forceinline__ long long block_exscan(long long v, long long* scratch /* kBlock/64 */,
                                                  long long* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  long long incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const long long t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  __syncthreads();
  if (lane == 63) scratch[wid] = incl;
  __syncthreads();
  long long base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kBlock / 64; ++i) {
    if (i < wid) base += scratch[i];
    tot += scratch[i];
  }
  *total = tot;
  return base + incl - v;
}

template <typename T>
__device__ __forceinline__ T ld_relaxed(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace di
