// D-iteration solve on gfx950: threshold rounds, one kernel launch per round.
//
// A round is the set form of the fluid/history recurrences (Section 2.2):
// every node whose score reaches the threshold theta_r (the threshold variant
// of Section 4.2) is taken at once, H_i += F_i, F_i = 0, and its fluid is
// pushed, d F_i p(j,i) to each child j.  Dangling nodes are taken like any
// other but push nothing (Section 3.4).
//
// The node set is cut into windows of 2^wlog consecutive ids; workgroup b owns
// window b for the whole solve.  Launch r of k_round, in workgroup b:
//   1. reduces the per-window partial sums of round r-1 (every workgroup does
//      this in the same order, so all reach bit-identical decisions without
//      any inter-workgroup communication): the stopping residual ||F||_1
//      (Theorem 2), the predicted remaining fluid and theta_r;
//   2. folds the pushes of round r-1 addressed to window b into an fp64 LDS
//      copy of its fluid (LDS atomics: a node hit k times is rounded once);
//   3. takes the nodes reaching theta_r and expands their out-links at once,
//      writing (local index, value) records into per-(source window,
//      destination window) segments.  A segment's place and size are fixed by
//      the graph (the number of links between the two windows), so a record's
//      slot is the segment start plus an LDS rank: no global atomics, no
//      fences;
//   4. stores its window's fluid and its partial sums.
// When round r-1 met the stop rule, launch r only folds (so the returned F, H
// again satisfy Theorem 1) and records the stop; later launches return at
// once.  The host launches rounds in chunks and reads the control block
// between chunks.
#include <algorithm>
#include <cmath>
#include <cstring>

#include <hip/hip_ext.h>

#include "kernels.h"

namespace di {

struct Workspace {
  int precision = 0, wlog = 0, nb = 0;
  int64_t n = 0, m = 0;
  DevBuf F, H, v, x, bstart, ctl;
  DevBuf pairs[2], cnt[2], slots;
  DevBuf soff, soffT, capT;  // nb x nb segment tables
  PinnedBuf hctl;
};

template <typename T>
struct DiArgs {
  int64_t n, m;
  int wlog, nb;
  const int64_t* row_ptr;
  const int32_t* deg;
  const int32_t* indeg;
  const int32_t* col;
  const double* w;
  const int64_t* bstart;  // [nb+1] first record of window w's region
  const int32_t* soff;    // [w][s] segment (s -> w) start within w's region
  const int32_t* soffT;   // [s][w] the same, source-major
  const int32_t* capT;    // [s][w] segment (s -> w) size = links from window s to window w
  T* F;
  double* H;
  PairT<T>* pairs[2];
  int32_t* cnt[2];        // [w][s] records written into segment (s -> w) in a round
  Slot* slots;            // [3][kSlots] round sums, round r uses set r % 3
  Ctl* ctl;
  double d, tol, c, theta0;
  int64_t max_rounds;
  int weighted;
};

// ------------------------------------------------------------ table setup

// E[w][s] = number of links from window s to window w.
__global__ void k_window_links(int64_t n, int wlog, int nb, const int64_t* __restrict__ row_ptr,
                               const int32_t* __restrict__ col, int32_t* __restrict__ E) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int s = (int)(i >> wlog);
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      const int w = col[e] >> wlog;
      atomicAdd(&E[(int64_t)w * nb + s], 1);
    }
  }
}

// soff[w][s] = exclusive prefix over s of E[w][s]; bstart[w] from in_ptr.
__global__ __launch_bounds__(kBlock) void k_segments(int64_t n, int wlog, int nb,
                                                     const int64_t* __restrict__ in_ptr,
                                                     const int32_t* __restrict__ E,
                                                     int32_t* __restrict__ soff,
                                                     int64_t* __restrict__ bstart,
                                                     int* __restrict__ err) {
  __shared__ long long s_scr[kBlock / 64];
  const int w = blockIdx.x;
  const int per = (nb + kBlock - 1) / kBlock;
  const int s0 = threadIdx.x * per;
  long long loc = 0;
  for (int k = 0; k < per; ++k)
    if (s0 + k < nb) loc += E[(int64_t)w * nb + s0 + k];
  long long tot = 0;
  long long run = block_exscan<kBlock>(loc, s_scr, &tot);
  for (int k = 0; k < per; ++k)
    if (s0 + k < nb) {
      soff[(int64_t)w * nb + s0 + k] = (int32_t)run;
      run += E[(int64_t)w * nb + s0 + k];
    }
  if (threadIdx.x == 0) {
    const int64_t lo = in_ptr[std::min((int64_t)w << wlog, n)];
    const int64_t hi = in_ptr[std::min(((int64_t)w + 1) << wlog, n)];
    bstart[w] = lo;
    if (w == nb - 1) bstart[nb] = hi;
    if (hi - lo != tot || hi - lo >= (1ll << 31)) atomicOr(err, 1);
  }
}

__global__ void k_transpose(int nb, const int32_t* __restrict__ E, const int32_t* __restrict__ soff,
                            int32_t* __restrict__ soffT, int32_t* __restrict__ capT) {
  const int64_t total = (int64_t)nb * nb;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += stride) {
    const int64_t w = k / nb, s = k % nb;
    soffT[s * nb + w] = soff[k];
    capT[s * nb + w] = E[k];
  }
}

// ------------------------------------------------------------------ kernels

// F = (1-d) V (V == NULL: uniform) and H = 0 unless resuming; control reset.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_init(DiArgs<T> a, const double* __restrict__ v,
                                                 int resume) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (!resume) {
    const double u = 1.0 / (double)a.n;
    for (int64_t i = t; i < a.n; i += stride) {
      a.F[i] = (T)((1.0 - a.d) * (v ? v[i] : u));
      a.H[i] = 0.0;
    }
  }
  for (int64_t k = t; k < 3 * kSlots; k += stride) {
    for (int f = 0; f < kSums; ++f) a.slots[k].sum[f] = 0.0;
    a.slots[k].mrem = 0;
  }
  if (t == 0) {
    Ctl* c = a.ctl;
    c->stop_round = -1;
    c->reason = 0;
    c->err = 0;
    c->nf = 0.0;
    c->theta = a.theta0;
    c->nodes_total = c->edges_total = 0;
    c->last_taken = c->last_edges = 0;
    for (int k = 0; k < 4; ++k) c->fl[k] = 0.0;
  }
}

// Score of a node holding fluid f: F itself (Section 4.2), or the ALGO-OP2 /
// ALGO-OP weights of Section 4.3.
template <int SCHED>
__device__ __forceinline__ double node_score(double f, int dg, int indeg) {
  if (SCHED == DI_SCHED_OP2) return f / ((double)dg + 1.0);
  if (SCHED == DI_SCHED_OP) return f / (((double)dg + 1.0) * ((double)indeg + 1.0));
  return f;
}

// In-place exclusive scan of arr[0..n) in LDS (NT threads); returns the total.
template <int NT>
__device__ long long lds_exscan(int32_t* arr, int n, long long* scr) {
  const int per = (n + NT - 1) / NT;
  const int s0 = threadIdx.x * per;
  long long loc = 0;
  for (int k = 0; k < per; ++k)
    if (s0 + k < n) loc += arr[s0 + k];
  long long tot = 0;
  long long run = block_exscan<NT>(loc, scr, &tot);
  for (int k = 0; k < per; ++k)
    if (s0 + k < n) {
      const int32_t v = arr[s0 + k];
      arr[s0 + k] = (int32_t)run;
      run += v;
    }
  __syncthreads();
  return tot;
}

// Largest i in [0, n) with a[i] <= x (a non-decreasing, a[0] <= x).
template <typename I>
__device__ __forceinline__ int upper_idx(const I* a, int n, long long x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((long long)a[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

constexpr int kRT = kRoundThreads;  // threads per round workgroup
constexpr int kU = 4;               // independent memory operations per thread per step
constexpr int kSuper = 2048;        // window nodes decided and expanded per pass
constexpr int kNPT = kSuper / kRT;  // nodes per thread per pass

// One round; mode 1 forces a fold-only launch (after an explicit single round).
template <typename T, int SCHED>
__global__ __launch_bounds__(kRT) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_round(DiArgs<T> a, int r,
                                                                                   int mode) {
  Ctl* ctl = a.ctl;
  // Launch r itself records stop_round = r-1; an earlier stop ends this launch.
  const int sr = ld_relaxed(&ctl->stop_round);
  if (sr >= 0 && sr < r - 1) return;

  extern __shared__ __align__(16) unsigned char smem[];
  const int W = 1 << a.wlog;
  const int nb = a.nb;
  double* win = reinterpret_cast<double*>(smem);             // [W]
  int64_t* s_base = reinterpret_cast<int64_t*>(win + W);      // [nb]
  int32_t* s_pre = reinterpret_cast<int32_t*>(s_base + nb);   // [nb+1] fold prefix, then ranks
  int32_t* s_soff = s_pre + (nb + 1);                         // [nb]
  int32_t* s_cap = s_soff + nb;                               // [nb]
  __shared__ int32_t s_beo[kSuper + 1];
  __shared__ int64_t s_brow[kSuper];
  __shared__ double s_bsh[kSuper];
  __shared__ double s_red[8 * (kRT / 64)];
  __shared__ long long s_scr[2 * (kRT / 64)];

  const int b = blockIdx.x;
  const int64_t j0 = (int64_t)b << a.wlog;
  const int wn = (int)min((int64_t)W, a.n - j0);
  const int tid = threadIdx.x;

  // Loads that do not depend on the round's decisions are issued first: this
  // window's fluid and, from round 1 on, its incoming segment counts/offsets.
  constexpr int kWinPer = 4;  // window values prefetched per thread (the rest load later)
  T fv[kWinPer];
#pragma unroll
  for (int k = 0; k < kWinPer; ++k) {
    const int q = tid + k * kRT;
    fv[k] = q < wn ? a.F[j0 + q] : (T)0;
  }
  const int32_t* cnt_in = a.cnt[(r - 1) & 1] + (int64_t)b * nb;
  int32_t c_own = 0, o_own = 0;  // first pass over sources (nb <= kRT in the common case)
  if (r >= 1 && tid < nb) {
    c_own = cnt_in[tid];
    o_own = a.soff[(int64_t)b * nb + tid];
  }

  // 1. Decisions from round r-1's partial sums (identical in every workgroup).
  double theta = a.theta0;
  bool stop = mode == 1;
  if (r >= 1) {
    const Slot* P = a.slots + ((r - 1) % 3) * kSlots;
    double v[kSums] = {0, 0, 0, 0, 0, 0, 0};  // nf, snd, sd, ssc, nnz, taken, edges
    double mrem = 0.0;
    if (tid < kSlots) {
      const Slot p = P[tid];
#pragma unroll
      for (int f = 0; f < kSums; ++f) v[f] = p.sum[f];
      mrem = __longlong_as_double((long long)p.mrem);
    }
    if (b == 0 && tid < kSlots) {  // set (r+1) % 3 is next used by launch r+1
      Slot* z = a.slots + ((r + 1) % 3) * kSlots + tid;
#pragma unroll
      for (int f = 0; f < kSums; ++f) z->sum[f] = 0.0;
      z->mrem = 0;
    }
    block_reduce_k<kRT, kSums>(v, mrem, s_red);
    const double nf = v[0], snd = v[1], sd = v[2], ssc = v[3], nnz = v[4], taken = v[5],
                 edges = v[6];
    int reason = 0;
    if (!isfinite(nf)) reason = 2;
    else if (nf < a.tol) reason = 1;
    else if ((int64_t)r >= a.max_rounds) reason = 3;
    if (reason) stop = true;
    // Remaining fluid after round r-1's pushes, in exact arithmetic: the
    // non-dangling senders keep d of what they send, the dangling ones none.
    const double R = nf - (1.0 - a.d) * snd - sd;
    // theta_r: c times the mean score of the nodes holding fluid, scaled by
    // the predicted decay of the total fluid.  After a round that took
    // nothing, fall back to the largest untaken score (at least the mean,
    // so the Lemma of Section 3.1 keeps its progress guarantee).
    theta = nnz > 0 ? a.c * (ssc / nnz) * (nf > 0 ? R / nf : 0.0) : 0.0;
    if (taken == 0 && theta > mrem) theta = mrem;
    if (b == 0 && tid == 0) {
      ctl->nodes_total += (long long)taken;
      ctl->edges_total += (long long)edges;
      ctl->last_taken = (long long)taken;
      ctl->last_edges = (long long)edges;
      ctl->theta = theta;
      ctl->nf = nf;
      if (stop) {
        ctl->reason = reason ? reason : 1;
        ctl->stop_round = r - 1;
      }
    }
  }

  // 2. Window fluid (fp64 in LDS) plus the pushes of round r-1.
#pragma unroll
  for (int k = 0; k < kWinPer; ++k) {
    const int q = tid + k * kRT;
    if (q < wn) win[q] = (double)fv[k];
  }
  for (int q = tid + kWinPer * kRT; q < wn; q += kRT) win[q] = (double)a.F[j0 + q];
  if (r >= 1) {
    if (tid < nb) {
      s_pre[tid] = c_own;
      s_soff[tid] = o_own;
    }
    for (int s = tid + kRT; s < nb; s += kRT) {
      s_pre[s] = cnt_in[s];
      s_soff[s] = a.soff[(int64_t)b * nb + s];
    }
    __syncthreads();
    const long long total = lds_exscan<kRT>(s_pre, nb, s_scr);
    const PairT<T>* pr = a.pairs[(r - 1) & 1];
    const int64_t base = a.bstart[b];
    for (long long i0 = tid; i0 < total; i0 += kU * kRT) {
      int64_t idx[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const long long i = i0 + (long long)u * kRT;
        idx[u] = -1;
        if (i < total) {
          const int s = upper_idx(s_pre, nb, i);
          idx[u] = base + s_soff[s] + (i - s_pre[s]);
        }
      }
      PairT<T> e[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u)
        if (idx[u] >= 0) e[u] = pr[idx[u]];
#pragma unroll
      for (int u = 0; u < kU; ++u)
        if (idx[u] >= 0 && e[u].loc < (uint32_t)wn) atomicAdd(&win[e[u].loc], (double)e[u].val);
    }
  }
  __syncthreads();
  if (stop) {
    for (int q = tid; q < wn; q += kRT) a.F[j0 + q] = (T)win[q];
    return;
  }

  // 3. Take and expand, one tile of kRT nodes at a time.
  for (int w = tid; w < nb; w += kRT) {
    s_pre[w] = 0;  // now: records written per destination window
    s_base[w] = a.bstart[w] + a.soffT[(int64_t)b * nb + w];
    s_cap[w] = a.capT[(int64_t)b * nb + w];
  }
  __syncthreads();
  PairT<T>* out = a.pairs[r & 1];
  const uint32_t wmask = (uint32_t)W - 1u;
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};  // nf, snd, sd, ssc, nnz, taken, edges
  double mrem = 0.0;
  for (int t0 = 0; t0 < wn; t0 += kSuper) {
    // A. Decide for kNPT nodes per thread, then issue all their loads at once.
    double f[kNPT];
    bool tk[kNPT];
#pragma unroll
    for (int u = 0; u < kNPT; ++u) {
      const int q = t0 + tid + u * kRT;
      f[u] = q < wn ? win[q] : 0.0;
      tk[u] = false;
      if (f[u] > 0.0) {
        const int64_t j = j0 + q;
        acc[0] += f[u];
        acc[4] += 1.0;
        int dg = -1;
        if (SCHED != DI_SCHED_MEAN) dg = a.deg[j];
        const double sc = node_score<SCHED>(f[u], dg, SCHED == DI_SCHED_OP ? a.indeg[j] : 0);
        acc[3] += sc;
        if (sc >= theta) tk[u] = true;
        else mrem = fmax(mrem, sc);
      } else if (f[u] != f[u]) {
        acc[0] = NAN;
      }
    }
    int64_t rs[kNPT];
    int dgs[kNPT];
    double h[kNPT];
#pragma unroll
    for (int u = 0; u < kNPT; ++u) {
      if (!tk[u]) continue;
      const int64_t j = j0 + t0 + tid + u * kRT;
      rs[u] = a.row_ptr[j];
      dgs[u] = a.deg[j];
      h[u] = a.H[j];
    }
    long long npush = 0, nedge = 0;
#pragma unroll
    for (int u = 0; u < kNPT; ++u) {
      if (!tk[u]) continue;
      const int q = t0 + tid + u * kRT;
      a.H[j0 + q] = h[u] + f[u];
      win[q] = 0.0;
      acc[5] += 1.0;
      if (dgs[u] > 0) {
        acc[1] += f[u];
        ++npush;
        nedge += dgs[u];
      } else {
        acc[2] += f[u];
      }
    }
    // B. Stage the pushing nodes (thread-major order) with their link offsets.
    long long slot = 0, eoff = 0, ntile = 0, etile = 0;
    block_exscan2<kRT>(npush, nedge, s_scr, &slot, &eoff, &ntile, &etile);
    if (ntile == 0) continue;  // uniform
#pragma unroll
    for (int u = 0; u < kNPT; ++u) {
      if (!tk[u] || dgs[u] == 0) continue;
      const long long dg = dgs[u];
      s_beo[slot] = (int32_t)eoff;
      s_brow[slot] = rs[u];
      s_bsh[slot] = a.weighted ? a.d * f[u] : a.d * f[u] / (double)dg;
      ++slot;
      eoff += dg;
    }
    __syncthreads();
    // C. Push every staged link: kU independent link reads per thread per step.
    const int bcount = (int)ntile;
    for (long long t00 = tid; t00 < etile; t00 += kU * kRT) {
      int64_t e[kU];
      int kk[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const long long t = t00 + (long long)u * kRT;
        e[u] = -1;
        if (t < etile) {
          kk[u] = upper_idx(s_beo, bcount, t);
          e[u] = s_brow[kk[u]] + (t - s_beo[kk[u]]);
        }
      }
      uint32_t dst[kU];
      double v[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u)
        if (e[u] >= 0) {
          dst[u] = (uint32_t)a.col[e[u]];
          v[u] = s_bsh[kk[u]];
          if (a.weighted) v[u] *= a.w[e[u]];
        }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        if (e[u] < 0) continue;
        const int w = (int)(dst[u] >> a.wlog);
        const int rank = atomicAdd(&s_pre[w], 1);
        if (rank < s_cap[w]) {
          PairT<T> pr;
          memset(&pr, 0, sizeof(pr));
          pr.loc = dst[u] & wmask;
          pr.val = (T)v[u];
          out[s_base[w] + rank] = pr;
        } else {
          atomicOr(&ctl->err, 2);
        }
      }
    }
    acc[6] += (double)etile;  // uniform: counted once below (thread 0 only)
    __syncthreads();
  }
  int32_t* cnt_out = a.cnt[r & 1];  // destination-major: these stores are posted
  for (int w = tid; w < nb; w += kRT) cnt_out[(int64_t)w * nb + b] = s_pre[w];
  for (int q = tid; q < wn; q += kRT) a.F[j0 + q] = (T)win[q];

  // 4. This window's sums, added into its slot.
  const double edges = acc[6];
  acc[6] = 0.0;
  block_reduce_k<kRT, kSums>(acc, mrem, s_red);
  if (tid == 0) {
    acc[6] = edges;
    Slot* sl = a.slots + (r % 3) * kSlots + (b % kSlots);
#pragma unroll
    for (int f = 0; f < kSums; ++f)
      if (acc[f] != 0.0) unsafeAtomicAdd(&sl->sum[f], acc[f]);
    if (mrem > 0.0) atomicMax(&sl->mrem, (unsigned long long)__double_as_longlong(mrem));
  }
}

// Flush sums: sum(H+F), sum(H), sum(F), sum over dangling nodes of H, as
// per-block partials spread over 256 slots of acc.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_flush_sum(DiArgs<T> a, double* __restrict__ acc) {
  __shared__ double s_red[kBlock / 64];
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * kBlock) {
    const double h = a.H[i], f = (double)a.F[i];
    s0 += h + f;
    s1 += h;
    s2 += f;
    if (a.deg[i] == 0) s3 += h;
  }
  s0 = block_sum(s0, s_red);
  s1 = block_sum(s1, s_red);
  s2 = block_sum(s2, s_red);
  s3 = block_sum(s3, s_red);
  if (threadIdx.x == 0) {
    double* slot = acc + 4 * (blockIdx.x & 255);
    unsafeAtomicAdd(slot + 0, s0);
    unsafeAtomicAdd(slot + 1, s1);
    unsafeAtomicAdd(slot + 2, s2);
    unsafeAtomicAdd(slot + 3, s3);
  }
}

// Reduce the 256 flush slots into ctl->fl (one block).
__global__ __launch_bounds__(kBlock) void k_flush_reduce(const double* __restrict__ acc, Ctl* ctl) {
  __shared__ double s_red[kBlock / 64];
  for (int k = 0; k < 4; ++k) {
    const double v = block_sum(acc[4 * threadIdx.x + k], s_red);
    if (threadIdx.x == 0) ctl->fl[k] = v;
  }
}

// x = (H + F) / sum(H + F)  (renormalisation of Section 3.4), or H + F.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_flush_write(DiArgs<T> a, double* __restrict__ x,
                                                        int normalize) {
  const double s = normalize ? a.ctl->fl[0] : 1.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * kBlock)
    x[i] = (a.H[i] + (double)a.F[i]) / s;
}

__global__ void k_zero(double* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// --------------------------------------------------------------- workspace

static double* flush_slots(Workspace* ws) {
  return reinterpret_cast<double*>(reinterpret_cast<char*>(ws->ctl.p) + 1024);
}

Workspace* acquire_workspace(Graph* g, int precision, int wlog) {
  {
    std::lock_guard<std::mutex> lk(g->ws_mu);
    for (size_t i = 0; i < g->ws_free.size(); ++i) {
      Workspace* ws = g->ws_free[i];
      if (ws->precision == precision && ws->wlog == wlog) {
        g->ws_free.erase(g->ws_free.begin() + i);
        return ws;
      }
    }
  }
  auto* ws = new Workspace();
  try {
    const int64_t n = g->n, m = g->m;
    const size_t fs = precision == DI_FP64 ? 8 : 4;
    const int nb = (int)((n + (1ll << wlog) - 1) >> wlog);
    const int64_t nb2 = (int64_t)nb * nb;
    static_assert(sizeof(Ctl) <= 1024, "control block layout");
    ws->precision = precision;
    ws->wlog = wlog;
    ws->nb = nb;
    ws->n = n;
    ws->m = m;
    ws->F.alloc(n * fs);
    ws->H.alloc(n * 8);
    ws->v.alloc(n * 8);
    ws->x.alloc(n * 8);
    ws->bstart.alloc((nb + 1) * 8);
    ws->ctl.alloc(1024 + 1024 * 8);  // Ctl, then 256 x 4 flush slots
    for (int k = 0; k < 2; ++k) {
      ws->pairs[k].alloc(std::max<int64_t>(m, 1) * (precision == DI_FP64 ? 16 : 8));
      ws->cnt[k].alloc(nb2 * 4);
    }
    ws->slots.alloc(3 * kSlots * sizeof(Slot));
    ws->soff.alloc(nb2 * 4);
    ws->soffT.alloc(nb2 * 4);
    ws->capT.alloc(nb2 * 4);
    ws->hctl.alloc(sizeof(Ctl));
    DevBuf E;
    E.alloc(nb2 * 4);
    DI_HIP(hipMemset(E.p, 0, nb2 * 4));
    DI_HIP(hipMemset(ws->ctl.p, 0, sizeof(Ctl)));
    const int gn = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
    k_window_links<<<gn, 256>>>(n, wlog, nb, g->row_ptr.as<int64_t>(), g->col.as<int32_t>(),
                                E.as<int32_t>());
    DI_HIP(hipGetLastError());
    k_segments<<<nb, kBlock>>>(n, wlog, nb, g->in_ptr.as<int64_t>(), E.as<int32_t>(),
                               ws->soff.as<int32_t>(), ws->bstart.as<int64_t>(),
                               &ws->ctl.as<Ctl>()->err);
    DI_HIP(hipGetLastError());
    const int gt = (int)std::max<int64_t>(1, std::min<int64_t>((nb2 + 255) / 256, 4096));
    k_transpose<<<gt, 256>>>(nb, E.as<int32_t>(), ws->soff.as<int32_t>(), ws->soffT.as<int32_t>(),
                             ws->capT.as<int32_t>());
    DI_HIP(hipGetLastError());
    DI_HIP(hipDeviceSynchronize());
    Ctl h;
    DI_HIP(hipMemcpy(&h, ws->ctl.p, sizeof(Ctl), hipMemcpyDeviceToHost));
    if (h.err) {
      set_error("window segment tables do not match the in-link counts");
      throw Fail{DI_EDEVICE};
    }
  } catch (...) {
    delete ws;
    throw;
  }
  return ws;
}

void release_workspace(Graph* g, Workspace* ws) {
  std::lock_guard<std::mutex> lk(g->ws_mu);
  if (g->ws_free.size() >= 4) {
    delete g->ws_free.front();
    g->ws_free.erase(g->ws_free.begin());
  }
  g->ws_free.push_back(ws);
}

void destroy_workspace(Workspace* ws) { delete ws; }

// Returns the workspace to the graph's pool once the stream has drained, so a
// failed call never hands out a workspace that kernels still use.
struct WsGuard {
  Graph* g;
  Workspace* ws;
  hipStream_t s;
  ~WsGuard() {
    if (!ws) return;
    if (hipStreamSynchronize(s) == hipSuccess) release_workspace(g, ws);
  }
};

// ------------------------------------------------------------- host driver

template <typename T>
static DiArgs<T> make_args(const Graph* g, Workspace* ws, double d, double tol, double c,
                           int64_t max_rounds, T* F, double* H) {
  DiArgs<T> a;
  memset(&a, 0, sizeof(a));
  a.n = g->n;
  a.m = g->m;
  a.wlog = ws->wlog;
  a.nb = ws->nb;
  a.row_ptr = g->row_ptr.as<int64_t>();
  a.deg = g->deg.as<int32_t>();
  a.indeg = g->indeg.as<int32_t>();
  a.col = g->col.as<int32_t>();
  a.w = g->weighted ? g->w.as<double>() : nullptr;
  a.weighted = g->weighted ? 1 : 0;
  a.bstart = ws->bstart.as<int64_t>();
  a.soff = ws->soff.as<int32_t>();
  a.soffT = ws->soffT.as<int32_t>();
  a.capT = ws->capT.as<int32_t>();
  a.F = F;
  a.H = H;
  for (int k = 0; k < 2; ++k) {
    a.pairs[k] = ws->pairs[k].as<PairT<T>>();
    a.cnt[k] = ws->cnt[k].as<int32_t>();
  }
  a.slots = ws->slots.as<Slot>();
  a.ctl = ws->ctl.as<Ctl>();
  a.d = d;
  a.tol = tol;
  a.c = c;
  a.theta0 = 0.0;
  a.max_rounds = max_rounds;
  return a;
}

static int grid_for(int64_t n, int cap) {
  int64_t b = (n + kBlock - 1) / kBlock;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

template <typename T, int SCHED>
static void launch_round_t(const DiArgs<T>& a, int r, int mode, hipStream_t s, LaunchTimer* lt) {
  const size_t smem = round_lds_bytes(a.wlog, a.nb);
  static size_t dyn_limit = 0;
  if (dyn_limit == 0) {
    // Dynamic LDS may use what the static part leaves of the workgroup limit.
    hipFuncAttributes fa;
    DI_HIP(hipFuncGetAttributes(&fa, (const void*)k_round<T, SCHED>));
    int dev = 0, lim = 0;
    DI_HIP(hipGetDevice(&dev));
    DI_HIP(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    dyn_limit = (size_t)lim - fa.sharedSizeBytes;
    DI_HIP(hipFuncSetAttribute((const void*)k_round<T, SCHED>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_limit));
  }
  DI_REQUIRE(smem <= dyn_limit, "window tables exceed the LDS available to the round kernel");
  if (lt && lt->on) {
    // The runtime stamps the kernel's own begin/end into the event pair.
    hipEvent_t e0, e1;
    lt->next(&e0, &e1);
    hipExtLaunchKernelGGL(k_round<T, SCHED>, dim3(a.nb), dim3(kRT), smem, s, e0, e1, 0, a, r,
                          mode);
  } else {
    k_round<T, SCHED><<<a.nb, kRT, smem, s>>>(a, r, mode);
  }
  DI_HIP(hipGetLastError());
}

template <typename T>
static void launch_round(const DiArgs<T>& a, int sched, int r, int mode, hipStream_t s,
                         LaunchTimer* lt = nullptr) {
  switch (sched) {
    case DI_SCHED_OP2: launch_round_t<T, DI_SCHED_OP2>(a, r, mode, s, lt); break;
    case DI_SCHED_OP: launch_round_t<T, DI_SCHED_OP>(a, r, mode, s, lt); break;
    default: launch_round_t<T, DI_SCHED_MEAN>(a, r, mode, s, lt); break;
  }
}

static void read_ctl(Workspace* ws, hipStream_t s) {
  DI_HIP(hipMemcpyAsync(ws->hctl.p, ws->ctl.p, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  DI_HIP(hipStreamSynchronize(s));
}

// Launches rounds until a launch records the stop (that launch also folds the
// last pushes, so (F, H) is again a state of the recurrences).
template <typename T>
static void run_rounds(const DiArgs<T>& a, Workspace* ws, int sched, int check_every,
                       hipStream_t s, LaunchTimer* lt) {
  Ctl* h = ws->hctl.as<Ctl>();
  int r = 0;
  int chunk = check_every > 0 ? check_every : 8;
  double nf_prev = -1.0;
  int r_prev = 0;
  for (;;) {
    for (int i = 0; i < chunk; ++i) launch_round(a, sched, r++, 0, s, lt);
    read_ctl(ws, s);
    if (h->stop_round >= 0) break;
    if (check_every == 0) {
      // Predict the rounds left from the observed per-round decay of ||F||_1.
      int next = 8;
      if (nf_prev > 0.0 && h->nf > 0.0 && h->nf < nf_prev && r > r_prev) {
        const double q = std::pow(h->nf / nf_prev, 1.0 / (r - r_prev));
        if (q > 0.0 && q < 1.0)
          next = (int)std::ceil(std::log(a.tol / h->nf) / std::log(q) * 1.15) + 2;
      }
      chunk = std::max(2, std::min(next, 64));
      nf_prev = h->nf;
      r_prev = r;
    }
  }
}

template <typename T>
static void flush(const DiArgs<T>& a, Workspace* ws, double* x, int normalize, hipStream_t s) {
  double* acc = flush_slots(ws);
  k_zero<<<4, 256, 0, s>>>(acc, 1024);
  DI_HIP(hipGetLastError());
  const int grid = grid_for(a.n, 1024);
  k_flush_sum<T><<<grid, kBlock, 0, s>>>(a, acc);
  DI_HIP(hipGetLastError());
  k_flush_reduce<<<1, kBlock, 0, s>>>(acc, a.ctl);
  DI_HIP(hipGetLastError());
  if (x) {
    k_flush_write<T><<<grid, kBlock, 0, s>>>(a, x, normalize);
    DI_HIP(hipGetLastError());
  }
}

template <typename T>
static di_status solve_impl(Graph* g, const double* v, const di_opts* o, double* x,
                            di_stats* st, hipStream_t s) {
  const di_tune* tn = o->tune;
  const int sched = tn ? tn->schedule : DI_SCHED_MEAN;
  DI_REQUIRE(sched >= 0 && sched <= 2, "unknown schedule");
  const double c = (tn && tn->c > 0.f) ? (double)tn->c : 1.0;
  const int wlog = window_log2_for(g->n, tn ? tn->window_log2 : 0);
  DI_REQUIRE(wlog > 0, "graph has too many nodes for the window tables");
  const int check_every = tn ? std::max(0, tn->check_every) : 0;
  const bool dev = (o->flags & DI_DEVICE_PTRS) != 0;
  const bool resume = (o->flags & DI_RESUME) != 0;
  const int64_t max_rounds = o->max_rounds > 0 ? o->max_rounds : 1000000;
  DI_REQUIRE(!resume || (o->state_f && o->state_h), "DI_RESUME needs state_f and state_h");
  if (v && !dev) validate_vector(v, g->n, "v");
  WsGuard guard{g, acquire_workspace(g, o->precision, wlog), s};
  Workspace* ws = guard.ws;
  const double* vdev = nullptr;
  if (v) {
    if (dev) {
      vdev = v;
    } else {
      DI_HIP(hipMemcpyAsync(ws->v.p, v, g->n * 8, hipMemcpyHostToDevice, s));
      vdev = ws->v.as<double>();
    }
  }
  T* F = resume ? static_cast<T*>(o->state_f) : ws->F.as<T>();
  double* H = resume ? o->state_h : ws->H.as<double>();
  DiArgs<T> a = make_args<T>(g, ws, o->d, o->tol, c, max_rounds, F, H);
  LaunchTimer lt(s, (o->flags & DI_TIMING) != 0);
  EventTimer timer(s);
  k_init<T><<<grid_for(g->n, 2048), kBlock, 0, s>>>(a, vdev, resume ? 1 : 0);
  DI_HIP(hipGetLastError());
  run_rounds(a, ws, sched, check_every, s, &lt);
  double* xo = x ? (dev ? x : ws->x.as<double>()) : nullptr;
  flush(a, ws, xo, o->normalize, s);
  const double secs = timer.stop();
  if (x && !dev) DI_HIP(hipMemcpyAsync(x, xo, g->n * 8, hipMemcpyDeviceToHost, s));
  read_ctl(ws, s);
  const Ctl* h = ws->hctl.as<Ctl>();
  if (st) {
    const double d = o->d;
    const double S = h->fl[0], nf = h->fl[2];
    st->residual_l1 = nf;
    st->err_bound_l1 = o->normalize ? (S > 0 ? 2.0 * d * nf / ((1.0 - d) * S) : 0.0)
                                    : d * nf / (1.0 - d);
    st->mass_drift = h->fl[1] + (h->fl[2] + d * h->fl[3]) / (1.0 - d) - 1.0;
    st->seconds = secs;
    st->rounds = h->stop_round + 1;
    st->nodes_diffused = h->nodes_total;
    st->edges_diffused = h->edges_total;
    // launches 0..stop_round take and expand; launch stop_round+1 folds.
    const size_t working = (size_t)h->stop_round + 2;
    st->kernel_seconds = lt.on ? lt.total(working) : 0.0;
    st->kernel_launches = lt.on ? (int64_t)working : 0;
  }
  if (h->err) {
    set_error("internal segment consistency check failed (code " + std::to_string(h->err) + ")");
    return DI_EDEVICE;
  }
  if (h->reason == 2) {
    set_error("non-finite residual");
    return DI_EDEVICE;
  }
  if (h->reason == 3) {
    set_error("max_rounds reached before ||F||_1 < tol");
    return DI_ENOTCONV;
  }
  return DI_OK;
}

template <typename T>
static void round_impl(Graph* g, double d, double theta, T* F, double* H, int64_t* tn,
                       int64_t* te, hipStream_t s) {
  const int wlog = window_log2_for(g->n, 0);
  DI_REQUIRE(wlog > 0, "graph has too many nodes for the window tables");
  WsGuard guard{g,
                acquire_workspace(g, std::is_same<T, double>::value ? DI_FP64 : DI_FP32_FLUID, wlog),
                s};
  Workspace* ws = guard.ws;
  DiArgs<T> a = make_args<T>(g, ws, d, 0.0, 1.0, (int64_t)1 << 40, F, H);
  a.theta0 = theta;
  k_init<T><<<grid_for(g->n, 2048), kBlock, 0, s>>>(a, nullptr, 1);
  DI_HIP(hipGetLastError());
  launch_round(a, DI_SCHED_MEAN, 0, 0, s);
  launch_round(a, DI_SCHED_MEAN, 1, 1, s);
  read_ctl(ws, s);
  const Ctl* h = ws->hctl.as<Ctl>();
  if (h->err) {
    set_error("internal segment consistency check failed");
    throw Fail{DI_EDEVICE};
  }
  if (tn) *tn = h->last_taken;
  if (te) *te = h->last_edges;
}

}  // namespace di

using namespace di;

extern "C" {

di_status di_solve(const di_graph* gc, const double* v, const di_opts* opts, double* x,
                   di_stats* stats, void* stream) {
  di_status rc = DI_OK;
  di_status g = guarded([&] {
    DI_REQUIRE(gc != nullptr, "graph is NULL");
    validate_d_tol(opts);
    Graph* g = const_cast<di_graph*>(gc);
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = opts->precision == DI_FP64 ? solve_impl<double>(g, v, opts, x, stats, s)
                                    : solve_impl<float>(g, v, opts, x, stats, s);
  });
  return g != DI_OK ? g : rc;
}

di_status di_diffuse_round(const di_graph* gc, int32_t precision, double d, double theta,
                           void* F, double* H, int64_t* taken_nodes, int64_t* taken_edges,
                           void* stream) {
  return guarded([&] {
    DI_REQUIRE(gc != nullptr, "graph is NULL");
    DI_REQUIRE(std::isfinite(d) && d >= 0.0 && d < 1.0, "d must satisfy 0 <= d < 1");
    DI_REQUIRE(!std::isnan(theta), "theta is NaN");
    DI_REQUIRE(F != nullptr && H != nullptr, "F and H must be device pointers");
    Graph* g = const_cast<di_graph*>(gc);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (precision == DI_FP64)
      round_impl<double>(g, d, theta, static_cast<double*>(F), H, taken_nodes, taken_edges, s);
    else if (precision == DI_FP32_FLUID)
      round_impl<float>(g, d, theta, static_cast<float*>(F), H, taken_nodes, taken_edges, s);
    else
      DI_REQUIRE(false, "unknown precision");
  });
}

}  // extern "C"
