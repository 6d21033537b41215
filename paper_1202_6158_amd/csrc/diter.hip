// D-iteration solve on gfx950: threshold rounds, one kernel launch per round.
//
// A round is the set form of the fluid/history recurrences (Section 2.2):
// every node whose score reaches the threshold theta_r (the threshold variant
// of Section 4.2) is taken at once, H_i += F_i, F_i = 0, and its fluid is
// pushed, d F_i p(j,i) to each child j.  Dangling nodes are taken like any
// other but push nothing (Section 3.3).
//
// The node set is cut into windows of 2^wlog consecutive ids; workgroup b owns
// window b for the whole solve.  Launch r of k_round, in workgroup b:
//   1. reduces the per-window partial sums of round r-1 (every workgroup does
//      this in the same order, so all reach bit-identical decisions without
//      any inter-workgroup communication): the stopping residual ||F||_1
//      (Theorem 2), the predicted remaining fluid and theta_r;
//   2. folds the pushes of round r-1 addressed to window b into an fp64 LDS
//      copy of its fluid (LDS atomics: a node hit k times is rounded once);
//   3. takes the nodes reaching theta_r (listed in node order in LDS) and
//      expands their out-links at once, 1024 nodes per pass, writing
//      (local index, value) records into per-(source window,
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
#include <atomic>
#include <cmath>
#include <cstring>
#include <type_traits>

#include <hip/hip_ext.h>

#include "kernels.h"

namespace di {

struct Workspace {
  int precision = 0, wlog = 0, nb = 0, nvec = 0;
  bool gt = false;  // segment tables read from global memory (not staged in LDS)
  int64_t n = 0, m = 0;
  DevBuf F, H, v, x, bstart, ctl, flacc, active;
  DevBuf pairs[2], cnt[2], slots;
  DevBuf soff, soffT, capT;  // nb x nb segment tables
  DevBuf front;              // frontier list of the whole-graph window (k_small)
  PinnedBuf hctl, hctl2;     // host copies of the control blocks (two in flight while polling)
  hipEvent_t ev[2] = {nullptr, nullptr};  // completion of those copies
  Workspace() = default;
  Workspace(const Workspace&) = delete;
  Workspace& operator=(const Workspace&) = delete;
  ~Workspace() {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
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
  // Per-vector state; vector vb (blockIdx.y) is at the given offsets.
  T* F;                   // [nvec][n]
  double* H;              // [nvec][n]
  PairT<T>* pairs[2];     // [nvec][mrec] records of even / odd rounds
  int32_t* cnt[2];        // [nvec][w][s] records written into segment (s -> w) in a round
  Slot* slots;            // [nvec][3][kSlots] round sums, round r uses set r % 3
  uint8_t* active;        // [nvec][nb] window held fluid after its last round
  Ctl* ctl;               // [nvec]
  double* flacc;          // [nvec][kFlushAcc] flush partial sums
  int64_t mrec;           // records per vector buffer
  int nvec;
  // Serving: blockIdx.y -> vector slot, and per-slot round index, d and tol
  // (NULL for solves and batches, which use blockIdx.y, the launch's round
  // index and the common d / tol).
  const int32_t* vmap;
  const int32_t* vround;
  const double* vd;
  const double* vtol;
  double d, tol, c, theta0;
  int64_t max_rounds;
  int weighted;
  int threads;  // round workgroup size (host side: selects the kernel instance)
  int gt;       // segment tables in global memory (host side: selects the kernel instance)
  int wlist;    // taken list: 1 whole window (after the state bytes), 0 one pass (staging), 2 none
  uint8_t* trace;        // [trace_rounds][n] taken sets of a traced solve (NULL: none)
  int64_t trace_rounds;
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

// F = (1-d) V (V == NULL: uniform) and H = 0 unless resuming, for vector
// blockIdx.y; control, round sums and window activity reset.  seeds != NULL
// (batches): F starts at zero and k_seed adds the seed fluid afterwards.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_init(DiArgs<T> a, const double* __restrict__ v,
                                                 int resume, int seeded) {
  const int vb = a.vmap ? a.vmap[blockIdx.y] : blockIdx.y;
  const double dv = a.vd ? a.vd[vb] : a.d;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  T* F = a.F + (int64_t)vb * a.n;
  double* H = a.H + (int64_t)vb * a.n;
  if (!resume) {
    const double u = 1.0 / (double)a.n;
    for (int64_t i = t; i < a.n; i += stride) {
      F[i] = seeded ? (T)0 : (T)((1.0 - dv) * (v ? v[i] : u));
      H[i] = 0.0;
    }
  }
  Slot* slots = a.slots + (int64_t)vb * 3 * kSlots;
  for (int64_t k = t; k < 3 * kSlots; k += stride) {
    for (int f = 0; f < kSums; ++f) slots[k].sum[f] = 0.0;
    slots[k].mrem = 0;
  }
  for (int64_t w = t; w < a.nb; w += stride) a.active[(int64_t)vb * a.nb + w] = seeded ? 0 : 1;
  // Record counts: rounds write only non-zero entries and their readers clear
  // them, so both buffers start at zero.
  const int64_t nb2 = (int64_t)a.nb * a.nb;
  for (int k = 0; k < 2; ++k) {
    int32_t* c = a.cnt[k] + vb * nb2;
    for (int64_t q = t; q < nb2; q += stride) c[q] = 0;
  }
  if (t == 0) {
    Ctl* c = a.ctl + vb;
    c->stop_round = -1;
    c->reason = 0;
    c->err = 0;
    c->bar = 0;
    c->nf = 0.0;
    c->theta = a.theta0;
    c->nodes_total = c->edges_total = 0;
    c->last_taken = c->last_edges = 0;
    for (int k = 0; k < kFlushSums; ++k) c->fl[k] = 0.0;
  }
}

// Seed fluid of a batch: vector b holds (1-d) w_k on seeds[ptr[b]..ptr[b+1])
// (w == NULL: uniform over the set); their windows start active.
template <typename T>
__global__ void k_seed(DiArgs<T> a, const int64_t* __restrict__ ptr, const int32_t* __restrict__ seeds,
                       const double* __restrict__ w) {
  const int vb = a.vmap ? a.vmap[blockIdx.x] : blockIdx.x;
  const double dv = a.vd ? a.vd[vb] : a.d;
  const int64_t s0 = ptr[blockIdx.x], s1 = ptr[blockIdx.x + 1];
  for (int64_t k = s0 + threadIdx.x; k < s1; k += blockDim.x) {
    const int32_t i = seeds[k];
    const double wt = w ? w[k] : 1.0 / (double)(s1 - s0);
    a.F[(int64_t)vb * a.n + i] = (T)((1.0 - dv) * wt);
    a.active[(int64_t)vb * a.nb + (i >> a.wlog)] = 1;
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

// Score sum and count of the nodes holding fluid in a resumed state: the
// first round of a resumed solve takes c times their mean score as its
// threshold (the rule of every later round) instead of 0, so that it does not
// take every node that kept a trace of fluid.  out[0..1] must start at zero.
template <typename T, int SCHED>
__global__ __launch_bounds__(kBlock) void k_resume_scores(DiArgs<T> a, double* __restrict__ out) {
  __shared__ double s_red[kBlock / 64];
  double ssc = 0.0, nnz = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * kBlock) {
    const double f = fabs((double)a.F[i]);
    if (f > 0.0) {
      const int dg = SCHED != DI_SCHED_MEAN ? a.deg[i] : -1;
      ssc += node_score<SCHED>(f, dg, SCHED == DI_SCHED_OP ? a.indeg[i] : 0);
      nnz += 1.0;
    }
  }
  ssc = block_sum(ssc, s_red);
  nnz = block_sum(nnz, s_red);
  if (threadIdx.x == 0) {
    unsafeAtomicAdd(&out[0], ssc);
    unsafeAtomicAdd(&out[1], nnz);
  }
}

// In-place exclusive scan of arr[0..n) in LDS (NT threads); returns the total.
// L: LDS-only barriers (see wg_barrier).
template <int NT, bool L = false>
__device__ long long lds_exscan(int32_t* arr, int n, long long* scr) {
  const int per = (n + NT - 1) / NT;
  const int s0 = threadIdx.x * per;
  long long loc = 0;
  for (int k = 0; k < per; ++k)
    if (s0 + k < n) loc += arr[s0 + k];
  long long tot = 0;
  long long run = block_exscan<NT, L>(loc, scr, &tot);
  for (int k = 0; k < per; ++k)
    if (s0 + k < n) {
      const int32_t v = arr[s0 + k];
      arr[s0 + k] = (int32_t)run;
      run += v;
    }
  wg_barrier<L>();
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

// Workgroups go to the 8 XCDs round-robin by linear id.  The round kernel
// maps linear ids to (vector column, window) so that each XCD gets a
// contiguous range of windows: neighbouring windows then share an L2, where
// their writes into the same lines of the count matrix and of the record
// regions can merge.  A bijection of [0, nb * columns).
__device__ __forceinline__ void xcd_window(int nb, int* col, int* win) {
  const long long total = (long long)nb * gridDim.y;
  const long long L = (long long)blockIdx.y * gridDim.x + blockIdx.x;
  const long long x = L & 7, k = L >> 3, base = total >> 3, rem = total & 7;
  const long long m = x * base + (x < rem ? x : rem) + k;
  *col = (int)(m / nb);
  *win = (int)(m - (long long)(*col) * nb);
}

constexpr int kRun = 4;             // consecutive records / links per thread per step
constexpr int kSuper = 1024;        // window nodes decided and expanded per pass

// One round; mode 1 forces a fold-only launch (after an explicit single round).
// NT threads per workgroup (512 or 1024: more loads in flight per window).
// GT: the per-window segment tables (record bases, capacities, fold offsets)
// are read from global memory where they are used instead of being staged in
// LDS, so that graphs with many windows fit (only the record counters and
// ranks stay in LDS).
template <typename T, int SCHED, int NT, bool GT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_round(DiArgs<T> a, int r,
                                                                                  int mode) {
  constexpr int kRT = NT;
  constexpr int kNPT = kSuper / NT;  // nodes per thread per pass
  int ycol, b;  // vector column of the launch, window
  xcd_window(a.nb, &ycol, &b);
  const int vb = a.vmap ? a.vmap[ycol] : ycol;  // vector (0 for a single solve)
  if (a.vround) r = a.vround[vb];
  const double d = a.vd ? a.vd[vb] : a.d;
  const double tol = a.vtol ? a.vtol[vb] : a.tol;
  Ctl* ctl = a.ctl + vb;
  T* const Fv = a.F + (int64_t)vb * a.n;
  double* const Hv = a.H + (int64_t)vb * a.n;
  Slot* const slots = a.slots + (int64_t)vb * 3 * kSlots;
  const int64_t nb2 = (int64_t)a.nb * a.nb;

  extern __shared__ __align__(16) unsigned char smem[];
  const int W = 1 << a.wlog;
  const int nb = a.nb;
  double* win = reinterpret_cast<double*>(smem);  // [W]
  int64_t* s_base = nullptr;                       // [nb] record base per destination (not GT)
  int32_t* s_pre;                                  // [nb+1] fold prefix, then ranks
  int32_t* s_soff = nullptr;                       // [nb] fold offsets per source (not GT)
  int32_t* s_cap = nullptr;                        // [nb] capacity per destination (not GT)
  // per node of the window: 0 not taken, 1 taken and not yet expanded, 2 expanded
  uint8_t* s_state;  // [W]
  if constexpr (GT) {
    s_pre = reinterpret_cast<int32_t*>(win + W);
    s_state = reinterpret_cast<uint8_t*>(s_pre + (nb + 1));
  } else {
    s_base = reinterpret_cast<int64_t*>(win + W);
    s_pre = reinterpret_cast<int32_t*>(s_base + nb);
    s_soff = s_pre + (nb + 1);
    s_cap = s_soff + nb;
    s_state = reinterpret_cast<uint8_t*>(s_cap + nb);
  }
  __shared__ int32_t s_beo[kSuper + 1];
  __shared__ int64_t s_brow[kSuper];
  __shared__ double s_bsh[kSuper];
  __shared__ double s_red[block_reduce_k_scratch<NT, kSums>()];
  __shared__ long long s_scr[2 * (kRT / 64)];
  __shared__ int s_lp;

  const int64_t j0 = (int64_t)b << a.wlog;
  const int wn = (int)min((int64_t)W, a.n - j0);
  const int tid = threadIdx.x;

  // Every load that does not depend on this round's decisions is issued
  // before the first wait: the stop flag, round r-1's sums, this window's
  // fluid, its incoming record counts and the tables of its outgoing segments.
  // (a plain load of a uniform address, so a scalar one: waiting for it does
  // not wait for the vector loads; a stop recorded by this very launch reads
  // either way as "not earlier")
  const int sr = ctl->stop_round;
  const Slot* P = slots + ((r + 2) % 3) * kSlots;  // set (r-1) % 3
  // These loads use clamped indices and no branch (the values past the ends
  // are dropped later), so that none of them waits for another: a load in a
  // branch whose value is used in it is followed by its own wait.
  const Slot p_own = P[min(tid, kSlots - 1)];  // round r-1's sums, slot tid
  constexpr int kWinPer = 4;  // window values prefetched per thread (the rest load later)
  T fv[kWinPer];
#pragma unroll
  for (int k = 0; k < kWinPer; ++k) fv[k] = Fv[j0 + min(tid + k * kRT, wn - 1)];
  const int was_active = a.active[(int64_t)vb * nb + b];
  int32_t* const cnt_in = a.cnt[(r - 1) & 1] + vb * nb2 + (int64_t)b * nb;
  // first pass over the windows (nb <= kRT usually)
  const int tw = min(tid, nb - 1);
  const int32_t c_own = cnt_in[tw];
  int32_t o_own = 0, cap_own = 0, sT_own = 0;
  int64_t bs_own = 0;
  if constexpr (!GT) {
    o_own = a.soff[(int64_t)b * nb + tw];
    bs_own = a.bstart[tw];
    sT_own = a.soffT[(int64_t)b * nb + tw];
    cap_own = a.capT[(int64_t)b * nb + tw];
  }

  // Launch r itself records stop_round = r-1; an earlier stop ends this
  // launch.  Its writes below are skipped and it returns after them, so that
  // the test does not hold back the loads above.
  const bool ended = sr >= 0 && sr < r - 1;

  // 1. Decisions from round r-1's partial sums (identical in every workgroup).
  double theta = a.theta0;
  bool stop = mode == 1;
  if (r >= 1) {
    if (b == 0 && tid < kSlots && !ended) {  // set (r+1) % 3 is next used by launch r+1
      Slot* z = slots + ((r + 1) % 3) * kSlots + tid;
#pragma unroll
      for (int f = 0; f < kSums; ++f) z->sum[f] = 0.0;
      z->mrem = 0;
    }
    const bool mine = tid < kSlots;
    double v[kSums];  // nf, snd, sd, ssc, nnz, taken, edges
#pragma unroll
    for (int f = 0; f < kSums; ++f) v[f] = mine ? p_own.sum[f] : 0.0;
    double mrem_prev = mine ? __longlong_as_double((long long)p_own.mrem) : 0.0;
    block_reduce_k<kRT, kSums, true>(v, mrem_prev, s_red);
    const double nf = v[0], snd = v[1], sd = v[2], ssc = v[3], nnz = v[4], taken = v[5],
                 edges = v[6];
    int reason = 0;
    if (!isfinite(nf)) reason = 2;
    else if (nf < tol) reason = 1;
    else if ((int64_t)r >= a.max_rounds) reason = 3;
    if (reason) stop = true;
    // Remaining fluid after round r-1's pushes, in exact arithmetic: the
    // non-dangling senders keep d of what they send, the dangling ones none.
    const double R = nf - (1.0 - d) * snd - sd;
    // theta_r: c times the mean score of the nodes holding fluid, scaled by
    // the predicted decay of the total fluid.  After a round that took
    // nothing, fall back to the largest untaken score (at least the mean,
    // so the Lemma of Section 3.1 keeps its progress guarantee).
    theta = nnz > 0 ? a.c * (ssc / nnz) * (nf > 0 ? R / nf : 0.0) : 0.0;
    if (taken == 0 && theta > mrem_prev) theta = mrem_prev;
    if (b == 0 && tid == 0 && !ended) {
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

  if (ended) return;

  // 2. Window fluid (fp64 in LDS) plus the pushes of round r-1.
#pragma unroll
  for (int k = 0; k < kWinPer; ++k) {
    const int q = tid + k * kRT;
    if (q < wn) win[q] = (double)fv[k];
  }
  // the rest of a large window, kWinPer values per thread at a time
  for (int q0 = tid + kWinPer * kRT; q0 < wn; q0 += kWinPer * kRT) {
    T fr[kWinPer];
#pragma unroll
    for (int k = 0; k < kWinPer; ++k) fr[k] = Fv[j0 + min(q0 + k * kRT, wn - 1)];
    // (this loop runs only when W > kWinPer * kRT: W / kRT is then a power
    // of two of at least 8, a multiple of kWinPer, so every q is inside the
    // window; entries past wn are written as zeros, read by nothing as fluid)
#pragma unroll
    for (int k = 0; k < kWinPer; ++k) {
      const int q = q0 + k * kRT;
      win[q] = q < wn ? (double)fr[k] : 0.0;
    }
  }
  if (tid < nb) {
    s_pre[tid] = r >= 1 ? c_own : 0;
    if constexpr (!GT) {
      s_soff[tid] = r >= 1 ? o_own : 0;
      s_base[tid] = bs_own + sT_own;
      s_cap[tid] = cap_own;
    }
  }
  // the rest of the windows, two per thread at a time (loads first)
  for (int s0 = tid + kRT; s0 < nb; s0 += 2 * kRT) {
    int32_t c2[2], o2[2] = {0, 0}, t2[2] = {0, 0}, k2[2] = {0, 0};
    int64_t b2[2] = {0, 0};
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int sc = min(s0 + u * kRT, nb - 1);
      c2[u] = cnt_in[sc];
      if constexpr (!GT) {
        o2[u] = a.soff[(int64_t)b * nb + sc];
        b2[u] = a.bstart[sc];
        t2[u] = a.soffT[(int64_t)b * nb + sc];
        k2[u] = a.capT[(int64_t)b * nb + sc];
      }
    }
    // (a clamped entry is written again with its own values: no branch)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int s = min(s0 + u * kRT, nb - 1);
      s_pre[s] = r >= 1 ? c2[u] : 0;
      if constexpr (!GT) {
        s_soff[s] = r >= 1 ? o2[u] : 0;
        s_base[s] = b2[u] + t2[u];
        s_cap[s] = k2[u];
      }
    }
  }
  wg_barrier<true>();
  long long total = 0;  // records addressed to this window in round r-1
  if (r >= 1) total = lds_exscan<kRT, true>(s_pre, nb, s_scr);
  if (total == 0 && !was_active) return;  // nothing held, nothing arrived: nothing to send
  if (total > 0) {
    const PairT<T>* pr = a.pairs[(r - 1) & 1] + (int64_t)vb * a.mrec;
    const int64_t base = a.bstart[b];
    // offset of segment (s -> this window) within the window's record region
    auto seg_off = [&](int s) -> int64_t {
      if constexpr (GT) return a.soff[(int64_t)b * nb + s];
      else return s_soff[s];
    };
    // Each thread takes kRun consecutive records: one search for the segment
    // of the first, then a forward walk over the segment boundaries.
    for (long long i0 = (long long)tid * kRun; i0 < total; i0 += (long long)kRT * kRun) {
      int s = upper_idx(s_pre, nb, i0);
      long long nxt = s + 1 < nb ? s_pre[s + 1] : total;
      int64_t sb = base + seg_off(s) - s_pre[s];  // record index = sb + i within segment s
      int64_t idx[kRun];
#pragma unroll
      for (int u = 0; u < kRun; ++u) {
        const long long i = i0 + u;
        idx[u] = -1;
        if (i < total) {
          while (i >= nxt) {
            ++s;
            nxt = s + 1 < nb ? s_pre[s + 1] : total;
            sb = base + seg_off(s) - s_pre[s];
          }
          idx[u] = sb + i;
        }
      }
      PairT<T> e[kRun];
#pragma unroll
      for (int u = 0; u < kRun; ++u)
        if (idx[u] >= 0) e[u] = pr[idx[u]];
#pragma unroll
      for (int u = 0; u < kRun; ++u)
        if (idx[u] >= 0 && e[u].loc < (uint32_t)wn) atomicAdd(&win[e[u].loc], (double)e[u].val);
    }
    // The counts are consumed: clear the row for the launch that next writes it.
    for (int s = tid; s < nb; s += kRT) cnt_in[s] = 0;
  }
  wg_barrier<true>();
  if (stop) {
    for (int q = tid; q < wn; q += kRT) Fv[j0 + q] = (T)win[q];
    return;
  }

  // 3. Take and expand, one tile of kRT nodes at a time.
  if (tid == 0) s_lp = 0;
  for (int w = tid; w < nb; w += kRT) s_pre[w] = 0;  // now: records written per destination
  wg_barrier<true>();
  int32_t* const cnt_out = a.cnt[r & 1] + vb * nb2;  // destination-major, non-zero entries only
  PairT<T>* out = a.pairs[r & 1] + (int64_t)vb * a.mrec;
  const uint32_t wmask = (uint32_t)W - 1u;
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};  // nf, snd, sd, ssc, nnz, taken, edges
  double mrem = 0.0;  // the largest untaken score of this window
  // A. Decide for every node of the window (LDS only) before any push, so a
  //    round takes one set S (reading 5) even though pushes that stay inside
  //    the window are applied to its LDS copy at once.  Bit k of tbits: this
  //    thread's k-th node was taken; s_chunk: taken nodes per 64-node chunk.
  int32_t* const s_chunk = s_beo;  // [W/64], free until the first pass
  // the taken list: [W] after the state bytes when the launch has room for
  // it, else [kSuper] in the staging area (free until the first pass's staging)
  uint16_t* const s_list = a.wlist == 1 ? reinterpret_cast<uint16_t*>(s_state + W)
                                        : reinterpret_cast<uint16_t*>(s_bsh);
  const int list_cap = a.wlist == 1 ? W : a.wlist == 0 ? kSuper : 0;
  uint32_t tbits = 0;
  // kDec nodes per thread at a time, so that their degree loads are in
  // flight together (one wait per step, not per node)
  constexpr int kDec = 4;
  for (int q0 = tid, k0 = 0; q0 < W; q0 += kDec * kRT, k0 += kDec) {
    double fq[kDec];
    int dg[kDec], in[kDec];
#pragma unroll
    for (int u = 0; u < kDec; ++u) {
      const int q = q0 + u * kRT;
      fq[u] = q < wn ? win[q] : 0.0;
      // unconditional loads (a clamped index past the window's end): no
      // branch separates them, so they are all issued before the first wait
      const int64_t j = j0 + min(q, wn - 1);
      dg[u] = -1;
      in[u] = 0;
      if (SCHED != DI_SCHED_MEAN) dg[u] = a.deg[j];
      if (SCHED == DI_SCHED_OP) in[u] = a.indeg[j];
    }
#pragma unroll
    for (int u = 0; u < kDec; ++u) {
      const int q = q0 + u * kRT;
      if (q >= W) break;  // uniform in a wave
      // Fluid may be signed after an update of the graph (Section 3.2): the
      // threshold and the residual use |F_i|.
      const double f = fq[u], af = fabs(f);
      uint8_t st = 0;
      if (af > 0.0) {
        acc[0] += af;
        acc[4] += 1.0;
        const double sc = node_score<SCHED>(af, dg[u], in[u]);
        acc[3] += sc;
        if (sc >= theta) st = 1;
        else mrem = fmax(mrem, sc);
      } else if (f != f) {
        acc[0] = NAN;
      }
      s_state[q] = st;
      if (W > kSuper) {  // uniform: a list can save passes only then
        tbits |= (uint32_t)st << (k0 + u);
        const unsigned long long m = __ballot(st != 0);
        if ((tid & 63) == 0) s_chunk[q >> 6] = __popcll(m);
      }
    }
  }
  wg_barrier<true>();
  // When the list can hold them, list the taken nodes in node order (chunk
  // offsets plus the rank within the chunk) and run the passes over the list;
  // otherwise every pass walks kSuper consecutive nodes.
  // (a window of at most kSuper nodes is one pass either way: no list)
  const long long ntk = W > kSuper ? lds_exscan<kRT, true>(s_chunk, W >> 6, s_scr) : 0;
  const bool use_list = W > kSuper && ntk <= list_cap;
  if (use_list && ntk > 0) {
    for (int q = tid, k = 0; q < W; q += kRT, ++k) {
      const bool t = (tbits >> k) & 1u;
      const unsigned long long m = __ballot(t);
      const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
      if (t) s_list[s_chunk[q >> 6] + rank] = (uint16_t)q;
    }
    wg_barrier<true>();
  }
  const int tlim = use_list ? (int)ntk : wn;
  int local_push = 0;  // some push stayed inside the window (its fluid is in LDS)
  for (int t0 = 0; t0 < tlim; t0 += kSuper) {
    // B. Take the pass's nodes of S: load their link ranges and histories.
    double f[kNPT];
    bool tk[kNPT];
    int qs[kNPT];
#pragma unroll
    for (int u = 0; u < kNPT; ++u) {
      const int i = t0 + tid + u * kRT;
      if (use_list) {
        tk[u] = i < tlim;
        qs[u] = tk[u] ? (int)s_list[i] : 0;
      } else {
        qs[u] = i;
        tk[u] = i < wn && s_state[i] == 1;
      }
      f[u] = tk[u] ? win[qs[u]] : 0.0;
    }
    int64_t rs[kNPT];
    int dgs[kNPT];
    double h[kNPT];
#pragma unroll
    for (int u = 0; u < kNPT; ++u) {
      if (!tk[u]) continue;
      const int64_t j = j0 + qs[u];
      rs[u] = a.row_ptr[j];
      dgs[u] = a.deg[j];
      h[u] = Hv[j];
    }
    long long npush = 0, nedge = 0;
#pragma unroll
    for (int u = 0; u < kNPT; ++u) {
      if (!tk[u]) continue;
      const int q = qs[u];
      Hv[j0 + q] = h[u] + f[u];
      win[q] = 0.0;
      s_state[q] = 2;
      if (a.trace && r < a.trace_rounds) a.trace[(int64_t)r * a.n + j0 + q] = 1;
      acc[5] += 1.0;
      if (dgs[u] > 0) {
        acc[1] += fabs(f[u]);
        ++npush;
        nedge += dgs[u];
      } else {
        acc[2] += fabs(f[u]);
      }
    }
    // C. Stage the pushing nodes (thread-major order) with their link offsets.
    long long slot = 0, eoff = 0, ntile = 0, etile = 0;
    block_exscan2<kRT, true>(npush, nedge, s_scr, &slot, &eoff, &ntile, &etile);
    if (ntile == 0) continue;  // uniform
#pragma unroll
    for (int u = 0; u < kNPT; ++u) {
      if (!tk[u] || dgs[u] == 0) continue;
      const long long dg = dgs[u];
      s_beo[slot] = (int32_t)eoff;
      s_brow[slot] = rs[u];
      s_bsh[slot] = a.weighted ? d * f[u] : d * f[u] / (double)dg;
      ++slot;
      eoff += dg;
    }
    wg_barrier<true>();
    // D. Push every staged link: each thread takes kRun consecutive links,
    //    one search for the node of the first, then a forward walk.  A link
    //    into this window whose target is not an S node still to be expanded
    //    adds to the LDS copy directly (the fluid F holds for the next round,
    //    rounded like a record); every other link writes a record.
    const int bcount = (int)ntile;
    for (long long t00 = (long long)tid * kRun; t00 < etile; t00 += (long long)kRT * kRun) {
      int k = upper_idx(s_beo, bcount, t00);
      long long nxt = k + 1 < bcount ? s_beo[k + 1] : etile;
      int64_t lb = s_brow[k] - s_beo[k];  // link index = lb + t for node k
      double sh = s_bsh[k];
      int64_t e[kRun];
      double v[kRun];
#pragma unroll
      for (int u = 0; u < kRun; ++u) {
        const long long t = t00 + u;
        e[u] = -1;
        if (t < etile) {
          while (t >= nxt) {
            ++k;
            nxt = k + 1 < bcount ? s_beo[k + 1] : etile;
            lb = s_brow[k] - s_beo[k];
            sh = s_bsh[k];
          }
          e[u] = lb + t;
          v[u] = sh;
        }
      }
      uint32_t dst[kRun];
#pragma unroll
      for (int u = 0; u < kRun; ++u)
        if (e[u] >= 0) {
          dst[u] = (uint32_t)a.col[e[u]];
          if (a.weighted) v[u] *= a.w[e[u]];
        }
#pragma unroll
      for (int u = 0; u < kRun; ++u) {
        if (e[u] < 0) continue;
        const int w = (int)(dst[u] >> a.wlog);
        if (w == b && s_state[dst[u] & wmask] != 1) {
          atomicAdd(&win[dst[u] & wmask], (double)(T)v[u]);
          local_push = 1;
          continue;
        }
        int cap;
        int64_t wbase;  // first record of segment (this window -> w)
        if constexpr (GT) {
          const int64_t q = (int64_t)b * nb + w;
          cap = a.capT[q];
          wbase = a.bstart[w] + a.soffT[q];
        } else {
          cap = s_cap[w];
          wbase = s_base[w];
        }
        const int rank = atomicAdd(&s_pre[w], 1);
        if (rank < cap) {
          PairT<T> pr;
          memset(&pr, 0, sizeof(pr));
          pr.loc = dst[u] & wmask;
          pr.val = (T)v[u];
          out[wbase + rank] = pr;
        } else {
          atomicOr(&ctl->err, 2);
        }
      }
    }
    acc[6] += (double)etile;  // uniform: counted once below (thread 0 only)
    wg_barrier<true>();
  }
  for (int w = tid; w < nb; w += kRT)
    if (s_pre[w] > 0) {
      int cap;
      if constexpr (GT) cap = a.capT[(int64_t)b * nb + w];
      else cap = s_cap[w];
      cnt_out[(int64_t)w * nb + b] = min(s_pre[w], cap);
    }
  for (int q = tid; q < wn; q += kRT) Fv[j0 + q] = (T)win[q];

  // 4. This window's sums, added into its slot.
  if (local_push) s_lp = 1;
  wg_barrier<true>();
  const int local_any = s_lp;
  const double edges = acc[6];
  acc[6] = 0.0;
  block_reduce_k<kRT, kSums, true>(acc, mrem, s_red);
  if (tid == 0) {
    acc[6] = edges;
    // the window stays active while some node keeps fluid: untaken, or
    // pushed inside the window this round
    a.active[(int64_t)vb * nb + b] = (acc[4] > acc[5] || local_any) ? 1 : 0;
    Slot* sl = slots + (r % 3) * kSlots + (b % kSlots);
#pragma unroll
    for (int f = 0; f < kSums; ++f)
      if (acc[f] != 0.0) unsafeAtomicAdd(&sl->sum[f], acc[f]);
    if (mrem > 0.0) atomicMax(&sl->mrem, (unsigned long long)__double_as_longlong(mrem));
  }
}

// Flush sums of vector blockIdx.y: sum(H+F), sum(H), sum|F|, sum over
// dangling nodes of H, sum(F), as per-block partials spread over 256 slots.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_flush_sum(DiArgs<T> a) {
  __shared__ double s_red[kBlock / 64];
  const int vb = a.vmap ? a.vmap[blockIdx.y] : blockIdx.y;
  const T* F = a.F + (int64_t)vb * a.n;
  const double* H = a.H + (int64_t)vb * a.n;
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * kBlock) {
    const double h = H[i], f = (double)F[i];
    s0 += h + f;
    s1 += h;
    s2 += fabs(f);
    if (a.deg[i] == 0) s3 += h;
    s4 += f;
  }
  s0 = block_sum(s0, s_red);
  s1 = block_sum(s1, s_red);
  s2 = block_sum(s2, s_red);
  s3 = block_sum(s3, s_red);
  s4 = block_sum(s4, s_red);
  if (threadIdx.x == 0) {
    double* slot = a.flacc + (int64_t)vb * kFlushAcc + kFlushSums * (blockIdx.x % kFlushSlots);
    unsafeAtomicAdd(slot + 0, s0);
    unsafeAtomicAdd(slot + 1, s1);
    unsafeAtomicAdd(slot + 2, s2);
    unsafeAtomicAdd(slot + 3, s3);
    unsafeAtomicAdd(slot + 4, s4);
  }
}

// Reduce the 256 flush slots of vector blockIdx.x into its ctl->fl.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_flush_reduce(DiArgs<T> a) {
  __shared__ double s_red[kBlock / 64];
  const int vb = a.vmap ? a.vmap[blockIdx.x] : blockIdx.x;
  const double* acc = a.flacc + (int64_t)vb * kFlushAcc;
  for (int k = 0; k < kFlushSums; ++k) {
    const double v = block_sum(acc[kFlushSums * threadIdx.x + k], s_red);
    if (threadIdx.x == 0) a.ctl[vb].fl[k] = v;
  }
}

// x = (H + F) / sum(H + F)  (renormalisation of Section 3.3), or H + F.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_flush_write(DiArgs<T> a, double* __restrict__ x,
                                                        int normalize) {
  const int vb = a.vmap ? a.vmap[blockIdx.y] : blockIdx.y;
  const T* F = a.F + (int64_t)vb * a.n;
  const double* H = a.H + (int64_t)vb * a.n;
  const double s = normalize ? a.ctl[vb].fl[0] : 1.0;
  double* xv = x + (int64_t)vb * a.n;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * kBlock)
    xv[i] = (H[i] + (double)F[i]) / s;
}

__global__ void k_zero(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// --------------------------------------------------------------- workspace

// Device bytes one vector of a solve holds (state, records, counts, sums).
static int64_t bytes_per_vector(int64_t n, int64_t m, int nb, int precision) {
  const int64_t fs = precision == DI_FP64 ? 8 : 4, ps = precision == DI_FP64 ? 16 : 8;
  return n * (fs + 8) + 2 * std::max<int64_t>(m, 1) * ps + 2 * (int64_t)nb * nb * 4 +
         3 * kSlots * (int64_t)sizeof(Slot) + nb + (int64_t)sizeof(Ctl) + kFlushAcc * 8;
}

// Workspace for nvec vectors of window 2^wlog (single solves use nvec = 1).
static Workspace* make_workspace(Graph* g, int precision, int wlog, int nvec, bool gt) {
  auto* ws = new Workspace();
  try {
    const int64_t n = g->n, m = g->m, mrec = std::max<int64_t>(m, 1);
    const size_t fs = precision == DI_FP64 ? 8 : 4;
    const int nb = (int)((n + (1ll << wlog) - 1) >> wlog);
    const int64_t nb2 = (int64_t)nb * nb;
    ws->precision = precision;
    ws->wlog = wlog;
    ws->gt = gt;
    ws->nb = nb;
    ws->nvec = nvec;
    ws->n = n;
    ws->m = m;
    ws->F.alloc(nvec * n * fs);
    ws->H.alloc(nvec * n * 8);
    if (nvec == 1) {
      ws->v.alloc(n * 8);
      ws->x.alloc(n * 8);
    }
    ws->bstart.alloc((nb + 1) * 8);
    ws->ctl.alloc(nvec * sizeof(Ctl));
    ws->flacc.alloc(nvec * kFlushAcc * 8);
    ws->active.alloc(nvec * (int64_t)nb);
    for (int k = 0; k < 2; ++k) {
      ws->pairs[k].alloc(nvec * mrec * (precision == DI_FP64 ? 16 : 8));
      ws->cnt[k].alloc(nvec * nb2 * 4);
    }
    ws->slots.alloc(nvec * 3 * kSlots * sizeof(Slot));
    ws->soff.alloc(nb2 * 4);
    ws->soffT.alloc(nb2 * 4);
    ws->capT.alloc(nb2 * 4);
    ws->hctl.alloc(nvec * sizeof(Ctl));
    ws->hctl2.alloc(nvec * sizeof(Ctl));
    for (hipEvent_t& e : ws->ev) DI_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    DevBuf E, err;
    E.alloc(nb2 * 4);
    err.alloc(sizeof(int));
    DI_HIP(hipMemset(E.p, 0, nb2 * 4));
    DI_HIP(hipMemset(err.p, 0, sizeof(int)));
    const int gn = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
    k_window_links<<<gn, 256>>>(n, wlog, nb, g->row_ptr.as<int64_t>(), g->col.as<int32_t>(),
                                E.as<int32_t>());
    DI_HIP(hipGetLastError());
    k_segments<<<nb, kBlock>>>(n, wlog, nb, g->in_ptr.as<int64_t>(), E.as<int32_t>(),
                               ws->soff.as<int32_t>(), ws->bstart.as<int64_t>(), err.as<int>());
    DI_HIP(hipGetLastError());
    const int gt = (int)std::max<int64_t>(1, std::min<int64_t>((nb2 + 255) / 256, 4096));
    k_transpose<<<gt, 256>>>(nb, E.as<int32_t>(), ws->soff.as<int32_t>(), ws->soffT.as<int32_t>(),
                             ws->capT.as<int32_t>());
    DI_HIP(hipGetLastError());
    DI_HIP(hipDeviceSynchronize());
    int h_err = 0;
    DI_HIP(hipMemcpy(&h_err, err.p, sizeof(int), hipMemcpyDeviceToHost));
    if (h_err) {
      set_error("window segment tables do not match the in-link counts");
      throw Fail{DI_EDEVICE};
    }
  } catch (...) {
    delete ws;
    throw;
  }
  return ws;
}

Workspace* acquire_workspace(Graph* g, int precision, int wlog, bool gt) {
  {
    std::lock_guard<std::mutex> lk(g->ws_mu);
    for (size_t i = 0; i < g->ws_free.size(); ++i) {
      Workspace* ws = g->ws_free[i];
      if (ws->precision == precision && ws->wlog == wlog && ws->gt == gt && ws->nvec == 1) {
        g->ws_free.erase(g->ws_free.begin() + i);
        return ws;
      }
    }
  }
  return make_workspace(g, precision, wlog, 1, gt);
}

// A workspace for at least nvec vectors (batches); reuses a cached one.
static Workspace* acquire_batch_workspace(Graph* g, int precision, int wlog, bool gt, int nvec) {
  {
    std::lock_guard<std::mutex> lk(g->ws_mu);
    for (size_t i = 0; i < g->ws_free.size(); ++i) {
      Workspace* ws = g->ws_free[i];
      if (ws->precision == precision && ws->wlog == wlog && ws->gt == gt && ws->nvec >= nvec &&
          ws->nvec > 1) {
        g->ws_free.erase(g->ws_free.begin() + i);
        return ws;
      }
    }
    // drop cached batch workspaces of other shapes before allocating a large one
    for (size_t i = 0; i < g->ws_free.size();) {
      if (g->ws_free[i]->nvec > 1) {
        delete g->ws_free[i];
        g->ws_free.erase(g->ws_free.begin() + i);
      } else {
        ++i;
      }
    }
  }
  return make_workspace(g, precision, wlog, nvec, gt);
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
                           int64_t max_rounds, T* F, double* H, int nvec) {
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
  a.mrec = std::max<int64_t>(g->m, 1);
  for (int k = 0; k < 2; ++k) {
    a.pairs[k] = ws->pairs[k].as<PairT<T>>();
    a.cnt[k] = ws->cnt[k].as<int32_t>();
  }
  a.slots = ws->slots.as<Slot>();
  a.active = ws->active.as<uint8_t>();
  a.ctl = ws->ctl.as<Ctl>();
  a.flacc = ws->flacc.as<double>();
  a.gt = ws->gt ? 1 : 0;
  a.nvec = nvec;
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

// Diagnostic switch (di_set_taken_list): 0 forces passes over consecutive nodes.
static std::atomic<int> g_taken_list{1};

template <typename T, int SCHED, int NT, bool GT = false>
static void launch_round_t(const DiArgs<T>& a0, int r, int mode, hipStream_t s, LaunchTimer* lt) {
  DiArgs<T> a = a0;
  size_t smem = round_lds_bytes(a.wlog, a.nb, GT);
  // Dynamic LDS may use what the static part leaves of the workgroup limit
  // (set once per kernel instance; thread-safe initialisation).
  // (The LDS limit of a workgroup is the LDS of a CU on gfx950.)
  static size_t lds_cu = 0;
  static const size_t dyn_limit = [] {
    hipFuncAttributes fa;
    DI_HIP(hipFuncGetAttributes(&fa, (const void*)k_round<T, SCHED, NT, GT>));
    int dev = 0, lim = 0;
    DI_HIP(hipGetDevice(&dev));
    DI_HIP(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const size_t dl = (size_t)lim - fa.sharedSizeBytes;
    DI_HIP(hipFuncSetAttribute((const void*)k_round<T, SCHED, NT, GT>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)dl));
    lds_cu = (size_t)lim;
    return dl;
  }();
  DI_REQUIRE(smem <= dyn_limit, "window tables exceed the LDS available to the round kernel");
  // A taken list of the whole window (2 bytes per node) when it fits and
  // costs no workgroups per CU (registers allow two 512-thread or one
  // 1024-thread workgroup).
  const size_t stat = lds_cu - dyn_limit;  // static LDS of this instance
  auto per_cu = [&](size_t dyn) {
    return std::min<size_t>(NT == 512 ? 2 : 1, lds_cu / (dyn + stat));
  };
  const size_t list_bytes = (size_t)2 << a.wlog;
  if (!g_taken_list.load(std::memory_order_relaxed)) {
    a.wlist = 2;
  } else {
    a.wlist = smem + list_bytes <= dyn_limit && per_cu(smem + list_bytes) >= per_cu(smem) ? 1 : 0;
    if (a.wlist == 1) smem += list_bytes;
  }
  const dim3 grid(a.nb, a.nvec);
  if (lt && lt->on) {
    // The runtime stamps the kernel's own begin/end into the event pair.
    hipEvent_t e0, e1;
    lt->next(&e0, &e1);
    hipExtLaunchKernelGGL(k_round<T, SCHED, NT, GT>, grid, dim3(NT), smem, s, e0, e1, 0, a, r,
                          mode);
  } else {
    k_round<T, SCHED, NT, GT><<<grid, NT, smem, s>>>(a, r, mode);
  }
  DI_HIP(hipGetLastError());
}

template <typename T>
static void launch_round(const DiArgs<T>& a, int sched, int r, int mode, hipStream_t s,
                         LaunchTimer* lt = nullptr) {
  if (a.gt) {  // segment tables in global memory: 1024-thread instances only
    switch (sched) {
      case DI_SCHED_OP2:
        launch_round_t<T, DI_SCHED_OP2, 1024, true>(a, r, mode, s, lt);
        break;
      case DI_SCHED_OP:
        launch_round_t<T, DI_SCHED_OP, 1024, true>(a, r, mode, s, lt);
        break;
      default:
        launch_round_t<T, DI_SCHED_MEAN, 1024, true>(a, r, mode, s, lt);
        break;
    }
    return;
  }
  switch (sched) {
    case DI_SCHED_OP2:
      if (a.threads == 1024) launch_round_t<T, DI_SCHED_OP2, 1024>(a, r, mode, s, lt);
      else launch_round_t<T, DI_SCHED_OP2, kRoundThreads>(a, r, mode, s, lt);
      break;
    case DI_SCHED_OP:
      if (a.threads == 1024) launch_round_t<T, DI_SCHED_OP, 1024>(a, r, mode, s, lt);
      else launch_round_t<T, DI_SCHED_OP, kRoundThreads>(a, r, mode, s, lt);
      break;
    default:
      if (a.threads == 1024) launch_round_t<T, DI_SCHED_MEAN, 1024>(a, r, mode, s, lt);
      else launch_round_t<T, DI_SCHED_MEAN, kRoundThreads>(a, r, mode, s, lt);
      break;
  }
}

static void read_ctl(Workspace* ws, int nvec, hipStream_t s) {
  DI_HIP(hipMemcpyAsync(ws->hctl.p, ws->ctl.p, nvec * sizeof(Ctl), hipMemcpyDeviceToHost, s));
  DI_HIP(hipStreamSynchronize(s));
}

// Launches rounds until every vector's launch has recorded its stop (that
// launch also folds the last pushes, so (F, H) is again a state of the
// recurrences).  Rounds go out in chunks, each followed by an asynchronous
// copy of the control blocks; while the host waits for one chunk's copy the
// next chunk is already queued, so the device never idles on the host.  Chunk
// sizes follow the observed per-round decay of ||F||_1; rounds launched after
// the stop return at once.
template <typename T>
static void run_rounds(const DiArgs<T>& a, Workspace* ws, int sched, int check_every,
                       hipStream_t s, LaunchTimer* lt) {
  Ctl* const hb[2] = {ws->hctl.as<Ctl>(), ws->hctl2.as<Ctl>()};
  const size_t cbytes = (size_t)a.nvec * sizeof(Ctl);
  int r = 0;
  int obs[2] = {0, 0};  // rounds launched before each buffer's copy
  auto launch_chunk = [&](int k, int slot) {
    for (int i = 0; i < k; ++i) launch_round(a, sched, r++, 0, s, lt);
    DI_HIP(hipMemcpyAsync(hb[slot], ws->ctl.p, cbytes, hipMemcpyDeviceToHost, s));
    DI_HIP(hipEventRecord(ws->ev[slot], s));
    obs[slot] = r;
  };
  const int fixed = check_every > 0 ? check_every : 0;
  int next = fixed ? fixed : 8;
  int cur = 0;
  launch_chunk(next, cur);
  double nf_prev = -1.0;
  int r_prev = 0;
  for (;;) {
    launch_chunk(next, 1 - cur);  // queued before looking at the previous chunk
    DI_HIP(hipEventSynchronize(ws->ev[cur]));
    const Ctl* h = hb[cur];
    double nf_max = 0.0;
    bool all = true;
    for (int v = 0; v < a.nvec; ++v) {
      if (h[v].stop_round < 0) {
        all = false;
        nf_max = std::max(nf_max, h[v].nf);
      }
    }
    if (all) break;
    if (!fixed) {
      // Rounds still needed after the observed one, predicted from the decay of
      // ||F||_1 of the slowest vector, minus those already queued behind it.
      int need = 8;
      if (nf_prev > 0.0 && nf_max > 0.0 && nf_max < nf_prev && obs[cur] > r_prev) {
        const double q = std::pow(nf_max / nf_prev, 1.0 / (obs[cur] - r_prev));
        if (q > 0.0 && q < 1.0)
          need = (int)std::ceil(std::log(a.tol / nf_max) / std::log(q) * 1.05) + 1;
      }
      nf_prev = nf_max;
      r_prev = obs[cur];
      next = std::max(2, std::min(need - (r - obs[cur]), 64));
    }
    cur = 1 - cur;
  }
}

// ------------------------------------------------- whole graph in one window

// Small graphs (n <= DI_SMALL_MAX_NODES): the whole fluid vector lives in the
// LDS of one 1024-thread workgroup (fp64), which runs every round itself,
// rounds separated by barriers instead of launches.  Round r: the fresh fp64
// ||F_r||_1 (Theorem 2 stop), the mean and the largest score of the nodes
// holding fluid; theta_r = c times that mean (never above the largest score,
// so every round takes a node).  Every node reaching theta_r is taken
// (H_i += F_i, F_i = 0) and, if it has out-links, listed in a frontier list in
// global memory (first link, degree, share), all before any push; the list is
// then pushed a chunk at a time through LDS staging, d F_i p(j,i) added into
// the LDS fluid (each push rounded to the fluid type first, as a stored record
// would be).  In fp32 the fluid is rounded to fp32 at the end of each round, as
// a stored F would be.
constexpr int kSmallThreads = 512;
constexpr int kSmallP = 4;  // frontier entries per thread per chunk, at most

struct FrontEntry {
  int64_t row;   // first out-link
  double share;  // d F_i / outdeg_i (weighted graphs: d F_i)
  int32_t deg;
  int32_t pad;
};

constexpr int kSmallRun = 8;  // consecutive links per thread per step of the push

template <typename T, int SCHED>
__global__ __launch_bounds__(kSmallThreads) void k_small(DiArgs<T> a, FrontEntry* __restrict__ front,
                                                         int chunk, int cache_deg) {
  constexpr int NT = kSmallThreads;
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = (int)a.n;
  double* f = reinterpret_cast<double*>(smem);                    // [n]
  int64_t* s_brow = reinterpret_cast<int64_t*>(f + n);            // [chunk]
  double* s_bsh = reinterpret_cast<double*>(s_brow + chunk);      // [chunk]
  int32_t* s_beo = reinterpret_cast<int32_t*>(s_bsh + chunk);     // [chunk + 1]
  int32_t* s_deg = s_beo + chunk + 1;                             // [n] when cache_deg
  __shared__ double s_red[block_reduce_k_scratch<NT, 4>()];
  __shared__ long long s_scr[2 * (NT / 64)];
  const int tid = threadIdx.x;
  const double d = a.d;
  const int P = chunk / NT;  // entries per thread per chunk
  if (cache_deg)
    for (int q = tid; q < n; q += NT) s_deg[q] = a.deg[q];
  auto degree = [&](int q) { return cache_deg ? s_deg[q] : a.deg[q]; };
  auto score = [&](int q, double af) {
    const int dg = SCHED != DI_SCHED_MEAN ? degree(q) : -1;
    return node_score<SCHED>(af, dg, SCHED == DI_SCHED_OP ? a.indeg[q] : 0);
  };
  // sums of the current fluid: ||F||_1, score sum, nodes holding fluid; max score
  double v[4], smax;
  auto sums = [&] {
    v[0] = v[1] = v[2] = v[3] = 0.0;
    smax = 0.0;
    for (int q = tid; q < n; q += NT) {
      const double af = fabs(f[q]);
      if (af > 0.0) {
        const double sc = score(q, af);
        v[0] += af;
        v[1] += sc;
        v[2] += 1.0;
        smax = fmax(smax, sc);
      } else if (f[q] != f[q]) {
        v[0] = NAN;
      }
    }
    block_reduce_k<NT, 4>(v, smax, s_red);
  };
  for (int q = tid; q < n; q += NT) f[q] = (double)a.F[q];
  __syncthreads();
  sums();
  long long nodes_total = 0, edges_total = 0, last_taken = 0, last_edges = 0;
  double theta = 0.0, nf = 0.0;
  int reason = 0;
  int64_t r = 0;
  for (;; ++r) {
    nf = v[0];
    if (!isfinite(nf)) reason = 2;
    else if (nf < a.tol) reason = 1;
    else if (r >= a.max_rounds) reason = 3;
    if (reason) break;  // uniform
    theta = fmin(a.c * v[1] / v[2], smax);
    // 1. take every node of S_r, all before any push: count this thread's
    //    pushing nodes and their links, place them (block scan), then take
    //    them and stage them -- straight into LDS when they fit one chunk,
    //    else into the frontier list
    long long mine = 0, mylinks = 0;
    for (int q = tid; q < n; q += NT) {
      const double af = fabs(f[q]);
      if (af > 0.0 && score(q, af) >= theta) {
        const int dg = degree(q);
        if (dg > 0) {
          ++mine;
          mylinks += dg;
        }
      }
    }
    long long pos = 0, eoff = 0, total = 0, etotal = 0;
    block_exscan2<NT>(mine, mylinks, s_scr, &pos, &eoff, &total, &etotal);
    const bool direct = total <= chunk;  // uniform
    double cnt[4] = {0.0, 0.0, 0.0, 0.0};  // taken, links
#pragma unroll 4
    for (int q = tid; q < n; q += NT) {
      const int64_t row = a.row_ptr[q];  // not behind the test: loads of several nodes overlap
      const double x = f[q], af = fabs(x);
      if (!(af > 0.0) || !(score(q, af) >= theta)) continue;
      const int dg = degree(q);
      f[q] = 0.0;
      unsafeAtomicAdd(&a.H[q], x);  // H_i += F_i (one writer per node; nothing waits on it)
      if (a.trace && r < a.trace_rounds) a.trace[r * a.n + q] = 1;
      cnt[0] += 1.0;
      cnt[1] += dg;
      if (dg > 0) {
        const double sh = a.weighted ? d * x : d * x / (double)dg;
        if (direct) {
          s_beo[pos] = (int32_t)eoff;
          s_brow[pos] = row;
          s_bsh[pos] = sh;
          eoff += dg;
        } else {
          FrontEntry e;
          e.row = row;
          e.share = sh;
          e.deg = dg;
          e.pad = 0;
          front[pos] = e;
        }
        ++pos;
      }
    }
    __syncthreads();  // the staging (or the list) and the zeroed fluid are complete
    // 2. push the staged nodes [0, cn) with their links [0, links)
    auto push = [&](int cn, long long links) {
      for (long long t00 = (long long)tid * kSmallRun; t00 < links;
           t00 += (long long)NT * kSmallRun) {
        int kk = upper_idx(s_beo, cn, t00);
        long long nxt = kk + 1 < cn ? s_beo[kk + 1] : links;
        int64_t lb = s_brow[kk] - s_beo[kk];
        double sh = s_bsh[kk];
        int64_t ei[kSmallRun];
        double pv[kSmallRun];
#pragma unroll
        for (int u = 0; u < kSmallRun; ++u) {
          const long long t = t00 + u;
          ei[u] = -1;
          if (t < links) {
            while (t >= nxt) {
              ++kk;
              nxt = kk + 1 < cn ? s_beo[kk + 1] : links;
              lb = s_brow[kk] - s_beo[kk];
              sh = s_bsh[kk];
            }
            ei[u] = lb + t;
            pv[u] = sh;
          }
        }
        int32_t dst[kSmallRun];
#pragma unroll
        for (int u = 0; u < kSmallRun; ++u)
          if (ei[u] >= 0) {
            dst[u] = a.col[ei[u]];
            if (a.weighted) pv[u] *= a.w[ei[u]];
          }
#pragma unroll
        for (int u = 0; u < kSmallRun; ++u)
          if (ei[u] >= 0) atomicAdd(&f[dst[u]], (double)(T)pv[u]);
      }
      __syncthreads();
    };
    if (direct) {
      if (total > 0) push((int)total, etotal);
    } else {
      // the list a chunk of P entries per thread at a time
      for (long long c0 = 0; c0 < total; c0 += chunk) {
        const int cn = (int)min((long long)chunk, total - c0);
        FrontEntry e[kSmallP];
        long long my_links = 0;
#pragma unroll
        for (int u = 0; u < kSmallP; ++u) {
          const int k = tid * P + u;
          e[u].deg = 0;
          if (u < P && k < cn) {
            e[u] = front[c0 + k];
            my_links += e[u].deg;
          }
        }
        long long lo = 0, links = 0;
        lo = block_exscan<NT>(my_links, s_scr, &links);
#pragma unroll
        for (int u = 0; u < kSmallP; ++u) {
          const int k = tid * P + u;
          if (u < P && k < cn) {
            s_beo[k] = (int32_t)lo;
            s_brow[k] = e[u].row;
            s_bsh[k] = e[u].share;
            lo += e[u].deg;
          }
        }
        __syncthreads();
        push(cn, links);
      }
    }
    // 3. the round's fluid as stored in the fluid type; the next round's sums
    if (!std::is_same<T, double>::value) {
      for (int q = tid; q < n; q += NT) f[q] = (double)(T)f[q];
      __syncthreads();
    }
    double unused = 0.0;
    block_reduce_k<NT, 4>(cnt, unused, s_red);
    last_taken = (long long)cnt[0];
    last_edges = (long long)cnt[1];
    nodes_total += last_taken;
    edges_total += last_edges;
    sums();
  }
  for (int q = tid; q < n; q += NT) a.F[q] = (T)f[q];
  if (tid == 0) {
    Ctl* c = a.ctl;
    c->stop_round = (int)r - 1;
    c->reason = reason;
    c->nf = nf;
    c->theta = theta;
    c->nodes_total = nodes_total;
    c->edges_total = edges_total;
    c->last_taken = last_taken;
    c->last_edges = last_edges;
  }
}

// LDS bytes of k_small for n nodes and a chunk of c frontier entries (plus
// the degrees when they are cached).
static size_t small_lds_bytes(int64_t n, int c, bool cache_deg = false) {
  return (size_t)n * 8 + (size_t)c * 16 + (size_t)(c + 1) * 4 + (cache_deg ? (size_t)n * 4 : 0);
}

template <typename T>
static void launch_small(const DiArgs<T>& a, Workspace* ws, int sched, hipStream_t s,
                         LaunchTimer* lt) {
  // the dynamic LDS limit of the kernel instances (set once): what the static
  // part leaves of the workgroup's 160 KiB
  static const size_t dyn_limit = [] {
    size_t lim = ~(size_t)0;
    auto one = [&](const void* k) {
      hipFuncAttributes fa;
      DI_HIP(hipFuncGetAttributes(&fa, k));
      int dev = 0, mx = 0;
      DI_HIP(hipGetDevice(&dev));
      DI_HIP(hipDeviceGetAttribute(&mx, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
      const size_t dl = (size_t)mx - fa.sharedSizeBytes;
      DI_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dl));
      lim = std::min(lim, dl);
    };
    one((const void*)k_small<T, DI_SCHED_MEAN>);
    one((const void*)k_small<T, DI_SCHED_OP2>);
    one((const void*)k_small<T, DI_SCHED_OP>);
    return lim;
  }();
  // largest chunk (a multiple of the block, at most kSmallP entries per thread)
  int chunk = kSmallP * kSmallThreads;
  while (chunk > kSmallThreads && small_lds_bytes(a.n, chunk) > dyn_limit) chunk -= kSmallThreads;
  DI_REQUIRE(small_lds_bytes(a.n, chunk) <= dyn_limit, "graph too large for the whole-graph window");
  // the degrees stay in LDS too when they fit beside a chunk of at least 1024
  int cache_deg = 0;
  for (int c = chunk; c >= std::min(chunk, 2 * kSmallThreads); c -= kSmallThreads)
    if (small_lds_bytes(a.n, c, true) <= dyn_limit) {
      chunk = c;
      cache_deg = 1;
      break;
    }
  const size_t smem = small_lds_bytes(a.n, chunk, cache_deg != 0);
  ws->front.alloc((size_t)a.n * sizeof(FrontEntry));
  FrontEntry* front = ws->front.as<FrontEntry>();
  auto go = [&](auto kern) {
    if (lt && lt->on) {
      hipEvent_t e0, e1;
      lt->next(&e0, &e1);
      hipExtLaunchKernelGGL(kern, dim3(1), dim3(kSmallThreads), smem, s, e0, e1, 0, a, front,
                            chunk, cache_deg);
    } else {
      kern<<<1, kSmallThreads, smem, s>>>(a, front, chunk, cache_deg);
    }
    DI_HIP(hipGetLastError());
  };
  if (sched == DI_SCHED_OP2) go(k_small<T, DI_SCHED_OP2>);
  else if (sched == DI_SCHED_OP) go(k_small<T, DI_SCHED_OP>);
  else go(k_small<T, DI_SCHED_MEAN>);
}

// ------------------------------------------- one launch for every round

// Graphs of at most kResMaxWindows windows: one cooperative launch runs every
// round of a single solve.  The workgroup of a window keeps the window's
// fluid and history (fp64), degrees, link offsets and, when they fit, its
// out-links in LDS for the whole solve; only what crosses windows goes
// through global memory: the records of cross-window pushes, their counts
// and the round sums.  Rounds are separated by a grid barrier instead of
// launches.  Round r computes what launch r of k_round computes (the same
// threshold and stop from the same sums, the same records and counts), so a
// round diffuses one set S (reading 5) and the stop is the fresh fp64
// ||F||_1 < tol of Theorem 2; in fp32 the fluid is rounded to fp32 at the end
// of each round, as a stored F would be.
constexpr int kResThreads = 256;
constexpr int kResMaxWindows = DI_PERSIST_MAX_WINDOWS;
constexpr int kResMaxWlog = 11;
constexpr int kResPass = 2 * kResThreads;  // taken nodes expanded per pass
constexpr int kResLinkCap = 24576;         // out-links of a window held in LDS, at most
constexpr int kResSpec = 8;                // speculative record reads per thread per round

// Grid barrier of co-resident workgroups: an arrival counter that grows by
// the number of workgroups every round (target = rounds so far x workgroups,
// both modulo 2^32).
// A wait longer than `limit` ticks of the constant-rate wall clock, or an
// abort seen while waiting, sets bit 4 of *err and returns false: every
// workgroup then leaves its loop at this or its next barrier.
__device__ bool grid_barrier(unsigned* bar, unsigned target, int* err, long long limit,
                             int* s_flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const long long t0 = wall_clock64();
    // (compared as a signed difference: correct across the counter's wrap)
    while ((int)(__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
      if ((__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 4) ||
          wall_clock64() - t0 > limit) {
        __hip_atomic_fetch_or(err, 4, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *s_flag = ok;
  }
  __syncthreads();
  return *s_flag != 0;
}

// LDS bytes of k_resident for 2^wlog-node windows, nb windows and link_cap
// cached out-links: fluid and history (8 B per node), link offsets, degrees,
// in-degrees (4 B each), taken list (2 B), state (1 B); per window 8 B record
// base, 4 B fold offset, 4 B capacity, 4 B counter, 4 B speculative-read
// prefix, 4 B received count.
static size_t res_lds_bytes(int wlog, int nb, int link_cap) {
  const size_t W = (size_t)1 << wlog;
  return 16 * W + 8 * (size_t)nb + 4 * (W + 1) + 8 * W + 8 * ((size_t)nb + 1) + 16 * (size_t)nb +
         2 * W + W + 4 * (size_t)link_cap;
}

template <typename T, int SCHED>
__global__ __launch_bounds__(kResThreads) void k_resident(DiArgs<T> a, int link_cap,
                                                          long long spin_limit) {
  constexpr int NT = kResThreads;
  constexpr int kNPT = kResPass / NT;
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const int W = 1 << a.wlog;
  const int nb = a.nb;
  const double d = a.d, tol = a.tol;
  Ctl* const ctl = a.ctl;
  Slot* const slots = a.slots;

  extern __shared__ __align__(16) unsigned char smem[];
  double* const win = reinterpret_cast<double*>(smem);      // [W] fluid
  double* const hist = win + W;                              // [W] history
  int64_t* const s_base = reinterpret_cast<int64_t*>(hist + W);  // [nb] record base per destination
  int32_t* const s_row = reinterpret_cast<int32_t*>(s_base + nb);  // [W+1] link offsets
  int32_t* const s_deg = s_row + W + 1;                      // [W]
  int32_t* const s_in = s_deg + W;                           // [W] (ALGO-OP)
  int32_t* const s_pre = s_in + W;                           // [nb+1] fold prefix, then ranks
  int32_t* const s_soff = s_pre + nb + 1;                    // [nb] fold offset per source
  int32_t* const s_cap = s_soff + nb;                        // [nb] capacity per destination
  int32_t* const s_kin = s_cap + nb;                         // [nb+1] speculative records per source
  int32_t* const s_cnt = s_kin + nb + 1;                     // [nb] records received per source
  uint16_t* const s_list = reinterpret_cast<uint16_t*>(s_cnt + nb);  // [W] taken list
  uint8_t* const s_state = reinterpret_cast<uint8_t*>(s_list + W);   // [W]
  int32_t* const s_col = reinterpret_cast<int32_t*>(s_state + W);    // [link_cap]
  __shared__ int32_t s_beo[kResPass + 1];
  __shared__ int32_t s_brow[kResPass];
  __shared__ double s_bsh[kResPass];
  __shared__ int32_t s_chunk[(1 << kResMaxWlog) / 64];
  __shared__ double s_red[block_reduce_k_scratch<NT, kSums>()];
  __shared__ long long s_scr[2 * (NT / 64)];
  __shared__ int s_flag;
  __shared__ int s_any, s_lp;  // records arrived this round; a push stayed in the window

  // The window, once.
  const int64_t j0 = (int64_t)b << a.wlog;
  const int wn = (int)min((int64_t)W, a.n - j0);
  const int64_t e0 = a.row_ptr[j0];
  const int nlinks = (int)(a.row_ptr[j0 + wn] - e0);
  const bool lcache = nlinks <= link_cap;
  for (int q = tid; q < W; q += NT) {
    const bool in = q < wn;
    const int64_t j = j0 + min(q, wn - 1);
    win[q] = in ? (double)a.F[j] : 0.0;
    hist[q] = in ? a.H[j] : 0.0;
    s_deg[q] = in ? a.deg[j] : 0;
    s_in[q] = in && SCHED == DI_SCHED_OP ? a.indeg[j] : 0;
    s_row[q] = in ? (int)(a.row_ptr[j] - e0) : nlinks;
  }
  if (tid == 0) s_row[W] = nlinks;
  if (lcache)
    for (int e = tid; e < nlinks; e += NT) s_col[e] = a.col[e0 + e];
  for (int w = tid; w < nb; w += NT) {
    s_soff[w] = a.soff[(int64_t)b * nb + w];
    s_base[w] = a.bstart[w] + a.soffT[(int64_t)b * nb + w];
    s_cap[w] = a.capT[(int64_t)b * nb + w];
  }
  // Records sent to this window are read speculatively: the first K of each
  // incoming segment (an equal share of kResSpec per thread) are loaded with
  // the round's counts, in one wait, and those past the count dropped; only
  // a segment that received more than K needs a second, dependent read.
  const int capin = tid < nb ? a.capT[(int64_t)tid * nb + b] : 0;  // links from window tid here
  const int nsrc = __syncthreads_count(capin > 0);
  const int K = nsrc > 0 ? kResSpec * NT / nsrc : 0;
  if (tid < nb) s_kin[tid] = min(capin, K);
  __syncthreads();
  const int spec_total = (int)lds_exscan<NT>(s_kin, nb, s_scr);
  if (tid == 0) s_kin[nb] = spec_total;
  __syncthreads();
  int sp_off[kResSpec], sp_src[kResSpec], sp_i[kResSpec];  // record offset, source, index in segment
#pragma unroll
  for (int u = 0; u < kResSpec; ++u) {
    const int slot = tid + u * NT;
    sp_src[u] = 0;
    sp_i[u] = INT_MAX;  // never below a count: an unused slot (its read is clamped and dropped)
    sp_off[u] = 0;
    if (slot < spec_total) {
      const int s = upper_idx(s_kin, nb, slot);
      sp_src[u] = s;
      sp_i[u] = slot - s_kin[s];
      sp_off[u] = s_soff[s] + sp_i[u];
    }
  }
  const int64_t rbase = a.bstart[b];  // first record of this window's region
  int active = a.active[b];
  const uint32_t wmask = (uint32_t)W - 1u;
  if (tid == 0) s_any = s_lp = 0;
  __syncthreads();

  for (int r = 0;; ++r) {
    // Round r-1's sums and the counts of the records it sent to this window
    // (clamped indices, no branch: one wait covers both).
    const Slot* P = slots + ((r + 2) % 3) * kSlots;
    const Slot p_own = P[min(tid, kSlots - 1)];
    int32_t* const cnt_in = a.cnt[(r - 1) & 1] + (int64_t)b * nb;
    const int32_t c_own = cnt_in[min(tid, nb - 1)];
    const PairT<T>* const pr = a.pairs[(r - 1) & 1];
    PairT<T> sp[kResSpec];
#pragma unroll
    for (int u = 0; u < kResSpec; ++u) sp[u] = pr[min(rbase + sp_off[u], a.mrec - 1)];

    // 1. Decisions from round r-1's sums (identical in every workgroup).
    double theta = a.theta0;
    bool stop = false;
    if (r >= 1) {
      if (b == 0 && tid < kSlots) {  // set (r+1) % 3 is next written in round r+1
        Slot* z = slots + ((r + 1) % 3) * kSlots + tid;
#pragma unroll
        for (int f = 0; f < kSums; ++f) z->sum[f] = 0.0;
        z->mrem = 0;
      }
      const bool mine = tid < kSlots;
      double v[kSums];  // nf, snd, sd, ssc, nnz, taken, edges
#pragma unroll
      for (int f = 0; f < kSums; ++f) v[f] = mine ? p_own.sum[f] : 0.0;
      double mrem_prev = mine ? __longlong_as_double((long long)p_own.mrem) : 0.0;
      block_reduce_k<NT, kSums, true>(v, mrem_prev, s_red);
      const double nf = v[0], snd = v[1], sd = v[2], ssc = v[3], nnz = v[4], taken = v[5],
                   edges = v[6];
      int reason = 0;
      if (!isfinite(nf)) reason = 2;
      else if (nf < tol) reason = 1;
      else if ((int64_t)r >= a.max_rounds) reason = 3;
      stop = reason != 0;
      const double R = nf - (1.0 - d) * snd - sd;
      theta = nnz > 0 ? a.c * (ssc / nnz) * (nf > 0 ? R / nf : 0.0) : 0.0;
      if (taken == 0 && theta > mrem_prev) theta = mrem_prev;
      if (b == 0 && tid == 0) {
        ctl->nodes_total += (long long)taken;
        ctl->edges_total += (long long)edges;
        ctl->last_taken = (long long)taken;
        ctl->last_edges = (long long)edges;
        ctl->theta = theta;
        ctl->nf = nf;
        if (stop) {
          ctl->reason = reason;
          ctl->stop_round = r - 1;
        }
      }
    }

    // 2. The pushes of round r-1 into this window: the speculative reads,
    //    then whatever a segment received beyond them.
    if (tid < nb) {
      const int c = r >= 1 ? c_own : 0;
      s_cnt[tid] = c;
      s_pre[tid] = max(c - (s_kin[tid + 1] - s_kin[tid]), 0);
      if (c > 0) s_any = 1;
    }
    wg_barrier<true>();
    const bool received = s_any != 0;
#pragma unroll
    for (int u = 0; u < kResSpec; ++u)
      if (sp_i[u] < s_cnt[sp_src[u]] && sp[u].loc < (uint32_t)wn)
        atomicAdd(&win[sp[u].loc], (double)sp[u].val);
    const long long rest = r >= 1 ? lds_exscan<NT, true>(s_pre, nb, s_scr) : 0;
    if (rest > 0) {
      const long long total = rest;
      for (long long i0 = (long long)tid * kRun; i0 < total; i0 += (long long)NT * kRun) {
        int s = upper_idx(s_pre, nb, i0);
        long long nxt = s + 1 < nb ? s_pre[s + 1] : total;
        int64_t sb = rbase + s_soff[s] + (s_kin[s + 1] - s_kin[s]) - s_pre[s];
        int64_t idx[kRun];
#pragma unroll
        for (int u = 0; u < kRun; ++u) {
          const long long i = i0 + u;
          idx[u] = -1;
          if (i < total) {
            while (i >= nxt) {
              ++s;
              nxt = s + 1 < nb ? s_pre[s + 1] : total;
              sb = rbase + s_soff[s] + (s_kin[s + 1] - s_kin[s]) - s_pre[s];
            }
            idx[u] = sb + i;
          }
        }
        PairT<T> e[kRun];
#pragma unroll
        for (int u = 0; u < kRun; ++u)
          if (idx[u] >= 0) e[u] = pr[idx[u]];
#pragma unroll
        for (int u = 0; u < kRun; ++u)
          if (idx[u] >= 0 && e[u].loc < (uint32_t)wn) atomicAdd(&win[e[u].loc], (double)e[u].val);
      }
    }
    // consumed: cleared for round r+1, which writes this row again
    if (r >= 1 && tid < nb && c_own != 0) cnt_in[tid] = 0;
    wg_barrier<true>();
    if (stop) break;  // uniform: every workgroup reads the same sums

    double acc[7] = {0, 0, 0, 0, 0, 0, 0};  // nf, snd, sd, ssc, nnz, taken, edges
    double mrem = 0.0;
    if (received || active) {  // uniform
      // 3. Decide for every node of the window (LDS only), then list the
      //    taken nodes in node order (per 64-node chunk: offset plus rank).
      uint32_t tbits = 0;
      for (int q = tid, k = 0; q < W; q += NT, ++k) {
        const double f = q < wn ? win[q] : 0.0, af = fabs(f);
        uint8_t st = 0;
        if (af > 0.0) {
          acc[0] += af;
          acc[4] += 1.0;
          const double sc = node_score<SCHED>(af, s_deg[q], s_in[q]);
          acc[3] += sc;
          if (sc >= theta) st = 1;
          else mrem = fmax(mrem, sc);
        } else if (f != f) {
          acc[0] = NAN;
        }
        s_state[q] = st;
        tbits |= (uint32_t)st << k;
        const unsigned long long m = __ballot(st != 0);
        if ((tid & 63) == 0) s_chunk[q >> 6] = __popcll(m);
      }
      wg_barrier<true>();
      const int ntk = (int)lds_exscan<NT, true>(s_chunk, W >> 6, s_scr);
      if (ntk > 0) {
        for (int q = tid, k = 0; q < W; q += NT, ++k) {
          const bool t = (tbits >> k) & 1u;
          const unsigned long long m = __ballot(t);
          const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
          if (t) s_list[s_chunk[q >> 6] + rank] = (uint16_t)q;
        }
      }
      for (int w = tid; w < nb; w += NT) s_pre[w] = 0;  // now: records written per destination
      wg_barrier<true>();
      int32_t* const cnt_out = a.cnt[r & 1];
      PairT<T>* const out = a.pairs[r & 1];
      for (int t0 = 0; t0 < ntk; t0 += kResPass) {
        // 4. Take the pass's nodes (H_i += F_i, F_i = 0) and stage the
        //    pushing ones with their link offsets and shares.
        long long npush = 0, nedge = 0;
        int qs[kNPT];
        double f[kNPT];
#pragma unroll
        for (int u = 0; u < kNPT; ++u) {
          const int i = t0 + tid + u * NT;
          qs[u] = -1;
          f[u] = 0.0;
          if (i >= ntk) continue;
          const int q = s_list[i];
          qs[u] = q;
          f[u] = win[q];
          hist[q] += f[u];
          win[q] = 0.0;
          s_state[q] = 2;
          if (a.trace && r < a.trace_rounds) a.trace[(int64_t)r * a.n + j0 + q] = 1;
          acc[5] += 1.0;
          const int dg = s_deg[q];
          if (dg > 0) {
            acc[1] += fabs(f[u]);
            ++npush;
            nedge += dg;
          } else {
            acc[2] += fabs(f[u]);
          }
        }
        long long slot = 0, eoff = 0, ntile = 0, etile = 0;
        block_exscan2<NT, true>(npush, nedge, s_scr, &slot, &eoff, &ntile, &etile);
        if (ntile == 0) continue;  // uniform
#pragma unroll
        for (int u = 0; u < kNPT; ++u) {
          if (qs[u] < 0 || s_deg[qs[u]] == 0) continue;
          const int dg = s_deg[qs[u]];
          s_beo[slot] = (int32_t)eoff;
          s_brow[slot] = s_row[qs[u]];
          s_bsh[slot] = a.weighted ? d * f[u] : d * f[u] / (double)dg;
          ++slot;
          eoff += dg;
        }
        wg_barrier<true>();
        // 5. Push every staged link (kRun consecutive links per thread): into
        //    the LDS fluid when the target is in this window and not a node
        //    of S still to be expanded, else as a record.
        const int bcount = (int)ntile;
        for (long long t00 = (long long)tid * kRun; t00 < etile; t00 += (long long)NT * kRun) {
          int k = upper_idx(s_beo, bcount, t00);
          long long nxt = k + 1 < bcount ? s_beo[k + 1] : etile;
          int lb = s_brow[k] - s_beo[k];  // window link index = lb + t for node k
          double sh = s_bsh[k];
          int e[kRun];
          double v[kRun];
#pragma unroll
          for (int u = 0; u < kRun; ++u) {
            const long long t = t00 + u;
            e[u] = -1;
            v[u] = 0.0;
            if (t < etile) {
              while (t >= nxt) {
                ++k;
                nxt = k + 1 < bcount ? s_beo[k + 1] : etile;
                lb = s_brow[k] - s_beo[k];
                sh = s_bsh[k];
              }
              e[u] = lb + (int)t;
              v[u] = sh;
            }
          }
          uint32_t dst[kRun];
#pragma unroll
          for (int u = 0; u < kRun; ++u)
            if (e[u] >= 0) {
              dst[u] = (uint32_t)(lcache ? s_col[e[u]] : a.col[e0 + e[u]]);
              if (a.weighted) v[u] *= a.w[e0 + e[u]];
            }
#pragma unroll
          for (int u = 0; u < kRun; ++u) {
            if (e[u] < 0) continue;
            const int w = (int)(dst[u] >> a.wlog);
            if (w == b && s_state[dst[u] & wmask] != 1) {
              atomicAdd(&win[dst[u] & wmask], (double)(T)v[u]);
              s_lp = 1;
              continue;
            }
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
        wg_barrier<true>();
      }
      for (int w = tid; w < nb; w += NT)
        if (s_pre[w] > 0) cnt_out[(int64_t)w * nb + b] = min(s_pre[w], s_cap[w]);
      if constexpr (std::is_same<T, float>::value)
        for (int q = tid; q < wn; q += NT) win[q] = (double)(float)win[q];
    }

    // 6. This window's sums, added into its slot; then wait for every window.
    const int local_any = s_lp;  // after the last pass's barrier
    const double edges = acc[6];
    acc[6] = 0.0;
    block_reduce_k<NT, kSums, true>(acc, mrem, s_red);
    active = (acc[4] > acc[5] || local_any) ? 1 : 0;
    if (tid == 0) {
      s_any = s_lp = 0;  // every thread read both before the reduction's barriers
      acc[6] = edges;
      Slot* sl = slots + (r % 3) * kSlots + (b % kSlots);
#pragma unroll
      for (int f = 0; f < kSums; ++f)
        if (acc[f] != 0.0) unsafeAtomicAdd(&sl->sum[f], acc[f]);
      if (mrem > 0.0) atomicMax(&sl->mrem, (unsigned long long)__double_as_longlong(mrem));
    }
    if (!grid_barrier(&ctl->bar, (unsigned)(r + 1) * (unsigned)nb,
                      &ctl->err, spin_limit, &s_flag))
      break;
  }
  for (int q = tid; q < wn; q += NT) {
    a.F[j0 + q] = (T)win[q];
    a.H[j0 + q] = hist[q];
  }
  if (tid == 0) a.active[b] = active;
}

// Diagnostic setting (di_set_persist_wait): the longest barrier wait, seconds.
static std::atomic<double> g_persist_wait_s{2.0};

// Whether a single solve at 2^wlog-node windows can run as one launch.
static bool resident_fits(int64_t n, int64_t m, int wlog, bool gt) {
  const int64_t nb = (n + (1ll << wlog) - 1) >> wlog;
  return !gt && wlog <= kResMaxWlog && nb <= kResMaxWindows && m < (1ll << 31) &&
         res_lds_bytes(wlog, (int)nb, 0) <= 120 * 1024;
}

bool persist_fits(int64_t n, int64_t m, int wlog) { return resident_fits(n, m, wlog, false); }

template <typename T>
static void launch_resident(const DiArgs<T>& a, int sched, hipStream_t s, LaunchTimer* lt) {
  DI_REQUIRE(a.nvec == 1 && a.nb <= kResMaxWindows && a.wlog <= kResMaxWlog,
             "the one-launch solve needs at most 128 windows of at most 2^11 nodes");
  // dynamic LDS limit of the three instances (set once) and the wall-clock rate
  static const size_t dyn_limit = [] {
    size_t lim = ~(size_t)0;
    auto one = [&](const void* k) {
      hipFuncAttributes fa;
      DI_HIP(hipFuncGetAttributes(&fa, k));
      int dev = 0, mx = 0;
      DI_HIP(hipGetDevice(&dev));
      DI_HIP(hipDeviceGetAttribute(&mx, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
      const size_t dl = (size_t)mx - fa.sharedSizeBytes;
      DI_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dl));
      lim = std::min(lim, dl);
    };
    one((const void*)k_resident<T, DI_SCHED_MEAN>);
    one((const void*)k_resident<T, DI_SCHED_OP2>);
    one((const void*)k_resident<T, DI_SCHED_OP>);
    return lim;
  }();
  static const long long ticks_per_s = [] {
    int dev = 0, khz = 0;
    DI_HIP(hipGetDevice(&dev));
    DI_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    return (long long)std::max(khz, 1) * 1000;
  }();
  const size_t base = res_lds_bytes(a.wlog, a.nb, 0);
  DI_REQUIRE(base <= dyn_limit, "window too large for the one-launch solve");
  // a barrier wait this long means a fault, not a slow round (di_set_persist_wait)
  int link_cap = (int)std::min<size_t>((dyn_limit - base) / 4, (size_t)kResLinkCap);
  const size_t smem = res_lds_bytes(a.wlog, a.nb, link_cap);
  long long limit = (long long)((double)ticks_per_s * g_persist_wait_s.load(std::memory_order_relaxed));
  DiArgs<T> args = a;
  void* params[] = {(void*)&args, (void*)&link_cap, (void*)&limit};
  const void* kern = sched == DI_SCHED_OP2  ? (const void*)k_resident<T, DI_SCHED_OP2>
                     : sched == DI_SCHED_OP ? (const void*)k_resident<T, DI_SCHED_OP>
                                            : (const void*)k_resident<T, DI_SCHED_MEAN>;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (lt && lt->on) {
    lt->next(&e0, &e1);
    DI_HIP(hipEventRecord(e0, s));
  }
  DI_HIP(hipLaunchCooperativeKernel(kern, dim3(a.nb), dim3(kResThreads), params, (unsigned)smem, s));
  if (e1) DI_HIP(hipEventRecord(e1, s));
}

// Zero the flush slots of the vectors of this launch (slot vmap[blockIdx.x]).
template <typename T>
__global__ void k_zero_flush(DiArgs<T> a) {
  const int vb = a.vmap ? a.vmap[blockIdx.x] : blockIdx.x;
  for (int k = threadIdx.x; k < kFlushAcc; k += blockDim.x) a.flacc[(int64_t)vb * kFlushAcc + k] = 0.0;
}

template <typename T>
static void flush(const DiArgs<T>& a, double* x, int normalize, hipStream_t s) {
  k_zero_flush<T><<<a.nvec, 256, 0, s>>>(a);
  DI_HIP(hipGetLastError());
  const dim3 grid(grid_for(a.n, 1024), a.nvec);
  k_flush_sum<T><<<grid, kBlock, 0, s>>>(a);
  DI_HIP(hipGetLastError());
  k_flush_reduce<T><<<a.nvec, kBlock, 0, s>>>(a);
  DI_HIP(hipGetLastError());
  if (x) {
    k_flush_write<T><<<grid, kBlock, 0, s>>>(a, x, normalize);
    DI_HIP(hipGetLastError());
  }
}

static void fill_stats(const Ctl& h, const di_opts* o, double secs, di_stats* st) {
  const double d = o->d;
  const double S = h.fl[0], nf = h.fl[2];
  st->residual_l1 = nf;
  st->err_bound_l1 = o->normalize ? (S > 0 ? 2.0 * d * nf / ((1.0 - d) * S) : 0.0)
                                  : d * nf / (1.0 - d);
  st->mass_drift = h.fl[1] + (h.fl[4] + d * h.fl[3]) / (1.0 - d) - 1.0;
  st->seconds = secs;
  st->rounds = h.stop_round + 1;
  st->nodes_diffused = h.nodes_total;
  st->edges_diffused = h.edges_total;
  st->kernel_seconds = 0.0;
  st->kernel_launches = 0;
}

static di_status status_of(const Ctl& h) {
  if (h.err & 4) {
    set_error("grid barrier of the one-launch solve timed out");
    return DI_EDEVICE;
  }
  if (h.err) {
    set_error("internal segment consistency check failed (code " + std::to_string(h.err) + ")");
    return DI_EDEVICE;
  }
  if (h.reason == 2) {
    set_error("non-finite residual");
    return DI_EDEVICE;
  }
  if (h.reason == 3) {
    set_error("max_rounds reached before ||F||_1 < tol");
    return DI_ENOTCONV;
  }
  return DI_OK;
}

struct TuneParams {
  int sched, wlog, check_every, threads;
  bool gt;
  bool whole;    // single solves: the whole graph in one workgroup's LDS (k_small)
  bool persist;  // single solves: one launch for every round (k_resident)
  double c;
};

// Knobs of a call: the caller's tune, else what di_autotune cached for this
// graph (mode DI_TUNE_SOLVE / DI_TUNE_BATCH, precision), else the defaults.
static TuneParams tune_params(Graph* g, const di_tune* tn, int mode, int precision) {
  di_tune cached;
  if (!tn) {
    std::lock_guard<std::mutex> lk(g->ws_mu);
    const int pi = precision == DI_FP64 ? 1 : 0;
    if (g->has_tuned[mode][pi]) {
      cached = g->tuned[mode][pi];
      tn = &cached;
    }
  }
  TuneParams p;
  p.sched = tn ? tn->schedule : DI_SCHED_MEAN;
  DI_REQUIRE(p.sched >= 0 && p.sched <= 2, "unknown schedule");
  p.c = (tn && tn->c > 0.f) ? (double)tn->c : 1.0;
  const int tables = tn ? tn->tables : 0;
  DI_REQUIRE(tables >= 0 && tables <= 2, "tables must be 0, 1 or 2");
  // The whole-graph window (single solves): when asked for, or autotuned.
  const bool asked = tn && tn->window_log2 == DI_WINDOW_WHOLE;
  const bool fits = g->n <= DI_SMALL_MAX_NODES && g->m < (1ll << 31);
  if (asked && mode == DI_TUNE_SOLVE)
    DI_REQUIRE(fits, "DI_WINDOW_WHOLE needs n <= DI_SMALL_MAX_NODES and fewer than 2^31 links");
  p.whole = mode == DI_TUNE_SOLVE && asked;
  p.gt = false;
  p.wlog = window_log2_for(g->n, p.whole ? 14 : (tn && !asked ? tn->window_log2 : 0), tables,
                           &p.gt);
  DI_REQUIRE(p.wlog > 0, "graph has too many nodes for the window tables");
  p.check_every = tn ? std::max(0, tn->check_every) : 0;
  p.threads = tn && tn->threads ? tn->threads : kRoundThreads;
  DI_REQUIRE(p.threads == 512 || p.threads == 1024, "threads must be 0, 512 or 1024");
  if (p.gt) p.threads = 1024;  // the only instance with tables in global memory
  p.persist = mode == DI_TUNE_SOLVE && tn && tn->persist;
  if (p.persist) {
    DI_REQUIRE(tn->persist == 1 && !p.whole, "persist must be 0 or 1 (not with DI_WINDOW_WHOLE)");
    // no window asked for: the smallest that allows it
    if (tn->window_log2 == 0)
      for (int k = p.wlog + 1; k <= kResMaxWlog && !resident_fits(g->n, g->m, p.wlog, p.gt); ++k)
        p.wlog = window_log2_for(g->n, k, tables, &p.gt);
    DI_REQUIRE(resident_fits(g->n, g->m, p.wlog, p.gt),
               "persist needs at most 128 windows of at most 2^11 nodes and fewer than 2^31 links");
  }
  return p;
}

template <typename T>
static di_status solve_impl(Graph* g, const double* v, const di_opts* o, double* x,
                            di_stats* st, hipStream_t s) {
  const TuneParams tp = tune_params(g, o->tune, DI_TUNE_SOLVE, o->precision);
  const bool dev = (o->flags & DI_DEVICE_PTRS) != 0;
  const bool resume = (o->flags & DI_RESUME) != 0;
  const int64_t max_rounds = o->max_rounds > 0 ? o->max_rounds : 1000000;
  DI_REQUIRE(!resume || (o->state_f && o->state_h), "DI_RESUME needs state_f and state_h");
  if (v && !dev) validate_vector(v, g->n, "v");
  WsGuard guard{g, acquire_workspace(g, o->precision, tp.wlog, tp.gt), s};
  Workspace* ws = guard.ws;
  // a device v: checked with the flush scratch (cleared again before the flush)
  if (v && dev)
    validate_device_vector(v, g->n, "v", ws->flacc.as<double>(), ws->hctl.as<double>(), s);
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
  DiArgs<T> a = make_args<T>(g, ws, o->d, o->tol, tp.c, max_rounds, F, H, 1);
  a.threads = tp.threads;
  if (o->flags & DI_TRACE) {
    DI_REQUIRE(o->trace_sets != nullptr && o->trace_rounds >= 0,
               "DI_TRACE needs trace_sets and trace_rounds >= 0");
    a.trace = o->trace_sets;
    a.trace_rounds = o->trace_rounds;
  }
  LaunchTimer lt(s, (o->flags & DI_TIMING) != 0);
  EventTimer timer(s);
  if (resume) {
    // first threshold from the resumed fluid (the flush scratch is cleared
    // again before the flush)
    double* acc = ws->flacc.as<double>();
    double* hacc = ws->hctl2.as<double>();
    DI_HIP(hipMemsetAsync(acc, 0, 2 * sizeof(double), s));
    const dim3 gr(grid_for(g->n, 128));
    if (tp.sched == DI_SCHED_OP2) k_resume_scores<T, DI_SCHED_OP2><<<gr, kBlock, 0, s>>>(a, acc);
    else if (tp.sched == DI_SCHED_OP) k_resume_scores<T, DI_SCHED_OP><<<gr, kBlock, 0, s>>>(a, acc);
    else k_resume_scores<T, DI_SCHED_MEAN><<<gr, kBlock, 0, s>>>(a, acc);
    DI_HIP(hipGetLastError());
    DI_HIP(hipMemcpyAsync(hacc, acc, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    DI_HIP(hipStreamSynchronize(s));
    if (hacc[1] > 0.0 && std::isfinite(hacc[0])) a.theta0 = tp.c * hacc[0] / hacc[1];
  }
  k_init<T><<<dim3(grid_for(g->n, 2048), 1), kBlock, 0, s>>>(a, vdev, resume ? 1 : 0, 0);
  DI_HIP(hipGetLastError());
  if (tp.whole) launch_small(a, ws, tp.sched, s, &lt);
  else if (tp.persist) launch_resident(a, tp.sched, s, &lt);
  else run_rounds(a, ws, tp.sched, tp.check_every, s, &lt);
  double* xo = x ? (dev ? x : ws->x.as<double>()) : nullptr;
  flush(a, xo, o->normalize, s);
  const double secs = timer.stop();
  if (x && !dev) DI_HIP(hipMemcpyAsync(x, xo, g->n * 8, hipMemcpyDeviceToHost, s));
  read_ctl(ws, 1, s);
  const Ctl* h = ws->hctl.as<Ctl>();
  if (st) {
    fill_stats(*h, o, secs, st);
    // launches 0..stop_round take and expand; launch stop_round+1 folds (the
    // whole-graph window and the one-launch solve: one launch).
    const size_t working = tp.whole || tp.persist ? 1 : (size_t)h->stop_round + 2;
    st->kernel_seconds = lt.on ? lt.total(working) : 0.0;
    st->kernel_launches = lt.on ? (int64_t)working : 0;
  }
  return status_of(*h);
}

// ------------------------------------------------------------------ top-k

constexpr int kTopBins = 2048;  // key prefix histogram (non-negative float bits >> shift)

// Histogram of key prefixes of x = H + F for slot vmap[blockIdx.y]; with
// parent >= 0 only keys whose (key >> 20) equals parent are counted.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_topk_hist(DiArgs<T> a, int shift, const int* parent,
                                                      int32_t* __restrict__ hist) {
  __shared__ int32_t h[kTopBins];
  for (int k = threadIdx.x; k < kTopBins; k += kBlock) h[k] = 0;
  __syncthreads();
  const int y = blockIdx.y, vb = a.vmap[y];
  const T* F = a.F + (int64_t)vb * a.n;
  const double* H = a.H + (int64_t)vb * a.n;
  const int par = parent ? parent[y] : -1;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n;
       i += (int64_t)gridDim.x * kBlock) {
    const uint32_t key = __float_as_uint((float)(H[i] + (double)F[i]));
    if (par >= 0 && (int)(key >> 20) != par) continue;
    atomicAdd(&h[(key >> shift) & (kTopBins - 1)], 1);
  }
  __syncthreads();
  int32_t* gh = hist + (int64_t)y * kTopBins;
  for (int k = threadIdx.x; k < kTopBins; k += kBlock)
    if (h[k]) atomicAdd(&gh[k], h[k]);
}

// Candidates of vector y: every i whose key >> 9 (a key prefix of 23 bits) is
// at least thr[y].  Those at or above hi[y] (fewer than kk by the choice of
// the thresholds) go to slots [0, kk); the rest, the entries of the
// threshold's own bin, to slots [kk, cap).  Counts: hcount[y], ecount[y]
// (the latter may exceed the room; the host then collects that vector again
// with k_topk_all).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_topk_collect(DiArgs<T> a, const uint32_t* thr,
                                                         const uint32_t* hi, int kk,
                                                         double* __restrict__ cval,
                                                         int32_t* __restrict__ cid,
                                                         int32_t* __restrict__ hcount,
                                                         int32_t* __restrict__ ecount, int cap) {
  const int y = blockIdx.y, vb = a.vmap[y];
  const T* F = a.F + (int64_t)vb * a.n;
  const double* H = a.H + (int64_t)vb * a.n;
  const uint32_t t = thr[y], th = hi[y];
  const int lane = threadIdx.x & 63;
  for (int64_t i0 = (int64_t)blockIdx.x * kBlock; i0 < a.n; i0 += (int64_t)gridDim.x * kBlock) {
    const int64_t i = i0 + threadIdx.x;
    double x = 0.0;
    uint32_t key = 0;
    if (i < a.n) {
      x = H[i] + (double)F[i];
      key = __float_as_uint((float)x) >> 9;
    }
    const bool take = i < a.n && key >= t;
    const bool top = take && key >= th;
    // one reservation per wave and class
    const unsigned long long mt = __ballot(top), me = __ballot(take && !top);
    if ((mt | me) == 0) continue;
    int bt = 0, be = 0;
    if (mt && lane == __ffsll((long long)mt) - 1) bt = atomicAdd(&hcount[y], __popcll(mt));
    if (me && lane == __ffsll((long long)me) - 1) be = atomicAdd(&ecount[y], __popcll(me));
    if (mt) bt = __shfl(bt, __ffsll((long long)mt) - 1, 64);
    if (me) be = __shfl(be, __ffsll((long long)me) - 1, 64);
    const unsigned long long below = (1ull << lane) - 1;
    int pos = -1;
    if (top) {
      const int p = bt + __popcll(mt & below);
      if (p < kk) pos = p;  // always: fewer than kk entries lie above the bin
    } else if (take) {
      const int p = be + __popcll(me & below);
      if (p < cap - kk) pos = kk + p;
    }
    if (pos >= 0) {
      cval[(int64_t)y * cap + pos] = x;
      cid[(int64_t)y * cap + pos] = (int32_t)i;
    }
  }
}

// Every i of vector vmap[y] whose key >> 9 is at least t, into out[0..) in
// any order (the caller sized out by the count the collection found).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_topk_all(DiArgs<T> a, int y, uint32_t t,
                                                     double* __restrict__ oval,
                                                     int32_t* __restrict__ oid,
                                                     int32_t* __restrict__ count, int64_t room) {
  const int vb = a.vmap[y];
  const T* F = a.F + (int64_t)vb * a.n;
  const double* H = a.H + (int64_t)vb * a.n;
  const int lane = threadIdx.x & 63;
  for (int64_t i0 = (int64_t)blockIdx.x * kBlock; i0 < a.n; i0 += (int64_t)gridDim.x * kBlock) {
    const int64_t i = i0 + threadIdx.x;
    double x = 0.0;
    bool take = false;
    if (i < a.n) {
      x = H[i] + (double)F[i];
      take = (__float_as_uint((float)x) >> 9) >= t;
    }
    const unsigned long long m = __ballot(take);
    if (m == 0) continue;
    int base = 0;
    if (lane == __ffsll((long long)m) - 1) base = atomicAdd(count, __popcll(m));
    base = __shfl(base, __ffsll((long long)m) - 1, 64);
    if (take) {
      const int64_t p = base + __popcll(m & ((1ull << lane) - 1));
      if (p < room) {
        oval[p] = x;
        oid[p] = (int32_t)i;
      }
    }
  }
}

// The kk largest entries of H+F of k vectors (a.vmap[0..k)) on the device:
// a histogram of the fp32 key's top bits picks a threshold bin that at least
// kk entries reach (refined by the next 11 bits when too many share its bin);
// the entries above that bin (fewer than kk) and those of the bin (as many as
// the room holds) are collected, and the host sorts that short list.  A
// vector whose threshold bin overflows the room (many equal or nearly equal
// values) has all its candidates collected again into a buffer of their
// exact count, so the result is exact in every case.
template <typename T>
class TopKT {
 public:
  static constexpr int kCap = 8192;  // candidates kept per vector

  void reserve(int cap) {
    hist_.alloc((int64_t)cap * kTopBins * 4);
    h_hist_.alloc((int64_t)cap * kTopBins * 4);
    par_.alloc(cap * 4);
    h_par_.alloc(cap * 4);
    thr_.alloc(cap * 8);
    h_thr_.alloc(cap * 8);
    ccount_.alloc(cap * 8);
    h_ccount_.alloc(cap * 8);
    cval_.alloc((int64_t)cap * kCap * 8);
    cid_.alloc((int64_t)cap * kCap * 4);
    h_cval_.alloc((int64_t)cap * kCap * 8);
    h_cid_.alloc((int64_t)cap * kCap * 4);
  }

  // out[q]: up to kk (value of H+F, node) pairs of vector a.vmap[q], largest
  // first, ties by node id; fewer when fewer entries are non-zero.
  void run(const DiArgs<T>& a, int k, int kk,
           std::vector<std::vector<std::pair<double, int32_t>>>& out, hipStream_t s) {
    DI_REQUIRE(kk >= 1 && kk <= 1024, "top-k size out of range");
    const int gx = grid_for(a.n, 512);
    DI_HIP(hipMemsetAsync(hist_.p, 0, (int64_t)k * kTopBins * 4, s));
    k_topk_hist<T><<<dim3(gx, k), kBlock, 0, s>>>(a, 20, nullptr, hist_.as<int32_t>());
    DI_HIP(hipGetLastError());
    DI_HIP(hipMemcpyAsync(h_hist_.p, hist_.p, (int64_t)k * kTopBins * 4, hipMemcpyDeviceToHost, s));
    DI_HIP(hipStreamSynchronize(s));
    const int32_t* hh = h_hist_.as<int32_t>();
    int32_t* par = h_par_.as<int32_t>();
    uint32_t* thr = h_thr_.as<uint32_t>();  // [0, k): bin threshold, [k, 2k): above the bin
    bool refine = false;
    std::vector<int64_t> above(k, 0);
    for (int q = 0; q < k; ++q) {
      const int32_t* h = hh + (int64_t)q * kTopBins;
      int64_t cum = 0;
      int b = kTopBins - 1;
      for (; b > 0; --b) {
        if (cum + h[b] >= kk) break;
        cum += h[b];
      }
      // fewer than kk non-zero entries: take every non-zero one (bins >= 1)
      par[q] = b >= 1 && cum + h[b] > kCap - kk ? b : -1;
      above[q] = cum;
      thr[q] = (uint32_t)std::max(b, 1) << 11;  // key >> 9 >= b << 11  <=>  key >> 20 >= b
      thr[k + q] = (uint32_t)(std::max(b, 1) + 1) << 11;
      if (par[q] >= 0) refine = true;
    }
    if (refine) {
      DI_HIP(hipMemcpyAsync(par_.p, h_par_.p, k * 4, hipMemcpyHostToDevice, s));
      DI_HIP(hipMemsetAsync(hist_.p, 0, (int64_t)k * kTopBins * 4, s));
      k_topk_hist<T><<<dim3(gx, k), kBlock, 0, s>>>(a, 9, par_.as<int32_t>(), hist_.as<int32_t>());
      DI_HIP(hipGetLastError());
      DI_HIP(hipMemcpyAsync(h_hist_.p, hist_.p, (int64_t)k * kTopBins * 4, hipMemcpyDeviceToHost,
                            s));
      DI_HIP(hipStreamSynchronize(s));
      for (int q = 0; q < k; ++q) {
        if (par[q] < 0) continue;
        const int32_t* h = hh + (int64_t)q * kTopBins;
        int64_t cum = above[q];
        int b = kTopBins - 1;
        for (; b > 0; --b) {
          if (cum + h[b] >= kk) break;
          cum += h[b];
        }
        thr[q] = ((uint32_t)par[q] << 11) | (uint32_t)b;
        thr[k + q] = thr[q] + 1;
      }
    }
    DI_HIP(hipMemcpyAsync(thr_.p, h_thr_.p, 2 * k * 4, hipMemcpyHostToDevice, s));
    DI_HIP(hipMemsetAsync(ccount_.p, 0, 2 * k * 4, s));
    int32_t* dcount = ccount_.as<int32_t>();
    k_topk_collect<T><<<dim3(gx, k), kBlock, 0, s>>>(a, thr_.as<uint32_t>(),
                                                      thr_.as<uint32_t>() + k, kk,
                                                      cval_.as<double>(), cid_.as<int32_t>(),
                                                      dcount, dcount + k, kCap);
    DI_HIP(hipGetLastError());
    DI_HIP(hipMemcpyAsync(h_ccount_.p, ccount_.p, 2 * k * 4, hipMemcpyDeviceToHost, s));
    DI_HIP(hipMemcpyAsync(h_cval_.p, cval_.p, (int64_t)k * kCap * 8, hipMemcpyDeviceToHost, s));
    DI_HIP(hipMemcpyAsync(h_cid_.p, cid_.p, (int64_t)k * kCap * 4, hipMemcpyDeviceToHost, s));
    DI_HIP(hipStreamSynchronize(s));
    const int32_t* hc = h_ccount_.as<int32_t>();
    const int32_t* ec = hc + k;
    auto by_rank = [](const std::pair<double, int32_t>& x, const std::pair<double, int32_t>& y) {
      return x.first > y.first || (x.first == y.first && x.second < y.second);
    };
    out.assign(k, {});
    for (int q = 0; q < k; ++q) {
      std::vector<std::pair<double, int32_t>>& v = out[q];
      if (hc[q] >= kk) {
        set_error("internal top-k threshold inconsistent");
        throw Fail{DI_EDEVICE};
      }
      if (ec[q] <= kCap - kk) {
        const double* cv = h_cval_.as<double>() + (int64_t)q * kCap;
        const int32_t* ci = h_cid_.as<int32_t>() + (int64_t)q * kCap;
        for (int t = 0; t < hc[q]; ++t) v.push_back({cv[t], ci[t]});
        for (int t = 0; t < ec[q]; ++t) v.push_back({cv[kk + t], ci[kk + t]});
      } else {
        // the threshold bin overflowed the room: every candidate, exactly
        const int64_t total = (int64_t)hc[q] + ec[q];
        DevBuf ov, oi, oc;
        ov.alloc(total * 8);
        oi.alloc(total * 4);
        oc.alloc(4);
        DI_HIP(hipMemsetAsync(oc.p, 0, 4, s));
        k_topk_all<T><<<gx, kBlock, 0, s>>>(a, q, thr[q], ov.as<double>(), oi.as<int32_t>(),
                                            oc.as<int32_t>(), total);
        DI_HIP(hipGetLastError());
        std::vector<double> hv(total);
        std::vector<int32_t> hi(total);
        DI_HIP(hipMemcpyAsync(hv.data(), ov.p, total * 8, hipMemcpyDeviceToHost, s));
        DI_HIP(hipMemcpyAsync(hi.data(), oi.p, total * 4, hipMemcpyDeviceToHost, s));
        DI_HIP(hipStreamSynchronize(s));
        v.resize(total);
        for (int64_t t = 0; t < total; ++t) v[t] = {hv[t], hi[t]};
      }
      if ((int)v.size() > kk) {
        std::partial_sort(v.begin(), v.begin() + kk, v.end(), by_rank);
        v.resize(kk);
      } else {
        std::sort(v.begin(), v.end(), by_rank);
      }
    }
  }

 private:
  DevBuf hist_, par_, thr_, ccount_, cval_, cid_;
  PinnedBuf h_hist_, h_par_, h_thr_, h_ccount_, h_cval_, h_cid_;
};

template <typename T>
static di_status batch_impl(Graph* g, int32_t B, const int64_t* seed_ptr, const int32_t* seeds,
                            const double* seed_w, const di_opts* o, double* x, di_stats* st,
                            hipStream_t s, int32_t topk = 0, int32_t* top_ids = nullptr,
                            double* top_x = nullptr) {
  const TuneParams tp = tune_params(g, o->tune, DI_TUNE_BATCH, o->precision);
  const bool dev = (o->flags & DI_DEVICE_PTRS) != 0;
  const int64_t n = g->n;
  const int64_t max_rounds = o->max_rounds > 0 ? o->max_rounds : 1000000;
  // Validation of the seed sets (host arrays).
  DI_REQUIRE(B >= 1, "B must be >= 1");
  DI_REQUIRE(seed_ptr && seeds, "seed_ptr and seeds are required");
  DI_REQUIRE(seed_ptr[0] == 0, "seed_ptr[0] must be 0");
  {
    std::vector<int32_t> tmp;
    for (int32_t b = 0; b < B; ++b) {
      DI_REQUIRE(seed_ptr[b + 1] > seed_ptr[b], "empty seed set");
      tmp.assign(seeds + seed_ptr[b], seeds + seed_ptr[b + 1]);
      double ws = 0.0;
      for (int64_t k = seed_ptr[b]; k < seed_ptr[b + 1]; ++k) {
        DI_REQUIRE(seeds[k] >= 0 && seeds[k] < n, "seed out of range");
        if (seed_w) {
          DI_REQUIRE(std::isfinite(seed_w[k]) && seed_w[k] >= 0.0,
                     "seed weight negative or not finite");
          ws += seed_w[k];
        }
      }
      if (seed_w) DI_REQUIRE(std::fabs(ws - 1.0) <= 1e-9, "seed weights of a set must sum to 1");
      std::sort(tmp.begin(), tmp.end());
      DI_REQUIRE(std::adjacent_find(tmp.begin(), tmp.end()) == tmp.end(), "repeated seed in a set");
    }
  }
  // Vectors per group: what 80% of the free device memory holds.
  size_t free_b = 0, total_b = 0;
  DI_HIP(hipMemGetInfo(&free_b, &total_b));
  const int nb = (int)((n + (1ll << tp.wlog) - 1) >> tp.wlog);
  const int64_t per = bytes_per_vector(n, g->m, nb, o->precision);
  int group = (int)std::max<int64_t>(1, std::min<int64_t>(B, (int64_t)(0.8 * (double)free_b) / per));
  WsGuard guard{g, acquire_batch_workspace(g, o->precision, tp.wlog, tp.gt, std::max(group, 2)),
                s};
  Workspace* ws = guard.ws;
  group = std::min(group, ws->nvec);
  DevBuf d_ptr, d_seeds, d_w, d_x;
  const int64_t nseeds = seed_ptr[B];
  d_ptr.alloc((B + 1) * 8);
  d_seeds.alloc(nseeds * 4);
  if (seed_w) d_w.alloc(nseeds * 8);
  if (x && !dev) d_x.alloc((int64_t)group * n * 8);
  // top-k outputs: the vectors of a group by identity slot map
  TopKT<T> tk;
  DevBuf ident;
  if (topk > 0) {
    tk.reserve(group);
    std::vector<int32_t> id(group);
    for (int k = 0; k < group; ++k) id[k] = k;
    ident.alloc(group * 4);
    DI_HIP(hipMemcpyAsync(ident.p, id.data(), group * 4, hipMemcpyHostToDevice, s));
    DI_HIP(hipStreamSynchronize(s));
  }
  di_status worst = DI_OK;
  for (int32_t b0 = 0; b0 < B; b0 += group) {
    const int gb = std::min<int32_t>(group, B - b0);
    // seed pointers of this group, rebased to 0
    std::vector<int64_t> ptr(gb + 1);
    for (int k = 0; k <= gb; ++k) ptr[k] = seed_ptr[b0 + k] - seed_ptr[b0];
    DI_HIP(hipMemcpyAsync(d_ptr.p, ptr.data(), (gb + 1) * 8, hipMemcpyHostToDevice, s));
    DI_HIP(hipMemcpyAsync(d_seeds.p, seeds + seed_ptr[b0], ptr[gb] * 4, hipMemcpyHostToDevice, s));
    if (seed_w)
      DI_HIP(hipMemcpyAsync(d_w.p, seed_w + seed_ptr[b0], ptr[gb] * 8, hipMemcpyHostToDevice, s));
    DiArgs<T> a = make_args<T>(g, ws, o->d, o->tol, tp.c, max_rounds, ws->F.as<T>(),
                               ws->H.as<double>(), gb);
    a.threads = tp.threads;
    EventTimer timer(s);
    k_init<T><<<dim3(grid_for(n, 256), gb), kBlock, 0, s>>>(a, nullptr, 0, 1);
    DI_HIP(hipGetLastError());
    k_seed<T><<<gb, 256, 0, s>>>(a, d_ptr.as<int64_t>(), d_seeds.as<int32_t>(),
                                  seed_w ? d_w.as<double>() : nullptr);
    DI_HIP(hipGetLastError());
    run_rounds(a, ws, tp.sched, tp.check_every, s, nullptr);
    double* xo = x ? (dev ? x + (int64_t)b0 * n : d_x.as<double>()) : nullptr;
    flush(a, xo, o->normalize, s);
    const double secs = timer.stop();
    if (x && !dev)
      DI_HIP(hipMemcpyAsync(x + (int64_t)b0 * n, xo, (int64_t)gb * n * 8, hipMemcpyDeviceToHost, s));
    read_ctl(ws, gb, s);
    const Ctl* h = ws->hctl.as<Ctl>();
    if (topk > 0) {
      DiArgs<T> at = a;
      at.vmap = ident.as<int32_t>();
      std::vector<std::vector<std::pair<double, int32_t>>> cand;
      tk.run(at, gb, (int)std::min<int64_t>(topk, n), cand, s);
      for (int k = 0; k < gb; ++k) {
        const double S = h[k].fl[0];
        const double scale = o->normalize && S > 0 ? 1.0 / S : 1.0;
        int32_t* ids = top_ids + (int64_t)(b0 + k) * topk;
        double* xs = top_x + (int64_t)(b0 + k) * topk;
        for (int t = 0; t < topk; ++t) {
          const bool has = t < (int)cand[k].size();
          ids[t] = has ? cand[k][t].second : -1;
          xs[t] = has ? cand[k][t].first * scale : 0.0;
        }
      }
    }
    for (int k = 0; k < gb; ++k) {
      if (st) fill_stats(h[k], o, secs, &st[b0 + k]);
      const di_status rc = status_of(h[k]);
      if (rc == DI_EDEVICE || (rc == DI_ENOTCONV && worst == DI_OK)) worst = rc;
    }
  }
  return worst;
}

template <typename T>
static void round_impl(Graph* g, double d, double theta, T* F, double* H, int64_t* tn,
                       int64_t* te, hipStream_t s) {
  bool gt = false;
  const int wlog = window_log2_for(g->n, 0, 0, &gt);
  DI_REQUIRE(wlog > 0, "graph has too many nodes for the window tables");
  WsGuard guard{g,
                acquire_workspace(g, std::is_same<T, double>::value ? DI_FP64 : DI_FP32_FLUID, wlog,
                                  gt),
                s};
  Workspace* ws = guard.ws;
  DiArgs<T> a = make_args<T>(g, ws, d, 0.0, 1.0, (int64_t)1 << 40, F, H, 1);
  a.theta0 = theta;
  k_init<T><<<dim3(grid_for(g->n, 2048), 1), kBlock, 0, s>>>(a, nullptr, 1, 0);
  DI_HIP(hipGetLastError());
  launch_round(a, DI_SCHED_MEAN, 0, 0, s);
  launch_round(a, DI_SCHED_MEAN, 1, 1, s);
  read_ctl(ws, 1, s);
  const Ctl* h = ws->hctl.as<Ctl>();
  if (h->err) {
    set_error("internal segment consistency check failed");
    throw Fail{DI_EDEVICE};
  }
  if (tn) *tn = h->last_taken;
  if (te) *te = h->last_edges;
}


// ---------------------------------------------------------- serving engine

int64_t slot_bytes(const Graph* g, int precision) {
  const int wlog = window_log2_for(g->n, 0, 0, nullptr);
  DI_REQUIRE(wlog > 0, "graph has too many nodes for the window tables");
  const int nb = (int)((g->n + (1ll << wlog) - 1) >> wlog);
  return bytes_per_vector(g->n, g->m, nb, precision);
}

constexpr int kMaxStepRounds = 16;  // rounds an engine step may launch

template <typename T>
class SlotPoolT : public SlotPool {
 public:
  SlotPoolT(Graph* g, int precision, int capacity, const di_tune* tune) : g_(g), cap_(capacity) {
    tp_ = tune_params(g, tune, DI_TUNE_BATCH, precision);
    ws_ = make_workspace(g, precision, tp_.wlog, capacity, tp_.gt);
    round_.assign(capacity, 0);
    d_.assign(capacity, 0.85);
    tol_.assign(capacity, 1e-6);
    vmap_.alloc(capacity * 4);
    vround_.alloc((size_t)kMaxStepRounds * capacity * 4);
    vd_.alloc(capacity * 8);
    vtol_.alloc(capacity * 8);
    h_vmap_.alloc(capacity * 4);
    h_vround_.alloc((size_t)kMaxStepRounds * capacity * 4);
    h_vd_.alloc(capacity * 8);
    h_vtol_.alloc(capacity * 8);
    topk_.reserve(capacity);
  }
  ~SlotPoolT() override { delete ws_; }
  int capacity() const override { return cap_; }
  int64_t bytes() const override {
    return (int64_t)cap_ * bytes_per_vector(g_->n, g_->m, ws_->nb, ws_->precision);
  }

  void admit(const std::vector<SlotInit>& inits, hipStream_t s) override {
    if (inits.empty()) return;
    const int k = (int)inits.size();
    std::vector<int64_t> ptr(k + 1, 0);
    std::vector<int32_t> seeds;
    std::vector<double> w;
    bool weighted = false;
    for (const SlotInit& in : inits) weighted |= !in.w.empty();
    int32_t* hv = h_vmap_.as<int32_t>();
    for (int q = 0; q < k; ++q) {
      const SlotInit& in = inits[q];
      hv[q] = in.slot;
      round_[in.slot] = 0;
      d_[in.slot] = in.d;
      tol_[in.slot] = in.tol;
      seeds.insert(seeds.end(), in.seeds.begin(), in.seeds.end());
      if (weighted) {
        if (in.w.empty()) w.insert(w.end(), in.seeds.size(), 1.0 / (double)in.seeds.size());
        else w.insert(w.end(), in.w.begin(), in.w.end());
      }
      ptr[q + 1] = (int64_t)seeds.size();
    }
    sptr_.alloc((k + 1) * 8);
    sseeds_.alloc(seeds.size() * 4);
    h_sptr_.alloc((k + 1) * 8);
    h_sseeds_.alloc(seeds.size() * 4);
    memcpy(h_sptr_.p, ptr.data(), (k + 1) * 8);
    memcpy(h_sseeds_.p, seeds.data(), seeds.size() * 4);
    if (weighted) {
      sw_.alloc(w.size() * 8);
      h_sw_.alloc(w.size() * 8);
      memcpy(h_sw_.p, w.data(), w.size() * 8);
    }
    memcpy(h_vd_.p, d_.data(), cap_ * 8);
    memcpy(h_vtol_.p, tol_.data(), cap_ * 8);
    DI_HIP(hipMemcpyAsync(vmap_.p, h_vmap_.p, k * 4, hipMemcpyHostToDevice, s));
    DI_HIP(hipMemcpyAsync(vd_.p, h_vd_.p, cap_ * 8, hipMemcpyHostToDevice, s));
    DI_HIP(hipMemcpyAsync(vtol_.p, h_vtol_.p, cap_ * 8, hipMemcpyHostToDevice, s));
    DI_HIP(hipMemcpyAsync(sptr_.p, h_sptr_.p, (k + 1) * 8, hipMemcpyHostToDevice, s));
    DI_HIP(hipMemcpyAsync(sseeds_.p, h_sseeds_.p, seeds.size() * 4, hipMemcpyHostToDevice, s));
    if (weighted) DI_HIP(hipMemcpyAsync(sw_.p, h_sw_.p, w.size() * 8, hipMemcpyHostToDevice, s));
    DiArgs<T> a = args(k);
    k_init<T><<<dim3(grid_for(g_->n, 256), k), kBlock, 0, s>>>(a, nullptr, 0, 1);
    DI_HIP(hipGetLastError());
    k_seed<T><<<k, 256, 0, s>>>(a, sptr_.as<int64_t>(), sseeds_.as<int32_t>(),
                                 weighted ? sw_.as<double>() : nullptr);
    DI_HIP(hipGetLastError());
    // the staging buffers above are reused by the next call: drain first
    DI_HIP(hipStreamSynchronize(s));
  }

  void step(const std::vector<int>& slots, int rounds, hipStream_t s) override {
    if (slots.empty() || rounds < 1) return;
    DI_REQUIRE(rounds <= kMaxStepRounds, "too many rounds per engine step");
    const int k = (int)slots.size();
    int32_t* hv = h_vmap_.as<int32_t>();
    int32_t* hr = h_vround_.as<int32_t>();  // [rounds][cap]: launch i runs round round_[q] + i
    for (int q = 0; q < k; ++q) hv[q] = slots[q];
    for (int i = 0; i < rounds; ++i)
      for (int q = 0; q < cap_; ++q) hr[i * cap_ + q] = round_[q] + i;
    DI_HIP(hipMemcpyAsync(vmap_.p, h_vmap_.p, k * 4, hipMemcpyHostToDevice, s));
    DI_HIP(hipMemcpyAsync(vround_.p, h_vround_.p, (size_t)rounds * cap_ * 4,
                          hipMemcpyHostToDevice, s));
    DiArgs<T> a = args(k);
    for (int i = 0; i < rounds; ++i) {
      a.vround = vround_.as<int32_t>() + (size_t)i * cap_;
      launch_round(a, tp_.sched, 0, 0, s);
    }
    for (int q : slots) round_[q] += rounds;
  }

  std::vector<int> stopped(const std::vector<int>& slots, hipStream_t s) override {
    read_ctl(ws_, cap_, s);
    const Ctl* h = ws_->hctl.as<Ctl>();
    std::vector<int> out;
    for (int q : slots)
      if (h[q].stop_round >= 0) out.push_back(q);
    return out;
  }

  void finish(const std::vector<int>& slots, int topk, std::vector<SlotResult>& out,
              hipStream_t s) override {
    if (slots.empty()) return;
    const int k = (int)slots.size();
    int32_t* hv = h_vmap_.as<int32_t>();
    for (int q = 0; q < k; ++q) hv[q] = slots[q];
    DI_HIP(hipMemcpyAsync(vmap_.p, h_vmap_.p, k * 4, hipMemcpyHostToDevice, s));
    DiArgs<T> a = args(k);
    flush(a, nullptr, 1, s);
    const int kk = (int)std::min<int64_t>(topk, g_->n);
    std::vector<std::vector<std::pair<double, int32_t>>> cand;
    topk_.run(a, k, kk, cand, s);
    read_ctl(ws_, cap_, s);
    const Ctl* hc = ws_->hctl.as<Ctl>();
    for (int q = 0; q < k; ++q) {
      const int slot = slots[q];
      const Ctl& c = hc[slot];
      SlotResult r;
      r.slot = slot;
      r.status = status_of(c);
      const double S = c.fl[0];
      for (const auto& e : cand[q]) {
        r.ids.push_back(e.second);
        r.x.push_back(S > 0 ? e.first / S : 0.0);
      }
      const double d = d_[slot], nf = c.fl[2];
      r.residual = nf;
      r.bound = S > 0 ? 2.0 * d * nf / ((1.0 - d) * S) : 0.0;
      r.rounds = c.stop_round + 1;
      r.edges = c.edges_total;
      out.push_back(std::move(r));
    }
  }

 private:
  DiArgs<T> args(int k) {
    DiArgs<T> a = make_args<T>(g_, ws_, 0.85, 1e-6, tp_.c, 1000000, ws_->F.as<T>(),
                               ws_->H.as<double>(), k);
    a.threads = tp_.threads;
    a.vmap = vmap_.as<int32_t>();
    a.vd = vd_.as<double>();
    a.vtol = vtol_.as<double>();
    return a;
  }
  Graph* g_;
  int cap_;
  TuneParams tp_;
  Workspace* ws_;
  std::vector<int> round_;
  std::vector<double> d_, tol_;
  TopKT<T> topk_;
  DevBuf vmap_, vround_, vd_, vtol_, sptr_, sseeds_, sw_;
  PinnedBuf h_vmap_, h_vround_, h_vd_, h_vtol_, h_sptr_, h_sseeds_, h_sw_;
};

SlotPool* make_slot_pool(Graph* g, int precision, int capacity, const di_tune* tune) {
  if (precision == DI_FP64) return new SlotPoolT<double>(g, precision, capacity, tune);
  return new SlotPoolT<float>(g, precision, capacity, tune);
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

di_status di_solve_batch_topk(const di_graph* gc, int32_t B, const int64_t* seed_ptr,
                              const int32_t* seeds, const double* seed_w, const di_opts* opts,
                              int32_t topk, int32_t* top_ids, double* top_x, di_stats* stats,
                              void* stream) {
  di_status rc = DI_OK;
  di_status g = guarded([&] {
    DI_REQUIRE(gc != nullptr, "graph is NULL");
    validate_d_tol(opts);
    DI_REQUIRE((opts->flags & DI_RESUME) == 0, "DI_RESUME is not supported for batches");
    DI_REQUIRE(topk >= 1 && topk <= 1024, "topk must be in [1, 1024]");
    DI_REQUIRE(top_ids != nullptr && top_x != nullptr, "top_ids and top_x are required");
    Graph* g = const_cast<di_graph*>(gc);
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = opts->precision == DI_FP64
             ? batch_impl<double>(g, B, seed_ptr, seeds, seed_w, opts, nullptr, stats, s, topk,
                                  top_ids, top_x)
             : batch_impl<float>(g, B, seed_ptr, seeds, seed_w, opts, nullptr, stats, s, topk,
                                 top_ids, top_x);
  });
  return g != DI_OK ? g : rc;
}

di_status di_solve_batch(const di_graph* gc, int32_t B, const int64_t* seed_ptr,
                         const int32_t* seeds, const double* seed_w, const di_opts* opts,
                         double* x, di_stats* stats, void* stream) {
  di_status rc = DI_OK;
  di_status g = guarded([&] {
    DI_REQUIRE(gc != nullptr, "graph is NULL");
    validate_d_tol(opts);
    DI_REQUIRE((opts->flags & DI_RESUME) == 0, "DI_RESUME is not supported for batches");
    Graph* g = const_cast<di_graph*>(gc);
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = opts->precision == DI_FP64
             ? batch_impl<double>(g, B, seed_ptr, seeds, seed_w, opts, x, stats, s)
             : batch_impl<float>(g, B, seed_ptr, seeds, seed_w, opts, x, stats, s);
  });
  return g != DI_OK ? g : rc;
}

di_status di_set_persist_wait(double seconds) {
  return guarded([&] {
    DI_REQUIRE(seconds >= 0.0 && seconds <= 60.0, "seconds must be within [0, 60]");
    g_persist_wait_s.store(seconds, std::memory_order_relaxed);
  });
}

di_status di_set_taken_list(int32_t enable) {
  return guarded([&] {
    DI_REQUIRE(enable == 0 || enable == 1, "enable must be 0 or 1");
    g_taken_list.store(enable, std::memory_order_relaxed);
  });
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
