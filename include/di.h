/*
 * di.h -- D-iteration PageRank on AMD MI355X (gfx950): the C ABI of libdi.so.
 *
 * Method: D. Hong, "Optimized on-line computation of PageRank algorithm"
 * (arXiv 1202.6158).  The library solves
 *
 *        X = d P X + (1-d) V                               (Section 2.1)
 *
 * for a non-negative N x N matrix P whose non-zero columns sum to one (column
 * i = the out-links of node i, P[j][i] = p(j,i)); zero columns (dangling
 * nodes) are allowed and are NOT completed (Section 3.3).  V is a normalised
 * non-negative vector (uniform for PageRank, a seed set for personalised
 * PageRank), 0 <= d < 1.
 *
 * The D-iteration keeps a fluid vector F (F_0 = (1-d)V) and a history H
 * (H_0 = 0).  Diffusing node i moves F_i into H_i and pushes d F_i p(j,i) to
 * each child j (the fluid/history recurrences of Section 2.2).  Any order of
 * diffusions converges to the same limit; this library diffuses, in each
 * round, every node whose fluid reaches an adaptive threshold (the threshold
 * variant of Section 4.2), all at once.  Theorem 2 makes ||F||_1 the stopping
 * residual.  The result is x = (H + F) / ||H + F||_1 (renormalisation of
 * Section 3.3), or the unnormalised H + F.
 *
 * Conventions for every entry point:
 *  - Nothing throws and nothing aborts.  Each call returns a di_status; on
 *    failure di_last_error() gives a message (thread-local, valid until the
 *    next call on the same thread).
 *  - `stream` is a hipStream_t (NULL = the null stream).  Work is ordered on
 *    it; a call returns after its results are complete (host outputs written,
 *    device outputs ready on the stream).
 *  - Vectors `v` and `x` are host pointers unless DI_DEVICE_PTRS is set in the
 *    options' flags, in which case they are device pointers (e.g. the
 *    data_ptr() of a torch tensor on the same device).  Caller-owned.  A
 *    device `v` gets the same checks as a host one, by a reduction on the
 *    call's stream.
 *  - Node ids are 0-based int32; N < 2^31 and nnz < 2^36.  Solves need the
 *    binned scatter's windows to fit: at most 16384 windows of 2^13 nodes, so
 *    N <= 134,217,728 (DI_EINVAL beyond; graphs above ~25M nodes keep the
 *    per-window tables in global memory, see di_tune.tables).
 */
#ifndef DI_H
#define DI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DI_OK = 0,
  DI_EINVAL = -1,     /* invalid argument (graph, vector, d, tol, seeds ...) */
  DI_ENOMEM = -2,     /* device allocation failed, or a request exceeds the memory budget */
  DI_EDEVICE = -3,    /* HIP runtime error, or a non-finite residual */
  DI_ENOTCONV = -4,   /* max_rounds reached: outputs and stats are still valid (H is a
                         lower bound of the limit with the reported error bound) */
  DI_EAGAIN = -5,     /* server: result not ready yet */
  DI_ECANCELED = -6,  /* server: request was cancelled */
  DI_EBUSY = -7       /* graph still referenced by a server */
} di_status;

typedef struct di_graph di_graph;   /* immutable device-resident graph */
typedef struct di_server di_server; /* continuous-batching PPR server */

/* precision */
enum {
  DI_FP32_FLUID = 0, /* fluid F and pushes in fp32; H, residuals, normalisation in fp64 */
  DI_FP64 = 1        /* everything in fp64 */
};

/* flags */
enum {
  DI_DEVICE_PTRS = 1u, /* v and x are device pointers (seed arrays are always host arrays) */
  DI_RESUME = 2u,      /* di_solve: start from the state passed in di_opts.state_f/state_h */
  DI_TIMING = 4u,      /* time every launch of the round (or product) kernel with HIP events
                          on the call's stream: fills kernel_seconds / kernel_launches */
  DI_TRACE = 8u        /* di_solve: record the set S_r each round takes in opts.trace_sets */
};

/* threshold schedule families (Section 4.2 threshold variant; Section 4.3 scores) */
enum {
  DI_SCHED_MEAN = 0, /* take i if F_i >= c * R / N_eff (R = remaining fluid) */
  DI_SCHED_OP2 = 1,  /* take i if F_i/(#out_i+1) >= c * mean of that score (ALGO-OP2) */
  DI_SCHED_OP = 2    /* take i if F_i/((#in_i+1)(#out_i+1)) >= c * mean (ALGO-OP) */
};

/* Tuning knobs (all optional; zero = library default). */
/* di_tune.window_log2: the whole graph is one window, held in the LDS of one
   workgroup that runs every round of a di_solve itself (rounds separated by
   barriers, not launches); graphs of at most DI_SMALL_MAX_NODES nodes and
   fewer than 2^31 links (DI_EINVAL otherwise).  di_autotune tries it for
   such graphs.  Batches and servers take it as the default window. */
#define DI_WINDOW_WHOLE (-1)
#define DI_SMALL_MAX_NODES 16384

typedef struct di_tune {
  int32_t schedule;    /* DI_SCHED_* */
  float c;             /* threshold factor (default 1.0) */
  int32_t window_log2; /* destination window of the binned scatter: 2^k nodes (8..14), or
                          DI_WINDOW_WHOLE */
  int32_t check_every; /* rounds between host checks of the device done flag (0 = adaptive) */
  int32_t threads;     /* round workgroup size: 512 (default, 0) or 1024 (more loads in flight) */
  int32_t tables;      /* per-window segment tables of the binned scatter: 0 = in LDS when they
                          fit, else in global memory (graphs above ~25M nodes); 1 = LDS only;
                          2 = global memory (runs 1024-thread workgroups) */
  int32_t persist;     /* di_solve only: 1 = one cooperative launch runs every round, each
                          window's fluid, history, degrees and (when they fit) out-links held
                          in its workgroup's LDS for the whole solve, rounds separated by a grid
                          barrier; graphs of at most DI_PERSIST_MAX_WINDOWS windows of at most
                          2^11 nodes (DI_EINVAL otherwise; window_log2 = 0 picks the smallest
                          window that allows it).  Same rounds, thresholds and stop as the
                          launch-per-round path.  A barrier wait past 2 s (a device fault, not a
                          slow round) ends every workgroup's loop and the call returns
                          DI_EDEVICE.  0 = one launch per round. */
} di_tune;
#define DI_PERSIST_MAX_WINDOWS 128

typedef struct di_opts {
  double d;           /* damping factor, 0 <= d < 1 */
  double tol;         /* stop when ||F||_1 < tol (tol > 0) */
  int32_t precision;  /* DI_FP32_FLUID or DI_FP64 */
  int32_t normalize;  /* 1: x = (H+F)/||H+F||_1;  0: x = H+F (approximates Y = (1-d)(I-dP)^-1 V) */
  int64_t max_rounds; /* 0 = 1,000,000 */
  const di_tune* tune; /* NULL = defaults */
  uint32_t flags;     /* DI_DEVICE_PTRS | DI_RESUME */
  uint32_t pad;
  void* state_f;      /* DI_RESUME: device fluid (float* or double* per precision), in/out */
  double* state_h;    /* DI_RESUME: device history (double*), in/out */
  uint8_t* trace_sets; /* DI_TRACE: device bytes [trace_rounds][n], zeroed by the caller;
                          byte (r, i) is set to 1 when round r takes node i */
  int64_t trace_rounds; /* DI_TRACE: rounds the trace holds (later rounds are not recorded) */
} di_opts;

typedef struct di_stats {
  double residual_l1;  /* ||F||_1 at the stop, summed afresh in fp64 (power: ||x_n - x_n-1||_1) */
  double err_bound_l1; /* bound on ||x - x*||_1: 2d r/((1-d)||H+F||_1) normalised, d r/(1-d) not */
  double mass_drift;   /* sum(H) + (sum(F) + d sum_{dangling} H)/(1-d) - sum(V): 0 in exact arithmetic */
  double seconds;      /* device time of the solve on the stream (HIP events) */
  int64_t rounds;      /* diffusion rounds (power: matrix products) */
  int64_t nodes_diffused; /* node diffusions that moved fluid */
  int64_t edges_diffused; /* elementary steps: out-links used (power: nnz per product) */
  double kernel_seconds;  /* DI_TIMING: summed device time of the launches that did work */
  int64_t kernel_launches; /* DI_TIMING: number of those launches (else 0) */
} di_stats;

/* ------------------------------------------------------------------ graph */

/*
 * Build a device-resident graph from source-ordered CSR (out-links):
 * the children of node i are col_idx[row_ptr[i] .. row_ptr[i+1]).  Repeated
 * links and self-loops are allowed and count with multiplicity.
 *   w == NULL: p(j,i) = 1/outdeg(i) per link (unweighted graph);
 *   else w[e] >= 0 is the weight of link e, and every non-dangling node's
 *   weights must sum to 1 within 1e-9 (columns of P, Section 2.1).
 * row_ptr: int64[n+1], col_idx: int32[nnz], w: double[nnz]; host pointers
 * (the library copies them; the caller keeps ownership).
 * Errors: DI_EINVAL if n < 1, nnz < 0, row_ptr[0] != 0, row_ptr not
 * non-decreasing, row_ptr[n] != nnz, a col_idx out of [0,n), a weight negative
 * or not finite, or a weight column sum off by more than 1e-9; DI_ENOMEM.
 */
di_status di_graph_create(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                          const double* w, void* stream, di_graph** out);
di_status di_graph_destroy(di_graph* g); /* DI_EBUSY while a server references it */

/*
 * The binned scatter's layout that solves on a graph of n nodes get under
 * the given knobs (tune may be NULL = defaults): windows of 2^window_log2
 * nodes, with the per-window segment tables in LDS (*global_tables = 0) or
 * read from global memory (1); tune->window_log2 = DI_WINDOW_WHOLE gives
 * DI_WINDOW_WHOLE (for n <= DI_SMALL_MAX_NODES).  Host only: touches no
 * device.  DI_EINVAL if no layout fits (n above 134,217,728 nodes, or
 * tune->tables = 1 above ~25M nodes, or DI_WINDOW_WHOLE above
 * DI_SMALL_MAX_NODES) or if an output pointer is NULL.
 */
di_status di_window_layout(int64_t n, const di_tune* tune, int32_t* window_log2,
                           int32_t* global_tables);
di_status di_graph_info(const di_graph* g, int64_t* n, int64_t* nnz, int64_t* n_dangling);

/*
 * Diagnostic switch, process-wide, for tests of a fallback path.  The round
 * kernel lists each window's taken nodes in LDS and expands them 1024 at a
 * time; when LDS has no room for the list (graphs near the size limit) it
 * expands passes of 1024 consecutive nodes instead.  enable = 0 forces that
 * fallback for every later launch, 1 (the default) restores the list.  It
 * changes the order in which a round's pushes are issued, not the set a
 * round takes.  DI_EINVAL unless enable is 0 or 1.  Host only.
 */
di_status di_set_taken_list(int32_t enable);

/*
 * Diagnostic setting, process-wide, for tests of a failure path.  A workgroup
 * of the one-launch solve (di_tune.persist) that waits longer than `seconds`
 * at a grid barrier (default 2; a wait that long means a device fault, not a
 * slow round) ends the solve: every workgroup leaves its loop and di_solve
 * returns DI_EDEVICE.  0 makes nearly every solve end that way, with every
 * workgroup exiting normally.  Later launches use the new value.  DI_EINVAL
 * unless 0 <= seconds <= 60.  Host only.
 */
di_status di_set_persist_wait(double seconds);

/* --------------------------------------------------------- single solves */

/*
 * D-iteration solve (Sections 2.2, 3.4, 4.2).  v: double[n] normalised
 * personalisation vector (NULL = uniform 1/N); x: double[n] result.
 * With DI_RESUME the state (opts->state_f, opts->state_h, device arrays of n
 * entries) replaces the initial F_0 = (1-d)V, H_0 = 0 and receives the final
 * state; v is then only used for mass_drift.
 * Errors: DI_EINVAL (d outside [0,1), tol <= 0, v negative / not finite / sum
 * not within 1e-9 of 1, bad precision), DI_ENOTCONV, DI_EDEVICE, DI_ENOMEM.
 */
di_status di_solve(const di_graph* g, const double* v, const di_opts* opts, double* x,
                   di_stats* stats, void* stream);

/*
 * Comparator: power iteration X_{n+1} = d P X_n + (1-d) V from X_0 = 0
 * (MAT-ITER, Sections 2.1 and 4), as a pull (gather) over in-links, without
 * dangling completion, stopped when ||X_n - X_{n-1}||_1 < tol; x is
 * normalised at the end when opts->normalize.  precision DI_FP64 gathers
 * fp64 iterates; DI_FP32_FLUID runs the delta form F_{n+1} = d P F_n with
 * fp32 F and an fp64 accumulation of X.  Same errors as di_solve.
 */
di_status di_power_solve(const di_graph* g, const double* v, const di_opts* opts, double* x,
                         di_stats* stats, void* stream);

/*
 * di_power_solve without any allocation, for callers that cannot allocate
 * device or pinned host memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arithmetic, kernels, results,
 * statistics and errors as di_power_solve, with these differences:
 *  - Its two iterates, per-link values and control block live in a fixed
 *    scratch array of DI_NOALLOC_SCRATCH_BYTES in device memory, one per GPU,
 *    held from the library's load until the process ends.  A graph of n
 *    nodes needs 32 n bytes (DI_FP64) or 24 n bytes (DI_FP32_FLUID) of it,
 *    plus 6.4 KB: larger graphs give DI_EINVAL (n above about 1.048e6 in
 *    fp64, 1.398e6 in fp32).
 *  - v and x must be device pointers: DI_DEVICE_PTRS is required (DI_EINVAL
 *    otherwise).  DI_TIMING is rejected; stats.seconds is host time.
 *  - The current device must be the graph's device.
 *  - Every call on one GPU shares that GPU's scratch and leaves its contents
 *    behind (the call initialises everything it reads): calls that overlap on
 *    one GPU, from several host threads or streams, race and must be
 *    serialised by the caller.
 *  - It calls no hipMalloc, hipHostMalloc, hipFree or other allocating routine
 *    (the control block's host copy is on the calling thread's stack).
 */
#define DI_NOALLOC_SCRATCH_BYTES (32u << 20)
di_status di_power_solve_noalloc(const di_graph* g, const double* v, const di_opts* opts,
                                 double* x, di_stats* stats, void* stream);

/*
 * One threshold round on caller-provided device state (the kernel step of a
 * di_solve round): every node with F_i != 0 and |F_i| >= theta (compared in
 * fp64) is taken -- H_i += F_i, F_i = 0 -- and its fluid is pushed,
 * d F_i p(j,i) to each child j (the set form of the Section 2.2 recurrences).
 * F: device float[n] (DI_FP32_FLUID) or double[n] (DI_FP64); H: device
 * double[n].  taken_nodes / taken_edges (host, may be NULL) receive |S| and
 * the out-links used.
 */
di_status di_diffuse_round(const di_graph* g, int32_t precision, double d, double theta,
                           void* F, double* H, int64_t* taken_nodes, int64_t* taken_edges,
                           void* stream);

/*
 * Graph update (the updating equation of Section 3.2).  The graph changes
 * from P (g_old) to P' (g_new), both with the same n, while a solve on P is
 * under way (or done) with device state F (float[n] for DI_FP32_FLUID,
 * double[n] for DI_FP64) and H (double[n]).  Adds d (P' - P) H to F (only
 * the out-link rows that differ between the graphs push, +H_i p'(j,i) and
 * -H_i p(j,i), summed in fp64; one rounding into F); afterwards
 * H + F = F_0 + d P' H holds (Theorem 1 for P'), and di_solve on g_new with
 * DI_RESUME and this state continues to the solution of X = d P' X + F_0
 * (Theorem 4).  The injected fluid may be negative: rounds take nodes on
 * |F_i|, the residual is ||F||_1.  F is updated in the order of `stream`
 * (the call does not wait for it).  DI_EINVAL if n differs.
 */
di_status di_inject_update(const di_graph* g_old, const di_graph* g_new, int32_t precision,
                           double d, void* F, const double* H, void* stream);

/* ---------------------------------------------------------------- batches */

/*
 * Personalised PageRank for B seed sets on one graph: B independent D-iteration
 * solves of X = dPX + (1-d)V_b, V_b being the personalisation vector of
 * Section 2.1 (the initial condition F_0 = (1-d)V_b of Section 2.2), each
 * stopped by Theorem 2's residual ||F_b||_1 < tol (Section 3.1) and
 * renormalised as Section 3.3 says when P has dangling columns.  Seed set b is
 * seeds[seed_ptr[b] .. seed_ptr[b+1]) (non-empty, ids in [0,n), no repeats);
 * V_b puts weight seed_w[k] on seeds[k] (seed_w NULL = uniform over the set;
 * otherwise each set's weights must sum to 1 within 1e-9).  opts applies to
 * every vector (each stops on its own ||F_b||_1 < tol).  x: B x n doubles,
 * row-major (x[b*n + i]); stats: B entries (may be NULL).  seed_ptr, seeds,
 * seed_w are host arrays.  DI_ENOTCONV if any vector hit max_rounds.
 */
di_status di_solve_batch(const di_graph* g, int32_t B, const int64_t* seed_ptr,
                         const int32_t* seeds, const double* seed_w, const di_opts* opts,
                         double* x, di_stats* stats, void* stream);

/*
 * di_solve_batch keeping only each vector's topk largest entries (the
 * same solves as di_solve_batch: V_b of Section 2.1, stop of Theorem 2 in
 * Section 3.1, renormalisation of Section 3.3; the B x n
 * result is never formed outside the device): top_ids int32[B*topk] holds
 * the node ids, largest value first, ties by id, and -1 past the vector's
 * last non-zero entry; top_x double[B*topk] the values (normalised as
 * opts->normalize says; 0 past the last non-zero entry).  Both host arrays,
 * row-major by vector.  Same seed sets, options and errors as
 * di_solve_batch; DI_EINVAL unless 1 <= topk <= 1024.
 */
di_status di_solve_batch_topk(const di_graph* g, int32_t B, const int64_t* seed_ptr,
                              const int32_t* seeds, const double* seed_w, const di_opts* opts,
                              int32_t topk, int32_t* top_ids, double* top_x, di_stats* stats,
                              void* stream);

/* -------------------------------------------------------------- autotuner */

#define DI_TUNE_SOLVE 0 /* tune single solves (uniform V) */
#define DI_TUNE_BATCH 1 /* tune batched / served personalised PageRank */

typedef struct di_tune_trial {
  di_tune tune;    /* the candidate */
  double seconds;  /* best device time per solve (DI_TUNE_BATCH: per vector) */
  int32_t status;  /* DI_OK, or why the candidate was discarded (e.g. DI_ENOTCONV) */
  int32_t pad;
} di_tune_trial;

/*
 * Picks the threshold schedule (Section 4.2 threshold variant, Section 4.3
 * OP / OP2 scores), the threshold factor c and the window size of the binned
 * scatter for this graph by timing trial solves on the device: first every
 * schedule x c in {1/32, 1/16, 1/8, 1/4, 1/2, 1, 2} at the default window,
 * then the best pair at larger and smaller windows, one size at a time in
 * each direction while the time improves, then the three fastest pairs of
 * the first step at the chosen window with 1024-thread workgroups; for
 * DI_TUNE_SOLVE on a graph of at most DI_SMALL_MAX_NODES
 * nodes, also every schedule x c in the whole-graph window (DI_WINDOW_WHOLE);
 * and for DI_TUNE_SOLVE on a graph that the one-launch solve takes
 * (di_tune.persist), every schedule x c at the smallest window it allows,
 * then the best pair at larger windows while the time improves.
 * Any schedule converges to the same limit (the order
 * independence of Sections 2.2 and 3.1), so only speed is compared.
 * The default knobs (mean, c = 1) run first; every other candidate gets at
 * most four times their rounds (at least 64, at most opts->max_rounds when
 * set) and is discarded if it does not converge within them.
 *
 * mode DI_TUNE_SOLVE times di_solve with uniform V and opts (d, tol,
 * precision).  DI_TUNE_BATCH times di_solve_batch on the B seed sets given
 * (host arrays as in di_solve_batch; required) and scores seconds per vector.
 * opts->tune and opts->flags are ignored.  Each candidate runs once untimed,
 * then twice timed; the faster run counts.
 *
 * The winner is written to *best and cached in the graph per (mode,
 * precision): later calls that pass no tune (di_solve: DI_TUNE_SOLVE;
 * di_solve_batch and servers created afterwards: DI_TUNE_BATCH) use it.
 * trials (may be NULL) receives up to max_trials entries; *n_trials (may be
 * NULL) the number of candidates timed.  DI_EINVAL for bad arguments,
 * DI_ENOTCONV if no candidate converged (nothing cached).
 */
di_status di_autotune(di_graph* g, int32_t mode, const di_opts* opts, int32_t B,
                      const int64_t* seed_ptr, const int32_t* seeds, di_tune* best,
                      di_tune_trial* trials, int32_t max_trials, int32_t* n_trials, void* stream);

/* ----------------------------------------------------------------- server */

typedef struct di_server_opts {
  int64_t hbm_budget_bytes; /* device bytes the server may hold for request state (0 = 32 GiB) */
  int32_t max_slots;        /* concurrent requests on the device (0 = 256) */
  int32_t topk;             /* results kept per request (0 = 100) */
  int32_t precision;        /* DI_FP32_FLUID or DI_FP64 */
  int32_t pad;
  const di_tune* tune;      /* NULL = defaults */
} di_server_opts;

typedef struct di_result {
  uint64_t req_id;
  int32_t status;          /* DI_OK, DI_ENOTCONV, DI_ECANCELED, DI_EDEVICE */
  int32_t k;               /* entries filled in top_ids / top_x */
  int32_t top_ids[1024];   /* highest-ranked nodes, best first (ties: lower id first) */
  double top_x[1024];      /* their normalised scores */
  double residual_l1, err_bound_l1;
  double t_submit, t_admit, t_done; /* seconds on the server's clock */
  int64_t rounds, edges_diffused;
} di_result;

typedef struct di_server_metrics {
  int64_t submitted, admitted, completed, cancelled, queued, active;
  int64_t hbm_in_use, hbm_budget;
  double p50_latency_s, p99_latency_s, qps;
} di_server_metrics;

/* Create a server of personalised PageRank requests: each request is a
   D-iteration solve of X = dPX + (1-d)V with V its seed set (the
   personalisation vector of Section 2.1), stopped by Theorem 2's residual
   ||F||_1 < tol (Section 3.1) and renormalised as in Section 3.3.  The server
   runs one scheduler thread and HIP stream per resident graph. */
di_status di_server_create(const di_server_opts* opts, di_server** out);
/* Register a resident graph (not copied; must outlive the server). */
di_status di_server_add_graph(di_server* s, const di_graph* g, int32_t* graph_id);
/* Enqueue a PPR request (thread-safe, non-blocking): V puts weight w[k] on
   seeds[k] (the personalisation vector of Section 2.1; w NULL = uniform over
   the seeds), d is the damping factor and the request stops when its
   ||F||_1 < tol (Theorem 2, Section 3.1).  seeds (and w) are host arrays
   copied at submit.  DI_EINVAL on bad input,
   DI_ENOMEM if one request can never fit the budget. */
di_status di_server_submit(di_server* s, int32_t graph_id, int32_t n_seeds, const int32_t* seeds,
                           const double* w, double d, double tol, uint64_t* req_id);
/* DI_EAGAIN while pending; otherwise fills *out and forgets the request. */
di_status di_server_poll(di_server* s, uint64_t req_id, di_result* out);
/* Block up to timeout_s (< 0 = forever); DI_EAGAIN on timeout. */
di_status di_server_wait(di_server* s, uint64_t req_id, double timeout_s, di_result* out);
di_status di_server_cancel(di_server* s, uint64_t req_id);
di_status di_server_stats(di_server* s, di_server_metrics* out);
di_status di_server_destroy(di_server* s);

/* ------------------------------------------------------------------ misc */

const char* di_last_error(void);
const char* di_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DI_H */
