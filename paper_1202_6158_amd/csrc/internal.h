// Internal declarations shared by the libdi translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/di.h"

namespace di {

// ---------------------------------------------------------------- errors

void set_error(const std::string& msg);
const std::string& last_error_ref();

struct Fail {
  di_status st;
};

#define DI_HIP(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      ::di::set_error(std::string(#call) + ": " + hipGetErrorString(e_));              \
      throw ::di::Fail{e_ == hipErrorOutOfMemory ? DI_ENOMEM : DI_EDEVICE};            \
    }                                                                                  \
  } while (0)

#define DI_REQUIRE(cond, msg)                   \
  do {                                          \
    if (!(cond)) {                              \
      ::di::set_error(msg);                     \
      throw ::di::Fail{DI_EINVAL};              \
    }                                           \
  } while (0)

// Runs f, mapping di::Fail and std exceptions to a status.
template <typename Fn>
di_status guarded(Fn&& f) {
  try {
    f();
    return DI_OK;
  } catch (const Fail& e) {
    return e.st;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return DI_ENOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return DI_EDEVICE;
  }
}

// Owning device buffer.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  void alloc(size_t n) {
    if (n <= bytes && p) return;
    release();
    if (n == 0) n = 16;
    DI_HIP(hipMalloc(&p, n));
    bytes = n;
  }
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

struct PinnedBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~PinnedBuf() {
    if (p) (void)hipHostFree(p);
  }
  void alloc(size_t n) {
    if (n <= bytes && p) return;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    DI_HIP(hipHostMalloc(&p, n, hipHostMallocDefault));
    bytes = n;
  }
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// --------------------------------------------------------------- constants

constexpr int kBlock = 256;        // threads per workgroup of the streaming kernels
constexpr int kRoundThreads = 512;   // threads per D-iteration round workgroup
constexpr int64_t kMaxNnz = 1ll << 36;  // links per graph
constexpr int kMaxBuckets = 4096;  // destination windows per solve, tables in LDS
constexpr int kMaxBucketsGlobal = 16384;  // the same, tables read from global memory
constexpr int kPullRows = 256;     // rows per pull block (one per thread)
constexpr int kPullNnz = 2048;     // staged in-links per pull block

// ----------------------------------------------------------------- graph

struct Workspace;

struct Graph {
  int64_t n = 0, m = 0, n_dangling = 0;
  bool weighted = false;
  int device = 0;
  // source-CSR (push side)
  DevBuf row_ptr;  // int64[n+1]
  DevBuf deg;      // int32[n] out-degree
  DevBuf col;      // int32[m]
  DevBuf w;        // double[m] (weighted graphs)
  DevBuf indeg;    // int32[n] in-degree (ALGO-OP score)
  // destination-CSR (pull side) and the window layout derived from it
  DevBuf in_ptr;   // int64[n+1]
  DevBuf in_src;   // int32[m]
  DevBuf in_w;     // double[m] (weighted graphs)
  DevBuf pull_blk; // int32[2*npull]: (first row, end row) of each pull block, longest first
  int64_t npull = 0;
  // reusable solve workspaces
  std::mutex ws_mu;
  std::vector<Workspace*> ws_free;
  int servers = 0;
  // Autotuned knobs per (mode, precision), used by calls that pass no tune.
  di_tune tuned[2][2] = {};
  bool has_tuned[2][2] = {};
  ~Graph();
};

// Window size (log2 nodes) of the binned scatter for a graph of n nodes: about
// 512 windows, the round kernel's LDS (fp64 window + per-window tables) within
// the workgroup limit, at most kMaxBuckets windows.  When no size fits (large
// graphs), or when tables == 2, the per-window segment tables stay in global
// memory and only the record counters sit in LDS (at most kMaxBucketsGlobal
// windows); tables == 1 forbids that.  *global_tables reports the choice;
// -1 if no size fits.
int window_log2_for(int64_t n, int requested, int tables, bool* global_tables);
// LDS bytes of the round kernel's dynamic part for window 2^wlog and nb windows.
size_t round_lds_bytes(int wlog, int nb, bool global_tables);
// Whether a single solve of an n-node, m-link graph at 2^wlog-node windows
// (LDS tables) can run every round in one launch (di_tune.persist).
bool persist_fits(int64_t n, int64_t m, int wlog);

// Workspaces (defined in diter.hip).
Workspace* acquire_workspace(Graph* g, int precision, int wlog, bool global_tables);
void release_workspace(Graph* g, Workspace* ws);
void destroy_workspace(Workspace* ws);

// ------------------------------------------------------------ serving engine

// One request's personalisation as the engine admits it into a slot.
struct SlotInit {
  int slot;
  double d, tol;
  std::vector<int32_t> seeds;
  std::vector<double> w;  // empty: uniform over the seeds
};

// Result of a finished slot.
struct SlotResult {
  int slot;
  int status;  // DI_OK, DI_ENOTCONV, DI_EDEVICE
  std::vector<int32_t> ids;
  std::vector<double> x;
  double residual, bound;
  int64_t rounds, edges;
};

// Device state for up to `capacity` concurrent personalised solves on one graph
// (defined in diter.hip).  Not thread-safe: one scheduler thread drives it.
class SlotPool {
 public:
  virtual ~SlotPool() = default;
  virtual int capacity() const = 0;
  virtual int64_t bytes() const = 0;
  // Initialise the slots of `inits` (F = (1-d)V, H = 0, control reset).
  virtual void admit(const std::vector<SlotInit>& inits, hipStream_t s) = 0;
  // `rounds` rounds in a row for every listed slot (each at its own round
  // index; a slot whose solve stops within them returns at once afterwards).
  virtual void step(const std::vector<int>& slots, int rounds, hipStream_t s) = 0;
  // Refresh the host copy of the slots' control blocks (synchronises s) and
  // return the slots among `slots` whose solve has stopped.
  virtual std::vector<int> stopped(const std::vector<int>& slots, hipStream_t s) = 0;
  // Flush and top-k of finished slots (synchronises s).
  virtual void finish(const std::vector<int>& slots, int topk, std::vector<SlotResult>& out,
                      hipStream_t s) = 0;
};

// Bytes of one slot of a pool on g.
int64_t slot_bytes(const Graph* g, int precision);
SlotPool* make_slot_pool(Graph* g, int precision, int capacity, const di_tune* tune);

// Validation helpers.
void validate_d_tol(const di_opts* o);
void validate_vector(const double* v, int64_t n, const char* what);
// The same checks on a device vector: reductions on stream s through dscratch
// (514 device doubles), read back into hscratch (2 pinned host doubles), then
// a sync of s.
void validate_device_vector(const double* v, int64_t n, const char* what, double* dscratch,
                            double* hscratch, hipStream_t s);

// Per-launch HIP event pairs on one stream (DI_TIMING).  Events come from a
// pool created before the timed region and grown in blocks; launches made
// with hipExtLaunchKernel fill them with the kernel's own begin/end times.
struct LaunchTimer {
  hipStream_t s;
  bool on;
  size_t used = 0;
  std::vector<hipEvent_t> a, b;
  LaunchTimer(hipStream_t st, bool enabled, size_t reserve = 256) : s(st), on(enabled) {
    if (on) grow(reserve);
  }
  void grow(size_t k) {
    for (size_t i = 0; i < k; ++i) {
      hipEvent_t e1, e2;
      DI_HIP(hipEventCreate(&e1));
      DI_HIP(hipEventCreate(&e2));
      a.push_back(e1);
      b.push_back(e2);
    }
  }
  // Event pair for the next launch (hipExtLaunchKernel records into them).
  void next(hipEvent_t* e0, hipEvent_t* e1) {
    if (used == a.size()) grow(256);
    *e0 = a[used];
    *e1 = b[used];
    ++used;
  }
  // Sum of the first `count` launches' durations (stream must have drained).
  double total(size_t count) {
    double t = 0.0;
    for (size_t i = 0; i < count && i < used; ++i) {
      float ms = 0.f;
      DI_HIP(hipEventElapsedTime(&ms, a[i], b[i]));
      t += ms * 1e-3;
    }
    return t;
  }
  ~LaunchTimer() {
    for (hipEvent_t e : a) (void)hipEventDestroy(e);
    for (hipEvent_t e : b) (void)hipEventDestroy(e);
  }
};

// Timing helper: records events around a region on a stream.
struct EventTimer {
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t s;
  explicit EventTimer(hipStream_t st) : s(st) {
    DI_HIP(hipEventCreate(&a));
    DI_HIP(hipEventCreate(&b));
    DI_HIP(hipEventRecord(a, s));
  }
  double stop() {
    DI_HIP(hipEventRecord(b, s));
    DI_HIP(hipEventSynchronize(b));
    float ms = 0.f;
    DI_HIP(hipEventElapsedTime(&ms, a, b));
    return ms * 1e-3;
  }
  ~EventTimer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

}  // namespace di

struct di_graph : di::Graph {};
