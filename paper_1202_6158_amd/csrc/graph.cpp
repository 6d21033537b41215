// Graph residency: validation, in-link transpose, device upload.
//
// P is given by its columns (the out-links of every node, Section 2.1).  The
// push side of the D-iteration uses them directly; the pull comparator and
// the destination windows of the binned scatter use the transpose (in-links),
// built here once with a stable counting sort so that every in-link row lists
// its sources in increasing order (deterministic pull sums).
#include <cmath>
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace di {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }
const std::string& last_error_ref() { return g_last_error; }

Graph::~Graph() {
  for (Workspace* ws : ws_free) destroy_workspace(ws);
}

size_t round_lds_bytes(int wlog, int nb, bool global_tables) {
  // fp64 window and a state byte per node; per window either the four segment
  // tables (base, count prefix / rank, offset, capacity: 20 bytes) or only the
  // count prefix / rank (4 bytes)
  return ((size_t)9 << wlog) + (size_t)(global_tables ? 4 : 20) * (nb + 1) + 16;
}

int window_log2_for(int64_t n, int requested, int tables, bool* global_tables) {
  // 160 KiB per workgroup minus the round kernel's static LDS (21.5 KiB at 512
  // threads, 21.6 KiB at 1024); the global-table layout always runs the
  // 1024-thread instance, which leaves it a little more
  constexpr size_t kLdsBudget = 136 * 1024, kLdsBudgetGlobal = 138 * 1024;
  int k0 = 8;
  if (requested >= 8) {
    k0 = std::min(requested, 14);
  } else {
    while (k0 < 14 && (n >> k0) > 512) ++k0;
  }
  auto nb_of = [&](int kk) { return (int)std::min<int64_t>((n + (1ll << kk) - 1) >> kk, 1 << 30); };
  for (const bool gt : {false, true}) {
    if ((gt && tables == 1) || (!gt && tables == 2)) continue;
    const int maxb = gt ? kMaxBucketsGlobal : kMaxBuckets;
    const size_t budget = gt ? kLdsBudgetGlobal : kLdsBudget;
    int k = k0;
    while (k > 8 && round_lds_bytes(k, nb_of(k), gt) > budget) --k;
    while (k < 14 && nb_of(k) > maxb) ++k;
    if (nb_of(k) <= maxb && round_lds_bytes(k, nb_of(k), gt) <= budget) {
      if (global_tables) *global_tables = gt;
      return k;
    }
  }
  return -1;
}

void validate_d_tol(const di_opts* o) {
  DI_REQUIRE(o != nullptr, "opts is NULL");
  DI_REQUIRE(std::isfinite(o->d) && o->d >= 0.0 && o->d < 1.0, "d must satisfy 0 <= d < 1");
  DI_REQUIRE(std::isfinite(o->tol) && o->tol > 0.0, "tol must be > 0");
  DI_REQUIRE(o->precision == DI_FP32_FLUID || o->precision == DI_FP64, "unknown precision");
  DI_REQUIRE(o->max_rounds >= 0, "max_rounds must be >= 0");
}

void validate_vector(const double* v, int64_t n, const char* what) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    DI_REQUIRE(std::isfinite(v[i]) && v[i] >= 0.0,
               std::string(what) + " has a negative or non-finite entry");
    s += v[i];
  }
  DI_REQUIRE(std::fabs(s - 1.0) <= 1e-9, std::string(what) + " does not sum to 1");
}

}  // namespace di

using namespace di;

extern "C" {

const char* di_last_error(void) { return last_error_ref().c_str(); }
const char* di_version(void) { return "libdi 0.1 (gfx950)"; }

di_status di_graph_create(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                          const double* w, void* stream, di_graph** out) {
  return guarded([&] {
    DI_REQUIRE(out != nullptr, "out is NULL");
    *out = nullptr;
    DI_REQUIRE(n >= 1 && n < (1ll << 31), "n must be in [1, 2^31)");
    DI_REQUIRE(nnz >= 0 && nnz < kMaxNnz, "nnz must be in [0, 2^36)");
    DI_REQUIRE(row_ptr != nullptr, "row_ptr is NULL");
    DI_REQUIRE(nnz == 0 || col_idx != nullptr, "col_idx is NULL");
    DI_REQUIRE(row_ptr[0] == 0, "row_ptr[0] must be 0");
    DI_REQUIRE(row_ptr[n] == nnz, "row_ptr[n] must equal nnz");
    int64_t dangling = 0;
    for (int64_t i = 0; i < n; ++i) {
      DI_REQUIRE(row_ptr[i + 1] >= row_ptr[i], "row_ptr must be non-decreasing");
      if (row_ptr[i + 1] == row_ptr[i]) ++dangling;
      DI_REQUIRE(row_ptr[i + 1] - row_ptr[i] < (1ll << 31), "out-degree too large");
    }
    std::vector<int32_t> indeg(n, 0);
    for (int64_t e = 0; e < nnz; ++e) {
      DI_REQUIRE(col_idx[e] >= 0 && col_idx[e] < n, "col_idx entry out of range");
      indeg[col_idx[e]] += 1;
    }
    if (w) {
      for (int64_t i = 0; i < n; ++i) {
        if (row_ptr[i + 1] == row_ptr[i]) continue;
        double s = 0.0;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
          DI_REQUIRE(std::isfinite(w[e]) && w[e] >= 0.0, "weight negative or not finite");
          s += w[e];
        }
        DI_REQUIRE(std::fabs(s - 1.0) <= 1e-9, "out-link weights of a node must sum to 1");
      }
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto* g = new di_graph();
    try {
      DI_HIP(hipGetDevice(&g->device));
      g->n = n;
      g->m = nnz;
      g->n_dangling = dangling;
      g->weighted = w != nullptr;
      std::vector<int32_t> deg(n);
      for (int64_t i = 0; i < n; ++i) deg[i] = (int32_t)(row_ptr[i + 1] - row_ptr[i]);
      // Stable counting sort of the links by destination -> in-link CSR.
      std::vector<int64_t> in_ptr(n + 1, 0);
      for (int64_t j = 0; j < n; ++j) in_ptr[j + 1] = in_ptr[j] + indeg[j];
      std::vector<int32_t> in_src(nnz > 0 ? nnz : 1);
      std::vector<double> in_w(w ? nnz : 0);
      {
        std::vector<int64_t> fill(in_ptr.begin(), in_ptr.end() - 1);
        for (int64_t i = 0; i < n; ++i)
          for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            int64_t slot = fill[col_idx[e]]++;
            in_src[slot] = (int32_t)i;
            if (w) in_w[slot] = w[e];
          }
      }
      // Pull blocks: up to kPullRows rows and kPullNnz in-links each; a row
      // with more in-links than that is a block of its own.  Stored as
      // (first row, end row) pairs, longest block first.
      std::vector<std::pair<int32_t, int32_t>> blocks;
      {
        int64_t r = 0;
        while (r < n) {
          int64_t r0 = r;
          int64_t nz = 0;
          while (r < n && r - r0 < kPullRows) {
            int64_t rn = in_ptr[r + 1] - in_ptr[r];
            if (r > r0 && nz + rn > kPullNnz) break;
            nz += rn;
            ++r;
            if (nz > kPullNnz) break;  // long row alone
          }
          blocks.emplace_back((int32_t)r0, (int32_t)r);
        }
      }
      std::stable_sort(blocks.begin(), blocks.end(), [&](const auto& x, const auto& y) {
        return in_ptr[x.second] - in_ptr[x.first] > in_ptr[y.second] - in_ptr[y.first];
      });
      std::vector<int32_t> blk;
      for (const auto& p : blocks) {
        blk.push_back(p.first);
        blk.push_back(p.second);
      }
      g->npull = (int64_t)blocks.size();
      g->row_ptr.alloc((n + 1) * 8);
      g->deg.alloc(n * 4);
      g->indeg.alloc(n * 4);
      g->col.alloc(std::max<int64_t>(nnz, 1) * 4);
      g->in_ptr.alloc((n + 1) * 8);
      g->in_src.alloc(std::max<int64_t>(nnz, 1) * 4);
      g->pull_blk.alloc(blk.size() * 4);
      DI_HIP(hipMemcpyAsync(g->row_ptr.p, row_ptr, (n + 1) * 8, hipMemcpyHostToDevice, s));
      DI_HIP(hipMemcpyAsync(g->deg.p, deg.data(), n * 4, hipMemcpyHostToDevice, s));
      DI_HIP(hipMemcpyAsync(g->indeg.p, indeg.data(), n * 4, hipMemcpyHostToDevice, s));
      if (nnz) DI_HIP(hipMemcpyAsync(g->col.p, col_idx, nnz * 4, hipMemcpyHostToDevice, s));
      DI_HIP(hipMemcpyAsync(g->in_ptr.p, in_ptr.data(), (n + 1) * 8, hipMemcpyHostToDevice, s));
      if (nnz) DI_HIP(hipMemcpyAsync(g->in_src.p, in_src.data(), nnz * 4, hipMemcpyHostToDevice, s));
      DI_HIP(hipMemcpyAsync(g->pull_blk.p, blk.data(), blk.size() * 4, hipMemcpyHostToDevice, s));
      if (w) {
        g->w.alloc(std::max<int64_t>(nnz, 1) * 8);
        g->in_w.alloc(std::max<int64_t>(nnz, 1) * 8);
        if (nnz) {
          DI_HIP(hipMemcpyAsync(g->w.p, w, nnz * 8, hipMemcpyHostToDevice, s));
          DI_HIP(hipMemcpyAsync(g->in_w.p, in_w.data(), nnz * 8, hipMemcpyHostToDevice, s));
        }
      }
      DI_HIP(hipStreamSynchronize(s));
    } catch (...) {
      delete g;
      throw;
    }
    *out = g;
  });
}

di_status di_graph_destroy(di_graph* g) {
  return guarded([&] {
    if (!g) return;
    if (g->servers > 0) {
      set_error("graph is still registered with a server");
      throw Fail{DI_EBUSY};
    }
    delete g;
  });
}

di_status di_window_layout(int64_t n, const di_tune* tune, int32_t* window_log2,
                           int32_t* global_tables) {
  return guarded([&] {
    DI_REQUIRE(window_log2 != nullptr && global_tables != nullptr, "NULL argument");
    DI_REQUIRE(n >= 1 && n < (1ll << 31), "n must be in [1, 2^31)");
    const int tables = tune ? tune->tables : 0;
    DI_REQUIRE(tables >= 0 && tables <= 2, "tables must be 0, 1 or 2");
    if (tune && tune->window_log2 == DI_WINDOW_WHOLE) {
      DI_REQUIRE(n <= DI_SMALL_MAX_NODES, "DI_WINDOW_WHOLE needs n <= DI_SMALL_MAX_NODES");
      *window_log2 = DI_WINDOW_WHOLE;
      *global_tables = 0;
      return;
    }
    bool gt = false;
    const int k = window_log2_for(n, tune ? tune->window_log2 : 0, tables, &gt);
    DI_REQUIRE(k > 0, "graph has too many nodes for the window tables");
    *window_log2 = k;
    *global_tables = gt ? 1 : 0;
  });
}

di_status di_graph_info(const di_graph* g, int64_t* n, int64_t* nnz, int64_t* n_dangling) {
  return guarded([&] {
    DI_REQUIRE(g != nullptr, "graph is NULL");
    if (n) *n = g->n;
    if (nnz) *nnz = g->m;
    if (n_dangling) *n_dangling = g->n_dangling;
  });
}

}  // extern "C"
