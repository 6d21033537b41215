// Seeded synthetic graph generator (input generation only).
//
// Produces directed graphs in source-ordered CSR form (out-links per node),
// the shape of the web graphs the D-iteration is evaluated on (Section 4):
// power-law out-degrees, power-law in-degrees through preferential attachment,
// a fixed fraction of dangling nodes (out-degree 0), and optionally a
// host-block ("web") locality structure.  It contains none of the PageRank
// arithmetic; both the CPU oracle and the GPU library consume its output.
//
// Every random draw comes from one std::mt19937_64 stream per phase, seeded
// from the caller's seed, so a (recipe, seed) pair always yields the same graph.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <random>
#include <vector>

namespace {

using rng_t = std::mt19937_64;

inline double unit(rng_t& g) {  // uniform in [0,1) with 53 random bits
  return (double)(g() >> 11) * (1.0 / 9007199254740992.0);
}
inline int64_t below(rng_t& g, int64_t n) {  // uniform integer in [0,n)
  return (int64_t)(g() % (uint64_t)n);
}

// Mean of the shifted Zipf law pmf(k) ∝ (k+s)^-alpha on [1,kmax].
double zipf_mean(double alpha, double s, int kmax) {
  double num = 0.0, den = 0.0;
  for (int k = 1; k <= kmax; ++k) {
    double w = std::pow(k + s, -alpha);
    num += k * w;
    den += w;
  }
  return num / den;
}

}  // namespace

extern "C" {

// Shift s >= 0 such that the shifted Zipf law on [1,kmax] has the given mean.
// Returns -1 if the mean is outside what a non-negative shift can reach.
double wl_zipf_shift(double alpha, int kmax, double mean) {
  double lo = 0.0, hi = 1.0;
  if (zipf_mean(alpha, lo, kmax) > mean) return -1.0;
  while (zipf_mean(alpha, hi, kmax) < mean) {
    hi *= 2.0;
    if (hi > 1e9) return -1.0;
  }
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (zipf_mean(alpha, mid, kmax) < mean) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

// Out-degrees: round(dangling*n) nodes chosen uniformly get degree 0; every
// other node draws from the shifted Zipf law (alpha, shift) on [1,kmax].
// outdeg must hold n entries.  Returns the edge count.
int64_t wl_outdeg(int64_t n, double alpha, double shift, int kmax,
                  double dangling, uint64_t seed, int32_t* outdeg) {
  rng_t g(seed * 0x9E3779B97F4A7C15ull + 1);
  std::vector<double> cdf(kmax);
  double acc = 0.0;
  for (int k = 1; k <= kmax; ++k) {
    acc += std::pow(k + shift, -alpha);
    cdf[k - 1] = acc;
  }
  for (auto& c : cdf) c /= acc;
  cdf[kmax - 1] = 1.0;
  int64_t nd = (int64_t)std::llround(dangling * (double)n);
  if (nd > n) nd = n;
  // Partial Fisher-Yates picks the dangling set.
  std::vector<int64_t> perm(n);
  for (int64_t i = 0; i < n; ++i) perm[i] = i;
  std::vector<uint8_t> is_dangling(n, 0);
  for (int64_t i = 0; i < nd; ++i) {
    int64_t j = i + below(g, n - i);
    std::swap(perm[i], perm[j]);
    is_dangling[perm[i]] = 1;
  }
  int64_t total = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (is_dangling[i]) { outdeg[i] = 0; continue; }
    double u = unit(g);
    int k = (int)(std::upper_bound(cdf.begin(), cdf.end(), u) - cdf.begin()) + 1;
    if (k > kmax) k = kmax;
    if (k > n - 1) k = (int)(n - 1);  // no self-loops, no multi-edges
    outdeg[i] = k;
    total += k;
  }
  return total;
}

// Targets for every edge slot.  row_ptr (n+1 entries) is the exclusive prefix
// sum of the out-degrees; col_idx receives row_ptr[n] targets, sorted within
// each row.  Nodes "arrive" in a random order and emit their out-links on
// arrival (a growing network, Price's preferential attachment); each link
//   - with probability p_intra (block > 0): goes to a uniform node of the
//     source's block of `block` consecutive ids, other than the source;
//   - else with probability p_uniform: goes to a uniform node (so that links
//     also point to nodes that arrive later and the graph has cycles);
//   - else goes to an arrived node j with P(j) ∝ indeg_so_far(j) + 1, drawn
//     as an urn: uniform over the a arrived nodes with probability a/(a+t),
//     else the target of a uniformly chosen earlier link (t links so far).
// Self-loops and repeated targets of one source are redrawn.  With about m
// attachment links per node this gives in-degrees with the power-law tail
// exponent 2 + 1/m of Price's model.
// Returns 0, or -1 if the degrees cannot be realised without repeats.
int wl_targets(int64_t n, const int64_t* row_ptr, int32_t* col_idx,
               int64_t block, double p_intra, double p_uniform, uint64_t seed) {
  const int64_t m = row_ptr[n];
  for (int64_t i = 0; i < n; ++i)
    if (row_ptr[i + 1] - row_ptr[i] > n - 1) return -1;
  rng_t g(seed * 0x9E3779B97F4A7C15ull + 2);
  std::vector<int32_t> arrival(n);
  for (int64_t i = 0; i < n; ++i) arrival[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; --i) std::swap(arrival[i], arrival[below(g, i + 1)]);
  std::vector<int32_t> placed(m);  // target of the t-th link in arrival order
  int64_t t = 0;
  for (int64_t a = 0; a < n; ++a) {
    const int32_t u = arrival[a];
    const int64_t arrived = a + 1;
    int32_t* row = col_idx + row_ptr[u];
    const int32_t deg = (int32_t)(row_ptr[u + 1] - row_ptr[u]);
    for (int32_t have = 0; have < deg; ++have) {
      auto taken = [&](int64_t v) {
        if (v == u) return true;
        for (int32_t q = 0; q < have; ++q)
          if (row[q] == v) return true;
        return false;
      };
      int64_t v = -1;
      for (int attempt = 0;; ++attempt) {
        if (attempt >= 64) {
          v = below(g, n);  // saturated neighbourhood: plain uniform redraw
        } else if (block > 0 && unit(g) < p_intra) {
          int64_t b0 = (u / block) * block;
          int64_t bn = std::min(block, n - b0);
          if (bn <= 1) {
            v = below(g, n);
          } else {
            v = b0 + below(g, bn - 1);
            if (v >= u) ++v;
          }
        } else if (unit(g) < p_uniform) {
          v = below(g, n);
        } else if (t == 0 || unit(g) * (double)(arrived + t) < (double)arrived) {
          v = arrival[below(g, arrived)];
        } else {
          v = placed[below(g, t)];
        }
        if (!taken(v)) break;
      }
      row[have] = (int32_t)v;
      placed[t++] = (int32_t)v;
    }
  }
  for (int64_t i = 0; i < n; ++i) std::sort(col_idx + row_ptr[i], col_idx + row_ptr[i + 1]);
  return 0;
}

}  // extern "C"
