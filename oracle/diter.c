/*
 * CPU oracle for the D-iteration PageRank solve -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, sequential fp64 code written from the paper ("Optimized on-line
 * computation of PageRank algorithm", D. Hong, arXiv 1202.6158).  It shares
 * no code with the GPU library and is used only by the tests, the smoke check
 * and the CPU baseline timing.  Nothing in the product path may call it.
 *
 * Problem (Section 2.1): P is an N x N non-negative matrix whose non-zero
 * columns sum to one; column i holds the out-links of node i.  For an
 * unweighted graph p(j,i) = m_ij / outdeg(i), where m_ij counts the links
 * i -> j (repeated links and self-loops count with multiplicity).  A node with
 * no out-link (dangling node) has a zero column and is NOT completed
 * (Section 3.3).  The solve targets X = dPX + (1-d)V, 0 <= d < 1.
 *
 * State (Section 2.2, fluid and history recurrences):
 *   F_0 = (1-d) V,  H_0 = 0.
 *   Diffusing node i:  sent = F_i;  H_i += sent;  F_i = 0;
 *                      if i is dangling the fluid only leaves the system,
 *                      else F_j += d * sent * p(j,i) for every child j.
 *   The running remaining-fluid scalar R starts at 1-d (for a normalised V)
 *   and loses (1-d)*sent per non-dangling diffusion and sent per dangling one
 *   (Section 3.3).
 * Stop: when the freshly summed ||F||_1 drops below tol (Theorem 2 makes
 * ||F||_1/(1-d) the L1 distance of H to the limit on graphs without dangling
 * nodes, and an upper bound otherwise).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int64_t picks;    /* diffusions that moved fluid (zero-fluid picks are free, Section 4.2) */
  int64_t edges;    /* elementary steps: one per out-link used (Section 4.2) */
  int64_t rounds;   /* set steps, sweeps or matrix products */
  double residual;  /* ||F||_1 summed afresh at exit (power iteration: last ||X_n - X_n-1||_1) */
  double running_r; /* the running scalar R of the algorithm */
  int32_t converged;
  int32_t pad;
} or_stats;

/* Orders of the diffusion sequence I (Section 4). */
enum {
  OR_PER = 0,   /* i_n = n mod N */
  OR_RAND = 1,  /* i_n uniform on {0..N-1} */
  OR_MAX = 2,   /* i_n = argmax F */
  OR_SWEEP = 3, /* sweeps over 0..N-1, diffusing every node whose fluid is at
                   least theta = c*||F||_1/N when visited; theta is recomputed
                   each sweep (the threshold variant of Section 4.2) */
  OR_OP = 4,    /* argmax F_i / ((#in_i + 1)(#out_i + 1))  (Section 4.3) */
  OR_OP2 = 5    /* argmax F_i / (#out_i + 1)               (Section 4.3) */
};

static double l1(int64_t n, const double* f) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += fabs(f[i]);
  return s;
}

/* One diffusion of node i, the inner body of ALGO-REF with the dangling rule. */
static void diffuse(int64_t i, const int64_t* rp, const int32_t* ci, double d,
                    double* F, double* H, double* R, or_stats* st) {
  double sent = F[i];
  if (sent == 0.0) return;
  H[i] += sent;
  F[i] = 0.0;
  int64_t deg = rp[i + 1] - rp[i];
  if (deg == 0) {
    *R -= sent;
  } else {
    double share = sent * d / (double)deg; /* sent * p(j,i) * d for one link */
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) F[ci[e]] += share;
    *R -= sent * (1.0 - d);
  }
  st->picks += 1;
  st->edges += deg;
}

static uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

/*
 * Sequential D-iteration (ALGO-REF with dangling nodes, Sections 2.2 and 3.3)
 * in one of the orders above.  F and H are in/out: the caller initialises them
 * (F = (1-d)V, H = 0 for a fresh solve; any state satisfying Theorem 1 to
 * resume).  r0 is the initial running R.  c is the threshold factor of
 * OR_SWEEP.  trace (may be NULL) receives ||F||_1 after each of the first
 * trace_len picks that moved fluid (used to check the Lemma of Section 3.1).
 * Returns 0 when converged, 1 when max_picks was reached first.
 */
int or_diter(int64_t n, const int64_t* rp, const int32_t* ci, double d, double tol,
             int order, double c, uint64_t seed, int64_t max_picks, double r0,
             double* F, double* H, double* trace, int64_t trace_len, or_stats* st) {
  memset(st, 0, sizeof(*st));
  double R = r0;
  double* w = NULL; /* per-node weight of OR_OP / OR_OP2 */
  if (order == OR_OP || order == OR_OP2) {
    w = (double*)calloc((size_t)n, sizeof(double));
    int64_t* indeg = (int64_t*)calloc((size_t)n, sizeof(int64_t));
    for (int64_t e = 0; e < rp[n]; ++e) indeg[ci[e]] += 1;
    for (int64_t i = 0; i < n; ++i) {
      double out = (double)(rp[i + 1] - rp[i]);
      w[i] = order == OR_OP ? 1.0 / (((double)indeg[i] + 1.0) * (out + 1.0)) : 1.0 / (out + 1.0);
    }
    free(indeg);
  }
  int64_t k = 0; /* picks made, including free zero-fluid ones */
  int64_t traced = 0;
  double theta = 0.0;
  int rc = 1;
  for (;;) {
    /* Stop test on the freshly summed fluid; the running R only says when to
       look (it equals ||F||_1 up to rounding). */
    if (R <= tol || k % n == 0) {
      if (l1(n, F) < tol) { rc = 0; break; }
    }
    if (st->picks >= max_picks) break;
    int64_t i;
    if (order == OR_PER) {
      i = k % n;
    } else if (order == OR_RAND) {
      i = (int64_t)(splitmix64(seed + (uint64_t)k) % (uint64_t)n);
    } else if (order == OR_MAX || order == OR_OP || order == OR_OP2) {
      i = 0;
      double best = -1.0;
      for (int64_t j = 0; j < n; ++j) {
        double s = w ? F[j] * w[j] : F[j];
        if (s > best) { best = s; i = j; }
      }
    } else { /* OR_SWEEP */
      i = k % n;
      if (i == 0) {
        /* New sweep: theta = c * ||F||_1 / N, but never above the largest
           fluid, which is at least the mean, so every sweep moves fluid. */
        double mx = 0.0;
        for (int64_t j = 0; j < n; ++j) mx = F[j] > mx ? F[j] : mx;
        theta = c * l1(n, F) / (double)n;
        if (theta > mx) theta = mx;
        st->rounds += 1;
      }
      if (!(F[i] >= theta)) { ++k; continue; }
    }
    ++k;
    int64_t before = st->picks;
    diffuse(i, rp, ci, d, F, H, &R, st);
    if (trace && st->picks > before && traced < trace_len) trace[traced++] = l1(n, F);
  }
  st->residual = l1(n, F);
  st->running_r = R;
  st->converged = rc == 0;
  free(w);
  return rc;
}

/*
 * One set step: every node of S = {i : F_i >= theta and F_i > 0} is diffused
 * at once, F <- (I - J_S + d P J_S) F and H <- H + J_S F, where J_S is the
 * diagonal selector of S (the recurrences of Section 2.2 with J_{i_n}
 * replaced by J_S; the induction proving Theorem 1 goes through unchanged).
 * F may hold single-precision values widened to double; the comparison
 * F_i >= theta is made in double on the values as given.  taken receives 1
 * for the nodes of S (may be NULL).  Returns |S|.
 */
int64_t or_set_step(int64_t n, const int64_t* rp, const int32_t* ci, double d,
                    double theta, double* F, double* H, uint8_t* taken, or_stats* st) {
  double* sent = (double*)calloc((size_t)n, sizeof(double));
  int64_t count = 0;
  for (int64_t i = 0; i < n; ++i) {
    int in = F[i] > 0.0 && F[i] >= theta;
    if (taken) taken[i] = (uint8_t)in;
    if (!in) continue;
    sent[i] = F[i];
    H[i] += F[i];
    F[i] = 0.0;
    ++count;
  }
  for (int64_t i = 0; i < n; ++i) {
    if (sent[i] == 0.0) continue;
    int64_t deg = rp[i + 1] - rp[i];
    if (deg == 0) {
      st->running_r -= sent[i];
    } else {
      double share = sent[i] * d / (double)deg;
      for (int64_t e = rp[i]; e < rp[i + 1]; ++e) F[ci[e]] += share;
      st->running_r -= sent[i] * (1.0 - d);
    }
    st->picks += 1;
    st->edges += deg;
  }
  st->rounds += 1;
  free(sent);
  return count;
}

/*
 * D-iteration by set steps with theta_r = c * ||F_r||_1 / N (the threshold
 * variant of Section 4.2 with the whole set taken at once).  If no node
 * reaches theta, theta is lowered to the largest fluid, which is at least the
 * mean (the Lemma of Section 3.1 then still applies).  c = 0 gives the
 * Jacobi form: every node with fluid diffuses in every round.
 */
int or_diter_sets(int64_t n, const int64_t* rp, const int32_t* ci, double d, double tol,
                  double c, int64_t max_rounds, double r0, double* F, double* H,
                  or_stats* st) {
  memset(st, 0, sizeof(*st));
  st->running_r = r0;
  int rc = 1;
  while (st->rounds < max_rounds) {
    double nf = l1(n, F);
    if (nf < tol) { rc = 0; break; }
    double theta = c * nf / (double)n;
    double mx = 0.0;
    for (int64_t i = 0; i < n; ++i) mx = F[i] > mx ? F[i] : mx;
    if (theta > mx) theta = mx;
    or_set_step(n, rp, ci, d, theta, F, H, NULL, st);
  }
  if (rc == 1 && l1(n, F) < tol) rc = 0;
  st->residual = l1(n, F);
  st->converged = rc == 0;
  return rc;
}

/*
 * MAT-ITER (Section 2.1 and 4): X_{n+1} = d P X_n + (1-d) V from X_0 = 0,
 * with no dangling completion, until ||X_n - X_{n-1}||_1 < tol.  x receives
 * the last iterate (not normalised).  Returns 0 when converged.
 */
int or_power(int64_t n, const int64_t* rp, const int32_t* ci, const double* v, double d,
             double tol, int64_t max_iter, double* x, or_stats* st) {
  memset(st, 0, sizeof(*st));
  double* y = (double*)malloc((size_t)n * sizeof(double));
  for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
  int rc = 1;
  while (st->rounds < max_iter) {
    for (int64_t j = 0; j < n; ++j) y[j] = (1.0 - d) * v[j];
    for (int64_t i = 0; i < n; ++i) {
      int64_t deg = rp[i + 1] - rp[i];
      if (deg == 0) continue;
      double share = d * x[i] / (double)deg;
      for (int64_t e = rp[i]; e < rp[i + 1]; ++e) y[ci[e]] += share;
    }
    double diff = 0.0;
    for (int64_t j = 0; j < n; ++j) diff += fabs(y[j] - x[j]);
    memcpy(x, y, (size_t)n * sizeof(double));
    st->rounds += 1;
    st->edges += rp[n];
    st->residual = diff;
    if (diff < tol) { rc = 0; break; }
  }
  st->converged = rc == 0;
  free(y);
  return rc;
}

/*
 * The same MAT-ITER on every host core (OpenMP), for the CPU baseline timing:
 * each product is taken as a pull over in-links, y_j = (1-d) v_j +
 * d sum_{i -> j} x_i / outdeg(i), one destination row per loop iteration, so
 * rows are independent and only the summation order differs from or_power.
 * The in-link lists are built first (a counting sort of the links by
 * destination).  *threads receives the number of threads used.
 */
int or_power_omp(int64_t n, const int64_t* rp, const int32_t* ci, const double* v, double d,
                 double tol, int64_t max_iter, double* x, or_stats* st, int32_t* threads) {
  memset(st, 0, sizeof(*st));
  const int64_t m = rp[n];
  int64_t* ip = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  int32_t* is = (int32_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
  double* z = (double*)malloc((size_t)n * sizeof(double));
  double* y = (double*)malloc((size_t)n * sizeof(double));
  for (int64_t e = 0; e < m; ++e) ip[ci[e] + 1] += 1;
  for (int64_t j = 0; j < n; ++j) ip[j + 1] += ip[j];
  int64_t* fill = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  memcpy(fill, ip, (size_t)n * sizeof(int64_t));
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) is[fill[ci[e]]++] = (int32_t)i;
  free(fill);
  int nt = 1;
#pragma omp parallel
  {
#pragma omp single
    nt = omp_get_num_threads();
  }
  *threads = nt;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
  int rc = 1;
  while (st->rounds < max_iter) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      const int64_t deg = rp[i + 1] - rp[i];
      z[i] = deg > 0 ? x[i] / (double)deg : 0.0;
    }
    double diff = 0.0;
#pragma omp parallel for schedule(dynamic, 4096) reduction(+ : diff)
    for (int64_t j = 0; j < n; ++j) {
      double acc = 0.0;
      for (int64_t e = ip[j]; e < ip[j + 1]; ++e) acc += z[is[e]];
      y[j] = (1.0 - d) * v[j] + d * acc;
      diff += fabs(y[j] - x[j]);
    }
    double* t = x;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) t[j] = y[j];
    st->rounds += 1;
    st->edges += m;
    st->residual = diff;
    if (diff < tol) { rc = 0; break; }
  }
  st->converged = rc == 0;
  free(ip);
  free(is);
  free(z);
  free(y);
  return rc;
}
