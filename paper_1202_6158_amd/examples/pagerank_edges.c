/*
 * PageRank of an edge list through the C ABI alone (no Python, no torch):
 * reads "src dst" pairs (0-based ids, one link per line) from a file, builds
 * the out-link CSR, solves X = dPX + (1-d)V with the D-iteration (host
 * buffers: the library copies V in and x out) and with the power iteration,
 * and prints the largest entries of both and the L1 distance between them.
 *
 *   pagerank_edges EDGES [d=0.85] [tol=1e-10] [top=10]
 *
 * Output, one record per line:
 *   n N links L
 *   diter rounds R links E residual F bound B
 *   power products P residual F bound B
 *   top RANK NODE X_DITER X_POWER
 *   l1 DIFF
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "di.h"

static int fail(const char* what, di_status st) {
  fprintf(stderr, "%s failed (%d): %s\n", what, (int)st, di_last_error());
  return 1;
}

int main(int argc, char** argv) {
  if (argc < 2) {
    fprintf(stderr, "usage: %s EDGES [d] [tol] [top]\n", argv[0]);
    return 2;
  }
  const double d = argc > 2 ? atof(argv[2]) : 0.85;
  const double tol = argc > 3 ? atof(argv[3]) : 1e-10;
  const int top = argc > 4 ? atoi(argv[4]) : 10;

  FILE* f = fopen(argv[1], "r");
  if (!f) {
    perror(argv[1]);
    return 2;
  }
  int64_t cap = 1 << 20, m = 0, n = 0;
  int32_t* src = malloc(cap * sizeof(int32_t));
  int32_t* dst = malloc(cap * sizeof(int32_t));
  long a, b;
  while (fscanf(f, "%ld %ld", &a, &b) == 2) {
    if (a < 0 || b < 0 || a >= INT32_MAX || b >= INT32_MAX) {
      fprintf(stderr, "bad node id on line %lld\n", (long long)m + 1);
      return 2;
    }
    if (m == cap) {
      cap *= 2;
      src = realloc(src, cap * sizeof(int32_t));
      dst = realloc(dst, cap * sizeof(int32_t));
    }
    src[m] = (int32_t)a;
    dst[m] = (int32_t)b;
    ++m;
    if (a + 1 > n) n = a + 1;
    if (b + 1 > n) n = b + 1;
  }
  fclose(f);
  if (n == 0) {
    fprintf(stderr, "no links read\n");
    return 2;
  }

  /* out-link CSR by a counting sort on the source (stable: file order kept) */
  int64_t* row_ptr = calloc(n + 1, sizeof(int64_t));
  int32_t* col = malloc((m > 0 ? m : 1) * sizeof(int32_t));
  for (int64_t e = 0; e < m; ++e) row_ptr[src[e] + 1]++;
  for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] += row_ptr[i];
  int64_t* fill = malloc(n * sizeof(int64_t));
  memcpy(fill, row_ptr, n * sizeof(int64_t));
  for (int64_t e = 0; e < m; ++e) col[fill[src[e]]++] = dst[e];
  free(fill);
  free(src);
  free(dst);
  printf("n %lld links %lld\n", (long long)n, (long long)m);

  di_graph* g = NULL;
  di_status st = di_graph_create(n, m, row_ptr, col, NULL, NULL, &g);
  if (st != DI_OK) return fail("di_graph_create", st);

  di_opts o;
  memset(&o, 0, sizeof(o));
  o.d = d;
  o.tol = tol;
  o.precision = DI_FP64;
  o.normalize = 1;
  double* x = malloc(n * sizeof(double));
  double* xp = malloc(n * sizeof(double));
  di_stats s, sp;
  st = di_solve(g, NULL, &o, x, &s, NULL); /* V = NULL: uniform; x: host buffer */
  if (st != DI_OK) return fail("di_solve", st);
  printf("diter rounds %lld links %lld residual %.6e bound %.6e\n", (long long)s.rounds,
         (long long)s.edges_diffused, s.residual_l1, s.err_bound_l1);
  st = di_power_solve(g, NULL, &o, xp, &sp, NULL);
  if (st != DI_OK) return fail("di_power_solve", st);
  printf("power products %lld residual %.6e bound %.6e\n", (long long)sp.rounds, sp.residual_l1,
         sp.err_bound_l1);

  /* the `top` largest entries of x (selection by repeated scans: top is small) */
  char* used = calloc(n, 1);
  for (int k = 0; k < top && k < n; ++k) {
    int64_t best = -1;
    for (int64_t i = 0; i < n; ++i)
      if (!used[i] && (best < 0 || x[i] > x[best])) best = i;
    used[best] = 1;
    printf("top %d %lld %.17g %.17g\n", k, (long long)best, x[best], xp[best]);
  }
  double l1 = 0.0;
  for (int64_t i = 0; i < n; ++i) l1 += x[i] > xp[i] ? x[i] - xp[i] : xp[i] - x[i];
  printf("l1 %.6e\n", l1);

  free(used);
  free(x);
  free(xp);
  free(row_ptr);
  free(col);
  di_graph_destroy(g);
  return 0;
}
