/*
 * Thread-sanitizer driver of the FP64 oracle (test infrastructure): the OpenMP loops of
 * qaoa_oracle.c run under ThreadSanitizer on a few small instances, and every result with
 * several threads must equal the one-thread result to rounding (the parallel loops only
 * split independent amplitudes and sum reductions).  Built and run by oracle/sanitize.py.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_cut_values(int n, int m, const int32_t *edges, const int32_t *wts, int32_t *out);
int orc_energy(int n, int m, const int32_t *edges, const int32_t *wts, int T, const int32_t *ti, const int32_t *tj,
               const double *tw, int p, const double *gamma, const double *beta, double *energy_terms,
               double *energy_direct, double *zz_out, double *norm_out);
int orc_energy_grad(int n, int m, const int32_t *edges, const int32_t *wts, int T, const int32_t *ti,
                    const int32_t *tj, const double *tw, int p, const double *gamma, const double *beta, double *energy,
                    double *dgamma, double *dbeta, double *final_dev);

typedef struct {
  double e, ed, nrm, g[8], b[8], dev;
} result;

static result run(int n, int m, const int32_t *edges, const int32_t *wts, int T, const int32_t *ti, const int32_t *tj,
                  const double *tw, int p, const double *gam, const double *bet) {
  result r;
  double zz[64];
  if (orc_energy(n, m, edges, wts, T, ti, tj, tw, p, gam, bet, &r.e, &r.ed, zz, &r.nrm) != 0) exit(2);
  double e2;
  if (orc_energy_grad(n, m, edges, wts, T, ti, tj, tw, p, gam, bet, &e2, r.g, r.b, &r.dev) != 0) exit(2);
  return r;
}

static int same(double a, double b) { return fabs(a - b) <= 1e-12 * (fabs(a) + fabs(b) + 1.0); }

int main(void) {
  int32_t edges[2 * 64], wts[64], ti[64], tj[64];
  double tw[64];
  int fails = 0;
  for (int c = 0; c < 3; ++c) {
    int n = 0, m = 0, p = 2;
    if (c == 0) {  /* cycle C_12 */
      n = 12;
      for (int v = 0; v < n; ++v, ++m) {
        edges[2 * m] = v;
        edges[2 * m + 1] = (v + 1) % n;
      }
    } else if (c == 1) {  /* K_8 */
      n = 8;
      p = 1;
      for (int u = 0; u < n; ++u)
        for (int v = u + 1; v < n; ++v, ++m) {
          edges[2 * m] = u;
          edges[2 * m + 1] = v;
        }
    } else {  /* star with 11 leaves */
      n = 12;
      p = 3;
      for (int v = 1; v < n; ++v, ++m) {
        edges[2 * m] = 0;
        edges[2 * m + 1] = v;
      }
    }
    for (int e = 0; e < m; ++e) {
      wts[e] = 1 + (e % 3);
      ti[e] = edges[2 * e];
      tj[e] = edges[2 * e + 1];
      tw[e] = wts[e];
    }
    const double gam[3] = {0.41, 1.3, 2.2}, bet[3] = {0.77, 0.35, 1.1};
    int32_t *cuts = (int32_t *)malloc(sizeof(int32_t) << n);
    orc_cut_values(n, m, edges, wts, cuts);
    free(cuts);
    omp_set_num_threads(1);
    result r1 = run(n, m, edges, wts, m, ti, tj, tw, p, gam, bet);
    omp_set_num_threads(4);
    result r4 = run(n, m, edges, wts, m, ti, tj, tw, p, gam, bet);
    int ok = same(r1.e, r4.e) && same(r1.ed, r4.ed) && same(r1.nrm, r4.nrm) && fabs(r4.nrm - 1.0) < 1e-12 &&
             r4.dev < 1e-12 && same(r1.e, r1.ed);
    for (int l = 0; l < p; ++l) ok = ok && same(r1.g[l], r4.g[l]) && same(r1.b[l], r4.b[l]);
    printf("case %d: n=%d m=%d p=%d energy %.15f %s\n", c, n, m, p, r4.e, ok ? "ok" : "MISMATCH");
    fails += !ok;
  }
  return fails ? 1 : 0;
}
