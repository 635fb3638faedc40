/*
 * Plain FP64 CPU statevector oracle for p-layer MaxCut QAOA.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code with the HIP library.
 *
 * What it computes (the plain definitions, written out without blocking,
 * fusion or reordering):
 *   - cut value C(z) = sum over edges (u,v) of w_uv [z_u != z_v]      (the eq. for H_P; w_uv = 1 unless
 *                                                                         integer weights are given)
 *   - ansatz |psi> = prod_{l=1..p} e^{-i beta_l H_M} e^{-i gamma_l H_C} |+>^n,
 *     layer 1 applied first, cost before mixer                          (QAOA section, eq. for |psi>_p;
 *                                                                         explicit order in eq. A2)
 *   - mixer e^{-i beta X_q} on every qubit q: (a,b) -> (cos b a - i sin b b, -i sin b a + cos b b)
 *   - expectation of an observable sum_t (w_t/2)(1 - Z_{i_t} Z_{j_t})  (F_p; H_red in
 *     "Reducing the Hamiltonian"; aggregation eq. in "The classical estimator cost")
 *   - gradient by the adjoint rule dE/dtheta = 2 Im <lambda|G|psi> for a gate e^{-i theta G}
 *     (lambda = the observable back-propagated to the gate), with G = H_C for gamma_l and
 *     G = sum_q X_q for beta_l.
 *
 * Conventions: vertex v = qubit v = bit v of the basis index z.  Complex numbers
 * are stored interleaved (re, im) in double arrays.  OpenMP parallelises the loops
 * over z; nothing else changes the arithmetic.
 */
#include <complex.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* cut value of z: sum over edges of w_e [bit u != bit v] (w_e = 1 when wts is NULL) */
static int cut_of(uint64_t z, int m, const int32_t *edges, const int32_t *wts) {
  int c = 0;
  for (int e = 0; e < m; ++e) {
    uint64_t bu = (z >> edges[2 * e]) & 1u, bv = (z >> edges[2 * e + 1]) & 1u;
    if (bu != bv) c += wts ? wts[e] : 1;
  }
  return c;
}

/* weighted term value h(z) = sum_t w_t [bit i_t != bit j_t] */
static double term_value(uint64_t z, int T, const int32_t *ti, const int32_t *tj, const double *tw) {
  double h = 0.0;
  for (int t = 0; t < T; ++t) {
    uint64_t a = (z >> ti[t]) & 1u, b = (z >> tj[t]) & 1u;
    if (a != b) h += tw[t];
  }
  return h;
}

int orc_cut_values(int n, int m, const int32_t *edges, const int32_t *wts, int32_t *out) {
  if (n < 1 || n > 30) return -1;
  uint64_t N = (uint64_t)1 << n;
#pragma omp parallel for schedule(static)
  for (int64_t z = 0; z < (int64_t)N; ++z) out[z] = cut_of((uint64_t)z, m, edges, wts);
  return 0;
}

int orc_term_values(int n, int T, const int32_t *ti, const int32_t *tj, const double *tw, double *out) {
  if (n < 1 || n > 30) return -1;
  uint64_t N = (uint64_t)1 << n;
#pragma omp parallel for schedule(static)
  for (int64_t z = 0; z < (int64_t)N; ++z) out[z] = term_value((uint64_t)z, T, ti, tj, tw);
  return 0;
}

/* psi(z) <- exp(-i gamma C(z)) psi(z); sign = +1 applies the gate, -1 its inverse */
static void apply_phase(cplx *psi, int n, int m, const int32_t *edges, const int32_t *wts, double gamma,
                        double sign) {
  uint64_t N = (uint64_t)1 << n;
#pragma omp parallel for schedule(static)
  for (int64_t z = 0; z < (int64_t)N; ++z) {
    double ang = -sign * gamma * (double)cut_of((uint64_t)z, m, edges, wts);
    psi[z] *= cos(ang) + I * sin(ang);
  }
}

/* e^{-i beta X_q} on qubit q (sign = -1: its inverse e^{+i beta X_q}) */
static void apply_rx(cplx *psi, int n, int q, double beta, double sign) {
  uint64_t N = (uint64_t)1 << n, bit = (uint64_t)1 << q;
  double c = cos(beta), s = sign * sin(beta);
#pragma omp parallel for schedule(static)
  for (int64_t z = 0; z < (int64_t)N; ++z) {
    if ((uint64_t)z & bit) continue;
    cplx a = psi[z], b = psi[(uint64_t)z | bit];
    psi[z] = c * a - I * s * b;
    psi[(uint64_t)z | bit] = -I * s * a + c * b;
  }
}

int orc_state(int n, int m, const int32_t *edges, const int32_t *wts, int p, const double *gamma, const double *beta,
              double *psi_out) {
  if (n < 1 || n > 30 || p < 0) return -1;
  uint64_t N = (uint64_t)1 << n;
  cplx *psi = (cplx *)psi_out;
  double amp = pow(2.0, -0.5 * n);
  for (uint64_t z = 0; z < N; ++z) psi[z] = amp;
  for (int l = 0; l < p; ++l) {
    apply_phase(psi, n, m, edges, wts, gamma[l], 1.0);
    for (int q = 0; q < n; ++q) apply_rx(psi, n, q, beta[l], 1.0);
  }
  return 0;
}

/* <Z_i Z_j> for each term; |psi|^2-weighted sum of (-1)^{z_i xor z_j} */
int orc_zz(int n, const double *psi_in, int T, const int32_t *ti, const int32_t *tj, double *zz_out) {
  const cplx *psi = (const cplx *)psi_in;
  uint64_t N = (uint64_t)1 << n;
  for (int t = 0; t < T; ++t) {
    double acc = 0.0;
#pragma omp parallel for reduction(+ : acc) schedule(static)
    for (int64_t z = 0; z < (int64_t)N; ++z) {
      double pr = creal(psi[z]) * creal(psi[z]) + cimag(psi[z]) * cimag(psi[z]);
      int odd = (int)((((uint64_t)z >> ti[t]) ^ ((uint64_t)z >> tj[t])) & 1u);
      acc += odd ? -pr : pr;
    }
    zz_out[t] = acc;
  }
  return 0;
}

/* energy = sum_t (w_t/2)(1 - <Z Z>_t); also the independent route sum_z |psi|^2 h(z) */
int orc_energy(int n, int m, const int32_t *edges, const int32_t *wts, int T, const int32_t *ti, const int32_t *tj,
               const double *tw, int p, const double *gamma, const double *beta, double *energy_terms, double *energy_direct,
               double *zz_out, double *norm_out) {
  if (n < 1 || n > 30) return -1;
  uint64_t N = (uint64_t)1 << n;
  double *buf = (double *)malloc(sizeof(double) * 2 * N);
  if (!buf) return -2;
  orc_state(n, m, edges, wts, p, gamma, beta, buf);
  double *zz = (double *)malloc(sizeof(double) * (T > 0 ? T : 1));
  orc_zz(n, buf, T, ti, tj, zz);
  double e = 0.0;
  for (int t = 0; t < T; ++t) e += 0.5 * tw[t] * (1.0 - zz[t]);
  const cplx *psi = (const cplx *)buf;
  double ed = 0.0, nrm = 0.0;
#pragma omp parallel for reduction(+ : ed, nrm) schedule(static)
  for (int64_t z = 0; z < (int64_t)N; ++z) {
    double pr = creal(psi[z]) * creal(psi[z]) + cimag(psi[z]) * cimag(psi[z]);
    ed += pr * term_value((uint64_t)z, T, ti, tj, tw);
    nrm += pr;
  }
  if (energy_terms) *energy_terms = e;
  if (energy_direct) *energy_direct = ed;
  if (norm_out) *norm_out = nrm;
  if (zz_out) memcpy(zz_out, zz, sizeof(double) * T);
  free(zz);
  free(buf);
  return 0;
}

/* Im sum_z conj(lam(z)) psi(z xor 2^q)  (the <lambda|X_q|psi> part of the beta gradient) */
static double im_lam_x_psi(const cplx *lam, const cplx *psi, int n, int q) {
  uint64_t N = (uint64_t)1 << n, bit = (uint64_t)1 << q;
  double acc = 0.0;
#pragma omp parallel for reduction(+ : acc) schedule(static)
  for (int64_t z = 0; z < (int64_t)N; ++z) acc += cimag(conj(lam[z]) * psi[(uint64_t)z ^ bit]);
  return acc;
}

/* Im sum_z conj(lam(z)) C(z) psi(z)  (the <lambda|H_C|psi> part of the gamma gradient) */
static double im_lam_c_psi(const cplx *lam, const cplx *psi, int n, int m, const int32_t *edges, const int32_t *wts) {
  uint64_t N = (uint64_t)1 << n;
  double acc = 0.0;
#pragma omp parallel for reduction(+ : acc) schedule(static)
  for (int64_t z = 0; z < (int64_t)N; ++z)
    acc += (double)cut_of((uint64_t)z, m, edges, wts) * cimag(conj(lam[z]) * psi[z]);
  return acc;
}

/*
 * Energy and gradient by the adjoint method.  Forward: build psi.  Set
 * lam = h * psi (h = the observable's diagonal).  Then walk the gates backwards:
 * for each gate e^{-i theta G}, record 2 Im <lam|G|psi> into dE/dtheta, then undo
 * the gate on both psi and lam.  The mixer's generator sum_q X_q is accumulated
 * qubit by qubit as the single-qubit gates are undone.
 */
int orc_energy_grad(int n, int m, const int32_t *edges, const int32_t *wts, int T, const int32_t *ti,
                    const int32_t *tj, const double *tw, int p, const double *gamma, const double *beta, double *energy,
                    double *dgamma, double *dbeta, double *final_dev) {
  if (n < 1 || n > 30 || p < 1) return -1;
  uint64_t N = (uint64_t)1 << n;
  cplx *psi = (cplx *)malloc(sizeof(cplx) * N);
  cplx *lam = (cplx *)malloc(sizeof(cplx) * N);
  if (!psi || !lam) {
    free(psi);
    free(lam);
    return -2;
  }
  orc_state(n, m, edges, wts, p, gamma, beta, (double *)psi);
  double e = 0.0;
#pragma omp parallel for reduction(+ : e) schedule(static)
  for (int64_t z = 0; z < (int64_t)N; ++z) {
    double h = term_value((uint64_t)z, T, ti, tj, tw);
    double pr = creal(psi[z]) * creal(psi[z]) + cimag(psi[z]) * cimag(psi[z]);
    e += pr * h;
    lam[z] = h * psi[z];
  }
  *energy = e;
  for (int l = p - 1; l >= 0; --l) {
    double gb = 0.0;
    for (int q = n - 1; q >= 0; --q) {
      gb += 2.0 * im_lam_x_psi(lam, psi, n, q);
      apply_rx(psi, n, q, beta[l], -1.0);
      apply_rx(lam, n, q, beta[l], -1.0);
    }
    dbeta[l] = gb;
    dgamma[l] = 2.0 * im_lam_c_psi(lam, psi, n, m, edges, wts);
    apply_phase(psi, n, m, edges, wts, gamma[l], -1.0);
    apply_phase(lam, n, m, edges, wts, gamma[l], -1.0);
  }
  if (final_dev) {
    /* after undoing every gate psi must be |+>^n again */
    double amp = pow(2.0, -0.5 * n), dev = 0.0;
    for (uint64_t z = 0; z < N; ++z) {
      double d = cabs(psi[z] - amp);
      if (d > dev) dev = d;
    }
    *final_dev = dev;
  }
  free(psi);
  free(lam);
  return 0;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* thread count of the following parallel loops (timing at a fixed count) */
void orc_set_num_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}
