/*
 * ranphy_ref.c — plain FP64 CPU oracle for the uplink receive hot path.
 *
 * TEST INFRASTRUCTURE ONLY: called by the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark; never by the product library.  Every step is the definition written
 * out in double precision; OpenMP only splits independent resource elements across threads.
 *
 * Readings taken where the paper is silent (it gives no DMRS layout, interpolation rule,
 * QAM mapping or LLR convention):
 *   - DMRS: comb C in frequency, optional length-2 time cover; port p sits on subcarriers
 *     k = (p mod C) + C j; the pilot value passed in already contains the cover code.
 *   - frequency interpolation: linear between a port's consecutive pilots, the nearest
 *     pilot held outside the first and last one;
 *   - time interpolation: linear in the symbol index between occasion centres
 *     s0 + (T-1)/2, held outside; a single occasion is held over the slot;
 *   - detector: linear MMSE with known noise variance per slot, unbiased per layer;
 *   - QAM: Gray square QAM in the 3GPP NR nested-sign structure, unit average energy;
 *   - LLR: max-log, positive when bit 0 is the more likely value.
 */
#include "ranphy_ref.h"

#include <complex.h>
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define REF_MAX_RX 64
#define REF_MAX_L 16

int ranphy_ref_version(void) { return 1; }

/* Threads an OpenMP loop of this library runs on (1 when built without OpenMP). */
int ranphy_ref_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads the following OpenMP loops of the calling thread use (n >= 1; no effect without
 * OpenMP).  Timing only: the results do not depend on the thread count. */
void ranphy_ref_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ------------------------------------------------------------------------------------- */
/* Descriptor helpers.                                                                    */
/* ------------------------------------------------------------------------------------- */

static int check_desc(const ranphy_ref_desc* d) {
  if (!d) return -1;
  if (d->n_prb < 1 || d->n_symb < 1 || d->n_symb > 14 || d->n_slots < 0) return -1;
  if (d->n_rx < 1 || d->n_rx > REF_MAX_RX) return -2;
  if (d->n_layers < 1 || d->n_layers > REF_MAX_L) return -2;
  if (d->qm != 2 && d->qm != 4 && d->qm != 6 && d->qm != 8) return -1;
  if (d->dmrs_comb < 1 || d->dmrs_td < 1 || d->dmrs_td > 2) return -1;
  if (d->n_occ < 1 || d->n_occ > 4) return -1;
  if (d->n_layers > d->dmrs_comb * d->dmrs_td) return -2;
  for (int o = 0; o < d->n_occ; ++o) {
    if (d->dmrs_sym0[o] < 0 || d->dmrs_sym0[o] + d->dmrs_td > d->n_symb) return -1;
    if (o > 0 && d->dmrs_sym0[o] < d->dmrs_sym0[o - 1] + d->dmrs_td) return -1;
  }
  return 0;
}

static int n_sc_of(const ranphy_ref_desc* d) { return 12 * d->n_prb; }

static int n_pilot_of(const ranphy_ref_desc* d) {
  return (n_sc_of(d) + d->dmrs_comb - 1) / d->dmrs_comb;
}

static int is_dmrs_symbol(const ranphy_ref_desc* d, int s) {
  for (int o = 0; o < d->n_occ; ++o)
    if (s >= d->dmrs_sym0[o] && s < d->dmrs_sym0[o] + d->dmrs_td) return 1;
  return 0;
}

/* Data symbols in ascending order; returns how many. */
static int data_symbols(const ranphy_ref_desc* d, int* out) {
  int n = 0;
  for (int s = 0; s < d->n_symb; ++s)
    if (!is_dmrs_symbol(d, s)) out[n++] = s;
  return n;
}

static cplx load_c64(const float* p, int64_t idx) {
  return (double)p[2 * idx] + I * (double)p[2 * idx + 1];
}

/* ------------------------------------------------------------------------------------- */
/* Least squares at the pilots, and frequency / time interpolation.                       */
/* ------------------------------------------------------------------------------------- */

/* LS estimate for port p, receive antenna r, occasion o at pilot index j:
 *   (1/T) sum_t y(s0 + t, k_j, r) conj(P(o, t, j, p)),  k_j = (p mod C) + C j.
 * Returns 0 when k_j falls beyond the last subcarrier. */
static cplx ls_at_pilot(const ranphy_ref_desc* d, const float* rx, const float* pilots, int slot,
                        int o, int j, int r, int p) {
  const int nsc = n_sc_of(d), C = d->dmrs_comb, T = d->dmrs_td, J = n_pilot_of(d);
  const int k = p % C + C * j;
  if (k >= nsc) return 0.0;
  cplx acc = 0.0;
  for (int t = 0; t < T; ++t) {
    const int s = d->dmrs_sym0[o] + t;
    const int64_t yi = (((int64_t)slot * d->n_symb + s) * nsc + k) * d->n_rx + r;
    const int64_t pi = ((((int64_t)slot * d->n_occ + o) * T + t) * J + j) * d->n_layers + p;
    acc += load_c64(rx, yi) * conj(load_c64(pilots, pi));
  }
  return acc / (double)T;
}

/* Number of pilots port p has within the n_sc subcarriers. */
static int port_pilots(const ranphy_ref_desc* d, int p) {
  const int c = p % d->dmrs_comb;
  return (n_sc_of(d) - c + d->dmrs_comb - 1) / d->dmrs_comb;
}

/* Frequency interpolation rule for port p at subcarrier k: the two pilot indices and the
 * weight a of the second one (value = (1 - a) v[j0] + a v[j1]). */
static void freq_rule(const ranphy_ref_desc* d, int p, int k, int* j0, int* j1, double* a) {
  const int C = d->dmrs_comb, c = p % C, Jp = port_pilots(d, p);
  const int first = c, last = c + C * (Jp - 1);
  if (k <= first) { *j0 = *j1 = 0; *a = 0.0; return; }
  if (k >= last) { *j0 = *j1 = Jp - 1; *a = 0.0; return; }
  const int j = (k - c) / C;
  *j0 = j;
  *j1 = j + 1;
  *a = (double)(k - c - C * j) / (double)C;
}

/* Time interpolation rule for symbol s: occasions o0, o1 and weight b of o1. */
static void time_rule(const ranphy_ref_desc* d, int s, int* o0, int* o1, double* b) {
  const int n = d->n_occ;
  double centre[4];
  for (int o = 0; o < n; ++o) centre[o] = d->dmrs_sym0[o] + 0.5 * (d->dmrs_td - 1);
  if (n == 1 || s <= centre[0]) { *o0 = *o1 = 0; *b = 0.0; return; }
  if (s >= centre[n - 1]) { *o0 = *o1 = n - 1; *b = 0.0; return; }
  for (int o = 0; o + 1 < n; ++o) {
    if (s >= centre[o] && s < centre[o + 1]) {
      *o0 = o;
      *o1 = o + 1;
      *b = (s - centre[o]) / (centre[o + 1] - centre[o]);
      return;
    }
  }
  *o0 = *o1 = n - 1;
  *b = 0.0;
}

int ranphy_ref_chest_ls(const ranphy_ref_desc* d, const float* rx, const float* pilots,
                        double* h, int h_res) {
  int rc = check_desc(d);
  if (rc) return rc;
  if (!rx || !pilots || !h) return -1;
  if (h_res != RANPHY_REF_H_PILOT && h_res != RANPHY_REF_H_FULL) return -1;
  const int nsc = n_sc_of(d), J = n_pilot_of(d), NR = d->n_rx, NL = d->n_layers;
  const int K = (h_res == RANPHY_REF_H_PILOT) ? J : nsc;
  const int64_t total = (int64_t)d->n_slots * d->n_occ * K;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < total; ++e) {
    const int slot = (int)(e / ((int64_t)d->n_occ * K));
    const int o = (int)((e / K) % d->n_occ);
    const int kk = (int)(e % K);
    for (int r = 0; r < NR; ++r) {
      for (int p = 0; p < NL; ++p) {
        cplx v;
        if (h_res == RANPHY_REF_H_PILOT) {
          v = ls_at_pilot(d, rx, pilots, slot, o, kk, r, p);
        } else {
          int j0, j1;
          double a;
          freq_rule(d, p, kk, &j0, &j1, &a);
          v = (1.0 - a) * ls_at_pilot(d, rx, pilots, slot, o, j0, r, p) +
              a * ls_at_pilot(d, rx, pilots, slot, o, j1, r, p);
        }
        const int64_t hi = ((e * NR) + r) * NL + p;
        h[2 * hi] = creal(v);
        h[2 * hi + 1] = cimag(v);
      }
    }
  }
  return 0;
}

/* Channel value at (slot, occasion, subcarrier, rx, port) from the caller's estimate. */
static cplx freq_value(const ranphy_ref_desc* d, const float* h, int h_res, int slot, int o,
                       int k, int r, int p) {
  const int NR = d->n_rx, NL = d->n_layers;
  if (h_res == RANPHY_REF_H_FULL) {
    const int64_t i = ((((int64_t)slot * d->n_occ + o) * n_sc_of(d) + k) * NR + r) * NL + p;
    return load_c64(h, i);
  }
  const int J = n_pilot_of(d);
  int j0, j1;
  double a;
  freq_rule(d, p, k, &j0, &j1, &a);
  const int64_t base = ((int64_t)slot * d->n_occ + o) * J;
  const cplx v0 = load_c64(h, ((base + j0) * NR + r) * NL + p);
  const cplx v1 = load_c64(h, ((base + j1) * NR + r) * NL + p);
  return (1.0 - a) * v0 + a * v1;
}

static void channel_matrix(const ranphy_ref_desc* d, const float* h, int h_res, int slot, int k,
                           int s, cplx* H) {
  int o0, o1;
  double b;
  time_rule(d, s, &o0, &o1, &b);
  for (int r = 0; r < d->n_rx; ++r)
    for (int p = 0; p < d->n_layers; ++p)
      H[r * d->n_layers + p] = (1.0 - b) * freq_value(d, h, h_res, slot, o0, k, r, p) +
                               b * freq_value(d, h, h_res, slot, o1, k, r, p);
}

int ranphy_ref_channel_at(const ranphy_ref_desc* d, const float* h, int h_res, int slot, int sc,
                          int symb, double* H) {
  int rc = check_desc(d);
  if (rc) return rc;
  if (!h || !H || slot < 0 || slot >= d->n_slots || sc < 0 || sc >= n_sc_of(d) || symb < 0 ||
      symb >= d->n_symb)
    return -1;
  cplx Hc[REF_MAX_RX * REF_MAX_L];
  channel_matrix(d, h, h_res, slot, sc, symb, Hc);
  for (int i = 0; i < d->n_rx * d->n_layers; ++i) {
    H[2 * i] = creal(Hc[i]);
    H[2 * i + 1] = cimag(Hc[i]);
  }
  return 0;
}

/* ------------------------------------------------------------------------------------- */
/* Dense complex LU with partial pivoting (Gaussian elimination written out).             */
/* ------------------------------------------------------------------------------------- */

/* Factor A (n x n, row-major) in place into P A = L U; returns 0, or 1 when a pivot is
 * zero relative to the matrix scale (numerically singular). */
static int lu_factor(int n, cplx* A, int* piv) {
  double scale = 0.0;
  for (int i = 0; i < n * n; ++i) scale = fmax(scale, cabs(A[i]));
  const double tiny = 64.0 * DBL_EPSILON * (scale > 0.0 ? scale : 1.0);
  for (int k = 0; k < n; ++k) {
    int best = k;
    for (int i = k + 1; i < n; ++i)
      if (cabs(A[i * n + k]) > cabs(A[best * n + k])) best = i;
    piv[k] = best;
    if (cabs(A[best * n + k]) <= tiny) return 1;
    if (best != k)
      for (int j = 0; j < n; ++j) {
        cplx t = A[k * n + j];
        A[k * n + j] = A[best * n + j];
        A[best * n + j] = t;
      }
    for (int i = k + 1; i < n; ++i) {
      const cplx m = A[i * n + k] / A[k * n + k];
      A[i * n + k] = m;
      for (int j = k + 1; j < n; ++j) A[i * n + j] -= m * A[k * n + j];
    }
  }
  return 0;
}

/* Solve A x = b with the factors: row swaps, forward substitution with unit L, backward
 * substitution with U.  b is overwritten by x. */
static void lu_solve(int n, const cplx* LU, const int* piv, cplx* b) {
  for (int k = 0; k < n; ++k)
    if (piv[k] != k) {
      cplx t = b[k];
      b[k] = b[piv[k]];
      b[piv[k]] = t;
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) b[i] -= LU[i * n + j] * b[j];
  for (int i = n - 1; i >= 0; --i) {
    for (int j = i + 1; j < n; ++j) b[i] -= LU[i * n + j] * b[j];
    b[i] /= LU[i * n + i];
  }
}

/* ------------------------------------------------------------------------------------- */
/* MMSE per resource element.                                                             */
/* ------------------------------------------------------------------------------------- */

int ranphy_ref_gram(int nr, int nl, const double* H, double s2, double* G) {
  if (nr < 1 || nl < 1 || !H || !G) return -1;
  for (int i = 0; i < nl; ++i)
    for (int j = 0; j < nl; ++j) {
      cplx acc = (i == j) ? s2 : 0.0;
      for (int r = 0; r < nr; ++r) {
        const cplx hi = H[2 * (r * nl + i)] + I * H[2 * (r * nl + i) + 1];
        const cplx hj = H[2 * (r * nl + j)] + I * H[2 * (r * nl + j) + 1];
        acc += conj(hi) * hj;
      }
      G[2 * (i * nl + j)] = creal(acc);
      G[2 * (i * nl + j) + 1] = cimag(acc);
    }
  return 0;
}

/* One resource element.  x_hat = (H^H H + s2 I)^-1 H^H y  (route LU) or
 * x_hat = H^H (H H^H + s2 I)^-1 y (route RCOV); mu = diag(W H); x~ = x_hat / mu;
 * nu2 = (1 - mu) / mu.  A singular system gives NaN x~ and mu, +inf nu2. */
static void mmse_one(int nr, int nl, const cplx* H, const cplx* y, double s2, int route,
                     cplx* xt, double* nv, double* mu) {
  cplx xhat[REF_MAX_L];
  double m[REF_MAX_L];
  int ok = 1;
  if (route == RANPHY_REF_ROUTE_LU) {
    cplx G[REF_MAX_L * REF_MAX_L];
    int piv[REF_MAX_L];
    for (int i = 0; i < nl; ++i) {
      for (int j = 0; j < nl; ++j) {
        cplx acc = (i == j) ? s2 : 0.0;
        for (int r = 0; r < nr; ++r) acc += conj(H[r * nl + i]) * H[r * nl + j];
        G[i * nl + j] = acc;
      }
      cplx z = 0.0;
      for (int r = 0; r < nr; ++r) z += conj(H[r * nl + i]) * y[r];
      xhat[i] = z;
    }
    if (lu_factor(nl, G, piv)) {
      ok = 0;
    } else {
      lu_solve(nl, G, piv, xhat);
      for (int l = 0; l < nl; ++l) {
        cplx e[REF_MAX_L];
        for (int i = 0; i < nl; ++i) e[i] = (i == l) ? 1.0 : 0.0;
        lu_solve(nl, G, piv, e); /* column l of G^-1 */
        m[l] = 1.0 - s2 * creal(e[l]);
      }
    }
  } else {
    cplx* R = (cplx*)malloc(sizeof(cplx) * nr * nr);
    cplx* v = (cplx*)malloc(sizeof(cplx) * nr);
    int* piv = (int*)malloc(sizeof(int) * nr);
    for (int a = 0; a < nr; ++a)
      for (int b = 0; b < nr; ++b) {
        cplx acc = (a == b) ? s2 : 0.0;
        for (int l = 0; l < nl; ++l) acc += H[a * nl + l] * conj(H[b * nl + l]);
        R[a * nr + b] = acc;
      }
    if (lu_factor(nr, R, piv)) {
      ok = 0;
    } else {
      for (int a = 0; a < nr; ++a) v[a] = y[a];
      lu_solve(nr, R, piv, v);
      for (int l = 0; l < nl; ++l) {
        cplx acc = 0.0;
        for (int a = 0; a < nr; ++a) acc += conj(H[a * nl + l]) * v[a];
        xhat[l] = acc;
        cplx* u = (cplx*)malloc(sizeof(cplx) * nr);
        for (int a = 0; a < nr; ++a) u[a] = H[a * nl + l];
        lu_solve(nr, R, piv, u);
        cplx q = 0.0;
        for (int a = 0; a < nr; ++a) q += conj(H[a * nl + l]) * u[a];
        m[l] = creal(q);
        free(u);
      }
    }
    free(R);
    free(v);
    free(piv);
  }
  for (int l = 0; l < nl; ++l) {
    if (!ok) {
      xt[l] = NAN + I * NAN;
      nv[l] = INFINITY;
      mu[l] = NAN;
    } else {
      mu[l] = m[l];
      xt[l] = xhat[l] / m[l];
      nv[l] = (1.0 - m[l]) / m[l];
    }
  }
}

int ranphy_ref_mmse_batch(int64_t n, int nr, int nl, const double* H, const double* y,
                          const double* s2, int route, double* x_tilde, double* nv,
                          double* mu) {
  if (n < 0 || nr < 1 || nr > REF_MAX_RX || nl < 1 || nl > REF_MAX_L) return -2;
  if (!H || !y || !s2 || !x_tilde || !nv || !mu) return -1;
  if (route != RANPHY_REF_ROUTE_LU && route != RANPHY_REF_ROUTE_RCOV) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < n; ++e) {
    cplx Hc[REF_MAX_RX * REF_MAX_L], yc[REF_MAX_RX], xt[REF_MAX_L];
    const double* He = H + 2 * e * nr * nl;
    const double* ye = y + 2 * e * nr;
    for (int i = 0; i < nr * nl; ++i) Hc[i] = He[2 * i] + I * He[2 * i + 1];
    for (int r = 0; r < nr; ++r) yc[r] = ye[2 * r] + I * ye[2 * r + 1];
    mmse_one(nr, nl, Hc, yc, s2[e], route, xt, nv + e * nl, mu + e * nl);
    for (int l = 0; l < nl; ++l) {
      x_tilde[2 * (e * nl + l)] = creal(xt[l]);
      x_tilde[2 * (e * nl + l) + 1] = cimag(xt[l]);
    }
  }
  return 0;
}

int ranphy_ref_mmse_detect(const ranphy_ref_desc* d, const float* rx, const float* h,
                           int h_res, const float* noise_var, double* x, double* nv,
                           int route) {
  int rc = check_desc(d);
  if (rc) return rc;
  if (!rx || !h || !noise_var || !x || !nv) return -1;
  if (h_res != RANPHY_REF_H_PILOT && h_res != RANPHY_REF_H_FULL) return -1;
  if (route != RANPHY_REF_ROUTE_LU && route != RANPHY_REF_ROUTE_RCOV) return -1;
  int dsym[14];
  const int nd = data_symbols(d, dsym);
  const int nsc = n_sc_of(d), NR = d->n_rx, NL = d->n_layers;
  const int64_t total = (int64_t)d->n_slots * nd * nsc;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t e = 0; e < total; ++e) {
    const int slot = (int)(e / ((int64_t)nd * nsc));
    const int di = (int)((e / nsc) % nd);
    const int k = (int)(e % nsc);
    const int s = dsym[di];
    cplx H[REF_MAX_RX * REF_MAX_L], y[REF_MAX_RX], xt[REF_MAX_L];
    double mu[REF_MAX_L];
    channel_matrix(d, h, h_res, slot, k, s, H);
    for (int r = 0; r < NR; ++r)
      y[r] = load_c64(rx, (((int64_t)slot * d->n_symb + s) * nsc + k) * NR + r);
    mmse_one(NR, NL, H, y, (double)noise_var[slot], route, xt, nv + e * NL, mu);
    for (int l = 0; l < NL; ++l) {
      x[2 * (e * NL + l)] = creal(xt[l]);
      x[2 * (e * NL + l) + 1] = cimag(xt[l]);
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------------------- */
/* Constellation and brute-force max-log demapping.                                       */
/* ------------------------------------------------------------------------------------- */

/* Gray PAM level of one axis from its bits c[0..m-1] (most significant first):
 * f(i) = (1 - 2 c_i) (2^(m-1-i) - f(i+1)),  f(m) = 0;  the level is f(0). */
static double pam_level(const int* c, int m) {
  double f = 0.0;
  for (int i = m - 1; i >= 0; --i) f = (1.0 - 2.0 * c[i]) * ((double)(1 << (m - 1 - i)) - f);
  return f;
}

int ranphy_ref_qam_points(int qm, double* pts) {
  if ((qm != 2 && qm != 4 && qm != 6 && qm != 8) || !pts) return -1;
  const int M = 1 << qm, m = qm / 2;
  const double norm = sqrt(2.0 * (M - 1) / 3.0);
  for (int i = 0; i < M; ++i) {
    int ci[4], cq[4];
    for (int b = 0; b < qm; ++b) {
      const int bit = (i >> (qm - 1 - b)) & 1; /* bit b of point i, b0 = MSB of i */
      if (b % 2 == 0) ci[b / 2] = bit; else cq[b / 2] = bit;
    }
    pts[2 * i] = pam_level(ci, m) / norm;
    pts[2 * i + 1] = pam_level(cq, m) / norm;
  }
  return 0;
}

static void llr_one(int qm, const double* pts, cplx x, double nv, double* llr) {
  const int M = 1 << qm;
  for (int b = 0; b < qm; ++b) {
    double d0 = INFINITY, d1 = INFINITY;
    for (int i = 0; i < M; ++i) {
      const double dr = creal(x) - pts[2 * i], di = cimag(x) - pts[2 * i + 1];
      const double dist = dr * dr + di * di;
      if ((i >> (qm - 1 - b)) & 1) d1 = fmin(d1, dist); else d0 = fmin(d0, dist);
    }
    llr[b] = (d1 - d0) / nv;
  }
}

int ranphy_ref_llr_batch(int64_t n, int qm, const double* x, const double* nv, double* llr) {
  double pts[2 * 256];
  if (ranphy_ref_qam_points(qm, pts)) return -1;
  if (n < 0 || !x || !nv || !llr) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < n; ++e)
    llr_one(qm, pts, x[2 * e] + I * x[2 * e + 1], nv[e], llr + e * qm);
  return 0;
}

int ranphy_ref_llr_demap(const ranphy_ref_desc* d, const float* x, const float* nv,
                         double* llr) {
  int rc = check_desc(d);
  if (rc) return rc;
  if (!x || !nv || !llr) return -1;
  double pts[2 * 256];
  ranphy_ref_qam_points(d->qm, pts);
  int dsym[14];
  const int nd = data_symbols(d, dsym);
  const int64_t n = (int64_t)d->n_slots * nd * n_sc_of(d) * d->n_layers;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < n; ++e)
    llr_one(d->qm, pts, load_c64(x, e), (double)nv[e], llr + e * d->qm);
  return 0;
}
