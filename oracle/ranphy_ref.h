/*
 * ranphy_ref — plain FP64 CPU oracle for the uplink receive hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or loads this
 * code; only the test suite, the smoke check and the CPU-baseline leg of the benchmark do.
 * It shares no source, header, table or helper with the GPU library.
 *
 * What it computes (all in double precision, loops written out, no blocking or fusion):
 *
 *   ranphy_ref_chest_ls     least-squares channel estimate at the DMRS pilot subcarriers
 *                           with time-cover despreading, optionally interpolated in
 *                           frequency to every subcarrier.  Channel estimation is named by
 *                           the paper (abstract; Sec. III-B) as a block suited to data-level
 *                           parallelism; the LS formula is the standard one.
 *   ranphy_ref_mmse_detect  per data resource element: channel by frequency then time
 *                           interpolation, x_hat = (H^H H + s2 I)^-1 H^H y solved by LU
 *                           decomposition with partial pivoting and forward/backward
 *                           substitution (the factorisation of Sec. IV / Fig. 4), or by the
 *                           received-covariance form x_hat = H^H (H H^H + s2 I)^-1 y (the
 *                           "R" of Sec. IV).  Unbiasing mu = diag(W H), x~ = x_hat / mu,
 *                           post-equalisation noise nu2 = (1 - mu) / mu.
 *   ranphy_ref_llr_demap    max-log LLR by brute force over all 2^Qm constellation points,
 *                           LLR = (min_{b=1} |x-s|^2 - min_{b=0} |x-s|^2) / nu2.
 *
 * Parity pins: every function here is pinned by CPU tests against closed forms, special
 * cases and brute force (see the test suite's oracle pin module).
 *
 * Layouts (row-major, slot outermost; complex = interleaved (re, im)):
 *   rx      [slot][symb][sc][rx]             complex64 (float pairs)
 *   pilots  [slot][occ][t][j][layer]         complex64, j < ceil(n_sc / comb)
 *   h PILOT [slot][occ][j][rx][layer]        (complex128 out of chest_ls, complex64 into
 *   h FULL  [slot][occ][sc][rx][layer]        mmse_detect: the GPU path's input bytes)
 *   x, nv   [slot][dsym][sc][layer]          complex128 / double out; complex64 / float in
 *   llr     [slot][dsym][sc][layer][qm]      double, LLR > 0 means bit 0 more likely
 *
 * Return value: 0 on success, -1 invalid argument, -2 unsupported shape.
 */
#ifndef RANPHY_REF_H
#define RANPHY_REF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n_prb;        /* resource blocks; 12 subcarriers each                */
  int32_t n_symb;       /* OFDM symbols per slot                               */
  int32_t n_rx;         /* receive antennas                                    */
  int32_t n_layers;     /* spatial layers (= DMRS ports 0..n_layers-1)         */
  int32_t qm;           /* bits per QAM symbol: 2, 4, 6, 8                      */
  int32_t dmrs_comb;    /* frequency comb C: port p on subcarriers p mod C + C j */
  int32_t dmrs_td;      /* DMRS symbols per occasion T (1 or 2, cover code)    */
  int32_t n_occ;        /* DMRS occasions                                      */
  int32_t dmrs_sym0[4]; /* first symbol of each occasion, ascending            */
  int32_t n_slots;      /* slots in the batch                                  */
} ranphy_ref_desc;

enum { RANPHY_REF_H_PILOT = 0, RANPHY_REF_H_FULL = 1 };
enum { RANPHY_REF_ROUTE_LU = 0, RANPHY_REF_ROUTE_RCOV = 1 };

int ranphy_ref_version(void);
int ranphy_ref_threads(void);
void ranphy_ref_set_threads(int n); /* timing only: later OpenMP loops of this thread */

/* Slot-level calls (host pointers). */
int ranphy_ref_chest_ls(const ranphy_ref_desc* d, const float* rx, const float* pilots,
                        double* h, int h_res);
int ranphy_ref_mmse_detect(const ranphy_ref_desc* d, const float* rx, const float* h,
                           int h_res, const float* noise_var, double* x, double* nv,
                           int route);
int ranphy_ref_llr_demap(const ranphy_ref_desc* d, const float* x, const float* nv,
                         double* llr);

/* Channel matrix H[rx][layer] (complex128) that the detector uses at (slot, sc, symb). */
int ranphy_ref_channel_at(const ranphy_ref_desc* d, const float* h, int h_res, int slot,
                          int sc, int symb, double* H);

/* Per-element primitives in double precision. */
int ranphy_ref_gram(int nr, int nl, const double* H, double s2, double* G);
int ranphy_ref_mmse_batch(int64_t n, int nr, int nl, const double* H, const double* y,
                          const double* s2, int route, double* x_tilde, double* nv,
                          double* mu);
int ranphy_ref_llr_batch(int64_t n, int qm, const double* x, const double* nv,
                         double* llr);
int ranphy_ref_qam_points(int qm, double* pts);

#ifdef __cplusplus
}
#endif
#endif
