/*
 * mpsw_debug.h -- test and measurement hooks of libmpsw.
 *
 * Not part of the stepping interface of mpsw.h: these calls expose internal
 * pieces (the fused Laplacian operator, the factorisation kernels on one
 * matrix, the rank network's plan for each bond) so that tests can hold them
 * against an independent implementation, and count or time the kernels of a
 * step for measurement.  Conventions as in mpsw.h.
 */
#ifndef MPSW_DEBUG_H
#define MPSW_DEBUG_H

#include "mpsw.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Kernel classes of mpsw_profile / mpsw_profile_read. */
enum {
  MPSW_KC_QR = 0,      /* Householder QR factorisations (L->R sweep and SVD) */
  MPSW_KC_JACOBI = 1,  /* one-sided Jacobi sweeps of the SVD */
  MPSW_KC_GEMM = 2,    /* contractions */
  MPSW_KC_APPLYQ = 3,  /* Q_{k-1} applied to U Sigma */
  MPSW_KC_APPLYV = 4,  /* reflectors applied to the right singular vectors */
  MPSW_KC_COUNT = 5
};

/* Launch statistics of one kernel class since the last mpsw_profile call. */
typedef struct {
  int64_t launches;  /* launches timed with events (0 unless this class is the timed one) */
  double total_ms;   /* summed event time of those launches */
  double alg_flops;  /* algorithmic flops of every launch of the class, all shots:
                        QR 2mn^2 - 2n^3/3 (m x n, m >= n); Jacobi 9c^3 (c x c factor);
                        GEMM 2MNK; reflector application 4mnr - 2n^2 r */
} mpsw_kprof;

/* Reset the counters of every class and time each launch of class `kclass`
 * (-1: none) with a pair of events on the state's stream until the next call.
 * Synchronises.  Errors: EINVAL, EHIP. */
int mpsw_profile(mpsw_state st, int kclass);

/* Read the counters of class `kclass`.  Synchronises.  Errors: EINVAL, EHIP. */
int mpsw_profile_read(mpsw_state st, int kclass, mpsw_kprof* out);

/* Host-only helper (no device work), used by the CPU tests: the fused
 * Laplacian MPO S_x+ + S_x- + S_z+ + S_z- - 4I (eqs. 6 and 16) the library
 * applies, for n-bit registers, a boundary, a site order (MPSW_SEQUENTIAL or
 * MPSW_INTERLEAVED) and ndim = 2 or 3 registers (three: the six shifts and
 * -6I).  Writes K+1 bonds into
 * `bonds` and, if `cores` is not NULL, the cores packed site after site, core k
 * of shape [w_k][w_{k+1}][s_out][s_in] row-major (at most `cap` doubles).
 * Returns the total number of core entries (>= 0) or a negative error code. */
int mpsw_debug_laplacian_mpo(int n, int boundary, int ordering, int ndim, int* bonds, double* cores, int64_t cap);

/* Test helper (device work on the current device, default stream): runs the
 * factorisation kernels of a rounding on one host matrix A (m x n row-major).
 * op 0: QR (m even); out1 receives Q (m x q, row-major), out2 R (q x n), where
 *       q = n for a tall A and q = m (Q = I, R = A) otherwise.
 * op 1: SVD without truncation (n even); out1 receives V^T (r x n), out2
 *       U Sigma (m x r), r = min(m, n), columns ordered by decreasing sigma.
 * Buffers are caller-owned host memory of at least m*n and max(m,n)^2 doubles.
 * Returns q (op 0) or r (op 1), or a negative error code. */
int mpsw_debug_factor(int op, int m, int n, const double* A, double* out1, double* out2);

/* The rank network's output and proposed rank (ceil(out chi_max) clamped to
 * [1, chi_max]) for bonds 1..K-1 of rounding `rounding` of shot `shot`, as
 * the learned-rank rounding computes them at the coming step (K-1 floats and
 * ints, host memory).  Synchronises.  Errors: EINVAL, ESTATE (no velocity or
 * no network installed), EHIP. */
int mpsw_debug_rank_plan(mpsw_state st, int shot, int rounding, float* outs, int* rhat);

/* Entries (i, j), i < rows, j < cols, of the Gaussian test matrix the
 * learned-rank rounding draws for bond `site` of rounding `rounding` at step
 * `step` of a state seeded `seed` (the counter-based generator of the
 * randomized range finder), written row-major into host memory.
 * Errors: EINVAL, EHIP. */
int mpsw_debug_sketch_normals(uint64_t seed, int step, int rounding, int site, int rows, int cols, double* out);

/* The learned-rank rounding's sketch of one bond matrix, run by the same
 * launches a state runs for a bond: A (m x n row-major host, n even, up to
 * 4096 x 4096) is sketched at width l (1 <= l <= 32, l <= m, n) with the
 * Gaussian test matrix of key (seed, step, rounding, site), then the SVD
 * stage on B = A Q, the FP64 residual ||A - B Q^T||_F^2 and the acceptance
 * rule with (eps, chi).  Outputs: sig (32 doubles: the singular values of B,
 * descending, 0 beyond l), stats (3 doubles: residual, discarded sketched
 * sigma^2, largest sketched sigma), rank (the kept rank) and accepted (0/1).
 * Synchronises the device.  Errors: EINVAL, ENOMEM, EHIP. */
int mpsw_debug_sketch(const double* A, int m, int n, int l, double eps, int chi, uint64_t seed, int step, int rounding,
                      int site, double* sig, double* stats, int* rank, int* accepted);

#ifdef __cplusplus
}
#endif
#endif /* MPSW_DEBUG_H */
