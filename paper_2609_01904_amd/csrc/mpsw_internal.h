// Internal structures shared by the kernels and the runtime of libmpsw.
//
// Memory model: a state ("group") holds B shots with the same number of sites
// K = 2n.  Every shot owns an arena of doubles with identical layout (all
// offsets below are relative to the shot's arena base, in doubles), and a
// block of ints holding its data-dependent dimensions (bonds, sweep ranks).
// Kernels read dimensions from device memory, so the launch sequence of a step
// is fixed and never waits for the host; each kernel is launched with a grid
// sized for the workspace capacities and blocks beyond the live sizes exit.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mpsw_debug.h"

#define MPSW_MAXK 24          // K = ndim n <= 22 is what the LDS allows
#define MPSW_NSLOT 5          // MPS buffers: 0..2 psi rotation, 3 = y, 4 = w
#define MPSW_SLOT_Y 3
#define MPSW_SLOT_W 4

// error bits raised on the device, reported by the host at the next sync
#define MPSW_DEV_ERR_CAP 1        // a live size exceeded a workspace capacity
#define MPSW_DEV_ERR_NONFINITE 2  // a singular value was not finite
#define MPSW_DEV_ERR_GRID 4       // a launch grid was smaller than the live work
#define MPSW_DEV_ERR_TIMEOUT 8    // a bounded inter-workgroup wait gave up

// Truncation-rank network: 34 inputs, two hidden layers of 128, one output.
#define MLP_NIN 34
#define MLP_NH 128
#define MLP_NPARAM (MLP_NIN * MLP_NH + MLP_NH + MLP_NH * MLP_NH + MLP_NH + MLP_NH + 1)
#define MPSW_RRF_MAXL 512         // widest randomized range finder sketch
#define MPSW_RRF_OVER 8           // oversampling of the sketch width

// Kernel classes for the algorithmic-flop counters and event timing are the
// MPSW_KC_* values of the public header.

// Per-shot synchronisation area (ints) used by the multi-workgroup kernels.
#define MPSW_SYNC_STRIDE 1024
#define MPSW_SYNC_BARRIER 0       // barrier arrival counter
#define MPSW_SYNC_ROT 8           // [64] rotations seen per Jacobi sweep
#define MPSW_SYNC_MAXREL 128      // [64] largest squared pair cosine per Jacobi sweep (float bits)
#define MPSW_SYNC_FLAGS 192       // [<= 832] panel-ready flags of the QR factorisation
#define MPSW_MAX_SWEEPS 60

// Per-shot integer block layout (offsets in ints).
struct ShotDimsLayout {
  static constexpr int bonds = 0;                                  // [NSLOT][MAXK+1]
  static constexpr int rin = bonds + MPSW_NSLOT * (MPSW_MAXK + 1); // input bonds of the rounding
  static constexpr int rt = rin + (MPSW_MAXK + 1);                 // left bonds after the QR sweep
  static constexpr int rho = rt + (MPSW_MAXK + 1);                 // bonds after the SVD sweep
  static constexpr int qid = rho + (MPSW_MAXK + 1);                // 1 if Q_k is the identity
  static constexpr int chi = qid + (MPSW_MAXK + 1);
  static constexpr int src_ix = chi + 1;
  static constexpr int src_iz = src_ix + 1;
  static constexpr int src_nt = src_iz + 1;
  static constexpr int maxbond = src_nt + 1;                       // [3] per rounding of the last step
  static constexpr int jac_sweeps = maxbond + 3;                   // most Jacobi sweeps since the last reset
  static constexpr int step = jac_sweeps + 1;                      // steps taken since the fields were set
  // learned-rank rounding (randomized range finder) of the current bond
  static constexpr int svd_n = step + 1;      // columns of the bond matrix the SVD stage sees (0: 2 rho_{k+1})
  static constexpr int rrf = svd_n + 1;       // 0: exact SVD, 1: sketch in progress, 2: sketch accepted
  static constexpr int rrf_l = rrf + 1;       // sketch width l = predicted rank + oversampling
  static constexpr int rrf_tries = rrf_l + 1; // bonds sketched since the fields were set
  static constexpr int fallbacks = rrf_tries + 1;  // sketches rejected (exact SVD taken)
  // per rounding and bond: after a rejected sketch the bond takes the exact
  // SVD until step rrf_skip, and the wait rrf_back doubles (1, 2, ..., 64)
  // with every further rejection; an accepted sketch resets it
  static constexpr int rrf_skip = fallbacks + 1;            // [3][MAXK]
  static constexpr int rrf_back = rrf_skip + 3 * MPSW_MAXK; // [3][MAXK]
  static constexpr int src_iy = rrf_back + 3 * MPSW_MAXK;   // source y (three-dimensional states)
  static constexpr int prank = src_iy + 1;                  // [3][MAXK] rank kept per rounding and bond, last step
  static constexpr int size = prank + 3 * MPSW_MAXK;
};

// Per-shot double block layout (offsets in doubles, separate small array).
struct ShotRealLayout {
  static constexpr int eps = 0;
  static constexpr int tail2 = 1;     // [3]
  static constexpr int sigma_log = 4; // [3][MAXK][32]: leading singular values of the last step
  static constexpr int alg_flops = sigma_log + 3 * MPSW_MAXK * 32;  // [MPSW_KC_COUNT] per kernel class
  static constexpr int rrf_res2 = alg_flops + 8; // ||M - B Q^T||_F^2: what the sketch of the bond matrix misses
  static constexpr int rrf_tail = rrf_res2 + 1;  // sum of the discarded sketched sigma^2
  static constexpr int rrf_sig1 = rrf_tail + 1;  // largest sketched sigma
  static constexpr int rrf_sum2 = rrf_sig1 + 1;  // sum of all sketched sigma^2 (= ||M Q||_F^2)
  static constexpr int size = rrf_sum2 + 1;
};

// Capacities (doubles) and offsets of one engine's buffers inside a shot arena.
struct EngineLayout {
  int64_t off_in[MPSW_MAXK], cap_in[MPSW_MAXK];   // explicit source cores
  int64_t off_q[MPSW_MAXK], cap_q[MPSW_MAXK];     // Householder vectors + R of the QR sweep
  int64_t off_qt[MPSW_MAXK], cap_qt[MPSW_MAXK];   // compact-WY T factors per panel
  int64_t off_X, cap_X;     // X_k = R_{k-1} S_k
  int64_t off_X2, cap_X2;   // X after the meeting product (c^2 rounding)
  int64_t off_R, cap_R;     // R factor carried to the right
  int64_t off_VL0, off_VL1, cap_VL;  // left halves of y, contracted site by site (ping-pong, 2^k x chi_k)
  int64_t off_WR0, off_WR1, cap_WR;  // right halves of y (ping-pong, chi_k x 2^(K-k))
  int64_t off_M, cap_M;     // bond matrix of the SVD sweep
  int64_t off_US, cap_US;   // U_r Sigma_r
  int64_t off_sA, cap_sA;   // Jacobi working matrix
  int64_t off_sA2, cap_sA2; // R1^T of a wide bond matrix
  int64_t off_qrS2, cap_qrS2, off_qrT2, cap_qrT2;  // second QR of a wide bond matrix
  int64_t off_Vp, cap_Vp;   // V'^T of a wide bond matrix
  int64_t off_Yv, cap_Yv;   // V = Q1 [V'; 0] work
  int64_t off_perm, cap_perm; // column order of the last SVD QR (stored as doubles)
  int64_t off_sJ, cap_sJ;   // Jacobi accumulated rotations
  int64_t off_qrS, cap_qrS; // Householder working matrix
  // randomized range finder (learned-rank rounding)
  int64_t off_Om, cap_Om;   // Gaussian test matrix Omega (rt x l)
  int64_t off_Ys, cap_Ys;   // row-space sketch / its orthonormal basis Q (2 rho x l)
  int64_t off_Zs, cap_Zs;   // column-space iterate, then B = M Q (rt x l)
  int64_t off_Mb, cap_Mb;   // copy of the bond matrix while its sketch is judged
  int64_t off_G, cap_G;     // l x l Gram matrix / Cholesky factor
  int64_t off_Tc, cap_Tc;   // core = W_r^T Q^T before it replaces the slot
  int64_t off_Rz, cap_Rz;   // B Q^T, the sketch's reconstruction of M (residual check)
  int64_t off_qrT, cap_qrT; // Householder tau
  int64_t stride;           // doubles per shot for this engine
  int maxdim;               // largest matrix side any factorization sees
};

struct DevCtx {
  int K, n, B;                                   // sites, bits per axis, shots
  int ndim;                                      // axes (2 or 3): K = ndim n
  int half;                                      // meeting site of the Kronecker rounding (K / 2)
  int boundary;
  int ordering;                                  // MPSW_SEQUENTIAL or MPSW_INTERLEAVED
  double lam2;
  int64_t mps_stride;                            // doubles per shot of the MPS arena
  double* mps;                                   // MPS arena base
  int64_t off_mps[MPSW_NSLOT][MPSW_MAXK];
  int64_t cap_mps[MPSW_NSLOT][MPSW_MAXK];
  int* dims;                                     // B * ShotDimsLayout::size
  double* reals;                                 // B * ShotRealLayout::size
  double* eng;                                   // engine arena base
  EngineLayout L;
  // c^2 diagonal (shared by all shots)
  const double* c2;
  const double* c2d;                             // c^2 as a dense field in site order (2^K)
  int64_t off_c2[MPSW_MAXK];
  int c2b[MPSW_MAXK + 1];
  // fused Laplacian MPO cores [wl][wr][2][2] (shared)
  const double* lapW;
  int off_W[MPSW_MAXK];
  int wb[MPSW_MAXK + 1];
  // per-shot wavelets (B * nt_max)
  const double* wavelet;
  int nt_max;
  // dense buffers for to_dense / from_dense (per shot, ping-pong)
  double* dense;
  int64_t dense_stride;
  int* err;
  int* sync;                                     // B * MPSW_SYNC_STRIDE
  // learned-rank rounding
  const float* mlp_w;                            // rank network parameters (MLP_NPARAM)
  unsigned long long seed;                       // of the Gaussian test matrices
  int rrf_over;                                  // oversampling p of the sketch width
  int rank_prev;                                 // 1: sketch at the previous step's rank, no network
};

__host__ __device__ inline int64_t mpsw_pow2(int e) { return (int64_t)1 << e; }
