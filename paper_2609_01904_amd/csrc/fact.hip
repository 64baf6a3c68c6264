// Multi-workgroup factorisations of libmpsw (gfx950):
//   k_qrf    blocked Householder QR of a tall unfolding, column blocks spread
//            over the workgroups of a shot, panels published through flags
//            (the owner of panel j+1 factors it as soon as reflector j reached
//            it; everybody else updates its own blocks meanwhile);
//   k_applyq applies the compact-WY reflectors of a QR to [U_r Sigma_r; 0];
//   k_jac    one-sided block Jacobi (Hestenes) on the thin orientation of a
//            bond matrix, block pairs held in LDS, pairs of blocks scheduled
//            round-robin across the workgroups of a shot;
//   k_jacfin singular values, ordering, truncation rule, new core.
// Inter-workgroup waits are bounded: a wait that exceeds its spin budget sets
// an error bit and proceeds, so no launch can hang the device.
#include "mpsw_device.h"

#include <math.h>

#include <algorithm>

namespace mpsw {

#define MPSW_SPIN_LIMIT (1 << 22)
#define MPSW_PERM_MAX 1024
#define QNT 1024   // threads of the QR-family kernels
#define MPSW_APPLY_LDS (16 * 256 + 256)   // doubles of LDS for apply_reflector
#define APNT 512   // threads of k_applyq, k_applyv, k_formq (8 waves, no register spills)

// s_waitcnt vmcnt(0), the export and LDS counters left at their maxima (GFX9
// encoding): every vector-memory operation of this wave has completed, the
// L2 write-back or invalidate of a fence included.
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Publication between the workgroups of one shot, which may sit on different
// XCDs (each with its own L2).  One thread of the producer releases (an
// agent-scope fence, i.e. an L2 write-back, then a relaxed flag update), one
// thread of the consumer acquires (relaxed spins, then an agent-scope fence,
// i.e. an L2 invalidate), and workgroup barriers order the other waves on
// both sides.  Two waits make that chain hold for every wave: before the
// producer's barrier every wave waits for its own stores, so the write-back
// covers all of them; and each fence's cache operation completes before the
// thread that issued it goes on to the flag or to the barrier, since a fence
// orders its cache operation only against later accesses of its own wave, not
// against those of the waves a barrier then releases.
__device__ __forceinline__ void release_agent() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  wait_vmem();
}
__device__ __forceinline__ void acquire_agent() {
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  wait_vmem();
}

// One thread waits until *p >= v (bounded).  The spin uses relaxed loads and
// a single acquire follows: an acquire load per spin would invalidate the L2
// of the waiting workgroup's XCD on every iteration, evicting the data every
// other workgroup on that XCD is working on.
__device__ void wait_geq(const DevCtx& c, const int* p, int v) {
  int it = 0;
  while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < v) {
    if ((++it & 127) == 0) {
      const int e = __hip_atomic_load(c.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (it > MPSW_SPIN_LIMIT || (e & MPSW_DEV_ERR_TIMEOUT)) {
        atomicOr(c.err, MPSW_DEV_ERR_TIMEOUT);
        return;
      }
    }
    __builtin_amdgcn_s_sleep(1);
  }
  acquire_agent();
}

// Barrier of the nwg workgroups of one shot (arrival counter, monotone):
// every wave's stores complete, then thread 0 releases them with its arrival
// and acquires the other workgroups' with its wait.
__device__ void shot_barrier(const DevCtx& c, int* ctr, int nwg, int& epoch) {
  wait_vmem();
  __syncthreads();
  if (nwg == 1) return;   // a lone workgroup: the workgroup barrier is all of it
  ++epoch;
  if (threadIdx.x == 0) {
    release_agent();
    __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    wait_geq(c, ctr, epoch * nwg);
  }
  __syncthreads();
}

__global__ void k_sync_reset(const DevCtx* __restrict__ cp) {
  const DevCtx& c = *cp;
  int* s = shot_sync(c, blockIdx.x);
  for (int i = threadIdx.x; i < MPSW_SYNC_STRIDE; i += blockDim.x) s[i] = 0;
}

// ---------------------------------------------------------------------------
// Block reflector application on the FP64 matrix cores, 1024 threads.
// V: unit lower trapezoidal (mj x bw), element (r, p) at V[r + ldv * p] for r > p.
// C: mj x bwc (bwc <= 16), element (r, q) at C[r * crs + q * ccs].
// C <- C - V op(T) V^T C with op(T) = T^T (trans) or T; T is bw x bw upper,
// row-major with leading dimension BW.
//
// Both products are 16 x 16 tiles of v_mfma_f64_16x16x4f64 (operand lanes:
// a = A[l % 16][l / 16], b = B[l / 16][l % 16]; result D[l / 16 + 4 v][l % 16]),
// padded with zeros beyond bw and bwc.  Phase 1 (W = V^T C) splits the rows
// over the 16 waves, four rows per product and UN products in flight per wave,
// then sums the 16 partial tiles in a fixed order; phase 2 (C -= V W2) gives
// each wave 16-row tiles of C.  wsp: LDS of >= 16 * 256 + 256 doubles.
// ---------------------------------------------------------------------------
typedef double mpsw_d4 __attribute__((ext_vector_type(4)));

template <int BW, int NWV = 16>
__device__ void apply_reflector(const double* __restrict__ V, int64_t ldv, double* C, int64_t crs, int64_t ccs,
                                int mj, int bw, int bwc, const double* __restrict__ T, bool trans, double* wsp,
                                int t0 = 0) {
  static_assert(BW <= 16, "panel wider than one matrix-core tile");
  const int t = threadIdx.x - t0, l = t & 63, wv = t >> 6;
  const int li = l & 15, lk = l >> 4;
  // unit lower trapezoid of V, zero beyond the panel width
  auto vfull = [&](int r, int p) -> double {
    if (r >= mj || p >= bw) return 0.0;
    const double v = V[r + ldv * p];   // inside the factored matrix for every r < mj
    return (r > p) ? v : ((r == p) ? 1.0 : 0.0);
  };
  constexpr int UN = 4;
  const int nsteps = (mj + 3) >> 2;
  mpsw_d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int s0 = wv; s0 < nsteps; s0 += NWV * UN) {
    double av[UN], bv[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const int r = 4 * (s0 + NWV * u) + lk;
      av[u] = vfull(r, li);
      bv[u] = (r < mj && li < bwc) ? C[(int64_t)r * crs + (int64_t)li * ccs] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UN; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) wsp[wv * 256 + (lk + 4 * v) * 16 + li] = acc[v];
  __syncthreads();
  double* W2 = wsp + NWV * 256;
  if (t < 256) {
    double s = 0.0;
    for (int w = 0; w < NWV; ++w) s += wsp[w * 256 + t];
    wsp[t] = s;   // W[p][q], p = t / 16, q = t % 16
  }
  __syncthreads();
  if (t < 256) {
    const int p = t >> 4, q = t & 15;
    double s = 0.0;
    if (p < bw) {
      if (trans) {   // (T^T W)[p][q] = sum_{s<=p} T[s][p] W[s][q]
        for (int s2 = 0; s2 <= p; ++s2) s = fma(T[s2 * BW + p], wsp[s2 * 16 + q], s);
      } else {       // (T W)[p][q] = sum_{s>=p} T[p][s] W[s][q]
        for (int s2 = p; s2 < bw; ++s2) s = fma(T[p * BW + s2], wsp[s2 * 16 + q], s);
      }
    }
    W2[t] = s;
  }
  __syncthreads();
  // phase 2: C[r][q] -= sum_p V[r][p] W2[p][q], 16-row tiles
  double bk[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) bk[kk] = W2[(4 * kk + lk) * 16 + li];
  const int ntile = (mj + 15) >> 4;
  for (int tb = wv; tb < ntile; tb += 2 * NWV) {
    double av[2][4], cv[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int r0 = 16 * (tb + NWV * h);
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) av[h][kk] = (4 * kk < bw) ? vfull(r0 + li, 4 * kk + lk) : 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + lk + 4 * v;
        cv[h][v] = (r < mj && li < bwc) ? C[(int64_t)r * crs + (int64_t)li * ccs] : 0.0;
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      mpsw_d4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) d = __builtin_amdgcn_mfma_f64_16x16x4f64(av[h][kk], bk[kk], d, 0, 0, 0);
      const int r0 = 16 * (tb + NWV * h);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + lk + 4 * v;
        if (r < mj && li < bwc) C[(int64_t)r * crs + (int64_t)li * ccs] = cv[h][v] - d[v];
      }
    }
  }
  wait_vmem();   // other waves read the updated columns next
  __syncthreads();
}

// ---------------------------------------------------------------------------
// One wave applies a staged panel's block reflector to one group of at most
// 16 columns: C -= V T^T (V^T C), all on the matrix cores, no workgroup
// synchronisation.  V (mj x bw, unit lower trapezoid; its strict lower part
// in Vl, column-major with leading dimension ldv) sits in LDS; C (mj x bwc,
// column-major, leading dimension ldc) and T (BW x BW row-major, upper
// triangular) in global memory.  The row sum of V^T C runs in any order, so
// lane (li, lk) takes rows 16 t + 4 lk + e of column li for both operands
// (4 contiguous doubles per lane); the update's rows are permuted the same
// way, so each lane writes 4 contiguous rows of its column.
// ---------------------------------------------------------------------------
template <int BW>
__device__ void apply_wave(const double* Vl, int ldv, int mj, int bw, double* C, int64_t ldc, int bwc,
                           const double* __restrict__ T) {
  const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
  // branch-free: every lane loads an in-range element, then selects
  auto vfull = [&](int rr, int p) -> double {
    const double x = Vl[min(rr, mj - 1) + ldv * min(p, bw - 1)];
    const bool in = rr < mj && p < bw;
    const double y = (in && rr > p) ? x : 0.0;
    return (in && rr == p) ? 1.0 : y;
  };
  const bool colok = li < bwc;
  // global address space: its loads are counted apart from the LDS reads, so
  // waiting for V does not wait for C
  typedef __attribute__((address_space(1))) double gdouble;
  gdouble* Cc = (gdouble*)(C + (int64_t)(colok ? li : 0) * ldc);   // column 0 stands in for idle lanes
  const int nchunk = (mj + 15) >> 4, nfull = mj >> 4;
  constexpr int UN = 2;   // chunks whose loads are in flight together
  // W = V^T C; acc[v] = W[lk + 4 v][li]
  mpsw_d4 acc = {0.0, 0.0, 0.0, 0.0};
  int tt = 0;
  for (; tt + UN <= nfull; tt += UN) {
    double cv[UN][4];
#pragma unroll
    for (int u = 0; u < UN; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) cv[u][e] = Cc[16 * (tt + u) + 4 * lk + e];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const int rb = 16 * (tt + u) + 4 * lk;
#pragma unroll
      for (int e = 0; e < 4; ++e)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(vfull(rb + e, li), colok ? cv[u][e] : 0.0, acc, 0, 0, 0);
    }
  }
  for (; tt < nchunk; ++tt) {
    const int rb = 16 * tt + 4 * lk;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const double cv = (colok && rb + e < mj) ? Cc[rb + e] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(vfull(rb + e, li), cv, acc, 0, 0, 0);
    }
  }
  // W2 = T^T W: the accumulator of W is the b operand of k-step v
  mpsw_d4 w2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int sidx = 4 * kk + lk;   // A2[li][sidx] = T[sidx][li], zero below the diagonal
    const double a = (sidx < BW && li < BW && sidx <= li && li < bw) ? T[sidx * BW + li] : 0.0;
    w2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, acc[kk], w2, 0, 0, 0);
  }
  // C -= V W2 in 16-row tiles; A's row i is tile row 4 (i % 4) + i / 4, so
  // lane (li, lk) owns rows 4 lk .. 4 lk + 3 of the tile in column li
  auto tile = [&](int rb0, const double (&cv)[4], bool full) {
    const int ra = rb0 + 4 * (li & 3) + (li >> 2);
    mpsw_d4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
      if (4 * kk < bw) d = __builtin_amdgcn_mfma_f64_16x16x4f64(vfull(ra, 4 * kk + lk), w2[kk], d, 0, 0, 0);
    const int rw = rb0 + 4 * lk;
    if (full) {
      if (colok) {
#pragma unroll
        for (int v = 0; v < 4; ++v) Cc[rw + v] = cv[v] - d[v];
      }
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (colok && rw + v < mj) Cc[rw + v] = cv[v] - d[v];
    }
  };
  tt = 0;
  for (; tt + UN <= nfull; tt += UN) {
    double cv[UN][4];
#pragma unroll
    for (int u = 0; u < UN; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) cv[u][e] = Cc[16 * (tt + u) + 4 * lk + e];
#pragma unroll
    for (int u = 0; u < UN; ++u) tile(16 * (tt + u), cv[u], true);
  }
  for (; tt < nchunk; ++tt) {
    const int rw = 16 * tt + 4 * lk;
    double cv[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) cv[e] = (colok && rw + e < mj) ? Cc[rw + e] : 0.0;
    tile(16 * tt, cv, false);
  }
}

// ---------------------------------------------------------------------------
// QR factorisation.  a.op = 0: QR sweep at site a.site (X or X2 -> Q slot,
// R buffer, rt/qid).  For the SVD of the bond matrix M (rt_k x 2 rho_{k+1}):
// a.op = 1 factors M = Q R when M is tall or square (R^T -> Jacobi buffer),
// else M^T = Q1 R1 (R1^T -> second buffer); a.op = 2 (wide M only) factors
// the square R1^T = Q2 R2 (R2^T -> Jacobi buffer).  The Jacobi sweep then
// always runs on the transposed triangular factor of a tall-or-square matrix.
// ---------------------------------------------------------------------------
template <int BW, int NT>
__device__ void factor_panel(const DevCtx& c, double* S, int m, int n, int j, double* T, double* lds,
                             double* red) {
  constexpr int RS = NT / BW;   // rows slices per column (RS >= 64: one or more waves per column)
  const int r0 = j * BW, mj = m - r0, c0 = j * BW;
  const int bw = min(BW, n - c0);
  const int t = threadIdx.x;
  double* Pn = lds;  // mj x bw, ld mj
  bulk_copy<8>(mj * bw, t, NT,
               [&](int e) { return S[r0 + (int)(e % mj) + (int64_t)m * (c0 + (int)(e / mj))]; },
               [&](int e, double v) { Pn[e] = v; });
  __shared__ double taus[16], betas[16], scales[16];
  __shared__ double part[NT / 64];
  __syncthreads();
  const int q = t / RS, rs = t % RS;
  const int lane = t & 63, wq = rs >> 6;   // wave index within the column group
  constexpr int WPC = RS / 64;             // waves per column
  // Column i: its Householder vector is kept unscaled in Pn until the panel
  // is done (v_r = scale_i * x_r); the update of columns q > i uses x_r * scale_i.
  __shared__ double wrow[16];   // deferred update of row i-1 of the trailing panel columns
  // s2 = |x_i below row i|^2 and dq = x_i . x_q below row i (same order in every thread)
  auto dots = [&](int i, double& s2, double& dq) {
    double d = 0.0;
    if (q >= i && q < bw) {
      const double* xi = Pn + (int64_t)mj * i;
      const double* xq = Pn + (int64_t)mj * q;
      for (int r = i + 1 + rs; r < mj; r += RS) d = fma(xi[r], xq[r], d);
    }
    d = wave_sum64(d);
    if (lane == 0) part[q * WPC + wq] = d;
    __syncthreads();
    s2 = 0.0;
    dq = 0.0;
    for (int u = 0; u < WPC; ++u) {
      s2 += part[i * WPC + u];
      dq += part[q * WPC + u];
    }
  };
  for (int i = 0; i < bw; ++i) {
    if (i > 0 && rs == 0 && q >= i && q < bw) Pn[(i - 1) + (int64_t)mj * q] -= wrow[q];
    double s2, dq;
    dots(i, s2, dq);
    double x0 = Pn[i + (int64_t)mj * i];
    // A column whose entries have fallen to about 1e-150 (the numerically
    // zero trailing part of a rank-deficient matrix) has squares in the
    // subnormal range, where s2 keeps only a few bits and the reflector would
    // not be orthogonal (tau |v|^2 != 2).  Such a column is scaled by 2^500
    // (exact) and summed again; tau and v do not depend on the scale, and
    // beta is scaled back.  The test reads the same values in every thread.
    double unscale = 1.0;
    if (s2 > 0.0 && fma(x0, x0, s2) < 0x1p-900) {
      __syncthreads();   // everyone has read part[] and x0
      if (q == i)
        for (int r = i + rs; r < mj; r += RS) Pn[r + (int64_t)mj * i] *= 0x1p500;
      __syncthreads();
      dots(i, s2, dq);
      x0 = Pn[i + (int64_t)mj * i];
      unscale = 0x1p-500;
    }
    double tau = 0.0, beta = x0, scale = 0.0;
    if (s2 > 0.0) {
      beta = -copysign(sqrt(x0 * x0 + s2), x0);
      tau = (beta - x0) / beta;
      scale = 1.0 / (x0 - beta);
    }
    double wqv = 0.0;
    if (q > i && q < bw && tau != 0.0) {
      double* xq = Pn + (int64_t)mj * q;
      const double* xi = Pn + (int64_t)mj * i;
      wqv = tau * (xq[i] + scale * dq);
      const double f = wqv * scale;
      for (int r = i + 1 + rs; r < mj; r += RS) xq[r] -= f * xi[r];
    }
    if (rs == 0 && q < 16) wrow[q] = wqv;   // row i of column q is read by the whole group above
    if (t == 0) {
      taus[i] = tau;
      betas[i] = beta * unscale;
      scales[i] = scale;
    }
    __syncthreads();
  }
  // (row bw-1 has no trailing panel columns, so nothing is pending here)
  // scale the vectors, put the diagonal of R in place
  for (int e = t; e < mj * bw; e += NT) {
    const int qq = e / mj, r = e % mj;
    if (r > qq) Pn[r + (int64_t)mj * qq] *= scales[qq];
  }
  __syncthreads();
  if (t < bw) Pn[t + (int64_t)mj * t] = betas[t];
  __syncthreads();
  // T (compact WY): T_ii = tau_i, T[0:i, i] = -tau_i T[0:i, 0:i] z, z_p = V[:,p]^T v_i
  double zp[BW];
#pragma unroll
  for (int p = 0; p < BW; ++p) zp[p] = 0.0;
  if (q < bw) {
    const int i = q;
    for (int r = i + 1 + rs; r < mj; r += RS) {
      const double vi = Pn[r + (int64_t)mj * i];
#pragma unroll
      for (int p = 0; p < BW; ++p)
        if (p < i) zp[p] = fma(Pn[r + (int64_t)mj * p], vi, zp[p]);
    }
  }
  __shared__ double Zp[16 * (NT / 64)];   // [BW][BW][WPC] wave partials of z
#pragma unroll
  for (int p = 0; p < BW; ++p) {
    const double v = wave_sum64(zp[p]);
    if (lane == 0) Zp[(p * BW + q) * WPC + wq] = v;
  }
  __syncthreads();
  // T = U^{-1} with U upper triangular, U_ii = 1/tau_i, U_pi = v_p^T v_i:
  // thread i solves U t = e_i for column i by back substitution, written with
  // the factor tau_p instead of a division so a zero tau yields a zero row.
  __shared__ double Us[16 * 16];
  if (t < BW * BW) {
    const int p = t / BW, i = t % BW;
    double x = 0.0;
    if (p < i && i < bw) {
      for (int u = 0; u < WPC; ++u) x += Zp[(p * BW + i) * WPC + u];
      x += Pn[i + (int64_t)mj * p];
    }
    Us[t] = x;
  }
  __syncthreads();
  if (t < bw) {
    const int i = t;
    double tc[BW];
#pragma unroll
    for (int p = BW - 1; p >= 0; --p) {
      double v = 0.0;
      if (p == i) {
        v = taus[p];
      } else if (p < i) {
        double s = 0.0;
#pragma unroll
        for (int s2 = p + 1; s2 < BW; ++s2)
          if (s2 <= i) s = fma(Us[p * BW + s2], tc[s2], s);
        v = -taus[p] * s;
      }
      tc[p] = v;
    }
#pragma unroll
    for (int p = 0; p < BW; ++p) T[(int64_t)j * BW * BW + p * BW + i] = tc[p];
  }
  for (int e = bw + t; e < BW; e += NT)   // unused columns of a ragged panel
    for (int p = 0; p < BW; ++p) T[(int64_t)j * BW * BW + p * BW + e] = 0.0;
  bulk_copy<8>(mj * bw, t, NT, [&](int e) { return Pn[e]; },
               [&](int e, double v) { S[r0 + (int)(e % mj) + (int64_t)m * (c0 + (int)(e / mj))] = v; });
  __syncthreads();
}

template <int BW>
__global__ __launch_bounds__(1024) void k_qrf(const DevCtx* __restrict__ cp, OpArgs a) {
  const DevCtx& c = *cp;
  const int shot = blockIdx.z, w = blockIdx.x, P = gridDim.x;
  int* dm = shot_dims(c, shot);
  double* E = shot_eng(c, shot);
  const EngineLayout& L = c.L;
  const int k = a.site;
  const bool sweep = (a.op == 0);
  const bool sketch = (a.op == 3);   // basis of a randomized range finder sketch
  int m, n;
  int64_t xr, xc;   // element (r, col) of the matrix to factor is X[r * xr + col * xc]
  const double* X;
  int64_t capX, capS, capT;
  double *S, *T, *Rout;
  int64_t capRout;
  if (sweep) {
    m = 2 * dm[DL::rt + k];
    n = dm[DL::rin + k + 1];
    X = E + (a.aux ? L.off_X2 : L.off_X);
    capX = a.aux ? L.cap_X2 : L.cap_X;
    xr = n; xc = 1;
    S = E + L.off_q[k];
    capS = L.cap_q[k];
    T = E + L.off_qt[k];
    capT = L.cap_qt[k];
    Rout = E + L.off_R;
    capRout = L.cap_R;
  } else if (sketch) {   // Y (2 rho_{k+1} x l, aux 0) or Z (rt_k x l, aux 1), row-major
    if (!gate_open(dm, a.gate)) return;
    m = a.aux ? dm[DL::rt + k] : 2 * dm[DL::rho + k + 1];
    n = dm[DL::rrf_l];
    X = E + (a.aux ? L.off_Zs : L.off_Ys);
    capX = a.aux ? L.cap_Zs : L.cap_Ys;
    xr = n; xc = 1;
    S = E + L.off_qrS;
    capS = L.cap_qrS;
    T = E + L.off_qrT;
    capT = L.cap_qrT;
    Rout = nullptr;
    capRout = 0;
    if (m < n) return;   // the planner never asks for a sketch wider than tall
  } else {
    // bond matrix M (mm x nn) = (rt_k x 2 rho_{k+1})
    if (!gate_open(dm, a.gate)) return;
    const int mm = dm[DL::rt + k], nn = svd_cols(dm, k);
    const bool tall = mm >= nn;
    if (a.op == 1) {   // M = Q R (tall) or M^T = Q1 R1 (wide)
      m = tall ? mm : nn;
      n = tall ? nn : mm;
      X = E + L.off_M;
      capX = L.cap_M;
      if (tall) { xr = nn; xc = 1; } else { xr = 1; xc = nn; }
      S = E + L.off_qrS;
      capS = L.cap_qrS;
      T = E + L.off_qrT;
      capT = L.cap_qrT;
      Rout = E + (tall ? L.off_sA : L.off_sA2);
      capRout = tall ? L.cap_sA : L.cap_sA2;
    } else {           // wide only: R1^T (mm x mm, column-major in sA2) = Q2 R2
      if (tall) return;
      m = n = mm;
      X = E + L.off_sA2;
      capX = L.cap_sA2;
      xr = 1; xc = mm;
      S = E + L.off_qrS2;
      capS = L.cap_qrS2;
      T = E + L.off_qrT2;
      capT = L.cap_qrT2;
      Rout = E + L.off_sA;
      capRout = L.cap_sA;
    }
  }
  const int t = threadIdx.x;
  if ((int64_t)m * n > capX) {
    if (w == 0 && t == 0) raise_err(c, MPSW_DEV_ERR_CAP);
    return;
  }
  if (sweep && m <= n) {
    double* R = E + L.off_R;
    if ((int64_t)m * n > L.cap_R) {
      if (w == 0 && t == 0) raise_err(c, MPSW_DEV_ERR_CAP);
      return;
    }
    for (int64_t e = (int64_t)w * QNT + t; e < (int64_t)m * n; e += (int64_t)P * QNT) R[e] = X[e];
    if (w == 0 && t == 0) {
      dm[DL::rt + k + 1] = m;
      dm[DL::qid + k] = 1;
    }
    return;
  }
  const int nbk = (n + BW - 1) / BW;
  if ((int64_t)m * n > capS || (int64_t)nbk * BW * BW > capT || nbk > (MPSW_SYNC_STRIDE - MPSW_SYNC_FLAGS) / 2 ||
      (Rout && (int64_t)n * n > capRout)) {
    if (w == 0 && t == 0) raise_err(c, MPSW_DEV_ERR_CAP);
    return;
  }
  if (w == 0 && t == 0)   // Householder QR of an m x n matrix, m >= n
    count_flops(c, shot, MPSW_KC_QR, 2.0 * m * (double)n * n - 2.0 * (double)n * n * n / 3.0);
  // the two QRs of one SVD use disjoint flag ranges
  int* flags = shot_sync(c, shot) + MPSW_SYNC_FLAGS + (a.op == 2 ? (MPSW_SYNC_STRIDE - MPSW_SYNC_FLAGS) / 2 : 0);
  extern __shared__ double lds[];
  __shared__ double red[2 * 16 * 16];
  // For the SVD the columns enter in order of decreasing norm (a one-shot
  // column pivoting): the Jacobi sweep on the transposed triangular factor
  // then converges in a few passes.  Every workgroup derives the same order;
  // workgroup 0 records it for k_jacfin.
  __shared__ double cnorm[MPSW_PERM_MAX];
  __shared__ int perm[MPSW_PERM_MAX];
  const bool pivot = !sweep && !sketch && n <= MPSW_PERM_MAX;
  if (pivot) {
    if (xr == 1) {          // columns contiguous: one wave per column
      const int lane = t & 63, wv = t >> 6;
      for (int j = wv; j < n; j += QNT / 64) {
        double s = 0.0;
        for (int r = lane; r < m; r += 64) {
          const double x = X[r + (int64_t)j * xc];
          s = fma(x, x, s);
        }
        s = wave_sum64(s);
        if (lane == 0) cnorm[j] = s;
      }
    } else {                // rows contiguous: 32 columns x 32 row slices per pass
      const int jj = t & 31, rsl = (t >> 6) * 2 + ((t >> 5) & 1), wv = t >> 6;
      for (int j0 = 0; j0 < n; j0 += 32) {
        const int j = j0 + jj;
        double s = 0.0;
        if (j < n)
          for (int r = rsl; r < m; r += 32) {
            const double x = X[(int64_t)r * xr + j];
            s = fma(x, x, s);
          }
        s += __shfl_xor(s, 32, 64);
        if ((t & 32) == 0) red[wv * 32 + jj] = s;
        __syncthreads();
        if (t < 32 && j0 + t < n) {
          double x = 0.0;
          for (int u = 0; u < QNT / 64; ++u) x += red[u * 32 + t];
          cnorm[j0 + t] = x;
        }
        __syncthreads();
      }
    }
    __syncthreads();
    // a NaN norm sorts last (key -1): the ranks stay a permutation, so no
    // column index is left unset whatever the data
    auto key = [](double x) { return (x == x) ? x : -1.0; };
    for (int j = t; j < n; j += QNT) {
      const double sj = key(cnorm[j]);
      int rank = 0;
      for (int i = 0; i < n; ++i) {
        const double si = key(cnorm[i]);
        rank += (si > sj) || (si == sj && i < j);
      }
      perm[rank] = j;
    }
    __syncthreads();
    if (w == 0) {
      double* pout = E + L.off_perm;
      for (int j = t; j < n; j += QNT) pout[j] = (double)perm[j];
    }
  }
  // Column blocks of BW are owned in groups of GB = 16 / BW adjacent blocks,
  // the groups cyclically over the P workgroups: a narrow panel's reflector
  // then reaches a whole 16-column matrix-core tile of trailing columns per
  // application.  The owner of block j factors panel j.
  constexpr int GB = 16 / BW;
  auto owner = [&](int blk) { return (blk / GB) % P; };
  // my column blocks into S (column-major m x n)
  for (int blk = 0; blk < nbk; ++blk) {
    if (owner(blk) != w) continue;
    const int c0 = blk * BW, bw = min(BW, n - c0);
    if (xc == 1 && !pivot) {
      bulk_copy<8>(m * bw, t, QNT,
                   [&](int e) { return X[(e / bw) * xr + c0 + (int)(e % bw)]; },
                   [&](int e, double v) { S[(e / bw) + (int64_t)m * (c0 + (int)(e % bw))] = v; });
    } else {
      bulk_copy<8>(m * bw, t, QNT,
                   [&](int e) {
                     const int qq = (int)(e / m), r = (int)(e % m);
                     const int src = pivot ? perm[c0 + qq] : c0 + qq;
                     return X[(int64_t)r * xr + (int64_t)src * xc];
                   },
                   [&](int e, double v) { S[(e % m) + (int64_t)m * (c0 + (int)(e / m))] = v; });
    }
  }
  wait_vmem();
  __syncthreads();
  auto publish = [&](int j) {   // see release_agent; a lone workgroup has no one to tell
    wait_vmem();
    __syncthreads();
    if (t == 0 && P > 1) {
      release_agent();
      __hip_atomic_store(flags + j, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  };
  // panel j's reflector on blocks b0..b1 (adjacent, at most 16 columns)
  auto apply = [&](int j, int b0, int b1) {
    const int r0 = j * BW, c0 = j * BW, bw = min(BW, n - c0);
    const int cb = b0 * BW, bwc = min((b1 - b0 + 1) * BW, n - cb);
    apply_reflector<BW>(S + r0 + (int64_t)m * c0, m, S + r0 + (int64_t)m * cb, 1, m, m - r0, bw, bwc,
                        T + (int64_t)j * BW * BW, true, lds);
  };
  if (owner(0) == w) {
    factor_panel<BW, QNT>(c, S, m, n, 0, T, lds, red);
    publish(0);
  }
  const int ngroups = (nbk + GB - 1) / GB;
  for (int j = 0; j < nbk; ++j) {
    if (owner(j) != w) {
      if (t == 0) wait_geq(c, flags + j, 1);
      __syncthreads();
    }
    const int j1 = j + 1;
    const bool own1 = (j1 < nbk) && (owner(j1) == w);
    if (own1) {   // the next panel first (lookahead)
      apply(j, j1, j1);
      factor_panel<BW, QNT>(c, S, m, n, j1, T, lds, red);
      publish(j1);
    }
    // my other trailing groups: panel j's reflectors staged in LDS (read after
    // the acquire of its flag), then one wave per group of up to 16 columns
    const int r0 = j * BW, mj = m - r0, bwj = min(BW, n - j * BW);
    const int ldv = mj | 1;   // odd: the 16 columns a load touches sit in distinct LDS banks
    __syncthreads();          // the LDS held the lookahead panel or the previous stage
    bulk_copy<8>(mj * bwj, t, QNT, [&](int e) { return S[r0 + (int)(e % mj) + (int64_t)m * (r0 + (int)(e / mj))]; },
                 [&](int e, double v) { lds[(e % mj) + ldv * (e / mj)] = v; });
    __syncthreads();
    int q = 0;
    for (int g = w; g < ngroups; g += P) {
      int lo = max(g * GB, j + 1);
      const int hi = min(g * GB + GB - 1, nbk - 1);
      if (own1 && lo <= j1 && j1 <= hi) lo = j1 + 1;
      if (lo > hi) continue;
      if (q++ % (QNT / 64) != (t >> 6)) continue;
      const int cb = lo * BW, bwc = min((hi - lo + 1) * BW, n - cb);
      apply_wave<BW>(lds, ldv, mj, bwj, S + r0 + (int64_t)m * cb, m, bwc, T + (int64_t)j * BW * BW);
    }
    // the next iteration's lookahead reuses the LDS and may read columns this
    // wave wrote: its stores complete first (a barrier alone does not wait)
    wait_vmem();
    __syncthreads();
  }
  // R (n x n) from my columns: row-major R (sweep) or R^T column-major (SVD)
  for (int blk = 0; blk < nbk && Rout; ++blk) {
    if (owner(blk) != w) continue;
    const int c0 = blk * BW, bw = min(BW, n - c0);
    bulk_copy<8>(n * bw, t, QNT,
                 [&](int e) {
                   const int r = (int)(e / bw), col = c0 + (int)(e % bw);
                   return (r <= col) ? S[r + (int64_t)m * col] : 0.0;
                 },
                 [&](int e, double v) {
                   const int r = (int)(e / bw), col = c0 + (int)(e % bw);
                   if (sweep) Rout[(int64_t)r * n + col] = v;
                   else Rout[col + (int64_t)n * r] = v;
                 });
  }
  if (sweep && w == 0 && t == 0) {
    dm[DL::rt + k + 1] = n;
    dm[DL::qid + k] = 0;
  }
}

// ---------------------------------------------------------------------------
// M_{k-1} (2 rt_{k-1} x rho_k) = Q_{k-1} [U_r Sigma_r; 0], column chunks of 8
// per workgroup, reflectors applied last to first.
// ---------------------------------------------------------------------------
template <int BW>
__global__ __launch_bounds__(APNT) void k_applyq(const DevCtx* __restrict__ cp, OpArgs a) {
  const DevCtx& c = *cp;
  const int shot = blockIdx.z, w = blockIdx.x;
  const int k = a.site;
  int* dm = shot_dims(c, shot);
  double* E = shot_eng(c, shot);
  const EngineLayout& L = c.L;
  const int rtp = dm[DL::rt + k - 1], n = dm[DL::rt + k], r = dm[DL::rho + k];
  const int m = 2 * rtp;
  const int t = threadIdx.x;
  const double* US = E + L.off_US;
  double* M = E + L.off_M;
  if ((int64_t)m * r > L.cap_M || (int64_t)n * r > L.cap_US) {
    if (w == 0 && t == 0) raise_err(c, MPSW_DEV_ERR_CAP);
    return;
  }
  constexpr int CW = 16;   // columns per workgroup: one matrix-core tile
  const int col0 = w * CW;
  if (col0 >= r) return;
  const int cw = min(CW, r - col0);
  if (dm[DL::qid + k - 1]) {  // identity: rt_k = 2 rt_{k-1}, same memory shape
    bulk_copy<8>(m * cw, t, APNT, [&](int e) { return US[(e / cw) * r + col0 + (int)(e % cw)]; },
                 [&](int e, double v) { M[(e / cw) * r + col0 + (int)(e % cw)] = v; });
    return;
  }
  const double* S = E + L.off_q[k - 1];
  const double* T = E + L.off_qt[k - 1];
  const int nbk = (n + BW - 1) / BW;
  if ((int64_t)m * n > L.cap_q[k - 1] || (int64_t)nbk * BW * BW > L.cap_qt[k - 1]) {
    if (t == 0) raise_err(c, MPSW_DEV_ERR_CAP);
    return;
  }
  extern __shared__ double wsp[];
  if (w == 0 && t == 0)   // n reflectors of length <= m applied to r columns
    count_flops(c, shot, MPSW_KC_APPLYQ, 4.0 * m * (double)n * r - 2.0 * (double)n * n * r);
  if (a.aux > 0 && m <= a.aux) {
    // the m x cw tile of M stays in LDS (row stride CW) across all panels:
    // read from U Sigma once, written to M once
    double* Ct = wsp + MPSW_APPLY_LDS;
    for (int e = t; e < m * CW; e += APNT) {
      const int row = e / CW, q = e % CW;
      Ct[e] = (row < n && q < cw) ? US[(int64_t)row * r + col0 + q] : 0.0;
    }
    __syncthreads();
    for (int j = nbk - 1; j >= 0; --j) {
      const int r0 = j * BW, c0 = j * BW, bw = min(BW, n - c0);
      apply_reflector<BW, APNT / 64>(S + r0 + (int64_t)m * c0, m, Ct + (int64_t)r0 * CW, CW, 1, m - r0, bw, cw,
                                     T + (int64_t)j * BW * BW, false, wsp);
    }
    for (int e = t; e < m * cw; e += APNT) {
      const int row = e / cw, q = e % cw;
      M[(int64_t)row * r + col0 + q] = Ct[row * CW + q];
    }
    return;
  }
  bulk_copy<8>(m * cw, t, APNT,
               [&](int e) { return (e / cw < n) ? US[(e / cw) * r + col0 + (int)(e % cw)] : 0.0; },
               [&](int e, double v) { M[(e / cw) * r + col0 + (int)(e % cw)] = v; });
  __syncthreads();
  for (int j = nbk - 1; j >= 0; --j) {
    const int r0 = j * BW, c0 = j * BW, bw = min(BW, n - c0);
    apply_reflector<BW, APNT / 64>(S + r0 + (int64_t)m * c0, m, M + (int64_t)r0 * r + col0, r, 1, m - r0, bw, cw,
                        T + (int64_t)j * BW * BW, false, wsp);
  }
}

// ---------------------------------------------------------------------------
// Wide bond matrix: V_r (n x r) = Q1 [V'_r; 0] with the reflectors of M^T =
// Q1 R1; V'^T (r x m) comes from k_jacfin, core k (r x n) = V_r^T.
// Column chunks of BW per workgroup.
// ---------------------------------------------------------------------------
template <int BW>
__global__ __launch_bounds__(APNT) void k_applyv(const DevCtx* __restrict__ cp, OpArgs a) {
  const DevCtx& c = *cp;
  const int shot = blockIdx.z, w = blockIdx.x;
  const int k = a.site;
  const int* dm = shot_dims(c, shot);
  double* E = shot_eng(c, shot);
  const EngineLayout& L = c.L;
  if (!gate_open(dm, a.gate)) return;
  const int m = dm[DL::rt + k], n = svd_cols(dm, k), r = dm[DL::rho + k];
  if (m >= n) return;
  const int t = threadIdx.x;
  const int col0 = w * 16;   // columns per workgroup: one matrix-core tile
  if (col0 >= r) return;
  const int cw = min(16, r - col0);
  const int nbk = (m + BW - 1) / BW;
  double* Y = E + L.off_Yv;           // n x r row-major work
  const double* Vp = E + L.off_Vp;    // r x m
  const double* S = E + L.off_qrS;    // reflectors of M^T (n x m, column-major)
  const double* T = E + L.off_qrT;
  double* core = shot_mps(c, shot) + c.off_mps[a.slot][k];
  if ((int64_t)n * r > L.cap_Yv || (int64_t)r * m > L.cap_Vp || (int64_t)n * m > L.cap_qrS ||
      (int64_t)nbk * BW * BW > L.cap_qrT || (int64_t)r * n > c.cap_mps[a.slot][k]) {
    if (t == 0) raise_err(c, MPSW_DEV_ERR_CAP);
    return;
  }
  extern __shared__ double wsp[];
  if (w == 0 && t == 0)   // m reflectors of length <= n applied to r columns
    count_flops(c, shot, MPSW_KC_APPLYV, 4.0 * n * (double)m * r - 2.0 * (double)m * m * r);
  bulk_copy<8>(n * cw, t, APNT,
               [&](int e) {
                 const int row = (int)(e / cw), qq = (int)(e % cw);
                 return (row < m) ? Vp[(int64_t)(col0 + qq) * m + row] : 0.0;
               },
               [&](int e, double v) { Y[(e / cw) * r + col0 + (int)(e % cw)] = v; });
  __syncthreads();
  for (int j = nbk - 1; j >= 0; --j) {
    const int r0 = j * BW, c0 = j * BW, bw = min(BW, m - c0);
    apply_reflector<BW, APNT / 64>(S + r0 + (int64_t)n * c0, n, Y + (int64_t)r0 * r + col0, r, 1, n - r0, bw, cw,
                        T + (int64_t)j * BW * BW, false, wsp);
  }
  bulk_copy<8>(n * cw, t, APNT, [&](int e) { return Y[(e % n) * r + col0 + (int)(e / n)]; },
               [&](int e, double v) { core[(int64_t)(col0 + (int)(e / n)) * n + (e % n)] = v; });
}

// ---------------------------------------------------------------------------
// Explicit orthonormal basis of a sketch: Q = H_0 ... H_{nb-1} [I_l; 0] from
// the reflectors k_qrf (op 3) left in qrS/qrT, written over the sketch
// (Y for aux 0, Z for aux 1; m x l row-major).  Column chunks of 16 per
// workgroup.
// ---------------------------------------------------------------------------
template <int BW>
__global__ __launch_bounds__(APNT) void k_formq(const DevCtx* __restrict__ cp, OpArgs a) {
  const DevCtx& c = *cp;
  const int shot = blockIdx.z, w = blockIdx.x;
  const int k = a.site;
  const int* dm = shot_dims(c, shot);
  if (!gate_open(dm, a.gate)) return;
  double* E = shot_eng(c, shot);
  const EngineLayout& L = c.L;
  const int m = a.aux ? dm[DL::rt + k] : 2 * dm[DL::rho + k + 1], l = dm[DL::rrf_l];
  const int t = threadIdx.x;
  const int col0 = w * 16;
  if (col0 >= l || m < l) return;
  const int cw = min(16, l - col0);
  const int nbk = (l + BW - 1) / BW;
  double* Q = E + (a.aux ? L.off_Zs : L.off_Ys);
  const double* S = E + L.off_qrS;
  const double* T = E + L.off_qrT;
  if ((int64_t)m * l > (a.aux ? L.cap_Zs : L.cap_Ys) || (int64_t)m * l > L.cap_qrS ||
      (int64_t)nbk * BW * BW > L.cap_qrT) {
    if (t == 0) raise_err(c, MPSW_DEV_ERR_CAP);
    return;
  }
  extern __shared__ double wsp[];
  bulk_copy<8>(m * cw, t, APNT, [&](int e) { return ((e / cw) == col0 + (e % cw)) ? 1.0 : 0.0; },
               [&](int e, double v) { Q[(int64_t)(e / cw) * l + col0 + (e % cw)] = v; });
  __syncthreads();
  for (int j = nbk - 1; j >= 0; --j) {
    const int r0 = j * BW, c0 = j * BW, bw = min(BW, l - c0);
    apply_reflector<BW, APNT / 64>(S + r0 + (int64_t)m * c0, m, Q + (int64_t)r0 * l + col0, l, 1, m - r0, bw, cw,
                        T + (int64_t)j * BW * BW, false, wsp);
  }
}

// ---------------------------------------------------------------------------
// One-sided block Jacobi on A = R^T (column-major c x c), R the triangular
// factor of the bond matrix M (rt_k x 2 rho_{k+1}) or of M^T, whichever is
// tall; c = min(rt_k, 2 rho_{k+1}).  The triangular preconditioning makes the
// sweeps converge in a handful of passes.  Blocks of b columns; in each round
// every active workgroup loads one pair of blocks into LDS and rotates all
// column pairs of the pair once.  Sweeps repeat until one rotates nothing.
// ---------------------------------------------------------------------------
// Rotation of one column pair by a group of 16 lanes (a DPP row); each lane
// keeps its EPL elements of both columns in registers (columns of length
// Lc <= 16 EPL; EPL = 0: any length, streamed from LDS).  Returns the squared
// cosine of the pair's angle, ga^2 / (al be), or -1 when either column is
// numerically zero; rotates when it exceeds tol2.
//
// The angle (Rutishauser's formulas) uses the hardware reciprocal and
// reciprocal square root, each refined by one Newton step: the tangent then
// carries a relative error of a few ulps, which only changes how far the pair
// is rotated, while cs = 1/sqrt(1+t^2), sn = cs t keep the rotation orthogonal
// to rounding.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  return r * fma(-x, r, 2.0);
}
__device__ __forceinline__ double rsq_nr(double x) {   // x >= 1 here
  const double y = __builtin_amdgcn_rsq(x);
  return y * fma(-0.5 * x * y, y, 1.5);
}

__device__ __forceinline__ bool jacobi_angle(double al, double be, double ga, double tol2, double floor2,
                                             double& rel2, double& cs, double& sn) {
  if (al <= floor2 || be <= floor2) {
    rel2 = -1.0;
    return false;
  }
  const double ab = al * be, g2 = ga * ga;
  rel2 = g2 * rcp_nr(ab);
  if (!(g2 > tol2 * ab)) return false;
  const double zeta = (be - al) * rcp_nr(2.0 * ga);
  double tt;
  if (fabs(zeta) > 1e100) {
    tt = 0.5 * rcp_nr(zeta);
  } else {
    const double q = fma(zeta, zeta, 1.0);
    tt = copysign(rcp_nr(fabs(zeta) + q * rsq_nr(q)), zeta);
  }
  cs = rsq_nr(fma(tt, tt, 1.0));
  sn = cs * tt;
  return true;
}

// Columns of 16 EPL rows (zero padded in LDS beyond the live length, so no
// element needs a bounds check).  The first column may live in registers (x).
template <int EPL>
__device__ __forceinline__ double rotate_reg(double (&x)[EPL], double* aq, int gl, double tol2, double floor2) {
  double y[EPL];
#pragma unroll
  for (int e = 0; e < EPL; ++e) y[e] = aq[gl + 16 * e];
  // NA accumulators per sum shorten the dependent chains
  constexpr int NA = (EPL < 4) ? EPL : 4;
  double al_[NA], be_[NA], ga_[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) al_[i] = be_[i] = ga_[i] = 0.0;
#pragma unroll
  for (int e = 0; e < EPL; ++e) {
    al_[e % NA] = fma(x[e], x[e], al_[e % NA]);
    be_[e % NA] = fma(y[e], y[e], be_[e % NA]);
    ga_[e % NA] = fma(x[e], y[e], ga_[e % NA]);
  }
#pragma unroll
  for (int i = 1; i < NA; ++i) {
    al_[0] += al_[i];
    be_[0] += be_[i];
    ga_[0] += ga_[i];
  }
  const double al = row_sum16(al_[0]), be = row_sum16(be_[0]), ga = row_sum16(ga_[0]);
  double rel2, cs, sn;
  if (!jacobi_angle(al, be, ga, tol2, floor2, rel2, cs, sn)) return rel2;
#pragma unroll
  for (int e = 0; e < EPL; ++e) {
    const double xe = x[e], ye = y[e];
    x[e] = cs * xe - sn * ye;
    aq[gl + 16 * e] = sn * xe + cs * ye;
  }
  return rel2;
}

template <int EPL>
__device__ __forceinline__ double rotate_pair(double* ap, double* aq, int gl, int Lc, double tol2, double floor2) {
  double x[EPL];
#pragma unroll
  for (int e = 0; e < EPL; ++e) x[e] = ap[gl + 16 * e];
  const double rel2 = rotate_reg<EPL>(x, aq, gl, tol2, floor2);
#pragma unroll
  for (int e = 0; e < EPL; ++e) ap[gl + 16 * e] = x[e];
  return rel2;
}

template <>
__device__ __forceinline__ double rotate_pair<0>(double* ap, double* aq, int gl, int Lc, double tol2, double floor2) {
  double al = 0.0, be = 0.0, ga = 0.0;
  for (int i = gl; i < Lc; i += 16) {
    const double x = ap[i], y = aq[i];
    al = fma(x, x, al);
    be = fma(y, y, be);
    ga = fma(x, y, ga);
  }
  al = row_sum16(al);
  be = row_sum16(be);
  ga = row_sum16(ga);
  double rel2, cs, sn;
  if (!jacobi_angle(al, be, ga, tol2, floor2, rel2, cs, sn)) return rel2;
  for (int i = gl; i < Lc; i += 16) {
    const double x = ap[i], y = aq[i];
    ap[i] = cs * x - sn * y;
    aq[i] = sn * x + cs * y;
  }
  return rel2;
}

// A sweep visits every column pair once: round 0 pairs the blocks and
// rotates all pairs among the 2b columns of a block pair (so every block's
// internal pairs are done), later rounds only the b x b cross pairs, b
// parallel rotations per step (block B_g meets A_{(g+s) mod na} at step s).
// A sweep whose largest pair cosine was below 1e-6 leaves cosines of order
// 1e-12 or less behind for separated singular values (quadratic
// convergence), so it is the last one.  Within a cluster of close values the
// cosines fall more slowly, but a rotation inside the kept (or the dropped)
// part leaves the rounding's result unchanged; a stricter rule (1e-12)
// changed no parity result (the n = 11 set-up TT-SVD, the C0 and C2
// trajectories agreed to the last printed digit) and cost one more sweep.
#define JNT 512   // threads of k_jac: 32 groups of 16 lanes, one column pair each per step

template <int EPL>
__global__ __launch_bounds__(JNT) void k_jac(const DevCtx* __restrict__ cp, OpArgs a, int b) {
  const DevCtx& c = *cp;
  const int shot = blockIdx.z, w = blockIdx.x, P = gridDim.x;
  const int k = a.site;
  int* dm = shot_dims(c, shot);
  double* E = shot_eng(c, shot);
  if (!gate_open(dm, a.gate)) return;
  const int m = dm[DL::rt + k], n = svd_cols(dm, k);
  const int cc = (m >= n) ? n : m;
  const int Lc = cc;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, nwv = blockDim.x >> 6;
  const int nb = (cc + b - 1) / b;
  const int nbe = nb + (nb & 1);
  const int pact = nbe / 2;
  int* sy = shot_sync(c, shot);
  int epoch = 0;
  const bool ok = ((int64_t)Lc * cc <= c.L.cap_sA) && b <= JNT / 16;
  if (!ok && w == 0 && t == 0) raise_err(c, (b > JNT / 16) ? MPSW_DEV_ERR_GRID : MPSW_DEV_ERR_CAP);
  double* A = E + c.L.off_sA;
  extern __shared__ double blk[];   // 2b columns, stride ldl
  // EPL > 0: columns padded with zeros to 16 EPL rows (rotations keep the
  // padding zero); the odd stride spreads the columns over the LDS banks
  const int ldl = (EPL > 0) ? 16 * EPL + 1 : Lc + 1;
  if (EPL > 0 && Lc > 16 * EPL) {
    if (w == 0 && t == 0) raise_err(c, MPSW_DEV_ERR_CAP);
    return;
  }
  for (int e = t; e < 2 * b * ldl; e += blockDim.x) blk[e] = 0.0;
  __syncthreads();
  __shared__ int nrot;
  __shared__ unsigned int maxrel;   // float bits of the largest squared cosine
  __shared__ double fro_red[16];
  const double tol = 1e-15 * sqrt((double)Lc), tol2 = tol * tol;
  // Columns below 1e-14 ||A||_F are numerically zero (rounding noise of the
  // factorisations): they are not rotated, since their direction cannot be
  // resolved and chasing it would never converge.
  double fro = 0.0;
  if (ok) bulk_copy<8>(Lc * cc, t, JNT, [&](int e) { return A[e]; }, [&](int, double v) { fro = fma(v, v, fro); });
  fro = wave_sum(fro);
  if (lane == 0) fro_red[wv] = fro;
  __syncthreads();
  fro = 0.0;
  for (int i = 0; i < nwv; ++i) fro += fro_red[i];
  const double floor2 = 1e-28 * fro;
  // every workgroup has read A for the norm before any of them rotates a block
  // of it, so all of them hold the same floor
  shot_barrier(c, sy + MPSW_SYNC_BARRIER, P, epoch);
  // the eigen stage of an SVD of a c x c factor, 9 c^3 by the standard count
  if (ok && w == 0 && t == 0) count_flops(c, shot, MPSW_KC_JACOBI, 9.0 * (double)cc * cc * cc);
  const int g = t >> 4, gl = t & 15, ng = JNT / 16;
  // rotations applied and the largest squared cosine seen, kept per group in
  // registers and merged once per round
  int myrot = 0;
  float mymax = 0.0f;
  auto note = [&](double rel2) {
    if (rel2 >= 0.0) {
      myrot += (rel2 > tol2) ? 1 : 0;
      mymax = fmaxf(mymax, (float)fmin(rel2, 1.0));
    }
  };
  for (int sweep = 0; sweep < MPSW_MAX_SWEEPS; ++sweep) {
    for (int rnd = 0; rnd < nbe - 1; ++rnd) {
      // the round's pact block pairs are disjoint: workgroup w takes pairs
      // w, w + P, ... one after the other (fewer workgroups than pairs trade
      // parallelism within a shot for fewer cross-workgroup barriers)
      for (int pw = w; ok && pw < pact && cc > 1; pw += P) {
        int bp, bq;
        if (pw == 0) { bp = rnd; bq = nbe - 1; }
        else { bp = (rnd + pw) % (nbe - 1); bq = (rnd - pw + (nbe - 1)) % (nbe - 1); }
        if (bp >= nb) { const int tmp = bp; bp = bq; bq = tmp; }
        const int np_ = (bp < nb) ? min(b, cc - bp * b) : 0;
        const int nq_ = (bq < nb) ? min(b, cc - bq * b) : 0;
        const int ncol = np_ + nq_;
        if (t == 0) { nrot = 0; maxrel = 0u; }
        auto gcol = [&](int jj) { return (jj < np_) ? bp * b + jj : bq * b + (jj - np_); };
        if constexpr (EPL > 0) {
          // columns padded to LP = 16 EPL rows (a power of two): element e is
          // (e / LP, e % LP) by shifts, and the padding rows receive zeros
          constexpr int LP = 16 * EPL;
          bulk_copy<32>(ncol * LP, t, JNT,
                        [&](int e) {
                          const int row = e & (LP - 1);
                          return (row < Lc) ? A[(int64_t)gcol(e / LP) * Lc + row] : 0.0;
                        },
                        [&](int e, double v) { blk[(e / LP) * ldl + (e & (LP - 1))] = v; });
        } else {
          bulk_copy<32>(ncol * Lc, t, blockDim.x,
                        [&](int e) { return A[(int64_t)gcol(e / Lc) * Lc + (e % Lc)]; },
                        [&](int e, double v) { blk[(e / Lc) * ldl + (e % Lc)] = v; });
        }
        __syncthreads();
        if (rnd == 0) {
          // internal pairs of both blocks at once: two round-robin
          // tournaments, the first hp pair slots for block P, the rest for Q
          const int npp = np_ + (np_ & 1), nqq = nq_ + (nq_ & 1);
          const int hp = npp / 2, hq = nqq / 2;
          const int nst = max(npp, nqq) - 1;
          for (int ir = 0; ir < nst; ++ir) {
            for (int pi = g; pi < hp + hq; pi += ng) {
              const bool inq = (pi >= hp);
              const int nn = inq ? nqq : npp, cnt = inq ? nq_ : np_, off = inq ? np_ : 0;
              const int pj = inq ? pi - hp : pi;
              if (ir >= nn - 1) continue;
              int p, q;
              if (pj == 0) { p = ir; q = nn - 1; }
              else { p = (ir + pj) % (nn - 1); q = (ir - pj + (nn - 1)) % (nn - 1); }
              if (p >= cnt || q >= cnt) continue;
              note(rotate_pair<EPL>(blk + (off + p) * ldl, blk + (off + q) * ldl, gl, Lc, tol2, floor2));
            }
            __syncthreads();
          }
        }
        if (np_ > 0 && nq_ > 0) {   // the b x b cross pairs
          const int na = max(np_, nq_), ns = min(np_, nq_);
          const int a0 = (np_ >= nq_) ? 0 : np_, s0 = (np_ >= nq_) ? np_ : 0;
          if constexpr (EPL > 0) {
            // Group g keeps column g of the smaller block in registers.  The
            // larger block is cut into chunks of 4 columns; in phase ph wave v
            // (groups 4v..4v+3) owns chunk (v + ph) mod nc alone and its four
            // groups meet the chunk's four columns in four steps, handing
            // columns to each other within the wave, so the workgroup only
            // synchronises between phases.  Active waves are v < ceil(ns/4)
            // <= nc, so no two waves own one chunk.
            double x[EPL];
            const bool act = g < ns;
            double* ap = blk + (s0 + g) * ldl;
            if (act) {
#pragma unroll
              for (int e = 0; e < EPL; ++e) x[e] = ap[gl + 16 * e];
            }
            const int nc = (na + 3) >> 2, wq = g >> 2, gi = g & 3;
            for (int ph = 0; ph < nc; ++ph) {
              const int ch = (wq + ph) % nc;
              for (int st = 0; st < 4; ++st) {
                const int col = 4 * ch + ((gi + st) & 3);
                if (act && col < na) note(rotate_reg<EPL>(x, blk + (a0 + col) * ldl, gl, tol2, floor2));
                // the column just written is read by the neighbouring group of
                // this wave in the next step
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
              }
              __syncthreads();
            }
            if (act) {
#pragma unroll
              for (int e = 0; e < EPL; ++e) ap[gl + 16 * e] = x[e];
            }
          } else {
            for (int s = 0; s < na; ++s) {
              if (g < ns) {
                const int p = s0 + g, q = a0 + (g + s) % na;
                note(rotate_pair<EPL>(blk + p * ldl, blk + q * ldl, gl, Lc, tol2, floor2));
              }
              __syncthreads();
            }
          }
        }
        if (gl == 0 && (myrot > 0 || mymax > 0.0f)) {
          atomicAdd(&nrot, myrot);
          atomicMax(&maxrel, __float_as_uint(mymax));
        }
        myrot = 0;
        mymax = 0.0f;
        __syncthreads();
        if constexpr (EPL > 0) {
          constexpr int LP = 16 * EPL;
          bulk_copy<32>(ncol * LP, t, JNT, [&](int e) { return blk[(e / LP) * ldl + (e & (LP - 1))]; },
                        [&](int e, double v) {
                          const int row = e & (LP - 1);
                          if (row < Lc) A[(int64_t)gcol(e / LP) * Lc + row] = v;
                        });
        } else {
          bulk_copy<32>(ncol * Lc, t, blockDim.x, [&](int e) { return blk[(e / Lc) * ldl + (e % Lc)]; },
                        [&](int e, double v) { A[(int64_t)gcol(e / Lc) * Lc + (e % Lc)] = v; });
        }
        if (t == 0) {
          if (nrot > 0) atomicAdd(sy + MPSW_SYNC_ROT + (sweep & 63), nrot);
          atomicMax((unsigned int*)sy + MPSW_SYNC_MAXREL + (sweep & 63), maxrel);
        }
        __syncthreads();   // the next pair's columns overwrite the LDS these were stored from
      }
      shot_barrier(c, sy + MPSW_SYNC_BARRIER, P, epoch);
    }
    // every workgroup reads the same final values after the barrier: each
    // workgroup's updates precede its arrival (release) and this one's barrier
    // acquired them, so relaxed atomic loads see them (an acquire load here
    // would invalidate the XCD's L2 once per wave)
    const int rot = __hip_atomic_load(sy + MPSW_SYNC_ROT + (sweep & 63), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const float mx = __uint_as_float((unsigned int)__hip_atomic_load(sy + MPSW_SYNC_MAXREL + (sweep & 63),
                                                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (rot == 0 || mx < 1e-12f || !ok || cc <= 1) {
      if (w == 0 && t == 0) atomicMax((int*)dm + DL::jac_sweeps, sweep + 1);
      break;
    }
  }
}

// Singular values (column norms of the converged A = R^T W), descending
// order, truncation rule, tail sum and log.  A's columns are sigma times the
// right singular vectors of the factored tall-or-square matrix: for a tall M
// they are the rows of core k; for a wide M they are V' (right singular
// vectors of R1^T), turned into V = Q1 V' by k_applyv.
#define JF_MAXC 4096
__global__ __launch_bounds__(256) void k_jacfin(const DevCtx* __restrict__ cp, OpArgs a) {
  const DevCtx& c = *cp;
  const int shot = blockIdx.z, k = a.site;
  int* dm = shot_dims(c, shot);
  double* re = shot_reals(c, shot);
  double* E = shot_eng(c, shot);
  if (!gate_open(dm, a.gate)) return;
  const int m = dm[DL::rt + k], n = svd_cols(dm, k);
  const bool tall = m >= n;
  const int cc = tall ? n : m, Lc = cc;
  __shared__ double sig[JF_MAXC];
  __shared__ int order[JF_MAXC];
  __shared__ int rank_s;
  if (cc > JF_MAXC || (int64_t)Lc * cc > c.L.cap_sA) {
    if (threadIdx.x == 0) raise_err(c, MPSW_DEV_ERR_CAP);
    return;
  }
  const double* A = E + c.L.off_sA;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, nwv = blockDim.x >> 6;
  for (int j = wv; j < cc; j += nwv) {
    const double* aj = A + (int64_t)j * Lc;
    double s = 0.0;
    for (int i = lane; i < Lc; i += 64) s = fma(aj[i], aj[i], s);
    s = wave_sum(s);
    if (lane == 0) sig[j] = sqrt(s);
  }
  __syncthreads();
  // a NaN sorts last (key -1): the order stays a permutation, and the
  // non-finite value is reported below
  auto key = [](double x) { return (x == x) ? x : -1.0; };
  for (int j = t; j < cc; j += blockDim.x) {
    const double sj = key(sig[j]);
    int r = 0;
    for (int i = 0; i < cc; ++i) {
      const double si = key(sig[i]);
      r += (si > sj) || (si == sj && i < j);
    }
    order[r] = j;
  }
  __syncthreads();
  if (t == 0) {
    const double s0 = sig[order[0]];
    const double eps = re[RL::eps];
    const int chi = dm[DL::chi];
    // Values below 1e-14 ||A||_F are rounding noise: the Jacobi sweep leaves
    // their columns unrotated (their directions cannot be resolved), so their
    // vectors are not orthogonal to the others and are never kept, whatever
    // eps (which matters for eps below about 1e-14 only).
    double fro2 = 0.0;
    for (int i = 0; i < cc; ++i) fro2 = fma(sig[order[i]], sig[order[i]], fro2);
    const double noise = 1e-14 * sqrt(fro2);
    int r = 0;
    bool finite = true;
    for (int i = 0; i < cc; ++i) {
      const double s = sig[order[i]];
      if (!(s == s) || isinf(s)) finite = false;
      if (s0 > 0.0 && s >= eps * s0 && s > noise) ++r;
    }
    if (!finite) raise_err(c, MPSW_DEV_ERR_NONFINITE);
    if (r > chi) r = chi;
    if (r < 1) r = 1;
    double tail = 0.0;
    for (int i = r; i < cc; ++i) {
      const double s = sig[order[i]];
      tail = fma(s, s, tail);
    }
    if (a.gate == GATE_SKETCH) {   // judged by k_rrf_accept before anything is kept
      double all = tail;
      for (int i = 0; i < r; ++i) all = fma(sig[order[i]], sig[order[i]], all);
      re[RL::rrf_tail] = tail;
      re[RL::rrf_sig1] = s0;
      re[RL::rrf_sum2] = all;
    } else if (a.aux >= 0 && a.aux < 3) {
      re[RL::tail2 + a.aux] += tail;
      if (cc > dm[DL::maxbond + a.aux]) dm[DL::maxbond + a.aux] = cc;
    }
    if (a.aux >= 0 && a.aux < 3) {
      double* lg = re + RL::sigma_log + (a.aux * MPSW_MAXK + k) * 32;
      for (int i = 0; i < 32; ++i) lg[i] = (i < cc) ? sig[order[i]] : 0.0;
      dm[DL::prank + a.aux * MPSW_MAXK + k] = r;   // a rejected sketch's rank is overwritten by the exact pass
    }
    rank_s = r;
  }
  __syncthreads();
  const int r = rank_s;
  // rows of V^T for the square-or-tall factor: the core itself (tall M) or
  // V'^T (r x m) to be rotated by Q1 (wide M)
  double* out = tall ? shot_mps(c, shot) + c.off_mps[a.slot][k] : E + c.L.off_Vp;
  const int64_t capo = tall ? c.cap_mps[a.slot][k] : c.L.cap_Vp;
  if ((int64_t)r * cc > capo) {
    if (t == 0) raise_err(c, MPSW_DEV_ERR_CAP);
    return;
  }
  // A's row l belongs to column perm[l] of the matrix the last QR factored
  const double* pv = E + c.L.off_perm;
  const bool pivoted = cc <= MPSW_PERM_MAX;
  for (int64_t e = t; e < (int64_t)r * cc; e += blockDim.x) {
    const int i = (int)(e / cc), l = (int)(e % cc);
    const int j = order[i];
    const double s = sig[j];
    const int dst = pivoted ? (int)pv[l] : l;
    out[(int64_t)i * cc + dst] = (s > 0.0) ? A[(int64_t)j * Lc + l] / s : ((l == i) ? 1.0 : 0.0);
  }
  if (t == 0) dm[DL::rho + k] = r;
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
void launch_sync_reset(const DevCtx* d, int nshots, hipStream_t s) {
  hipLaunchKernelGGL(k_sync_reset, dim3(nshots), dim3(256), 0, s, d);
}

void launch_qrf(const DevCtx* d, const OpArgs& a, int bw, int nwg, int nshots, size_t lds, hipStream_t s) {
  // the panel with one spare row (the staged reflectors' odd leading
  // dimension), or the reflector workspace of the lookahead application
  lds = std::max(lds + (size_t)bw * sizeof(double), (size_t)MPSW_APPLY_LDS * sizeof(double));
  if (bw == 16)
    hipLaunchKernelGGL(k_qrf<16>, dim3(nwg, 1, nshots), dim3(QNT), lds, s, d, a);
  else if (bw == 8)
    hipLaunchKernelGGL(k_qrf<8>, dim3(nwg, 1, nshots), dim3(QNT), lds, s, d, a);
  else
    hipLaunchKernelGGL(k_qrf<4>, dim3(nwg, 1, nshots), dim3(QNT), lds, s, d, a);
}

void launch_applyq(const DevCtx* d, const OpArgs& a, int bw, int nwg, int nshots, hipStream_t s) {
  // a.aux > 0: rows of the LDS-resident column tile (16 columns)
  const size_t lds = (size_t)(MPSW_APPLY_LDS + (a.aux > 0 ? 16 * a.aux : 0)) * sizeof(double);
  if (bw == 16)
    hipLaunchKernelGGL(k_applyq<16>, dim3(nwg, 1, nshots), dim3(APNT), lds, s, d, a);
  else if (bw == 8)
    hipLaunchKernelGGL(k_applyq<8>, dim3(nwg, 1, nshots), dim3(APNT), lds, s, d, a);
  else
    hipLaunchKernelGGL(k_applyq<4>, dim3(nwg, 1, nshots), dim3(APNT), lds, s, d, a);
}

void launch_applyv(const DevCtx* d, const OpArgs& a, int bw, int nwg, int nshots, hipStream_t s) {
  const size_t lds = (size_t)MPSW_APPLY_LDS * sizeof(double);
  if (bw == 16)
    hipLaunchKernelGGL(k_applyv<16>, dim3(nwg, 1, nshots), dim3(APNT), lds, s, d, a);
  else if (bw == 8)
    hipLaunchKernelGGL(k_applyv<8>, dim3(nwg, 1, nshots), dim3(APNT), lds, s, d, a);
  else
    hipLaunchKernelGGL(k_applyv<4>, dim3(nwg, 1, nshots), dim3(APNT), lds, s, d, a);
}

void launch_formq(const DevCtx* d, const OpArgs& a, int bw, int nwg, int nshots, hipStream_t s) {
  const size_t lds = (size_t)MPSW_APPLY_LDS * sizeof(double);
  if (bw == 16)
    hipLaunchKernelGGL(k_formq<16>, dim3(nwg, 1, nshots), dim3(APNT), lds, s, d, a);
  else if (bw == 8)
    hipLaunchKernelGGL(k_formq<8>, dim3(nwg, 1, nshots), dim3(APNT), lds, s, d, a);
  else
    hipLaunchKernelGGL(k_formq<4>, dim3(nwg, 1, nshots), dim3(APNT), lds, s, d, a);
}

// Rows a Jacobi column occupies in LDS for a column length of at most lcap.
int jac_rows(int64_t lcap) {
  for (int r = 32; r <= 512; r <<= 1)
    if (lcap <= r) return r;
  return (int)lcap;
}

void launch_jac(const DevCtx* d, const OpArgs& a, int b, int nwg, int nshots, size_t lds, int64_t lcap, hipStream_t s) {
  (void)lds;
  const dim3 g(nwg, 1, nshots), blk(JNT);
  const size_t bytes = (size_t)2 * b * (jac_rows(lcap) + 1) * sizeof(double);
  if (lcap <= 32) hipLaunchKernelGGL(k_jac<2>, g, blk, bytes, s, d, a, b);
  else if (lcap <= 64) hipLaunchKernelGGL(k_jac<4>, g, blk, bytes, s, d, a, b);
  else if (lcap <= 128) hipLaunchKernelGGL(k_jac<8>, g, blk, bytes, s, d, a, b);
  else if (lcap <= 256) hipLaunchKernelGGL(k_jac<16>, g, blk, bytes, s, d, a, b);
  else if (lcap <= 512) hipLaunchKernelGGL(k_jac<32>, g, blk, bytes, s, d, a, b);
  else hipLaunchKernelGGL(k_jac<0>, g, blk, bytes, s, d, a, b);
}

void launch_jacfin(const DevCtx* d, const OpArgs& a, int nshots, hipStream_t s) {
  hipLaunchKernelGGL(k_jacfin, dim3(1, 1, nshots), dim3(256), 0, s, d, a);
}

void set_lds_limits(size_t bytes) {
  (void)hipFuncSetAttribute((const void*)k_qrf<16>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  (void)hipFuncSetAttribute((const void*)k_applyq<16>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  (void)hipFuncSetAttribute((const void*)k_applyq<8>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  (void)hipFuncSetAttribute((const void*)k_applyq<4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  (void)hipFuncSetAttribute((const void*)k_qrf<8>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  (void)hipFuncSetAttribute((const void*)k_qrf<4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  (void)hipFuncSetAttribute((const void*)k_jac<2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  (void)hipFuncSetAttribute((const void*)k_jac<4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  (void)hipFuncSetAttribute((const void*)k_jac<8>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  (void)hipFuncSetAttribute((const void*)k_jac<16>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  (void)hipFuncSetAttribute((const void*)k_jac<32>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  (void)hipFuncSetAttribute((const void*)k_jac<0>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace mpsw
