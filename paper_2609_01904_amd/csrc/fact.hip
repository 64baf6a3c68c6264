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

namespace mpsw {

#define MPSW_SPIN_LIMIT (1 << 22)

__device__ __forceinline__ int ld_acquire(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// One thread waits until *p >= v (bounded).
__device__ void wait_geq(const DevCtx& c, const int* p, int v) {
  int it = 0;
  while (ld_acquire(p) < v) {
    if ((++it & 127) == 0) {
      const int e = __hip_atomic_load(c.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (it > MPSW_SPIN_LIMIT || (e & MPSW_DEV_ERR_TIMEOUT)) {
        atomicOr(c.err, MPSW_DEV_ERR_TIMEOUT);
        return;
      }
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// Barrier of the nwg workgroups of one shot (arrival counter, monotone).
__device__ void shot_barrier(const DevCtx& c, int* ctr, int nwg, int& epoch) {
  __threadfence();
  __syncthreads();
  ++epoch;
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    wait_geq(c, ctr, epoch * nwg);
  }
  __syncthreads();
  __threadfence();
}

__global__ void k_sync_reset(const DevCtx* __restrict__ cp) {
  const DevCtx& c = *cp;
  int* s = shot_sync(c, blockIdx.x);
  for (int i = threadIdx.x; i < MPSW_SYNC_STRIDE; i += blockDim.x) s[i] = 0;
}

// ---------------------------------------------------------------------------
// Block reflector application on column-major storage.
// V: unit lower trapezoidal (mj x bw), element (r, p) at V[r + ldv * p] for r > p.
// C: mj x bwc, element (r, q) at C[r * crs + q * ccs].
// C <- C - V op(T) V^T C with op(T) = T^T (trans) or T; T is bw x bw upper, row-major ld BW.
// Thread layout: t = q * RS + rs (RS = 256 / BW rows slices per column).
// ---------------------------------------------------------------------------
template <int BW>
__device__ void apply_reflector(const double* __restrict__ V, int64_t ldv, double* C, int64_t crs, int64_t ccs,
                                int mj, int bw, int bwc, const double* __restrict__ T, bool trans,
                                double* red /* LDS >= 2*BW*BW */) {
  constexpr int RS = 256 / BW;
  const int t = threadIdx.x;
  const int q = t / RS, rs = t % RS;
  double acc[BW];
#pragma unroll
  for (int p = 0; p < BW; ++p) acc[p] = 0.0;
  if (q < bwc) {
    for (int r = rs; r < mj; r += RS) {
      const double cv = C[(int64_t)r * crs + (int64_t)q * ccs];
#pragma unroll
      for (int p = 0; p < BW; ++p) {
        double v = 0.0;
        if (p < bw) v = (r > p) ? V[r + ldv * p] : ((r == p) ? 1.0 : 0.0);
        acc[p] = fma(v, cv, acc[p]);
      }
    }
  }
  // reduce over the RS row slices (RS lanes of one wave share q)
#pragma unroll
  for (int p = 0; p < BW; ++p) {
    double v = acc[p];
    for (int off = RS / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    acc[p] = v;
  }
  double* W = red;           // BW x BW
  double* W2 = red + BW * BW;
  if (rs == 0) {
#pragma unroll
    for (int p = 0; p < BW; ++p) W[p * BW + q] = acc[p];
  }
  __syncthreads();
  if (t < BW * BW) {
    const int p = t / BW, qq = t % BW;
    double s = 0.0;
    if (trans) {   // (T^T W)[p][q] = sum_{s<=p} T[s][p] W[s][q]
      for (int s2 = 0; s2 <= p && s2 < bw; ++s2) s = fma(T[s2 * BW + p], W[s2 * BW + qq], s);
    } else {       // (T W)[p][q] = sum_{s>=p} T[p][s] W[s][q]
      for (int s2 = p; s2 < bw; ++s2) s = fma(T[p * BW + s2], W[s2 * BW + qq], s);
    }
    W2[p * BW + qq] = s;
  }
  __syncthreads();
  if (q < bwc) {
    double w2[BW];
#pragma unroll
    for (int p = 0; p < BW; ++p) w2[p] = W2[p * BW + q];
    for (int r = rs; r < mj; r += RS) {
      double s = 0.0;
#pragma unroll
      for (int p = 0; p < BW; ++p) {
        if (p < bw) {
          const double v = (r > p) ? V[r + ldv * p] : ((r == p) ? 1.0 : 0.0);
          s = fma(v, w2[p], s);
        }
      }
      C[(int64_t)r * crs + (int64_t)q * ccs] -= s;
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// QR factorisation.  a.op = 0: QR sweep at site a.site (X or X2 -> Q slot,
// R buffer, rt/qid).  For the SVD of the bond matrix M (rt_k x 2 rho_{k+1}):
// a.op = 1 factors M = Q R when M is tall or square (R^T -> Jacobi buffer),
// else M^T = Q1 R1 (R1^T -> second buffer); a.op = 2 (wide M only) factors
// the square R1^T = Q2 R2 (R2^T -> Jacobi buffer).  The Jacobi sweep then
// always runs on the transposed triangular factor of a tall-or-square matrix.
// ---------------------------------------------------------------------------
template <int BW>
__device__ void factor_panel(const DevCtx& c, double* S, int m, int n, int j, double* T, double* lds,
                             double* red) {
  constexpr int RS = 256 / BW;
  const int r0 = j * BW, mj = m - r0, c0 = j * BW;
  const int bw = min(BW, n - c0);
  const int t = threadIdx.x;
  double* Pn = lds;  // mj x bw, ld mj
  for (int e = t; e < mj * bw; e += 256) {
    const int qq = e / mj, r = e % mj;
    Pn[r + (int64_t)mj * qq] = S[r0 + r + (int64_t)m * (c0 + qq)];
  }
  __shared__ double taus[16];
  __syncthreads();
  const int q = t / RS, rs = t % RS;
  for (int i = 0; i < bw; ++i) {
    // d_q = sum_{r>i} x_r P[r][q] for q >= i (d_i is the squared norm below the diagonal)
    double d = 0.0;
    if (q >= i && q < bw) {
      for (int r = i + 1 + rs; r < mj; r += RS) d = fma(Pn[r + (int64_t)mj * i], Pn[r + (int64_t)mj * q], d);
    }
    for (int off = RS / 2; off > 0; off >>= 1) d += __shfl_xor(d, off, 64);
    if (rs == 0) red[q] = d;
    __syncthreads();
    const double s2 = red[i];
    const double x0 = Pn[i + (int64_t)mj * i];
    double tau = 0.0, beta = x0, scale = 0.0;
    if (s2 > 0.0) {
      beta = -copysign(sqrt(x0 * x0 + s2), x0);
      tau = (beta - x0) / beta;
      scale = 1.0 / (x0 - beta);
    }
    double wq = 0.0;
    if (q > i && q < bw) wq = tau * (Pn[i + (int64_t)mj * q] + scale * red[q]);
    __syncthreads();
    // column i -> Householder vector, columns q > i updated
    if (q == i) {
      for (int r = i + 1 + rs; r < mj; r += RS) Pn[r + (int64_t)mj * i] *= scale;
    }
    __syncthreads();
    if (q > i && q < bw && tau != 0.0) {
      for (int r = i + 1 + rs; r < mj; r += RS) Pn[r + (int64_t)mj * q] -= wq * Pn[r + (int64_t)mj * i];
      if (rs == 0) Pn[i + (int64_t)mj * q] -= wq;
    }
    if (t == 0) {
      Pn[i + (int64_t)mj * i] = beta;
      taus[i] = tau;
    }
    __syncthreads();
  }
  // T (compact WY): T_ii = tau_i, T[0:i, i] = -tau_i T[0:i, 0:i] z, z_p = V[:,p]^T v_i
  // z for all p < i via the same slice layout: thread (q = i, rs) sums rows > i.
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
#pragma unroll
  for (int p = 0; p < BW; ++p) {
    double v = zp[p];
    for (int off = RS / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    zp[p] = v;
  }
  __shared__ double Z[16 * 16];
  if (rs == 0 && q < bw) {
#pragma unroll
    for (int p = 0; p < BW; ++p) Z[p * BW + q] = (p < q) ? zp[p] + Pn[q + (int64_t)mj * p] : 0.0;
  }
  __syncthreads();
  if (t == 0) {
    double Tl[BW * BW];
    for (int e = 0; e < BW * BW; ++e) Tl[e] = 0.0;
    for (int i = 0; i < bw; ++i) {
      Tl[i * BW + i] = taus[i];
      for (int p = 0; p < i; ++p) {
        double s = 0.0;
        for (int s2 = p; s2 < i; ++s2) s = fma(Tl[p * BW + s2], Z[s2 * BW + i], s);
        Tl[p * BW + i] = -taus[i] * s;
      }
    }
    for (int e = 0; e < BW * BW; ++e) T[(int64_t)j * BW * BW + e] = Tl[e];
  }
  for (int e = t; e < mj * bw; e += 256) {
    const int qq = e / mj, r = e % mj;
    S[r0 + r + (int64_t)m * (c0 + qq)] = Pn[r + (int64_t)mj * qq];
  }
  __syncthreads();
}

template <int BW>
__global__ __launch_bounds__(256) void k_qrf(const DevCtx* __restrict__ cp, OpArgs a) {
  const DevCtx& c = *cp;
  const int shot = blockIdx.z, w = blockIdx.x, P = gridDim.x;
  int* dm = shot_dims(c, shot);
  double* E = shot_eng(c, shot);
  const EngineLayout& L = c.L;
  const int k = a.site;
  const bool sweep = (a.op == 0);
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
  } else {
    // bond matrix M (mm x nn) = (rt_k x 2 rho_{k+1})
    const int mm = dm[DL::rt + k], nn = 2 * dm[DL::rho + k + 1];
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
    for (int64_t e = (int64_t)w * 256 + t; e < (int64_t)m * n; e += (int64_t)P * 256) R[e] = X[e];
    if (w == 0 && t == 0) {
      dm[DL::rt + k + 1] = m;
      dm[DL::qid + k] = 1;
    }
    return;
  }
  const int nbk = (n + BW - 1) / BW;
  if ((int64_t)m * n > capS || (int64_t)nbk * BW * BW > capT || nbk > (MPSW_SYNC_STRIDE - MPSW_SYNC_FLAGS) / 2 ||
      (int64_t)n * n > capRout) {
    if (w == 0 && t == 0) raise_err(c, MPSW_DEV_ERR_CAP);
    return;
  }
  // the two QRs of one SVD use disjoint flag ranges
  int* flags = shot_sync(c, shot) + MPSW_SYNC_FLAGS + (a.op == 2 ? (MPSW_SYNC_STRIDE - MPSW_SYNC_FLAGS) / 2 : 0);
  extern __shared__ double lds[];
  __shared__ double red[2 * 16 * 16];
  // my column blocks into S (column-major m x n)
  for (int blk = w; blk < nbk; blk += P) {
    const int c0 = blk * BW, bw = min(BW, n - c0);
    if (xc == 1) {
      for (int e = t; e < m * bw; e += 256) {
        const int r = e / bw, qq = e % bw;
        S[r + (int64_t)m * (c0 + qq)] = X[(int64_t)r * xr + c0 + qq];
      }
    } else {
      for (int e = t; e < m * bw; e += 256) {
        const int qq = e / m, r = e % m;
        S[r + (int64_t)m * (c0 + qq)] = X[(int64_t)r * xr + (int64_t)(c0 + qq) * xc];
      }
    }
  }
  __syncthreads();
  auto publish = [&](int j) {
    __threadfence();
    __syncthreads();
    if (t == 0) __hip_atomic_store(flags + j, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  };
  auto apply = [&](int j, int blk) {
    const int r0 = j * BW, c0 = j * BW, bw = min(BW, n - c0);
    const int cb = blk * BW, bwc = min(BW, n - cb);
    apply_reflector<BW>(S + r0 + (int64_t)m * c0, m, S + r0 + (int64_t)m * cb, 1, m, m - r0, bw, bwc,
                        T + (int64_t)j * BW * BW, true, red);
  };
  if (w == 0) {
    factor_panel<BW>(c, S, m, n, 0, T, lds, red);
    publish(0);
  }
  for (int j = 0; j < nbk; ++j) {
    if (j % P != w) {
      if (t == 0) wait_geq(c, flags + j, 1);
      __syncthreads();
      __threadfence();
    }
    const int j1 = j + 1;
    const bool own1 = (j1 < nbk) && (j1 % P == w);
    if (own1) {
      apply(j, j1);
      factor_panel<BW>(c, S, m, n, j1, T, lds, red);
      publish(j1);
    }
    int first = w;
    while (first <= j) first += P;
    for (int blk = first; blk < nbk; blk += P) {
      if (own1 && blk == j1) continue;
      apply(j, blk);
    }
  }
  // R (n x n) from my columns: row-major R (sweep) or R^T column-major (SVD)
  for (int blk = w; blk < nbk; blk += P) {
    const int c0 = blk * BW, bw = min(BW, n - c0);
    for (int e = t; e < n * bw; e += 256) {
      const int r = e / bw, qq = e % bw, col = c0 + qq;
      const double v = (r <= col) ? S[r + (int64_t)m * col] : 0.0;
      if (sweep) Rout[(int64_t)r * n + col] = v;
      else Rout[col + (int64_t)n * r] = v;
    }
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
__global__ __launch_bounds__(256) void k_applyq(const DevCtx* __restrict__ cp, OpArgs a) {
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
  constexpr int CW = BW;
  const int col0 = w * CW;
  if (col0 >= r) return;
  const int cw = min(CW, r - col0);
  if (dm[DL::qid + k - 1]) {  // identity: rt_k = 2 rt_{k-1}, same memory shape
    for (int e = t; e < m * cw; e += 256) {
      const int row = e / cw, qq = e % cw;
      M[(int64_t)row * r + col0 + qq] = US[(int64_t)row * r + col0 + qq];
    }
    return;
  }
  const double* S = E + L.off_q[k - 1];
  const double* T = E + L.off_qt[k - 1];
  const int nbk = (n + BW - 1) / BW;
  if ((int64_t)m * n > L.cap_q[k - 1] || (int64_t)nbk * BW * BW > L.cap_qt[k - 1]) {
    if (t == 0) raise_err(c, MPSW_DEV_ERR_CAP);
    return;
  }
  __shared__ double red[2 * 16 * 16];
  for (int e = t; e < m * cw; e += 256) {
    const int row = e / cw, qq = e % cw;
    M[(int64_t)row * r + col0 + qq] = (row < n) ? US[(int64_t)row * r + col0 + qq] : 0.0;
  }
  __syncthreads();
  for (int j = nbk - 1; j >= 0; --j) {
    const int r0 = j * BW, c0 = j * BW, bw = min(BW, n - c0);
    apply_reflector<BW>(S + r0 + (int64_t)m * c0, m, M + (int64_t)r0 * r + col0, r, 1, m - r0, bw, cw,
                        T + (int64_t)j * BW * BW, false, red);
  }
}

// ---------------------------------------------------------------------------
// Wide bond matrix: V_r (n x r) = Q1 [V'_r; 0] with the reflectors of M^T =
// Q1 R1; V'^T (r x m) comes from k_jacfin, core k (r x n) = V_r^T.
// Column chunks of BW per workgroup.
// ---------------------------------------------------------------------------
template <int BW>
__global__ __launch_bounds__(256) void k_applyv(const DevCtx* __restrict__ cp, OpArgs a) {
  const DevCtx& c = *cp;
  const int shot = blockIdx.z, w = blockIdx.x;
  const int k = a.site;
  const int* dm = shot_dims(c, shot);
  double* E = shot_eng(c, shot);
  const EngineLayout& L = c.L;
  const int m = dm[DL::rt + k], n = 2 * dm[DL::rho + k + 1], r = dm[DL::rho + k];
  if (m >= n) return;
  const int t = threadIdx.x;
  const int col0 = w * BW;
  if (col0 >= r) return;
  const int cw = min(BW, r - col0);
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
  __shared__ double red[2 * 16 * 16];
  for (int e = t; e < n * cw; e += 256) {
    const int row = e / cw, qq = e % cw;
    Y[(int64_t)row * r + col0 + qq] = (row < m) ? Vp[(int64_t)(col0 + qq) * m + row] : 0.0;
  }
  __syncthreads();
  for (int j = nbk - 1; j >= 0; --j) {
    const int r0 = j * BW, c0 = j * BW, bw = min(BW, m - c0);
    apply_reflector<BW>(S + r0 + (int64_t)n * c0, n, Y + (int64_t)r0 * r + col0, r, 1, n - r0, bw, cw,
                        T + (int64_t)j * BW * BW, false, red);
  }
  for (int e = t; e < n * cw; e += 256) {
    const int qq = e / n, row = e % n;
    core[(int64_t)(col0 + qq) * n + row] = Y[(int64_t)row * r + col0 + qq];
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
__global__ __launch_bounds__(512) void k_jac(const DevCtx* __restrict__ cp, OpArgs a, int b) {
  const DevCtx& c = *cp;
  const int shot = blockIdx.z, w = blockIdx.x, P = gridDim.x;
  const int k = a.site;
  const int* dm = shot_dims(c, shot);
  double* E = shot_eng(c, shot);
  const int m = dm[DL::rt + k], n = 2 * dm[DL::rho + k + 1];
  const int cc = (m >= n) ? n : m;
  const int Lc = cc;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, nwv = blockDim.x >> 6;
  const int nb = (cc + b - 1) / b;
  const int nbe = nb + (nb & 1);
  const int pact = nbe / 2;
  int* sy = shot_sync(c, shot);
  int epoch = 0;
  const bool ok = ((int64_t)Lc * cc <= c.L.cap_sA) && pact <= P;
  if (!ok && w == 0 && t == 0) raise_err(c, (pact > P) ? MPSW_DEV_ERR_GRID : MPSW_DEV_ERR_CAP);
  double* A = E + c.L.off_sA;
  extern __shared__ double blk[];   // 2b columns, stride ldl
  const int ldl = Lc + 1;
  __shared__ int nrot;
  const double tol = 1e-15 * sqrt((double)Lc);
  for (int sweep = 0; sweep < MPSW_MAX_SWEEPS; ++sweep) {
    for (int rnd = 0; rnd < nbe - 1; ++rnd) {
      if (ok && w < pact && cc > 1) {
        int bp, bq;
        if (w == 0) { bp = rnd; bq = nbe - 1; }
        else { bp = (rnd + w) % (nbe - 1); bq = (rnd - w + (nbe - 1)) % (nbe - 1); }
        if (bp >= nb) { const int tmp = bp; bp = bq; bq = tmp; }
        const int np_ = (bp < nb) ? min(b, cc - bp * b) : 0;
        const int nq_ = (bq < nb) ? min(b, cc - bq * b) : 0;
        const int ncol = np_ + nq_;
        if (t == 0) nrot = 0;
        // load
        for (int e = t; e < ncol * Lc; e += blockDim.x) {
          const int jj = e / Lc, i = e % Lc;
          const int gcol = (jj < np_) ? bp * b + jj : bq * b + (jj - np_);
          blk[jj * ldl + i] = A[(int64_t)gcol * Lc + i];
        }
        __syncthreads();
        // one cyclic pass over all column pairs of the loaded block pair
        const int npl = ncol + (ncol & 1);
        for (int ir = 0; ir < npl - 1; ++ir) {
          for (int pi = wv; pi < npl / 2; pi += nwv) {
            int p, q;
            if (pi == 0) { p = ir; q = npl - 1; }
            else { p = (ir + pi) % (npl - 1); q = (ir - pi + (npl - 1)) % (npl - 1); }
            if (p >= ncol || q >= ncol) continue;
            double* ap = blk + p * ldl;
            double* aq = blk + q * ldl;
            double al = 0.0, be = 0.0, ga = 0.0;
            for (int i = lane; i < Lc; i += 64) {
              const double x = ap[i], y = aq[i];
              al = fma(x, x, al);
              be = fma(y, y, be);
              ga = fma(x, y, ga);
            }
            al = wave_sum(al);
            be = wave_sum(be);
            ga = wave_sum(ga);
            if (al == 0.0 || be == 0.0 || fabs(ga) <= tol * sqrt(al) * sqrt(be)) continue;
            const double zeta = (be - al) / (2.0 * ga);
            double tt;
            if (fabs(zeta) > 1e100) tt = 0.5 / zeta;
            else tt = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
            for (int i = lane; i < Lc; i += 64) {
              const double x = ap[i], y = aq[i];
              ap[i] = cs * x - sn * y;
              aq[i] = sn * x + cs * y;
            }
            if (lane == 0) atomicAdd(&nrot, 1);
          }
          __syncthreads();
        }
        // store
        for (int e = t; e < ncol * Lc; e += blockDim.x) {
          const int jj = e / Lc, i = e % Lc;
          const int gcol = (jj < np_) ? bp * b + jj : bq * b + (jj - np_);
          A[(int64_t)gcol * Lc + i] = blk[jj * ldl + i];
        }
        if (t == 0 && nrot > 0) atomicAdd(sy + MPSW_SYNC_ROT + (sweep & 63), nrot);
      }
      shot_barrier(c, sy + MPSW_SYNC_BARRIER, P, epoch);
    }
    // every workgroup reads the same final count after the barrier
    const int rot = ld_acquire(sy + MPSW_SYNC_ROT + (sweep & 63));
    if (rot == 0 || !ok || cc <= 1) break;
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
  const int m = dm[DL::rt + k], n = 2 * dm[DL::rho + k + 1];
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
  for (int j = t; j < cc; j += blockDim.x) {
    const double sj = sig[j];
    int r = 0;
    for (int i = 0; i < cc; ++i) {
      const double si = sig[i];
      r += (si > sj) || (si == sj && i < j);
    }
    order[r] = j;
  }
  __syncthreads();
  if (t == 0) {
    const double s0 = sig[order[0]];
    const double eps = re[RL::eps];
    const int chi = dm[DL::chi];
    int r = 0;
    bool finite = true;
    for (int i = 0; i < cc; ++i) {
      const double s = sig[order[i]];
      if (!(s == s) || isinf(s)) finite = false;
      if (s0 > 0.0 && s >= eps * s0) ++r;
    }
    if (!finite) raise_err(c, MPSW_DEV_ERR_NONFINITE);
    if (r > chi) r = chi;
    if (r < 1) r = 1;
    double tail = 0.0;
    for (int i = r; i < cc; ++i) {
      const double s = sig[order[i]];
      tail = fma(s, s, tail);
    }
    if (a.aux >= 0 && a.aux < 3) {
      re[RL::tail2 + a.aux] += tail;
      double* lg = re + RL::sigma_log + (a.aux * MPSW_MAXK + k) * 32;
      for (int i = 0; i < 32; ++i) lg[i] = (i < cc) ? sig[order[i]] : 0.0;
      if (cc > dm[DL::maxbond + a.aux]) dm[DL::maxbond + a.aux] = cc;
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
  for (int64_t e = t; e < (int64_t)r * cc; e += blockDim.x) {
    const int i = (int)(e / cc), l = (int)(e % cc);
    const int j = order[i];
    const double s = sig[j];
    out[e] = (s > 0.0) ? A[(int64_t)j * Lc + l] / s : ((l == i) ? 1.0 : 0.0);
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
  if (bw == 16)
    hipLaunchKernelGGL(k_qrf<16>, dim3(nwg, 1, nshots), dim3(256), lds, s, d, a);
  else if (bw == 8)
    hipLaunchKernelGGL(k_qrf<8>, dim3(nwg, 1, nshots), dim3(256), lds, s, d, a);
  else
    hipLaunchKernelGGL(k_qrf<4>, dim3(nwg, 1, nshots), dim3(256), lds, s, d, a);
}

void launch_applyq(const DevCtx* d, const OpArgs& a, int bw, int nwg, int nshots, hipStream_t s) {
  if (bw == 16)
    hipLaunchKernelGGL(k_applyq<16>, dim3(nwg, 1, nshots), dim3(256), 0, s, d, a);
  else if (bw == 8)
    hipLaunchKernelGGL(k_applyq<8>, dim3(nwg, 1, nshots), dim3(256), 0, s, d, a);
  else
    hipLaunchKernelGGL(k_applyq<4>, dim3(nwg, 1, nshots), dim3(256), 0, s, d, a);
}

void launch_applyv(const DevCtx* d, const OpArgs& a, int bw, int nwg, int nshots, hipStream_t s) {
  if (bw == 16)
    hipLaunchKernelGGL(k_applyv<16>, dim3(nwg, 1, nshots), dim3(256), 0, s, d, a);
  else if (bw == 8)
    hipLaunchKernelGGL(k_applyv<8>, dim3(nwg, 1, nshots), dim3(256), 0, s, d, a);
  else
    hipLaunchKernelGGL(k_applyv<4>, dim3(nwg, 1, nshots), dim3(256), 0, s, d, a);
}

void launch_jac(const DevCtx* d, const OpArgs& a, int b, int nwg, int nshots, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL(k_jac, dim3(nwg, 1, nshots), dim3(512), lds, s, d, a, b);
}

void launch_jacfin(const DevCtx* d, const OpArgs& a, int nshots, hipStream_t s) {
  hipLaunchKernelGGL(k_jacfin, dim3(1, 1, nshots), dim3(256), 0, s, d, a);
}

void set_lds_limits(size_t bytes) {
  (void)hipFuncSetAttribute((const void*)k_qrf<16>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  (void)hipFuncSetAttribute((const void*)k_qrf<8>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  (void)hipFuncSetAttribute((const void*)k_qrf<4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  (void)hipFuncSetAttribute((const void*)k_jac, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace mpsw
