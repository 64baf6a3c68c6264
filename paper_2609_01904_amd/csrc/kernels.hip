// Device kernels of libmpsw (gfx950).
//
// Every kernel takes the group context (DevCtx, in device memory) and an OpArgs
// value.  Shapes are read from the per-shot dimension blocks, so all launches
// of a step are fixed and can be replayed without host involvement; blocks
// whose tile or batch entry lies beyond the live shape return immediately.
// Every write is checked against the capacity of its buffer; an overflow sets
// an error bit instead of writing.
#include "mpsw_device.h"

#include <math.h>

namespace mpsw {

// ---------------------------------------------------------------------------
// GEMM planning: one descriptor per (shot, batch entry)
// ---------------------------------------------------------------------------
struct GemmDesc {
  const double* A;
  const double* B;
  double* C;
  int M, N, K;
  int64_t ars, acs, brs, bcs, crs;
  int nbatch;
  int copy;     // C <- B (M x N), A unused
  int64_t capC; // capacity of the destination buffer from C onwards
  const double* hmul;  // if set, C[i][j] = (A B)[i][j] * hmul[i * hrs + j] (an elementwise factor)
  int64_t hrs;
};

__device__ __forceinline__ const double* mps_core(const DevCtx& c, int shot, int slot, int k) {
  return shot_mps(c, shot) + c.off_mps[slot][k];
}

// Fills d for shot/batch z; returns false when there is nothing to do.
__device__ bool plan_gemm(const DevCtx& c, const OpArgs& a, int shot, int z, int dz, GemmDesc& d) {
  const int* dm = shot_dims(c, shot);
  double* E = shot_eng(c, shot);
  const EngineLayout& L = c.L;
  const int k = a.site;
  const int K = c.K;
  d.copy = 0;
  d.nbatch = 1;
  d.hmul = nullptr;
  d.hrs = 0;
  switch (a.op) {
    case G_L2R_EXPLICIT: {  // X_k = R (rt_k x rin_k) * IN_k (rin_k x 2 rin_{k+1})
      const int rt = dm[DL::rt + k], r0 = dm[DL::rin + k], r1 = dm[DL::rin + k + 1];
      d.M = rt; d.K = r0; d.N = 2 * r1;
      d.A = E + L.off_R; d.ars = r0; d.acs = 1;
      d.B = E + L.off_in[k]; d.brs = 2 * r1; d.bcs = 1;
      if (a.aux == 1) { d.C = E + L.off_M; d.capC = L.cap_M; }  // last site feeds the SVD sweep
      else { d.C = E + L.off_X; d.capC = L.cap_X; }
      d.crs = d.N;
      if ((int64_t)r0 * 2 * r1 > L.cap_in[k] || (int64_t)rt * r0 > L.cap_R) { raise_err(c, MPSW_DEV_ERR_CAP); return false; }
      break;
    }
    case G_COPY_RX: {  // identity source: X_k = R_{k-1} viewed as (2 rt_k x rin_{k+1})
      const int rt = dm[DL::rt + k], r0 = dm[DL::rin + k];
      d.copy = 1; d.M = rt; d.N = r0; d.K = 0;
      d.B = E + L.off_R; d.brs = r0; d.bcs = 1;
      if (a.aux == 1) { d.C = E + L.off_M; d.capC = L.cap_M; }
      else { d.C = E + L.off_X; d.capC = L.cap_X; }
      d.crs = r0;
      if ((int64_t)rt * r0 > L.cap_R) { raise_err(c, MPSW_DEV_ERR_CAP); return false; }
      break;
    }
    case G_US: {  // U_r Sigma_r (rt_k x rho_k) = M_k (rt_k x 2rho_{k+1}) * core_k^T
      const int m = dm[DL::rt + k], nn = svd_cols(dm, k), r = dm[DL::rho + k];
      d.M = m; d.K = nn; d.N = r;
      d.A = E + L.off_M; d.ars = nn; d.acs = 1;
      d.B = mps_core(c, shot, a.slot, k); d.brs = 1; d.bcs = nn;
      d.C = E + L.off_US; d.crs = r; d.capC = L.cap_US;
      if ((int64_t)m * nn > L.cap_M || (int64_t)r * nn > c.cap_mps[a.slot][k]) { raise_err(c, MPSW_DEV_ERR_CAP); return false; }
      break;
    }
    // randomized range finder of the bond matrix M (rt_k x 2 rho_{k+1}, row-major
    // in M), sketch width l: Omega (rt x l), Y (2 rho x l), Z (rt x l), G (l x l)
    case G_RRF_Y: {  // Y = M^T Omega (aux 0) or M^T Z (aux 1)
      const int m = dm[DL::rt + k], nn = 2 * dm[DL::rho + k + 1], l = dm[DL::rrf_l];
      d.M = nn; d.K = m; d.N = l;
      d.A = E + L.off_M; d.ars = 1; d.acs = nn;
      d.B = E + (a.aux ? L.off_Zs : L.off_Om); d.brs = l; d.bcs = 1;
      d.C = E + L.off_Ys; d.crs = l; d.capC = L.cap_Ys;
      if ((int64_t)m * nn > L.cap_M || (int64_t)m * l > (a.aux ? L.cap_Zs : L.cap_Om)) { raise_err(c, MPSW_DEV_ERR_CAP); return false; }
      break;
    }
    case G_RRF_Z: {  // Z = M Q (Q = orthonormal Y)
      const int m = dm[DL::rt + k], nn = 2 * dm[DL::rho + k + 1], l = dm[DL::rrf_l];
      d.M = m; d.K = nn; d.N = l;
      d.A = E + L.off_M; d.ars = nn; d.acs = 1;
      d.B = E + L.off_Ys; d.brs = l; d.bcs = 1;
      d.C = E + L.off_Zs; d.crs = l; d.capC = L.cap_Zs;
      if ((int64_t)m * nn > L.cap_M || (int64_t)nn * l > L.cap_Ys) { raise_err(c, MPSW_DEV_ERR_CAP); return false; }
      break;
    }
    case G_RRF_CORE: {  // core (r x 2 rho) = core_small (r x l) Q^T; Q is 2 rho x l row-major
      const int nn = 2 * dm[DL::rho + k + 1], l = dm[DL::rrf_l], r = dm[DL::rho + k];
      d.M = r; d.K = l; d.N = nn;
      d.A = mps_core(c, shot, a.slot, k); d.ars = l; d.acs = 1;
      d.B = E + L.off_Ys; d.brs = 1; d.bcs = l;
      d.C = E + L.off_Tc; d.crs = nn; d.capC = L.cap_Tc;
      if ((int64_t)r * l > c.cap_mps[a.slot][k] || (int64_t)nn * l > L.cap_Ys) { raise_err(c, MPSW_DEV_ERR_CAP); return false; }
      break;
    }
    case G_RRF_RES: {  // Rz (rt x 2 rho) = B (rt x l) Q^T; B = M Q is in Zs, Q (2 rho x l) in Ys
      const int m = dm[DL::rt + k], nn = 2 * dm[DL::rho + k + 1], l = dm[DL::rrf_l];
      d.M = m; d.K = l; d.N = nn;
      d.A = E + L.off_Zs; d.ars = l; d.acs = 1;
      d.B = E + L.off_Ys; d.brs = 1; d.bcs = l;
      d.C = E + L.off_Rz; d.crs = nn; d.capC = L.cap_Rz;
      if ((int64_t)m * l > L.cap_Zs || (int64_t)nn * l > L.cap_Ys) { raise_err(c, MPSW_DEV_ERR_CAP); return false; }
      break;
    }
    // The Hadamard product C^2 . y formed in its middle unfolding: with n the
    // meeting site, (C^2 . y)[x, z] = c^2[x, z] y[x, z] for x the first n
    // sites and z the rest, and y[x, z] = (V_n W_n)[x, z] with V_n (2^n x chi_n)
    // and W_n (chi_n x 2^(K-n)) its two halves contracted.
    case G_HALF_L: {  // V_{k+1} (2^k x 2 chi_{k+1}) = V_k (2^k x chi_k) * Y_k (chi_k x 2 chi_{k+1}), k < n
      const int ck = dm[DL::bonds + MPSW_SLOT_Y * (MPSW_MAXK + 1) + k];
      const int c1 = dm[DL::bonds + MPSW_SLOT_Y * (MPSW_MAXK + 1) + k + 1];
      const int64_t rows = mpsw_pow2(k);
      d.M = (int)rows; d.K = ck; d.N = 2 * c1;
      d.A = E + ((k & 1) ? L.off_VL1 : L.off_VL0); d.ars = ck; d.acs = 1;
      d.B = mps_core(c, shot, MPSW_SLOT_Y, k); d.brs = 2 * c1; d.bcs = 1;
      d.C = E + ((k & 1) ? L.off_VL0 : L.off_VL1); d.crs = 2 * c1; d.capC = L.cap_VL;
      if (rows * ck > L.cap_VL) { raise_err(c, MPSW_DEV_ERR_CAP); return false; }
      break;
    }
    case G_HALF_R: {  // W_k (2 chi_k x 2^(K-k-1)) = Y_k (2 chi_k x chi_{k+1}) * W_{k+1} (chi_{k+1} x 2^(K-k-1)), k >= n
      const int ck = dm[DL::bonds + MPSW_SLOT_Y * (MPSW_MAXK + 1) + k];
      const int c1 = dm[DL::bonds + MPSW_SLOT_Y * (MPSW_MAXK + 1) + k + 1];
      const int q = (int)mpsw_pow2(K - k - 1);
      const bool in1 = ((K - k - 1) & 1) != 0;
      d.M = 2 * ck; d.K = c1; d.N = q;
      d.A = mps_core(c, shot, MPSW_SLOT_Y, k); d.ars = c1; d.acs = 1;
      d.B = E + (in1 ? L.off_WR1 : L.off_WR0); d.brs = q; d.bcs = 1;
      d.C = E + (in1 ? L.off_WR0 : L.off_WR1); d.crs = q; d.capC = L.cap_WR;
      if ((int64_t)c1 * q > L.cap_WR) { raise_err(c, MPSW_DEV_ERR_CAP); return false; }
      break;
    }
    case G_MEET_H: {  // X2 (2^n x 2^(K-n)) = (V_n W_n) .* c^2, at site n-1 = k
      const int n = k + 1;
      const int cn = dm[DL::bonds + MPSW_SLOT_Y * (MPSW_MAXK + 1) + n];
      const int64_t rows = mpsw_pow2(n), q = mpsw_pow2(K - n);
      d.M = (int)rows; d.K = cn; d.N = (int)q;
      d.A = E + ((n & 1) ? L.off_VL1 : L.off_VL0); d.ars = cn; d.acs = 1;
      d.B = E + (((K - n) & 1) ? L.off_WR1 : L.off_WR0); d.brs = q; d.bcs = 1;
      d.C = E + L.off_X2; d.crs = q; d.capC = L.cap_X2;
      d.hmul = c.c2d; d.hrs = q;
      if (rows * cn > L.cap_VL || (int64_t)cn * q > L.cap_WR || c.c2d == nullptr) { raise_err(c, MPSW_DEV_ERR_CAP); return false; }
      break;
    }
    case G_DENSE: {  // V_{k+1} (2^k x 2 r_{k+1}) = V_k (2^k x r_k) * G_k (r_k x 2 r_{k+1})
      int r0, r1;
      const double* G;
      if (a.slot < 0) { r0 = c.c2b[k]; r1 = c.c2b[k + 1]; G = c.c2 + c.off_c2[k]; }
      else {
        r0 = dm[DL::bonds + a.slot * (MPSW_MAXK + 1) + k];
        r1 = dm[DL::bonds + a.slot * (MPSW_MAXK + 1) + k + 1];
        G = mps_core(c, shot, a.slot, k);
      }
      const int64_t rows = mpsw_pow2(k);
      double* D = c.dense + (int64_t)dz * c.dense_stride;
      const int64_t half = c.dense_stride / 2;
      d.M = (int)rows; d.K = r0; d.N = 2 * r1;
      d.A = D + ((k & 1) ? half : 0); d.ars = r0; d.acs = 1;
      d.B = G; d.brs = 2 * r1; d.bcs = 1;
      d.C = D + ((k & 1) ? 0 : half); d.crs = 2 * r1; d.capC = half;
      if (rows * r0 > half) { raise_err(c, MPSW_DEV_ERR_CAP); return false; }
      break;
    }
    default:
      return false;
  }
  if (d.M <= 0 || d.N <= 0) return false;
  if ((int64_t)(d.M - 1) * d.crs + d.N > d.capC) { raise_err(c, MPSW_DEV_ERR_CAP); return false; }
  return true;
}

// C = A * B on the matrix cores: TS x TS output tiles per 256-thread
// workgroup (TS = 64), each wave a quarter (2 x 2 tiles of 16 x 16); K in
// slices of KS = 16 staged through two LDS buffers as FP64, the next slice's
// global loads in flight while the current one is multiplied.  Lane layouts (checked on the
// device): f64 16x16x4 and f32 16x16x4 take a = A[l%16][l/16], b = B[l/16][l%16];
// bf16 16x16x16 takes a[q] = A[l%16][4(l/16)+q], b[q] = B[4(l/16)+q][l%16];
// results are D[l/16 + 4v][l%16] (f64) and D[4(l/16) + v][l%16] (f32 accumulators).
// In the FP32 and BF16 modes each slice's FP32 sums are added into FP64
// accumulators, so the FP32 rounding of long sums is confined to 16 terms.
typedef double gd4 __attribute__((ext_vector_type(4)));
typedef float gf4 __attribute__((ext_vector_type(4)));
typedef short gs4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_rne(float x) {   // round to nearest even (finite x)
  const unsigned u = __float_as_uint(x);
  return (short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_val(short h) { return __uint_as_float(((unsigned)(unsigned short)h) << 16); }

template <int MODE, int TS, int KS>
__global__ __launch_bounds__(256, (MODE == GEMM_FP64) ? 4 : 2) void k_gemm(const DevCtx* __restrict__ cp, OpArgs a) {
  static_assert(TS == 64 || (TS == 128 && MODE == GEMM_FP64), "128-wide tiles are FP64 only");
  static_assert(KS == 16 || (KS == 32 && MODE == GEMM_FP64), "FP32 sums cover 16-deep slices");
  constexpr int EU = TS * KS / 256;   // elements of each slice per thread
  constexpr int NTL = TS / 32;  // 16 x 16 tiles per wave and dimension
  const DevCtx& c = *cp;
  const int shot = (a.shot >= 0) ? a.shot : (int)blockIdx.z, z = blockIdx.y;
  if (!gate_open(shot_dims(c, shot), a.gate)) return;
  GemmDesc d;
  if (!plan_gemm(c, a, shot, z, blockIdx.z, d)) return;
  if (z == 0 && blockIdx.x == 0 && threadIdx.x == 0 && d.nbatch > (int)gridDim.y) raise_err(c, MPSW_DEV_ERR_GRID);
  const int tn = (d.N + TS - 1) / TS, tm = (d.M + TS - 1) / TS;
  if (blockIdx.x == 0 && threadIdx.x == 0 && (int64_t)tm * tn > (int64_t)gridDim.x) raise_err(c, MPSW_DEV_ERR_GRID);
  if (blockIdx.x == 0 && threadIdx.x == 0 && !d.copy) count_flops(c, shot, MPSW_KC_GEMM, 2.0 * d.M * d.N * d.K);
  if ((int)blockIdx.x >= tm * tn) return;
  const int m0 = (blockIdx.x / tn) * TS, n0 = (blockIdx.x % tn) * TS;
  const int t = threadIdx.x;

  if (d.copy) {
    for (int e = t; e < TS * TS; e += 256) {
      const int i = m0 + e / TS, j = n0 + e % TS;
      if (i < d.M && j < d.N) d.C[(int64_t)i * d.crs + j] = d.B[(int64_t)i * d.brs + (int64_t)j * d.bcs];
    }
    return;
  }

  __shared__ double As[2][KS][TS + 2];   // two buffers: slice i is multiplied
  __shared__ double Bs[2][KS][TS + 2];   // while slice i + 1 is stored
  const bool a_k_fast = (d.acs == 1);
  const bool b_n_fast = (d.bcs == 1);
  // element u (0..EU-1) of this thread's share of the A and B slices
  auto a_idx = [&](int u, int& mm, int& kk) {
    const int e = t + 256 * u;
    if (a_k_fast) { kk = e % KS; mm = e / KS; } else { mm = e % TS; kk = e / TS; }
  };
  auto b_idx = [&](int u, int& nn, int& kk) {
    const int e = t + 256 * u;
    if (b_n_fast) { nn = e % TS; kk = e / TS; } else { kk = e % KS; nn = e / KS; }
  };
  double ra[EU], rb[EU];
  // per element: offset of its k = 0 entry (every operand spans fewer than
  // 2^31 elements) or -1 outside the tile's rows/columns, and its k within a
  // slice; a slice at k0 adds k0 times the k stride
  int aoff[EU], boff[EU], akk[EU], bkk[EU];
#pragma unroll
  for (int u = 0; u < EU; ++u) {
    int mm, kk, nn, kb;
    a_idx(u, mm, kk);
    b_idx(u, nn, kb);
    const int gi = m0 + mm, gj = n0 + nn;
    aoff[u] = (gi < d.M) ? (int)((int64_t)gi * d.ars + (int64_t)kk * d.acs) : -1;
    boff[u] = (gj < d.N) ? (int)((int64_t)kb * d.brs + (int64_t)gj * d.bcs) : -1;
    akk[u] = kk;
    bkk[u] = kb;
  }
  const int acs = (int)d.acs, brs = (int)d.brs;
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < EU; ++u) {
      ra[u] = (aoff[u] >= 0 && k0 + akk[u] < d.K) ? d.A[aoff[u] + k0 * acs] : 0.0;
      rb[u] = (boff[u] >= 0 && k0 + bkk[u] < d.K) ? d.B[boff[u] + k0 * brs] : 0.0;
    }
  };
  const int l = t & 63, w = t >> 6, li = l & 15, lq = l >> 4;
  const int wm = (w >> 1) * (TS / 2), wn = (w & 1) * (TS / 2);
  gd4 acc64[NTL][NTL];
  gf4 acc32[NTL][NTL];
#pragma unroll
  for (int i = 0; i < NTL; ++i)
#pragma unroll
    for (int j = 0; j < NTL; ++j) {
      acc64[i][j] = gd4{0.0, 0.0, 0.0, 0.0};
      acc32[i][j] = gf4{0.0f, 0.0f, 0.0f, 0.0f};
    }
  auto stash = [&](int buf) {
#pragma unroll
    for (int u = 0; u < EU; ++u) {
      int mm, kk, nn, kb;
      a_idx(u, mm, kk);
      b_idx(u, nn, kb);
      As[buf][kk][mm] = ra[u];
      Bs[buf][kb][nn] = rb[u];
    }
  };
  fetch(0);
  stash(0);
  __syncthreads();
  for (int k0 = 0, cur = 0; k0 < d.K; k0 += KS, cur ^= 1) {
    // one barrier per slice: the buffer written here was last read before
    // the previous barrier
    const bool more = (k0 + KS < d.K);
    if (more) fetch(k0 + KS);   // next slice in flight during the products
    if (MODE == GEMM_FP64 || MODE == GEMM_FP32) {
#pragma unroll
      for (int ks = 0; ks < KS / 4; ++ks) {
        const int kr = 4 * ks + lq;
#pragma unroll
        for (int i = 0; i < NTL; ++i)
#pragma unroll
          for (int j = 0; j < NTL; ++j) {
            const double av = As[cur][kr][wm + 16 * i + li], bv = Bs[cur][kr][wn + 16 * j + li];
            if (MODE == GEMM_FP64)
              acc64[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc64[i][j], 0, 0, 0);
            else
              acc32[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)av, (float)bv, acc32[i][j], 0, 0, 0);
          }
      }
    } else {   // BF16 x 6: three BF16 parts per operand, six of the nine partial products
      gs4 ap[3][NTL], bp[3][NTL];
#pragma unroll
      for (int i = 0; i < NTL; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float x = (float)As[cur][4 * lq + q][wm + 16 * i + li];
          float y = (float)Bs[cur][4 * lq + q][wn + 16 * i + li];
#pragma unroll
          for (int p = 0; p < 3; ++p) {
            const short hx = bf16_rne(x), hy = bf16_rne(y);
            ap[p][i][q] = hx;
            bp[p][i][q] = hy;
            x -= bf16_val(hx);
            y -= bf16_val(hy);
          }
        }
      // smallest terms first: lo.hi, hi.lo (2^-18), mid.mid, mid.hi, hi.mid (2^-9), hi.hi;
      // the dropped mid.lo, lo.mid, lo.lo are below 2^-26 of the product
#pragma unroll
      for (int i = 0; i < NTL; ++i)
#pragma unroll
        for (int j = 0; j < NTL; ++j) {
          acc32[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ap[2][i], bp[0][j], acc32[i][j], 0, 0, 0);
          acc32[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ap[0][i], bp[2][j], acc32[i][j], 0, 0, 0);
          acc32[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ap[1][i], bp[1][j], acc32[i][j], 0, 0, 0);
          acc32[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ap[1][i], bp[0][j], acc32[i][j], 0, 0, 0);
          acc32[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ap[0][i], bp[1][j], acc32[i][j], 0, 0, 0);
          acc32[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ap[0][i], bp[0][j], acc32[i][j], 0, 0, 0);
        }
    }
    if (MODE != GEMM_FP64) {   // FP32 sums of one 16-deep slice, accumulated across slices in FP64
#pragma unroll
      for (int i = 0; i < NTL; ++i)
#pragma unroll
        for (int j = 0; j < NTL; ++j) {
#pragma unroll
          for (int v = 0; v < 4; ++v) acc64[i][j][v] += (double)acc32[i][j][v];
          acc32[i][j] = gf4{0.0f, 0.0f, 0.0f, 0.0f};
        }
    }
    if (more) stash(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < NTL; ++i)
#pragma unroll
    for (int j = 0; j < NTL; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = m0 + wm + 16 * i + ((MODE == GEMM_FP64) ? (lq + 4 * v) : (4 * lq + v));
        const int gj = n0 + wn + 16 * j + li;
        if (gi < d.M && gj < d.N)
          d.C[(int64_t)gi * d.crs + gj] = d.hmul ? acc64[i][j][v] * d.hmul[(int64_t)gi * d.hrs + gj] : acc64[i][j][v];
      }
}

// ---------------------------------------------------------------------------
// Prepare a rounding: input bonds, sweep start values.
// ---------------------------------------------------------------------------
__global__ void k_prepare(const DevCtx* __restrict__ cp, OpArgs a) {
  const DevCtx& c = *cp;
  const int shot = blockIdx.x * blockDim.x + threadIdx.x;
  if (shot >= c.B) return;
  int* dm = shot_dims(c, shot);
  const int K = c.K, n = c.half;   // the Kronecker rounding's sweeps meet at site n
  const int* bonds = dm + DL::bonds;
  auto B = [&](int slot, int k) { return bonds[slot * (MPSW_MAXK + 1) + k]; };
  for (int k = 0; k <= K; ++k) {
    int r;
    switch (a.op) {
      case P_LAPLACE: r = c.wb[k] * B(a.slot, k); break;
      // the Hadamard product is formed in its middle unfolding: the left half
      // is held in the identity basis (bond 2^k), the right half densely
      case P_C2: r = (k < n) ? (int)mpsw_pow2(k) : (int)mpsw_pow2(K - k); break;
      case P_SUM:
        r = (k == 0 || k == K) ? 1 : B(a.slot, k) + B(a.slot2, k) + B(MPSW_SLOT_W, k) + 1;
        break;
      default: r = (int)mpsw_pow2(K - k); break;  // dense input
    }
    dm[DL::rin + k] = r;
  }
  dm[DL::rt + 0] = 1;
  dm[DL::rho + K] = 1;
  if (a.op == P_C2)   // sites 0..n-2 merge without a factorisation: Q_k = I, rt_{k+1} = 2 rt_k
    for (int k = 0; k + 1 < n; ++k) {
      dm[DL::rt + k + 1] = (int)mpsw_pow2(k + 1);
      dm[DL::qid + k] = 1;
    }
  if (a.aux >= 0 && a.aux < 3) {
    shot_reals(c, shot)[RL::tail2 + a.aux] = 0.0;
    dm[DL::maxbond + a.aux] = 0;
  }
}

// Initial R: R_0 = [1], or the dense tensor (1 x 2^K) for a dense input.
__global__ void k_init_R(const DevCtx* __restrict__ cp, OpArgs a) {
  const DevCtx& c = *cp;
  const int shot = blockIdx.y;
  double* R = shot_eng(c, shot) + c.L.off_R;
  if (a.op == P_C2 && blockIdx.x == 0 && threadIdx.x == 0) {   // V_0 = W_K = [1]
    shot_eng(c, shot)[c.L.off_VL0] = 1.0;
    shot_eng(c, shot)[c.L.off_WR0] = 1.0;
  }
  if (a.op == P_DENSE) {
    const int64_t total = mpsw_pow2(c.K);
    if (total > c.L.cap_R || total > c.dense_stride) { if (threadIdx.x == 0 && blockIdx.x == 0) raise_err(c, MPSW_DEV_ERR_CAP); return; }
    const double* src = c.dense + (int64_t)shot * c.dense_stride;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
      R[e] = src[e];
  } else if (blockIdx.x == 0 && threadIdx.x == 0) {
    R[0] = 1.0;
  }
}

// ---------------------------------------------------------------------------
// Laplacian MPO applied to psi: IN_k[(al,i), s', (be,j)] = sum_s W_k[al,be,s',s] G_k[i,s,j]
// ---------------------------------------------------------------------------
__global__ void k_pack_lap(const DevCtx* __restrict__ cp, OpArgs a) {
  const DevCtx& c = *cp;
  const int k = blockIdx.y, shot = blockIdx.z;
  const int* dm = shot_dims(c, shot);
  const int c0 = dm[DL::bonds + a.slot * (MPSW_MAXK + 1) + k];
  const int c1 = dm[DL::bonds + a.slot * (MPSW_MAXK + 1) + k + 1];
  const int w0 = c.wb[k], w1 = c.wb[k + 1];
  const int r0 = w0 * c0, r1 = w1 * c1;
  const int64_t total = (int64_t)r0 * 2 * r1;
  if (total > c.L.cap_in[k]) { if (blockIdx.x == 0 && threadIdx.x == 0) raise_err(c, MPSW_DEV_ERR_CAP); return; }
  const double* G = mps_core(c, shot, a.slot, k);
  const double* W = c.lapW + c.off_W[k];
  double* out = shot_eng(c, shot) + c.L.off_in[k];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int col = (int)(e % r1);
    const int sp = (int)((e / r1) & 1);
    const int row = (int)(e / (2 * (int64_t)r1));
    const int al = row / c0, i = row - al * c0;
    const int be = col / c1, j = col - be * c1;
    const double* w = W + ((al * w1 + be) * 2 + sp) * 2;
    const double g0 = G[((int64_t)i * 2 + 0) * c1 + j];
    const double g1 = G[((int64_t)i * 2 + 1) * c1 + j];
    out[e] = w[0] * g0 + w[1] * g1;
  }
}

// ---------------------------------------------------------------------------
// Direct sum 2 psi^k - psi^{k-1} + lambda^2 w + s_k e_src (block cores)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double sum_term(const DevCtx& c, int shot, int slot, int k, int i, int s, int j,
                                           int r0, int r1) {
  (void)r0;
  return mps_core(c, shot, slot, k)[((int64_t)i * 2 + s) * r1 + j];
}

__global__ void k_pack_sum(const DevCtx* __restrict__ cp, OpArgs a) {
  const DevCtx& c = *cp;
  const int k = blockIdx.y, shot = blockIdx.z;
  const int K = c.K, n = c.n;
  const int* dm = shot_dims(c, shot);
  const int slots[3] = {a.slot, a.slot2, MPSW_SLOT_W};
  int b0[3], b1[3];
  for (int t = 0; t < 3; ++t) {
    b0[t] = dm[DL::bonds + slots[t] * (MPSW_MAXK + 1) + k];
    b1[t] = dm[DL::bonds + slots[t] * (MPSW_MAXK + 1) + k + 1];
  }
  const int r0 = dm[DL::rin + k], r1 = dm[DL::rin + k + 1];
  const int64_t total = (int64_t)r0 * 2 * r1;
  if (total > c.L.cap_in[k]) { if (blockIdx.x == 0 && threadIdx.x == 0) raise_err(c, MPSW_DEV_ERR_CAP); return; }
  // source coefficient and bit
  double ssrc = 0.0;
  const int nt = dm[DL::src_nt];
  // the step index lives on the device, so a captured step replays correctly
  const int stp = dm[DL::step];
  if (stp >= 0 && stp < nt && stp < c.nt_max) ssrc = c.wavelet[(int64_t)shot * c.nt_max + stp];
  // site k holds bit b of axis r: registers in order (sequential) or bits of
  // equal significance side by side (interleaved); the last axis is z
  const int nd = c.ndim;
  const int r = (c.ordering == MPSW_INTERLEAVED) ? k % nd : k / n;
  const int b = (c.ordering == MPSW_INTERLEAVED) ? n - 1 - k / nd : n - 1 - k % n;
  const int coord = (r == 0) ? dm[DL::src_ix] : (r == nd - 1) ? dm[DL::src_iz] : dm[DL::src_iy];
  const int bit = (coord >> b) & 1;
  const double coef[3] = {2.0, -1.0, c.lam2};
  double* out = shot_eng(c, shot) + c.L.off_in[k];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int col = (int)(e % r1);
    const int s = (int)((e / r1) & 1);
    const int row = (int)(e / (2 * (int64_t)r1));
    double v = 0.0;
    if (k == 0) {            // concatenate along the right bond, coefficients here
      int off = 0, t = 0;
      for (; t < 3; ++t) { if (col < off + b1[t]) break; off += b1[t]; }
      if (t < 3) v = coef[t] * sum_term(c, shot, slots[t], k, 0, s, col - off, b0[t], b1[t]);
      else v = (s == bit) ? ssrc : 0.0;
    } else if (k == K - 1) { // stack along the left bond
      int off = 0, t = 0;
      for (; t < 3; ++t) { if (row < off + b0[t]) break; off += b0[t]; }
      if (t < 3) v = sum_term(c, shot, slots[t], k, row - off, s, 0, b0[t], b1[t]);
      else v = (s == bit) ? 1.0 : 0.0;
    } else {                 // block diagonal
      int ro = 0, co = 0, t = 0;
      for (; t < 3; ++t) {
        if (row < ro + b0[t]) break;
        ro += b0[t];
        co += b1[t];
      }
      if (t < 3) {
        if (col >= co && col < co + b1[t]) v = sum_term(c, shot, slots[t], k, row - ro, s, col - co, b0[t], b1[t]);
      } else {
        if (col == co) v = (s == bit) ? 1.0 : 0.0;
      }
    }
    out[e] = v;
  }
}

// Core 0 of the rounded state and its bonds.
__global__ void k_finish(const DevCtx* __restrict__ cp, OpArgs a) {
  const DevCtx& c = *cp;
  const int shot = blockIdx.z;
  int* dm = shot_dims(c, shot);
  const int r1 = dm[DL::rho + 1];
  const double* M = shot_eng(c, shot) + c.L.off_M;
  double* out = shot_mps(c, shot) + c.off_mps[a.slot][0];
  if ((int64_t)2 * r1 > c.cap_mps[a.slot][0]) { if (threadIdx.x == 0) raise_err(c, MPSW_DEV_ERR_CAP); return; }
  for (int e = threadIdx.x; e < 2 * r1; e += blockDim.x) out[e] = M[e];
  __syncthreads();
  if (threadIdx.x == 0) {
    int* b = dm + DL::bonds + a.slot * (MPSW_MAXK + 1);
    b[0] = 1;
    for (int k = 1; k < c.K; ++k) b[k] = dm[DL::rho + k];
    b[c.K] = 1;
    if (a.aux == 1) dm[DL::step] += 1;   // last rounding of a time step
  }
}

// V_0 = [1] for to_dense.
__global__ void k_dense_init(const DevCtx* __restrict__ cp) {
  const DevCtx& c = *cp;
  const int shot = blockIdx.x;
  if (threadIdx.x == 0) c.dense[(int64_t)shot * c.dense_stride] = 1.0;
}

// Zero state (bond 1, zero cores) in a slot.
__global__ void k_zero_state(const DevCtx* __restrict__ cp, OpArgs a) {
  const DevCtx& c = *cp;
  const int shot = blockIdx.x;
  if (a.shot >= 0 && shot != a.shot) return;
  int* b = shot_dims(c, shot) + DL::bonds + a.slot * (MPSW_MAXK + 1);
  for (int k = threadIdx.x; k < c.K; k += blockDim.x) {
    double* core = shot_mps(c, shot) + c.off_mps[a.slot][k];
    core[0] = 0.0;
    core[1] = 0.0;
  }
  for (int k = threadIdx.x; k <= c.K; k += blockDim.x) b[k] = 1;
}

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------
void launch_gemm(const DevCtx* d, const OpArgs& a, int64_t mcap, int64_t ncap, int grid_batch, int nshots, hipStream_t s) {
  if (grid_batch <= 0) return;
  const int64_t nt = std::max<int64_t>(1, ((mcap + 63) / 64) * ((ncap + 63) / 64));
  const dim3 g((unsigned)nt, grid_batch, nshots);
  if (a.mode == GEMM_FP32) hipLaunchKernelGGL((k_gemm<GEMM_FP32, 64, 16>), g, dim3(256), 0, s, d, a);
  else if (a.mode == GEMM_BF16X6) hipLaunchKernelGGL((k_gemm<GEMM_BF16X6, 64, 16>), g, dim3(256), 0, s, d, a);
  else hipLaunchKernelGGL((k_gemm<GEMM_FP64, 64, 16>), g, dim3(256), 0, s, d, a);
}
void launch_prepare(const DevCtx* d, const OpArgs& a, int nshots, hipStream_t s) {
  hipLaunchKernelGGL(k_prepare, dim3((nshots + 63) / 64), dim3(64), 0, s, d, a);
}
void launch_init_R(const DevCtx* d, const OpArgs& a, int nshots, hipStream_t s) {
  hipLaunchKernelGGL(k_init_R, dim3(a.op == P_DENSE ? 256 : 1, nshots), dim3(256), 0, s, d, a);
}
void launch_pack_lap(const DevCtx* d, const OpArgs& a, int K, int nshots, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_lap, dim3(blocks, K, nshots), dim3(256), 0, s, d, a);
}
void launch_pack_sum(const DevCtx* d, const OpArgs& a, int K, int nshots, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_sum, dim3(blocks, K, nshots), dim3(256), 0, s, d, a);
}
void launch_finish(const DevCtx* d, const OpArgs& a, int nshots, hipStream_t s) {
  hipLaunchKernelGGL(k_finish, dim3(1, 1, nshots), dim3(256), 0, s, d, a);
}
void launch_dense_init(const DevCtx* d, int nshots, hipStream_t s) {
  hipLaunchKernelGGL(k_dense_init, dim3(nshots), dim3(64), 0, s, d);
}
void launch_zero_state(const DevCtx* d, const OpArgs& a, int nshots, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_state, dim3(nshots), dim3(64), 0, s, d, a);
}

}  // namespace mpsw
