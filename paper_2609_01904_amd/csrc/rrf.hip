// Learned-rank rounding of libmpsw: the network proposes a rank for each bond
// of the SVD sweep, a randomized range finder (Halko, Martinsson and Tropp
// 2011, one power iteration) sketches the bond matrix at that width, the SVD
// stage runs on the sketch, and a FP64 residual test accepts the result or
// restores the bond matrix for the exact SVD.
//
// Sketch of the row space of M (rt x 2 rho): Y = M^T Omega, Q_Y = orth(Y),
// Z = M Q_Y, Q_Z = orth(Z), Y = M^T Q_Z, Q = orth(Y), B = M Q (rt x l).  The
// SVD of B = U S W^T gives M ~ U S (Q W)^T; the core is W_r^T Q^T and
// U_r S_r = B W_r.
//
// Acceptance, with sigma-hat the singular values of B (all <= those of M),
// res2 = ||M - B Q^T||_F^2 the energy outside the sketch (formed in FP64 from
// M and the sketch, not as ||M||^2 - ||B||^2, whose rounding noise of about
// 1e-16 ||M||^2 would swamp (eps sigma_1)^2 at small eps), r the rank the
// truncation rule keeps from sigma-hat:
//   rank below the cap: r < l and res2 <= (eps sigma-hat_1)^2, so everything
//     the sketch missed lies below the cutoff (the Frobenius norm bounds the
//     spectral one, so this is at least as strict as a spectral-norm test);
//   rank at the cap: res2 <= 0.21 T with T the in-sketch tail beyond the cap;
//     the kept error T + res2 is then within 1.1 of the optimal one, which is
//     at least T.
// The Gaussian test matrix comes from a counter-based generator: entry (i, j)
// of the sketch of bond k in rounding j' at step t hashes the key
// ((((t * 3 + j') * 64 + k) * 4096 + i) * 1024 + j) with SplitMix64 (Steele,
// Lea and Flood 2014) into two uniforms and a Box-Muller normal.
#include "mpsw_device.h"

#include <math.h>

#include <algorithm>

namespace mpsw {

__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__device__ __forceinline__ double sketch_normal(unsigned long long seed, int step, int rnd, int site, int i, int j) {
  const unsigned long long key =
      (((((unsigned long long)step * 3ull + (unsigned long long)rnd) * 64ull + (unsigned long long)site) * 4096ull +
        (unsigned long long)i) * 1024ull + (unsigned long long)j);
  const double u1 = (double)((splitmix64(seed ^ (2ull * key)) >> 11) + 1ull) * 0x1.0p-53;   // (0, 1]
  const double u2 = (double)(splitmix64(seed ^ (2ull * key + 1ull)) >> 11) * 0x1.0p-53;     // [0, 1)
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// Network input of bond k of rounding rnd for the coming step, thread j < 34
// writes x[j]: log10(sigma_i / sigma_1) of the bond's leading singular values
// at the previous step (-30 where absent or zero), k / K, min(step, 10^4) / 1000.
__device__ __forceinline__ void rank_features(const DevCtx& c, const int* dm, const double* re, int rnd, int k,
                                              float* x, int j) {
  const double* lg = re + RL::sigma_log + (rnd * MPSW_MAXK + k) * 32;
  if (j < 32) x[j] = (lg[0] > 0.0 && lg[j] > 0.0) ? (float)fmax(log10(lg[j] / lg[0]), -30.0) : -30.0f;
  if (j == 32) x[32] = (float)k / (float)c.K;
  if (j == 33) x[33] = (float)min(dm[DL::step], 10000) / 1000.0f;
}

// The network (34 -> 128 -> 128 -> 1, ReLU) on x by MLP_NH threads; the
// output is valid in thread 0.  h1, h2: MLP_NH floats of LDS each.
__device__ __forceinline__ float rank_net(const float* __restrict__ W, const float* x, float* h1, float* h2, int j) {
  float z = W[MLP_NIN * MLP_NH + j];
  for (int i = 0; i < MLP_NIN; ++i) z = fmaf(x[i], W[i * MLP_NH + j], z);
  h1[j] = fmaxf(z, 0.0f);
  __syncthreads();
  const int ow2 = MLP_NIN * MLP_NH + MLP_NH, ob2 = ow2 + MLP_NH * MLP_NH, ow3 = ob2 + MLP_NH;
  z = W[ob2 + j];
  for (int i = 0; i < MLP_NH; ++i) z = fmaf(h1[i], W[ow2 + i * MLP_NH + j], z);
  h2[j] = fmaxf(z, 0.0f) * W[ow3 + j];
  __syncthreads();
  float o = 0.0f;
  if (j == 0) {
    o = W[ow3 + MLP_NH];
    for (int i = 0; i < MLP_NH; ++i) o += h2[i];
  }
  return o;
}

// The rank the network proposes for output o: ceil(o chi), clamped to [1, chi].
__device__ __forceinline__ int rank_of(float o, int chi) { return max(1, min(chi, (int)ceilf(o * (float)chi))); }

// Per shot: features of the bond from the previous step's sigma log, the
// network's rank, the sketch width.  a.aux = rounding index.
__global__ __launch_bounds__(MLP_NH) void k_rrf_plan(const DevCtx* __restrict__ cp, OpArgs a) {
  const DevCtx& c = *cp;
  const int shot = blockIdx.z, k = a.site, j = threadIdx.x;
  int* dm = shot_dims(c, shot);
  const double* re = shot_reals(c, shot);
  __shared__ float x[MLP_NIN], h1[MLP_NH], h2[MLP_NH];
  const int m = dm[DL::rt + k], nn = 2 * dm[DL::rho + k + 1], cc = min(m, nn);
  const int chi = dm[DL::chi];
  const double* lg = re + RL::sigma_log + (a.aux * MPSW_MAXK + k) * 32;
  rank_features(c, dm, re, a.aux, k, x, j);
  __syncthreads();
  // the network's rank, or (baseline mode, no network) the rank this bond
  // kept in this rounding at the previous step
  const float o = c.rank_prev ? 0.0f : rank_net(c.mlp_w, x, h1, h2, j);
  if (j == 0) {
    // (0 in baseline mode while the bond has no rank of a previous step: no sketch)
    const int rhat = c.rank_prev ? dm[DL::prank + a.aux * MPSW_MAXK + k] : rank_of(o, chi);
    const int l = rhat + c.rrf_over;
    // a sketch pays off only well below the full width and below the cap (a
    // capped bond's flat tail rarely lets the residual test certify the
    // capped error), and needs a sigma log
    const bool waiting = (a.aux >= 0 && a.aux < 3) && dm[DL::step] < dm[DL::rrf_skip + a.aux * MPSW_MAXK + k];
    const int ok = (lg[0] > 0.0) && (rhat >= 1) && (rhat < chi) && (l <= MPSW_RRF_MAXL) && (4 * l <= 3 * cc) && m >= l && nn >= l &&
                   !waiting;
    dm[DL::rrf] = ok ? 1 : 0;
    dm[DL::rrf_l] = ok ? l : 0;
    dm[DL::svd_n] = 0;
    if (ok) dm[DL::rrf_tries] += 1;
  }
}

// For one shot and rounding, every bond k = 1..K-1 (block k): the network's
// input, output and proposed rank, exactly as k_rrf_plan forms them at the
// coming step (outs and rhat only when a network is installed).
__global__ __launch_bounds__(MLP_NH) void k_rank_export(const DevCtx* __restrict__ cp, int shot, int rnd,
                                                        float* feats, float* outs, int* rhat) {
  const DevCtx& c = *cp;
  const int k = blockIdx.x + 1, j = threadIdx.x;
  const int* dm = shot_dims(c, shot);
  const double* re = shot_reals(c, shot);
  __shared__ float x[MLP_NIN], h1[MLP_NH], h2[MLP_NH];
  rank_features(c, dm, re, rnd, k, x, j);
  __syncthreads();
  if (j < MLP_NIN) feats[k * MLP_NIN + j] = x[j];
  if (c.mlp_w == nullptr) return;
  const float o = rank_net(c.mlp_w, x, h1, h2, j);
  if (j == 0) {
    outs[k] = o;
    rhat[k] = rank_of(o, dm[DL::chi]);
  }
}

// Omega (rt x l), row-major.
__global__ void k_gauss(const DevCtx* __restrict__ cp, OpArgs a) {
  const DevCtx& c = *cp;
  const int shot = blockIdx.z, k = a.site;
  const int* dm = shot_dims(c, shot);
  if (!gate_open(dm, a.gate)) return;
  const int m = dm[DL::rt + k], l = dm[DL::rrf_l];
  if ((int64_t)m * l > c.L.cap_Om) {
    if (blockIdx.x == 0 && threadIdx.x == 0) raise_err(c, MPSW_DEV_ERR_CAP);
    return;
  }
  double* Om = shot_eng(c, shot) + c.L.off_Om;
  const int step = dm[DL::step];
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < m * l; e += gridDim.x * blockDim.x)
    Om[e] = sketch_normal(c.seed, step, a.aux, k, e / l, e % l);
}

// The test matrix entries of one key (seed, step, rounding, site), rows x cols.
__global__ void k_sketch_normals(unsigned long long seed, int step, int rnd, int site, int rows, int cols,
                                 double* out) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < rows * cols; e += gridDim.x * blockDim.x)
    out[e] = sketch_normal(seed, step, rnd, site, e / cols, e % cols);
}

// Keep a copy of M while its sketch is judged (k_rrf_swap_in then puts
// B = M Q in its place; two launches, so no block overwrites M before every
// block has copied it).
__global__ void k_rrf_swap(const DevCtx* __restrict__ cp, OpArgs a) {
  const DevCtx& c = *cp;
  const int shot = blockIdx.z, k = a.site;
  int* dm = shot_dims(c, shot);
  if (!gate_open(dm, a.gate)) return;
  const int m = dm[DL::rt + k], nn = 2 * dm[DL::rho + k + 1];
  double* E = shot_eng(c, shot);
  if ((int64_t)m * nn > c.L.cap_Mb) {
    if (blockIdx.x == 0 && threadIdx.x == 0) raise_err(c, MPSW_DEV_ERR_CAP);
    return;
  }
  const double* M = E + c.L.off_M;
  double* Mb = E + c.L.off_Mb;
  const int t = blockIdx.x * blockDim.x + threadIdx.x, nt = gridDim.x * blockDim.x;
  bulk_copy<8>(m * nn, t, nt, [&](int e) { return M[e]; }, [&](int e, double v) { Mb[e] = v; });
}

__global__ void k_rrf_swap_in(const DevCtx* __restrict__ cp, OpArgs a) {
  const DevCtx& c = *cp;
  const int shot = blockIdx.z, k = a.site;
  int* dm = shot_dims(c, shot);
  if (!gate_open(dm, a.gate)) return;
  const int m = dm[DL::rt + k], l = dm[DL::rrf_l];
  double* E = shot_eng(c, shot);
  if ((int64_t)m * l > c.L.cap_M) return;
  double* M = E + c.L.off_M;
  const double* Z = E + c.L.off_Zs;
  const int t = blockIdx.x * blockDim.x + threadIdx.x, nt = gridDim.x * blockDim.x;
  bulk_copy<8>(m * l, t, nt, [&](int e) { return Z[e]; }, [&](int e, double v) { M[e] = v; });
  if (t == 0) dm[DL::svd_n] = l;
}

// res2 = ||M - B Q^T||_F^2 from the kept copy of M and the product B Q^T
// (one workgroup per shot, fixed summation order).
__global__ __launch_bounds__(256) void k_rrf_resid(const DevCtx* __restrict__ cp, OpArgs a) {
  const DevCtx& c = *cp;
  const int shot = blockIdx.z, k = a.site;
  const int* dm = shot_dims(c, shot);
  if (!gate_open(dm, a.gate)) return;
  const int m = dm[DL::rt + k], nn = 2 * dm[DL::rho + k + 1];
  const double* E = shot_eng(c, shot);
  __shared__ double red[4];
  double s = 0.0;
  if ((int64_t)m * nn <= c.L.cap_Mb && (int64_t)m * nn <= c.L.cap_Rz) {
    const double* Mb = E + c.L.off_Mb;
    const double* Rz = E + c.L.off_Rz;
    for (int e = threadIdx.x; e < m * nn; e += 256) {
      const double d = Mb[e] - Rz[e];
      s = fma(d, d, s);
    }
  } else if (threadIdx.x == 0) {
    raise_err(c, MPSW_DEV_ERR_CAP);
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) shot_reals(c, shot)[RL::rrf_res2] = s;
}

// Accept the sketch or restore M for the exact SVD (every block takes the
// same decision from the same values; block 0 records it).
__global__ void k_rrf_accept(const DevCtx* __restrict__ cp, OpArgs a) {
  const DevCtx& c = *cp;
  const int shot = blockIdx.z, k = a.site;
  int* dm = shot_dims(c, shot);
  if (!gate_open(dm, a.gate)) return;
  double* re = shot_reals(c, shot);
  const int m = dm[DL::rt + k], nn = 2 * dm[DL::rho + k + 1], l = dm[DL::rrf_l];
  const int r = dm[DL::rho + k], chi = dm[DL::chi];
  const double res2 = re[RL::rrf_res2];
  const double eps = re[RL::eps], s1 = re[RL::rrf_sig1], tail = re[RL::rrf_tail];
  const bool capped = (r >= chi);
  const bool accept = capped ? (res2 <= 0.21 * tail) : (r < l && res2 <= (eps * s1) * (eps * s1));
  const int t = blockIdx.x * blockDim.x + threadIdx.x, nt = gridDim.x * blockDim.x;
  if (!accept) {
    double* E = shot_eng(c, shot);
    double* M = E + c.L.off_M;
    const double* Mb = E + c.L.off_Mb;
    bulk_copy<8>(m * nn, t, nt, [&](int e) { return Mb[e]; }, [&](int e, double v) { M[e] = v; });
  }
  __syncthreads();
  if (t == 0) {
    if (accept) {
      if (a.aux >= 0 && a.aux < 3) re[RL::tail2 + a.aux] += tail + res2;
    } else {
      dm[DL::fallbacks] += 1;
    }
  }
}

// After the grid of k_rrf_accept: the gate state (separate launch so that no
// block of the restore reads a half-updated state).
__global__ void k_rrf_settle(const DevCtx* __restrict__ cp, OpArgs a) {
  const DevCtx& c = *cp;
  const int shot = blockIdx.x * blockDim.x + threadIdx.x;
  if (shot >= c.B) return;
  int* dm = shot_dims(c, shot);
  double* re = shot_reals(c, shot);
  if (dm[DL::rrf] != 1) return;
  const int k = a.site;
  const int l = dm[DL::rrf_l], r = dm[DL::rho + k], chi = dm[DL::chi];
  const double res2 = re[RL::rrf_res2];
  const double eps = re[RL::eps], s1 = re[RL::rrf_sig1], tail = re[RL::rrf_tail];
  const bool capped = (r >= chi);
  const bool accept = capped ? (res2 <= 0.21 * tail) : (r < l && res2 <= (eps * s1) * (eps * s1));
  dm[DL::rrf] = accept ? 2 : 0;
  if (!accept) dm[DL::svd_n] = 0;
  if (a.aux >= 0 && a.aux < 3) {
    const int jk = a.aux * MPSW_MAXK + k;
    if (accept) {
      dm[DL::rrf_back + jk] = 0;
    } else {
      const int b = min(64, max(1, 2 * dm[DL::rrf_back + jk]));
      dm[DL::rrf_back + jk] = b;
      dm[DL::rrf_skip + jk] = dm[DL::step] + 1 + b;
    }
  }
}

// core slot <- Tc (r x 2 rho), after the sketch was accepted.
__global__ void k_rrf_core(const DevCtx* __restrict__ cp, OpArgs a) {
  const DevCtx& c = *cp;
  const int shot = blockIdx.z, k = a.site;
  int* dm = shot_dims(c, shot);
  if (!gate_open(dm, a.gate)) return;
  const int nn = 2 * dm[DL::rho + k + 1], r = dm[DL::rho + k];
  if ((int64_t)r * nn > c.cap_mps[a.slot][k] || (int64_t)r * nn > c.L.cap_Tc) {
    if (blockIdx.x == 0 && threadIdx.x == 0) raise_err(c, MPSW_DEV_ERR_CAP);
    return;
  }
  double* core = shot_mps(c, shot) + c.off_mps[a.slot][k];
  const double* Tc = shot_eng(c, shot) + c.L.off_Tc;
  const int t = blockIdx.x * blockDim.x + threadIdx.x, nt = gridDim.x * blockDim.x;
  bulk_copy<8>(r * nn, t, nt, [&](int e) { return Tc[e]; }, [&](int e, double v) { core[e] = v; });
  if (t == 0) dm[DL::svd_n] = 0;
}

// The bond is done: back to the exact state for the next one.
__global__ void k_rrf_clear(const DevCtx* __restrict__ cp) {
  const DevCtx& c = *cp;
  const int shot = blockIdx.x * blockDim.x + threadIdx.x;
  if (shot >= c.B) return;
  int* dm = shot_dims(c, shot);
  dm[DL::rrf] = 0;
  dm[DL::svd_n] = 0;
}

void launch_rrf_plan(const DevCtx* d, const OpArgs& a, int nshots, hipStream_t s) {
  hipLaunchKernelGGL(k_rrf_plan, dim3(1, 1, nshots), dim3(MLP_NH), 0, s, d, a);
}
void launch_gauss(const DevCtx* d, const OpArgs& a, int64_t cap, int nshots, hipStream_t s) {
  const int blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (cap + 255) / 256));
  hipLaunchKernelGGL(k_gauss, dim3(blocks, 1, nshots), dim3(256), 0, s, d, a);
}
void launch_rrf_swap(const DevCtx* d, const OpArgs& a, int64_t cap, int nshots, hipStream_t s) {
  const int blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (cap + 2047) / 2048));
  hipLaunchKernelGGL(k_rrf_swap, dim3(blocks, 1, nshots), dim3(256), 0, s, d, a);
  hipLaunchKernelGGL(k_rrf_swap_in, dim3(blocks, 1, nshots), dim3(256), 0, s, d, a);
}
void launch_rrf_accept(const DevCtx* d, const OpArgs& a, int64_t cap, int nshots, hipStream_t s) {
  const int blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (cap + 2047) / 2048));
  hipLaunchKernelGGL(k_rrf_accept, dim3(blocks, 1, nshots), dim3(256), 0, s, d, a);
  hipLaunchKernelGGL(k_rrf_settle, dim3((nshots + 63) / 64), dim3(64), 0, s, d, a);
}
void launch_sketch_normals(unsigned long long seed, int step, int rnd, int site, int rows, int cols, double* out,
                           hipStream_t s) {
  const int blocks = std::max(1, std::min(1024, (rows * cols + 255) / 256));
  hipLaunchKernelGGL(k_sketch_normals, dim3(blocks), dim3(256), 0, s, seed, step, rnd, site, rows, cols, out);
}
void launch_rrf_resid(const DevCtx* d, const OpArgs& a, int nshots, hipStream_t s) {
  hipLaunchKernelGGL(k_rrf_resid, dim3(1, 1, nshots), dim3(256), 0, s, d, a);
}
void launch_rank_export(const DevCtx* d, int shot, int rnd, int K, float* feats, float* outs, int* rhat,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_rank_export, dim3(K - 1), dim3(MLP_NH), 0, s, d, shot, rnd, feats, outs, rhat);
}
void launch_rrf_core(const DevCtx* d, const OpArgs& a, int64_t cap, int nshots, hipStream_t s) {
  const int blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (cap + 2047) / 2048));
  hipLaunchKernelGGL(k_rrf_core, dim3(blocks, 1, nshots), dim3(256), 0, s, d, a);
  hipLaunchKernelGGL(k_rrf_clear, dim3((nshots + 63) / 64), dim3(64), 0, s, d);
}

}  // namespace mpsw
