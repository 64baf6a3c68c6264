// Device helpers shared by the kernel files of libmpsw.
#pragma once
#include "mpsw_kernels.h"

namespace mpsw {

using DL = ShotDimsLayout;
using RL = ShotRealLayout;

__device__ __forceinline__ int* shot_dims(const DevCtx& c, int shot) { return c.dims + (int64_t)shot * DL::size; }
__device__ __forceinline__ double* shot_reals(const DevCtx& c, int shot) { return c.reals + (int64_t)shot * RL::size; }
__device__ __forceinline__ double* shot_eng(const DevCtx& c, int shot) { return c.eng + (int64_t)shot * c.L.stride; }
__device__ __forceinline__ double* shot_mps(const DevCtx& c, int shot) { return c.mps + (int64_t)shot * c.mps_stride; }
__device__ __forceinline__ void raise_err(const DevCtx& c, int bit) { atomicOr(c.err, bit); }
// Algorithmic flops of one launch (counted once per shot by one thread).
__device__ __forceinline__ void count_flops(const DevCtx& c, int shot, int cls, double f) {
  atomicAdd(shot_reals(c, shot) + ShotRealLayout::alg_flops + cls, f);
}

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// block-wide sum for 256 threads; `red` has >= 4 doubles of LDS
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = blockDim.x >> 6;
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}


// Sum over each row of 16 lanes with DPP row rotations and quad permutes
// (every lane of the row receives the sum).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  // the patterns used here (row rotations, quad permutations) give every lane
  // a source lane, so no old value is merged and none needs initialising
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double row_sum16(double v) {
  v += dpp_f64<0x128>(v);  // row_ror:8
  v += dpp_f64<0x124>(v);  // row_ror:4
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  return v;
}
// Sum over the 64 lanes of a wave (row sums, then across the four rows).
__device__ __forceinline__ double wave_sum64(double v) {
  v = row_sum16(v);
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// Element-wise transfer of n items, dst(e, src(e)), with U independent loads in
// flight per thread before any of them is used: a loop with one load per
// iteration pays a full memory latency per iteration.
// Indices are 32-bit (every buffer here holds < 2^31 elements).
template <int U, class Src, class Dst>
__device__ __forceinline__ void bulk_copy(int n, int t, int nt, Src src, Dst dst) {
  for (int b = t; b < n; b += nt * U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = b + u * nt;
      v[u] = (e < n) ? src(e) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = b + u * nt;
      if (e < n) dst(e, v[u]);
    }
  }
}

// Columns of the bond matrix of site k the SVD stage factors: 2 rho_{k+1},
// or the sketch width while a randomized range finder result is judged.
__device__ __forceinline__ int svd_cols(const int* dm, int k) {
  const int o = dm[ShotDimsLayout::svd_n];
  return (o > 0) ? o : 2 * dm[ShotDimsLayout::rho + k + 1];
}
// Whether a launch with this gate runs for the shot's current bond.
__device__ __forceinline__ bool gate_open(const int* dm, int gate) {
  const int s = dm[ShotDimsLayout::rrf];
  switch (gate) {
    case GATE_SKETCH: return s == 1;
    case GATE_EXACT: return s != 2;
    case GATE_ACCEPTED: return s == 2;
    default: return true;
  }
}

__device__ __forceinline__ int* shot_sync(const DevCtx& c, int shot) { return c.sync + (int64_t)shot * MPSW_SYNC_STRIDE; }

}  // namespace mpsw
