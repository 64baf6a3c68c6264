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


__device__ __forceinline__ int* shot_sync(const DevCtx& c, int shot) { return c.sync + (int64_t)shot * MPSW_SYNC_STRIDE; }

}  // namespace mpsw
