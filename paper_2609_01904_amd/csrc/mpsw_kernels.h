// Kernel entry points and operation codes of libmpsw.
#pragma once
#include "mpsw_internal.h"

namespace mpsw {

// GEMM-shaped operations (planned on the device from the live bonds).
enum GemmOp {
  G_L2R_EXPLICIT = 1,  // X_k = R_{k-1} S_k with explicit source cores
  G_COPY_RX,           // identity source: X_k = R_{k-1}
  G_DENSE,             // dense contraction step V_{k+1} = V_k G_k
  G_US,                // U_r Sigma_r = M_k V_r
  G_RRF_Y,             // Y = M^T Omega (aux 0) or Y = M^T Z (aux 1): row-space sketch
  G_RRF_Z,             // Z = M Q: column-space iterate (aux 0) or B = M Q (aux 1)
  G_RRF_CORE,          // Tc = core_small Q^T (r x l times l x 2 rho)
  G_RRF_RES,           // Rz = B Q^T (rt x l times l x 2 rho): the sketch's reconstruction of M
  G_HALF_L,            // V_{k+1} = V_k Y_k: the left half of y contracted up to the middle site
  G_HALF_R,            // W_k = Y_k W_{k+1}: the right half of y contracted down to the middle site
  G_MEET_H             // X2 = (V_n W_n) .* c^2: the Hadamard product's middle unfolding
};

// Gates of the SVD-stage launches (OpArgs.gate) in the learned-rank rounding.
enum Gate { GATE_ALWAYS = 0, GATE_SKETCH = 1, GATE_EXACT = 2, GATE_ACCEPTED = 3 };

// Arithmetic of the contractions (k_gemm); storage is FP64 in every mode.
enum GemmMode {
  GEMM_FP64 = 0,   // FP64 matrix cores
  GEMM_FP32 = 1,   // operands rounded to FP32, FP32 matrix cores, FP32 accumulation
  GEMM_BF16X6 = 2  // operands split x = hi + mid + lo in BF16, six of the nine partial products, FP32 accumulation
};

// Rounding input kinds (k_prepare / k_init_R).
enum PrepOp { P_LAPLACE = 1, P_C2, P_SUM, P_DENSE };

struct OpArgs {
  int op;
  int site;
  int slot;    // MPS slot read (pack) or written (svd, finish); -1 = c^2 operator (dense)
  int slot2;   // second MPS slot (direct sum: psi^{k-1})
  int aux;     // op-specific flag (buffer select, rounding index)
  int step;    // step index (source sample)
  int shot;    // restrict to one shot (-1 = all)
  int mode;    // contraction arithmetic of k_gemm: GEMM_FP64, GEMM_FP32 or GEMM_BF16X6
  int gate;    // Gate: run only while the bond's sketch state allows it
};

// Contraction launch over output capacities mcap x ncap (64 x 64 tiles).
void launch_gemm(const DevCtx* d, const OpArgs& a, int64_t mcap, int64_t ncap, int grid_batch, int nshots, hipStream_t s);
void launch_prepare(const DevCtx* d, const OpArgs& a, int nshots, hipStream_t s);
void launch_init_R(const DevCtx* d, const OpArgs& a, int nshots, hipStream_t s);
void launch_pack_lap(const DevCtx* d, const OpArgs& a, int K, int nshots, int blocks, hipStream_t s);
void launch_pack_sum(const DevCtx* d, const OpArgs& a, int K, int nshots, int blocks, hipStream_t s);
void launch_sync_reset(const DevCtx* d, int nshots, hipStream_t s);
void launch_qrf(const DevCtx* d, const OpArgs& a, int bw, int nwg, int nshots, size_t lds, hipStream_t s);
void launch_applyq(const DevCtx* d, const OpArgs& a, int bw, int nwg, int nshots, hipStream_t s);
void launch_applyv(const DevCtx* d, const OpArgs& a, int bw, int nwg, int nshots, hipStream_t s);
void launch_jac(const DevCtx* d, const OpArgs& a, int b, int nwg, int nshots, size_t lds, int64_t lcap, hipStream_t s);
int jac_rows(int64_t lcap);
void launch_jacfin(const DevCtx* d, const OpArgs& a, int nshots, hipStream_t s);
void set_lds_limits(size_t bytes);
void launch_formq(const DevCtx* d, const OpArgs& a, int bw, int nwg, int nshots, hipStream_t s);
void launch_rrf_plan(const DevCtx* d, const OpArgs& a, int nshots, hipStream_t s);
void launch_gauss(const DevCtx* d, const OpArgs& a, int64_t cap, int nshots, hipStream_t s);
void launch_rrf_swap(const DevCtx* d, const OpArgs& a, int64_t cap, int nshots, hipStream_t s);
void launch_rrf_accept(const DevCtx* d, const OpArgs& a, int64_t cap, int nshots, hipStream_t s);
void launch_rrf_resid(const DevCtx* d, const OpArgs& a, int nshots, hipStream_t s);
void launch_sketch_normals(unsigned long long seed, int step, int rnd, int site, int rows, int cols, double* out,
                           hipStream_t s);
void launch_rank_export(const DevCtx* d, int shot, int rnd, int K, float* feats, float* outs, int* rhat,
                        hipStream_t s);
void launch_rrf_core(const DevCtx* d, const OpArgs& a, int64_t cap, int nshots, hipStream_t s);
void launch_finish(const DevCtx* d, const OpArgs& a, int nshots, hipStream_t s);
void launch_dense_init(const DevCtx* d, int nshots, hipStream_t s);
void launch_zero_state(const DevCtx* d, const OpArgs& a, int nshots, hipStream_t s);

}  // namespace mpsw
