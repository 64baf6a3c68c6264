/*
 * mpsw.h -- C ABI of the MI355X quantics-MPS acoustic wave stepper.
 *
 * Method: Nemeth & Vattay, "Quantum Circuit and Tensor Network Implementation
 * of the 2D Acoustic Wave Equation".  A field u[x, z] on a 2^n x 2^n grid
 * (Sec. 2) is held as a matrix product state over K = 2n binary sites
 * (Sec. 4.1, eq. 8); sites 1..n are the bits x_{n-1}..x_0 of the horizontal
 * index (most significant first), sites n+1..2n the bits z_{n-1}..z_0 (eq. 3).
 * A state may instead use the interleaved order x_{n-1} z_{n-1} ... x_0 z_0
 * (bits of equal significance side by side); it holds the same fields and
 * changes only the ranks the roundings keep.
 * One call of mpsw_step advances eq. 17,
 *
 *   psi^{k+1} = 2 psi^k - psi^{k-1} + lambda^2 C^2 (S_x+ + S_x- + S_z+ + S_z- - 4 I) psi^k,
 *
 * with the shift MPOs of Sec. 4.2 (eqs. 9-15), the diagonal c^2 MPO of
 * Sec. 4.3, and a compression (left-to-right QR sweep, then right-to-left SVD
 * sweep discarding sigma_i < eps * sigma_max and capping the bond at chi_max,
 * Sec. 4.3) after each of the three operator applications:
 *
 *   y = round(L psi^k);  w = round(C^2 y);  psi^{k+1} = round(2 psi^k - psi^{k-1} + lambda^2 w + s_k e_src).
 *
 * Conventions (all entry points):
 *   - return 0 (MPSW_OK) on success, a negative MPSW_E* code on failure; the
 *     message of the last failure on the calling thread is mpsw_last_error();
 *   - host arrays passed in are borrowed for the duration of the call only;
 *   - dense fields are float64, 4^n entries, flat index x * 2^n + z (three-
 *     dimensional states: 8^n entries, flat index (x * 2^n + y) * 2^n + z);
 *   - all device work of a state is ordered on the HIP stream given at
 *     creation (NULL = the default stream); entry points that return data to
 *     the host synchronise that stream;
 *   - a state is not thread-safe; distinct states are independent.
 * All computation runs in the library's HIP kernels on the current device.
 */
#ifndef MPSW_H
#define MPSW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MPSW_OK = 0,
  MPSW_EINVAL = -1,     /* bad argument */
  MPSW_ENOMEM = -2,     /* device allocation failed or a size exceeds the workspace */
  MPSW_EHIP = -3,       /* a HIP runtime call failed */
  MPSW_ESTATE = -4,     /* call out of order (e.g. step before set_velocity) */
  MPSW_ECFL = -5,       /* lambda^2 * max(c^2) * ndim > 1: the scheme is unstable */
  MPSW_ENONFINITE = -6  /* a non-finite value was produced (detected at a sync) */
};

/* Contraction precision.  QR, Jacobi SVD, truncation and storage stay FP64.
   MPSW_FP32: operands rounded to FP32, FP32 matrix-core products.
   MPSW_BF16: each operand split into three BF16 parts (hi + mid + lo), six of
   the nine partial products on BF16 matrix cores (the refinement terms carry
   what one BF16 part drops).  In both, FP32 sums of 16-deep slices are
   accumulated in FP64. */
enum { MPSW_FP64 = 0, MPSW_FP32 = 1, MPSW_BF16 = 2 };
enum { MPSW_PERIODIC = 0, MPSW_OPEN = 1 };                     /* shift boundary */
enum { MPSW_SEQUENTIAL = 0, MPSW_INTERLEAVED = 1 };            /* site order */
/* truncation rank mode: the exact SVD of every bond (Sec. 4.3); a randomized
 * range finder at the rank the network proposes; or at the bond's kept rank of
 * the previous step, with no network (the baseline the network is judged
 * against).  The two sketch modes share the width rule, the residual test and
 * the exact fallback described at mpsw_rank_model_set. */
enum { MPSW_RANK_EXACT = 0, MPSW_RANK_LEARNED = 1, MPSW_RANK_PREVIOUS = 2 };

typedef struct mpsw_config {
  int n;              /* grid 2^n x 2^n, 1 <= n <= 11; K = 2n sites (the tallest QR of a
                         rounding has 2^(K/2+1) rows, and a panel of it must fit in LDS) */
  int chi_max;        /* bond cap of every rounding, >= 1 */
  double eps;         /* relative singular-value cutoff, >= 0 */
  double lambda;      /* mesh ratio dt/dh of eq. 2, > 0 */
  int precision;      /* MPSW_FP64 | MPSW_FP32 | MPSW_BF16 */
  int boundary;       /* MPSW_PERIODIC (cyclic shifts) | MPSW_OPEN (eq. 11 as printed) */
  int rank_mode;      /* MPSW_RANK_EXACT | MPSW_RANK_LEARNED | MPSW_RANK_PREVIOUS */
  uint64_t seed;      /* seed of the library's own random sketches */
  int ordering;       /* MPSW_SEQUENTIAL (x bits, then z bits; eq. 3) | MPSW_INTERLEAVED
                         (x_{n-1} z_{n-1} ... x_0 z_0).  Dense fields passed in and out
                         are u[x, z] in either order; MPS cores given to
                         mpsw_set_velocity_mpo are in the state's site order */
  int ndim;           /* 2 (0 means 2): the paper's u[x, z], K = 2n sites; or 3: u[x, y, z]
                         on a 2^n cube, K = 3n sites (registers x, y, z), the seven-point
                         Laplacian with -6I, n <= 7 */
} mpsw_config;

typedef struct mpsw_state_s* mpsw_state;

typedef struct mpsw_stats {
  int64_t step;            /* steps taken by this shot since its fields were set (or creation) */
  int nsites;              /* K */
  int bonds[64];           /* bonds of psi^k, K+1 entries */
  int max_exact_bond[3];   /* largest bond before truncation in the last step, per rounding */
  double tail2[3];         /* discarded sum of squared singular values in the last step,
                              summed over bonds, per rounding */
  int64_t fallbacks;       /* learned-rank mode: sketches rejected (the exact SVD ran) */
  int max_jacobi_sweeps;   /* most one-sided Jacobi sweeps any bond needed since creation */
  int64_t sketches;        /* learned-rank mode: bonds sketched by the randomized range finder */
} mpsw_stats;

/* Create a state for one shot: a 2^n x 2^n grid (Sec. 2) held as a K = 2n site
 * MPS (Sec. 4.1), with psi^0 = psi^{-1} = 0 (bond 1).  lambda is the mesh
 * ratio dt/dh of eq. 2; eps and chi_max are the cutoff and bond cap of the
 * compression of Sec. 4.3.  hip_stream: a hipStream_t or NULL.  Allocates the
 * device workspace for the worst-case bonds of this (n, chi_max) with
 * hipMalloc.  *out receives the handle (owned by the caller, released with
 * mpsw_destroy).  Errors: EINVAL, ENOMEM, EHIP. */
int mpsw_create_state(const mpsw_config* cfg, void* hip_stream, mpsw_state* out);

/* Batch of nshots shots with the same n sharing one c^2 model; shot i uses
 * cfgs[i] (chi_max and eps may differ per shot; n, lambda, precision, boundary,
 * rank mode and site order must agree).  Steps of a batch advance all shots together.  Errors as above. */
int mpsw_create_batch(const mpsw_config* cfgs, int nshots, void* hip_stream, mpsw_state* out);

/* Device memory supplied by the caller (for instance a framework's caching
 * allocator): alloc returns device memory of at least `bytes` bytes, aligned
 * to 256 bytes, on the current device, or NULL when it cannot (the library
 * then fails with ENOMEM); free gives back a block alloc returned, with the
 * size it was asked for.  ctx is passed through.  Both are called only from
 * within the library's entry points on the calling thread, never from device
 * work; a block is freed only after the state's stream has finished with it. */
typedef struct mpsw_allocator {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, size_t bytes, void* ctx);
  void* ctx;
} mpsw_allocator;

/* mpsw_create_batch whose every device allocation over the state's life
 * (workspace, MPS arena, c^2 operator, set-up temporaries) goes through
 * `alloc` (NULL: hipMalloc / hipFree).  The allocator must outlive the state.
 * Errors: EINVAL (an allocator without both functions), ENOMEM, EHIP. */
int mpsw_create_batch_ex(const mpsw_config* cfgs, int nshots, void* hip_stream, const mpsw_allocator* alloc,
                         mpsw_state* out);

/* Set c^2 from its dense field (host, 4^n or 8^n float64, all > 0).  The diagonal
 * c^2 operator is built on the device as the right-to-left truncated TT-SVD of
 * c^2 (taken in the state's site order) with relative cutoff eps_c and no
 * bond cap (Sec. 4.3: the velocity field encoded as a diagonal MPO).  Errors: EINVAL (non-positive or
 * non-finite c^2), ECFL, ENOMEM, EHIP. */
int mpsw_set_velocity_dense(mpsw_state st, const double* c2, double eps_c);

/* Set c^2 directly as the cores of its diagonal (host, float64):
 * bonds[0..K] with bonds[0] = bonds[K] = 1, cores packed site after site,
 * core k row-major of shape (bonds[k], 2, bonds[k+1]), site k of the state's
 * site order.  CFL is checked on the
 * reconstructed field.  Errors: EINVAL, ECFL, ENOMEM, EHIP. */
int mpsw_set_velocity_mpo(mpsw_state st, const int* bonds, const double* cores);

/* Point source for shot `shot` at grid point (ix, iz), the source term of the
 * wave equation (Sec. 2) entering the update sum of eq. 17 as a bond-1
 * product state (the impulse of the run in Sec. 5 is wavelet = {1, 0, ...}):
 * step j (counted from creation, or from the shot's last mpsw_set_fields or
 * mpsw_set_cores) adds wavelet[j] * e_(ix,iz) to psi^{j+1}; steps j >= nt
 * add nothing.  The host array is copied.  Errors: EINVAL (also for a
 * three-dimensional state). */
int mpsw_set_source(mpsw_state st, int shot, int ix, int iz, int nt, const double* wavelet);
/* The same at grid point (ix, iy, iz) of a three-dimensional state.
 * Errors: EINVAL (also for a two-dimensional state). */
int mpsw_set_source_3d(mpsw_state st, int shot, int ix, int iy, int iz, int nt, const double* wavelet);

/* Initial fields of shot `shot` from dense host arrays (NULL = zero); each is
 * stored as its right-to-left TT-SVD with the shot's (eps, chi_max).
 * Restarts the shot's step counter (its source clock) at 0 and clears its
 * learned-rank sketch back-offs.  Errors: EINVAL (also for a non-finite
 * value), ENOMEM, EHIP. */
int mpsw_set_fields(mpsw_state st, int shot, const double* u_prev, const double* u_cur);

/* Checkpoint of shot `shot`: the cores of psi^k (which = 0) or psi^{k-1}
 * (which = 1) as they are held (Sec. 4.1, eq. 8), into host memory: bonds
 * receives K+1 ints, cores (if not NULL) the cores packed site after site,
 * core k row-major of shape (bonds[k], 2, bonds[k+1]), at most `cap`
 * doubles.  Returns the number of doubles of the cores (>= 0) or a negative
 * error code.  The shot's step counter is mpsw_stats.step.  Synchronises.
 * Errors: EINVAL (cap too small), EHIP, ENONFINITE. */
int mpsw_get_cores(mpsw_state st, int shot, int which, int* bonds, double* cores, int64_t cap);

/* Resume shot `shot` from a checkpoint: psi^{k-1} and psi^k are set to the
 * given cores exactly (no rounding; same packing as mpsw_get_cores, host
 * memory borrowed for the call) and the shot's step counter (its source
 * clock) to `step`.  Every bond must lie in [1, min(chi_cap, 2^k, 2^(K-k))],
 * chi_cap the largest chi_max of the state.  Stepping on from here repeats,
 * bit for bit, what the checkpointed state would have done.
 * Errors: EINVAL, EHIP. */
int mpsw_set_cores(mpsw_state st, int shot, int64_t step, const int* bonds_prev, const double* cores_prev,
                   const int* bonds_cur, const double* cores_cur);

/* Enqueue k >= 0 steps of eq. 17 on the state's stream (asynchronous).
 * Errors: ESTATE (no velocity set), EINVAL, EHIP. */
int mpsw_step(mpsw_state st, int k);

/* Graph mode (on != 0): mpsw_step replays captured HIP graphs, three steps
 * (one turn of the psi slot rotation) per launch, capturing on first use
 * and again after a velocity change; remaining steps run eagerly.  Results
 * are identical to eager stepping.  Errors: EINVAL, EHIP. */
int mpsw_set_graph_mode(mpsw_state st, int on);

/* A group steps several states together (states may differ in n; shots of a
 * state may differ in chi_max and eps) as one HIP graph with one branch per
 * state, launched on `hip_stream`.  The states stay owned by the caller and
 * must outlive the group. */
typedef struct mpsw_group_s* mpsw_group;
int mpsw_group_create(const mpsw_state* states, int nstates, void* hip_stream, mpsw_group* out);
/* Enqueue k steps of every state (asynchronous; ordered after, and before,
 * the work already enqueued on each state's own stream).  Errors: EINVAL,
 * ESTATE, EHIP. */
int mpsw_group_step(mpsw_group g, int k);
int mpsw_group_destroy(mpsw_group g);

/* Write the dense field of shot `shot` (which = 0: u^k, 1: u^{k-1}; 2: the c^2
 * operator's diagonal; 3, 4: y and w of the last step) into the caller's
 * buffer of 4^n (8^n) float64 (host memory, or device memory if
 * out_is_device != 0): the contraction of the chain of eq. 8 (Sec. 4.1), in
 * the grid layout of eq. 3.  Synchronises the stream; reports ENONFINITE if
 * any entry is not finite.  Errors: EINVAL, EHIP, ENONFINITE. */
int mpsw_to_dense(mpsw_state st, int shot, int which, double* out, int out_is_device);

/* Bonds (K+1 ints) of shot `shot`'s psi^k (which = 0), psi^{k-1} (1) or of
 * the c^2 operator (2).  Synchronises.  Errors: EINVAL, EHIP. */
int mpsw_get_bonds(mpsw_state st, int shot, int which, int* bonds);

/* Statistics of shot `shot` after the last step: the bonds the compression of
 * Sec. 4.3 kept, and per rounding the largest bond before truncation and the
 * discarded sum of squared singular values (the truncation error of the
 * rule "discard sigma_i < eps sigma_max, cap at chi_max", summed in FP64 over
 * the bonds).  Synchronises and reports device-side failures of the steps
 * enqueued so far: ENOMEM (a live size exceeded a workspace), ENONFINITE,
 * EHIP (a bounded inter-workgroup wait gave up). */
int mpsw_get_stats(mpsw_state st, int shot, mpsw_stats* out);

/* Autotuner of the launch shapes for this state's bucket (grid, chi cap,
 * shot count, precision): times `steps` steps from the current state for
 * each candidate Jacobi block width (rule, 8, 16, 32 columns) and then each
 * cap on the workgroups per shot of a QR factorisation (32, 16, 8, 4, 3, 2, 1;
 * the same cap bounds the workgroups of a Jacobi sweep, one per block pair
 * of a round at most, each taking several pairs in turn when fewer), then
 * each block width again at the chosen cap, keeps
 * the fastest pair, and restores the state exactly as it was (fields, bonds,
 * step counters).  The chosen values are returned if the pointers are not
 * NULL.  Synchronises.  Errors: EINVAL, ESTATE, ENOMEM, EHIP. */
int mpsw_autotune(mpsw_state st, int steps, int* qr_nwg, int* jac_block);

/* Set the launch shapes mpsw_autotune chooses, without timing: the cap on the
 * workgroups per shot of a QR factorisation and a Jacobi sweep (1..32) and the Jacobi block
 * width (0 = rule from the column count, or 8, 16, 32).  For reusing a shape
 * tuned earlier on another state of the same bucket; the shapes change the
 * order of the factorisations' sums, so results agree with another shape to
 * rounding, and with the same shape bit for bit.  Captured step graphs are
 * dropped.  Errors: EINVAL. */
int mpsw_set_launch_shapes(mpsw_state st, int qr_nwg, int jac_block);

/* Learned-rank rounding (rank_mode MPSW_RANK_LEARNED): for every bond of the
 * SVD sweep the rank network (parameters w, MPSW_MLP_NPARAM floats, host
 * memory copied) proposes r from the bond's leading singular values at the
 * previous step; when r is below chi_max and r + 8 at most 3/4 of the bond
 * matrix's smaller side, a randomized range finder of width r + 8 with one
 * power iteration sketches the bond matrix (Gaussian test matrix from the
 * state's seed), the SVD stage runs on the sketch, and a FP64 residual test
 * keeps it or runs the exact SVD (counted in mpsw_stats.fallbacks).  Required before
 * stepping a learned-rank state.  A MPSW_RANK_PREVIOUS state takes r as the
 * rank the same bond kept in the same rounding at the previous step and needs
 * no network.  Errors: EINVAL, EHIP. */
int mpsw_rank_model_set(mpsw_state st, const float* w, int nw);

/* Network inputs of bonds 1..K-1 of rounding `rounding` (0: L psi, 1: c^2 y,
 * 2: the sum) of shot `shot`, exactly as the learned-rank rounding forms them
 * for the coming step: row k-1 holds log10(sigma_i / sigma_1) for the 32
 * leading singular values of bond k in the last step (-30 where absent),
 * k / K and min(step, 10^4) / 1000 (34 floats per row, host memory, (K-1) x 34).
 * Used to log training data: the label of a row is the rank the rule keeps
 * at that bond in the coming step.  Synchronises.  Errors: EINVAL, ESTATE
 * (no velocity set), EHIP. */
int mpsw_get_rank_features(mpsw_state st, int shot, int rounding, float* feats);

/* The leading 32 singular values (descending, 0 where absent) of every bond
 * of rounding `rounding` (0: L psi, 1: c^2 y, 2: the sum) in the last step of
 * shot `shot`: out[k * 32 + i] for k = 0..K-1 (row k is bond k, the SVD of
 * site k; row 0 is unused).  Synchronises.  Errors: EINVAL, EHIP. */
int mpsw_get_sigma_log(mpsw_state st, int shot, int rounding, double* out);

/* Number of shots and sites of the state. */
int mpsw_get_shape(mpsw_state st, int* nshots, int* nsites);

/* Free all device memory of the state.  NULL is accepted. */
int mpsw_destroy(mpsw_state st);

/* Message of the last failure on the calling thread ("" if none). */
const char* mpsw_last_error(void);

/* Truncation-rank network (34 -> 128 -> 128 -> 1, ReLU, FP32), trained and
 * evaluated on the GPU.  X: m x 34 features (row-major), y: m targets (rank /
 * chi_max), w: the MPSW_MLP_NPARAM parameters W1 (34 x 128, input by output),
 * b1, W2 (128 x 128), b2, W3 (128), b3.  Loss: mean of wt (out - y)^2 with
 * wt = alpha where out < y, else 1.  All pointers are host memory borrowed for
 * the call.  Errors: EINVAL, ENOMEM, EHIP. */
#define MPSW_MLP_NPARAM 21121
/* Loss and gradient at w (gradient in the parameter order). */
int mpsw_mlp_grad(const float* X, const float* y, int m, float alpha, const float* w, float* grad, float* loss);
/* Initial parameters: He-scaled normal weights (variance 2 / fan-in for the
 * ReLU layers, 1 / fan-in for the output layer; a 64-bit Mersenne twister
 * from `seed`), zero biases.  Host only.  Errors: EINVAL. */
int mpsw_mlp_init(uint64_t seed, float* w);
/* `epochs` full-batch Adam steps from w (updated in place) at learning rate lr. */
int mpsw_mlp_train(const float* X, const float* y, int m, int epochs, float lr, float alpha, float* w);
/* mpsw_mlp_grad for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid allocation): X, y,
 * w, grad and loss are DEVICE pointers owned by the caller (same layouts as
 * mpsw_mlp_grad), and the per-chunk partial sums live in a static device
 * array of the library (about 21.6 MB per device, held until the process
 * ends), so m is at most 8192.  Enqueued on hip_stream (NULL = the default
 * stream), asynchronous, no allocation, no synchronisation; the results
 * equal mpsw_mlp_grad's bit for bit.  All calls on one device share the
 * scratch array: calls that overlap on one device (different streams or
 * threads without ordering) race.  Errors: EINVAL (null pointer, m outside
 * [1, 8192]), EHIP. */
int mpsw_mlp_grad_noalloc(const float* X, const float* y, int m, float alpha, const float* w, float* grad,
                          float* loss, void* hip_stream);
/* Network outputs for m feature rows. */
int mpsw_mlp_forward(const float* X, int m, const float* w, float* out);

#ifdef __cplusplus
}
#endif
#endif /* MPSW_H */
