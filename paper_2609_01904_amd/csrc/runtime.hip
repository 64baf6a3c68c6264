// Host runtime and C ABI of libmpsw.
//
// A state ("group") owns B shots of the same grid size.  Its step is a fixed
// sequence of kernel launches on the caller's stream (see run_step): three
// roundings, each an optional pack kernel, a left-to-right sweep of
// (contraction, QR-or-merge) pairs and a right-to-left sweep of (SVD, absorb)
// pairs.  Workspace capacities are computed from the worst-case bonds of the
// configuration; the kernels read the live bonds from device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/mpsw_debug.h"
#include "mpsw_kernels.h"

using namespace mpsw;
using DL = ShotDimsLayout;
using RL = ShotRealLayout;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(MPSW_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));         \
  } while (0)

inline int64_t p2(int e) { return (int64_t)1 << e; }

}  // namespace

namespace mpsw {
// Records the message returned by mpsw_last_error (for the other source files).
int set_last_error(int code, const char* msg) { return fail(code, msg); }
}  // namespace mpsw

namespace {
inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Dense fields cross the boundary as u[x, z] (flat x 2^n + z), or u[x, y, z].
// In the sequential site order that flat index is the site index; in the
// interleaved order bit m of axis r sits at bit ndim m + (ndim - 1 - r) of the
// site index.  These two copies move a field between the two layouts.
std::vector<int64_t> spread_bits(int n, int ndim) {
  std::vector<int64_t> sp((size_t)1 << n, 0);
  for (int64_t v = 0; v < ((int64_t)1 << n); ++v)
    for (int m = 0; m < n; ++m) sp[v] |= ((v >> m) & 1) << (ndim * m);
  return sp;
}
int64_t site_index(const std::vector<int64_t>& sp, int n, int ndim, int64_t flat) {
  const int64_t mask = ((int64_t)1 << n) - 1;
  int64_t idx = 0;
  for (int r = 0; r < ndim; ++r) idx |= sp[(flat >> (n * (ndim - 1 - r))) & mask] << (ndim - 1 - r);
  return idx;
}
void field_to_sites(const double* u, int n, int ndim, double* t) {
  const auto sp = spread_bits(n, ndim);
  const int64_t total = (int64_t)1 << (n * ndim);
  for (int64_t f = 0; f < total; ++f) t[site_index(sp, n, ndim, f)] = u[f];
}
void sites_to_field(const double* t, int n, int ndim, double* u) {
  const auto sp = spread_bits(n, ndim);
  const int64_t total = (int64_t)1 << (n * ndim);
  for (int64_t f = 0; f < total; ++f) u[f] = t[site_index(sp, n, ndim, f)];
}

// ---------------------------------------------------------------------------
// The fused Laplacian MPO (eqs. 6, 16: the four shifts and -4I; in three
// dimensions the six shifts and -6I) in site order: the registers x, z (or
// x, y, z) one after the other, MSB first (eq. 3), or their bits interleaved.
// It is a finite automaton read from the last site to the first; the bond
// carries what the sites to the right did: P (no shift yet), the carry of an
// S+ or the borrow of an S- still pending in register r (C_r, B_r), D (shift
// finished, or the -2 ndim I term).  The last register's shift enters at the
// right end (the last site is its least significant bit); P passes every site
// and may start the shift of another register at that register's least
// significant bit.  A site passes the other registers' pending carries on
// unchanged.  A pending carry at a register's top bit wraps (periodic) or is
// dropped (open, the terminal core of eq. 11 as printed).  States that no
// path from both ends reaches are pruned: in two dimensions bonds 3 inside
// the x register, 2 at the x|z cut and 4 inside the z register (sequential),
// at most 5 interleaved.
// ---------------------------------------------------------------------------
struct LapMPO {
  std::vector<int> bonds;                  // K+1
  std::vector<std::vector<double>> cores;  // [wl][wr][2][2]
};

LapMPO build_laplacian_mpo(int n, int boundary, int ordering, int ndim) {
  const int K = ndim * n;
  // states: P = 0, C_r = 1 + 2r, B_r = 2 + 2r, D = NS - 1
  const int NS = 2 + 2 * ndim, P = 0, D = NS - 1;
  const double I2[2][2] = {{1, 0}, {0, 1}};
  const double SP[2][2] = {{0, 0}, {1, 0}};  // |1><0|
  const double SM[2][2] = {{0, 1}, {0, 0}};  // |0><1|
  const bool periodic = boundary == MPSW_PERIODIC;
  const bool il = ordering == MPSW_INTERLEAVED;
  auto reg = [&](int k) { return il ? k % ndim : k / n; };
  auto bit = [&](int k) { return il ? n - 1 - k / ndim : n - 1 - k % n; };
  // T[k][out][in][s'][s]
  std::vector<std::vector<double>> T(K, std::vector<double>((size_t)NS * NS * 4, 0.0));
  auto add = [&](int k, int out, int in, const double (*op)[2]) {
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) T[k][((out * NS + in) * 2 + a) * 2 + b] += op[a][b];
  };
  for (int k = 0; k < K; ++k) {
    const int r = reg(k);
    add(k, D, D, I2);
    add(k, P, P, I2);
    for (int q = 0; q < ndim; ++q) {
      const int C = 1 + 2 * q, Bs = 2 + 2 * q;
      if (q == r) {
        add(k, C, C, SM);    // bit 1 -> 0, carry moves on
        add(k, D, C, SP);    // bit 0 -> 1, carry absorbed
        add(k, Bs, Bs, SP);  // bit 0 -> 1, borrow moves on
        add(k, D, Bs, SM);   // bit 1 -> 0, borrow absorbed
      } else {               // another register's carry and borrow pass
        add(k, C, C, I2);
        add(k, Bs, Bs, I2);
      }
    }
    if (bit(k) == 0 && r < ndim - 1) {   // P starts this register's shift here
      add(k, D, P, SP);
      add(k, D, P, SM);
      add(k, 1 + 2 * r, P, SM);
      add(k, 2 + 2 * r, P, SP);
    }
    if (bit(k) == n - 1) {   // top bit: a pending carry/borrow wraps or is dropped
      const int C = 1 + 2 * r, Bs = 2 + 2 * r;
      for (int in = 0; in < NS; ++in)
        for (int e = 0; e < 4; ++e) {
          double& cv = T[k][((size_t)C * NS + in) * 4 + e];
          double& bv = T[k][((size_t)Bs * NS + in) * 4 + e];
          if (periodic) T[k][((size_t)D * NS + in) * 4 + e] += cv + bv;
          cv = 0.0;
          bv = 0.0;
        }
    }
  }
  // the left end keeps the finished terms; the last register's shift and the
  // -2 ndim I term enter at the right end
  std::vector<double> left(NS, 0.0), right(NS, 0.0);
  left[D] = 1.0;
  right[P] = 1.0;
  right[1 + 2 * (ndim - 1)] = right[2 + 2 * (ndim - 1)] = 1.0;
  right[D] = -2.0 * ndim;
  // dense cores with bonds 1, NS, ..., NS, 1
  std::vector<int> wl(K), wr(K);
  std::vector<std::vector<double>> W(K);
  for (int k = 0; k < K; ++k) {
    wl[k] = (k == 0) ? 1 : NS;
    wr[k] = (k == K - 1) ? 1 : NS;
    W[k].assign((size_t)wl[k] * wr[k] * 4, 0.0);
    for (int o = 0; o < wl[k]; ++o)
      for (int i = 0; i < wr[k]; ++i)
        for (int e = 0; e < 4; ++e) {
          double v = 0.0;
          for (int oo = 0; oo < NS; ++oo) {
            if (k != 0 && oo != o) continue;
            const double lw = (k == 0) ? left[oo] : 1.0;
            for (int ii = 0; ii < NS; ++ii) {
              if (k != K - 1 && ii != i) continue;
              const double rw = (k == K - 1) ? right[ii] : 1.0;
              v += lw * rw * T[k][(oo * NS + ii) * 4 + e];
            }
          }
          W[k][((size_t)o * wr[k] + i) * 4 + e] = v;
        }
  }
  // keep the states of each bond that a chain of nonzero transitions reaches
  // from the left end and from the right end
  auto nz = [&](int k, int o, int i) {
    for (int e = 0; e < 4; ++e)
      if (W[k][((size_t)o * wr[k] + i) * 4 + e] != 0.0) return true;
    return false;
  };
  std::vector<std::vector<char>> fromL(K + 1, std::vector<char>(NS, 0)), fromR(K + 1, std::vector<char>(NS, 0));
  fromL[0][0] = 1;
  for (int b = 1; b <= K; ++b)
    for (int s = 0; s < wr[b - 1]; ++s)
      for (int o = 0; o < wl[b - 1]; ++o)
        if (fromL[b - 1][o] && nz(b - 1, o, s)) { fromL[b][s] = 1; break; }
  fromR[K][0] = 1;
  for (int b = K - 1; b >= 0; --b)
    for (int s = 0; s < wl[b]; ++s)
      for (int i = 0; i < wr[b]; ++i)
        if (fromR[b + 1][i] && nz(b, s, i)) { fromR[b][s] = 1; break; }
  std::vector<std::vector<int>> keep(K + 1);
  keep[0] = {0};
  keep[K] = {0};
  for (int b = 1; b < K; ++b)
    for (int s = 0; s < NS; ++s)
      if (fromL[b][s] && fromR[b][s]) keep[b].push_back(s);
  LapMPO out;
  out.bonds.resize(K + 1);
  for (int b = 0; b <= K; ++b) out.bonds[b] = (int)keep[b].size();
  out.cores.resize(K);
  for (int k = 0; k < K; ++k) {
    const auto& kl = keep[k];
    const auto& kr = keep[k + 1];
    out.cores[k].assign(kl.size() * kr.size() * 4, 0.0);
    for (size_t o = 0; o < kl.size(); ++o)
      for (size_t i = 0; i < kr.size(); ++i)
        for (int e = 0; e < 4; ++e)
          out.cores[k][(o * kr.size() + i) * 4 + e] = W[k][((size_t)kl[o] * wr[k] + kr[i]) * 4 + e];
  }
  return out;
}

// ---------------------------------------------------------------------------
// Capacity planning
// ---------------------------------------------------------------------------
struct SweepCaps {
  std::vector<int64_t> rin, rt, rho;
  bool explicit_in = false;   // source cores are materialised in the IN buffers
};

SweepCaps sweep_caps(const std::vector<int64_t>& rin, int K, int64_t chi) {
  SweepCaps s;
  s.rin = rin;
  s.rt.assign(K + 1, 1);
  for (int k = 0; k + 1 <= K - 1; ++k) s.rt[k + 1] = std::min(2 * s.rt[k], rin[k + 1]);
  s.rho.assign(K + 1, 1);
  for (int k = K - 1; k >= 1; --k) s.rho[k] = std::min({chi, s.rt[k], 2 * s.rho[k + 1]});
  return s;
}

struct Plan {
  int K, half;   // sites; where the two sweeps of the Kronecker rounding meet
  std::vector<SweepCaps> sw;   // roundings handled by this engine
  std::vector<int64_t> Rmax;   // state bond caps (y feeding the Kronecker rounding)
  std::vector<int> D;          // c^2 bonds (empty when no Kronecker rounding)
  bool kron = false;
  int64_t rrf_l = 0;           // widest sketch of the learned-rank rounding (0: exact only)
};

void add64(int64_t& off, int64_t& field_off, int64_t cap) {
  field_off = off;
  off += (cap + 31) & ~(int64_t)31;   // 256-byte aligned sub-buffers
}

// Fills the engine layout for the roundings in p and returns the per-shot stride.
void layout_engine(const Plan& p, EngineLayout& L) {
  const int K = p.K, n = p.half;
  std::memset(&L, 0, sizeof(L));
  int64_t capX = 1, capX2 = 1, capR = 1, capM = 2, capUS = 1, capSA = 2, capSJ = 1,
          capQRS = 1, capQRT = 1, capSA2 = 1, capQRS2 = 1, capQRT2 = 1, capVp = 1, capYv = 1;
  std::vector<int64_t> capIn(K, 1), capQ(K, 1), capQT(K, 1);
  int maxdim = 1;
  for (const auto& s : p.sw) {
    for (int k = 0; k < K; ++k) {
      if (s.explicit_in) capIn[k] = std::max(capIn[k], s.rin[k] * 2 * s.rin[k + 1]);
      if (k <= K - 2) {
        capQ[k] = std::max(capQ[k], 2 * s.rt[k] * s.rin[k + 1]);
        capQT[k] = std::max(capQT[k], (s.rin[k + 1] + 16) * 16);
        capX = std::max(capX, 2 * s.rt[k] * s.rin[k + 1]);
        capR = std::max(capR, s.rt[k + 1] * s.rin[k + 1]);
      }
      capR = std::max(capR, s.rt[k] * s.rin[k]);
      if (k >= 1) {
        capM = std::max(capM, s.rt[k] * 2 * s.rho[k + 1]);
        capUS = std::max(capUS, s.rt[k] * s.rho[k]);
        capSA = std::max(capSA, s.rt[k] * 2 * s.rho[k + 1]);
        capQRS = std::max(capQRS, s.rt[k] * 2 * s.rho[k + 1]);
        capQRT = std::max(capQRT, (2 * s.rho[k + 1] + 16) * 16);
        const int64_t cc = std::min(s.rt[k], 2 * s.rho[k + 1]);
        capSA2 = std::max(capSA2, cc * cc);
        capQRS2 = std::max(capQRS2, cc * cc);
        capQRT2 = std::max(capQRT2, (cc + 16) * 16);
        capVp = std::max(capVp, s.rho[k] * cc);
        capYv = std::max(capYv, 2 * s.rho[k + 1] * s.rho[k]);
        maxdim = (int)std::max<int64_t>(maxdim, std::max(s.rt[k], 2 * s.rho[k + 1]));
      }
      capM = std::max(capM, 2 * s.rho[1]);
    }
  }
  int64_t capVL = 1, capWR = 1;
  if (p.kron) {   // the c^2 rounding (listed last): y's two halves and the middle unfolding
    const auto& s = p.sw.back();
    for (int k = 0; k <= n; ++k) capVL = std::max(capVL, p2(k) * p.Rmax[k]);
    for (int k = n; k <= K; ++k) capWR = std::max(capWR, p.Rmax[k] * p2(K - k));
    capX2 = 2 * s.rt[n - 1] * p2(K - n);
  }
  int64_t off = 0;
  for (int k = 0; k < K; ++k) { L.cap_in[k] = capIn[k]; add64(off, L.off_in[k], capIn[k]); }
  for (int k = 0; k < K; ++k) { L.cap_q[k] = capQ[k]; add64(off, L.off_q[k], capQ[k]); }
  for (int k = 0; k < K; ++k) { L.cap_qt[k] = capQT[k]; add64(off, L.off_qt[k], capQT[k]); }
  L.cap_X = capX; add64(off, L.off_X, capX);
  L.cap_X2 = capX2; add64(off, L.off_X2, capX2);
  L.cap_R = capR; add64(off, L.off_R, capR);
  L.cap_VL = capVL; add64(off, L.off_VL0, capVL); add64(off, L.off_VL1, capVL);
  L.cap_WR = capWR; add64(off, L.off_WR0, capWR); add64(off, L.off_WR1, capWR);
  L.cap_M = capM; add64(off, L.off_M, capM);
  L.cap_US = capUS; add64(off, L.off_US, capUS);
  L.cap_sA = capSA; add64(off, L.off_sA, capSA);
  L.cap_sJ = capSJ; add64(off, L.off_sJ, capSJ);
  L.cap_sA2 = capSA2; add64(off, L.off_sA2, capSA2);
  L.cap_qrS2 = capQRS2; add64(off, L.off_qrS2, capQRS2);
  L.cap_qrT2 = capQRT2; add64(off, L.off_qrT2, capQRT2);
  L.cap_Vp = capVp; add64(off, L.off_Vp, capVp);
  L.cap_Yv = capYv; add64(off, L.off_Yv, capYv);
  L.cap_perm = 4096; add64(off, L.off_perm, 4096);
  if (p.rrf_l > 0) {   // the sketch bases reuse the Householder buffers
    int64_t mx = 1;
    for (const auto& s : p.sw)
      for (int k = 1; k < K; ++k) mx = std::max(mx, std::max(s.rt[k], 2 * s.rho[k + 1]));
    capQRS = std::max(capQRS, mx * p.rrf_l);
    capQRT = std::max(capQRT, (p.rrf_l + 16) * 16);
  }
  L.cap_qrS = capQRS; add64(off, L.off_qrS, capQRS);
  L.cap_qrT = capQRT; add64(off, L.off_qrT, capQRT);
  if (p.rrf_l > 0) {   // randomized range finder buffers
    int64_t mrt = 1, m2r = 1, mchi = 1;
    for (const auto& s : p.sw)
      for (int k = 1; k < K; ++k) {
        mrt = std::max(mrt, s.rt[k]);
        m2r = std::max(m2r, 2 * s.rho[k + 1]);
        mchi = std::max(mchi, s.rho[k]);
      }
    L.cap_Om = mrt * p.rrf_l; add64(off, L.off_Om, L.cap_Om);
    L.cap_Ys = m2r * p.rrf_l; add64(off, L.off_Ys, L.cap_Ys);
    L.cap_Zs = mrt * p.rrf_l; add64(off, L.off_Zs, L.cap_Zs);
    L.cap_Mb = capM; add64(off, L.off_Mb, capM);
    L.cap_Tc = mchi * m2r; add64(off, L.off_Tc, L.cap_Tc);
    L.cap_Rz = capM; add64(off, L.off_Rz, capM);
  }
  L.stride = off;
  L.maxdim = maxdim;
}

// Launch grids per op and site, from the capacity bonds of each rounding.
struct Grids {
  // [rounding][site]
  std::vector<std::vector<int>> l2r, copyrx, absorb;
  std::vector<int> kl1_t, kl1_b, kl2_t, kl2_b, kr1_t, kr2_t, kr2_b;
  int meet = 0;
};

// ---------------------------------------------------------------------------
// The state
// ---------------------------------------------------------------------------
struct Engine {
  DevCtx h{};            // host mirror of the device context
  DevCtx* d = nullptr;   // device copy
  double* eng = nullptr;
  Plan plan;
  std::vector<SweepCaps> sw;
};

}  // namespace

struct mpsw_state_s {
  // n bits per axis, ndim axes, K = ndim n sites; the two sweeps of the
  // Kronecker rounding meet at site half = K / 2
  int B = 1, n = 0, K = 0, ndim = 2, half = 0;
  std::vector<mpsw_config> cfg;
  hipStream_t stream = nullptr;
  int chi_cap = 1;
  LapMPO lap;
  // device allocations
  double* mps = nullptr;
  int* dims = nullptr;
  double* reals = nullptr;
  double* c2 = nullptr;
  double* c2d = nullptr;   // c^2 as a dense field in site order (the middle unfolding of the c^2 rounding)
  double* lapW = nullptr;
  double* wavelet = nullptr;
  double* dense = nullptr;
  int* err = nullptr;
  int* sync = nullptr;
  std::vector<int> c2b;
  int nt_max = 0;
  std::vector<std::vector<double>> wavelets;
  Engine eng;              // step engine (after the velocity is known)
  bool have_velocity = false;
  int cur = 0, prev = 1, nxt = 2;
  int64_t step = 0;
  std::vector<int64_t> Rmax;
  int64_t mps_stride = 0;
  int64_t off_mps[MPSW_NSLOT][MPSW_MAXK];
  int64_t cap_mps[MPSW_NSLOT][MPSW_MAXK];
  Grids g;
  // captured steps: one graph of three steps (a full turn of the psi slot
  // rotation) per rotation phase, replayed by mpsw_step in graph mode
  int gemm_mode = 0;                   // GemmMode of the step's contractions
  int tune_qr_nwg = 32;                // most workgroups per shot of a QR factorisation
  int tune_jac_b = 0;                  // Jacobi block width (0: rule from the column count)
  bool learned = false;                // sketched rounding (rank network or previous rank + sketch)
  bool rank_prev = false;              // the sketch rank is the previous step's, no network
  float* mlp_w = nullptr;              // rank network parameters on the device
  bool have_model = false;
  bool graph_mode = false;
  int engine_gen = 0;                  // bumped whenever the step engine is rebuilt
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec[3] = {nullptr, nullptr, nullptr};
  // device memory: the caller's allocator (torch's caching allocator, an
  // arena) when one was given at creation, else hipMalloc / hipFree
  mpsw_allocator alloc{};
  bool has_alloc = false;
  std::unordered_map<void*, size_t> alloc_sizes;
  // event timing of one kernel class (mpsw_profile)
  int prof_cls = -1;
  std::vector<hipEvent_t> prof_ev;
  size_t prof_used = 0;
};

// Device allocations of a state go through the caller's allocator if it gave one.
template <class T>
hipError_t st_malloc(mpsw_state st, T** p, size_t bytes) {
  *p = nullptr;
  if (st == nullptr || !st->has_alloc) return hipMalloc((void**)p, bytes);
  void* q = st->alloc.alloc(std::max<size_t>(bytes, 1), st->alloc.ctx);
  if (q == nullptr) return hipErrorOutOfMemory;
  st->alloc_sizes[q] = bytes;
  *p = (T*)q;
  return hipSuccess;
}

void st_free(mpsw_state st, void* p) {
  if (p == nullptr) return;
  // teardown: a failing free or synchronisation leaves nothing to undo, so
  // their status is dropped here (and below) on purpose
  if (st == nullptr || !st->has_alloc) {
    (void)hipFree(p);
    return;
  }
  // the caller may hand the block to other work at once: nothing of this
  // state's may still be using it
  if (st->stream) (void)hipStreamSynchronize(st->stream);
  else (void)hipDeviceSynchronize();
  auto it = st->alloc_sizes.find(p);
  const size_t bytes = (it != st->alloc_sizes.end()) ? it->second : 0;
  if (it != st->alloc_sizes.end()) st->alloc_sizes.erase(it);
  st->alloc.free(p, bytes, st->alloc.ctx);
}

static void drop_graphs(mpsw_state st) {
  for (int i = 0; i < 3; ++i)
    if (st->gexec[i]) {
      (void)hipGraphExecDestroy(st->gexec[i]);
      st->gexec[i] = nullptr;
    }
}

namespace {

int check_dev_err(mpsw_state st) {
  int e = 0;
  HIP_TRY(hipMemcpyAsync(&e, st->err, sizeof(int), hipMemcpyDeviceToHost, st->stream));
  HIP_TRY(hipStreamSynchronize(st->stream));
  if (e & MPSW_DEV_ERR_NONFINITE) return fail(MPSW_ENONFINITE, "non-finite singular value encountered");
  if (e & (MPSW_DEV_ERR_CAP | MPSW_DEV_ERR_GRID))
    return fail(MPSW_ENOMEM, "a live size exceeded the workspace (device error bits " + std::to_string(e) + ")");
  if (e & MPSW_DEV_ERR_TIMEOUT)
    return fail(MPSW_EHIP, "a bounded inter-workgroup wait gave up (device error bits " + std::to_string(e) + ")");
  return MPSW_OK;
}

// Brackets the launches of kernel class `cls` with events when it is the
// timed class.
template <class F>
void prof(mpsw_state st, int cls, hipStream_t s, F&& launch) {
  if (st->prof_cls != cls) {
    launch();
    return;
  }
  while (st->prof_ev.size() < st->prof_used + 2) {
    hipEvent_t ev;
    if (hipEventCreate(&ev) != hipSuccess) {
      launch();
      return;
    }
    st->prof_ev.push_back(ev);
  }
  // a failed record surfaces when mpsw_profile_read reads the pair
  (void)hipEventRecord(st->prof_ev[st->prof_used], s);
  launch();
  (void)hipEventRecord(st->prof_ev[st->prof_used + 1], s);
  st->prof_used += 2;
}

// device context for the main (step) engine
void fill_ctx(mpsw_state st, DevCtx& h, double* eng, const EngineLayout& L) {
  std::memset(&h, 0, sizeof(h));
  h.K = st->K;
  h.n = st->n;
  h.ndim = st->ndim;
  h.half = st->half;
  h.B = st->B;
  h.boundary = st->cfg[0].boundary;
  h.ordering = st->cfg[0].ordering;
  h.lam2 = st->cfg[0].lambda * st->cfg[0].lambda;
  h.mps_stride = st->mps_stride;
  h.mps = st->mps;
  std::memcpy(h.off_mps, st->off_mps, sizeof(h.off_mps));
  std::memcpy(h.cap_mps, st->cap_mps, sizeof(h.cap_mps));
  h.dims = st->dims;
  h.reals = st->reals;
  h.eng = eng;
  h.L = L;
  h.c2 = st->c2;
  h.c2d = st->c2d;
  int64_t off = 0;
  for (int k = 0; k < st->K && !st->c2b.empty(); ++k) {
    h.off_c2[k] = off;
    off += (int64_t)st->c2b[k] * 2 * st->c2b[k + 1];
  }
  for (int k = 0; k <= st->K; ++k) h.c2b[k] = st->c2b.empty() ? 1 : st->c2b[k];
  h.lapW = st->lapW;
  int woff = 0;
  for (int k = 0; k < st->K; ++k) {
    h.off_W[k] = woff;
    woff += st->lap.bonds[k] * st->lap.bonds[k + 1] * 4;
  }
  for (int k = 0; k <= st->K; ++k) h.wb[k] = st->lap.bonds[k];
  h.wavelet = st->wavelet;
  h.nt_max = st->nt_max;
  h.dense = st->dense;
  h.dense_stride = 2 * p2(st->K);
  h.err = st->err;
  h.sync = st->sync;
  h.mlp_w = st->mlp_w;
  h.seed = (unsigned long long)st->cfg[0].seed;
  h.rrf_over = MPSW_RRF_OVER;
  h.rank_prev = st->rank_prev ? 1 : 0;
}

int upload_ctx(Engine& e, hipStream_t s, mpsw_state st = nullptr) {
  if (!e.d) HIP_TRY(st_malloc(st, &e.d, sizeof(DevCtx)));
  HIP_TRY(hipMemcpyAsync(e.d, &e.h, sizeof(DevCtx), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return MPSW_OK;
}


size_t g_lds_limit = 0;   // bytes of LDS a workgroup may allocate on this device

size_t lds_limit() {
  if (g_lds_limit == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) v = 65536;
    g_lds_limit = (size_t)v;
    set_lds_limits(g_lds_limit);
    (void)hipGetLastError();   // the attribute is advisory on this platform; clear any status it left
  }
  return g_lds_limit;
}

// Householder panel width for a QR whose row count is at most mcap: the panel
// ((mcap + 1) x bw doubles: one spare row for an odd leading dimension) lives
// in LDS.
int qr_panel(int64_t mcap) {
  const size_t lim = lds_limit() - 24576;   // static LDS of the kernel
  for (int bw = 16; bw >= 4; bw >>= 1)
    if ((size_t)(mcap + 1) * bw * 8 <= lim) return bw;
  return 0;
}

// Jacobi block width for columns of length at most lcap: a block pair
// (2 bw columns of lcap+1 doubles) lives in LDS.
// About 16 blocks per sweep spread a sweep over 8 workgroups; every block
// pair's rotations are a sequence of b-wide steps, so smaller blocks only add
// rounds (and barriers) without shortening the sequence.
int jac_block(int64_t lcap, int prefer = 0) {
  const size_t lim = lds_limit() - 1024;   // static LDS of the kernel
  int want = 4;   // 32 groups of 16 lanes: at most 32 pairs per step
  while (want < 16 && want * 16 < lcap) want <<= 1;
  if (prefer >= 1 && prefer <= 32) want = prefer;   // autotuned
  for (int b = want; b >= 1; b >>= 1)
    if ((size_t)2 * b * (jac_rows(lcap) + 1) * 8 <= lim) return b;
  return 0;
}

// ---------------------------------------------------------------------------
// Rounding launch sequences
// ---------------------------------------------------------------------------
enum Kind { K_LAPLACE = 0, K_C2 = 1, K_SUM = 2, K_DENSE = 3 };

// Every factorisation of a rounding with these capacities fits the LDS of
// one workgroup (panel of the QR, block pair of the Jacobi sweep).
int check_fits(const SweepCaps& s, int K) {
  for (int k = 0; k + 1 < K; ++k)
    if (qr_panel(2 * s.rt[k]) == 0) return fail(MPSW_ENOMEM, "QR panel exceeds the LDS of a workgroup");
  for (int k = K - 1; k >= 1; --k) {
    if (qr_panel(std::max(s.rt[k], 2 * s.rho[k + 1])) == 0 || qr_panel(std::min(s.rt[k], 2 * s.rho[k + 1])) == 0)
      return fail(MPSW_ENOMEM, "QR panel exceeds the LDS of a workgroup");
    if (jac_block(std::min(s.rt[k], 2 * s.rho[k + 1])) == 0)
      return fail(MPSW_ENOMEM, "Jacobi block exceeds the LDS of a workgroup");
  }
  return MPSW_OK;
}

// L->R sweep then R->L sweep for one rounding; output into MPS slot out_slot.
void run_rounding(mpsw_state st, Engine& e, int kind, const SweepCaps& s, int out_slot, int log_idx,
                  int slot_a, int slot_b, int step, int nshots, hipStream_t strm) {
  const int K = st->K, n = st->half;
  const DevCtx* d = e.d;
  // contractions of a time step run in the state's precision; set-up (dense
  // fields to MPS) always in FP64
  const int gmode = (kind == K_DENSE) ? GEMM_FP64 : st->gemm_mode;
  OpArgs a{};
  a.shot = -1;
  a.aux = log_idx;
  a.slot = slot_a;
  a.slot2 = slot_b;
  a.step = step;
  a.op = (kind == K_LAPLACE) ? P_LAPLACE : (kind == K_C2) ? P_C2 : (kind == K_SUM) ? P_SUM : P_DENSE;
  launch_prepare(d, a, nshots, strm);
  if (kind == K_LAPLACE) {
    int64_t mx = 1;
    for (int k = 0; k < K; ++k) mx = std::max(mx, s.rin[k] * 2 * s.rin[k + 1]);
    launch_pack_lap(d, a, K, nshots, std::min<int64_t>(1024, cdiv(mx, 256)), strm);
  } else if (kind == K_SUM) {
    int64_t mx = 1;
    for (int k = 0; k < K; ++k) mx = std::max(mx, s.rin[k] * 2 * s.rin[k + 1]);
    launch_pack_sum(d, a, K, nshots, std::min<int64_t>(1024, cdiv(mx, 256)), strm);
  }
  launch_init_R(d, a, nshots, strm);

  const auto& R = st->Rmax;
  if (kind == K_C2) {
    // the halves of y, for the Hadamard product's middle unfolding
    for (int k = K - 1; k >= n; --k) {
      OpArgs g{};
      g.mode = gmode;
      g.shot = -1;
      g.site = k;
      g.op = G_HALF_R;
      prof(st, MPSW_KC_GEMM, strm, [&] { launch_gemm(d, g, 2 * R[k], p2(K - k - 1), 1, nshots, strm); });
    }
    for (int k = 0; k < n; ++k) {
      OpArgs g{};
      g.mode = gmode;
      g.shot = -1;
      g.site = k;
      g.op = G_HALF_L;
      prof(st, MPSW_KC_GEMM, strm, [&] { launch_gemm(d, g, p2(k), 2 * R[k + 1], 1, nshots, strm); });
    }
  }
  for (int k = 0; k < K; ++k) {
    OpArgs g{};
    g.mode = gmode;
    g.shot = -1;
    g.site = k;
    const bool last = (k == K - 1);
    bool meet = false;
    if (kind == K_LAPLACE || kind == K_SUM) {
      g.op = G_L2R_EXPLICIT;
      g.aux = last ? 1 : 0;
      prof(st, MPSW_KC_GEMM, strm, [&] { launch_gemm(d, g, s.rt[k], 2 * s.rin[k + 1], 1, nshots, strm); });
    } else if (kind == K_C2 && k < n) {
      if (k < n - 1) continue;   // the identity merges of sites 0..n-2 were set by k_prepare
      g.op = G_MEET_H;
      prof(st, MPSW_KC_GEMM, strm, [&] { launch_gemm(d, g, p2(n), p2(K - n), 1, nshots, strm); });
      meet = true;
    } else {
      g.op = G_COPY_RX;
      g.aux = last ? 1 : 0;
      prof(st, MPSW_KC_GEMM, strm, [&] { launch_gemm(d, g, s.rt[k], s.rin[k], 1, nshots, strm); });
    }
    if (!last) {
      const int64_t mcap = 2 * s.rt[k], ncap = s.rin[k + 1];
      const int bw = qr_panel(mcap);
      const int nwg = (int)std::min<int64_t>(st->tune_qr_nwg, std::max<int64_t>(1, cdiv(ncap, bw)));
      OpArgs q{};
      q.shot = -1;
      q.site = k;
      q.op = 0;
      q.aux = meet ? 1 : 0;
      launch_sync_reset(d, nshots, strm);
      prof(st, MPSW_KC_QR, strm, [&] { launch_qrf(d, q, bw, nwg, nshots, (size_t)mcap * bw * 8, strm); });
    }
  }
  const bool learned = st->learned && kind != K_DENSE && e.plan.rrf_l > 0;
  for (int k = K - 1; k >= 1; --k) {
    // SVD stage of the bond matrix M (rt_k x ncols): QR preconditioning,
    // Jacobi, truncation, V, U Sigma = M V.  `ncap` bounds the column count.
    auto svd_stage = [&](int gate, int64_t ncap) {
      const int64_t rows = std::max(s.rt[k], ncap);   // rows of the factored orientation
      const int64_t ccap = std::min(s.rt[k], ncap);
      OpArgs v{};
      v.shot = -1;
      v.site = k;
      v.slot = out_slot;
      v.aux = log_idx;
      v.gate = gate;
      launch_sync_reset(d, nshots, strm);
      const int bw1 = qr_panel(rows), bw2 = qr_panel(ccap);
      OpArgs q = v;
      q.op = 1;
      prof(st, MPSW_KC_QR, strm, [&] { launch_qrf(d, q, bw1, (int)std::min<int64_t>(st->tune_qr_nwg, std::max<int64_t>(1, cdiv(ccap, bw1))), nshots,
                 (size_t)rows * bw1 * 8, strm); });
      q.op = 2;
      prof(st, MPSW_KC_QR, strm, [&] { launch_qrf(d, q, bw2, (int)std::min<int64_t>(st->tune_qr_nwg, std::max<int64_t>(1, cdiv(ccap, bw2))), nshots,
                 (size_t)ccap * bw2 * 8, strm); });
      const int b = jac_block(ccap, st->tune_jac_b);
      const int64_t nb = cdiv(ccap, b);
      // workgroups per shot: one per block pair of a round, at most the QR's
      // tuned count (a large batch fills the chip with one per shot)
      const int jnwg = (int)std::max<int64_t>(1, std::min<int64_t>(st->tune_qr_nwg, (nb + (nb & 1)) / 2));
      prof(st, MPSW_KC_JACOBI, strm, [&] { launch_jac(d, v, b, jnwg, nshots, (size_t)2 * b * (ccap + 1) * 8, ccap, strm); });
      launch_jacfin(d, v, nshots, strm);
      prof(st, MPSW_KC_APPLYV, strm, [&] { launch_applyv(d, v, bw1, std::max(1, cdiv(s.rho[k], 16)), nshots, strm); });
      OpArgs g{};
      g.mode = gmode;
      g.gate = gate;
      g.shot = -1;
      g.site = k;
      g.slot = out_slot;
      g.op = G_US;
      prof(st, MPSW_KC_GEMM, strm, [&] { launch_gemm(d, g, s.rt[k], s.rho[k], 1, nshots, strm); });
    };
    const int64_t n2cap = 2 * s.rho[k + 1];
    if (learned) {
      // randomized range finder at the width the rank network proposes
      const int64_t lcap = std::min<int64_t>(e.plan.rrf_l, n2cap);
      OpArgs r{};
      r.shot = -1;
      r.site = k;
      r.slot = out_slot;
      r.aux = log_idx;
      r.gate = GATE_SKETCH;
      launch_rrf_plan(d, r, nshots, strm);
      launch_gauss(d, r, s.rt[k] * lcap, nshots, strm);
      OpArgs g{};
      g.mode = gmode;
      g.gate = GATE_SKETCH;
      g.shot = -1;
      g.site = k;
      auto orth = [&](int which, int64_t mcap) {   // Q of Y (0) or Z (1), in place
        OpArgs q = r;
        q.op = 3;
        q.aux = which;
        const int bw = qr_panel(mcap);
        launch_sync_reset(d, nshots, strm);
        prof(st, MPSW_KC_QR, strm, [&] { launch_qrf(d, q, bw, (int)std::min<int64_t>(st->tune_qr_nwg, std::max<int64_t>(1, cdiv(lcap, bw))), nshots,
                   (size_t)mcap * bw * 8, strm); });
        prof(st, MPSW_KC_APPLYQ, strm, [&] { launch_formq(d, q, bw, std::max(1, cdiv(lcap, 16)), nshots, strm); });
      };
      g.op = G_RRF_Y;
      g.aux = 0;
      prof(st, MPSW_KC_GEMM, strm, [&] { launch_gemm(d, g, n2cap, lcap, 1, nshots, strm); });
      orth(0, n2cap);
      g.op = G_RRF_Z;
      prof(st, MPSW_KC_GEMM, strm, [&] { launch_gemm(d, g, s.rt[k], lcap, 1, nshots, strm); });
      orth(1, s.rt[k]);
      g.op = G_RRF_Y;
      g.aux = 1;
      prof(st, MPSW_KC_GEMM, strm, [&] { launch_gemm(d, g, n2cap, lcap, 1, nshots, strm); });
      orth(0, n2cap);
      g.op = G_RRF_Z;   // B = M Q
      prof(st, MPSW_KC_GEMM, strm, [&] { launch_gemm(d, g, s.rt[k], lcap, 1, nshots, strm); });
      launch_rrf_swap(d, r, s.rt[k] * n2cap, nshots, strm);
      svd_stage(GATE_SKETCH, lcap);
      // the residual M - B Q^T in FP64 whatever the contraction precision
      g.op = G_RRF_RES;
      g.mode = GEMM_FP64;
      prof(st, MPSW_KC_GEMM, strm, [&] { launch_gemm(d, g, s.rt[k], n2cap, 1, nshots, strm); });
      g.mode = gmode;
      launch_rrf_resid(d, r, nshots, strm);
      launch_rrf_accept(d, r, s.rt[k] * n2cap, nshots, strm);
      svd_stage(GATE_EXACT, n2cap);
      g.op = G_RRF_CORE;
      g.gate = GATE_ACCEPTED;
      g.slot = out_slot;
      prof(st, MPSW_KC_GEMM, strm, [&] { launch_gemm(d, g, s.rho[k], n2cap, 1, nshots, strm); });
      OpArgs cr = r;
      cr.gate = GATE_ACCEPTED;
      launch_rrf_core(d, cr, s.rho[k] * n2cap, nshots, strm);
    } else {
      svd_stage(GATE_ALWAYS, n2cap);
    }
    OpArgs ap{};
    ap.shot = -1;
    ap.site = k;
    const int bwq = qr_panel(2 * s.rt[k - 1]);
    // the 16-column tile of M in LDS when it fits beside the reflector workspace
    const int64_t mq = 2 * s.rt[k - 1];
    if ((size_t)(16 * 256 + 256 + 16 * mq) * sizeof(double) <= lds_limit()) ap.aux = (int)mq;   // 16 * 256 + 256: the reflector workspace
    prof(st, MPSW_KC_APPLYQ, strm, [&] { launch_applyq(d, ap, bwq, std::max(1, cdiv(s.rho[k], 16)), nshots, strm); });
  }
  OpArgs f{};
  f.shot = -1;
  f.slot = out_slot;
  f.aux = (kind == K_SUM) ? 1 : 0;   // the sum rounding ends a time step
  launch_finish(d, f, nshots, strm);
}

std::vector<int64_t> state_rmax(int K, int64_t chi) {
  std::vector<int64_t> r(K + 1);
  for (int k = 0; k <= K; ++k) r[k] = std::min({chi, p2(k), p2(K - k)});
  return r;
}

// Dense field(s) -> MPS by the right-to-left truncated TT-SVD, run on a
// temporary single-shot engine.  out_slot of shot `shot` of st receives the
// result when to_velocity is false; otherwise the cores become the c^2 operator.
int dense_to_mps(mpsw_state st, const double* host_field, double eps, int64_t chi, int shot, int out_slot,
                 bool to_velocity) {
  const int K = st->K;
  const int64_t N = p2(K);
  // temporary group-like context with one shot
  std::vector<int64_t> rin(K + 1);
  for (int k = 0; k <= K; ++k) rin[k] = p2(K - k);
  SweepCaps s = sweep_caps(rin, K, chi);
  Plan p;
  p.K = K;
  p.half = st->half;
  p.sw = {s};
  EngineLayout L;
  layout_engine(p, L);
  // one output slot with caps from the rho bounds
  int64_t mps_stride = 0;
  int64_t offs[MPSW_MAXK], caps[MPSW_MAXK];
  for (int k = 0; k < K; ++k) {
    caps[k] = s.rho[k] * 2 * s.rho[k + 1];
    if (k == 0) caps[k] = 2 * s.rho[1];
    offs[k] = mps_stride;
    mps_stride += (caps[k] + 31) & ~(int64_t)31;
  }
  double *eng = nullptr, *mps = nullptr, *dense = nullptr, *reals = nullptr;
  int* dims = nullptr;
  int rc = MPSW_OK;
  auto cleanup = [&]() {
    st_free(st, eng);
    st_free(st, mps);
    st_free(st, dense);
    st_free(st, reals);
    st_free(st, dims);
  };
  if (st_malloc(st, &eng, L.stride * sizeof(double)) != hipSuccess ||
      st_malloc(st, &mps, mps_stride * sizeof(double)) != hipSuccess ||
      st_malloc(st, &dense, 2 * N * sizeof(double)) != hipSuccess ||
      st_malloc(st, &reals, RL::size * sizeof(double)) != hipSuccess ||
      st_malloc(st, &dims, DL::size * sizeof(int)) != hipSuccess) {
    cleanup();
    return fail(MPSW_ENOMEM, "dense_to_mps: device allocation failed");
  }
  Engine e;
  DevCtx& h = e.h;
  std::memset(&h, 0, sizeof(h));
  h.K = K;
  h.n = st->n;
  h.ndim = st->ndim;
  h.half = st->half;
  h.B = 1;
  h.mps = mps;
  h.mps_stride = mps_stride;
  for (int k = 0; k < K; ++k) { h.off_mps[0][k] = offs[k]; h.cap_mps[0][k] = caps[k]; }
  h.dims = dims;
  h.reals = reals;
  h.eng = eng;
  h.L = L;
  for (int k = 0; k <= K; ++k) { h.c2b[k] = 1; h.wb[k] = 1; }
  h.dense = dense;
  h.dense_stride = 2 * N;
  h.err = st->err;
  h.sync = st->sync;
  std::vector<int> hd(DL::size, 0);
  hd[DL::chi] = (int)std::min<int64_t>(chi, 1 << 30);
  std::vector<double> hr(RL::size, 0.0);
  hr[RL::eps] = eps;
  hipStream_t s0 = st->stream;
  std::vector<double> sites;   // the field in site order (interleaved states)
  if (st->cfg[0].ordering == MPSW_INTERLEAVED) {
    sites.resize(N);
    field_to_sites(host_field, st->n, st->ndim, sites.data());
    host_field = sites.data();
  }
  if (hipMemcpyAsync(dims, hd.data(), DL::size * sizeof(int), hipMemcpyHostToDevice, s0) != hipSuccess ||
      hipMemcpyAsync(reals, hr.data(), RL::size * sizeof(double), hipMemcpyHostToDevice, s0) != hipSuccess ||
      hipMemcpyAsync(dense, host_field, N * sizeof(double), hipMemcpyHostToDevice, s0) != hipSuccess) {
    cleanup();
    return fail(MPSW_EHIP, "dense_to_mps: upload failed");
  }
  if ((rc = upload_ctx(e, s0, st)) != MPSW_OK) { cleanup(); return rc; }
  if ((rc = check_fits(s, K)) != MPSW_OK) { cleanup(); st_free(st, e.d); return rc; }
  // swap in the temporary engine: run_rounding uses st only for K/n/c2b/Rmax
  run_rounding(st, e, K_DENSE, s, 0, -1, 0, 0, 0, 1, s0);
  {
    const hipError_t le = hipGetLastError();
    if (le != hipSuccess) {
      cleanup();
      st_free(st, e.d);
      return fail(MPSW_EHIP, std::string("dense_to_mps: launch failed: ") + hipGetErrorString(le) +
                                 " (LDS limit " + std::to_string(lds_limit()) + ")");
    }
  }
  if ((rc = check_dev_err(st)) != MPSW_OK) { cleanup(); st_free(st, e.d); return rc; }
  // bonds of the result
  std::vector<int> dd(DL::size);
  hipError_t herr = hipMemcpy(dd.data(), dims, DL::size * sizeof(int), hipMemcpyDeviceToHost);
  if (herr != hipSuccess) { cleanup(); st_free(st, e.d); return fail(MPSW_EHIP, std::string("dense_to_mps: ") + hipGetErrorString(herr)); }
  auto chk = [&](hipError_t x) { if (herr == hipSuccess) herr = x; };
  std::vector<int> bonds(K + 1);
  for (int k = 0; k <= K; ++k) bonds[k] = dd[DL::bonds + k];
  if (to_velocity) {
    int64_t tot = 0;
    for (int k = 0; k < K; ++k) tot += (int64_t)bonds[k] * 2 * bonds[k + 1];
    st_free(st, st->c2);
    st->c2 = nullptr;
    if (st_malloc(st, &st->c2, tot * sizeof(double)) != hipSuccess) { cleanup(); st_free(st, e.d); return fail(MPSW_ENOMEM, "c2 alloc"); }
    int64_t o = 0;
    for (int k = 0; k < K; ++k) {
      const int64_t sz = (int64_t)bonds[k] * 2 * bonds[k + 1];
      chk(hipMemcpyAsync(st->c2 + o, mps + offs[k], sz * sizeof(double), hipMemcpyDeviceToDevice, s0));
      o += sz;
    }
    st->c2b = bonds;
  } else {
    for (int k = 0; k < K; ++k) {
      const int64_t sz = (int64_t)bonds[k] * 2 * bonds[k + 1];
      if (sz > st->cap_mps[out_slot][k]) { cleanup(); st_free(st, e.d); return fail(MPSW_ENOMEM, "field rank exceeds chi_max caps"); }
      chk(hipMemcpyAsync(st->mps + shot * st->mps_stride + st->off_mps[out_slot][k], mps + offs[k], sz * sizeof(double),
                         hipMemcpyDeviceToDevice, s0));
    }
    // bonds into the main dims block
    chk(hipMemcpyAsync(st->dims + (int64_t)shot * DL::size + DL::bonds + out_slot * (MPSW_MAXK + 1), bonds.data(),
                       (K + 1) * sizeof(int), hipMemcpyHostToDevice, s0));
  }
  chk(hipStreamSynchronize(s0));
  cleanup();
  st_free(st, e.d);
  if (herr != hipSuccess) return fail(MPSW_EHIP, std::string("dense_to_mps: ") + hipGetErrorString(herr));
  return MPSW_OK;
}

int contract_dense(mpsw_state st, int shot, int slot, std::vector<double>& out);

// c^2 as a dense field in site order, contracted from its operator cores.
int upload_c2_dense(mpsw_state st, const std::vector<double>& v) {
  if (!st->c2d) HIP_TRY(st_malloc(st, &st->c2d, (size_t)p2(st->K) * sizeof(double)));
  HIP_TRY(hipMemcpy(st->c2d, v.data(), (size_t)p2(st->K) * sizeof(double), hipMemcpyHostToDevice));
  return MPSW_OK;
}

// Build the step engine once c^2 is known.
int build_step_engine(mpsw_state st) {
  drop_graphs(st);
  ++st->engine_gen;
  const int K = st->K, n = st->half;
  Engine& e = st->eng;
  if (e.eng) { st_free(st, e.eng); e.eng = nullptr; }
  const auto& R = st->Rmax;
  std::vector<int64_t> r1(K + 1), r2(K + 1), r3(K + 1);
  for (int k = 0; k <= K; ++k) {
    r1[k] = (int64_t)st->lap.bonds[k] * R[k];
    r2[k] = (k < n) ? p2(k) : p2(K - k);   // identity basis on the left, dense on the right
    r3[k] = (k == 0 || k == K) ? 1 : 3 * R[k] + 1;
  }
  e.sw = {sweep_caps(r1, K, st->chi_cap), sweep_caps(r3, K, st->chi_cap), sweep_caps(r2, K, st->chi_cap)};
  e.sw[0].explicit_in = true;
  e.sw[1].explicit_in = true;
  for (auto& s : e.sw) {
    const int rc = check_fits(s, K);
    if (rc != MPSW_OK) return rc;
  }
  e.plan.K = K;
  e.plan.half = n;
  e.plan.sw = e.sw;
  e.plan.Rmax = R;
  e.plan.D = st->c2b;
  e.plan.kron = true;
  e.plan.rrf_l = st->learned ? std::min<int64_t>(st->chi_cap + MPSW_RRF_OVER, MPSW_RRF_MAXL) : 0;
  EngineLayout L;
  layout_engine(e.plan, L);
  if (st_malloc(st, &e.eng, (size_t)L.stride * st->B * sizeof(double)) != hipSuccess)
    return fail(MPSW_ENOMEM, "step workspace allocation failed (" + std::to_string(L.stride * st->B * 8 / (1 << 20)) + " MiB)");
  fill_ctx(st, e.h, e.eng, L);
  return upload_ctx(e, st->stream, st);
}

int upload_lap(mpsw_state st) {
  std::vector<double> w;
  for (auto& c : st->lap.cores) w.insert(w.end(), c.begin(), c.end());
  HIP_TRY(st_malloc(st, &st->lapW, std::max<size_t>(1, w.size()) * sizeof(double)));
  HIP_TRY(hipMemcpy(st->lapW, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice));
  return MPSW_OK;
}

int create_group(const mpsw_config* cfgs, int nshots, void* stream, const mpsw_allocator* alloc, mpsw_state* out) {
  if (!cfgs || !out || nshots < 1) return fail(MPSW_EINVAL, "null argument or nshots < 1");
  if (alloc && (!alloc->alloc || !alloc->free)) return fail(MPSW_EINVAL, "allocator needs both alloc and free");
  const mpsw_config& c0 = cfgs[0];
  for (int i = 0; i < nshots; ++i) {
    const mpsw_config& c = cfgs[i];
    const int nd = c.ndim ? c.ndim : 2;
    if (nd != 2 && nd != 3) return fail(MPSW_EINVAL, "ndim must be 2 or 3");
    if (c.n < 1 || c.n * nd > 22) return fail(MPSW_EINVAL, "n must be in [1, 11] (two dimensions) or [1, 7] (three)");
    if (c.chi_max < 1) return fail(MPSW_EINVAL, "chi_max must be >= 1");
    if (!(c.eps >= 0.0) || !std::isfinite(c.eps)) return fail(MPSW_EINVAL, "eps must be finite and >= 0");
    if (!(c.lambda > 0.0) || !std::isfinite(c.lambda)) return fail(MPSW_EINVAL, "lambda must be > 0");
    if (c.precision != MPSW_FP64 && c.precision != MPSW_FP32 && c.precision != MPSW_BF16)
      return fail(MPSW_EINVAL, "unknown precision");
    if (c.boundary != MPSW_PERIODIC && c.boundary != MPSW_OPEN) return fail(MPSW_EINVAL, "unknown boundary");
    if (c.rank_mode != MPSW_RANK_EXACT && c.rank_mode != MPSW_RANK_LEARNED && c.rank_mode != MPSW_RANK_PREVIOUS)
      return fail(MPSW_EINVAL, "unknown rank mode");
    if (c.ordering != MPSW_SEQUENTIAL && c.ordering != MPSW_INTERLEAVED) return fail(MPSW_EINVAL, "unknown site order");
    if (c.n != c0.n || c.lambda != c0.lambda || c.precision != c0.precision || c.boundary != c0.boundary ||
        c.rank_mode != c0.rank_mode || c.ordering != c0.ordering || nd != (c0.ndim ? c0.ndim : 2))
      return fail(MPSW_EINVAL, "shots of one batch must share n, ndim, lambda, precision, boundary, rank mode and site order");
  }
  mpsw_state st = new mpsw_state_s();
  if (alloc) {
    st->alloc = *alloc;
    st->has_alloc = true;
  }
  st->B = nshots;
  st->gemm_mode = (c0.precision == MPSW_FP32) ? GEMM_FP32 : (c0.precision == MPSW_BF16) ? GEMM_BF16X6 : GEMM_FP64;
  st->learned = (c0.rank_mode != MPSW_RANK_EXACT);
  st->rank_prev = (c0.rank_mode == MPSW_RANK_PREVIOUS);
  st->n = c0.n;
  st->ndim = c0.ndim ? c0.ndim : 2;
  st->K = st->ndim * c0.n;
  st->half = st->K / 2;
  st->cfg.assign(cfgs, cfgs + nshots);
  st->stream = (hipStream_t)stream;
  st->chi_cap = 1;
  for (int i = 0; i < nshots; ++i) st->chi_cap = std::max(st->chi_cap, cfgs[i].chi_max);
  const int K = st->K;
  st->lap = build_laplacian_mpo(st->n, c0.boundary, c0.ordering, st->ndim);
  st->Rmax = state_rmax(K, st->chi_cap);
  // MPS slots
  int64_t off = 0;
  for (int s = 0; s < MPSW_NSLOT; ++s)
    for (int k = 0; k < K; ++k) {
      st->cap_mps[s][k] = std::max<int64_t>(2, st->Rmax[k] * 2 * st->Rmax[k + 1]);
      st->off_mps[s][k] = off;
      off += (st->cap_mps[s][k] + 31) & ~(int64_t)31;
    }
  st->mps_stride = off;
  int rc;
  auto bail = [&](int code) {
    mpsw_destroy(st);
    return code;
  };
  if (st_malloc(st, &st->mps, (size_t)st->mps_stride * nshots * sizeof(double)) != hipSuccess ||
      st_malloc(st, &st->dims, (size_t)DL::size * nshots * sizeof(int)) != hipSuccess ||
      st_malloc(st, &st->reals, (size_t)RL::size * nshots * sizeof(double)) != hipSuccess ||
      st_malloc(st, &st->err, sizeof(int)) != hipSuccess ||
      st_malloc(st, &st->sync, (size_t)MPSW_SYNC_STRIDE * nshots * sizeof(int)) != hipSuccess ||
      st_malloc(st, &st->dense, (size_t)2 * p2(K) * sizeof(double)) != hipSuccess)
    return bail(fail(MPSW_ENOMEM, "state allocation failed"));
  if ((rc = upload_lap(st)) != MPSW_OK) return bail(rc);
  std::vector<int> hd((size_t)DL::size * nshots, 0);
  std::vector<double> hr((size_t)RL::size * nshots, 0.0);
  for (int i = 0; i < nshots; ++i) {
    int* d = hd.data() + (size_t)i * DL::size;
    for (int s = 0; s < MPSW_NSLOT; ++s)
      for (int k = 0; k <= K; ++k) d[DL::bonds + s * (MPSW_MAXK + 1) + k] = 1;
    d[DL::chi] = cfgs[i].chi_max;
    hr[(size_t)i * RL::size + RL::eps] = cfgs[i].eps;
  }
  if (hipMemcpy(st->dims, hd.data(), hd.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(st->reals, hr.data(), hr.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(st->err, 0, sizeof(int)) != hipSuccess ||
      hipMemset(st->mps, 0, (size_t)st->mps_stride * nshots * sizeof(double)) != hipSuccess)
    return bail(fail(MPSW_EHIP, "state initialisation failed"));
  st->wavelets.assign(nshots, {});
  *out = st;
  return MPSW_OK;
}

int upload_wavelets(mpsw_state st) {
  int ntm = 1;
  for (auto& w : st->wavelets) ntm = std::max<int>(ntm, (int)w.size());
  std::vector<double> buf((size_t)ntm * st->B, 0.0);
  for (int i = 0; i < st->B; ++i) std::copy(st->wavelets[i].begin(), st->wavelets[i].end(), buf.begin() + (size_t)i * ntm);
  st_free(st, st->wavelet);
  st->wavelet = nullptr;
  HIP_TRY(st_malloc(st, &st->wavelet, buf.size() * sizeof(double)));
  HIP_TRY(hipMemcpy(st->wavelet, buf.data(), buf.size() * sizeof(double), hipMemcpyHostToDevice));
  st->nt_max = ntm;
  if (st->eng.eng) {
    st->eng.h.wavelet = st->wavelet;
    st->eng.h.nt_max = ntm;
    return upload_ctx(st->eng, st->stream, st);
  }
  return MPSW_OK;
}

// to_dense of shot `shot`: slot >= 0 or -1 for c^2.  Result in a host vector.
int contract_dense(mpsw_state st, int shot, int slot, std::vector<double>& out) {
  const int K = st->K;
  Engine& e = st->eng;
  Engine tmp;
  Engine* use = &e;
  if (!e.eng || slot < 0) {  // no engine yet, or the c^2 operator (which may just have changed): a fresh context
    EngineLayout L;
    std::memset(&L, 0, sizeof(L));
    fill_ctx(st, tmp.h, nullptr, L);
    int rc = upload_ctx(tmp, st->stream, st);
    if (rc != MPSW_OK) return rc;
    use = &tmp;
  }
  launch_dense_init(use->d, 1, st->stream);
  for (int k = 0; k < K; ++k) {
    OpArgs g{};
    g.op = G_DENSE;
    g.site = k;
    g.slot = slot;
    g.shot = shot;
    const int64_t r1 = (slot < 0) ? st->c2b[k + 1] : st->Rmax[k + 1];
    launch_gemm(use->d, g, p2(k), 2 * r1, 1, 1, st->stream);
  }
  out.resize(p2(K));
  const int64_t half = p2(K);
  const double* src = st->dense + (((K - 1) & 1) ? 0 : half);
  HIP_TRY(hipMemcpyAsync(out.data(), src, half * sizeof(double), hipMemcpyDeviceToHost, st->stream));
  int rc = check_dev_err(st);
  if (tmp.d) st_free(st, tmp.d);
  return rc;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* mpsw_last_error(void) { return g_last_error.c_str(); }

int mpsw_create_state(const mpsw_config* cfg, void* hip_stream, mpsw_state* out) {
  return create_group(cfg, 1, hip_stream, nullptr, out);
}

int mpsw_create_batch(const mpsw_config* cfgs, int nshots, void* hip_stream, mpsw_state* out) {
  return create_group(cfgs, nshots, hip_stream, nullptr, out);
}

int mpsw_create_batch_ex(const mpsw_config* cfgs, int nshots, void* hip_stream, const mpsw_allocator* alloc,
                         mpsw_state* out) {
  return create_group(cfgs, nshots, hip_stream, alloc, out);
}

int mpsw_get_cores(mpsw_state st, int shot, int which, int* bonds, double* cores, int64_t cap) {
  if (!st || !bonds) return fail(MPSW_EINVAL, "null argument");
  if (shot < 0 || shot >= st->B || which < 0 || which > 1) return fail(MPSW_EINVAL, "shot or field out of range");
  const int K = st->K, slot = which ? st->prev : st->cur;
  HIP_TRY(hipStreamSynchronize(st->stream));
  std::vector<int> dd(DL::size);
  HIP_TRY(hipMemcpy(dd.data(), st->dims + (int64_t)shot * DL::size, DL::size * sizeof(int), hipMemcpyDeviceToHost));
  int64_t tot = 0;
  for (int k = 0; k <= K; ++k) bonds[k] = dd[DL::bonds + slot * (MPSW_MAXK + 1) + k];
  for (int k = 0; k < K; ++k) tot += (int64_t)bonds[k] * 2 * bonds[k + 1];
  if (tot > INT32_MAX) return fail(MPSW_EINVAL, "cores exceed the int range");
  if (cores) {
    if (cap < tot) return fail(MPSW_EINVAL, "cores buffer too small (" + std::to_string(tot) + " doubles needed)");
    int64_t o = 0;
    for (int k = 0; k < K; ++k) {
      const int64_t sz = (int64_t)bonds[k] * 2 * bonds[k + 1];
      HIP_TRY(hipMemcpy(cores + o, st->mps + (int64_t)shot * st->mps_stride + st->off_mps[slot][k], sz * sizeof(double),
                        hipMemcpyDeviceToHost));
      o += sz;
    }
  }
  const int rc = check_dev_err(st);
  return rc == MPSW_OK ? (int)tot : rc;
}

int mpsw_set_cores(mpsw_state st, int shot, int64_t step, const int* bonds_prev, const double* cores_prev,
                   const int* bonds_cur, const double* cores_cur) {
  if (!st || !bonds_prev || !cores_prev || !bonds_cur || !cores_cur) return fail(MPSW_EINVAL, "null argument");
  if (shot < 0 || shot >= st->B) return fail(MPSW_EINVAL, "shot out of range");
  if (step < 0 || step > (1 << 30)) return fail(MPSW_EINVAL, "step out of range");
  const int K = st->K;
  const int* bs[2] = {bonds_prev, bonds_cur};
  const double* cs[2] = {cores_prev, cores_cur};
  const int slots[2] = {st->prev, st->cur};
  for (int t = 0; t < 2; ++t) {
    if (bs[t][0] != 1 || bs[t][K] != 1) return fail(MPSW_EINVAL, "bonds[0] and bonds[K] must be 1");
    for (int k = 1; k < K; ++k)
      if (bs[t][k] < 1 || bs[t][k] > st->Rmax[k]) return fail(MPSW_EINVAL, "bond outside [1, min(chi, 2^k, 2^(K-k))]");
    for (int k = 0; k < K; ++k)
      if ((int64_t)bs[t][k] * 2 * bs[t][k + 1] > st->cap_mps[slots[t]][k]) return fail(MPSW_EINVAL, "core exceeds its slot");
  }
  HIP_TRY(hipStreamSynchronize(st->stream));
  std::vector<int> dd(DL::size);
  HIP_TRY(hipMemcpy(dd.data(), st->dims + (int64_t)shot * DL::size, DL::size * sizeof(int), hipMemcpyDeviceToHost));
  for (int t = 0; t < 2; ++t) {
    int64_t o = 0;
    for (int k = 0; k < K; ++k) {
      const int64_t sz = (int64_t)bs[t][k] * 2 * bs[t][k + 1];
      HIP_TRY(hipMemcpy(st->mps + (int64_t)shot * st->mps_stride + st->off_mps[slots[t]][k], cs[t] + o,
                        sz * sizeof(double), hipMemcpyHostToDevice));
      o += sz;
    }
    for (int k = 0; k <= K; ++k) dd[DL::bonds + slots[t] * (MPSW_MAXK + 1) + k] = bs[t][k];
  }
  // the shot's source clock is the checkpoint's; its sketch back-offs restart
  dd[DL::step] = (int)step;
  for (int i = 0; i < 6 * MPSW_MAXK; ++i) dd[DL::rrf_skip + i] = 0;
  for (int i = 0; i < 3 * MPSW_MAXK; ++i) dd[DL::prank + i] = 0;
  HIP_TRY(hipMemcpy(st->dims + (int64_t)shot * DL::size, dd.data(), DL::size * sizeof(int), hipMemcpyHostToDevice));
  return MPSW_OK;
}

int mpsw_destroy(mpsw_state st) {
  if (!st) return MPSW_OK;
  // teardown: errors of the synchronisation and the frees are dropped
  if (st->stream) (void)hipStreamSynchronize(st->stream);
  else (void)hipDeviceSynchronize();
  st_free(st, st->mps);
  st_free(st, st->dims);
  st_free(st, st->reals);
  st_free(st, st->c2);
  st_free(st, st->c2d);
  st_free(st, st->lapW);
  st_free(st, st->wavelet);
  st_free(st, st->dense);
  st_free(st, st->err);
  st_free(st, st->sync);
  st_free(st, st->eng.eng);
  st_free(st, st->eng.d);
  st_free(st, st->mlp_w);
  for (hipEvent_t ev : st->prof_ev) (void)hipEventDestroy(ev);
  drop_graphs(st);
  if (st->cap_stream) (void)hipStreamDestroy(st->cap_stream);
  delete st;
  return MPSW_OK;
}

int mpsw_get_shape(mpsw_state st, int* nshots, int* nsites) {
  if (!st) return fail(MPSW_EINVAL, "null state");
  if (nshots) *nshots = st->B;
  if (nsites) *nsites = st->K;
  return MPSW_OK;
}

int mpsw_set_velocity_dense(mpsw_state st, const double* c2, double eps_c) {
  if (!st || !c2) return fail(MPSW_EINVAL, "null argument");
  if (!(eps_c >= 0.0)) return fail(MPSW_EINVAL, "eps_c must be >= 0");
  const int64_t N = p2(st->K);
  double mx = 0.0;
  for (int64_t i = 0; i < N; ++i) {
    if (!(c2[i] > 0.0) || !std::isfinite(c2[i])) return fail(MPSW_EINVAL, "c^2 must be finite and > 0");
    mx = std::max(mx, c2[i]);
  }
  const double lam = st->cfg[0].lambda;
  if (lam * lam * mx * st->ndim > 1.0) return fail(MPSW_ECFL, "CFL violated: lambda^2 max(c^2) ndim > 1");
  int rc = dense_to_mps(st, c2, eps_c, p2(st->K), 0, 0, true);
  if (rc != MPSW_OK) return rc;
  std::vector<double> dense;
  if ((rc = contract_dense(st, 0, -1, dense)) != MPSW_OK || (rc = upload_c2_dense(st, dense)) != MPSW_OK) return rc;
  if ((rc = build_step_engine(st)) != MPSW_OK) return rc;
  st->have_velocity = true;
  return MPSW_OK;
}

int mpsw_set_velocity_mpo(mpsw_state st, const int* bonds, const double* cores) {
  if (!st || !bonds || !cores) return fail(MPSW_EINVAL, "null argument");
  const int K = st->K;
  if (bonds[0] != 1 || bonds[K] != 1) return fail(MPSW_EINVAL, "bonds[0] and bonds[K] must be 1");
  int64_t tot = 0;
  for (int k = 0; k < K; ++k) {
    if (bonds[k + 1] < 1 || bonds[k + 1] > (1 << 20)) return fail(MPSW_EINVAL, "bad bond");
    tot += (int64_t)bonds[k] * 2 * bonds[k + 1];
  }
  st_free(st, st->c2);
  st->c2 = nullptr;
  HIP_TRY(st_malloc(st, &st->c2, tot * sizeof(double)));
  HIP_TRY(hipMemcpy(st->c2, cores, tot * sizeof(double), hipMemcpyHostToDevice));
  st->c2b.assign(bonds, bonds + K + 1);
  std::vector<double> dense;
  int rc = contract_dense(st, 0, -1, dense);
  if (rc != MPSW_OK) return rc;
  double mx = 0.0;
  for (double v : dense) {
    if (!std::isfinite(v)) return fail(MPSW_EINVAL, "non-finite c^2");
    mx = std::max(mx, v);
  }
  const double lam = st->cfg[0].lambda;
  if (lam * lam * mx * st->ndim > 1.0) return fail(MPSW_ECFL, "CFL violated: lambda^2 max(c^2) ndim > 1");
  if ((rc = upload_c2_dense(st, dense)) != MPSW_OK) return rc;
  if ((rc = build_step_engine(st)) != MPSW_OK) return rc;
  st->have_velocity = true;
  return MPSW_OK;
}

namespace {
int set_source_at(mpsw_state st, int shot, int ix, int iy, int iz, int nt, const double* wavelet) {
  const int N = 1 << st->n;
  if (shot < 0 || shot >= st->B) return fail(MPSW_EINVAL, "shot out of range");
  if (ix < 0 || ix >= N || iy < 0 || iy >= N || iz < 0 || iz >= N) return fail(MPSW_EINVAL, "source outside the grid");
  if (nt < 0 || (nt > 0 && !wavelet)) return fail(MPSW_EINVAL, "bad wavelet");
  st->wavelets[shot].assign(wavelet, wavelet + nt);
  int vals[3] = {ix, iz, nt};
  HIP_TRY(hipMemcpy(st->dims + (int64_t)shot * DL::size + DL::src_ix, vals, sizeof(vals), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(st->dims + (int64_t)shot * DL::size + DL::src_iy, &iy, sizeof(int), hipMemcpyHostToDevice));
  return upload_wavelets(st);
}
}  // namespace

int mpsw_set_source(mpsw_state st, int shot, int ix, int iz, int nt, const double* wavelet) {
  if (!st) return fail(MPSW_EINVAL, "null state");
  if (st->ndim != 2) return fail(MPSW_EINVAL, "a three-dimensional state takes mpsw_set_source_3d");
  return set_source_at(st, shot, ix, 0, iz, nt, wavelet);
}

int mpsw_set_source_3d(mpsw_state st, int shot, int ix, int iy, int iz, int nt, const double* wavelet) {
  if (!st) return fail(MPSW_EINVAL, "null state");
  if (st->ndim != 3) return fail(MPSW_EINVAL, "a two-dimensional state takes mpsw_set_source");
  return set_source_at(st, shot, ix, iy, iz, nt, wavelet);
}

int mpsw_set_fields(mpsw_state st, int shot, const double* u_prev, const double* u_cur) {
  if (!st) return fail(MPSW_EINVAL, "null state");
  if (shot < 0 || shot >= st->B) return fail(MPSW_EINVAL, "shot out of range");
  const double* fields[2] = {u_prev, u_cur};
  const int64_t N = p2(st->K);
  for (int t = 0; t < 2; ++t)
    if (fields[t])
      for (int64_t i = 0; i < N; ++i)
        if (!std::isfinite(fields[t][i])) return fail(MPSW_EINVAL, "non-finite field value");
  const int slots[2] = {st->prev, st->cur};
  for (int t = 0; t < 2; ++t) {
    if (!fields[t]) {
      Engine tmp;
      EngineLayout L;
      std::memset(&L, 0, sizeof(L));
      fill_ctx(st, tmp.h, nullptr, L);
      int rc = upload_ctx(tmp, st->stream, st);
      if (rc != MPSW_OK) return rc;
      OpArgs a{};
      a.slot = slots[t];
      a.shot = shot;
      launch_zero_state(tmp.d, a, st->B, st->stream);
      const hipError_t ze = hipStreamSynchronize(st->stream);
      st_free(st, tmp.d);
      if (ze != hipSuccess) return fail(MPSW_EHIP, std::string("set_fields: ") + hipGetErrorString(ze));
      continue;
    }
    int rc = dense_to_mps(st, fields[t], st->cfg[shot].eps, st->cfg[shot].chi_max, shot, slots[t], false);
    if (rc != MPSW_OK) return rc;
  }
  const int zero = 0;   // this shot's source clock restarts, and so do the sketch back-offs
  HIP_TRY(hipMemcpy(st->dims + (int64_t)shot * DL::size + DL::step, &zero, sizeof(int), hipMemcpyHostToDevice));
  HIP_TRY(hipMemset(st->dims + (int64_t)shot * DL::size + DL::rrf_skip, 0, sizeof(int) * 6 * MPSW_MAXK));
  HIP_TRY(hipMemset(st->dims + (int64_t)shot * DL::size + DL::prank, 0, sizeof(int) * 3 * MPSW_MAXK));
  st->step = 0;
  return MPSW_OK;
}

namespace {

// Enqueue one time step (eq. 17: three roundings) on strm and turn the slot
// rotation on the host.
void enqueue_step(mpsw_state st, hipStream_t strm) {
  Engine& e = st->eng;
  const int step = (int)std::min<int64_t>(st->step, 1 << 30);
  run_rounding(st, e, K_LAPLACE, e.sw[0], MPSW_SLOT_Y, 0, st->cur, 0, step, st->B, strm);
  run_rounding(st, e, K_C2, e.sw[2], MPSW_SLOT_W, 1, 0, 0, step, st->B, strm);
  run_rounding(st, e, K_SUM, e.sw[1], st->nxt, 2, st->cur, st->prev, step, st->B, strm);
  const int old_prev = st->prev;
  st->prev = st->cur;
  st->cur = st->nxt;
  st->nxt = old_prev;
  ++st->step;
}

int ensure_cap_stream(mpsw_state st) {
  if (!st->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&st->cap_stream, hipStreamNonBlocking));
  return MPSW_OK;
}

// Capture three steps of st on the capture stream into *exec (the host-side
// slot rotation returns to the same phase; nothing executes until launch).
int capture_three_steps(mpsw_state st, hipStream_t cap, hipGraphExec_t* exec) {
  const int saved_prof = st->prof_cls;
  st->prof_cls = -1;   // no event nodes inside a graph
  hipGraph_t graph = nullptr;
  HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  for (int i = 0; i < 3; ++i) enqueue_step(st, cap);
  st->step -= 3;   // counted when the graph is launched
  const hipError_t ce = hipStreamEndCapture(cap, &graph);
  st->prof_cls = saved_prof;
  if (ce != hipSuccess) return fail(MPSW_EHIP, std::string("step capture failed: ") + hipGetErrorString(ce));
  const hipError_t ie = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);   // the executable graph no longer needs it
  if (ie != hipSuccess) return fail(MPSW_EHIP, std::string("graph instantiation failed: ") + hipGetErrorString(ie));
  return MPSW_OK;
}

}  // namespace

int mpsw_step(mpsw_state st, int k) {
  if (!st) return fail(MPSW_EINVAL, "null state");
  if (k < 0) return fail(MPSW_EINVAL, "k must be >= 0");
  if (!st->have_velocity) return fail(MPSW_ESTATE, "set the velocity before stepping");
  if (st->learned && !st->rank_prev && !st->have_model) return fail(MPSW_ESTATE, "set the rank model before stepping a learned-rank state");
  if (st->graph_mode) {
    int rc = ensure_cap_stream(st);
    if (rc != MPSW_OK) return rc;
    for (; k >= 3; k -= 3) {
      const int phase = st->cur;
      if (!st->gexec[phase] && (rc = capture_three_steps(st, st->cap_stream, &st->gexec[phase])) != MPSW_OK)
        return rc;
      HIP_TRY(hipGraphLaunch(st->gexec[phase], st->stream));
      st->step += 3;
    }
  }
  for (int it = 0; it < k; ++it) enqueue_step(st, st->stream);
  HIP_TRY(hipGetLastError());
  return MPSW_OK;
}

int mpsw_set_graph_mode(mpsw_state st, int on) {
  if (!st) return fail(MPSW_EINVAL, "null state");
  st->graph_mode = (on != 0);
  if (!st->graph_mode) drop_graphs(st);
  return MPSW_OK;
}

// ---------------------------------------------------------------------------
// Groups: several states (different grids n, different chi per shot) stepped
// by one graph with one branch per state.
// ---------------------------------------------------------------------------
struct mpsw_group_s {
  std::vector<mpsw_state> states;
  hipStream_t stream = nullptr;        // the caller's stream (launches)
  hipStream_t cap = nullptr;           // capture origin
  std::vector<hipStream_t> branch;     // one capture stream per state
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;        // capture joins; reused to order the states' streams
  hipGraphExec_t exec = nullptr;
  std::vector<int> phases;             // slot phases the graph was captured at
  std::vector<int> gens;               // engine generations the graph was captured with
};

int mpsw_group_create(const mpsw_state* states, int nstates, void* stream, mpsw_group* out) {
  if (!states || nstates < 1 || !out) return fail(MPSW_EINVAL, "null argument or nstates < 1");
  for (int i = 0; i < nstates; ++i) {
    if (!states[i]) return fail(MPSW_EINVAL, "null state in group");
    for (int j = 0; j < i; ++j)
      if (states[j] == states[i]) return fail(MPSW_EINVAL, "a state appears twice in the group");
  }
  mpsw_group g = new mpsw_group_s();
  g->states.assign(states, states + nstates);
  g->stream = (hipStream_t)stream;
  g->branch.assign(nstates, nullptr);
  g->join.assign(nstates, nullptr);
  bool ok = hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&g->fork, hipEventDisableTiming) == hipSuccess;
  for (int i = 0; ok && i < nstates; ++i)
    ok = hipStreamCreateWithFlags(&g->branch[i], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&g->join[i], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    mpsw_group_destroy(g);
    return fail(MPSW_EHIP, "group stream or event creation failed");
  }
  *out = g;
  return MPSW_OK;
}

int mpsw_group_step(mpsw_group g, int k) {
  if (!g) return fail(MPSW_EINVAL, "null group");
  if (k < 0) return fail(MPSW_EINVAL, "k must be >= 0");
  const int ns = (int)g->states.size();
  for (mpsw_state st : g->states) {
    if (!st->have_velocity) return fail(MPSW_ESTATE, "set the velocity of every state before stepping");
    if (st->learned && !st->rank_prev && !st->have_model) return fail(MPSW_ESTATE, "set the rank model of every learned-rank state");
  }
  // order after the states' own pending work
  for (int i = 0; i < ns; ++i) {
    HIP_TRY(hipEventRecord(g->join[i], g->states[i]->stream));
    HIP_TRY(hipStreamWaitEvent(g->stream, g->join[i], 0));
  }
  for (; k >= 3; k -= 3) {
    std::vector<int> ph(ns), gen(ns);
    for (int i = 0; i < ns; ++i) {
      ph[i] = g->states[i]->cur;
      gen[i] = g->states[i]->engine_gen;
    }
    if (!g->exec || ph != g->phases || gen != g->gens) {
      if (g->exec) (void)hipGraphExecDestroy(g->exec);
      g->exec = nullptr;
      hipGraph_t graph = nullptr;
      HIP_TRY(hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal));
      hipError_t ce = hipEventRecord(g->fork, g->cap);
      std::vector<int> saved(ns);
      for (int i = 0; i < ns && ce == hipSuccess; ++i) {
        mpsw_state st = g->states[i];
        ce = hipStreamWaitEvent(g->branch[i], g->fork, 0);
        if (ce != hipSuccess) break;
        saved[i] = st->prof_cls;
        st->prof_cls = -1;
        for (int s = 0; s < 3; ++s) enqueue_step(st, g->branch[i]);
        st->step -= 3;
        st->prof_cls = saved[i];
        ce = hipEventRecord(g->join[i], g->branch[i]);
        if (ce == hipSuccess) ce = hipStreamWaitEvent(g->cap, g->join[i], 0);
      }
      const hipError_t ee = hipStreamEndCapture(g->cap, &graph);
      if (ce != hipSuccess || ee != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(MPSW_EHIP, std::string("group capture failed: ") + hipGetErrorString(ce != hipSuccess ? ce : ee));
      }
      const hipError_t ie = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ie != hipSuccess) return fail(MPSW_EHIP, std::string("graph instantiation failed: ") + hipGetErrorString(ie));
      g->phases = ph;
      g->gens = gen;
    }
    HIP_TRY(hipGraphLaunch(g->exec, g->stream));
    for (mpsw_state st : g->states) st->step += 3;
  }
  // remaining steps eagerly, then hand the states back to their own streams
  for (int i = 0; i < ns && k > 0; ++i) {
    HIP_TRY(hipEventRecord(g->join[i], g->stream));
    HIP_TRY(hipStreamWaitEvent(g->branch[i], g->join[i], 0));
    for (int s = 0; s < k; ++s) enqueue_step(g->states[i], g->branch[i]);
    HIP_TRY(hipEventRecord(g->join[i], g->branch[i]));
    HIP_TRY(hipStreamWaitEvent(g->stream, g->join[i], 0));
  }
  HIP_TRY(hipEventRecord(g->fork, g->stream));
  for (mpsw_state st : g->states) HIP_TRY(hipStreamWaitEvent(st->stream, g->fork, 0));
  HIP_TRY(hipGetLastError());
  return MPSW_OK;
}

int mpsw_group_destroy(mpsw_group g) {
  if (!g) return MPSW_OK;
  // teardown: errors of the synchronisation and the destroys are dropped
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  else (void)hipDeviceSynchronize();
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  for (hipStream_t s : g->branch)
    if (s) (void)hipStreamDestroy(s);
  for (hipEvent_t e : g->join)
    if (e) (void)hipEventDestroy(e);
  if (g->fork) (void)hipEventDestroy(g->fork);
  if (g->cap) (void)hipStreamDestroy(g->cap);
  delete g;
  return MPSW_OK;
}

int mpsw_to_dense(mpsw_state st, int shot, int which, double* out, int out_is_device) {
  if (!st || !out) return fail(MPSW_EINVAL, "null argument");
  if (shot < 0 || shot >= st->B) return fail(MPSW_EINVAL, "shot out of range");
  int slot;
  switch (which) {
    case 0: slot = st->cur; break;
    case 1: slot = st->prev; break;
    case 2: slot = -1; break;
    case 3: slot = MPSW_SLOT_Y; break;
    case 4: slot = MPSW_SLOT_W; break;
    default: return fail(MPSW_EINVAL, "which must be 0..4");
  }
  if (slot < 0 && st->c2b.empty()) return fail(MPSW_ESTATE, "no velocity set");
  std::vector<double> host;
  int rc = contract_dense(st, shot, slot, host);
  if (rc != MPSW_OK) return rc;
  if (st->cfg[0].ordering == MPSW_INTERLEAVED) {
    std::vector<double> u(host.size());
    sites_to_field(host.data(), st->n, st->ndim, u.data());
    host.swap(u);
  }
  for (double v : host)
    if (!std::isfinite(v)) return fail(MPSW_ENONFINITE, "non-finite value in the field");
  if (out_is_device) {
    HIP_TRY(hipMemcpy(out, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice));
  } else {
    std::memcpy(out, host.data(), host.size() * sizeof(double));
  }
  return MPSW_OK;
}

int mpsw_get_bonds(mpsw_state st, int shot, int which, int* bonds) {
  if (!st || !bonds) return fail(MPSW_EINVAL, "null argument");
  if (shot < 0 || shot >= st->B) return fail(MPSW_EINVAL, "shot out of range");
  if (which == 2) {
    if (st->c2b.empty()) return fail(MPSW_ESTATE, "no velocity set");
    std::copy(st->c2b.begin(), st->c2b.end(), bonds);
    return MPSW_OK;
  }
  int slot;
  switch (which) {
    case 0: slot = st->cur; break;
    case 1: slot = st->prev; break;
    case 3: slot = MPSW_SLOT_Y; break;
    case 4: slot = MPSW_SLOT_W; break;
    default: return fail(MPSW_EINVAL, "which must be 0..4");
  }
  HIP_TRY(hipStreamSynchronize(st->stream));
  HIP_TRY(hipMemcpy(bonds, st->dims + (int64_t)shot * DL::size + DL::bonds + slot * (MPSW_MAXK + 1),
                    (st->K + 1) * sizeof(int), hipMemcpyDeviceToHost));
  return check_dev_err(st);
}

int mpsw_get_stats(mpsw_state st, int shot, mpsw_stats* out) {
  if (!st || !out) return fail(MPSW_EINVAL, "null argument");
  if (shot < 0 || shot >= st->B) return fail(MPSW_EINVAL, "shot out of range");
  int rc = check_dev_err(st);
  if (rc != MPSW_OK) return rc;
  std::vector<int> d(DL::size);
  std::vector<double> r(RL::size);
  HIP_TRY(hipMemcpy(d.data(), st->dims + (int64_t)shot * DL::size, DL::size * sizeof(int), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(r.data(), st->reals + (int64_t)shot * RL::size, RL::size * sizeof(double), hipMemcpyDeviceToHost));
  std::memset(out, 0, sizeof(*out));
  out->step = d[DL::step];
  out->nsites = st->K;
  for (int k = 0; k <= st->K; ++k) out->bonds[k] = d[DL::bonds + st->cur * (MPSW_MAXK + 1) + k];
  for (int i = 0; i < 3; ++i) {
    out->max_exact_bond[i] = d[DL::maxbond + i];
    out->tail2[i] = r[RL::tail2 + i];
  }
  out->fallbacks = d[DL::fallbacks];
  out->max_jacobi_sweeps = d[DL::jac_sweeps];
  out->sketches = d[DL::rrf_tries];
  return MPSW_OK;
}

// Test hook: run the factorisation kernels of a rounding on one matrix.
//   op 0: QR of A (m x n, m even): Q (m x q) into out1, R (q x n) into out2, q = min(m, n)
//         (the identity merge when m <= n: Q = I, R = A);
//   op 1: SVD of A (m x n, n even): out1 = V^T (r x n), out2 = U Sigma (m x r),
//         r = min(m, n) (no truncation); returns r.
int mpsw_autotune(mpsw_state st, int steps, int* qr_nwg, int* jac_block_out) {
  if (!st || steps < 1) return fail(MPSW_EINVAL, "null state or steps < 1");
  if (!st->have_velocity) return fail(MPSW_ESTATE, "set the velocity before tuning");
  if (st->learned && !st->rank_prev && !st->have_model) return fail(MPSW_ESTATE, "set the rank model before tuning");
  HIP_TRY(hipStreamSynchronize(st->stream));
  // snapshot of everything a step changes: MPS arena, dims, reals, rotation
  const size_t nm = (size_t)st->mps_stride * st->B, nd = (size_t)DL::size * st->B, nr = (size_t)RL::size * st->B;
  double *sm = nullptr, *sr = nullptr;
  int* sd = nullptr;
  auto cleanup = [&]() {
    st_free(st, sm);
    st_free(st, sd);
    st_free(st, sr);
  };
  if (st_malloc(st, &sm, nm * 8) != hipSuccess || st_malloc(st, &sd, nd * 4) != hipSuccess ||
      st_malloc(st, &sr, nr * 8) != hipSuccess) {
    cleanup();
    return fail(MPSW_ENOMEM, "tuning snapshot");
  }
  const int cur = st->cur, prev = st->prev, nxt = st->nxt;
  const int64_t step0 = st->step;
  const bool graph = st->graph_mode;
  st->graph_mode = false;
  auto save = [&]() {
    return hipMemcpy(sm, st->mps, nm * 8, hipMemcpyDeviceToDevice) == hipSuccess &&
           hipMemcpy(sd, st->dims, nd * 4, hipMemcpyDeviceToDevice) == hipSuccess &&
           hipMemcpy(sr, st->reals, nr * 8, hipMemcpyDeviceToDevice) == hipSuccess;
  };
  auto restore = [&]() {
    st->cur = cur; st->prev = prev; st->nxt = nxt; st->step = step0;
    return hipMemcpy(st->mps, sm, nm * 8, hipMemcpyDeviceToDevice) == hipSuccess &&
           hipMemcpy(st->dims, sd, nd * 4, hipMemcpyDeviceToDevice) == hipSuccess &&
           hipMemcpy(st->reals, sr, nr * 8, hipMemcpyDeviceToDevice) == hipSuccess &&
           hipDeviceSynchronize() == hipSuccess;
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float best = 1e30f;
  int best_q = st->tune_qr_nwg, best_b = st->tune_jac_b;
  bool ok = save() && hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
  auto trial = [&](int q, int b) {
    if (!ok) return;
    st->tune_qr_nwg = q;
    st->tune_jac_b = b;
    ok = restore();
    if (!ok) return;
    ok = hipEventRecord(e0, st->stream) == hipSuccess;
    for (int i = 0; ok && i < steps; ++i) enqueue_step(st, st->stream);
    ok = ok && hipEventRecord(e1, st->stream) == hipSuccess;
    ok = ok && hipEventSynchronize(e1) == hipSuccess;
    float ms = 0.0f;
    if (ok) ok = hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
    if (ok && ms < best) {
      best = ms;
      best_q = q;
      best_b = b;
    }
  };
  // one factor at a time: the Jacobi block width, then the workgroups per
  // shot, then the block width again at that count (the count also bounds
  // the Jacobi workgroups, which changes what the width trades)
  for (int b : {0, 8, 16, 32}) trial(32, b);
  const int bb = best_b;
  for (int q : {16, 8, 4, 3, 2, 1}) trial(q, bb);
  const int bq = best_q;
  for (int b : {0, 8, 16, 32})
    if (bq != 32 && b != bb) trial(bq, b);   // (bq, bb) and every (32, b) were timed above
  st->tune_qr_nwg = best_q;
  st->tune_jac_b = best_b;
  if (ok) ok = restore();
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  cleanup();
  st->graph_mode = graph;
  drop_graphs(st);
  if (!ok) return fail(MPSW_EHIP, "tuning run failed");
  int rc = check_dev_err(st);
  if (rc != MPSW_OK) return rc;
  if (qr_nwg) *qr_nwg = best_q;
  if (jac_block_out) *jac_block_out = best_b;
  return MPSW_OK;
}

int mpsw_set_launch_shapes(mpsw_state st, int qr_nwg, int jac_block) {
  if (!st) return fail(MPSW_EINVAL, "null state");
  if (qr_nwg < 1 || qr_nwg > 32) return fail(MPSW_EINVAL, "qr_nwg must be in 1..32");
  if (jac_block != 0 && jac_block != 8 && jac_block != 16 && jac_block != 32)
    return fail(MPSW_EINVAL, "jac_block must be 0, 8, 16 or 32");
  st->tune_qr_nwg = qr_nwg;
  st->tune_jac_b = jac_block;
  drop_graphs(st);   // captured steps hold the old grids
  return MPSW_OK;
}

int mpsw_rank_model_set(mpsw_state st, const float* w, int nw) {
  if (!st || !w || nw != MLP_NPARAM) return fail(MPSW_EINVAL, "null argument or wrong parameter count");
  if (!st->mlp_w) HIP_TRY(st_malloc(st, &st->mlp_w, MLP_NPARAM * sizeof(float)));
  HIP_TRY(hipMemcpy(st->mlp_w, w, MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice));
  st->have_model = true;
  if (st->have_velocity) {   // the step engine's context points at the parameters
    st->eng.h.mlp_w = st->mlp_w;
    int rc = upload_ctx(st->eng, st->stream, st);
    if (rc != MPSW_OK) return rc;
    drop_graphs(st);
  }
  return MPSW_OK;
}

// Network inputs (and, with a network installed, outputs and ranks) of every
// bond of one rounding, as the learned-rank rounding forms them at the next step.
static int rank_export(mpsw_state st, int shot, int rounding, float* feats, float* outs, int* rhat) {
  if (!st) return fail(MPSW_EINVAL, "null state");
  if (shot < 0 || shot >= st->B || rounding < 0 || rounding > 2) return fail(MPSW_EINVAL, "shot or rounding out of range");
  if (!st->have_velocity) return fail(MPSW_ESTATE, "no velocity set");
  const int K = st->K;
  if (K < 2) return fail(MPSW_EINVAL, "a single site has no bond");
  const size_t nf = (size_t)K * MLP_NIN, nb = (size_t)K;
  char* buf = nullptr;
  HIP_TRY(st_malloc(st, &buf, nf * sizeof(float) + nb * (sizeof(float) + sizeof(int))));
  float* df = (float*)buf;
  float* dout = df + nf;
  int* dr = (int*)(dout + nb);
  hipError_t e = hipMemsetAsync(buf, 0, nf * sizeof(float) + nb * (sizeof(float) + sizeof(int)), st->stream);
  if (e == hipSuccess) launch_rank_export(st->eng.d, shot, rounding, K, df, dout, dr, st->stream);
  std::vector<float> hf(nf), ho(nb);
  std::vector<int> hr(nb);
  if (e == hipSuccess) e = hipMemcpyAsync(hf.data(), df, nf * sizeof(float), hipMemcpyDeviceToHost, st->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(ho.data(), dout, nb * sizeof(float), hipMemcpyDeviceToHost, st->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(hr.data(), dr, nb * sizeof(int), hipMemcpyDeviceToHost, st->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
  st_free(st, buf);
  if (e != hipSuccess) return fail(MPSW_EHIP, hipGetErrorString(e));
  for (int k = 1; k < K; ++k) {
    if (feats) std::memcpy(feats + (size_t)(k - 1) * MLP_NIN, hf.data() + (size_t)k * MLP_NIN, MLP_NIN * sizeof(float));
    if (outs) outs[k - 1] = ho[k];
    if (rhat) rhat[k - 1] = hr[k];
  }
  return check_dev_err(st);
}

int mpsw_get_rank_features(mpsw_state st, int shot, int rounding, float* feats) {
  if (!feats) return fail(MPSW_EINVAL, "null argument");
  return rank_export(st, shot, rounding, feats, nullptr, nullptr);
}

int mpsw_debug_sketch_normals(uint64_t seed, int step, int rounding, int site, int rows, int cols, double* out) {
  if (!out || rows < 1 || cols < 1 || rows > 4096 || cols > 1024 || step < 0 || rounding < 0 || site < 0)
    return fail(MPSW_EINVAL, "bad argument");
  double* d = nullptr;
  HIP_TRY(hipMalloc(&d, (size_t)rows * cols * sizeof(double)));
  launch_sketch_normals((unsigned long long)seed, step, rounding, site, rows, cols, d, nullptr);
  hipError_t e = hipMemcpy(out, d, (size_t)rows * cols * sizeof(double), hipMemcpyDeviceToHost);
  (void)hipFree(d);
  if (e != hipSuccess) return fail(MPSW_EHIP, hipGetErrorString(e));
  return MPSW_OK;
}

int mpsw_debug_rank_plan(mpsw_state st, int shot, int rounding, float* outs, int* rhat) {
  if (!outs || !rhat) return fail(MPSW_EINVAL, "null argument");
  if (st && !st->have_model) return fail(MPSW_ESTATE, "no rank network installed");
  return rank_export(st, shot, rounding, nullptr, outs, rhat);
}

int mpsw_get_sigma_log(mpsw_state st, int shot, int rounding, double* out) {
  if (!st || !out) return fail(MPSW_EINVAL, "null argument");
  if (shot < 0 || shot >= st->B || rounding < 0 || rounding > 2) return fail(MPSW_EINVAL, "shot or rounding out of range");
  HIP_TRY(hipStreamSynchronize(st->stream));
  std::vector<double> r(RL::size);
  HIP_TRY(hipMemcpy(r.data(), st->reals + (int64_t)shot * RL::size, RL::size * sizeof(double), hipMemcpyDeviceToHost));
  for (int k = 0; k < st->K; ++k)
    for (int i = 0; i < 32; ++i) out[k * 32 + i] = r[RL::sigma_log + (rounding * MPSW_MAXK + k) * 32 + i];
  return MPSW_OK;
}

int mpsw_profile(mpsw_state st, int kclass) {
  if (!st || kclass < -1 || kclass >= MPSW_KC_COUNT) return fail(MPSW_EINVAL, "invalid state or kernel class");
  HIP_TRY(hipStreamSynchronize(st->stream));
  std::vector<double> r((size_t)RL::size * st->B);
  HIP_TRY(hipMemcpy(r.data(), st->reals, r.size() * sizeof(double), hipMemcpyDeviceToHost));
  for (int i = 0; i < st->B; ++i)
    for (int c = 0; c < MPSW_KC_COUNT; ++c) r[(size_t)i * RL::size + RL::alg_flops + c] = 0.0;
  HIP_TRY(hipMemcpy(st->reals, r.data(), r.size() * sizeof(double), hipMemcpyHostToDevice));
  st->prof_cls = kclass;
  st->prof_used = 0;
  return MPSW_OK;
}

int mpsw_profile_read(mpsw_state st, int kclass, mpsw_kprof* out) {
  if (!st || !out || kclass < 0 || kclass >= MPSW_KC_COUNT) return fail(MPSW_EINVAL, "invalid arguments");
  HIP_TRY(hipStreamSynchronize(st->stream));
  std::vector<double> r((size_t)RL::size * st->B);
  HIP_TRY(hipMemcpy(r.data(), st->reals, r.size() * sizeof(double), hipMemcpyDeviceToHost));
  out->alg_flops = 0.0;
  for (int i = 0; i < st->B; ++i) out->alg_flops += r[(size_t)i * RL::size + RL::alg_flops + kclass];
  out->launches = 0;
  out->total_ms = 0.0;
  if (kclass == st->prof_cls) {
    for (size_t i = 0; i + 1 < st->prof_used; i += 2) {
      float ms = 0.0f;
      HIP_TRY(hipEventElapsedTime(&ms, st->prof_ev[i], st->prof_ev[i + 1]));
      out->total_ms += ms;
      ++out->launches;
    }
  }
  return MPSW_OK;
}

int mpsw_debug_factor(int op, int m, int n, const double* A, double* out1, double* out2) {
  if (!A || !out1 || !out2 || m < 1 || n < 1 || m > 4096 || n > 4096) return fail(MPSW_EINVAL, "bad argument");
  if (op == 0 && (m & 1)) return fail(MPSW_EINVAL, "QR test needs an even row count");
  if (op == 1 && (n & 1)) return fail(MPSW_EINVAL, "SVD test needs an even column count");
  if (op != 0 && op != 1) return fail(MPSW_EINVAL, "op must be 0 or 1");
  const int K = 4;
  // capacities: one rounding whose site 0 (QR) / site 1 (SVD) sees the matrix
  SweepCaps s;
  s.rin.assign(K + 1, 1);
  s.rt.assign(K + 1, 1);
  s.rho.assign(K + 1, 1);
  const int64_t q = std::min(m, n);
  if (op == 0) {
    s.rt[0] = m / 2; s.rin[1] = n; s.rt[1] = std::max<int64_t>(q, m / 2); s.rho[1] = n;
  } else {
    s.rt[1] = m; s.rho[2] = n / 2; s.rho[1] = q; s.rt[0] = std::max<int64_t>(1, m / 2);
  }
  Plan p;
  p.K = K;
  p.half = 2;
  p.sw = {s};
  EngineLayout L;
  layout_engine(p, L);
  L.cap_X = std::max<int64_t>(L.cap_X, (int64_t)m * n);
  L.cap_M = std::max<int64_t>(L.cap_M, (int64_t)m * std::max(n, m));
  L.cap_R = std::max<int64_t>(L.cap_R, (int64_t)m * n);
  L.cap_US = std::max<int64_t>(L.cap_US, (int64_t)m * std::max(n, m));
  L.cap_sA = std::max<int64_t>(L.cap_sA, (int64_t)m * n);
  L.cap_qrS = std::max<int64_t>(L.cap_qrS, (int64_t)m * n);
  L.cap_qrT = std::max<int64_t>(L.cap_qrT, (int64_t)(std::max(m, n) + 16) * 16);
  L.cap_sA2 = std::max<int64_t>(L.cap_sA2, q * q);
  L.cap_qrS2 = std::max<int64_t>(L.cap_qrS2, q * q);
  L.cap_qrT2 = std::max<int64_t>(L.cap_qrT2, (q + 16) * 16);
  L.cap_Vp = std::max<int64_t>(L.cap_Vp, q * q);
  L.cap_Yv = std::max<int64_t>(L.cap_Yv, (int64_t)std::max(m, n) * q);
  L.cap_q[0] = std::max<int64_t>(L.cap_q[0], (int64_t)m * n);
  L.cap_qt[0] = std::max<int64_t>(L.cap_qt[0], (int64_t)(n + 16) * 16);
  int64_t off = 0;
  auto place = [&](int64_t& o, int64_t cap) { o = off; off += (cap + 31) & ~(int64_t)31; };
  for (int k = 0; k < K; ++k) { place(L.off_in[k], L.cap_in[k]); place(L.off_q[k], L.cap_q[k]); place(L.off_qt[k], L.cap_qt[k]); }
  place(L.off_X, L.cap_X); place(L.off_X2, L.cap_X2); place(L.off_R, L.cap_R);
  place(L.off_M, L.cap_M); place(L.off_US, L.cap_US);
  place(L.off_sA, L.cap_sA); place(L.off_sJ, L.cap_sJ); place(L.off_qrS, L.cap_qrS); place(L.off_qrT, L.cap_qrT);
  place(L.off_sA2, L.cap_sA2); place(L.off_qrS2, L.cap_qrS2); place(L.off_qrT2, L.cap_qrT2);
  place(L.off_Vp, L.cap_Vp); place(L.off_Yv, L.cap_Yv);
  L.cap_perm = 4096; place(L.off_perm, L.cap_perm);
  L.stride = off;
  const int64_t core_cap = (int64_t)q * n + 2;
  double *eng = nullptr, *mps = nullptr, *reals = nullptr;
  int *dims = nullptr, *err = nullptr, *sync = nullptr;
  auto cleanup = [&]() {
    for (void* p : {(void*)eng, (void*)mps, (void*)reals, (void*)dims, (void*)err, (void*)sync}) (void)hipFree(p);
  };
  hipError_t herr = hipSuccess;   // the first failing copy or synchronisation
  auto chk = [&](hipError_t x) { if (herr == hipSuccess) herr = x; };
  if (hipMalloc(&eng, L.stride * 8) || hipMalloc(&mps, core_cap * 8) || hipMalloc(&reals, RL::size * 8) ||
      hipMalloc(&dims, DL::size * 4) || hipMalloc(&err, 4) || hipMalloc(&sync, MPSW_SYNC_STRIDE * 4)) {
    cleanup();
    return fail(MPSW_ENOMEM, "debug_factor: allocation failed");
  }
  Engine e;
  DevCtx& h = e.h;
  std::memset(&h, 0, sizeof(h));
  h.K = K; h.n = 2; h.half = 2; h.ndim = 2; h.B = 1;
  h.mps = mps; h.mps_stride = core_cap;
  for (int k = 0; k < K; ++k) { h.off_mps[0][k] = 0; h.cap_mps[0][k] = core_cap; }
  h.dims = dims; h.reals = reals; h.eng = eng; h.L = L; h.err = err; h.sync = sync;
  for (int k = 0; k <= K; ++k) { h.c2b[k] = 1; h.wb[k] = 1; }
  std::vector<int> hd(DL::size, 0);
  std::vector<double> hr(RL::size, 0.0);
  hd[DL::chi] = 1 << 30;
  hr[RL::eps] = 0.0;
  if (op == 0) { hd[DL::rt + 0] = m / 2; hd[DL::rin + 1] = n; }
  else { hd[DL::rt + 1] = m; hd[DL::rho + 2] = n / 2; }
  chk(hipMemcpy(dims, hd.data(), DL::size * 4, hipMemcpyHostToDevice));
  chk(hipMemcpy(reals, hr.data(), RL::size * 8, hipMemcpyHostToDevice));
  chk(hipMemset(err, 0, 4));
  chk(hipMemcpy(eng + (op == 0 ? L.off_X : L.off_M), A, (size_t)m * n * 8, hipMemcpyHostToDevice));
  if (herr != hipSuccess) { cleanup(); return fail(MPSW_EHIP, std::string("debug_factor: ") + hipGetErrorString(herr)); }
  int rc = upload_ctx(e, nullptr);
  if (rc != MPSW_OK) { cleanup(); return rc; }
  hipStream_t s0 = nullptr;
  int ret = 0;
  if (op == 0) {
    const int bw = qr_panel(m);
    if (bw == 0) { cleanup(); (void)hipFree(e.d); return fail(MPSW_ENOMEM, "matrix too tall for LDS"); }
    OpArgs a{};
    a.shot = -1; a.site = 0; a.op = 0;
    launch_sync_reset(e.d, 1, s0);
    launch_qrf(e.d, a, bw, (int)std::min<int64_t>(32, std::max<int64_t>(1, cdiv(n, bw))), 1, (size_t)m * bw * 8, s0);
    // Q = Q_0 [I_q; 0] through the absorb kernel: US = I (q x q), rho_1 = q
    std::vector<int> d1(DL::size);
    chk(hipMemcpy(d1.data(), dims, DL::size * 4, hipMemcpyDeviceToHost));
    const int rt1 = (herr == hipSuccess) ? d1[DL::rt + 1] : 0;
    if (rt1 < 1 || rt1 > std::min(m, n)) {   // nothing is copied out unless the rank is sane
      cleanup();
      (void)hipFree(e.d);
      return fail(MPSW_EHIP, "debug_factor: QR rank not read back");
    }
    std::vector<double> I((size_t)rt1 * rt1, 0.0);
    for (int i = 0; i < rt1; ++i) I[(size_t)i * rt1 + i] = 1.0;
    chk(hipMemcpy(eng + L.off_US, I.data(), I.size() * 8, hipMemcpyHostToDevice));
    d1[DL::rho + 1] = rt1;
    chk(hipMemcpy(dims, d1.data(), DL::size * 4, hipMemcpyHostToDevice));
    OpArgs ap{};
    ap.shot = -1; ap.site = 1;
    launch_applyq(e.d, ap, bw, std::max(1, cdiv(rt1, 16)), 1, s0);
    chk(hipDeviceSynchronize());
    chk(hipMemcpy(out1, eng + L.off_M, (size_t)m * rt1 * 8, hipMemcpyDeviceToHost));
    chk(hipMemcpy(out2, eng + L.off_R, (size_t)rt1 * n * 8, hipMemcpyDeviceToHost));
    ret = rt1;
  } else {
    OpArgs v{};
    v.shot = -1; v.site = 1; v.slot = 0; v.aux = -1;
    launch_sync_reset(e.d, 1, s0);
    const int rows = std::max(m, n);
    const int bw = qr_panel(rows);
    if (bw == 0) { cleanup(); (void)hipFree(e.d); return fail(MPSW_ENOMEM, "matrix too tall for LDS"); }
    OpArgs qa = v;
    qa.op = 1;
    launch_qrf(e.d, qa, bw, (int)std::min<int64_t>(32, std::max<int64_t>(1, cdiv(q, bw))), 1, (size_t)rows * bw * 8, s0);
    const int bw2 = qr_panel(q);
    qa.op = 2;
    launch_qrf(e.d, qa, bw2, (int)std::min<int64_t>(32, std::max<int64_t>(1, cdiv(q, bw2))), 1, (size_t)q * bw2 * 8, s0);
    const int b = jac_block(q);
    if (b == 0) { cleanup(); (void)hipFree(e.d); return fail(MPSW_ENOMEM, "columns too long for LDS"); }
    const int64_t nb = cdiv(q, b);
    launch_jac(e.d, v, b, (int)std::max<int64_t>(1, (nb + (nb & 1)) / 2), 1, (size_t)2 * b * (q + 1) * 8, q, s0);
    launch_jacfin(e.d, v, 1, s0);
    launch_applyv(e.d, v, bw, std::max<int>(1, cdiv(q, 16)), 1, s0);
    OpArgs g{};
    g.shot = -1; g.site = 1; g.slot = 0; g.op = G_US;
    launch_gemm(e.d, g, m, q, 1, 1, s0);
    chk(hipDeviceSynchronize());
    std::vector<int> d1(DL::size);
    chk(hipMemcpy(d1.data(), dims, DL::size * 4, hipMemcpyDeviceToHost));
    const int r = (herr == hipSuccess) ? d1[DL::rho + 1] : -1;
    if (r >= 0 && r <= q) {   // nothing is copied out unless the rank is sane
      chk(hipMemcpy(out1, mps, (size_t)r * n * 8, hipMemcpyDeviceToHost));
      chk(hipMemcpy(out2, eng + L.off_US, (size_t)m * r * 8, hipMemcpyDeviceToHost));
    } else if (herr == hipSuccess) {
      herr = hipErrorInvalidValue;
    }
    ret = r;
  }
  int he = 0;
  chk(hipMemcpy(&he, err, 4, hipMemcpyDeviceToHost));
  const hipError_t le = hipGetLastError();
  cleanup();
  (void)hipFree(e.d);
  if (herr != hipSuccess) return fail(MPSW_EHIP, std::string("debug_factor: ") + hipGetErrorString(herr));
  if (le != hipSuccess) return fail(MPSW_EHIP, std::string("debug_factor: ") + hipGetErrorString(le));
  if (he) return fail(MPSW_ENOMEM, "debug_factor: device error bits " + std::to_string(he));
  return ret;
}

// Host-side helper exported for tests: the fused Laplacian MPO cores
// ([wl][wr][s'][s] per site, packed) and bonds (K+1) for a register of n bits.
int mpsw_debug_sketch(const double* A, int m, int n, int l, double eps, int chi, uint64_t seed, int step, int rounding,
                      int site, double* sig, double* stats, int* rank, int* accepted) {
  if (!A || !sig || !stats || !rank || !accepted) return fail(MPSW_EINVAL, "null argument");
  if (m < 2 || n < 2 || (n & 1) || m > 4096 || n > 4096 || l < 1 || l > 32 || l > m || l > n || chi < 1 ||
      !(eps >= 0.0) || rounding < 0 || rounding > 2 || site < 1 || site > MPSW_MAXK - 2 || step < 0)
    return fail(MPSW_EINVAL, "bad argument");
  const int k = site, K = site + 1;
  SweepCaps sc;
  sc.rin.assign(K + 1, 1);
  sc.rt.assign(K + 1, 1);
  sc.rho.assign(K + 1, 1);
  sc.rt[k] = m;
  sc.rho[k + 1] = n / 2;
  sc.rho[k] = l;
  Plan p;
  p.K = K;
  p.half = std::max(1, K / 2);
  p.sw = {sc};
  p.rrf_l = l;
  EngineLayout L;
  layout_engine(p, L);
  const int64_t core_cap = (int64_t)l * n + 2;
  double *eng = nullptr, *mps = nullptr, *reals = nullptr;
  int *dims = nullptr, *err = nullptr, *sync = nullptr;
  auto cleanup = [&]() {
    for (void* p : {(void*)eng, (void*)mps, (void*)reals, (void*)dims, (void*)err, (void*)sync}) (void)hipFree(p);
  };
  hipError_t herr = hipSuccess;   // the first failing copy or synchronisation
  auto chk = [&](hipError_t x) { if (herr == hipSuccess) herr = x; };
  if (hipMalloc(&eng, L.stride * 8) || hipMalloc(&mps, core_cap * 8) || hipMalloc(&reals, RL::size * 8) ||
      hipMalloc(&dims, DL::size * 4) || hipMalloc(&err, 4) || hipMalloc(&sync, MPSW_SYNC_STRIDE * 4)) {
    cleanup();
    return fail(MPSW_ENOMEM, "debug_sketch: allocation failed");
  }
  Engine e;
  DevCtx& h = e.h;
  std::memset(&h, 0, sizeof(h));
  h.K = K; h.n = std::max(1, K / 2); h.half = h.n; h.ndim = 2; h.B = 1;
  h.mps = mps; h.mps_stride = core_cap;
  for (int q = 0; q < K; ++q) { h.off_mps[0][q] = 0; h.cap_mps[0][q] = core_cap; }
  h.dims = dims; h.reals = reals; h.eng = eng; h.L = L; h.err = err; h.sync = sync;
  h.seed = (unsigned long long)seed;
  h.rrf_over = MPSW_RRF_OVER;
  for (int q = 0; q <= K; ++q) { h.c2b[q] = 1; h.wb[q] = 1; }
  // the plan of the sketch set by hand: width l, this step
  std::vector<int> hd(DL::size, 0);
  std::vector<double> hr(RL::size, 0.0);
  hd[DL::chi] = chi;
  hd[DL::rt + k] = m;
  hd[DL::rho + k + 1] = n / 2;
  hd[DL::step] = step;
  hd[DL::rrf] = 1;
  hd[DL::rrf_l] = l;
  hr[RL::eps] = eps;
  chk(hipMemcpy(dims, hd.data(), DL::size * 4, hipMemcpyHostToDevice));
  chk(hipMemcpy(reals, hr.data(), RL::size * 8, hipMemcpyHostToDevice));
  chk(hipMemset(err, 0, 4));
  chk(hipMemcpy(eng + L.off_M, A, (size_t)m * n * 8, hipMemcpyHostToDevice));
  if (herr != hipSuccess) { cleanup(); return fail(MPSW_EHIP, std::string("debug_sketch: ") + hipGetErrorString(herr)); }
  int rc = upload_ctx(e, nullptr);
  if (rc != MPSW_OK) { cleanup(); return rc; }
  hipStream_t s0 = nullptr;
  const DevCtx* d = e.d;
  // the launch sequence of the learned-rank rounding for one bond (sketch,
  // SVD stage on B = M Q, residual, acceptance)
  OpArgs r{};
  r.shot = -1; r.site = k; r.slot = 0; r.aux = rounding; r.gate = GATE_SKETCH;
  launch_gauss(d, r, (int64_t)m * l, 1, s0);
  OpArgs g{};
  g.mode = GEMM_FP64; g.gate = GATE_SKETCH; g.shot = -1; g.site = k;
  auto orth = [&](int which, int64_t mcap) {
    OpArgs q = r;
    q.op = 3;
    q.aux = which;
    const int bw = qr_panel(mcap);
    launch_sync_reset(d, 1, s0);
    launch_qrf(d, q, bw, std::max(1, cdiv(l, bw)), 1, (size_t)mcap * bw * 8, s0);
    launch_formq(d, q, bw, std::max(1, cdiv(l, 16)), 1, s0);
  };
  g.op = G_RRF_Y; g.aux = 0;
  launch_gemm(d, g, n, l, 1, 1, s0);
  orth(0, n);
  g.op = G_RRF_Z;
  launch_gemm(d, g, m, l, 1, 1, s0);
  orth(1, m);
  g.op = G_RRF_Y; g.aux = 1;
  launch_gemm(d, g, n, l, 1, 1, s0);
  orth(0, n);
  g.op = G_RRF_Z;
  launch_gemm(d, g, m, l, 1, 1, s0);
  launch_rrf_swap(d, r, (int64_t)m * n, 1, s0);
  {
    const int64_t rows = std::max<int64_t>(m, l), ccap = std::min<int64_t>(m, l);
    OpArgs v{};
    v.shot = -1; v.site = k; v.slot = 0; v.aux = rounding; v.gate = GATE_SKETCH;
    launch_sync_reset(d, 1, s0);
    const int bw1 = qr_panel(rows), bw2 = qr_panel(ccap);
    OpArgs q = v;
    q.op = 1;
    launch_qrf(d, q, bw1, std::max(1, cdiv(ccap, bw1)), 1, (size_t)rows * bw1 * 8, s0);
    q.op = 2;
    launch_qrf(d, q, bw2, std::max(1, cdiv(ccap, bw2)), 1, (size_t)ccap * bw2 * 8, s0);
    const int b = jac_block(ccap);
    const int64_t nb = cdiv(ccap, b);
    launch_jac(d, v, b, (int)std::max<int64_t>(1, (nb + (nb & 1)) / 2), 1, (size_t)2 * b * (ccap + 1) * 8, ccap, s0);
    launch_jacfin(d, v, 1, s0);
    launch_applyv(d, v, bw1, std::max(1, cdiv(l, 16)), 1, s0);
    OpArgs gu{};
    gu.mode = GEMM_FP64; gu.gate = GATE_SKETCH; gu.shot = -1; gu.site = k; gu.slot = 0; gu.op = G_US;
    launch_gemm(d, gu, m, l, 1, 1, s0);
  }
  g.op = G_RRF_RES;
  launch_gemm(d, g, m, n, 1, 1, s0);
  launch_rrf_resid(d, r, 1, s0);
  launch_rrf_accept(d, r, (int64_t)m * n, 1, s0);
  chk(hipDeviceSynchronize());
  std::vector<int> d1(DL::size, 0);
  std::vector<double> r1(RL::size, 0.0);
  chk(hipMemcpy(d1.data(), dims, DL::size * 4, hipMemcpyDeviceToHost));
  chk(hipMemcpy(r1.data(), reals, RL::size * 8, hipMemcpyDeviceToHost));
  for (int i = 0; i < 32; ++i) sig[i] = r1[RL::sigma_log + (rounding * MPSW_MAXK + k) * 32 + i];
  stats[0] = r1[RL::rrf_res2];
  stats[1] = r1[RL::rrf_tail];
  stats[2] = r1[RL::rrf_sig1];
  *rank = d1[DL::rho + k];
  *accepted = (d1[DL::rrf] == 2) ? 1 : 0;
  int he = 0;
  chk(hipMemcpy(&he, err, 4, hipMemcpyDeviceToHost));
  const hipError_t le = hipGetLastError();
  cleanup();
  (void)hipFree(e.d);
  if (herr != hipSuccess) return fail(MPSW_EHIP, std::string("debug_sketch: ") + hipGetErrorString(herr));
  if (le != hipSuccess) return fail(MPSW_EHIP, std::string("debug_sketch: ") + hipGetErrorString(le));
  if (he) return fail(MPSW_ENOMEM, "debug_sketch: device error bits " + std::to_string(he));
  return MPSW_OK;
}

int mpsw_debug_laplacian_mpo(int n, int boundary, int ordering, int ndim, int* bonds, double* cores, int64_t cap) {
  if ((ndim != 2 && ndim != 3) || n < 1 || n * ndim > 22 || !bonds) return fail(MPSW_EINVAL, "bad argument");
  if (ordering != MPSW_SEQUENTIAL && ordering != MPSW_INTERLEAVED) return fail(MPSW_EINVAL, "unknown site order");
  LapMPO m = build_laplacian_mpo(n, boundary, ordering, ndim);
  std::copy(m.bonds.begin(), m.bonds.end(), bonds);
  int64_t o = 0;
  for (auto& c : m.cores) {
    if (cores) {
      if (o + (int64_t)c.size() > cap) return fail(MPSW_ENOMEM, "cores buffer too small");
      std::copy(c.begin(), c.end(), cores + o);
    }
    o += (int64_t)c.size();
  }
  return (int)o;
}

}  // extern "C"
