// Truncation-rank network of libmpsw: forward, backward and Adam training on
// the GPU (FP32), and the per-bond rank prediction used by the learned-rank
// rounding.
//
// Network (34 -> 128 -> 128 -> 1, ReLU): out = relu(relu(x W1 + b1) W2 + b2) W3
// + b3, read as rank / chi_max.  Loss: mean of w (out - y)^2, w = alpha where
// out < y (under-prediction costs an exact-SVD fallback), else 1.  Parameters
// are one flat FP32 vector: W1 (34 x 128, input by output), b1, W2 (128 x 128),
// b2, W3 (128), b3.
//
// Training kernels work on chunks of MLP_S samples per 128-thread workgroup
// (thread j = hidden unit j); each chunk writes its own partial gradient and
// a reduction sums the chunks in a fixed order, so gradients are reproducible.
#include "mpsw_device.h"
#include "../../include/mpsw_debug.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <random>
#include <string>
#include <vector>

namespace mpsw {

constexpr int MLP_S = 32;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + MLP_NIN * MLP_NH, OFF_W2 = OFF_B1 + MLP_NH,
              OFF_B2 = OFF_W2 + MLP_NH * MLP_NH, OFF_W3 = OFF_B2 + MLP_NH, OFF_B3 = OFF_W3 + MLP_NH;
static_assert(OFF_B3 + 1 == MLP_NPARAM, "parameter layout");

// Forward (and with BWD the backward) pass of one chunk of samples.
template <bool BWD>
__global__ __launch_bounds__(MLP_NH) void k_mlp(const float* __restrict__ X, const float* __restrict__ y, int m,
                                                float alpha, const float* __restrict__ W, float* out,
                                                float* gpart, float* lpart) {
  __shared__ float xs[MLP_S][MLP_NIN];
  __shared__ float h1[MLP_S][MLP_NH], h2[MLP_S][MLP_NH], dz[MLP_S][MLP_NH];
  __shared__ float outs[MLP_S], dout[MLP_S];
  const int j = threadIdx.x, chunk = blockIdx.x;
  const int s0 = chunk * MLP_S, ns = min(MLP_S, m - s0);
  for (int e = j; e < MLP_S * MLP_NIN; e += MLP_NH) {
    const int s = e / MLP_NIN, i = e % MLP_NIN;
    xs[s][i] = (s < ns) ? X[(int64_t)(s0 + s) * MLP_NIN + i] : 0.0f;
  }
  __syncthreads();
  // layer 1
  {
    float w1[MLP_NIN];
#pragma unroll
    for (int i = 0; i < MLP_NIN; ++i) w1[i] = W[OFF_W1 + i * MLP_NH + j];
    const float b = W[OFF_B1 + j];
    for (int s = 0; s < MLP_S; ++s) {
      float z = b;
#pragma unroll
      for (int i = 0; i < MLP_NIN; ++i) z = fmaf(xs[s][i], w1[i], z);
      h1[s][j] = fmaxf(z, 0.0f);
    }
  }
  __syncthreads();
  // layer 2
  float acc[MLP_S];
  {
    const float b = W[OFF_B2 + j];
#pragma unroll
    for (int s = 0; s < MLP_S; ++s) acc[s] = b;
    for (int i = 0; i < MLP_NH; ++i) {
      const float w = W[OFF_W2 + i * MLP_NH + j];
#pragma unroll
      for (int s = 0; s < MLP_S; ++s) acc[s] = fmaf(h1[s][i], w, acc[s]);
    }
#pragma unroll
    for (int s = 0; s < MLP_S; ++s) h2[s][j] = fmaxf(acc[s], 0.0f);
  }
  // output: products into dz, then one thread per sample sums its row
  const float w3 = W[OFF_W3 + j];
#pragma unroll
  for (int s = 0; s < MLP_S; ++s) dz[s][j] = fmaxf(acc[s], 0.0f) * w3;
  __syncthreads();
  if (j < MLP_S) {
    float o = W[OFF_B3];
    for (int u = 0; u < MLP_NH; ++u) o += dz[j][u];
    outs[j] = o;
    float d = 0.0f, l = 0.0f;
    if (j < ns) {
      d = o - y[s0 + j];
      const float wt = (d < 0.0f) ? alpha : 1.0f;
      l = wt * d * d;
      d = 2.0f * wt * d / (float)m;
      if (out) out[s0 + j] = o;
    }
    dout[j] = d;
    dz[j][0] = l;   // row 0 of dz is free again after this thread's sum
  }
  __syncthreads();
  if (j == 0 && lpart) {
    float l = 0.0f;
    for (int s = 0; s < ns; ++s) l += dz[s][0];
    lpart[chunk] = l / (float)m;
  }
  if (!BWD) return;
  float* g = gpart + (int64_t)chunk * MLP_NPARAM;
  __syncthreads();
  // W3, b3 and dz2 = dout W3 relu'(z2)
  {
    float gw3 = 0.0f;
    for (int s = 0; s < MLP_S; ++s) {
      gw3 = fmaf(h2[s][j], dout[s], gw3);
      dz[s][j] = (h2[s][j] > 0.0f) ? dout[s] * w3 : 0.0f;
    }
    g[OFF_W3 + j] = gw3;
    if (j == 0) {
      float gb = 0.0f;
      for (int s = 0; s < MLP_S; ++s) gb += dout[s];
      g[OFF_B3] = gb;
    }
  }
  __syncthreads();
  // W2, b2
  for (int i = 0; i < MLP_NH; ++i) {
    float gw = 0.0f;
    for (int s = 0; s < MLP_S; ++s) gw = fmaf(h1[s][i], dz[s][j], gw);
    g[OFF_W2 + i * MLP_NH + j] = gw;
  }
  {
    float gb = 0.0f;
    for (int s = 0; s < MLP_S; ++s) gb += dz[s][j];
    g[OFF_B2 + j] = gb;
  }
  // dz1 (thread i = j): sum_u dz2[s][u] W2[i][u], masked by relu'(z1)
  for (int s = 0; s < MLP_S; ++s) acc[s] = 0.0f;
  for (int u = 0; u < MLP_NH; ++u) {
    const float w = W[OFF_W2 + j * MLP_NH + u];
#pragma unroll
    for (int s = 0; s < MLP_S; ++s) acc[s] = fmaf(dz[s][u], w, acc[s]);
  }
  __syncthreads();   // every read of dz2 is done
#pragma unroll
  for (int s = 0; s < MLP_S; ++s) dz[s][j] = (h1[s][j] > 0.0f) ? acc[s] : 0.0f;
  __syncthreads();
  for (int i = 0; i < MLP_NIN; ++i) {
    float gw = 0.0f;
    for (int s = 0; s < MLP_S; ++s) gw = fmaf(xs[s][i], dz[s][j], gw);
    g[OFF_W1 + i * MLP_NH + j] = gw;
  }
  {
    float gb = 0.0f;
    for (int s = 0; s < MLP_S; ++s) gb += dz[s][j];
    g[OFF_B1 + j] = gb;
  }
}

// grad[p] = sum over chunks (fixed order); loss likewise.
__global__ void k_mlp_reduce(const float* __restrict__ gpart, const float* __restrict__ lpart, int nchunk,
                             float* grad, float* loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < MLP_NPARAM) {
    float s = 0.0f;
    for (int c = 0; c < nchunk; ++c) s += gpart[(int64_t)c * MLP_NPARAM + p];
    grad[p] = s;
  }
  if (p == 0) {
    float l = 0.0f;
    for (int c = 0; c < nchunk; ++c) l += lpart[c];
    *loss = l;
  }
}

// Adam (Kingma & Ba 2015) with bias correction; t counts from 1.
__global__ void k_adam(float* W, const float* __restrict__ grad, float* m1, float* m2, float lr, int t) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= MLP_NPARAM) return;
  const float b1 = 0.9f, b2 = 0.999f, e = 1e-8f;
  const float gv = grad[p];
  const float a = b1 * m1[p] + (1.0f - b1) * gv;
  const float b = b2 * m2[p] + (1.0f - b2) * gv * gv;
  m1[p] = a;
  m2[p] = b;
  const float ah = a / (1.0f - powf(b1, (float)t)), bh = b / (1.0f - powf(b2, (float)t));
  W[p] -= lr * ah / (sqrtf(bh) + e);
}

// Scratch of the allocation-free gradient call: the per-chunk partial
// gradients and losses of up to MLP_STATIC_MAX_ROWS samples.  One copy per
// device, held until the process ends; every call overwrites all of what it
// reads (each chunk writes its whole partial, the reduction writes the whole
// gradient), so nothing needs clearing between calls.
constexpr int MLP_STATIC_MAX_ROWS = 8192;
constexpr int MLP_STATIC_CHUNKS = MLP_STATIC_MAX_ROWS / MLP_S;
static __device__ __align__(256) float scratch[(size_t)MLP_STATIC_CHUNKS * MLP_NPARAM + MLP_STATIC_CHUNKS];

}  // namespace mpsw

using namespace mpsw;

namespace mpsw {
int set_last_error(int code, const char* msg);
}

namespace {

int mlp_fail(int code, const std::string& msg) { return mpsw::set_last_error(code, msg.c_str()); }

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);   // teardown: nothing to do with an error here
  }
  bool alloc(size_t bytes) { return hipMalloc(&p, bytes) == hipSuccess; }
  float* f() { return (float*)p; }
};

int run_mlp(const float* X, const float* y, int m, float alpha, float* w, int epochs, float lr, float* grad_out,
            float* loss_out, float* out_pred) {
  if (!X || !w || m < 1) return mlp_fail(MPSW_EINVAL, "null argument or m < 1");
  const bool need_y = (epochs > 0) || grad_out || loss_out;
  if (need_y && !y) return mlp_fail(MPSW_EINVAL, "labels required");
  const int nchunk = (m + MLP_S - 1) / MLP_S;
  DevBuf dX, dy, dW, dg, dgp, dlp, dl, dm1, dm2, dout;
  if (!dX.alloc((size_t)m * MLP_NIN * 4) || !dy.alloc((size_t)m * 4) || !dW.alloc(MLP_NPARAM * 4) ||
      !dg.alloc(MLP_NPARAM * 4) || !dgp.alloc((size_t)nchunk * MLP_NPARAM * 4) || !dlp.alloc((size_t)nchunk * 4) ||
      !dl.alloc(4) || !dm1.alloc(MLP_NPARAM * 4) || !dm2.alloc(MLP_NPARAM * 4) ||
      (out_pred && !dout.alloc((size_t)m * 4)))
    return mlp_fail(MPSW_ENOMEM, "network buffers");
  if (hipMemcpy(dX.p, X, (size_t)m * MLP_NIN * 4, hipMemcpyHostToDevice) != hipSuccess ||
      (y && hipMemcpy(dy.p, y, (size_t)m * 4, hipMemcpyHostToDevice) != hipSuccess) ||
      hipMemcpy(dW.p, w, MLP_NPARAM * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(dm1.p, 0, MLP_NPARAM * 4) != hipSuccess || hipMemset(dm2.p, 0, MLP_NPARAM * 4) != hipSuccess ||
      (!y && hipMemset(dy.p, 0, (size_t)m * 4) != hipSuccess))
    return mlp_fail(MPSW_EHIP, "network upload");
  const int rb = (MLP_NPARAM + 255) / 256;
  for (int ep = 1; ep <= epochs; ++ep) {
    hipLaunchKernelGGL(k_mlp<true>, dim3(nchunk), dim3(MLP_NH), 0, 0, dX.f(), dy.f(), m, alpha, dW.f(), nullptr,
                       dgp.f(), dlp.f());
    hipLaunchKernelGGL(k_mlp_reduce, dim3(rb), dim3(256), 0, 0, dgp.f(), dlp.f(), nchunk, dg.f(), dl.f());
    hipLaunchKernelGGL(k_adam, dim3(rb), dim3(256), 0, 0, dW.f(), dg.f(), dm1.f(), dm2.f(), lr, ep);
  }
  // final pass: loss, gradient, predictions at the returned weights
  hipLaunchKernelGGL(k_mlp<true>, dim3(nchunk), dim3(MLP_NH), 0, 0, dX.f(), dy.f(), m, alpha, dW.f(),
                     out_pred ? dout.f() : nullptr, dgp.f(), dlp.f());
  hipLaunchKernelGGL(k_mlp_reduce, dim3(rb), dim3(256), 0, 0, dgp.f(), dlp.f(), nchunk, dg.f(), dl.f());
  if (hipGetLastError() != hipSuccess) return mlp_fail(MPSW_EHIP, "network kernels failed to launch");
  if (hipMemcpy(w, dW.p, MLP_NPARAM * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      (grad_out && hipMemcpy(grad_out, dg.p, MLP_NPARAM * 4, hipMemcpyDeviceToHost) != hipSuccess) ||
      (loss_out && hipMemcpy(loss_out, dl.p, 4, hipMemcpyDeviceToHost) != hipSuccess) ||
      (out_pred && hipMemcpy(out_pred, dout.p, (size_t)m * 4, hipMemcpyDeviceToHost) != hipSuccess))
    return mlp_fail(MPSW_EHIP, "network download");
  return MPSW_OK;
}

}  // namespace

extern "C" {

int mpsw_mlp_grad(const float* X, const float* y, int m, float alpha, const float* w, float* grad, float* loss) {
  if (!w || !grad || !loss) return mlp_fail(MPSW_EINVAL, "null argument");
  std::vector<float> wc(w, w + MLP_NPARAM);
  return run_mlp(X, y, m, alpha, wc.data(), 0, 0.0f, grad, loss, nullptr);
}

int mpsw_mlp_train(const float* X, const float* y, int m, int epochs, float lr, float alpha, float* w) {
  if (epochs < 0 || !(lr > 0.0f)) return mlp_fail(MPSW_EINVAL, "epochs must be >= 0 and lr > 0");
  return run_mlp(X, y, m, alpha, w, epochs, lr, nullptr, nullptr, nullptr);
}

int mpsw_mlp_grad_noalloc(const float* X, const float* y, int m, float alpha, const float* w, float* grad,
                          float* loss, void* hip_stream) {
  if (!X || !y || !w || !grad || !loss) return mlp_fail(MPSW_EINVAL, "null argument");
  if (m < 1 || m > MLP_STATIC_MAX_ROWS)
    return mlp_fail(MPSW_EINVAL, "m must be in [1, " + std::to_string(MLP_STATIC_MAX_ROWS) + "] for the static scratch");
  // the device address of this device's copy of the scratch array, looked up
  // once per device with that device current (the array's name in host code
  // is not a device address)
  static std::mutex mu;
  static float* addr[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return mlp_fail(MPSW_EHIP, "no current device");
  float* sp = nullptr;
  {
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) return mlp_fail(MPSW_EHIP, std::string("scratch address: ") + hipGetErrorString(e));
      addr[dev] = (float*)p;
    }
    sp = addr[dev];
  }
  hipStream_t s = (hipStream_t)hip_stream;
  const int nchunk = (m + MLP_S - 1) / MLP_S;
  float* gpart = sp;
  float* lpart = sp + (size_t)MLP_STATIC_CHUNKS * MLP_NPARAM;
  hipLaunchKernelGGL(k_mlp<true>, dim3(nchunk), dim3(MLP_NH), 0, s, X, y, m, alpha, w, nullptr, gpart, lpart);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, gpart, lpart, nchunk, grad, loss);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return mlp_fail(MPSW_EHIP, std::string("network kernels: ") + hipGetErrorString(e));
  return MPSW_OK;
}

int mpsw_mlp_init(uint64_t seed, float* w) {
  // He-scaled normal weights (variance 2 / fan-in for the ReLU layers, 1 / fan-in
  // for the output), zero biases, in the parameter order of the header
  if (!w) return mlp_fail(MPSW_EINVAL, "null argument");
  std::mt19937_64 gen(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  auto fill = [&](int off, int count, double sd) {
    for (int i = 0; i < count; ++i) w[off + i] = (float)(sd * nd(gen));
  };
  std::fill(w, w + MLP_NPARAM, 0.0f);
  fill(OFF_W1, MLP_NIN * MLP_NH, std::sqrt(2.0 / MLP_NIN));
  fill(OFF_W2, MLP_NH * MLP_NH, std::sqrt(2.0 / MLP_NH));
  fill(OFF_W3, MLP_NH, std::sqrt(1.0 / MLP_NH));
  return MPSW_OK;
}

int mpsw_mlp_forward(const float* X, int m, const float* w, float* out) {
  if (!w || !out) return mlp_fail(MPSW_EINVAL, "null argument");
  std::vector<float> wc(w, w + MLP_NPARAM);
  return run_mlp(X, nullptr, m, 1.0f, wc.data(), 0, 0.0f, nullptr, nullptr, out);
}

}  // extern "C"
