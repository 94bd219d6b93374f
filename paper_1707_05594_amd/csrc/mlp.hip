// Small multilayer perceptron for the learned TTM-tree cost model: forward,
// backward and Adam on the GPU.
//
// Model: x' = (x - mu) / sigma, h1 = relu(W1 x' + b1), h2 = relu(W2 h1 + b2),
// y = w3 . h2 + b3, with x in R^D (node features), hidden width H and one
// output (log of the node's time).  Loss: mean squared error over the batch.
// Parameters are FP32 and stored flat in the order W1 (H x D, row-major), b1,
// W2 (H x H), b2, w3 (H), b3.  Every reduction runs in a fixed order, so
// results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <vector>

#include "internal.h"
#include "tucker.h"

struct tk_mlp {
  int D = 0, H = 0;
  int64_t P = 0;
  int cap = 0;  // rows the activation buffers hold
  float* params = nullptr;
  float* grad = nullptr;
  float* m1 = nullptr;  // Adam first moment
  float* m2 = nullptr;  // Adam second moment
  float* mu = nullptr;
  float* sigma = nullptr;
  float* X = nullptr;   // cap x D
  float* y = nullptr;   // cap targets
  float* Z1 = nullptr;  // cap x H pre-activations (layer 1)
  float* A1 = nullptr;
  float* Z2 = nullptr;
  float* A2 = nullptr;
  float* out = nullptr;   // cap predictions
  float* dout = nullptr;  // cap
  float* dZ2 = nullptr;   // cap x H
  float* dZ1 = nullptr;   // cap x H
  float* loss = nullptr;  // 1
  int64_t adam_t = 0;
  hipStream_t st = nullptr;

  ~tk_mlp() {
    float* ptrs[] = {params, grad, m1, m2, mu, sigma, X, y, Z1, A1, Z2, A2, out, dout, dZ2, dZ1, loss};
    for (float* p : ptrs)
      if (p) (void)hipFree(p);
    if (st) (void)hipStreamDestroy(st);
  }
  int64_t off_b1() const { return (int64_t)H * D; }
  int64_t off_W2() const { return off_b1() + H; }
  int64_t off_b2() const { return off_W2() + (int64_t)H * H; }
  int64_t off_w3() const { return off_b2() + H; }
  int64_t off_b3() const { return off_w3() + H; }
};

namespace tk {
namespace {

constexpr int kThreads = 256;

// Z[r, j] = sum_i W[j, i] x[r, i] + b[j]; A = relu(Z).  With mu/sigma set, x
// is standardised on the fly.  Thread per (r, j).
__global__ void dense_fwd(const float* __restrict__ X, int n, int I, const float* __restrict__ W,
                          const float* __restrict__ b, int J, float* __restrict__ Z,
                          float* __restrict__ A, const float* __restrict__ mu,
                          const float* __restrict__ sig, int relu) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * J) return;
  const int r = (int)(e / J), j = (int)(e % J);
  float acc = b[j];
  const float* x = X + (int64_t)r * I;
  const float* w = W + (int64_t)j * I;
  for (int i = 0; i < I; ++i) {
    const float xi = mu ? (x[i] - mu[i]) / sig[i] : x[i];
    acc = fmaf(w[i], xi, acc);
  }
  if (Z) Z[e] = acc;
  A[e] = relu ? fmaxf(acc, 0.f) : acc;
}

// dy[r] = 2 (pred[r] - y[r]) / n and loss = mean (pred - y)^2 (one block).
__global__ void mse_grad(const float* __restrict__ pred, const float* __restrict__ y, int n,
                         float* __restrict__ dy, float* __restrict__ loss) {
  __shared__ float red[kThreads];
  float s = 0.f;
  for (int r = threadIdx.x; r < n; r += kThreads) {
    const float d = pred[r] - y[r];
    dy[r] = 2.f * d / (float)n;
    s = fmaf(d, d, s);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] / (float)n;
}

// dX[r, i] = (sum_j dZ[r, j] W[j, i]) * [Zprev[r, i] > 0].  Thread per (r, i).
__global__ void dense_bwd_in(const float* __restrict__ dZ, int n, int J, const float* __restrict__ W,
                             int I, const float* __restrict__ Zprev, float* __restrict__ dX) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * I) return;
  const int r = (int)(e / I), i = (int)(e % I);
  float acc = 0.f;
  const float* dz = dZ + (int64_t)r * J;
  for (int j = 0; j < J; ++j) acc = fmaf(dz[j], W[(int64_t)j * I + i], acc);
  dX[e] = Zprev[e] > 0.f ? acc : 0.f;
}

// dW[j, i] = sum_r dZ[r, j] x[r, i] (thread per (j, i)); db[j] = sum_r dZ[r, j]
// (threads j < J of the extra row of blocks).  x standardised as in the forward.
__global__ void dense_bwd_w(const float* __restrict__ dZ, int n, int J, const float* __restrict__ Xin,
                            int I, float* __restrict__ dW, float* __restrict__ db,
                            const float* __restrict__ mu, const float* __restrict__ sig) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (int64_t)J * I) {
    const int j = (int)(e / I), i = (int)(e % I);
    float acc = 0.f;
    for (int r = 0; r < n; ++r) {
      const float x = Xin[(int64_t)r * I + i];
      const float xi = mu ? (x - mu[i]) / sig[i] : x;
      acc = fmaf(dZ[(int64_t)r * J + j], xi, acc);
    }
    dW[e] = acc;
  } else if (e < (int64_t)J * I + J) {
    const int j = (int)(e - (int64_t)J * I);
    float acc = 0.f;
    for (int r = 0; r < n; ++r) acc += dZ[(int64_t)r * J + j];
    db[j] = acc;
  }
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// p -= lr (m / bc1) / (sqrt(v / bc2) + eps) with bc = 1 - beta^t.
__global__ void adam_step(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                          float* __restrict__ v, int64_t P, float lr, float b1, float b2, float eps,
                          float bc1, float bc2) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= P) return;
  const float gi = g[e];
  const float mi = b1 * m[e] + (1.f - b1) * gi;
  const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  p[e] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

int dalloc_f(float** p, int64_t n) {
  if (hipMalloc((void**)p, sizeof(float) * (size_t)std::max<int64_t>(n, 1)) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(TK_ENOMEM, "device allocation of %lld floats failed", (long long)n);
  }
  return TK_OK;
}

int ensure_rows(tk_mlp* m, int n) {
  if (n <= m->cap) return TK_OK;
  float** bufs[] = {&m->X, &m->y, &m->Z1, &m->A1, &m->Z2, &m->A2, &m->out, &m->dout, &m->dZ2, &m->dZ1};
  for (float** b : bufs)
    if (*b) {
      (void)hipFree(*b);
      *b = nullptr;
    }
  m->cap = 0;
  const int64_t H = m->H, D = m->D;
  const int64_t sizes[] = {n * D, n, n * H, n * H, n * H, n * H, n, n, n * H, n * H};
  for (int i = 0; i < 10; ++i)
    if (int rc = dalloc_f(bufs[i], sizes[i])) return rc;
  m->cap = n;
  return TK_OK;
}

hipError_t forward(tk_mlp* m, int n) {
  const int D = m->D, H = m->H;
  const float* P = m->params;
  hipLaunchKernelGGL(dense_fwd, dim3(blocks_for((int64_t)n * H)), dim3(kThreads), 0, m->st, m->X, n,
                     D, P, P + m->off_b1(), H, m->Z1, m->A1, m->mu, m->sigma, 1);
  hipLaunchKernelGGL(dense_fwd, dim3(blocks_for((int64_t)n * H)), dim3(kThreads), 0, m->st, m->A1, n,
                     H, P + m->off_W2(), P + m->off_b2(), H, m->Z2, m->A2, (const float*)nullptr,
                     (const float*)nullptr, 1);
  hipLaunchKernelGGL(dense_fwd, dim3(blocks_for(n)), dim3(kThreads), 0, m->st, m->A2, n, H,
                     P + m->off_w3(), P + m->off_b3(), 1, (float*)nullptr, m->out,
                     (const float*)nullptr, (const float*)nullptr, 0);
  return hipGetLastError();
}

hipError_t backward(tk_mlp* m, int n, float* loss_dst) {
  const int D = m->D, H = m->H;
  const float* P = m->params;
  float* G = m->grad;
  hipLaunchKernelGGL(mse_grad, dim3(1), dim3(kThreads), 0, m->st, m->out, m->y, n, m->dout, loss_dst);
  // output layer: dw3 = sum_r dout[r] A2[r, :], db3 = sum dout
  hipLaunchKernelGGL(dense_bwd_w, dim3(blocks_for(H + 1)), dim3(kThreads), 0, m->st, m->dout, n, 1,
                     m->A2, H, G + m->off_w3(), G + m->off_b3(), (const float*)nullptr,
                     (const float*)nullptr);
  hipLaunchKernelGGL(dense_bwd_in, dim3(blocks_for((int64_t)n * H)), dim3(kThreads), 0, m->st,
                     m->dout, n, 1, P + m->off_w3(), H, m->Z2, m->dZ2);
  hipLaunchKernelGGL(dense_bwd_w, dim3(blocks_for((int64_t)H * H + H)), dim3(kThreads), 0, m->st,
                     m->dZ2, n, H, m->A1, H, G + m->off_W2(), G + m->off_b2(),
                     (const float*)nullptr, (const float*)nullptr);
  hipLaunchKernelGGL(dense_bwd_in, dim3(blocks_for((int64_t)n * H)), dim3(kThreads), 0, m->st,
                     m->dZ2, n, H, P + m->off_W2(), H, m->Z1, m->dZ1);
  hipLaunchKernelGGL(dense_bwd_w, dim3(blocks_for((int64_t)H * D + H)), dim3(kThreads), 0, m->st,
                     m->dZ1, n, H, m->X, D, G, G + m->off_b1(), m->mu, m->sigma);
  return hipGetLastError();
}

int upload_batch(tk_mlp* m, const float* X, const float* y, int n) {
  if (int rc = ensure_rows(m, n)) return rc;
  TK_HIP(hipMemcpyAsync(m->X, X, sizeof(float) * (size_t)n * m->D, hipMemcpyHostToDevice, m->st));
  if (y) TK_HIP(hipMemcpyAsync(m->y, y, sizeof(float) * (size_t)n, hipMemcpyHostToDevice, m->st));
  return TK_OK;
}

}  // namespace

// Predictions for n device-resident rows of features (used by the planner).
int mlp_forward_host(tk_mlp* m, const float* X_host, int n, float* y_host) {
  if (int rc = upload_batch(m, X_host, nullptr, n)) return rc;
  TK_HIP(forward(m, n));
  TK_HIP(hipMemcpyAsync(y_host, m->out, sizeof(float) * (size_t)n, hipMemcpyDeviceToHost, m->st));
  TK_HIP(hipStreamSynchronize(m->st));
  return TK_OK;
}

}  // namespace tk

using namespace tk;

extern "C" int64_t tk_mlp_param_count(int in_dim, int hidden) {
  if (in_dim < 1 || hidden < 1) return 0;
  const int64_t D = in_dim, H = hidden;
  return H * D + H + H * H + H + H + 1;
}

extern "C" int tk_mlp_create(int in_dim, int hidden, const float* params_host, tk_mlp** out) {
  clear_error();
  if (!out || !params_host) return fail(TK_EINVAL, "null pointer");
  *out = nullptr;
  if (in_dim < 1 || in_dim > 256 || hidden < 1 || hidden > 1024)
    return fail(TK_EINVAL, "in_dim=%d hidden=%d outside [1,256] x [1,1024]", in_dim, hidden);
  tk_mlp* m = new (std::nothrow) tk_mlp;
  if (!m) return fail(TK_ENOMEM, "model allocation failed");
  m->D = in_dim;
  m->H = hidden;
  m->P = tk_mlp_param_count(in_dim, hidden);
  auto bail = [&](int rc) {
    delete m;
    return rc;
  };
  if (hipStreamCreateWithFlags(&m->st, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    return bail(fail(TK_EDEVICE, "stream creation failed"));
  }
  for (float** b : {&m->params, &m->grad, &m->m1, &m->m2})
    if (int rc = dalloc_f(b, m->P)) return bail(rc);
  if (int rc = dalloc_f(&m->loss, 1)) return bail(rc);
  if (hipMemcpy(m->params, params_host, sizeof(float) * (size_t)m->P, hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemset(m->m1, 0, sizeof(float) * (size_t)m->P) != hipSuccess ||
      hipMemset(m->m2, 0, sizeof(float) * (size_t)m->P) != hipSuccess) {
    (void)hipGetLastError();
    return bail(fail(TK_EDEVICE, "parameter upload failed"));
  }
  *out = m;
  return TK_OK;
}

extern "C" int tk_mlp_set_norm(tk_mlp* m, const float* mu, const float* sigma) {
  clear_error();
  if (!m || !mu || !sigma) return fail(TK_EINVAL, "null pointer");
  for (int i = 0; i < m->D; ++i)
    if (!(sigma[i] > 0.f) || !std::isfinite(mu[i]))
      return fail(TK_EINVAL, "sigma[%d] must be positive and mu finite", i);
  if (!m->mu) {
    if (int rc = dalloc_f(&m->mu, m->D)) return rc;
    if (int rc = dalloc_f(&m->sigma, m->D)) return rc;
  }
  TK_HIP(hipMemcpy(m->mu, mu, sizeof(float) * m->D, hipMemcpyHostToDevice));
  TK_HIP(hipMemcpy(m->sigma, sigma, sizeof(float) * m->D, hipMemcpyHostToDevice));
  return TK_OK;
}

extern "C" int tk_mlp_fit_norm(tk_mlp* m, const float* X_host, int n) {
  clear_error();
  if (!m || !X_host) return fail(TK_EINVAL, "null pointer");
  if (n < 1) return fail(TK_EINVAL, "n=%d < 1", n);
  std::vector<float> mu(m->D), sigma(m->D);
  for (int i = 0; i < m->D; ++i) {
    double sum = 0.0;
    for (int r = 0; r < n; ++r) sum += (double)X_host[(size_t)r * m->D + i];
    const double mean = sum / n;
    double ss = 0.0;
    for (int r = 0; r < n; ++r) {
      const double d = (double)X_host[(size_t)r * m->D + i] - mean;
      ss += d * d;
    }
    const double sd = std::sqrt(ss / n);
    if (!std::isfinite(mean) || !std::isfinite(sd))
      return fail(TK_EINVAL, "feature %d is not finite", i);
    mu[i] = (float)mean;
    sigma[i] = sd > 1e-6 ? (float)sd : 1.f;  // constant feature: leave it unscaled
  }
  return tk_mlp_set_norm(m, mu.data(), sigma.data());
}

extern "C" int tk_mlp_get_params(const tk_mlp* m, float* host) {
  clear_error();
  if (!m || !host) return fail(TK_EINVAL, "null pointer");
  TK_HIP(hipStreamSynchronize(m->st));
  TK_HIP(hipMemcpy(host, m->params, sizeof(float) * (size_t)m->P, hipMemcpyDeviceToHost));
  return TK_OK;
}

extern "C" int tk_mlp_set_params(tk_mlp* m, const float* host) {
  clear_error();
  if (!m || !host) return fail(TK_EINVAL, "null pointer");
  TK_HIP(hipStreamSynchronize(m->st));
  TK_HIP(hipMemcpy(m->params, host, sizeof(float) * (size_t)m->P, hipMemcpyHostToDevice));
  TK_HIP(hipMemset(m->m1, 0, sizeof(float) * (size_t)m->P));
  TK_HIP(hipMemset(m->m2, 0, sizeof(float) * (size_t)m->P));
  m->adam_t = 0;
  return TK_OK;
}

extern "C" int tk_mlp_forward(tk_mlp* m, const float* X_host, int n, float* y_host) {
  clear_error();
  if (!m || !X_host || !y_host) return fail(TK_EINVAL, "null pointer");
  if (n < 1) return fail(TK_EINVAL, "n=%d < 1", n);
  return mlp_forward_host(m, X_host, n, y_host);
}

extern "C" int tk_mlp_loss_grad(tk_mlp* m, const float* X_host, const float* y_host, int n,
                                float* loss_host, float* grad_host) {
  clear_error();
  if (!m || !X_host || !y_host) return fail(TK_EINVAL, "null pointer");
  if (n < 1) return fail(TK_EINVAL, "n=%d < 1", n);
  if (int rc = upload_batch(m, X_host, y_host, n)) return rc;
  TK_HIP(forward(m, n));
  TK_HIP(backward(m, n, m->loss));
  if (loss_host)
    TK_HIP(hipMemcpyAsync(loss_host, m->loss, sizeof(float), hipMemcpyDeviceToHost, m->st));
  if (grad_host)
    TK_HIP(hipMemcpyAsync(grad_host, m->grad, sizeof(float) * (size_t)m->P, hipMemcpyDeviceToHost,
                          m->st));
  TK_HIP(hipStreamSynchronize(m->st));
  return TK_OK;
}

extern "C" int tk_mlp_train(tk_mlp* m, const float* X_host, const float* y_host, int n, int steps,
                            float lr, float* loss_host) {
  clear_error();
  if (!m || !X_host || !y_host) return fail(TK_EINVAL, "null pointer");
  if (n < 1 || steps < 1) return fail(TK_EINVAL, "n=%d steps=%d must be >= 1", n, steps);
  if (!(lr > 0.f)) return fail(TK_EINVAL, "lr must be positive");
  if (int rc = upload_batch(m, X_host, y_host, n)) return rc;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  float* losses = nullptr;  // one loss per step, copied out at the end
  if (int rc = dalloc_f(&losses, steps)) return rc;
  hipError_t e = hipSuccess;
  for (int t = 0; t < steps && e == hipSuccess; ++t) {
    e = forward(m, n);
    if (e == hipSuccess) e = backward(m, n, losses + t);
    if (e != hipSuccess) break;
    ++m->adam_t;
    const double bc1 = 1.0 - std::pow(0.9, (double)m->adam_t);
    const double bc2 = 1.0 - std::pow(0.999, (double)m->adam_t);
    hipLaunchKernelGGL(adam_step, dim3(blocks_for(m->P)), dim3(kThreads), 0, m->st, m->params,
                       m->grad, m->m1, m->m2, m->P, lr, b1, b2, eps, (float)bc1, (float)bc2);
    e = hipGetLastError();
  }
  if (e == hipSuccess && loss_host)
    e = hipMemcpyAsync(loss_host, losses, sizeof(float) * (size_t)steps, hipMemcpyDeviceToHost,
                       m->st);
  if (e == hipSuccess) e = hipStreamSynchronize(m->st);
  (void)hipFree(losses);
  if (e != hipSuccess) return fail(TK_EDEVICE, "training failed: %s", hipGetErrorString(e));
  return TK_OK;
}

extern "C" void tk_mlp_free(tk_mlp* m) { delete m; }
