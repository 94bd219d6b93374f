// Small device kernels around the TTM tree: FP64 sums of squares (||T||,
// ||G||, Sec. 2.2 error), factor conversion, fills, and the explicit residual
// ||T - G x_1 F_1 ... x_N F_N|| accumulated without forming the recovered
// tensor.  Every reduction is two-stage with a fixed partition and a fixed
// summation order (deterministic).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.h"
#include "internal.h"
#include "kernels.h"

namespace tk {

constexpr int kRedBlocks = 1024;

template <typename T>
__global__ __launch_bounds__(256) void sumsq_partial(const T* __restrict__ x, int64_t n,
                                                     double* __restrict__ part) {
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = min(n, lo + per);
  double s = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
    const double v = Elem<T>::to_f64(x[i]);
    s = fma(v, v, s);
  }
  s = wave_sum(s);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void sum_final(const double* __restrict__ part, int n,
                                                 double* __restrict__ out) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  s = wave_sum(s);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = (red[0] + red[1]) + (red[2] + red[3]);
}

hipError_t launch_sumsq(int dtype, const void* x, int64_t n, double* part, double* out,
                        hipStream_t st) {
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(kRedBlocks, (n + 255) / 256));
  if (dtype == TK_F64)
    hipLaunchKernelGGL(sumsq_partial<double>, dim3(blocks), dim3(256), 0, st, (const double*)x, n,
                       part);
  else if (dtype == TK_F32)
    hipLaunchKernelGGL(sumsq_partial<float>, dim3(blocks), dim3(256), 0, st, (const float*)x, n,
                       part);
  else if (dtype == TK_F16)
    hipLaunchKernelGGL(sumsq_partial<_Float16>, dim3(blocks), dim3(256), 0, st,
                       (const _Float16*)x, n, part);
  else
    hipLaunchKernelGGL(sumsq_partial<uint16_t>, dim3(blocks), dim3(256), 0, st,
                       (const uint16_t*)x, n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_final, dim3(1), dim3(256), 0, st, part, blocks, out);
  return hipGetLastError();
}

int sumsq_partials() { return kRedBlocks; }

__global__ void f64_to_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}
__global__ void f32_to_f64(const float* __restrict__ a, double* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (double)a[i];
}
__global__ void fill_f64(double* __restrict__ a, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

hipError_t launch_convert(int from, int to, const void* a, void* b, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (from == TK_F64 && to == TK_F32)
    hipLaunchKernelGGL(f64_to_f32, dim3(blocks), dim3(256), 0, st, (const double*)a, (float*)b, n);
  else if (from == TK_F32 && to == TK_F64)
    hipLaunchKernelGGL(f32_to_f64, dim3(blocks), dim3(256), 0, st, (const float*)a, (double*)b, n);
  else if (from == to)
    return hipMemcpyAsync(b, a, n * (from == TK_F64 ? 8 : (from == TK_F32 ? 4 : 2)),
                          hipMemcpyDeviceToDevice, st);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

__global__ void copy_f64(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

hipError_t launch_copy_f64(const double* a, double* b, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(copy_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, n);
  return hipGetLastError();
}

// Block s: out[s] = sum of squares of x[off[s] .. off[s + 1]), FP64, fixed order.
__global__ __launch_bounds__(256) void sumsq_segments(const float* __restrict__ x,
                                                      const int64_t* __restrict__ off,
                                                      double* __restrict__ out) {
  __shared__ double red[256];
  const int64_t b = off[blockIdx.x], e = off[blockIdx.x + 1];
  double s = 0.0;
  for (int64_t i = b + threadIdx.x; i < e; i += 256) {
    const double v = x[i];
    s = fma(v, v, s);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

hipError_t launch_sumsq_segments(const float* x, const int64_t* off, int count, double* out,
                                 hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(sumsq_segments, dim3(count), dim3(256), 0, st, x, off, out);
  return hipGetLastError();
}

__global__ void fill_i32(int* __restrict__ a, int64_t n, int v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

hipError_t launch_fill_int(int* a, int64_t n, int v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, n, v);
  return hipGetLastError();
}

hipError_t launch_fill(double* a, int64_t n, double v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, n, v);
  return hipGetLastError();
}

// Residual of the last expansion step: with Zp = G x_1 F_1 ... x_{N-1} F_{N-1}
// except mode 0 (row-major [K0, R]) and F0 (L0 x K0), accumulate
// sum_{i0, r} (T[i0, r] - sum_k F0[i0, k] Zp[k, r])^2 in FP64.
template <typename T>
__global__ __launch_bounds__(256) void residual_partial(const T* __restrict__ Tt,
                                                        const double* __restrict__ Zp,
                                                        const double* __restrict__ F0, int L0,
                                                        int K0, int64_t R,
                                                        double* __restrict__ part) {
  const int64_t n = (int64_t)L0 * R;
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = min(n, lo + per);
  double s = 0.0;
  for (int64_t e = lo + threadIdx.x; e < hi; e += 256) {
    const int64_t i0 = e / R;
    const int64_t r = e - i0 * R;
    double z = 0.0;
    for (int k = 0; k < K0; ++k) z = fma(F0[i0 * K0 + k], Zp[(int64_t)k * R + r], z);
    const double d = Elem<T>::to_f64(Tt[e]) - z;
    s = fma(d, d, s);
  }
  s = wave_sum(s);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

hipError_t launch_residual(int dtype, const void* Tt, const double* Zp, const double* F0, int L0,
                           int K0, int64_t R, double* part, double* out, hipStream_t st) {
  const int blocks = kRedBlocks;
  if (dtype == TK_F64)
    hipLaunchKernelGGL(residual_partial<double>, dim3(blocks), dim3(256), 0, st,
                       (const double*)Tt, Zp, F0, L0, K0, R, part);
  else if (dtype == TK_F32)
    hipLaunchKernelGGL(residual_partial<float>, dim3(blocks), dim3(256), 0, st, (const float*)Tt,
                       Zp, F0, L0, K0, R, part);
  else if (dtype == TK_F16)
    hipLaunchKernelGGL(residual_partial<_Float16>, dim3(blocks), dim3(256), 0, st,
                       (const _Float16*)Tt, Zp, F0, L0, K0, R, part);
  else
    hipLaunchKernelGGL(residual_partial<uint16_t>, dim3(blocks), dim3(256), 0, st,
                       (const uint16_t*)Tt, Zp, F0, L0, K0, R, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_final, dim3(1), dim3(256), 0, st, part, blocks, out);
  return hipGetLastError();
}

}  // namespace tk
