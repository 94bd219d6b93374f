// Gram matrix of a mode-n unfolding (Sec. 5: the SVD step is computed from
// the Gram matrix Y_(n) Y_(n)^T followed by an eigen-decomposition).
//
// With Y viewed row-major as [A, L, B], the unfolding's columns are the
// pairs c = (a, b), and
//     S[i, j] = sum_{a, b} Y[a, i, b] * Y[a, j, b].
// The columns are cut into fixed chunks; every block computes one 64 x 64
// tile (i-tile <= j-tile, symmetry) of one chunk's partial Gram with FP64
// FMAs on LDS-staged rows (FP32/BF16 inputs convert exactly to FP64, so the
// products are exact and only the FP64 sums round).  A second kernel adds the
// chunk partials in fixed chunk order and mirrors the tile: the result is
// bitwise deterministic for a given shape.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.h"
#include "internal.h"
#include "kernels.h"

namespace tk {

constexpr int kGT = 64;  // tile rows
constexpr int kGC = 32;  // columns per LDS step

__device__ __forceinline__ void pair_of(int p, int T, int* ti, int* tj) {
  int i = 0;
  while (p >= T - i) {
    p -= T - i;
    ++i;
  }
  *ti = i;
  *tj = i + p;
}

template <typename TIn>
__device__ __forceinline__ void gram_load_tile(double (*X)[kGT], const TIn* __restrict__ Y,
                                               int L, int64_t B, int row0, int64_t cs,
                                               int64_t cend) {
  // kGC * kGT / 256 = 8 elements per thread, all loads issued before the stores
  const int tid = threadIdx.x;
  constexpr int kPer = kGC * kGT / 256;
  double v[kPer];
  if (B == 1) {
    // Y[a, l]: rows of one column are contiguous -> threads walk rows fastest
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + 256 * u;
      const int rr = e % kGT, cc = e / kGT;
      const int64_t c = cs + cc;
      const int row = row0 + rr;
      v[u] = (c < cend && row < L) ? Elem<TIn>::to_f64(Y[c * L + row]) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + 256 * u;
      X[e / kGT][e % kGT] = v[u];
    }
  } else {
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + 256 * u;
      const int cc = e % kGC, rr = e / kGC;
      const int64_t c = cs + cc;
      const int row = row0 + rr;
      double x = 0.0;
      if (c < cend && row < L) {
        const int64_t a = c / B;
        const int64_t b = c - a * B;
        x = Elem<TIn>::to_f64(Y[(a * L + row) * B + b]);
      }
      v[u] = x;
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + 256 * u;
      X[e % kGC][e / kGC] = v[u];
    }
  }
}

// Partial Gram of column chunk `chunk` for tile pair `pair` -> one 64 x 64
// block of `part`.
template <typename TIn>
__device__ __forceinline__ void gram_partial_body(const TIn* __restrict__ Y, int L, int64_t B,
                                                  int64_t C, int64_t cchunk, int T, int npairs,
                                                  double* __restrict__ part, int chunk, int pair,
                                                  double (*Xi)[kGT], double (*Xj)[kGT]) {
  int ti, tj;
  pair_of(pair, T, &ti, &tj);
  const int64_t cbeg = (int64_t)chunk * cchunk;
  const int64_t cend = min(C, cbeg + cchunk);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int s = 0; s < 4; ++s) acc[r][s] = 0.0;
  const bool diag = (ti == tj);
  for (int64_t cs = cbeg; cs < cend; cs += kGC) {
    __syncthreads();
    gram_load_tile<TIn>(Xi, Y, L, B, ti * kGT, cs, cend);
    if (!diag) gram_load_tile<TIn>(Xj, Y, L, B, tj * kGT, cs, cend);
    __syncthreads();
    double (*Xb)[kGT] = diag ? Xi : Xj;
#pragma unroll 4
    for (int cc = 0; cc < kGC; ++cc) {
      double ai[4], bj[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) ai[r] = Xi[cc][4 * ty + r];
#pragma unroll
      for (int s = 0; s < 4; ++s) bj[s] = Xb[cc][4 * tx + s];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int s = 0; s < 4; ++s) acc[r][s] = fma(ai[r], bj[s], acc[r][s]);
    }
  }
  double* out = part + ((int64_t)chunk * npairs + pair) * (kGT * kGT);
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int s = 0; s < 4; ++s) out[(4 * ty + r) * kGT + 4 * tx + s] = acc[r][s];
}

template <typename TIn>
__global__ __launch_bounds__(256) void gram_partial(const TIn* __restrict__ Y, int L, int64_t B,
                                                    int64_t C, int64_t cchunk, int T,
                                                    int npairs, double* __restrict__ part) {
  __shared__ double Xi[kGC][kGT];
  __shared__ double Xj[kGC][kGT];
  gram_partial_body<TIn>(Y, L, B, C, cchunk, T, npairs, part, blockIdx.x, blockIdx.y, Xi, Xj);
}

// Grouped Gram (batched HOOI): block b computes item b = (matrix, chunk, pair).
template <typename TIn>
__global__ __launch_bounds__(256) void gram_grouped_partial(const GramDesc* __restrict__ mats,
                                                            const int4* __restrict__ items) {
  __shared__ double Xi[kGC][kGT];
  __shared__ double Xj[kGC][kGT];
  const int4 w = items[blockIdx.x];
  const GramDesc d = mats[w.x];
  gram_partial_body<TIn>((const TIn*)d.Y, d.L, d.B, d.C, d.cchunk, d.T, d.npairs, d.part, w.y,
                         w.z, Xi, Xj);
}

__global__ void gram_reduce(const double* __restrict__ part, int L, int T, int npairs,
                            int nchunks, double* __restrict__ S) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)L * L) return;
  int i = (int)(e / L), j = (int)(e % L);
  int ii = i, jj = j;
  if (ii / kGT > jj / kGT) {
    ii = j;
    jj = i;
  }
  const int ti = ii / kGT, tj = jj / kGT;
  const int p = ti * T - ti * (ti - 1) / 2 + (tj - ti);
  const int li = ii - ti * kGT, lj = jj - tj * kGT;
  double s = 0.0;
  for (int ch = 0; ch < nchunks; ++ch)
    s += part[((int64_t)ch * npairs + p) * (kGT * kGT) + li * kGT + lj];
  S[e] = s;
}

// Element e of the concatenated L_m x L_m results of all matrices: matrix m
// with elem_off[m] <= e < elem_off[m + 1] (binary search), then as gram_reduce.
__global__ void gram_grouped_reduce(const GramDesc* __restrict__ mats,
                                    const int64_t* __restrict__ elem_off, int n_mats) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= elem_off[n_mats]) return;
  int lo = 0, hi = n_mats - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (elem_off[mid] <= e)
      lo = mid;
    else
      hi = mid - 1;
  }
  const GramDesc d = mats[lo];
  const int64_t r = e - elem_off[lo];
  const int L = d.L;
  const int i = (int)(r / L), j = (int)(r % L);
  int ii = i, jj = j;
  if (ii / kGT > jj / kGT) {
    ii = j;
    jj = i;
  }
  const int ti = ii / kGT, tj = jj / kGT;
  const int p = ti * d.T - ti * (ti - 1) / 2 + (tj - ti);
  const int li = ii - ti * kGT, lj = jj - tj * kGT;
  double s = 0.0;
  for (int ch = 0; ch < d.nchunks; ++ch)
    s += d.part[((int64_t)ch * d.npairs + p) * (kGT * kGT) + li * kGT + lj];
  d.S[r] = s;
}

namespace {
struct GramGeom {
  int T, npairs;
  int64_t cchunk, nchunks;
};
GramGeom gram_geom(int64_t L, int64_t C) {
  GramGeom g;
  g.T = (int)((L + kGT - 1) / kGT);
  g.npairs = g.T * (g.T + 1) / 2;
  const int64_t target = std::max<int64_t>(1, 4096 / g.npairs);
  int64_t cc = (C + target - 1) / target;
  cc = std::max<int64_t>(cc, 128);
  cc = (cc + kGC - 1) / kGC * kGC;
  g.cchunk = cc;
  g.nchunks = (C + cc - 1) / cc;
  return g;
}
}  // namespace

void gram_geometry(int64_t L, int64_t C, int64_t target_blocks, GramDesc* d) {
  GramGeom g = gram_geom(L, C);
  if (target_blocks > 0) {
    // batched: aim for `target_blocks` blocks per matrix instead of 4096
    int64_t cc = (C + std::max<int64_t>(1, target_blocks / g.npairs) - 1) /
                 std::max<int64_t>(1, target_blocks / g.npairs);
    cc = std::max<int64_t>(cc, 128);
    cc = (cc + kGC - 1) / kGC * kGC;
    g.cchunk = cc;
    g.nchunks = (C + cc - 1) / cc;
  }
  d->L = (int)L;
  d->C = C;
  d->T = g.T;
  d->npairs = g.npairs;
  d->cchunk = g.cchunk;
  d->nchunks = (int)g.nchunks;
}

hipError_t launch_gram_grouped(int in_dtype, const GramDesc* mats, const int4* items,
                               int n_items, const int64_t* elem_off, int n_mats,
                               int64_t total_elems, hipStream_t st) {
  if (n_items == 0) return hipSuccess;
  if (in_dtype == TK_F32)
    hipLaunchKernelGGL(gram_grouped_partial<float>, dim3(n_items), dim3(256), 0, st, mats, items);
  else
    hipLaunchKernelGGL(gram_grouped_partial<uint16_t>, dim3(n_items), dim3(256), 0, st, mats,
                       items);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gram_grouped_reduce, dim3((unsigned)((total_elems + 255) / 256)), dim3(256),
                     0, st, mats, elem_off, n_mats);
  return hipGetLastError();
}

size_t gram_workspace_elems(int64_t L, int64_t C) {
  GramGeom g = gram_geom(L, C);
  return (size_t)g.nchunks * g.npairs * kGT * kGT;
}

hipError_t launch_gram(int in_dtype, const void* Y, int64_t A, int64_t L, int64_t B, double* S,
                       double* part, hipStream_t st) {
  const int64_t C = A * B;
  if (C == 0) return launch_fill(S, L * L, 0.0, st);
  GramGeom g = gram_geom(L, C);
  dim3 grid((unsigned)g.nchunks, (unsigned)g.npairs);
  if (in_dtype == TK_F64)
    hipLaunchKernelGGL(gram_partial<double>, grid, dim3(256), 0, st, (const double*)Y, (int)L, B,
                       C, g.cchunk, g.T, g.npairs, part);
  else if (in_dtype == TK_F32)
    hipLaunchKernelGGL(gram_partial<float>, grid, dim3(256), 0, st, (const float*)Y, (int)L, B, C,
                       g.cchunk, g.T, g.npairs, part);
  else
    hipLaunchKernelGGL(gram_partial<uint16_t>, grid, dim3(256), 0, st, (const uint16_t*)Y,
                       (int)L, B, C, g.cchunk, g.T, g.npairs, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n = L * L;
  hipLaunchKernelGGL(gram_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, part,
                     (int)L, g.T, g.npairs, (int)g.nchunks, S);
  return hipGetLastError();
}

}  // namespace tk
