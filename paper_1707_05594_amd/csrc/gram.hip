// Gram matrix of a mode-n unfolding (Sec. 5: the SVD step is computed from
// the Gram matrix Y_(n) Y_(n)^T followed by an eigen-decomposition).
//
// With Y viewed row-major as [A, L, B], the unfolding's columns are the
// pairs c = (a, b), and
//     S[i, j] = sum_{a, b} Y[a, i, b] * Y[a, j, b].
// The columns are cut into fixed chunks; every block computes one 64 x 64
// tile (i-tile <= j-tile, symmetry) of one chunk's partial Gram with FP64
// MFMAs on LDS-staged rows (FP32/BF16 inputs convert exactly to FP64, so the
// products are exact and only the FP64 sums round).  A second kernel adds the
// chunk partials in a fixed order and mirrors the tile: the result is bitwise
// deterministic for a given shape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "device.h"
#include "internal.h"
#include "kernels.h"

namespace tk {

constexpr int kGT = 64;       // tile rows
constexpr int kGC = 32;       // columns per LDS step
constexpr int kGP = kGT + 1;  // LDS pitch (doubles): column-fastest stores spread over banks

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void pair_of(int p, int T, int* ti, int* tj) {
  int i = 0;
  while (p >= T - i) {
    p -= T - i;
    ++i;
  }
  *ti = i;
  *tj = i + p;
}

// One kGC-column step of a 64-row tile: 8 elements per thread in their
// stored type (converted to FP64, exactly, when written to LDS); zeros past
// the chunk's end and past row L.  B == 1: Y[a, l],
// a column's rows are contiguous and threads walk rows fastest; otherwise
// consecutive columns (b) are contiguous and threads walk columns fastest, so
// a thread keeps one column c = (a, b) for the whole step: `col` points at
// row 0 of it, advanced by the caller from step to step.
template <typename TIn>
__device__ __forceinline__ void gram_load_step(TIn (&v)[8], const TIn* __restrict__ Y, int L,
                                               int64_t B, int row0, int64_t cs, int64_t cend,
                                               const TIn* __restrict__ col) {
  const int tid = threadIdx.x;
  if (B == 1) {
    const int row = row0 + tid % kGT;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t c = cs + tid / kGT + 4 * u;
      v[u] = (c < cend && row < L) ? Y[c * L + row] : TIn(0);
    }
  } else {
    const bool in = cs + tid % kGC < cend;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int row = row0 + tid / kGC + 8 * u;
      v[u] = (in && row < L) ? col[(int64_t)row * B] : TIn(0);
    }
  }
}

// Column walker of a thread for B > 1: c = (a, b) -> pointer to Y[a, 0, b];
// one division at the start, then steps of kGC columns.
template <typename TIn>
struct GramCol {
  int64_t a, b;
  __device__ __forceinline__ void start(int64_t c, int64_t B) {
    a = c / B;
    b = c - a * B;
  }
  __device__ __forceinline__ void step(int64_t B) {
    b += kGC;
    while (b >= B) {
      b -= B;
      ++a;
    }
  }
  __device__ __forceinline__ const TIn* ptr(const TIn* Y, int L, int64_t B) const {
    return Y + a * L * B + b;
  }
};
template <typename TIn>
__device__ __forceinline__ void gram_store_step(double (*X)[kGP], const TIn (&v)[8], bool b1) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const double x = Elem<TIn>::to_f64(v[u]);
    if (b1)
      X[tid / kGT + 4 * u][tid % kGT] = x;
    else
      X[tid % kGC][tid / kGC + 8 * u] = x;
  }
}

__device__ __forceinline__ d4 mfma_f64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// (4 waves per SIMD for 2- and 4-byte inputs; FP64 raw sets need the
// registers of 2.)
// Partial Gram of column chunk `chunk` for tile pair `pair` -> one 64 x 64
// block of `part` (row index in tile ti, column index in tile tj).  Wave w
// owns the 32 x 32 quadrant (w / 2, w % 2) as 2 x 2 blocks of
// v_mfma_f64_16x16x4_f64: per four columns, lane l supplies row l % 16 of
// column l / 16 for both operands (A = the ti rows, B = the tj rows), and
// holds D[l / 16 + 4 r][l % 16] in register r.  16-row blocks entirely past
// row L are skipped.  Loads run two steps ahead of the multiplications.
template <typename TIn>
__device__ __forceinline__ void gram_partial_body(const TIn* __restrict__ Y, int L, int64_t B,
                                                  int64_t C, int64_t cchunk, int T, int npairs,
                                                  double* __restrict__ part, int chunk, int pair,
                                                  double (*Xi)[kGP], double (*Xj)[kGP]) {
  int ti, tj;
  pair_of(pair, T, &ti, &tj);
  const int64_t cbeg = (int64_t)chunk * cchunk;
  const int64_t cend = min(C, cbeg + cchunk);
  const bool diag = (ti == tj);
  const bool b1 = B == 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rq = (wave >> 1) * 32, cq = (wave & 1) * 32;
  const bool vi0 = ti * kGT + rq < L, vi1 = ti * kGT + rq + 16 < L;
  const bool vj0 = tj * kGT + cq < L, vj1 = tj * kGT + cq + 16 < L;
  d4 acc00 = {0.0, 0.0, 0.0, 0.0}, acc01 = acc00, acc10 = acc00, acc11 = acc00;
  double (*Xb)[kGP] = diag ? Xi : Xj;

  // steps s = 0, 1, 2, ... of kGC columns; step s's elements are loaded two
  // steps ahead into raw set s % 2 (loads in step order, one column walker)
  GramCol<TIn> cw;
  if (!b1) cw.start(cbeg + threadIdx.x % kGC, B);
  TIn ri[2][8], rj[2][8];
  auto load = [&](int set, int64_t cs) {
    gram_load_step<TIn>(ri[set], Y, L, B, ti * kGT, cs, cend, cw.ptr(Y, L, B));
    if (!diag) gram_load_step<TIn>(rj[set], Y, L, B, tj * kGT, cs, cend, cw.ptr(Y, L, B));
    if (!b1) cw.step(B);
  };
  const int r = lane & 15, k4 = lane >> 4;
  auto multiply = [&]() {
#pragma unroll
    for (int k = 0; k < kGC; k += 4) {
      const double a0 = Xi[k + k4][rq + r], a1 = Xi[k + k4][rq + 16 + r];
      const double b0 = Xb[k + k4][cq + r], b1v = Xb[k + k4][cq + 16 + r];
      if (vi0 && vj0) acc00 = mfma_f64(a0, b0, acc00);
      if (vi0 && vj1) acc01 = mfma_f64(a0, b1v, acc01);
      if (vi1 && vj0) acc10 = mfma_f64(a1, b0, acc10);
      if (vi1 && vj1) acc11 = mfma_f64(a1, b1v, acc11);
    }
  };
  auto step = [&](int set, int64_t cs) {
    __syncthreads();  // the previous step has been multiplied
    gram_store_step<TIn>(Xi, ri[set], b1);
    if (!diag) gram_store_step<TIn>(Xj, rj[set], b1);
    __syncthreads();
    if (cs + 2 * kGC < cend) load(set, cs + 2 * kGC);
    multiply();
  };
  load(0, cbeg);
  if (cbeg + kGC < cend) load(1, cbeg + kGC);
  for (int64_t cs = cbeg; cs < cend; cs += 2 * kGC) {
    step(0, cs);
    if (cs + kGC < cend) step(1, cs + kGC);
  }
  double* out = part + ((int64_t)chunk * npairs + pair) * (kGT * kGT);
  const int i0 = rq + k4, j0 = cq + r;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    out[(i0 + 4 * q) * kGT + j0] = acc00[q];
    out[(i0 + 4 * q) * kGT + j0 + 16] = acc01[q];
    out[(i0 + 16 + 4 * q) * kGT + j0] = acc10[q];
    out[(i0 + 16 + 4 * q) * kGT + j0 + 16] = acc11[q];
  }
}

template <typename TIn>
__global__ __launch_bounds__(256, sizeof(TIn) == 8 ? 2 : 4) void gram_partial(
    const TIn* __restrict__ Y, int L, int64_t B, int64_t C, int64_t cchunk, int T, int npairs,
    double* __restrict__ part) {
  __shared__ double Xi[kGC][kGP];
  __shared__ double Xj[kGC][kGP];
  gram_partial_body<TIn>(Y, L, B, C, cchunk, T, npairs, part, blockIdx.x, blockIdx.y, Xi, Xj);
}

// Grouped Gram (batched HOOI): block b computes item b = (matrix, chunk, pair).
template <typename TIn>
__global__ __launch_bounds__(256, sizeof(TIn) == 8 ? 2 : 4) void gram_grouped_partial(
    const GramDesc* __restrict__ mats, const int4* __restrict__ items) {
  __shared__ double Xi[kGC][kGP];
  __shared__ double Xj[kGC][kGP];
  const int4 w = items[blockIdx.x];
  const GramDesc d = mats[w.x];
  gram_partial_body<TIn>(global_ptr((const TIn*)d.Y), d.L, d.B, d.C, d.cchunk, d.T, d.npairs,
                         global_ptr(d.part), w.y, w.z, Xi, Xj);
}

// Sum over chunks of element (i, j) of an L x L Gram: kRG thread groups of
// kRE elements; group g adds chunks g, g + kRG, ... in order, then the group
// sums are added in group order (a fixed order for a given shape).
constexpr int kRG = 8, kRE = 32;

__device__ __forceinline__ double gram_chunk_sum(const double* __restrict__ part, int T,
                                                 int npairs, int nchunks, int i, int j, int g) {
  int ii = i, jj = j;
  if (ii / kGT > jj / kGT) {
    ii = j;
    jj = i;
  }
  const int ti = ii / kGT, tj = jj / kGT;
  const int p = ti * T - ti * (ti - 1) / 2 + (tj - ti);
  const int64_t off = (int64_t)p * (kGT * kGT) + (ii - ti * kGT) * kGT + (jj - tj * kGT);
  const int64_t stride = (int64_t)npairs * (kGT * kGT);
  // chunks g, g + kRG, ... added in that order; eight loads issued together
  double s = 0.0;
  for (int ch0 = g; ch0 < nchunks; ch0 += 8 * kRG) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int ch = ch0 + u * kRG;
      v[u] = ch < nchunks ? part[ch * stride + off] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (ch0 + u * kRG < nchunks) s += v[u];
  }
  return s;
}

__device__ __forceinline__ double combine_groups(double s, double (*red)[kRE]) {
  const int g = threadIdx.x / kRE, q = threadIdx.x % kRE;
  red[g][q] = s;
  __syncthreads();
  double t = 0.0;
  if (g == 0)
#pragma unroll
    for (int h = 0; h < kRG; ++h) t += red[h][q];
  return t;
}

__global__ __launch_bounds__(256) void gram_reduce(const double* __restrict__ part, int L, int T,
                                                   int npairs, int nchunks,
                                                   double* __restrict__ S) {
  __shared__ double red[kRG][kRE];
  const int g = threadIdx.x / kRE, q = threadIdx.x % kRE;
  const int64_t e = (int64_t)blockIdx.x * kRE + q;
  const bool ok = e < (int64_t)L * L;
  const double s = ok ? gram_chunk_sum(part, T, npairs, nchunks, (int)(e / L), (int)(e % L), g)
                      : 0.0;
  const double t = combine_groups(s, red);
  if (g == 0 && ok) S[e] = t;
}

// Element e of the concatenated L_m x L_m results of all matrices: matrix m
// with elem_off[m] <= e < elem_off[m + 1] (binary search), one thread per
// element.  The thread adds the chunks in gram_reduce's order (group g's chunks
// g, g + kRG, ... in order, then the kRG group sums in group order), so both
// reductions give the same bits for the same partials.
__global__ __launch_bounds__(256) void gram_grouped_reduce(const GramDesc* __restrict__ mats,
                                                           const int64_t* __restrict__ elem_off,
                                                           int n_mats) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
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
  const int64_t rel = e - elem_off[lo];
  int ii = (int)(rel / d.L), jj = (int)(rel % d.L);
  if (ii / kGT > jj / kGT) {
    const int t = ii;
    ii = jj;
    jj = t;
  }
  const int ti = ii / kGT, tj = jj / kGT;
  const int p = ti * d.T - ti * (ti - 1) / 2 + (tj - ti);
  const double* src =
      global_ptr(d.part) + (int64_t)p * (kGT * kGT) + (ii - ti * kGT) * kGT + (jj - tj * kGT);
  const int64_t stride = (int64_t)d.npairs * (kGT * kGT);
  double t = 0.0;
  if (d.nchunks <= kRG) {
    // one chunk per group: the group sums are the chunks themselves
    double v[kRG];
#pragma unroll
    for (int g = 0; g < kRG; ++g) v[g] = g < d.nchunks ? src[g * stride] : 0.0;
#pragma unroll
    for (int g = 0; g < kRG; ++g) t += v[g];
  } else {
    for (int g = 0; g < kRG; ++g) {
      double s = 0.0;
      for (int ch = g; ch < d.nchunks; ch += kRG) s += src[ch * stride];
      t += s;
    }
  }
  global_ptr(d.S)[rel] = t;
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
  hipLaunchKernelGGL(gram_grouped_reduce, dim3((unsigned)((total_elems + 255) / 256)),
                     dim3(256), 0, st, mats, elem_off, n_mats);
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
  else if (in_dtype == TK_F16)
    hipLaunchKernelGGL(gram_partial<_Float16>, grid, dim3(256), 0, st, (const _Float16*)Y,
                       (int)L, B, C, g.cchunk, g.T, g.npairs, part);
  else
    hipLaunchKernelGGL(gram_partial<uint16_t>, grid, dim3(256), 0, st, (const uint16_t*)Y,
                       (int)L, B, C, g.cchunk, g.T, g.npairs, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n = L * L;
  hipLaunchKernelGGL(gram_reduce, dim3((unsigned)((n + kRE - 1) / kRE)), dim3(256), 0, st, part,
                     (int)L, g.T, g.npairs, (int)g.nchunks, S);
  return hipGetLastError();
}

}  // namespace tk

// ---------------------------------------------------------------------------
// Allocation-free Gram: the chunk partials live in a file-scope device array
// instead of memory allocated per call.  The array's name is a host-side
// stand-in in host code; its device address comes from hipGetSymbolAddress,
// taken once per device with that device current, and only that address is
// passed to the kernels.
// ---------------------------------------------------------------------------
namespace tk {
namespace {

constexpr size_t kGramScratchDoubles = (size_t)4 << 20;  // 32 MiB per device
__device__ __align__(256) double scratch[kGramScratchDoubles];

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kScratchDevices] = {};

// Device address of this device's scratch array (looked up on first use).
int scratch_ptr(double** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchDevices)
    return fail(TK_EDEVICE, "no current device for the Gram scratch area");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(TK_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return TK_OK;
}

}  // namespace
}  // namespace tk

extern "C" int tk_gram_noalloc(int in_dtype, const void* Y, int64_t A, int64_t L, int64_t B,
                               double* S, void* stream) {
  using namespace tk;
  clear_error();
  if (!Y || !S) return fail(TK_EINVAL, "null pointer");
  if (A < 1 || L < 1 || B < 1) return fail(TK_EINVAL, "sizes must be >= 1");
  if (L > 1024) return fail(TK_EUNSUPPORTED, "L > 1024");
  if (in_dtype < TK_F64 || in_dtype > TK_F16) return fail(TK_EINVAL, "unknown dtype %d", in_dtype);
  const int64_t C = A * B;
  GramGeom g = gram_geom(L, C);
  const size_t per_chunk = (size_t)g.npairs * kGT * kGT;
  if (per_chunk > kGramScratchDoubles)
    return fail(TK_EUNSUPPORTED,
                "L=%lld needs %zu doubles of partials per column chunk; the allocation-free "
                "Gram holds %zu",
                (long long)L, per_chunk, kGramScratchDoubles);
  // fewer, longer column chunks when the partials would not fit
  const int64_t max_chunks = (int64_t)(kGramScratchDoubles / per_chunk);
  if (g.nchunks > max_chunks) {
    int64_t cc = (C + max_chunks - 1) / max_chunks;
    cc = (cc + kGC - 1) / kGC * kGC;
    g.cchunk = cc;
    g.nchunks = (C + cc - 1) / cc;
  }
  double* part = nullptr;
  if (int rc = scratch_ptr(&part)) return rc;
  hipStream_t st = (hipStream_t)stream;
  dim3 grid((unsigned)g.nchunks, (unsigned)g.npairs);
  if (in_dtype == TK_F64)
    hipLaunchKernelGGL(gram_partial<double>, grid, dim3(256), 0, st, (const double*)Y, (int)L, B,
                       C, g.cchunk, g.T, g.npairs, part);
  else if (in_dtype == TK_F32)
    hipLaunchKernelGGL(gram_partial<float>, grid, dim3(256), 0, st, (const float*)Y, (int)L, B, C,
                       g.cchunk, g.T, g.npairs, part);
  else if (in_dtype == TK_F16)
    hipLaunchKernelGGL(gram_partial<_Float16>, grid, dim3(256), 0, st, (const _Float16*)Y,
                       (int)L, B, C, g.cchunk, g.T, g.npairs, part);
  else
    hipLaunchKernelGGL(gram_partial<uint16_t>, grid, dim3(256), 0, st, (const uint16_t*)Y,
                       (int)L, B, C, g.cchunk, g.T, g.npairs, part);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    const int64_t n = L * L;
    hipLaunchKernelGGL(gram_reduce, dim3((unsigned)((n + kRE - 1) / kRE)), dim3(256), 0, st, part,
                       (int)L, g.T, g.npairs, (int)g.nchunks, S);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return fail(TK_EDEVICE, "gram: %s", hipGetErrorString(e));
  return TK_OK;
}
