// TTM node kernels (Sec. 2.1): Out = In x_n F^T without unfolding.
//
// A node multiplies its input along mode n by the transpose of the L x K
// factor F.  Seen row-major as [A, L, B] (A = product of the lengths before
// mode n, B = after it) the operation is, for every "column" (a, b),
//
//     Out[a, k, b] = sum_l F[l, k] * In[a, l, b],      0 <= k < K,
//
// i.e. F^T applied to every mode-n fiber.  Columns with consecutive b are
// contiguous in memory, so a wave that owns consecutive columns reads In with
// unit stride (coalesced) for every l and writes Out the same way.
//
// FP32 arithmetic runs on v_mfma_f32_4x4x1_16b_f32: sixteen independent 4x4
// outer products per instruction.  Block beta (lanes 4*beta..4*beta+3) takes
// its 4 A-values (four k's of one F row, identical for every block) and 4
// B-values (four columns, one per lane); lane i receives D[m][i%4] for
// m = 0..3, i.e. four k's of its own column.  K is covered in groups of four,
// so only K mod 4 rows are ever padded (K = 20 wastes nothing), unlike
// 16- or 32-row tiles.  A lane loads four consecutive b of one row with one
// 16-byte load and issues one MFMA per component, so each lane ends up with
// four consecutive b for each k and stores them with one 16-byte store.
//
// FP64 arithmetic (FP64 storage) uses plain FP64 FMAs on an LDS-staged tile.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "device.h"
#include "internal.h"
#include "kernels.h"

namespace tk {

__device__ __forceinline__ f4 mfma4x4x1(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}

// Stage the factor slice used by this block in LDS as FT[r][l][g] = F[l, k0+4g+r]
// (zero beyond K), so that lane i reads its A-values FT[i%4][l][0..KG-1]
// contiguously.
template <int KG>
__device__ __forceinline__ void stage_factor(float* FT, const float* __restrict__ F, int L,
                                             int Kt, int k0) {
  const int total = 4 * L * KG;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int g = e % KG;
    const int t = e / KG;
    const int l = t % L;
    const int r = t / L;
    const int k = k0 + 4 * g + r;
    FT[e] = (k < Kt) ? F[(int64_t)l * Kt + k] : 0.f;
  }
}

// ------------------------------------------------------------------ wide path --
// Requires B % 4 == 0.  A wave owns 256 consecutive columns; lane i owns
// columns c0 + 4i .. c0 + 4i + 3 (same a, consecutive b).  grid.y splits K
// into chunks of 4*KG rows.  NT: the input is streamed (read once, e.g. T at
// the root), so its loads bypass cache retention.
// MFMA chain of one wide-path lane over rows [l0, l1) of its four columns
// (input at p, row stride B); acc[g][j][m] is output k = k0 + 4g + m of
// column j.  Software-pipelined: U rows are in flight from the start, and
// each row's registers are refilled with the row U further on as soon as the
// MFMAs that consume them are issued, so U loads stay outstanding while the
// MFMAs run; the factor values of the next row are read from LDS one row
// ahead.  Rows wait in registers as loaded (2-byte inputs: two registers per
// row, converted at use).
template <int KG, typename TIn, bool NT>
__device__ __forceinline__ void wide_chain(const TIn* __restrict__ p, int64_t B,
                                           const float* __restrict__ ft, int l0, int l1,
                                           f4 (&acc)[KG][4]) {
  typedef typename Raw4<TIn>::type R;
  constexpr int U = 8;
  int l = l0;
  if (l + U <= l1) {
    R x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = load4_raw<NT>(p + (int64_t)(l + u) * B);
    float fa[KG];
#pragma unroll
    for (int g = 0; g < KG; ++g) fa[g] = ft[l * KG + g];
    // rows l .. l + U - 1 in registers; rows up to l + 2U - 1 < l1 exist
    for (; l + 2 * U <= l1; l += U) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        float fn[KG];
#pragma unroll
        for (int g = 0; g < KG; ++g) fn[g] = ft[(l + u + 1) * KG + g];
        const f4 xv = raw4_to_f32<TIn>(x[u]);
#pragma unroll
        for (int g = 0; g < KG; ++g)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[g][j] = mfma4x4x1(fa[g], xv[j], acc[g][j]);
        x[u] = load4_raw<NT>(p + (int64_t)(l + U + u) * B);
#pragma unroll
        for (int g = 0; g < KG; ++g) fa[g] = fn[g];
        // one row per group: the refill stays behind its row's MFMAs
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    // the last batch in registers: nothing further to fetch
#pragma unroll
    for (int u = 0; u < U; ++u) {
      float fn[KG];
      if (u + 1 < U) {
#pragma unroll
        for (int g = 0; g < KG; ++g) fn[g] = ft[(l + u + 1) * KG + g];
      }
      const f4 xv = raw4_to_f32<TIn>(x[u]);
#pragma unroll
      for (int g = 0; g < KG; ++g)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[g][j] = mfma4x4x1(fa[g], xv[j], acc[g][j]);
      if (u + 1 < U) {
#pragma unroll
        for (int g = 0; g < KG; ++g) fa[g] = fn[g];
      }
    }
    l += U;
  }
  for (; l < l1; ++l) {
    const f4 x = load4_f32<NT>(p + (int64_t)l * B);
#pragma unroll
    for (int g = 0; g < KG; ++g) {
      const float fa = ft[l * KG + g];
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[g][j] = mfma4x4x1(fa, x[j], acc[g][j]);
    }
  }
}

template <int KG>
__device__ __forceinline__ void wide_store(float* __restrict__ out, int64_t a, int64_t b,
                                           int64_t B, int Kt, int k0, const f4 (&acc)[KG][4]) {
  float* q = out + (a * Kt) * B + b;
#pragma unroll
  for (int g = 0; g < KG; ++g)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int k = k0 + 4 * g + m;
      if (k < Kt) {
        f4 v = {acc[g][0][m], acc[g][1][m], acc[g][2][m], acc[g][3][m]};
        *reinterpret_cast<f4*>(q + (int64_t)k * B) = v;
      }
    }
}

template <int KG, typename TIn, bool NT>
__device__ __forceinline__ void wide_body(const TIn* __restrict__ in, const float* __restrict__ F,
                                          float* __restrict__ out, int64_t C, int L, int64_t B,
                                          int Kt, int64_t blk, int k0, float* smem) {
  stage_factor<KG>(smem, F, L, Kt, k0);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t c = (blk * 4 + wave) * 256 + 4 * lane;
  if ((blk * 4 + wave) * 256 >= C) return;  // whole wave idle
  const bool active = c < C;
  // lanes past the end read row a = 0 (always in bounds) and store nothing:
  // the loads stay unconditional, so they are issued back to back
  const int64_t a = active ? c / B : 0;
  const int64_t b = active ? c - a * B : 0;
  const TIn* p = in + (a * L) * B + b;
  const float* ft = smem + (lane & 3) * L * KG;

  f4 acc[KG][4];
#pragma unroll
  for (int g = 0; g < KG; ++g)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[g][j] = f4{0.f, 0.f, 0.f, 0.f};
  wide_chain<KG, TIn, NT>(p, B, ft, 0, L, acc);
  if (active) wide_store<KG>(out, a, b, B, Kt, k0, acc);
}

// Split-L variant for grids too small to fill the chip: the four waves of a
// block share 256 columns and take four contiguous ranges of rows l (whole
// batches of eight); waves 1..3 leave their partial sums in LDS, over the
// factor slice once every wave is done with it, and wave 0 adds them in wave
// order (a fixed order) and stores.  The input is still read once.
constexpr int kSplitLMaxKG = 5;  // 3 partial sets of 16 KG floats per lane fit in 64 KB
constexpr size_t splitl_lds(int L, int KG) {
  return std::max((size_t)16 * L * KG, (size_t)3 * 16 * KG * 64 * sizeof(float));
}

template <int KG, typename TIn, bool NT>
__device__ __forceinline__ void wide_splitl_body(const TIn* __restrict__ in,
                                                 const float* __restrict__ F,
                                                 float* __restrict__ out, int64_t C, int L,
                                                 int64_t B, int Kt, int64_t blk, int k0,
                                                 float* smem) {
  static_assert(KG <= kSplitLMaxKG, "partials exceed the LDS budget");
  stage_factor<KG>(smem, F, L, Kt, k0);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t c = blk * 256 + 4 * lane;
  const bool active = c < C;
  const int64_t a = active ? c / B : 0;
  const int64_t b = active ? c - a * B : 0;
  const TIn* p = in + (a * L) * B + b;
  const float* ft = smem + (lane & 3) * L * KG;
  const int lq = ((L + 3) / 4 + 7) / 8 * 8;
  const int l0 = min(L, wave * lq), l1 = min(L, l0 + lq);

  f4 acc[KG][4];
#pragma unroll
  for (int g = 0; g < KG; ++g)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[g][j] = f4{0.f, 0.f, 0.f, 0.f};
  wide_chain<KG, TIn, NT>(p, B, ft, l0, l1, acc);
  __syncthreads();  // every wave is done with the factor slice
  // partial set w - 1, element e = (g, j, m): red[((w - 1) * 16 KG + e) * 64 + lane]
  if (wave > 0) {
    float* red = smem + (wave - 1) * 16 * KG * 64 + lane;
#pragma unroll
    for (int g = 0; g < KG; ++g)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int m = 0; m < 4; ++m) red[((g * 4 + j) * 4 + m) * 64] = acc[g][j][m];
  }
  __syncthreads();
  if (wave != 0) return;
  // one K-group at a time, partial sets in wave order (few live registers)
#pragma unroll
  for (int g = 0; g < KG; ++g) {
    const float* red = smem + g * 16 * 64 + lane;
#pragma unroll 1
    for (int w = 0; w < 3; ++w) {
      float v[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) v[e] = red[(w * 16 * KG + e) * 64];
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int m = 0; m < 4; ++m) acc[g][j][m] += v[j * 4 + m];
    }
  }
  if (active) wide_store<KG>(out, a, b, B, Kt, k0, acc);
}

template <int KG, typename TIn, bool NT>
__global__ __launch_bounds__(256) void ttm_wide_splitl_f32(const TIn* __restrict__ in,
                                                           const float* __restrict__ F,
                                                           float* __restrict__ out, int64_t C,
                                                           int L, int64_t B, int Kt) {
  extern __shared__ float smem[];
  if constexpr (KG <= kSplitLMaxKG)
    wide_splitl_body<KG, TIn, NT>(in, F, out, C, L, B, Kt, blockIdx.x, blockIdx.y * 4 * KG, smem);
}

// Four waves per SIMD where the accumulators leave room (KG <= 4: the
// pipelined chain holds 16 KG accumulators, 32 input registers and the
// factor values of two rows).
constexpr int wide_min_waves(int KG) { return KG <= 4 ? 4 : 1; }

template <int KG, typename TIn, bool NT>
__global__ __launch_bounds__(256, wide_min_waves(KG)) void ttm_wide_f32(const TIn* __restrict__ in,
                                                    const float* __restrict__ F,
                                                    float* __restrict__ out, int64_t C, int L,
                                                    int64_t B, int Kt) {
  extern __shared__ float smem[];
  wide_body<KG, TIn, NT>(in, F, out, C, L, B, Kt, blockIdx.x, blockIdx.y * 4 * KG, smem);
}

// Wide variant with 4-byte loads, for runs of B (>= 32) that cannot be read
// 16 bytes at a time (B % 4 != 0, or an unaligned base): lane i of wave w
// owns the flattened columns c = 256 w + i + 64 j, j = 0..3, each with its
// own (a, b); every load instruction reads 64 consecutive columns of one row
// l (one run of B, or the end of one and the start of the next).
constexpr int kWideScalarMinB = 32;

template <int KG, typename TIn, bool NT>
__device__ __forceinline__ void wide_scalar_body(const TIn* __restrict__ in,
                                                 const float* __restrict__ F,
                                                 float* __restrict__ out, int64_t C, int L,
                                                 int64_t B, int Kt, int64_t blk, int k0,
                                                 float* smem) {
  stage_factor<KG>(smem, F, L, Kt, k0);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t c0 = (blk * 4 + wave) * 256;
  if (c0 >= C) return;  // whole wave idle
  const TIn* p[4];
  int64_t q[4];
  bool act[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t c = c0 + lane + 64 * j;
    act[j] = c < C;
    // columns past the end read column 0 (always in bounds) and store nothing
    const int64_t a = act[j] ? c / B : 0;
    const int64_t b = act[j] ? c - a * B : 0;
    p[j] = in + (a * L) * B + b;
    q[j] = (a * Kt) * B + b;
  }
  const float* ft = smem + (lane & 3) * L * KG;
  f4 acc[KG][4];
#pragma unroll
  for (int g = 0; g < KG; ++g)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[g][j] = f4{0.f, 0.f, 0.f, 0.f};
  constexpr int U = 8;
  auto ld = [&](const TIn* a) -> float {
    if constexpr (NT)
      return Elem<TIn>::to_f32(__builtin_nontemporal_load(a));
    else
      return Elem<TIn>::to_f32(*a);
  };
  // software-pipelined like the wide chain: U rows in flight, each row's
  // registers refilled with the row U further on once its MFMAs are issued
  int l = 0;
  if (U <= L) {
    float x[U][4];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int j = 0; j < 4; ++j) x[u][j] = ld(p[j] + (int64_t)u * B);
    for (; l + 2 * U <= L; l += U) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int g = 0; g < KG; ++g) {
          const float fa = ft[(l + u) * KG + g];
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[g][j] = mfma4x4x1(fa, x[u][j], acc[g][j]);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) x[u][j] = ld(p[j] + (int64_t)(l + U + u) * B);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int g = 0; g < KG; ++g) {
        const float fa = ft[(l + u) * KG + g];
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[g][j] = mfma4x4x1(fa, x[u][j], acc[g][j]);
      }
    l += U;
  }
  for (; l < L; ++l) {
    float x[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = ld(p[j] + (int64_t)l * B);
#pragma unroll
    for (int g = 0; g < KG; ++g) {
      const float fa = ft[l * KG + g];
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[g][j] = mfma4x4x1(fa, x[j], acc[g][j]);
    }
  }
#pragma unroll
  for (int g = 0; g < KG; ++g)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int k = k0 + 4 * g + m;
      if (k < Kt)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (act[j]) out[q[j] + (int64_t)k * B] = acc[g][j][m];
    }
}

template <int KG, typename TIn, bool NT>
__global__ __launch_bounds__(256) void ttm_wide_scalar_f32(const TIn* __restrict__ in,
                                                           const float* __restrict__ F,
                                                           float* __restrict__ out, int64_t C,
                                                           int L, int64_t B, int Kt) {
  extern __shared__ float smem[];
  wide_scalar_body<KG, TIn, NT>(in, F, out, C, L, B, Kt, blockIdx.x, blockIdx.y * 4 * KG, smem);
}

// ------------------------------------------------------------- large ranks --
// Wide grids whose rank needs more than one LDS-resident factor slice (the
// real tensors' K_n of 80-306): the slice of 4 KG factor columns is staged
// kLkRows rows at a time (a block barrier per chunk of rows), so KG is not
// capped by L; and the K-chunks of one 1024-column tile run as consecutive
// work items of one XCD (blocks are mapped chunk-fastest within each XCD's
// share of the grid), so the tile's input comes from HBM once and from that
// XCD's L2 for the other K-chunks, which read the same rows at about the same
// time.  SCALAR: lane i of wave w owns flattened columns 256 w + i + 64 j
// (4-byte loads, any B); else lane i owns columns 256 w + 4 i .. + 3 (16-byte
// loads, B % 4 == 0, aligned).  Normal loads: the K-chunks re-read the input.
constexpr int kLkRows = 64;

template <int KG>
__device__ __forceinline__ void stage_factor_rows(float* FT, const float* __restrict__ F, int l0,
                                                  int l1, int Kt, int k0) {
  // FT[(r * kLkRows + (l - l0)) * KG + g] = F[l, k0 + 4 g + r] (0 past K or l1)
  constexpr int total = 4 * kLkRows * KG;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int g = e % KG;
    const int t = e / KG;
    const int l = l0 + t % kLkRows;
    const int r = t / kLkRows;
    const int k = k0 + 4 * g + r;
    FT[e] = (k < Kt && l < l1) ? F[(int64_t)l * Kt + k] : 0.f;
  }
}

template <int KG, typename TIn, bool SCALAR>
__global__ __launch_bounds__(256) void ttm_lk_f32(const TIn* __restrict__ in,
                                                  const float* __restrict__ F,
                                                  float* __restrict__ out, int64_t C, int L,
                                                  int64_t B, int Kt, int chunks, int64_t nwork,
                                                  int64_t per_xcd) {
  extern __shared__ float smem[];
  const int64_t w = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (w >= nwork) return;  // the whole block: no barrier is skipped by part of it
  const int64_t blk = w / chunks;
  const int k0 = (int)(w - blk * chunks) * 4 * KG;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t c0 = (blk * 4 + wave) * 256;
  const bool live = c0 < C;  // idle waves still take part in the staging barriers
  const TIn* p[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t c = SCALAR ? c0 + lane + 64 * j : c0 + 4 * lane + j;
    // columns past the end read column 0 (always in bounds) and store nothing
    const int64_t a = c < C ? c / B : 0;
    const int64_t b = c < C ? c - a * B : 0;
    p[j] = in + (a * L) * B + b;
  }
  f4 acc[KG][4];
#pragma unroll
  for (int g = 0; g < KG; ++g)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[g][j] = f4{0.f, 0.f, 0.f, 0.f};
  for (int l0 = 0; l0 < L; l0 += kLkRows) {
    const int l1 = min(L, l0 + kLkRows);
    __syncthreads();  // every wave is done with the previous rows' factor
    stage_factor_rows<KG>(smem, F, l0, l1, Kt, k0);
    __syncthreads();
    if (!live) continue;
    const float* ft = smem + (lane & 3) * kLkRows * KG - l0 * KG;
    if constexpr (SCALAR) {
      constexpr int U = 8;
      int l = l0;
      for (; l + U <= l1; l += U) {
        float x[U][4];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int j = 0; j < 4; ++j) x[u][j] = Elem<TIn>::to_f32(p[j][(int64_t)(l + u) * B]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int g = 0; g < KG; ++g) {
            const float fa = ft[(l + u) * KG + g];
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[g][j] = mfma4x4x1(fa, x[u][j], acc[g][j]);
          }
      }
      for (; l < l1; ++l) {
        float x[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) x[j] = Elem<TIn>::to_f32(p[j][(int64_t)l * B]);
#pragma unroll
        for (int g = 0; g < KG; ++g) {
          const float fa = ft[l * KG + g];
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[g][j] = mfma4x4x1(fa, x[j], acc[g][j]);
        }
      }
    } else {
      wide_chain<KG, TIn, false>(p[0], B, ft, l0, l1, acc);
    }
  }
  if (!live) return;
  if constexpr (SCALAR) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t c = c0 + lane + 64 * j;
      if (c >= C) continue;
      const int64_t a = c / B;
      float* q = out + (a * Kt) * B + (c - a * B);
#pragma unroll
      for (int g = 0; g < KG; ++g)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int k = k0 + 4 * g + m;
          if (k < Kt) q[(int64_t)k * B] = acc[g][j][m];
        }
    }
  } else {
    const int64_t c = c0 + 4 * lane;
    if (c < C) {
      const int64_t a = c / B;
      wide_store<KG>(out, a, c - a * B, B, Kt, k0, acc);
    }
  }
}

// Slab-aligned variant for runs of B (<= 256) that are not whole 128-byte
// lines while every slab In[a, :, :] starts on a line: a wave takes
// 64 / (B / 4) whole slabs, B / 4 lanes each (the rest idle), so no cache
// line is shared with another wave and the input can be streamed.
template <int KG, typename TIn, bool NT>
__global__ __launch_bounds__(256) void ttm_wide_slab_f32(const TIn* __restrict__ in,
                                                         const float* __restrict__ F,
                                                         float* __restrict__ out, int64_t A,
                                                         int L, int64_t B, int Kt) {
  extern __shared__ float smem[];
  const int k0 = blockIdx.y * 4 * KG;
  stage_factor<KG>(smem, F, L, Kt, k0);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int lpa = (int)(B / 4), apw = 64 / lpa;
  const int64_t a0 = ((int64_t)blockIdx.x * 4 + wave) * apw;
  if (a0 >= A) return;  // whole wave idle
  const int al = lane / lpa;
  const bool active = al < apw && a0 + al < A;
  // idle lanes read slab a0 (always in bounds) and store nothing
  const int64_t a = active ? a0 + al : a0;
  const int64_t b = active ? 4 * (lane % lpa) : 0;
  const TIn* p = in + (a * L) * B + b;
  const float* ft = smem + (lane & 3) * L * KG;
  f4 acc[KG][4];
#pragma unroll
  for (int g = 0; g < KG; ++g)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[g][j] = f4{0.f, 0.f, 0.f, 0.f};
  wide_chain<KG, TIn, NT>(p, B, ft, 0, L, acc);
  if (active) wide_store<KG>(out, a, b, B, Kt, k0, acc);
}

// ------------------------------------------------------------------- row path --
// B == 1 (the last mode): Out[a, k] = sum_l In[a, l] F[l, k], rows of In
// contiguous.  In a 4x4x1 MFMA the B operand of lane i is a value of its own
// row a, the A operands (four k's of row l of F) are the same for every block,
// so lane i accumulates four k's of row a.
//
// Direct variant, for rows too long to stage the factor slice beside the row
// tiles below: requires L % 4 == 0.  Lane i owns row a = 256*block + thread
// and walks it with 16-byte loads (eight in flight); each load feeds four
// MFMAs, one per l.  Every load instruction touches 64 rows, so it moves less
// than the staged variant.
template <int KG, typename TIn, bool NT>
__device__ __forceinline__ void rows_direct_body(const TIn* __restrict__ in, const float* __restrict__ F,
                                          float* __restrict__ out, int64_t A, int L, int Kt,
                                          int64_t blk, int k0, float* smem) {
  stage_factor<KG>(smem, F, L, Kt, k0);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t wave_row0 = blk * 256 + (threadIdx.x & ~63);
  if (wave_row0 >= A) return;  // whole wave idle
  const int64_t a = wave_row0 + lane;
  const bool active = a < A;
  const TIn* p = in + (active ? a : 0) * L;  // lanes past the end re-read row 0
  const float* ft = smem + (lane & 3) * L * KG;

  f4 acc[KG];
#pragma unroll
  for (int g = 0; g < KG; ++g) acc[g] = f4{0.f, 0.f, 0.f, 0.f};

  constexpr int U = 8;
  int l = 0;
  for (; l + 4 * U <= L; l += 4 * U) {
    f4 x[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      x[u] = load4_f32<NT>(p + l + 4 * u);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int g = 0; g < KG; ++g)
          acc[g] = mfma4x4x1(ft[(l + 4 * u + j) * KG + g], x[u][j], acc[g]);
  }
  for (; l < L; l += 4) {
    const f4 x = load4_f32<NT>(p + l);
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int g = 0; g < KG; ++g) acc[g] = mfma4x4x1(ft[(l + j) * KG + g], x[j], acc[g]);
  }
  if (!active) return;
  float* q = out + a * Kt;
#pragma unroll
  for (int g = 0; g < KG; ++g)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int k = k0 + 4 * g + m;
      if (k < Kt) q[k] = acc[g][m];
    }
}

template <int KG, typename TIn, bool NT>
__global__ __launch_bounds__(256) void ttm_rows_direct_f32(const TIn* __restrict__ in,
                                                           const float* __restrict__ F,
                                                           float* __restrict__ out, int64_t A,
                                                           int L, int Kt) {
  extern __shared__ float smem[];
  rows_direct_body<KG, TIn, NT>(in, F, out, A, L, Kt, blockIdx.x, blockIdx.y * 4 * KG, smem);
}

// Staged variants: a wave owns 64 consecutive rows and reads them
// cooperatively in chunks of kRowLC columns into a padded LDS tile of its own
// (pitch kRowLC + 1, so the 64 lanes reading one column hit distinct banks);
// then every lane runs the MFMA chain over its own row.
constexpr int kRowLC = 32;
constexpr int kRowPitch = kRowLC + 1;
constexpr size_t kRowStageBytes = (size_t)4 * 64 * kRowPitch * sizeof(float);  // 4 waves

// Orders this wave's LDS accesses for the compiler; the LDS itself executes
// one wave's accesses in issue order, so no wait is needed between them.
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// A wave reads its 64 rows chunk by chunk with every load instruction
// covering whole row segments: V4 (L % 4 == 0, rows aligned for
// four-element loads) -- load slot u of a lane is four columns of row
// 8u + lane/8, so eight lanes read 128 contiguous bytes of FP32; otherwise
// (odd L, or an unaligned base) one element per load -- slot u is column
// lane % 32 of row 2u + lane/32, so 32 lanes read one row's 32 consecutive
// elements.  The next chunk's loads are issued before the current chunk's
// MFMAs, and the tile is private to the wave: after the factor is staged the
// waves of a block never wait for each other.
template <int KG, typename TIn, bool NT, bool V4 = true>
__device__ __forceinline__ void rows_body(const TIn* __restrict__ in, const float* __restrict__ F,
                                          float* __restrict__ out, int64_t A, int L, int Kt,
                                          int64_t blk, int k0, float* smem) {
  stage_factor<KG>(smem, F, L, Kt, k0);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t row0 = blk * 256 + wave * 64;
  if (row0 >= A) return;  // whole wave idle
  const int nrows = (int)min((int64_t)64, A - row0);
  float* Xs = smem + 4 * L * KG + wave * 64 * kRowPitch;
  const float* ft = smem + (lane & 3) * L * KG;
  const TIn* base = in + row0 * (int64_t)L;

  f4 acc[KG];
#pragma unroll
  for (int g = 0; g < KG; ++g) acc[g] = f4{0.f, 0.f, 0.f, 0.f};

  // slots past the wave's last row re-read that row; in a short last chunk,
  // lanes past its end re-read its last columns
  constexpr int kSlots = V4 ? 8 : 32;
  using Slot = typename std::conditional<V4, f4, float>::type;
  Slot v[kSlots];
  const int rq = V4 ? lane >> 3 : lane >> 5;                  // row within a slot's group
  const int cq = V4 ? 4 * (lane & 7) : lane & (kRowLC - 1);   // first column
  constexpr int kRowStep = V4 ? 8 : 2;                        // rows between slots
  auto load_chunk = [&](int l0) {
    const int lc = min(kRowLC, L - l0);
    const int c = l0 + min(cq, lc - (V4 ? 4 : 1));
#pragma unroll
    for (int u = 0; u < kSlots; ++u) {
      const TIn* pr = base + (int64_t)min(kRowStep * u + rq, nrows - 1) * L + c;
      if constexpr (V4) {
        v[u] = load4_f32<NT>(pr);
      } else if constexpr (NT) {
        v[u] = Elem<TIn>::to_f32(__builtin_nontemporal_load(pr));
      } else {
        v[u] = Elem<TIn>::to_f32(*pr);
      }
    }
  };
  load_chunk(0);
  const float* xr = Xs + lane * kRowPitch;
  for (int l0 = 0; l0 < L; l0 += kRowLC) {
    wave_lds_fence();  // the previous chunk's reads are issued before these writes
#pragma unroll
    for (int u = 0; u < kSlots; ++u) {
      float* xs = Xs + (kRowStep * u + rq) * kRowPitch + cq;
      if constexpr (V4) {
#pragma unroll
        for (int j = 0; j < 4; ++j) xs[j] = v[u][j];
      } else {
        xs[0] = v[u];
      }
    }
    wave_lds_fence();
    if (l0 + kRowLC < L) load_chunk(l0 + kRowLC);
    if (L - l0 >= kRowLC) {
#pragma unroll
      for (int c = 0; c < kRowLC; ++c)
#pragma unroll
        for (int g = 0; g < KG; ++g) acc[g] = mfma4x4x1(ft[(l0 + c) * KG + g], xr[c], acc[g]);
    } else {
      for (int c = 0; c < L - l0; ++c)
#pragma unroll
        for (int g = 0; g < KG; ++g) acc[g] = mfma4x4x1(ft[(l0 + c) * KG + g], xr[c], acc[g]);
    }
  }
  if (lane >= nrows) return;
  float* q = out + (row0 + lane) * Kt;
  if (Kt % 4 == 0 && (uintptr_t)out % 16 == 0) {
#pragma unroll
    for (int g = 0; g < KG; ++g)
      if (k0 + 4 * g < Kt) *reinterpret_cast<f4*>(q + k0 + 4 * g) = acc[g];
  } else {
#pragma unroll
    for (int g = 0; g < KG; ++g)
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int k = k0 + 4 * g + m;
        if (k < Kt) q[k] = acc[g][m];
      }
  }
}

template <int KG, typename TIn, bool NT, bool V4>
__global__ __launch_bounds__(256) void ttm_rows_f32(const TIn* __restrict__ in,
                                                    const float* __restrict__ F,
                                                    float* __restrict__ out, int64_t A, int L,
                                                    int Kt) {
  extern __shared__ float smem[];
  rows_body<KG, TIn, NT, V4>(in, F, out, A, L, Kt, blockIdx.x, blockIdx.y * 4 * KG, smem);
}

// Single-element row body with block barriers around each chunk (one element
// per load, eight rows' 32 consecutive elements per load instruction), kept
// for the grouped kernel: there the barrier-free body above measured slower
// (the persistent kernel's register budget is shared by all bodies).
template <int KG, typename TIn, bool NT>
__device__ __forceinline__ void rows_lds_body(const TIn* __restrict__ in,
                                              const float* __restrict__ F,
                                              float* __restrict__ out, int64_t A, int L, int Kt,
                                              int64_t blk, int k0, float* smem) {
  float* FT = smem;
  stage_factor<KG>(FT, F, L, Kt, k0);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  float* Xs = smem + 4 * L * KG + wave * 64 * kRowPitch;
  const int64_t row0 = blk * 256 + wave * 64;
  const int nrows = (int)max((int64_t)0, min((int64_t)64, A - row0));  // rows of this wave
  const float* ft = FT + (lane & 3) * L * KG;

  f4 acc[KG];
#pragma unroll
  for (int g = 0; g < KG; ++g) acc[g] = f4{0.f, 0.f, 0.f, 0.f};

  for (int l0 = 0; l0 < L; l0 += kRowLC) {
    const int lc = min(kRowLC, L - l0);
    __syncthreads();  // the previous chunk has been consumed (and FT staged)
    constexpr int kPer = 64 * kRowLC / 64;  // one element per load
    float v[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int q = lane + 64 * u;
      const int r = q / kRowLC, c = q % kRowLC;
      v[u] = (r < nrows && c < lc) ? Elem<TIn>::to_f32(in[(row0 + r) * L + l0 + c]) : 0.f;
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int q = lane + 64 * u;
      Xs[(q / kRowLC) * kRowPitch + q % kRowLC] = v[u];
    }
    __syncthreads();
    for (int c = 0; c < lc; ++c) {
      const float x = Xs[lane * kRowPitch + c];
#pragma unroll
      for (int g = 0; g < KG; ++g) acc[g] = mfma4x4x1(ft[(l0 + c) * KG + g], x, acc[g]);
    }
  }
  if (lane >= nrows) return;
  float* q = out + (row0 + lane) * Kt;
#pragma unroll
  for (int g = 0; g < KG; ++g)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int k = k0 + 4 * g + m;
      if (k < Kt) q[k] = acc[g][m];
    }
}

// ------------------------------------------------------------- BF16 MFMA paths --
// TK_C_BF16: both operands rounded to bfloat16 (round to nearest even), FP32
// accumulation, on v_mfma_f32_4x4x4_16b_bf16: the 4x4x1 block structure of the
// FP32 path with a reduction depth of four, so each MFMA consumes four
// consecutive l of one column.  Lanes load the same coalesced 16-byte row
// pieces as the FP32 wide path (four rows l..l+3) and transpose them in
// registers into per-column operands; a row-path lane reads four consecutive
// l of its own row directly.
// TK_C_BF16X3: split-precision, a ~ a_hi + a_lo with a_hi = bf16(a),
// a_lo = bf16(a - a_hi); a*b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi (three MFMAs,
// the dropped a_lo b_lo term is ~2^-16 of the product).  A BF16-stored input
// has no low part, so only two products remain.
// The factor is staged in LDS already split and packed: entry (r, lb, g) holds
// F[4lb..4lb+3, k0 + 4g + r] as four bfloat16.
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
  bf2 v = {(__bf16)a, (__bf16)b};  // hardware round-to-nearest-even pack on gfx950
  return __builtin_bit_cast(uint32_t, v);
}
__device__ __forceinline__ float bf16_low_f32(uint32_t u) { return __uint_as_float(u << 16); }
__device__ __forceinline__ float bf16_high_f32(uint32_t u) { return __uint_as_float(u & 0xFFFF0000u); }
__device__ __forceinline__ s4 as_s4(uint2 v) { return __builtin_bit_cast(s4, v); }
__device__ __forceinline__ f4 mfma4x4x4bf16(s4 a, s4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(a, b, c, 0, 0, 0);
}
// hi/lo packs of four consecutive reduction values
__device__ __forceinline__ void split4(float x0, float x1, float x2, float x3, uint2& hi,
                                      uint2& lo) {
  hi.x = pack_bf16(x0, x1);
  hi.y = pack_bf16(x2, x3);
  lo.x = pack_bf16(x0 - bf16_low_f32(hi.x), x1 - bf16_high_f32(hi.x));
  lo.y = pack_bf16(x2 - bf16_low_f32(hi.y), x3 - bf16_high_f32(hi.y));
}

template <int KG, bool X3, bool F3 = false>
__device__ __forceinline__ void stage_factor_bf16(uint2* FH, uint2* FL, uint2* FL2,
                                                  const float* __restrict__ F, int L, int LB,
                                                  int Kt, int k0) {
  const int total = 4 * LB * KG;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int g = e % KG;
    const int t = e / KG;
    const int lb = t % LB;
    const int r = t / LB;
    const int k = k0 + 4 * g + r;
    float f[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int l = 4 * lb + q;
      f[q] = (k < Kt && l < L) ? F[(int64_t)l * Kt + k] : 0.f;
    }
    uint2 hi, lo;
    split4(f[0], f[1], f[2], f[3], hi, lo);
    FH[e] = hi;
    if (X3) FL[e] = lo;
    if constexpr (F3) {
      // third term: f - hi - lo (both differences exact in FP32) is exactly a
      // bfloat16, so hi + lo + lo2 reproduces the FP32 factor bit for bit
      uint2 lo2;
      lo2.x = pack_bf16(f[0] - bf16_low_f32(hi.x) - bf16_low_f32(lo.x),
                        f[1] - bf16_high_f32(hi.x) - bf16_high_f32(lo.x));
      lo2.y = pack_bf16(f[2] - bf16_low_f32(hi.y) - bf16_low_f32(lo.y),
                        f[3] - bf16_high_f32(hi.y) - bf16_high_f32(lo.y));
      FL2[e] = lo2;
    }
  }
}

// One block of four rows x[q] (q = l mod 4) of the lane's four columns:
// column j's operand is the four values x[0..3][j].
template <int KG, bool X3, bool kSplitIn, bool F3 = false>
__device__ __forceinline__ void wide_bf16_block(f4 (&acc)[KG][4], const f4 (&x)[4],
                                                const uint2* fh, const uint2* fl,
                                                const uint2* fl2 = nullptr) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    uint2 bh, bl;
    split4(x[0][j], x[1][j], x[2][j], x[3][j], bh, bl);
#pragma unroll
    for (int g = 0; g < KG; ++g) {
      const uint2 ah = fh[g];
      acc[g][j] = mfma4x4x4bf16(as_s4(ah), as_s4(bh), acc[g][j]);
      if (X3) {
        acc[g][j] = mfma4x4x4bf16(as_s4(fl[g]), as_s4(bh), acc[g][j]);
        if (kSplitIn) acc[g][j] = mfma4x4x4bf16(as_s4(ah), as_s4(bl), acc[g][j]);
      }
      if (F3) acc[g][j] = mfma4x4x4bf16(as_s4(fl2[g]), as_s4(bh), acc[g][j]);
    }
  }
}

// Wide path (B % 4 == 0): lane owns columns c0 + 4i .. c0 + 4i + 3.
template <int KG, typename TIn, bool NT, bool X3, bool OutBF16, bool F3 = false>
__global__ __launch_bounds__(256) void ttm_wide_bf16(const TIn* __restrict__ in,
                                                     const float* __restrict__ F,
                                                     void* __restrict__ out_, int64_t C, int L,
                                                     int64_t B, int Kt) {
  extern __shared__ uint2 sfb[];
  const int LB = (L + 3) / 4;
  uint2* FH = sfb;
  uint2* FL = sfb + 4 * LB * KG;
  uint2* FL2 = sfb + 8 * LB * KG;
  const int k0 = blockIdx.y * 4 * KG;
  stage_factor_bf16<KG, X3, F3>(FH, FL, FL2, F, L, LB, Kt, k0);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t c = ((int64_t)blockIdx.x * 4 + wave) * 256 + 4 * lane;
  if (((int64_t)blockIdx.x * 4 + wave) * 256 >= C) return;
  const bool active = c < C;
  const int64_t a = active ? c / B : 0;
  const int64_t b = active ? c - a * B : 0;
  const TIn* p = in + (a * L) * B + b;
  const uint2* fh = FH + (lane & 3) * LB * KG;
  const uint2* fl = FL + (lane & 3) * LB * KG;
  const uint2* fl2 = FL2 + (lane & 3) * LB * KG;
  constexpr bool kSplitIn = X3 && std::is_same<TIn, float>::value;

  f4 acc[KG][4];
#pragma unroll
  for (int g = 0; g < KG; ++g)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[g][j] = f4{0.f, 0.f, 0.f, 0.f};

  // blocks of four rows per step: 8 (FP32 input) or 16 (BF16 input) loads in flight
  constexpr int U = (sizeof(TIn) == 2 && KG <= 8) ? 4 : 2;
  const int LF = L / 4;  // blocks with all four rows inside L
  int lb = 0;
  for (; lb + U <= LF; lb += U) {
    f4 x[U][4];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) x[u][q] = load4_f32<NT>(p + (int64_t)(4 * (lb + u) + q) * B);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; ++u)
      wide_bf16_block<KG, X3, kSplitIn, F3>(acc, x[u], fh + (lb + u) * KG, fl + (lb + u) * KG,
                                            fl2 + (lb + u) * KG);
  }
  for (; lb < LB; ++lb) {  // remaining blocks, the last one possibly ragged
    f4 x[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int l = 4 * lb + q;
      x[q] = l < L ? load4_f32<NT>(p + (int64_t)l * B) : f4{0.f, 0.f, 0.f, 0.f};
    }
    wide_bf16_block<KG, X3, kSplitIn, F3>(acc, x, fh + lb * KG, fl + lb * KG, fl2 + lb * KG);
  }
  if (!active) return;
  const int64_t q0 = (a * Kt) * B + b;
#pragma unroll
  for (int g = 0; g < KG; ++g)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int k = k0 + 4 * g + m;
      if (k < Kt) {
        if constexpr (OutBF16) {
          // BF16 output (rounded as the next BF16 node would round it on load)
          uint2 v = {pack_bf16(acc[g][0][m], acc[g][1][m]), pack_bf16(acc[g][2][m], acc[g][3][m])};
          *reinterpret_cast<uint2*>((uint16_t*)out_ + q0 + (int64_t)k * B) = v;
        } else {
          f4 v = {acc[g][0][m], acc[g][1][m], acc[g][2][m], acc[g][3][m]};
          *reinterpret_cast<f4*>((float*)out_ + q0 + (int64_t)k * B) = v;
        }
      }
    }
}

template <int KG, bool X3, bool kSplitIn>
__device__ __forceinline__ void rows_bf16_block(f4 (&acc)[KG], const f4 x, const uint2* fh,
                                                const uint2* fl) {
  uint2 bh, bl;
  split4(x[0], x[1], x[2], x[3], bh, bl);
#pragma unroll
  for (int g = 0; g < KG; ++g) {
    const uint2 ah = fh[g];
    acc[g] = mfma4x4x4bf16(as_s4(ah), as_s4(bh), acc[g]);
    if (X3) {
      acc[g] = mfma4x4x4bf16(as_s4(fl[g]), as_s4(bh), acc[g]);
      if (kSplitIn) acc[g] = mfma4x4x4bf16(as_s4(ah), as_s4(bl), acc[g]);
    }
  }
}

// Row path (B == 1, L % 4 == 0): lane owns row a; four consecutive l of its
// row form one MFMA operand as loaded.
template <int KG, typename TIn, bool NT, bool X3, bool OutBF16>
__global__ __launch_bounds__(256) void ttm_rows_bf16(const TIn* __restrict__ in,
                                                     const float* __restrict__ F,
                                                     void* __restrict__ out_, int64_t A, int L,
                                                     int Kt) {
  extern __shared__ uint2 sfb[];
  const int LB = L / 4;
  uint2* FH = sfb;
  uint2* FL = sfb + 4 * LB * KG;
  const int k0 = blockIdx.y * 4 * KG;
  stage_factor_bf16<KG, X3>(FH, FL, nullptr, F, L, LB, Kt, k0);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t wave_row0 = (int64_t)blockIdx.x * 256 + (threadIdx.x & ~63);
  if (wave_row0 >= A) return;
  const int64_t a = wave_row0 + lane;
  const bool active = a < A;
  const TIn* p = in + (active ? a : 0) * L;  // lanes past the end re-read row 0
  const uint2* fh = FH + (lane & 3) * LB * KG;
  const uint2* fl = FL + (lane & 3) * LB * KG;
  constexpr bool kSplitIn = X3 && std::is_same<TIn, float>::value;

  f4 acc[KG];
#pragma unroll
  for (int g = 0; g < KG; ++g) acc[g] = f4{0.f, 0.f, 0.f, 0.f};

  constexpr int U = 8;
  int lb = 0;
  for (; lb + U <= LB; lb += U) {
    f4 x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = load4_f32<NT>(p + 4 * (lb + u));
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; ++u)
      rows_bf16_block<KG, X3, kSplitIn>(acc, x[u], fh + (lb + u) * KG, fl + (lb + u) * KG);
  }
  for (; lb < LB; ++lb)
    rows_bf16_block<KG, X3, kSplitIn>(acc, load4_f32<NT>(p + 4 * lb), fh + lb * KG, fl + lb * KG);
  if (!active) return;
#pragma unroll
  for (int g = 0; g < KG; ++g)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int k = k0 + 4 * g + m;
      if (k < Kt) {
        if constexpr (OutBF16)
          ((__bf16*)out_)[a * Kt + k] = (__bf16)acc[g][m];
        else
          ((float*)out_)[a * Kt + k] = acc[g][m];
      }
    }
}

// ------------------------------------------------------------------ tile path --
// Any B.  A block owns a tile of na consecutive a's times nb consecutive b's
// (na * nb <= 256 columns, one per thread).  The tile's rows of In are staged
// through LDS in chunks of LC rows with loads in memory order (runs of nb
// contiguous elements), then each thread reads its column from LDS.
constexpr int kTileLC = 32;

// One tile of na x nb output columns (all K rows of the K-chunk at k0):
// index `tile` = at * nbt + bt over a-tiles and b-tiles of the node.
template <int KG, typename TIn>
__device__ __forceinline__ void tile_body(const TIn* __restrict__ in, const float* __restrict__ F,
                                          float* __restrict__ out, int64_t A, int L, int64_t B,
                                          int Kt, int na, int nb, int64_t nbt, int64_t tile,
                                          int k0, float* smem) {
  float* FT = smem;
  float* X = smem + 4 * L * KG;  // [kTileLC][256]
  stage_factor<KG>(FT, F, L, Kt, k0);
  const int64_t at = tile / nbt;
  const int64_t bt = tile - at * nbt;
  const int64_t a0 = at * na;
  const int64_t b0 = bt * nb;
  const int nav = (int)min((int64_t)na, A - a0);
  const int nbv = (int)min((int64_t)nb, B - b0);
  const int col = threadIdx.x;
  const int a_loc = col / nb;
  const int b_loc = col - a_loc * nb;
  const bool active = a_loc < nav && b_loc < nbv;
  const int lane = threadIdx.x & 63;
  const float* ft = FT + (lane & 3) * L * KG;

  f4 acc[KG];
#pragma unroll
  for (int g = 0; g < KG; ++g) acc[g] = f4{0.f, 0.f, 0.f, 0.f};

  if (nb >= 64) {
    // runs of >= 64 consecutive b: thread `col` reads its own column for every
    // l (for each l the block reads nav runs of nbv consecutive values), all
    // loads of a chunk in flight, and feeds the MFMAs from registers
    __syncthreads();  // factor staged
    const TIn* src = in + ((a0 + a_loc) * L) * B + b0 + b_loc;
    for (int l0 = 0; l0 < L; l0 += kTileLC) {
      const int lc = min(kTileLC, L - l0);
      float v[kTileLC];
#pragma unroll
      for (int ll = 0; ll < kTileLC; ++ll)
        v[ll] = (active && ll < lc) ? Elem<TIn>::to_f32(src[(int64_t)(l0 + ll) * B]) : 0.f;
#pragma unroll
      for (int ll = 0; ll < kTileLC; ++ll) {
        if (ll < lc) {
#pragma unroll
          for (int g = 0; g < KG; ++g) acc[g] = mfma4x4x1(ft[(l0 + ll) * KG + g], v[ll], acc[g]);
        }
      }
    }
  } else {
    for (int l0 = 0; l0 < L; l0 += kTileLC) {
      const int lc = min(kTileLC, L - l0);
      __syncthreads();
      const int total = nav * lc * nbv;
      // short runs: consecutive threads walk b, then l, then a (contiguous
      // memory for B < nb); eight loads in flight per thread before the stores
      for (int e0 = threadIdx.x; e0 < total; e0 += 256 * 8) {
        float v[8];
        int dst[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = e0 + u * 256;
          dst[u] = -1;
          if (e < total) {
            const int bb = e % nbv;
            const int t = e / nbv;
            const int ll = t % lc;
            const int aa = t / lc;
            dst[u] = ll * 256 + aa * nb + bb;
            v[u] = Elem<TIn>::to_f32(in[((a0 + aa) * L + (l0 + ll)) * B + b0 + bb]);
          }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (dst[u] >= 0) X[dst[u]] = v[u];
      }
      __syncthreads();
      for (int ll = 0; ll < lc; ++ll) {
        const float x = active ? X[ll * 256 + col] : 0.f;
#pragma unroll
        for (int g = 0; g < KG; ++g) acc[g] = mfma4x4x1(ft[(l0 + ll) * KG + g], x, acc[g]);
      }
    }
  }
  if (!active) return;
  float* q = out + ((a0 + a_loc) * Kt) * B + b0 + b_loc;
#pragma unroll
  for (int g = 0; g < KG; ++g)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int k = k0 + 4 * g + m;
      if (k < Kt) q[(int64_t)k * B] = acc[g][m];
    }
}

template <int KG, typename TIn>
__global__ __launch_bounds__(256) void ttm_tile_f32(const TIn* __restrict__ in,
                                                    const float* __restrict__ F,
                                                    float* __restrict__ out, int64_t A, int L,
                                                    int64_t B, int Kt, int na, int nb,
                                                    int64_t nbt) {
  extern __shared__ float smem[];
  tile_body<KG, TIn>(in, F, out, A, L, B, Kt, na, nb, nbt, blockIdx.x, blockIdx.y * 4 * KG, smem);
}

// Grouped TTM for batched HOOI: the (node, tile) items of many nodes, drained
// from a device queue by a persistent grid.  Each block takes the next item
// with one atomic increment; every block leaves once the queue is empty.
// Nodes have K <= 16 (one K-chunk of four groups) and L <= Lmax.  Held to
// three waves per SIMD (the LDS of a block allows three per CU), which the
// bodies reach without spilling.
template <typename TIn, bool NT>
__global__ __launch_bounds__(256, 3) void ttm_grouped(const TtmNodeDesc* __restrict__ nodes,
                                                   const int2* __restrict__ items, int n_items,
                                                   int* __restrict__ counter) {
  extern __shared__ float smem[];
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int it = s_item;
    __syncthreads();  // every thread has read s_item and finished the previous item
    if (it >= n_items) break;
    const int2 w = items[it];
    TtmNodeDesc d = nodes[w.x];
    d.in = global_ptr(d.in);
    d.F = global_ptr(d.F);
    d.out = global_ptr(d.out);
    // streaming loads only where no 128-byte line is shared between runs
    const bool nt = NT && d.lines;
    if (d.path == kGroupedWide) {
      if (nt)
        wide_body<4, TIn, true>((const TIn*)d.in, d.F, d.out, d.A * d.B, d.L, d.B, d.K, w.y, 0,
                                smem);
      else
        wide_body<4, TIn, false>((const TIn*)d.in, d.F, d.out, d.A * d.B, d.L, d.B, d.K, w.y, 0,
                                 smem);
    } else if (d.path == kGroupedWideScalar) {
      if (nt)
        wide_scalar_body<4, TIn, true>((const TIn*)d.in, d.F, d.out, d.A * d.B, d.L, d.B, d.K,
                                       w.y, 0, smem);
      else
        wide_scalar_body<4, TIn, false>((const TIn*)d.in, d.F, d.out, d.A * d.B, d.L, d.B, d.K,
                                        w.y, 0, smem);
    } else if (d.path == kGroupedRows) {
      if (nt)
        rows_body<4, TIn, true>((const TIn*)d.in, d.F, d.out, d.A, d.L, d.K, w.y, 0, smem);
      else
        rows_body<4, TIn, false>((const TIn*)d.in, d.F, d.out, d.A, d.L, d.K, w.y, 0, smem);
    } else if (d.path == kGroupedRowsScalar) {
      rows_lds_body<4, TIn, false>((const TIn*)d.in, d.F, d.out, d.A, d.L, d.K, w.y, 0, smem);
    } else if (d.path == kGroupedRowsDirect) {
      if (nt)
        rows_direct_body<4, TIn, true>((const TIn*)d.in, d.F, d.out, d.A, d.L, d.K, w.y, 0, smem);
      else
        rows_direct_body<4, TIn, false>((const TIn*)d.in, d.F, d.out, d.A, d.L, d.K, w.y, 0,
                                        smem);
    } else
      tile_body<4, TIn>((const TIn*)d.in, d.F, d.out, d.A, d.L, d.B, d.K, d.na, d.nb, d.nbt, w.y,
                        0, smem);
  }
}

// Persistent grouped launch for the B == 1 nodes whose rows cannot be read 16
// bytes at a time (odd L): the barrier-free single-element row body (each
// wave its own LDS tile, the next chunk prefetched into registers), in a
// kernel of its own so that the registers it needs do not set the occupancy
// of the grouped kernel's other bodies.
template <typename TIn, bool NT>
__global__ __launch_bounds__(256) void ttm_grouped_rows(const TtmNodeDesc* __restrict__ nodes,
                                                        const int2* __restrict__ items,
                                                        int n_items, int* __restrict__ counter) {
  extern __shared__ float smem[];
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int it = s_item;
    __syncthreads();  // every thread has read s_item and finished the previous item
    if (it >= n_items) break;
    const int2 w = items[it];
    const TtmNodeDesc d = nodes[w.x];
    rows_body<4, TIn, NT, false>(global_ptr((const TIn*)d.in), global_ptr(d.F),
                                 global_ptr(d.out), d.A, d.L, d.K, w.y, 0, smem);
  }
}

// ------------------------------------------------------------------ FP64 path --
// Same tiling; each thread accumulates KC outputs of its column in FP64.
constexpr int kF64LC = 16;

template <int KC, typename TIn>
__global__ __launch_bounds__(256) void ttm_tile_f64(const TIn* __restrict__ in,
                                                    const double* __restrict__ F,
                                                    double* __restrict__ out, int64_t A, int L,
                                                    int64_t B, int Kt, int na, int nb,
                                                    int64_t nbt) {
  extern __shared__ double dsm[];
  double* Fs = dsm;              // [L][KC]
  double* X = dsm + L * KC;      // [kF64LC][256]
  const int k0 = blockIdx.y * KC;
  for (int e = threadIdx.x; e < L * KC; e += 256) {
    const int kk = e % KC, l = e / KC;
    Fs[e] = (k0 + kk < Kt) ? F[(int64_t)l * Kt + k0 + kk] : 0.0;
  }
  const int64_t at = blockIdx.x / nbt;
  const int64_t bt = blockIdx.x - at * nbt;
  const int64_t a0 = at * na;
  const int64_t b0 = bt * nb;
  const int nav = (int)min((int64_t)na, A - a0);
  const int nbv = (int)min((int64_t)nb, B - b0);
  const int col = threadIdx.x;
  const int a_loc = col / nb;
  const int b_loc = col - a_loc * nb;
  const bool active = a_loc < nav && b_loc < nbv;
  double acc[KC];
#pragma unroll
  for (int k = 0; k < KC; ++k) acc[k] = 0.0;
  for (int l0 = 0; l0 < L; l0 += kF64LC) {
    const int lc = min(kF64LC, L - l0);
    __syncthreads();
    const int total = nav * lc * nbv;
    for (int e = threadIdx.x; e < total; e += 256) {
      const int bb = e % nbv;
      const int t = e / nbv;
      const int ll = t % lc;
      const int aa = t / lc;
      X[ll * 256 + aa * nb + bb] =
          Elem<TIn>::to_f64(in[((a0 + aa) * L + (l0 + ll)) * B + b0 + bb]);
    }
    __syncthreads();
    if (active) {
      for (int ll = 0; ll < lc; ++ll) {
        const double x = X[ll * 256 + col];
        const double* fr = Fs + (l0 + ll) * KC;
#pragma unroll
        for (int k = 0; k < KC; ++k) acc[k] = fma(fr[k], x, acc[k]);
      }
    }
  }
  if (!active) return;
  double* q = out + ((a0 + a_loc) * Kt) * B + b0 + b_loc;
#pragma unroll
  for (int k = 0; k < KC; ++k)
    if (k0 + k < Kt) q[(int64_t)(k0 + k) * B] = acc[k];
}

// ------------------------------------------------------------------ launchers --
namespace {

constexpr int kLdsBudget = 64 * 1024;

enum class Path { kWide, kWideSplitL, kWideScalar, kRows, kTile };

template <typename TIn>
Path choose_path(const TIn* in, const float* out, int64_t B) {
  const bool in_al = (uintptr_t)in % (4 * sizeof(TIn)) == 0;
  if (B % 4 == 0 && B >= 16 && in_al && (uintptr_t)out % 16 == 0) return Path::kWide;
  if (B == 1) return Path::kRows;  // direct, or staged through LDS (short or unaligned rows)
  if (B >= kWideScalarMinB) return Path::kWideScalar;
  return Path::kTile;
}

// K-group instances compiled for the MFMA paths (KG groups of four outputs).
constexpr int kInst[] = {1, 2, 3, 4, 5, 6, 8, 12, 16};

int64_t grid_blocks(Path path, int64_t A, int64_t B) {
  if (path == Path::kWide) return (A * B + 1023) / 1024;
  if (path == Path::kWideSplitL) return (A * B + 255) / 256;
  if (path == Path::kWideScalar) return (A * B + 1023) / 1024;
  if (path == Path::kRows) return (A + 255) / 256;
  return 0;
}

// The smallest instance covering ceil(K/4) groups if it fits in `kg_cap`
// (the groups whose factor slice fits in LDS), else the largest that fits
// (K is then covered by several chunks).  Grids of fewer blocks than CUs
// trade a larger KG for more K-chunks (more blocks; the input is re-read
// from cache).
int pick_kg(int64_t K, int kg_cap, int64_t blocks) {
  const int need = (int)((K + 3) / 4);
  int kg = 1;
  for (int c : kInst)
    if (c <= kg_cap) kg = c;  // largest fitting instance
  for (int c : kInst)
    if (c >= need && c <= kg_cap) {
      kg = c;
      break;
    }
  if (blocks > 0 && blocks < 256 && need > 1) {
    // cut K into balanced chunks (2, 3, ... groups of ceil(need/chunks))
    // until the grid covers the chip
    for (int chunks = 2; chunks <= need; ++chunks) {
      const int want = (need + chunks - 1) / chunks;
      int pick = 0;
      for (int c : kInst)
        if (c >= want && c <= kg_cap) {
          pick = c;
          break;
        }
      if (pick == 0) break;
      kg = pick;
      if (blocks * ((need + kg - 1) / kg) >= 256) break;
    }
  }
  return kg;
}

// Rows that the 16-byte row body can read: L % 4 == 0, base aligned for
// four-element loads.
template <typename TIn>
bool rows_v4(const TIn* in, int64_t L) {
  return L % 4 == 0 && (uintptr_t)in % (4 * sizeof(TIn)) == 0;
}

template <typename TIn, int KG, bool NT>
hipError_t launch_f32_kg(Path path, const TIn* in, int64_t A, int L, int64_t B, const float* F,
                         int K, float* out, hipStream_t st) {
  const int chunks = (K + 4 * KG - 1) / (4 * KG);
  if (path == Path::kWide) {
    const int64_t C = A * B;
    const size_t lds = (size_t)16 * L * KG;
    dim3 grid((unsigned)((C + 1023) / 1024), (unsigned)chunks);
    // runs of B that are not whole 128-byte lines share their boundary lines
    // with a neighbouring wave: whole slabs per wave when that keeps >= 3/4
    // of the lanes busy and slabs start on lines (then streaming is safe),
    // else normal loads, which keep those lines cached.  Slabs only for FP32
    // input: with 8 bytes per lane and idle lanes, BF16 rows load too little
    // per instruction (measured slower than normal loads).
    const bool line_runs = (B * sizeof(TIn)) % 128 == 0;
    const int64_t lpa = B / 4;
    const bool slab = sizeof(TIn) == 4 && !line_runs && B <= 256 && (64 / lpa) * lpa >= 48 &&
                      ((int64_t)L * B * sizeof(TIn)) % 128 == 0;
    if (slab) {
      const int64_t apb = 4 * (64 / lpa);  // slabs per block
      dim3 sgrid((unsigned)((A + apb - 1) / apb), (unsigned)chunks);
      if (NT)
        hipLaunchKernelGGL((ttm_wide_slab_f32<KG, TIn, true>), sgrid, dim3(256), lds, st, in, F,
                           out, A, L, B, K);
      else
        hipLaunchKernelGGL((ttm_wide_slab_f32<KG, TIn, false>), sgrid, dim3(256), lds, st, in, F,
                           out, A, L, B, K);
    } else if (NT && line_runs) {
      hipLaunchKernelGGL((ttm_wide_f32<KG, TIn, true>), grid, dim3(256), lds, st, in, F, out, C,
                         L, B, K);
    } else {
      hipLaunchKernelGGL((ttm_wide_f32<KG, TIn, false>), grid, dim3(256), lds, st, in, F, out, C,
                         L, B, K);
    }
  } else if (path == Path::kWideScalar) {
    // runs of B % 4 != 0 elements are never whole 128-byte lines: consecutive
    // rows share their boundary lines, so the loads stay normal (cached)
    const int64_t C = A * B;
    dim3 grid((unsigned)((C + 1023) / 1024), (unsigned)chunks);
    hipLaunchKernelGGL((ttm_wide_scalar_f32<KG, TIn, false>), grid, dim3(256),
                       (size_t)16 * L * KG, st, in, F, out, C, L, B, K);
  } else if (path == Path::kWideSplitL) {
    if (KG > kSplitLMaxKG || splitl_lds(L, KG) > (size_t)kLdsBudget) return hipErrorInvalidValue;
    const int64_t C = A * B;
    dim3 grid((unsigned)((C + 255) / 256), (unsigned)chunks);
    if (NT && (B * sizeof(TIn)) % 128 == 0)
      hipLaunchKernelGGL((ttm_wide_splitl_f32<KG, TIn, true>), grid, dim3(256),
                         splitl_lds(L, KG), st, in, F, out, C, L, B, K);
    else
      hipLaunchKernelGGL((ttm_wide_splitl_f32<KG, TIn, false>), grid, dim3(256),
                         splitl_lds(L, KG), st, in, F, out, C, L, B, K);
  } else if (path == Path::kRows) {
    dim3 grid((unsigned)((A + 255) / 256), (unsigned)chunks);
    const size_t staged = (size_t)16 * L * KG + kRowStageBytes;
    // rows that are not whole 128-byte lines share a line with the next
    // column chunk: normal loads keep it cached until then
    const bool nt = NT && (L * sizeof(TIn)) % 128 == 0;
    if (!rows_v4(in, L)) {
      if (staged > (size_t)kLdsBudget) return hipErrorInvalidValue;  // launch_f32 prevents it
      if (nt)
        hipLaunchKernelGGL((ttm_rows_f32<KG, TIn, true, false>), grid, dim3(256), staged, st, in,
                           F, out, A, L, K);
      else
        hipLaunchKernelGGL((ttm_rows_f32<KG, TIn, false, false>), grid, dim3(256), staged, st, in,
                           F, out, A, L, K);
    } else if (staged <= (size_t)kLdsBudget) {
      if (nt)
        hipLaunchKernelGGL((ttm_rows_f32<KG, TIn, true, true>), grid, dim3(256), staged, st, in,
                           F, out, A, L, K);
      else
        hipLaunchKernelGGL((ttm_rows_f32<KG, TIn, false, true>), grid, dim3(256), staged, st, in,
                           F, out, A, L, K);
    } else {  // the factor slice leaves no room for the row tiles
      const size_t lds = (size_t)16 * L * KG;
      hipLaunchKernelGGL((ttm_rows_direct_f32<KG, TIn, NT>), grid, dim3(256), lds, st, in, F,
                         out, A, L, K);
    }
  } else {
    const int nb = (int)std::min<int64_t>(B, 256);
    const int na = 256 / nb;
    const int64_t nbt = (B + nb - 1) / nb;
    const int64_t nat = (A + na - 1) / na;
    const size_t lds = (size_t)16 * L * KG + (size_t)4 * kTileLC * 256;
    dim3 grid((unsigned)(nat * nbt), (unsigned)chunks);
    hipLaunchKernelGGL((ttm_tile_f32<KG, TIn>), grid, dim3(256), lds, st, in, F, out, A, L, B,
                       K, na, nb, nbt);
  }
  return hipGetLastError();
}

template <typename TIn, bool NT>
hipError_t launch_f32_nt(Path path, int kg, const TIn* in, int64_t A, int L, int64_t B,
                         const float* F, int K, float* out, hipStream_t st) {
  switch (kg) {
    case 1: return launch_f32_kg<TIn, 1, NT>(path, in, A, L, B, F, K, out, st);
    case 2: return launch_f32_kg<TIn, 2, NT>(path, in, A, L, B, F, K, out, st);
    case 3: return launch_f32_kg<TIn, 3, NT>(path, in, A, L, B, F, K, out, st);
    case 4: return launch_f32_kg<TIn, 4, NT>(path, in, A, L, B, F, K, out, st);
    case 5: return launch_f32_kg<TIn, 5, NT>(path, in, A, L, B, F, K, out, st);
    case 6: return launch_f32_kg<TIn, 6, NT>(path, in, A, L, B, F, K, out, st);
    case 8: return launch_f32_kg<TIn, 8, NT>(path, in, A, L, B, F, K, out, st);
    case 12: return launch_f32_kg<TIn, 12, NT>(path, in, A, L, B, F, K, out, st);
    default: return launch_f32_kg<TIn, 16, NT>(path, in, A, L, B, F, K, out, st);
  }
}

// Tile override: TK_TILE_SPLITK halves the K-group instance (twice the
// K-chunks, so more blocks that re-read the input from cache).
int split_kg(int kg) {
  int pick = 1;
  for (int c : kInst)
    if (c <= std::max(1, kg / 2)) pick = c;
  return pick;
}

template <typename TIn, int KG, bool SCALAR>
hipError_t launch_lk_kg(const TIn* in, int64_t A, int L, int64_t B, const float* F, int K,
                        float* out, hipStream_t st) {
  const int64_t C = A * B;
  const int chunks = (K + 4 * KG - 1) / (4 * KG);
  const int64_t nwork = ((C + 1023) / 1024) * chunks;
  const int64_t per_xcd = (nwork + 7) / 8;
  if (8 * per_xcd > (int64_t)INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL((ttm_lk_f32<KG, TIn, SCALAR>), dim3((unsigned)(8 * per_xcd)), dim3(256),
                     (size_t)16 * kLkRows * KG, st, in, F, out, C, L, B, K, chunks, nwork,
                     per_xcd);
  return hipGetLastError();
}

// Large-rank launch: the 16-byte body takes chunks of up to 12 K-groups (48
// factor columns, accumulators in 248 VGPRs, two waves per SIMD), 8 groups
// when that gives the same number of chunks; the 4-byte body keeps four
// pointers and takes 8 groups (at 12 it would hold one wave per SIMD).
template <typename TIn>
hipError_t launch_lk(bool wide, const TIn* in, int64_t A, int L, int64_t B, const float* F, int K,
                     float* out, hipStream_t st) {
  const int need = (K + 3) / 4;
  if (!wide) return launch_lk_kg<TIn, 8, true>(in, A, L, B, F, K, out, st);
  const int chunks = (need + 11) / 12;
  if (8 * chunks >= need) return launch_lk_kg<TIn, 8, false>(in, A, L, B, F, K, out, st);
  return launch_lk_kg<TIn, 12, false>(in, A, L, B, F, K, out, st);
}

// ---------------------------------------------------------- short-slab path --
// Nodes whose slabs In[a, :, :] are short (L <= 32, and B = 1 or B < 32 and
// not a wide-path B; the real tensors' small trailing modes): a wave owns
// G = 64 / B whole consecutive slabs, so its input (G L B elements) and its
// output (G K B) are each one contiguous range.  The wave reads its input
// range with consecutive loads (64 lanes, contiguous bytes per instruction)
// into its own LDS area, runs the MFMA chain with one column (a, b) per lane
// (the wide body's pattern), writes the outputs into the same LDS area in
// their memory order and stores the range with consecutive stores.  The row
// and tile bodies read 32-column chunks per row and store K scattered
// elements per row, which leaves most lanes idle on rows of 4 to 16
// elements.
constexpr int kShortMaxL = 32;
constexpr int kShortMaxKG = 8;
constexpr int kShortLoads = 32;  // 64 L / 64 element loads per lane at most

// q = e / d for 0 <= e < 2^22, d >= 1, inv = 1.0f / d (the float quotient is
// off by at most one and is corrected).
__device__ __forceinline__ int short_div(int e, int d, float inv) {
  int q = (int)((float)e * inv);
  const int r = e - q * d;
  if (r < 0)
    --q;
  else if (r >= d)
    ++q;
  return q;
}

template <int KG, typename TIn, bool NT, bool PAD>
__global__ __launch_bounds__(256) void ttm_short_f32(const TIn* __restrict__ in,
                                                     const float* __restrict__ F,
                                                     float* __restrict__ out, int64_t A, int L,
                                                     int B, int Kt, int G, int wbuf) {
  extern __shared__ float smem[];
  float* ft_all = smem;  // FT[r][l][g], 4 L KG
  stage_factor<KG>(ft_all, F, L, Kt, 0);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float* buf = smem + 4 * L * KG + wave * wbuf;  // this wave's area
  const int64_t a0 = ((int64_t)blockIdx.x * 4 + wave) * G;
  if (a0 >= A) return;  // whole wave idle
  // a slab length that is a multiple of 16 puts the lanes reading one row l
  // of their columns (or writing one output k) on at most 4 banks: such
  // slabs sit in LDS at pitch + 1 (PAD variant).  Shorter power-of-two
  // factors conflict less than the index division costs, so the variant
  // without padding keeps both packed.
  const int LB = L * B, KB = Kt * B;
  const int P = PAD && LB % 16 == 0 ? LB + 1 : LB;
  const int Q = PAD && KB % 16 == 0 ? KB + 1 : KB;
  const float inv_lb = 1.0f / (float)LB, inv_kb = 1.0f / (float)KB;
  const int ga = (int)min<int64_t>(G, A - a0);
  const int n_in = ga * LB;  // <= 64 L
  const TIn* src = in + a0 * LB;
  float v[kShortLoads];
#pragma unroll
  for (int u = 0; u < kShortLoads; ++u) {
    const int i = u * 64 + lane;
    if (i < n_in) {
      if constexpr (NT)
        v[u] = Elem<TIn>::to_f32(__builtin_nontemporal_load(src + i));
      else
        v[u] = Elem<TIn>::to_f32(src[i]);
    }
  }
#pragma unroll
  for (int u = 0; u < kShortLoads; ++u) {
    const int i = u * 64 + lane;
    if (i < n_in) {
      if constexpr (PAD)
        buf[i + short_div(i, LB, inv_lb) * (P - LB)] = v[u];
      else
        buf[i] = v[u];
    }
  }
  wave_lds_fence();
  // lane = column c = s B + b of slab a0 + s (lanes past G B read column 0
  // and store nothing)
  const bool act = lane < ga * B;
  const int sl = act ? lane / B : 0, b = act ? lane - sl * B : 0;
  const float* xcol = buf + sl * P + b;
  const float* ft = ft_all + (lane & 3) * L * KG;
  f4 acc[KG];
#pragma unroll
  for (int g = 0; g < KG; ++g) acc[g] = f4{0.f, 0.f, 0.f, 0.f};
  for (int l = 0; l < L; ++l) {
    const float x = xcol[l * B];
#pragma unroll
    for (int g = 0; g < KG; ++g) acc[g] = mfma4x4x1(ft[l * KG + g], x, acc[g]);
  }
  wave_lds_fence();  // every lane's reads are issued before the area is rewritten
  if (act) {
#pragma unroll
    for (int g = 0; g < KG; ++g)
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int k = 4 * g + m;
        if (k < Kt) buf[sl * Q + k * B + b] = acc[g][m];
      }
  }
  wave_lds_fence();
  const int n_out = ga * KB;  // <= 64 Kt
  float* dst = out + a0 * KB;
  for (int i = lane; i < n_out; i += 64) {
    if constexpr (PAD)
      dst[i] = buf[i + short_div(i, KB, inv_kb) * (Q - KB)];
    else
      dst[i] = buf[i];
  }
}

// Short-slab path: L <= 32, K <= 32, B = 1 or a B the row and tile bodies
// would take (below 32).
bool short_applies(int64_t L, int64_t B, int64_t K) {
  return L >= 1 && L <= kShortMaxL && K >= 1 && K <= 4 * kShortMaxKG && B >= 1 && B < 32;
}

template <typename TIn, int KG>
hipError_t launch_short_kg(const TIn* in, int64_t A, int L, int B, const float* F, int K,
                           float* out, hipStream_t st) {
  const int G = 64 / B;
  const int wbuf = G * (B * std::max(L, K) + 1);  // slabs at pitch + 1 at most
  const size_t lds = sizeof(float) * ((size_t)4 * L * KG + (size_t)4 * wbuf);
  const int64_t groups = (A + G - 1) / G;
  const int64_t blocks = (groups + 3) / 4;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  // streaming loads only where each wave's input range is whole 128-byte lines
  const bool nt = (uintptr_t)in % 128 == 0 && ((int64_t)G * L * B * sizeof(TIn)) % 128 == 0;
  const bool pad = (L * B) % 16 == 0 || (K * B) % 16 == 0;
#define TK_SHORT(NT_, PAD_)                                                                 \
  hipLaunchKernelGGL((ttm_short_f32<KG, TIn, NT_, PAD_>), dim3((unsigned)blocks), dim3(256), \
                     lds, st, in, F, out, A, L, B, K, G, wbuf)
  if (nt) {
    if (pad)
      TK_SHORT(true, true);
    else
      TK_SHORT(true, false);
  } else {
    if (pad)
      TK_SHORT(false, true);
    else
      TK_SHORT(false, false);
  }
#undef TK_SHORT
  return hipGetLastError();
}

template <typename TIn>
hipError_t launch_short(const TIn* in, int64_t A, int L, int B, const float* F, int K, float* out,
                        hipStream_t st) {
  switch ((K + 3) / 4) {
    case 1: return launch_short_kg<TIn, 1>(in, A, L, B, F, K, out, st);
    case 2: return launch_short_kg<TIn, 2>(in, A, L, B, F, K, out, st);
    case 3: return launch_short_kg<TIn, 3>(in, A, L, B, F, K, out, st);
    case 4: return launch_short_kg<TIn, 4>(in, A, L, B, F, K, out, st);
    case 5:
    case 6: return launch_short_kg<TIn, 6>(in, A, L, B, F, K, out, st);
    default: return launch_short_kg<TIn, 8>(in, A, L, B, F, K, out, st);
  }
}

template <typename TIn>
hipError_t launch_f32(const TIn* in, int64_t A, int L, int64_t B, const float* F, int K,
                      float* out, bool stream_in, int tile, hipStream_t st) {
  // LDS holds 16 * L * KG bytes of factor (+32 KB of tile for the tile path).
  Path path = tile == TK_TILE_STAGED ? Path::kTile : choose_path(in, out, B);
  // short slabs: the short-slab body, except rows of 16 or more elements read
  // 16 bytes at a time with K <= L / 2, where the row body measured faster
  // (L = 16 and 32 with K = 4 or 8: 10-15%)
  if (tile == TK_TILE_AUTO && (path == Path::kRows || path == Path::kTile) &&
      short_applies(L, B, K) &&
      !(path == Path::kRows && rows_v4(in, L) && L >= 16 && 2 * K <= L))
    return launch_short<TIn>(in, A, L, (int)B, F, K, out, st);
  // LDS beside the factor slice: the staged tile, or the row tiles when one
  // K-group fits beside them (else 16-byte rows are read directly, and
  // single-element rows take the tile path)
  const bool row_stage = (size_t)16 * L + kRowStageBytes <= (size_t)kLdsBudget;
  if (path == Path::kRows && !rows_v4(in, L) && !row_stage) path = Path::kTile;
  const int stage = (path == Path::kRows && row_stage) ? (int)kRowStageBytes
                    : path == Path::kTile              ? 4 * kTileLC * 256
                                                       : 0;
  int kg_cap = std::max(1, (kLdsBudget - std::max(stage, 4 * kTileLC * 256)) / (16 * L));
  // a wide grid that leaves CUs idle splits L over the waves of a block
  // (when at least one K-group of the factor slice fits beside the partials)
  if (path == Path::kWide && tile == TK_TILE_AUTO && grid_blocks(path, A, B) < 256 &&
      splitl_lds(L, 1) <= (size_t)kLdsBudget) {
    path = Path::kWideSplitL;
    kg_cap = std::max(1, std::min(kSplitLMaxKG, kLdsBudget / (16 * L)));
  }
  int kg = pick_kg(K, kg_cap, grid_blocks(path, A, B));
  // ranks of 32 and more that would need several K-chunks of the capped
  // instance: the large-rank kernel (any B except rows, which keep theirs)
  if (tile == TK_TILE_AUTO && K >= 32 && (K + 3) / 4 > kg &&
      (path == Path::kWide || path == Path::kWideScalar || path == Path::kTile))
    return launch_lk<TIn>(path == Path::kWide, in, A, L, B, F, K, out, st);
  if (tile == TK_TILE_SPLITK) kg = split_kg(kg);
  if (stream_in)
    return launch_f32_nt<TIn, true>(path, kg, in, A, L, B, F, K, out, st);
  return launch_f32_nt<TIn, false>(path, kg, in, A, L, B, F, K, out, st);
}

// 16 groups x 4 columns of accumulators exceed the register file of the BF16
// wide kernel (it spills); wider K is covered by more chunks.
constexpr int kWideBf16MaxKG = 12;

template <typename TIn, int KG, bool NT, bool X3, bool OutBF16, bool F3 = false>
hipError_t launch_bf16_kg(Path path, const TIn* in, int64_t A, int L, int64_t B, const float* F,
                          int K, void* out, hipStream_t st) {
  const int chunks = (K + 4 * KG - 1) / (4 * KG);
  const size_t lds = (size_t)32 * ((L + 3) / 4) * KG * (F3 ? 3 : X3 ? 2 : 1);
  if (path == Path::kWide) {
    if constexpr (KG <= kWideBf16MaxKG) {
      const int64_t C = A * B;
      dim3 grid((unsigned)((C + 1023) / 1024), (unsigned)chunks);
      hipLaunchKernelGGL((ttm_wide_bf16<KG, TIn, NT, X3, OutBF16, F3>), grid, dim3(256), lds, st,
                         in, F, out, C, L, B, K);
    } else {
      return hipErrorInvalidValue;  // not reached: launch_bf16 caps the wide KG
    }
  } else {
    if constexpr (F3) return hipErrorInvalidValue;  // the exact split runs the wide kernel only
    dim3 grid((unsigned)((A + 255) / 256), (unsigned)chunks);
    hipLaunchKernelGGL((ttm_rows_bf16<KG, TIn, NT, X3, OutBF16>), grid, dim3(256), lds, st, in, F,
                       out, A, L, K);
  }
  return hipGetLastError();
}

template <typename TIn, bool NT, bool X3, bool OutBF16, bool F3 = false>
hipError_t launch_bf16_nt(Path path, int kg, const TIn* in, int64_t A, int L, int64_t B,
                          const float* F, int K, void* out, hipStream_t st) {
#define TK_BF16_KG(G) \
  return launch_bf16_kg<TIn, G, NT, X3, OutBF16, F3>(path, in, A, L, B, F, K, out, st)
  switch (kg) {
    case 1: TK_BF16_KG(1);
    case 2: TK_BF16_KG(2);
    case 3: TK_BF16_KG(3);
    case 4: TK_BF16_KG(4);
    case 5: TK_BF16_KG(5);
    case 6: TK_BF16_KG(6);
    case 8: TK_BF16_KG(8);
    case 12: TK_BF16_KG(12);
    default: TK_BF16_KG(16);
  }
#undef TK_BF16_KG
}

// BF16 / split-BF16 compute.  Nodes that need the tile path (B not a multiple
// of four, or B == 1 with L not a multiple of four) run the FP32 tile kernel:
// at least as accurate as the mode asks for.
// True when a TK_C_BF16 node with these operands runs a BF16 kernel (wide or
// row), which can also write its output in BF16.
// Wide grids too small to fill the chip run the FP32 split-L kernel instead
// (it reads the input once; the BF16 kernel would re-read it per K-chunk).
template <typename TIn>
bool bf16_kernel_applies(const TIn* in, const void* out, int64_t A, int64_t L, int64_t B,
                         int tile) {
  if (tile == TK_TILE_STAGED) return false;
  const Path path = choose_path(in, (const float*)out, B);
  const bool rows_ok = L % 4 == 0 && (uintptr_t)in % (4 * sizeof(TIn)) == 0;
  const bool small_wide = grid_blocks(Path::kWide, A, B) < 256 && splitl_lds(L, 1) <=
                          (size_t)kLdsBudget;
  return (path == Path::kWide && (tile != TK_TILE_AUTO || !small_wide)) ||
         (path == Path::kRows && rows_ok);
}

template <typename TIn>
hipError_t launch_bf16(const TIn* in, int64_t A, int L, int64_t B, const float* F, int K,
                       void* out, bool stream_in, bool x3, bool out_bf16, int tile,
                       hipStream_t st, bool f3 = false) {
  const Path path = tile == TK_TILE_STAGED ? Path::kTile : choose_path(in, (float*)out, B);
  // the BF16 row kernel reads four consecutive l per lane: L % 4 == 0, aligned
  if (!bf16_kernel_applies(in, out, A, L, B, tile)) {
    if (out_bf16) return hipErrorInvalidValue;  // callers ask for BF16 output only here
    return launch_f32<TIn>(in, A, L, B, F, K, (float*)out, stream_in, tile, st);
  }
  if (out_bf16 && x3) return hipErrorInvalidValue;
  const int per_group = 32 * ((L + 3) / 4) * (f3 ? 3 : x3 ? 2 : 1);  // LDS bytes per K-group
  int kg_cap = std::max(1, kLdsBudget / per_group);
  if (path == Path::kWide) kg_cap = std::min(kg_cap, kWideBf16MaxKG);
  int kg = pick_kg(K, kg_cap, grid_blocks(path, A, B));
  if (tile == TK_TILE_SPLITK) kg = split_kg(kg);
  // a run (B columns, or a row of L) that is not a whole number of 128-byte
  // lines shares its boundary lines with a neighbouring wave: normal loads
  if ((path == Path::kWide ? B : (int64_t)L) * (int64_t)sizeof(TIn) % 128 != 0) stream_in = false;
  if (f3) {
    // exact three-term factor split on BF16 input (wide path only)
    if constexpr (std::is_same<TIn, uint16_t>::value) {
      if (path != Path::kWide || out_bf16) return hipErrorInvalidValue;
      if (stream_in)
        return launch_bf16_nt<TIn, true, true, false, true>(path, kg, in, A, L, B, F, K, out, st);
      return launch_bf16_nt<TIn, false, true, false, true>(path, kg, in, A, L, B, F, K, out, st);
    } else {
      return hipErrorInvalidValue;
    }
  }
  if (stream_in) {
    if (x3) return launch_bf16_nt<TIn, true, true, false>(path, kg, in, A, L, B, F, K, out, st);
    if (out_bf16)
      return launch_bf16_nt<TIn, true, false, true>(path, kg, in, A, L, B, F, K, out, st);
    return launch_bf16_nt<TIn, true, false, false>(path, kg, in, A, L, B, F, K, out, st);
  }
  if (x3) return launch_bf16_nt<TIn, false, true, false>(path, kg, in, A, L, B, F, K, out, st);
  if (out_bf16)
    return launch_bf16_nt<TIn, false, false, true>(path, kg, in, A, L, B, F, K, out, st);
  return launch_bf16_nt<TIn, false, false, false>(path, kg, in, A, L, B, F, K, out, st);
}

template <int KC>
hipError_t launch_f64_kc(const double* in, int64_t A, int L, int64_t B, const double* F, int K,
                         double* out, hipStream_t st) {
  const int chunks = (K + KC - 1) / KC;
  const int nb = (int)std::min<int64_t>(B, 256);
  const int na = 256 / nb;
  const int64_t nbt = (B + nb - 1) / nb;
  const int64_t nat = (A + na - 1) / na;
  const size_t lds = (size_t)8 * L * KC + (size_t)8 * kF64LC * 256;
  dim3 grid((unsigned)(nat * nbt), (unsigned)chunks);
  hipLaunchKernelGGL((ttm_tile_f64<KC, double>), grid, dim3(256), lds, st, in, F, out, A, L, B,
                     K, na, nb, nbt);
  return hipGetLastError();
}

}  // namespace

// Longest rows the grouped kernel stages through LDS (factor slice of four
// K-groups plus the row tiles within the LDS budget).
constexpr int kGroupedRowStageMaxL = (int)((kLdsBudget - kRowStageBytes) / (16 * 4));
int ttm_grouped_row_stage_max_L() { return kGroupedRowStageMaxL; }

void ttm_grouped_geometry(const void* in, const float* out, int in_bytes, int64_t A, int64_t L,
                          int64_t B, TtmNodeDesc* d, int64_t* tiles) {
  const bool in_al = (uintptr_t)in % (4 * (uintptr_t)in_bytes) == 0;
  d->nb = (int)std::min<int64_t>(B, 256);
  d->na = 256 / d->nb;
  d->nbt = (B + d->nb - 1) / d->nb;
  if (B % 4 == 0 && B >= 16 && in_al && (uintptr_t)out % 16 == 0) {
    d->path = kGroupedWide;  // 1024 columns per item
    *tiles = (A * B + 1023) / 1024;
  } else if (B == 1 && ((L % 4 == 0 && in_al) || L <= kGroupedRowStageMaxL)) {
    // 256 rows per item: through LDS (16-byte or single loads) or direct
    if (L > kGroupedRowStageMaxL)
      d->path = kGroupedRowsDirect;
    else
      d->path = L % 4 == 0 && in_al ? kGroupedRows : kGroupedRowsScalar;
    *tiles = (A + 255) / 256;
  } else if (B >= kWideScalarMinB) {
    d->path = kGroupedWideScalar;  // 1024 columns per item, 4-byte loads
    *tiles = (A * B + 1023) / 1024;
  } else {
    d->path = kGroupedTile;
    *tiles = ((A + d->na - 1) / d->na) * d->nbt;
  }
  const int64_t run = (d->path == kGroupedRows || d->path == kGroupedRowsDirect ||
                       d->path == kGroupedRowsScalar)
                          ? L
                          : B;
  d->lines = (d->path != kGroupedTile && (run * in_bytes) % 128 == 0 &&
              (uintptr_t)in % 128 == 0)
                 ? 1
                 : 0;
}

size_t ttm_grouped_lds(int Lmax) {
  const size_t factor = (size_t)16 * Lmax * 4;
  const size_t rows = (size_t)16 * std::min(Lmax, kGroupedRowStageMaxL) * 4 + kRowStageBytes;
  return std::max(factor + (size_t)4 * kTileLC * 256, rows);
}

hipError_t launch_ttm_grouped(int in_dtype, const TtmNodeDesc* nodes, const int2* items,
                              int n_items, int* counter, int Lmax, int grid, bool stream_in,
                              hipStream_t st) {
  if (n_items == 0) return hipSuccess;
  const size_t lds = ttm_grouped_lds(Lmax);
  if (lds > (size_t)kLdsBudget) return hipErrorInvalidValue;
  grid = std::max(1, std::min(grid, n_items));
#define TK_GROUPED(T, NT_)                                                                \
  hipLaunchKernelGGL((ttm_grouped<T, NT_>), dim3(grid), dim3(256), lds, st, nodes, items, \
                     n_items, counter)
  if (in_dtype == TK_F32) {
    if (stream_in)
      TK_GROUPED(float, true);
    else
      TK_GROUPED(float, false);
  } else {
    if (stream_in)
      TK_GROUPED(uint16_t, true);
    else
      TK_GROUPED(uint16_t, false);
  }
#undef TK_GROUPED
  return hipGetLastError();
}

size_t ttm_grouped_rows_lds(int Lmax) { return (size_t)16 * Lmax * 4 + kRowStageBytes; }

hipError_t launch_ttm_grouped_rows(int in_dtype, const TtmNodeDesc* nodes, const int2* items,
                                   int n_items, int* counter, int Lmax, int grid, bool stream_in,
                                   hipStream_t st) {
  if (n_items == 0) return hipSuccess;
  const size_t lds = ttm_grouped_rows_lds(Lmax);
  if (lds > (size_t)kLdsBudget) return hipErrorInvalidValue;
  grid = std::max(1, std::min(grid, n_items));
  // odd-length rows never end on a 128-byte line: consecutive rows share their
  // boundary lines, so the loads stay normal (cached) even for an input read
  // once, which non-temporal loads would fetch twice
  (void)stream_in;
  if (in_dtype == TK_F32)
    hipLaunchKernelGGL((ttm_grouped_rows<float, false>), dim3(grid), dim3(256), lds, st, nodes,
                       items, n_items, counter);
  else
    hipLaunchKernelGGL((ttm_grouped_rows<uint16_t, false>), dim3(grid), dim3(256), lds, st,
                       nodes, items, n_items, counter);
  return hipGetLastError();
}

// Largest L the TTM kernels accept (factor slice of at least one K-group in LDS).
int ttm_max_L() { return (kLdsBudget - 4 * kTileLC * 256) / 16; }

bool ttm_bf16_output_ok(int in_dtype, int compute, const void* in, int64_t A, int64_t L,
                        int64_t B, const void* out, int tile) {
  if (compute != TK_C_BF16) return false;
  if (in_dtype == TK_F32) return bf16_kernel_applies((const float*)in, out, A, L, B, tile);
  if (in_dtype == TK_BF16) return bf16_kernel_applies((const uint16_t*)in, out, A, L, B, tile);
  return false;
}

hipError_t launch_ttm(int in_dtype, int compute, const void* in, int64_t A, int64_t L, int64_t B,
                      const void* F, int64_t K, void* out, hipStream_t st, bool stream_in,
                      int tile, int out_dtype) {
  if (out_dtype == TK_BF16 && !ttm_bf16_output_ok(in_dtype, compute, in, A, L, B, out, tile))
    return hipErrorInvalidValue;
  if (A * B == 0 || K == 0) return hipSuccess;
  if (compute == TK_C_FP64) {
    const int Li = (int)L;
    const int kc_cap = std::max(1, (kLdsBudget - 8 * kF64LC * 256) / (8 * Li));
    if (K <= 8 || kc_cap < 16)
      return launch_f64_kc<8>((const double*)in, A, Li, B, (const double*)F, (int)K,
                              (double*)out, st);
    if (K <= 16 || kc_cap < 32)
      return launch_f64_kc<16>((const double*)in, A, Li, B, (const double*)F, (int)K,
                               (double*)out, st);
    return launch_f64_kc<32>((const double*)in, A, Li, B, (const double*)F, (int)K,
                             (double*)out, st);
  }
  if (compute == TK_C_BF16 || compute == TK_C_BF16X3) {
    if (in_dtype == TK_F16) return hipErrorInvalidValue;  // FP16 storage: FP32 compute only
    const bool x3 = compute == TK_C_BF16X3;
    const bool ob = out_dtype == TK_BF16;
    if (in_dtype == TK_F32)
      return launch_bf16<float>((const float*)in, A, (int)L, B, (const float*)F, (int)K, out,
                                stream_in, x3, ob, tile, st);
    return launch_bf16<uint16_t>((const uint16_t*)in, A, (int)L, B, (const float*)F, (int)K, out,
                                 stream_in, x3, ob, tile, st);
  }
  if (in_dtype == TK_F32)
    return launch_f32<float>((const float*)in, A, (int)L, B, (const float*)F, (int)K,
                             (float*)out, stream_in, tile, st);
  // FP32 compute on FP16 input: the FP32 kernels, converting on load
  if (in_dtype == TK_F16)
    return launch_f32<_Float16>((const _Float16*)in, A, (int)L, B, (const float*)F, (int)K,
                                (float*)out, stream_in, tile, st);
  // FP32 compute on BF16 input: on wide grids that fill the chip, BF16 MFMAs
  // with the factor split exactly into three bfloat16 terms (the products of
  // bfloat16 pairs are exact in FP32, so this matches an FP32 MFMA chain up
  // to the order of the FP32 accumulation); otherwise the FP32 kernels
  const uint16_t* in16 = (const uint16_t*)in;
  if (tile == TK_TILE_AUTO && choose_path(in16, (const float*)out, B) == Path::kWide &&
      grid_blocks(Path::kWide, A, B) >= 256)
    return launch_bf16<uint16_t>(in16, A, (int)L, B, (const float*)F, (int)K, out, stream_in,
                                 true, false, tile, st, true);
  return launch_f32<uint16_t>(in16, A, (int)L, B, (const float*)F, (int)K, (float*)out,
                              stream_in, tile, st);
}

}  // namespace tk
