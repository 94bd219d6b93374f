// Both root TTMs of a TTM-tree in one pass over T.
//
// A node's output is computed once and reused by every child (Sec. 3.1); at
// the root the "output" is T itself, and each root child reads all of it.
// When the root has two children, along modes p < q, one kernel can stream T
// once and form both outputs.  With T seen row-major as [A, Lp, M, Lq, B]
// (A, M, B: products of the lengths before p, between p and q, after q):
//
//   Outp[a, kp, m, lq, b] = sum_lp Fp[lp, kp] T[a, lp, m, lq, b]   ([A, Kp, M, Lq, B])
//   Outq[a, lp, m, kq, b] = sum_lq Fq[lq, kq] T[a, lp, m, lq, b]   ([A, Lp, M, Kq, B])
//
// A block owns one tile (a, m, four consecutive b) and walks lp.  Lane
// (beta, i) of wave w holds rows lq = 64 w + 4 beta + j (j = 0..3) at column
// b = i, i.e. a 4 x 4 patch per group of four lanes, so both products run on
// v_mfma_f32_4x4x1_16b_f32 from the same registers:
//   * Outp: the group's outer products F[lp, 4g + r] x T[.., lq, b] accumulate
//     over lp in registers (four k's of four rows per lane, K <= 20);
//   * Outq: the outer products Fq[lq, 4g + r] x T[.., lq, b] summed over the
//     group's four rows give per-group partial sums, which the block adds
//     over its 64 groups through LDS in a fixed order (deterministic) and
//     writes once per lp.
// Tiles are mapped XCD by XCD (block id modulo 8 picks the XCD, the quotient
// the slot), so the tiles that share T's cache lines (neighbouring b) run on
// one XCD at the same time and the lines are fetched from HBM once.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.h"
#include "internal.h"
#include "kernels.h"

namespace tk {

namespace {

constexpr int kPairThreads = 256;
constexpr int kPairRows = 256;   // Lq limit: one row group per lane quad
constexpr int kPairPre = 5;      // lp steps whose loads are in flight
// Partial sums in LDS, partial-major: partial p of output o at p * kRedPitch
// + o.  kRedPitch = 84 = 4 (mod 64): the 64 lanes of a store (16 groups x 4
// outputs) hit 64 different banks, and the readers (one thread per output)
// read consecutive words at every step.
constexpr int kRedPitch = 84;

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}

// Block barrier for LDS traffic only: this wave's LDS accesses complete
// (lgkmcnt(0)), then s_barrier.  Unlike __syncthreads() it does not wait for
// outstanding global loads, so the prefetched steps stay in flight across
// it.  The wavefront-scope fences emit no instruction; they keep the compiler
// from moving LDS accesses across the barrier.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_s_waitcnt(0xc07f);
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int KGP, int KGQ>
__global__ __launch_bounds__(kPairThreads, 2) void ttm_pair_f32(
    const float* __restrict__ in, int Lp, int64_t M, int Lq, int64_t B,
    const float* __restrict__ Fp, int Kp, const float* __restrict__ Fq, int Kq,
    float* __restrict__ outp, float* __restrict__ outq, int64_t ntiles, int64_t per_xcd) {
  extern __shared__ float lds[];
  float* FTp = lds;                            // [4][Lp][KGP]: Fp[lp, 4g + r]
  // [KGQ][4][Lqp]: Fq[lq, 4g + r], rows padded to Lqp = 1 (mod 4) so that
  // the 64 lanes of a read (16 row groups x 4 r) hit different banks
  const int Lqp = (Lq + 3) / 4 * 4 + 1;
  float* FTq = FTp + 4 * Lp * KGP;
  float* red = FTq + KGQ * 4 * Lqp;            // 2 x [64][kRedPitch]
  const int64_t t = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (t >= ntiles) return;  // the whole block
  const int tid = threadIdx.x;
  for (int e = tid; e < 4 * Lp * KGP; e += kPairThreads) {
    const int g = e % KGP, lp = (e / KGP) % Lp, r = e / (KGP * Lp);
    const int k = 4 * g + r;
    FTp[e] = k < Kp ? Fp[(int64_t)lp * Kp + k] : 0.f;
  }
  for (int e = tid; e < KGQ * 4 * Lqp; e += kPairThreads) {
    const int lq = e % Lqp, k = e / Lqp;
    FTq[e] = (k < Kq && lq < Lq) ? Fq[(int64_t)lq * Kq + k] : 0.f;
  }
  __syncthreads();

  const int64_t nbc = B / 4;
  const int64_t bc = t % nbc;
  const int64_t am = t / nbc;
  const int64_t m = am % M;
  const int64_t a = am / M;
  const int lane = tid & 63, wave = tid >> 6;
  const int beta = lane >> 2, i = lane & 3;
  const int row0 = wave * 64 + 4 * beta;
  const int64_t lpstride = M * Lq * B;
  // rows past Lq load row Lq - 1 (an address in bounds) and are zeroed, and
  // prefetches past the last lp load step Lp - 1: every load is unconditional,
  // so the loads of kPairPre steps stay in flight in program order
  bool ok[4];
  int frow[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    ok[j] = row0 + j < Lq;
    frow[j] = min(row0 + j, Lq - 1);
  }
  // block-uniform base of the tile and 32-bit per-lane offsets, so a load is
  // one scalar base plus one offset register
  const float* tile = in + ((a * Lp) * M + m) * (int64_t)Lq * B + 4 * bc;
  uint32_t off[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) off[j] = (uint32_t)(frow[j] * B + i);
  const float* ftp = FTp + i * Lp * KGP;

  f4 accp[KGP][4];
#pragma unroll
  for (int g = 0; g < KGP; ++g)
#pragma unroll
    for (int j = 0; j < 4; ++j) accp[g][j] = f4{0.f, 0.f, 0.f, 0.f};

  float y[kPairPre][4];
  auto load = [&](int s, int lp) {
    const float* p = tile + (int64_t)min(lp, Lp - 1) * lpstride;
#pragma unroll
    for (int j = 0; j < 4; ++j) y[s][j] = p[off[j]];
  };
  float* qout = outq + ((a * Lp) * M + m) * (int64_t)Kq * B + 4 * bc;
  // one lp step on the loads of slot s; then slot s fetches step lp + kPairPre
  auto step = [&](int s, int lp, bool prefetch) {
    float x[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = ok[j] ? y[s][j] : 0.f;
    if (prefetch) load(s, lp + kPairPre);
    // Outp: accumulate over lp
#pragma unroll
    for (int g = 0; g < KGP; ++g) {
      const float fa = ftp[lp * KGP + g];
#pragma unroll
      for (int j = 0; j < 4; ++j) accp[g][j] = mfma4(fa, x[j], accp[g][j]);
    }
    // Outq: this group's four rows
    f4 accq[KGQ];
#pragma unroll
    for (int g = 0; g < KGQ; ++g) accq[g] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float* fq = FTq + i * Lqp + frow[j];
#pragma unroll
      for (int g = 0; g < KGQ; ++g) accq[g] = mfma4(fq[4 * g * Lqp], x[j], accq[g]);
    }
    // partial sums of output (kq = 4 g + r, b = i) -> red[o][wave * 16 + beta];
    // the two buffers alternate, so a buffer is written again only after the
    // next step's barrier, when its readers are done
    float* rb = red + (lp & 1) * (64 * kRedPitch);
#pragma unroll
    for (int g = 0; g < KGQ; ++g)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        rb[(wave * 16 + beta) * kRedPitch + (4 * g + r) * 4 + i] = accq[g][r];
    lds_barrier();
    if (tid < 16 * KGQ) {
      const float* pr = rb + tid;
      float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
#pragma unroll
      for (int q = 0; q < 64; q += 4) {
        s0 += pr[q * kRedPitch];
        s1 += pr[(q + 1) * kRedPitch];
        s2 += pr[(q + 2) * kRedPitch];
        s3 += pr[(q + 3) * kRedPitch];
      }
      const int kq = tid >> 2, b = tid & 3;
      if (kq < Kq) qout[((int64_t)lp * M * Kq + kq) * B + b] = (s0 + s1) + (s2 + s3);
    }
    // keep the steps apart in the schedule (interleaving them only lengthens
    // register live ranges; the loads are already kPairPre steps ahead)
    __builtin_amdgcn_sched_barrier(0);
  };
#pragma unroll
  for (int s = 0; s < kPairPre; ++s) load(s, s);
  int lp0 = 0;
  for (; lp0 + kPairPre <= Lp; lp0 += kPairPre) {
#pragma unroll
    for (int s = 0; s < kPairPre; ++s) step(s, lp0 + s, true);
  }
#pragma unroll
  for (int s = 0; s < kPairPre; ++s)
    if (lp0 + s < Lp) step(s, lp0 + s, false);

  float* pout = outp + (a * Kp * M + m) * (int64_t)Lq * B + 4 * bc + i;
#pragma unroll
  for (int g = 0; g < KGP; ++g)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int kp = 4 * g + r;
      if (kp >= Kp) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (ok[j]) pout[((int64_t)kp * M * Lq + row0 + j) * B] = accp[g][j][r];
    }
}

// q = e / d and *rem = e % d for 0 <= e < 2^22, d >= 1, inv = 1.0f / d: the
// float quotient is off by at most one and is corrected.
__device__ __forceinline__ int small_divmod(int e, int d, float inv, int* rem) {
  int q = (int)((float)e * inv);
  int r = e - q * d;
  if (r < 0) {
    --q;
    r += d;
  } else if (r >= d) {
    ++q;
    r -= d;
  }
  *rem = r;
  return q;
}

// ---- the two trailing modes (M = 1, B = 1): slabs T[a] of Lp x Lq elements
// A block stages NA consecutive slabs (contiguous in T) in LDS with 16-byte
// loads, then forms both outputs from LDS on the VALU:
//   Outq[a, lp, kq] = sum_lq T[a, lp, lq] Fq[lq, kq]   (thread per row (a, lp))
//   Outp[a, kp, lq] = sum_lp Fp[lp, kp] T[a, lp, lq]   (thread per column (a, lq))
// Each element of T is read from HBM once and from LDS twice.  The rows of a
// slab sit at an odd LDS pitch, so row walks and column walks are both free
// of bank conflicts.  Kp, Kq <= 8 (the factors live in registers).
template <int KP, int KQ>
__global__ __launch_bounds__(kPairThreads) void ttm_pair_tail_f32(
    const float* __restrict__ in, int64_t A, int Lp, int Lq, const float* __restrict__ Fp,
    int Kp, const float* __restrict__ Fq, int Kq, float* __restrict__ outp,
    float* __restrict__ outq, int NA) {
  extern __shared__ float lds[];
  const int pitch = Lq | 1;
  const int slab = Lp * pitch;
  float* S = lds;                        // NA x Lp x pitch
  float* FpS = S + NA * slab;            // Lp x KP
  float* FqS = FpS + Lp * KP;            // Lq x KQ
  const int tid = threadIdx.x;
  for (int e = tid; e < Lp * KP; e += kPairThreads) {
    const int l = e / KP, k = e % KP;
    FpS[e] = k < Kp ? Fp[l * Kp + k] : 0.f;
  }
  for (int e = tid; e < Lq * KQ; e += kPairThreads) {
    const int l = e / KQ, k = e % KQ;
    FqS[e] = k < Kq ? Fq[l * Kq + k] : 0.f;
  }
  const int64_t a0 = (int64_t)blockIdx.x * NA;
  const int na = (int)min<int64_t>(NA, A - a0);
  const int per = Lp * Lq;
  const int n = na * per;  // at most 6144 + 2048 elements
  const float* src = in + a0 * per;
  const float inv_per = 1.0f / (float)per, inv_lq = 1.0f / (float)Lq;
  // 16-byte loads of the contiguous chunk (per % 4 == 0: every slab, hence
  // the chunk, starts on 16 bytes), scattered into the padded rows.  The
  // slab, row and column of an element come from one small-integer division
  // pair per four elements (float reciprocals, corrected to exact)
  for (int v = tid; v < n / 4; v += kPairThreads) {
    const f4 x = *reinterpret_cast<const f4*>(src + 4 * v);
    int r;
    const int as = small_divmod(4 * v, per, inv_per, &r);
    int col;
    int row = small_divmod(r, Lq, inv_lq, &col);
    float* srow = S + as * slab;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      srow[row * pitch + col] = x[c];
      if (++col == Lq) {  // a slab ends on a row end (per = Lp * Lq)
        col = 0;
        if (++row == Lp) {
          row = 0;
          srow += slab;
        }
      }
    }
  }
  __syncthreads();
  // rows (a, lp) -> Outq
  for (int row = tid; row < na * Lp; row += kPairThreads) {
    const int as = row / Lp, lp = row % Lp;
    const float* sr = S + as * slab + lp * pitch;
    float acc[KQ];
#pragma unroll
    for (int k = 0; k < KQ; ++k) acc[k] = 0.f;
    for (int lq = 0; lq < Lq; ++lq) {
      const float x = sr[lq];
#pragma unroll
      for (int k = 0; k < KQ; ++k) acc[k] = fmaf(x, FqS[lq * KQ + k], acc[k]);
    }
    float* q = outq + ((a0 + as) * Lp + lp) * (int64_t)Kq;
#pragma unroll
    for (int k = 0; k < KQ; ++k)
      if (k < Kq) q[k] = acc[k];
  }
  // columns (a, lq) -> Outp
  for (int col = tid; col < na * Lq; col += kPairThreads) {
    const int as = col / Lq, lq = col % Lq;
    const float* sc = S + as * slab + lq;
    float acc[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) acc[k] = 0.f;
    for (int lp = 0; lp < Lp; ++lp) {
      const float x = sc[lp * pitch];
#pragma unroll
      for (int k = 0; k < KP; ++k) acc[k] = fmaf(x, FpS[lp * KP + k], acc[k]);
    }
    float* o = outp + (a0 + as) * (int64_t)Kp * Lq + lq;
#pragma unroll
    for (int k = 0; k < KP; ++k)
      if (k < Kp) o[(int64_t)k * Lq] = acc[k];
  }
}

// ---- the two trailing modes, slabs too large for one block's LDS: T[a] of
// Lp x Lq elements (Lq % 4 == 0, Lq <= 256), ranks up to 20.  A block owns
// NA consecutive slabs and streams them through LDS in chunks of R rows
// (R a multiple of 4, R Lq <= 4096, R <= 16), the 16-byte loads of the next chunk in
// flight while the current one is used.  LDS rows have 256 columns (zeros
// past Lq, written once) at the odd pitch 257: column walks and row walks
// are both free of bank conflicts, and each wave's quarter of a row is a
// fixed 64 columns.
// From the same LDS rows both outputs run on v_mfma_f32_4x4x1_16b_f32:
//   * Outp[a, kp, lq]: lane lq = 64 w + i of wave w accumulates
//     Fp[lp, 4g + r] x T[a, lp, lq] over every row lp of the slab (the wide
//     body's pattern, one column per lane, KGP accumulators);
//   * Outq[a, lp, kq]: the 16 blocks of an MFMA are (rank group g, row quad
//     q) pairs of the chunk (KGQ groups x R / 4 quads); wave w sums over its
//     quarter of the columns lq, with the factor entries Fq[lq, 4g + r] it
//     needs held in registers for the whole block, and the four waves'
//     partial sums are added in wave order through LDS and stored once per
//     chunk (deterministic).
constexpr int kSlabMaxLq = 256;
constexpr int kSlabPitch = kSlabMaxLq + 1;
constexpr int kSlabJw = kSlabMaxLq / 4;  // columns per wave in the Outq sums
constexpr int kSlabChunk = 4096;         // elements of T per chunk
constexpr int kSlabMaxFp = 2560;         // Lp * KGP: the staged Fp within 40 KB

template <int KGP, int KGQ, bool NT>
__global__ __launch_bounds__(kPairThreads) void ttm_pair_slab_f32(
    const float* __restrict__ in, int64_t A, int Lp, int Lq, int R,
    const float* __restrict__ Fp, int Kp, const float* __restrict__ Fq, int Kq,
    float* __restrict__ outp, float* __restrict__ outq, int NA) {
  extern __shared__ float lds[];
  constexpr int pitch = kSlabPitch;
  float* S = lds;                   // R x pitch: the current chunk
  float* FpS = S + R * pitch;       // FT[r][lp][g] = Fp[lp, 4g + r]
  float* red = FpS + 4 * Lp * KGP;  // [wave][m][lane] partial sums of Outq
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < R * pitch; e += kPairThreads) S[e] = 0.f;  // padding stays zero
  for (int e = tid; e < 4 * Lp * KGP; e += kPairThreads) {
    const int g = e % KGP, t = e / KGP, l = t % Lp, r = t / Lp;
    const int k = 4 * g + r;
    FpS[e] = k < Kp ? Fp[(int64_t)l * Kp + k] : 0.f;
  }
  // Outq: block beta = lane / 4 is (group gq, row quad qq) when beta < KGQ Qn
  const int Qn = R / 4;
  const int beta = lane >> 2, kr = lane & 3;
  const bool qblk = beta < KGQ * Qn;
  const int gq = qblk ? beta / Qn : 0, qq = qblk ? beta % Qn : 0;
  const int kq = 4 * gq + kr;
  const int j0 = wave * kSlabJw;  // this wave's columns j0 .. j0 + 63 (zeros past Lq)
  float fq[kSlabJw];
#pragma unroll
  for (int t = 0; t < kSlabJw; ++t)
    fq[t] = (j0 + t < Lq && qblk && kq < Kq) ? Fq[(int64_t)(j0 + t) * Kq + kq] : 0.f;
  // Outp: this lane's column (lanes past Lq read the last column, store nothing)
  const int jp = wave * 64 + lane;
  const int jc = min(jp, Lq - 1);
  const float* ft = FpS + kr * Lp * KGP;
  const int nchunk = (Lp + R - 1) / R;
  const int64_t a0 = (int64_t)blockIdx.x * NA;
  const int na = (int)min<int64_t>(NA, A - a0);
  const int total = na * nchunk;
  const float inv_lq = 1.0f / (float)Lq;
  const int nv_full = R * Lq / 4;  // 16-byte vectors per full chunk (<= 1024)
  // f4 v = tid + 256 u (u < 4) of chunk s
  auto fetch = [&](int s, f4 (&pre)[4]) {
    const int as = s / nchunk, c = s - as * nchunk;
    const int rc = min(R, Lp - c * R);
    const float* src = in + ((a0 + as) * Lp + (int64_t)c * R) * Lq;
    const int nv = rc * Lq / 4;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int v = tid + kPairThreads * u;
      if (v < nv) {
        if constexpr (NT)
          pre[u] = __builtin_nontemporal_load(reinterpret_cast<const f4*>(src) + v);
        else
          pre[u] = reinterpret_cast<const f4*>(src)[v];
      } else {
        pre[u] = f4{0.f, 0.f, 0.f, 0.f};  // rows past Lp in the last chunk
      }
    }
  };
  f4 pre[4];
  if (total > 0) fetch(0, pre);
  f4 accp[KGP];
#pragma unroll
  for (int g = 0; g < KGP; ++g) accp[g] = f4{0.f, 0.f, 0.f, 0.f};
  __syncthreads();  // FpS staged
  for (int s = 0; s < total; ++s) {
    const int as = s / nchunk, c = s - as * nchunk;
    const int i0 = c * R, rc = min(R, Lp - i0);
    // the chunk into LDS (all R rows: zeros past Lp)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int v = tid + kPairThreads * u;
      if (v < nv_full) {
        int col;
        const int row = small_divmod(4 * v, Lq, inv_lq, &col);
        float* d = S + row * pitch + col;
        d[0] = pre[u][0];
        d[1] = pre[u][1];
        d[2] = pre[u][2];
        d[3] = pre[u][3];
      }
    }
    __syncthreads();
    if (s + 1 < total) fetch(s + 1, pre);
    // Outp: rows i0 .. i0 + rc - 1 of this slab
    for (int r = 0; r < rc; ++r) {
      const float x = S[r * pitch + jc];
      const float* f = ft + (i0 + r) * KGP;
#pragma unroll
      for (int g = 0; g < KGP; ++g) accp[g] = mfma4(f[g], x, accp[g]);
    }
    // Outq partial sums over this wave's 64 columns (two chains, even and
    // odd columns, so consecutive MFMAs do not wait on each other)
    f4 aq = f4{0.f, 0.f, 0.f, 0.f}, aq1 = f4{0.f, 0.f, 0.f, 0.f};
    const float* srow = S + (4 * qq + kr) * pitch + j0;
#pragma unroll
    for (int t = 0; t < kSlabJw; t += 2) {
      aq = mfma4(fq[t], srow[t], aq);
      aq1 = mfma4(fq[t + 1], srow[t + 1], aq1);
    }
    aq += aq1;
#pragma unroll
    for (int m = 0; m < 4; ++m) red[(wave * 4 + m) * 64 + lane] = aq[m];
    __syncthreads();
    {
      // thread (m, l): register m of lane l, summed over the waves in order
      const int m = tid >> 6, l = tid & 63;
      const float v = ((red[(0 * 4 + m) * 64 + l] + red[(1 * 4 + m) * 64 + l]) +
                       red[(2 * 4 + m) * 64 + l]) +
                      red[(3 * 4 + m) * 64 + l];
      const int b2 = l >> 2, n = l & 3;
      if (b2 < KGQ * Qn) {
        const int row = 4 * (b2 % Qn) + n, k = 4 * (b2 / Qn) + m;
        if (row < rc && k < Kq) outq[((a0 + as) * Lp + i0 + row) * Kq + k] = v;
      }
    }
    if (c == nchunk - 1) {
      // the slab is done: Outp[a, kp, lq]
      if (jp < Lq) {
        float* o = outp + (a0 + as) * (int64_t)Kp * Lq + jp;
#pragma unroll
        for (int g = 0; g < KGP; ++g)
#pragma unroll
          for (int m = 0; m < 4; ++m)
            if (4 * g + m < Kp) o[(int64_t)(4 * g + m) * Lq] = accp[g][m];
      }
#pragma unroll
      for (int g = 0; g < KGP; ++g) accp[g] = f4{0.f, 0.f, 0.f, 0.f};
    }
  }
}

// Rows per chunk: a multiple of 4 with KGQ (R / 4) <= 16 blocks per MFMA,
// R Lq <= 4096 elements, and R <= 16 (R x 257 floats of LDS beside a staged
// Fp of up to 40 KB).
int slab_rows(int Lq, int KGQ) {
  const int quads = std::min(std::min(16 / KGQ, kSlabChunk / (4 * Lq)), 4);
  return 4 * std::max(1, quads);
}

size_t slab_lds(int Lp, int KGP, int R) {
  return sizeof(float) * ((size_t)R * kSlabPitch + (size_t)4 * Lp * KGP + (size_t)4 * 4 * 64);
}

bool slab_applies(int64_t A, int64_t Lp, int64_t M, int64_t Lq, int64_t B, int64_t Kp,
                  int64_t Kq) {
  if (M != 1 || B != 1 || A < 1 || Lp < 1) return false;
  if (Lq < 4 || Lq > kSlabMaxLq || Lq % 4 != 0) return false;
  if (Kp < 1 || Kq < 1 || Kp > 20 || Kq > 20) return false;
  if (Lp * ((Kp + 3) / 4) > kSlabMaxFp) return false;
  return A * Lp * Lq < ((int64_t)1 << 40);
}

template <int KGP, int KGQ>
hipError_t launch_slab(const float* in, int64_t A, int Lp, int Lq, const float* Fp, int Kp,
                       const float* Fq, int Kq, float* outp, float* outq, hipStream_t st) {
  const int R = slab_rows(Lq, KGQ);
  const size_t lds = slab_lds(Lp, KGP, R);
  // a few slabs per block where there are many (the staging of the factors
  // is paid once per block), at least 8192 blocks otherwise
  const int NA = (int)std::max<int64_t>(1, std::min<int64_t>(4, A / 8192));
  const unsigned grid = (unsigned)((A + NA - 1) / NA);
  // streaming loads where every chunk and slab is whole 128-byte lines
  const bool nt = ((uintptr_t)in % 128 == 0) && ((int64_t)R * Lq * 4) % 128 == 0 &&
                  ((int64_t)Lp * Lq * 4) % 128 == 0;
  if (nt)
    hipLaunchKernelGGL((ttm_pair_slab_f32<KGP, KGQ, true>), dim3(grid), dim3(kPairThreads), lds,
                       st, in, A, Lp, Lq, R, Fp, Kp, Fq, Kq, outp, outq, NA);
  else
    hipLaunchKernelGGL((ttm_pair_slab_f32<KGP, KGQ, false>), dim3(grid), dim3(kPairThreads),
                       lds, st, in, A, Lp, Lq, R, Fp, Kp, Fq, Kq, outp, outq, NA);
  return hipGetLastError();
}

int tail_na(int Lp, int Lq) { return std::max(1, 6144 / (Lp * Lq)); }

size_t tail_lds(int Lp, int Lq, int NA) {
  return sizeof(float) * ((size_t)NA * Lp * (Lq | 1) + (size_t)Lp * 8 + (size_t)Lq * 8);
}

bool tail_applies(int64_t A, int64_t Lp, int64_t M, int64_t Lq, int64_t B, int64_t Kp,
                  int64_t Kq) {
  return M == 1 && B == 1 && Lp * Lq <= 2048 && (Lp * Lq) % 4 == 0 && Kp <= 8 && Kq <= 8 &&
         A >= 4096 && tail_lds((int)Lp, (int)Lq, tail_na((int)Lp, (int)Lq)) <= 64 * 1024;
}

template <int KP, int KQ>
hipError_t launch_tail(const float* in, int64_t A, int Lp, int Lq, const float* Fp, int Kp,
                       const float* Fq, int Kq, float* outp, float* outq, hipStream_t st) {
  const int NA = tail_na(Lp, Lq);
  const size_t lds = tail_lds(Lp, Lq, NA);
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)ttm_pair_tail_f32<KP, KQ>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL((ttm_pair_tail_f32<KP, KQ>), dim3((unsigned)((A + NA - 1) / NA)),
                     dim3(kPairThreads), lds, st, in, A, Lp, Lq, Fp, Kp, Fq, Kq, outp, outq, NA);
  return hipGetLastError();
}

size_t pair_lds(int Lp, int Lq, int KGP, int KGQ) {
  const size_t Lqp = (size_t)(Lq + 3) / 4 * 4 + 1;
  return sizeof(float) * ((size_t)4 * Lp * KGP + (size_t)KGQ * 4 * Lqp +
                          (size_t)2 * 64 * kRedPitch);
}

template <int KGP, int KGQ>
hipError_t launch_pair_kg(const float* in, int64_t A, int Lp, int64_t M, int Lq, int64_t B,
                          const float* Fp, int Kp, const float* Fq, int Kq, float* outp,
                          float* outq, hipStream_t st) {
  const size_t lds = pair_lds(Lp, Lq, KGP, KGQ);
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)ttm_pair_f32<KGP, KGQ>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 80 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int64_t ntiles = A * M * (B / 4);
  const int64_t per_xcd = (ntiles + 7) / 8;
  hipLaunchKernelGGL((ttm_pair_f32<KGP, KGQ>), dim3((unsigned)(8 * per_xcd)),
                     dim3(kPairThreads), lds, st, in, Lp, M, Lq, B, Fp, Kp, Fq, Kq, outp, outq,
                     ntiles, per_xcd);
  return hipGetLastError();
}

}  // namespace

int ttm_pair_kind(int in_dtype, int compute, const void* in, int64_t A, int64_t Lp, int64_t M,
                  int64_t Lq, int64_t B, int64_t Kp, int64_t Kq, const void* outp,
                  const void* outq) {
  if (in_dtype != TK_F32 || compute != TK_C_FP32) return 0;
  if (((uintptr_t)in | (uintptr_t)outp | (uintptr_t)outq) % 16 != 0) return 0;
  if (tail_applies(A, Lp, M, Lq, B, Kp, Kq)) return 2;
  if (slab_applies(A, Lp, M, Lq, B, Kp, Kq)) return 3;
  return ttm_pair_applies(in_dtype, compute, in, A, Lp, M, Lq, B, Kp, Kq, outp, outq) ? 1 : 0;
}

bool ttm_pair_applies(int in_dtype, int compute, const void* in, int64_t A, int64_t Lp,
                      int64_t M, int64_t Lq, int64_t B, int64_t Kp, int64_t Kq,
                      const void* outp, const void* outq) {
  if (in_dtype != TK_F32 || compute != TK_C_FP32) return false;
  if ((tail_applies(A, Lp, M, Lq, B, Kp, Kq) || slab_applies(A, Lp, M, Lq, B, Kp, Kq)) &&
      ((uintptr_t)in | (uintptr_t)outp | (uintptr_t)outq) % 16 == 0)
    return true;
  if (B % 4 != 0 || Lq > kPairRows || Lq < 1 || Lp < 1) return false;
  if (Lq * B >= ((int64_t)1 << 31)) return false;  // per-lane offsets are 32-bit
  if (Kp < 1 || Kq < 1 || Kp > 20 || Kq > 20) return false;
  if (((uintptr_t)in | (uintptr_t)outp | (uintptr_t)outq) % 16 != 0) return false;
  const int KGP = (int)((Kp + 3) / 4), KGQ = (int)((Kq + 3) / 4);
  if (pair_lds((int)Lp, (int)Lq, KGP, KGQ) > 80 * 1024) return false;
  // enough tiles to fill the chip twice over
  return A * M * (B / 4) >= 2048;
}

hipError_t launch_ttm_pair(const float* in, int64_t A, int64_t Lp, int64_t M, int64_t Lq,
                           int64_t B, const float* Fp, int64_t Kp, const float* Fq, int64_t Kq,
                           float* outp, float* outq, hipStream_t st) {
  if (tail_applies(A, Lp, M, Lq, B, Kp, Kq)) {
    const int kp = Kp <= 4 ? 4 : 8, kq = Kq <= 4 ? 4 : 8;
    if (kp == 4 && kq == 4)
      return launch_tail<4, 4>(in, A, (int)Lp, (int)Lq, Fp, (int)Kp, Fq, (int)Kq, outp, outq, st);
    if (kp == 4)
      return launch_tail<4, 8>(in, A, (int)Lp, (int)Lq, Fp, (int)Kp, Fq, (int)Kq, outp, outq, st);
    if (kq == 4)
      return launch_tail<8, 4>(in, A, (int)Lp, (int)Lq, Fp, (int)Kp, Fq, (int)Kq, outp, outq, st);
    return launch_tail<8, 8>(in, A, (int)Lp, (int)Lq, Fp, (int)Kp, Fq, (int)Kq, outp, outq, st);
  }
  if (slab_applies(A, Lp, M, Lq, B, Kp, Kq)) {
    const int kgp = (int)((Kp + 3) / 4), kgq = (int)((Kq + 3) / 4);
#define TK_SLAB_CASE(P, Q)                                                                 \
  if (kgp == P && kgq == Q)                                                                \
    return launch_slab<P, Q>(in, A, (int)Lp, (int)Lq, Fp, (int)Kp, Fq, (int)Kq, outp, outq, st);
#define TK_SLAB_ROW(P) \
  TK_SLAB_CASE(P, 1) TK_SLAB_CASE(P, 2) TK_SLAB_CASE(P, 3) TK_SLAB_CASE(P, 4) TK_SLAB_CASE(P, 5)
    TK_SLAB_ROW(1)
    TK_SLAB_ROW(2)
    TK_SLAB_ROW(3)
    TK_SLAB_ROW(4)
    TK_SLAB_ROW(5)
#undef TK_SLAB_ROW
#undef TK_SLAB_CASE
    return hipErrorInvalidValue;
  }
  const int kgp = (int)((Kp + 3) / 4), kgq = (int)((Kq + 3) / 4);
#define TK_PAIR_CASE(P, Q)                                                                 \
  if (kgp == P && kgq == Q)                                                                \
    return launch_pair_kg<P, Q>(in, A, (int)Lp, M, (int)Lq, B, Fp, (int)Kp, Fq, (int)Kq, outp, \
                                outq, st);
#define TK_PAIR_ROW(P) \
  TK_PAIR_CASE(P, 1) TK_PAIR_CASE(P, 2) TK_PAIR_CASE(P, 3) TK_PAIR_CASE(P, 4) TK_PAIR_CASE(P, 5)
  TK_PAIR_ROW(1)
  TK_PAIR_ROW(2)
  TK_PAIR_ROW(3)
  TK_PAIR_ROW(4)
  TK_PAIR_ROW(5)
#undef TK_PAIR_ROW
#undef TK_PAIR_CASE
  return hipErrorInvalidValue;
}

}  // namespace tk
