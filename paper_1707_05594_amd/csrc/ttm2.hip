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
constexpr int kRedPitch = 65;    // LDS pitch of one output's 64 partial sums

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
  float* FTq = FTp + 4 * Lp * KGP;             // [Lq][KGQ][4]: Fq[lq, 4g + r]
  float* red = FTq + Lq * KGQ * 4;             // 2 x [16 KGQ][kRedPitch]
  const int64_t t = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (t >= ntiles) return;  // the whole block
  const int tid = threadIdx.x;
  for (int e = tid; e < 4 * Lp * KGP; e += kPairThreads) {
    const int g = e % KGP, lp = (e / KGP) % Lp, r = e / (KGP * Lp);
    const int k = 4 * g + r;
    FTp[e] = k < Kp ? Fp[(int64_t)lp * Kp + k] : 0.f;
  }
  for (int e = tid; e < Lq * KGQ * 4; e += kPairThreads) {
    const int r = e % 4, g = (e / 4) % KGQ, lq = e / (4 * KGQ);
    const int k = 4 * g + r;
    FTq[e] = k < Kq ? Fq[(int64_t)lq * Kq + k] : 0.f;
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
      const float* fq = FTq + frow[j] * KGQ * 4 + i;
#pragma unroll
      for (int g = 0; g < KGQ; ++g) accq[g] = mfma4(fq[4 * g], x[j], accq[g]);
    }
    // partial sums of output (kq = 4 g + r, b = i) -> red[o][wave * 16 + beta];
    // the two buffers alternate, so a buffer is written again only after the
    // next step's barrier, when its readers are done
    float* rb = red + (lp & 1) * (16 * KGQ * kRedPitch);
#pragma unroll
    for (int g = 0; g < KGQ; ++g)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        rb[((4 * g + r) * 4 + i) * kRedPitch + wave * 16 + beta] = accq[g][r];
    lds_barrier();
    if (tid < 16 * KGQ) {
      const float* pr = rb + tid * kRedPitch;
      float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
#pragma unroll
      for (int q = 0; q < 64; q += 4) {
        s0 += pr[q];
        s1 += pr[q + 1];
        s2 += pr[q + 2];
        s3 += pr[q + 3];
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

size_t pair_lds(int Lp, int Lq, int KGP, int KGQ) {
  return sizeof(float) * ((size_t)4 * Lp * KGP + (size_t)Lq * KGQ * 4 +
                          (size_t)2 * 16 * KGQ * kRedPitch);
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

bool ttm_pair_applies(int in_dtype, int compute, const void* in, int64_t A, int64_t Lp,
                      int64_t M, int64_t Lq, int64_t B, int64_t Kp, int64_t Kq,
                      const void* outp, const void* outq) {
  if (in_dtype != TK_F32 || compute != TK_C_FP32) return false;
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
