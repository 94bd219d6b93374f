// Leading eigenvectors of the Gram matrices, FP64 (the EVD after the Gram
// product, Sec. 5; F~_n = leading K_n left singular vectors, Fig. 2).
//
// One workgroup per matrix.  Subspace iteration with Rayleigh-Ritz on a block
// of p >= K columns:
//
//   V = orth(start)
//   loop:  W = S V
//          H = V^T W,  H = Z diag(theta) Z^T   (cyclic Jacobi)
//          V <- V Z,  W <- W Z           (Ritz pairs, theta descending)
//          stop when ||W_j - theta_j V_j|| <= tol * theta_0 for every j < K
//          V = orth(W)                   (power step)
//
// A warm start begins from the previous factors alone (p = K): the Ritz
// matrix is then nearly diagonal and Jacobi converges in one or two sweeps.
// If that has not converged after `maxit` steps, the block grows to p_max
// with deterministic fill columns for up to another `maxit` steps.  A cold
// start uses p_max from the outset; p = L makes the Rayleigh-Ritz step a full
// Jacobi eigen-decomposition (used when L is small).
// orth() is Cholesky-QR applied twice to column-normalised blocks; a column
// whose normalised Cholesky pivot vanishes (rank deficiency) is zeroed.
// Output: the first K Ritz vectors, each with its largest-magnitude entry
// (lowest row on ties) made positive, and their eigenvalues.
//
// The kernel is instantiated for a padded block width PS (a multiple of 8,
// PS >= p): V, W have row stride PS, H and Z are PS x PS, and every loop runs
// over PS columns with static bounds (the columns p..PS-1 hold zeros, Z holds
// the identity there), so loads are batched instead of serialised behind
// guards.  V and W live in LDS when they fit, else in a global work area.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "device.h"
#include "internal.h"
#include "kernels.h"

namespace tk {

constexpr int kEigPMax = 64;
constexpr int kEigThreads = 256;
constexpr int kEigLdsMax = 160 * 1024;

__device__ __forceinline__ double hash_unit(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  x ^= x >> 31;
  return (double)(x >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

struct EigSmall {
  double theta[kEigPMax];
  double dscale[kEigPMax];
  double red[4 * kEigPMax];
  double cs_c[kEigPMax];  // Cholesky reciprocals (cholqr_pass)
  // rotations of one Jacobi round: pair q = (pair_a[q] < pair_b[q]), cosine, sine
  int pair_a[kEigPMax / 2], pair_b[kEigPMax / 2];
  double pair_c[kEigPMax / 2], pair_s[kEigPMax / 2];
  int perm[kEigPMax];
  int flag;
  double minpiv;
};

template <int PS>
struct EigMem {
  double* H;   // PS x PS (LDS)
  double* Z;   // PS x PS (LDS)
  double* H2;  // PS x PS (LDS)
  double* V;   // L x PS (LDS or global)
  double* W;   // L x PS
  EigSmall* sm;
};

// Sum over the block of per-thread vectors v[0..PS-1] -> out[0..PS-1].
template <int PS>
__device__ __forceinline__ void block_sum_vec(const double (&v)[PS], double* red, double* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < PS; ++j) {
    const double s = wave_sum(v[j]);
    if (lane == 0) red[wave * kEigPMax + j] = s;
  }
  __syncthreads();
  if (threadIdx.x < PS) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < 4; ++w) s += red[w * kEigPMax + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// out[a][b] = sum_i X[i][a] * Y[i][b] for a <= b (PS x PS, symmetric fill).
// Each thread owns one (a, b) pair and walks the rows with 16-byte loads.
template <int PS, bool SYM_AVG>
__device__ __forceinline__ void crossprod(const double* X, const double* Y, int L, double* out) {
  constexpr int NP = PS * (PS + 1) / 2;
  for (int e = threadIdx.x; e < NP; e += kEigThreads) {
    int a = 0, rem = e;
    while (rem >= PS - a) {
      rem -= PS - a;
      ++a;
    }
    const int b = a + rem;
    double s0 = 0.0, s1 = 0.0, t0 = 0.0, t1 = 0.0;
    int i = 0;
    for (; i + 1 < L; i += 2) {
      s0 = fma(X[i * PS + a], Y[i * PS + b], s0);
      s1 = fma(X[(i + 1) * PS + a], Y[(i + 1) * PS + b], s1);
      if (SYM_AVG) {
        t0 = fma(X[i * PS + b], Y[i * PS + a], t0);
        t1 = fma(X[(i + 1) * PS + b], Y[(i + 1) * PS + a], t1);
      }
    }
    if (i < L) {
      s0 = fma(X[i * PS + a], Y[i * PS + b], s0);
      if (SYM_AVG) t0 = fma(X[i * PS + b], Y[i * PS + a], t0);
    }
    const double v = SYM_AVG ? 0.5 * ((s0 + s1) + (t0 + t1)) : (s0 + s1);
    out[a * PS + b] = v;
    out[b * PS + a] = v;
  }
}

// One Cholesky-QR pass on V (L x PS), in place.
template <int PS>
__device__ __forceinline__ void cholqr_pass(EigMem<PS>& m, int L) {
  double* V = m.V;
  double* H = m.H;
  EigSmall& sh = *m.sm;
  const int tid = threadIdx.x;
  crossprod<PS, false>(V, V, L, H);
  __syncthreads();
  // Cholesky of D G D (D = diag(G)^{-1/2}), lower factor in place, whole block
  if (tid < PS) {
    const double d = H[tid * PS + tid];
    sh.dscale[tid] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < PS * PS; e += kEigThreads) H[e] *= sh.dscale[e / PS] * sh.dscale[e % PS];
  __syncthreads();
  double minpiv = 1.0;  // smallest normalised pivot of a live column (same in every thread)
  for (int j = 0; j < PS; ++j) {
    const double piv = H[j * PS + j];
    const bool dead = !(piv > 1e-15) || sh.dscale[j] == 0.0;
    if (sh.dscale[j] != 0.0) minpiv = fmin(minpiv, piv);
    const double inv = dead ? 0.0 : 1.0 / sqrt(piv);
    __syncthreads();  // every thread has read the pivot
    if (tid > j && tid < PS) H[tid * PS + j] *= inv;
    if (tid == 0) H[j * PS + j] = dead ? 0.0 : sqrt(piv);
    __syncthreads();
    // trailing update of the lower triangle, rows and columns j+1..PS-1
    const int w = PS - j - 1;
    for (int e = tid; e < w * w; e += kEigThreads) {
      const int i = j + 1 + e / w;
      const int k = j + 1 + e % w;
      if (k <= i) H[i * PS + k] -= H[i * PS + j] * H[k * PS + j];
    }
    __syncthreads();
  }
  // reciprocal diagonal for the solve (cs_c is free outside the Jacobi sweep)
  if (tid < PS) {
    const double r = H[tid * PS + tid];
    sh.cs_c[tid] = r > 0.0 ? 1.0 / r : 0.0;
  }
  if (tid == 0) sh.minpiv = minpiv;
  __syncthreads();
  // V <- V M with M = D R^{-1} (R = transpose of the lower factor Lc in H): row
  // i of the result solves x R = v D.  Column c of M follows from the earlier
  // ones, M(:,c) = (d_c e_c - sum_{k<c} M(:,k) Lc[c][k]) / Lc[c][c]; thread j
  // builds row j of M in H2 (a dead column has a zero reciprocal: zero column).
  double* M = m.H2;
  if (tid < PS) {
    const int j = tid;
    for (int c = 0; c < PS; ++c) {
      double acc = (j == c) ? sh.dscale[c] : 0.0;
      for (int k = j; k < c; ++k) acc -= M[j * PS + k] * H[c * PS + k];
      M[j * PS + c] = acc * sh.cs_c[c];
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < L; i += kEigThreads) {
    double x[PS];
#pragma unroll
    for (int j = 0; j < PS; ++j) x[j] = V[i * PS + j];
#pragma unroll 2
    for (int c = 0; c < PS; ++c) {
      double sx = 0.0;
#pragma unroll
      for (int j = 0; j < PS; ++j) sx = fma(x[j], M[j * PS + c], sx);
      V[i * PS + c] = sx;
    }
  }
  __syncthreads();
}

// Cholesky-QR, repeated once unless the first pass saw a well-conditioned
// block (every normalised pivot >= 1/2, i.e. each column keeps at least
// 1/sqrt(2) of its norm outside the span of the previous ones): then one pass
// already leaves V orthonormal to rounding.
template <int PS>
__device__ __forceinline__ void orth(EigMem<PS>& m, int L) {
  cholqr_pass<PS>(m, L);
  if (m.sm->minpiv < 0.5) cholqr_pass<PS>(m, L);
}

// Cyclic Jacobi (round-robin pairs) on H (PS x PS) by the whole block; Z
// accumulates the rotations.  A round rotates PS / 2 disjoint pairs at once:
// with J the product of the round's rotations, H <- J^T H J is applied by 2 x 2
// blocks -- the block of row pair P and column pair R depends only on its own
// four entries and the two pairs' rotations, so one thread reads it once and
// rewrites it in place -- and Z <- Z J by the two columns of each pair.
template <int PS>
__device__ __forceinline__ void jacobi_block(EigMem<PS>& m, int maxsweep) {
  constexpr int NP = PS / 2;
  EigSmall& sh = *m.sm;
  const int tid = threadIdx.x;
  double* Z = m.Z;
  double* H = m.H;
  for (int e = tid; e < PS * PS; e += kEigThreads) Z[e] = (e / PS == e % PS) ? 1.0 : 0.0;
  __syncthreads();
  for (int sweep = 0; sweep < maxsweep; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int e = tid; e < PS * PS; e += kEigThreads) {
      const double v = H[e];
      if (e / PS == e % PS)
        dia += v * v;
      else
        off += v * v;
    }
    off = wave_sum(off);
    dia = wave_sum(dia);
    if ((tid & 63) == 0) {
      sh.red[2 * (tid >> 6)] = off;
      sh.red[2 * (tid >> 6) + 1] = dia;
    }
    __syncthreads();
    off = (sh.red[0] + sh.red[2]) + (sh.red[4] + sh.red[6]);
    dia = (sh.red[1] + sh.red[3]) + (sh.red[5] + sh.red[7]);
    __syncthreads();
    // off-diagonal norm <= 1e-13 of the diagonal's: the Ritz pairs are then
    // exact to far below the residual test that decides convergence
    if (off <= 1e-26 * dia || off == 0.0) break;
    for (int r = 0; r < PS - 1; ++r) {
      if (tid < NP) {
        auto slot = [&](int q) { return q == 0 ? 0 : 1 + (q - 1 + r) % (PS - 1); };
        int a = slot(tid), b = slot(PS - 1 - tid);
        if (a > b) {
          const int t = a;
          a = b;
          b = t;
        }
        double c = 1.0, s = 0.0;
        const double apq = H[a * PS + b];
        if (apq != 0.0) {
          const double tau = (H[b * PS + b] - H[a * PS + a]) / (2.0 * apq);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
        }
        // rotation: J[a][a] = c, J[b][a] = -s, J[a][b] = s, J[b][b] = c
        sh.pair_a[tid] = a;
        sh.pair_b[tid] = b;
        sh.pair_c[tid] = c;
        sh.pair_s[tid] = s;
      }
      __syncthreads();
      for (int w = tid; w < NP * NP; w += kEigThreads) {
        const int P = w / NP, R = w % NP;
        const int aP = sh.pair_a[P], bP = sh.pair_b[P], aR = sh.pair_a[R], bR = sh.pair_b[R];
        const double cP = sh.pair_c[P], sP = sh.pair_s[P], cR = sh.pair_c[R], sR = sh.pair_s[R];
        const double haa = H[aP * PS + aR], hab = H[aP * PS + bR];
        const double hba = H[bP * PS + aR], hbb = H[bP * PS + bR];
        // rows: x = a takes (c, -s) with its partner, x = b takes (c, +s); columns alike
        double naa = cP * cR * haa - cP * sR * hab - sP * cR * hba + sP * sR * hbb;
        double nab = cP * cR * hab + cP * sR * haa - sP * cR * hbb - sP * sR * hba;
        double nba = cP * cR * hba - cP * sR * hbb + sP * cR * haa - sP * sR * hab;
        const double nbb = cP * cR * hbb + cP * sR * hba + sP * cR * hab + sP * sR * haa;
        if (P == R) nab = nba = 0.0;  // the annihilated pair
        H[aP * PS + aR] = naa;
        H[aP * PS + bR] = nab;
        H[bP * PS + aR] = nba;
        H[bP * PS + bR] = nbb;
      }
      for (int w = tid; w < PS * NP; w += kEigThreads) {
        const int i = w / NP, P = w % NP;
        const int a = sh.pair_a[P], b = sh.pair_b[P];
        const double c = sh.pair_c[P], s = sh.pair_s[P];
        const double za = Z[i * PS + a], zb = Z[i * PS + b];
        Z[i * PS + a] = c * za - s * zb;
        Z[i * PS + b] = c * zb + s * za;
      }
      __syncthreads();
    }
  }
}

// kLds: V and W live in LDS (a compile-time choice, so that every access to
// them is an LDS instruction rather than a generic one).
template <int PS, bool kLds>
__global__ __launch_bounds__(kEigThreads) void eig_subspace(
    const EigJob* __restrict__ jobs, int job0, const double* __restrict__ S_base,
    const double* __restrict__ V0_base, double* __restrict__ F_base, double* __restrict__ ev_base,
    double* __restrict__ work_base, int* __restrict__ status, int* __restrict__ iters_out,
    int maxit, double tol, double* __restrict__ basis_base) {
  extern __shared__ double dyn[];
  __shared__ EigSmall small;
  const int mi = job0 + blockIdx.x;
  const EigJob job = jobs[mi];
  const int L = job.L, K = job.K, pmax = job.p;
  const double* S = S_base + job.S_off;
  const double* V0 = job.V0_off >= 0 ? V0_base + job.V0_off : nullptr;
  double* F = F_base + job.F_off;
  double* ev = ev_base + job.ev_off;
  const int tid = threadIdx.x;

  EigMem<PS> m;
  m.H = dyn;
  m.Z = dyn + PS * PS;
  m.H2 = dyn + 2 * PS * PS;
  if constexpr (kLds)
    m.V = dyn + 3 * PS * PS;
  else
    m.V = work_base + job.work_off;
  m.W = m.V + (int64_t)L * PS;
  m.sm = &small;
  EigSmall& sh = small;

  // start block: p = L (full Jacobi) when L <= p_max, from the stored basis
  // on a warm solve (else the identity); warm: the K previous factors; cold:
  // p_max columns
  int p;
  if (pmax == L)
    p = L;
  else if (V0)
    p = K;
  else
    p = pmax;
  double* basis = (p == L && job.basis_off >= 0 && basis_base) ? basis_base + job.basis_off
                                                                : nullptr;
  const bool warm_basis = basis && V0;
  bool grown = (p == pmax);
  for (int e = tid; e < L * PS; e += kEigThreads) {
    const int i = e / PS, j = e % PS;
    double v = 0.0;
    if (j < p) {
      if (p == L)
        v = warm_basis ? basis[i * L + j] : ((i == j) ? 1.0 : 0.0);
      else if (V0 && j < K)
        v = V0[(int64_t)i * K + j];
      else
        v = hash_unit(((uint64_t)mi << 40) ^ ((uint64_t)i << 20) ^ (uint64_t)j);
    }
    m.V[e] = v;
  }
  __syncthreads();
  if (p < L || warm_basis) orth<PS>(m, L);

  int converged = 0;
  int used = 0;
  for (int it = 0; it < 2 * maxit; ++it) {
    used = it;
    if (it == maxit && !grown) {
      // not converged with the small block: add fill columns up to p_max
      for (int e = tid; e < L * PS; e += kEigThreads) {
        const int i = e / PS, j = e % PS;
        if (j >= p && j < pmax)
          m.V[e] = hash_unit(((uint64_t)(mi + 7777) << 40) ^ ((uint64_t)i << 20) ^ (uint64_t)j);
      }
      p = pmax;
      grown = true;
      __syncthreads();
      orth<PS>(m, L);
    } else if (it == maxit) {
      break;
    }
    double* V = m.V;
    double* W = m.W;
    // ---- W = S V (S symmetric: threads walk rows i, reading S[l][i] coalesced),
    // in column chunks of kCW so the accumulators stay in registers
    // one pass over S for blocks up to 32 columns, else chunks that divide PS
    constexpr int kCW = PS <= 32 ? PS : (PS % 16 == 0 ? 16 : 8);
    static_assert(PS % kCW == 0, "column chunks must tile the padded width");
    for (int i = tid; i < L; i += kEigThreads) {
      for (int c0 = 0; c0 < PS; c0 += kCW) {
        double acc[kCW];
#pragma unroll
        for (int j = 0; j < kCW; ++j) acc[j] = 0.0;
        constexpr int kPre = 8;
        for (int l0 = 0; l0 < L; l0 += kPre) {
          double sv[kPre];
#pragma unroll
          for (int u = 0; u < kPre; ++u) sv[u] = (l0 + u < L) ? S[(int64_t)(l0 + u) * L + i] : 0.0;
#pragma unroll
          for (int u = 0; u < kPre; ++u) {
            const int l = min(l0 + u, L - 1);  // sv is 0 past the end
            const double* vr = V + l * PS + c0;
#pragma unroll
            for (int j = 0; j < kCW; ++j) acc[j] = fma(sv[u], vr[j], acc[j]);
          }
        }
#pragma unroll
        for (int j = 0; j < kCW; ++j) W[i * PS + c0 + j] = acc[j];
      }
    }
    __syncthreads();
    // ---- H = V^T W (symmetrised)
    crossprod<PS, true>(V, W, L, m.H);
    __syncthreads();
    jacobi_block<PS>(m, 30);
    if (tid < PS) sh.theta[tid] = m.H[tid * PS + tid];
    __syncthreads();
    if (tid < PS) {
      const int j = tid;
      const double tj = sh.theta[j];
      int rank = 0;
      for (int i = 0; i < PS; ++i) {
        const double ti = sh.theta[i];
        // padded columns (j >= p) rank last
        const bool before = (i < p) && ((j >= p) || ti > tj || (ti == tj && i < j));
        rank += before || (j >= p && i >= p && i < j);
      }
      sh.perm[rank] = j;
    }
    __syncthreads();
    // ---- Ritz vectors: V <- V Z(:, perm), W <- W Z(:, perm), one block at a time
    for (int pass = 0; pass < 2; ++pass) {
      double* X = pass == 0 ? V : W;
      for (int i = tid; i < L; i += kEigThreads) {
        double x[PS];
#pragma unroll
        for (int j = 0; j < PS; ++j) x[j] = X[i * PS + j];
#pragma unroll 2
        for (int c = 0; c < PS; ++c) {
          const int src = sh.perm[c];
          double sx = 0.0;
#pragma unroll
          for (int j = 0; j < PS; ++j) sx = fma(x[j], m.Z[j * PS + src], sx);
          X[i * PS + c] = sx;
        }
      }
    }
    __syncthreads();
    // ---- residuals of the leading K Ritz pairs (column chunks of kCW)
    {
      for (int c0 = 0; c0 < PS; c0 += kCW) {
        double part[kCW];
#pragma unroll
        for (int j = 0; j < kCW; ++j) part[j] = 0.0;
        for (int i = tid; i < L; i += kEigThreads) {
#pragma unroll
          for (int j = 0; j < kCW; ++j) {
            const double r = W[i * PS + c0 + j] - sh.theta[sh.perm[c0 + j]] * V[i * PS + c0 + j];
            part[j] = fma(r, r, part[j]);
          }
        }
        block_sum_vec<kCW>(part, sh.red, sh.dscale + c0);
      }
      if (tid == 0) {
        const double t0 = fabs(sh.theta[sh.perm[0]]);
        double worst = 0.0;
        bool finite = true;
        for (int j = 0; j < K; ++j) {
          worst = fmax(worst, sqrt(sh.dscale[j]));
          finite = finite && isfinite(sh.dscale[j]);
        }
        sh.flag = !finite ? 2 : (worst <= tol * fmax(t0, 1e-300) ? 1 : 0);
      }
      __syncthreads();
    }
    if (sh.flag == 2) {
      converged = -1;
      break;
    }
    if (sh.flag == 1) {
      converged = 1;
      break;
    }
    // ---- power step: V = orth(W)
    for (int e = tid; e < L * PS; e += kEigThreads) V[e] = W[e];
    __syncthreads();
    orth<PS>(m, L);
  }

  // ---- output: the basis (p = L), first K columns with the sign rule, eigenvalues
  const double* V = m.V;
  if (basis && converged == 1)
    for (int e = tid; e < L * L; e += kEigThreads) basis[e] = V[(e / L) * PS + e % L];
  for (int j = 0; j < K; ++j) {
    double best = -1.0;
    int bi = 0x7fffffff;
    for (int i = tid; i < L; i += kEigThreads) {
      const double a = fabs(V[i * PS + j]);
      if (a > best || (a == best && i < bi)) {
        best = a;
        bi = i;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if ((tid & 63) == 0) {
      sh.red[(tid >> 6) * 2] = best;
      sh.red[(tid >> 6) * 2 + 1] = (double)bi;
    }
    __syncthreads();
    if (tid == 0) {
      double b = sh.red[0];
      int i0 = (int)sh.red[1];
      for (int w = 1; w < 4; ++w) {
        const double ob = sh.red[2 * w];
        const int oi = (int)sh.red[2 * w + 1];
        if (ob > b || (ob == b && oi < i0)) {
          b = ob;
          i0 = oi;
        }
      }
      sh.dscale[0] = V[i0 * PS + j] < 0.0 ? -1.0 : 1.0;
    }
    __syncthreads();
    const double sg = sh.dscale[0];
    for (int i = tid; i < L; i += kEigThreads) F[(int64_t)i * K + j] = sg * V[i * PS + j];
    __syncthreads();
  }
  if (tid < K) ev[tid] = sh.theta[sh.perm[tid]];
  // failures only: callers clear the status array before a sequence of solves
  if (tid == 0 && converged != 1) status[mi] = converged < 0 ? 2 : 1;
  if (tid == 0 && iters_out) iters_out[mi] = used + 1;
}

// Up to L = 64 the block is the whole space (p = L), so every solve is a full
// Jacobi eigen-decomposition: exact in one step whatever the eigenvalue gaps,
// which matters when the trailing K_n eigenvalues sit in an almost flat noise
// spectrum (a planted core of lower numerical rank than K_n).  Larger L uses
// subspace iteration with a block of K + 16 columns (at most 48).
int eig_block_size(int L, int K, int64_t rank_bound) {
  if (L <= kEigPMax) return L;
  int64_t p = K + 16;
  p = std::min<int64_t>(p, 48);
  p = std::min<int64_t>(p, L);
  p = std::min<int64_t>(p, std::max<int64_t>(rank_bound, K));
  return (int)std::max<int64_t>(p, K);
}

namespace {

int padded(int p) { return (p + 7) / 8 * 8; }

size_t eig_lds_bytes(int L, int PS, bool vw_in_lds) {
  return sizeof(double) * ((size_t)3 * PS * PS + (vw_in_lds ? (size_t)2 * L * PS : 0));
}

int g_lds_limit = 0;  // dynamic LDS bytes available to one workgroup

template <int PS>
hipError_t set_attr(int lim) {
  hipError_t e = hipFuncSetAttribute((const void*)eig_subspace<PS, true>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)eig_subspace<PS, false>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, lim);
}

hipError_t init_lds_limit() {
  if (g_lds_limit != 0) return hipSuccess;
  int dev = 0, per_block = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return e;
  int lim = std::min(per_block, kEigLdsMax) - (int)sizeof(EigSmall);
  if (lim > 64 * 1024) {
    hipError_t a = set_attr<8>(lim);
    if (a == hipSuccess) a = set_attr<16>(lim);
    if (a == hipSuccess) a = set_attr<24>(lim);
    if (a == hipSuccess) a = set_attr<32>(lim);
    if (a == hipSuccess) a = set_attr<40>(lim);
    if (a == hipSuccess) a = set_attr<48>(lim);
    if (a == hipSuccess) a = set_attr<56>(lim);
    if (a == hipSuccess) a = set_attr<64>(lim);
    if (a != hipSuccess) {
      (void)hipGetLastError();
      lim = 64 * 1024 - (int)sizeof(EigSmall);
    }
  }
  g_lds_limit = lim;
  return hipSuccess;
}

template <int PS>
void launch_ps(int count, const EigJob* jobs_dev, int job0, int Lmax, const double* S_base,
               const double* V0_base, double* F_base, double* ev_base, double* work_base,
               int* status, int* iters, int maxit, double tol, hipStream_t st,
               double* basis_base) {
  const bool in_lds = eig_lds_bytes(Lmax, PS, true) <= (size_t)g_lds_limit;
  const size_t lds = eig_lds_bytes(Lmax, PS, in_lds);
  if (in_lds)
    hipLaunchKernelGGL((eig_subspace<PS, true>), dim3(count), dim3(kEigThreads), lds, st,
                       jobs_dev, job0, S_base, V0_base, F_base, ev_base, work_base, status, iters,
                       maxit, tol, basis_base);
  else
    hipLaunchKernelGGL((eig_subspace<PS, false>), dim3(count), dim3(kEigThreads), lds, st,
                       jobs_dev, job0, S_base, V0_base, F_base, ev_base, work_base, status, iters,
                       maxit, tol, basis_base);
}

}  // namespace

size_t eig_work_elems(int L, int p) { return (size_t)2 * L * padded(p); }

hipError_t launch_eig(int count, const EigJob* jobs_dev, int job0, int Lmax, int pmax,
                      const double* S_base, const double* V0_base, double* F_base,
                      double* ev_base, double* work_base, int* status, int* iters, int maxit,
                      double tol, hipStream_t st, double* basis_base) {
  if (count == 0) return hipSuccess;
  hipError_t e = init_lds_limit();
  if (e != hipSuccess) return e;
  const int PS = padded(pmax);
#define TK_EIG_CASE(P)                                                                    \
  case P:                                                                                 \
    launch_ps<P>(count, jobs_dev, job0, Lmax, S_base, V0_base, F_base, ev_base, work_base, \
                 status, iters, maxit, tol, st, basis_base);                              \
    break;
  switch (PS) {
    TK_EIG_CASE(8)
    TK_EIG_CASE(16)
    TK_EIG_CASE(24)
    TK_EIG_CASE(32)
    TK_EIG_CASE(40)
    TK_EIG_CASE(48)
    TK_EIG_CASE(56)
    TK_EIG_CASE(64)
    default:
      return hipErrorInvalidValue;
  }
#undef TK_EIG_CASE
  return hipGetLastError();
}

int eig_max_K() { return 48; }

void eig_identity_bases(const std::vector<EigJob>& jobs, std::vector<double>* out) {
  size_t n = 0;
  for (const EigJob& j : jobs)
    if (j.basis_off >= 0) n = std::max(n, (size_t)j.basis_off + (size_t)j.L * j.L);
  out->assign(n, 0.0);
  for (const EigJob& j : jobs)
    if (j.basis_off >= 0)
      for (int i = 0; i < j.L; ++i) (*out)[(size_t)j.basis_off + (size_t)i * j.L + i] = 1.0;
}

}  // namespace tk
