// Leading eigenvectors of the Gram matrices, FP64 (the EVD after the Gram
// product, Sec. 5; F~_n = leading K_n left singular vectors, Fig. 2).
//
// One workgroup per matrix.  Subspace iteration with Rayleigh-Ritz on a block
// of p >= K columns:
//
//   V = orth(start)                     start = previous factor + fill columns
//   loop:  W = S V
//          H = V^T W,  H = Z diag(theta) Z^T   (Jacobi, one wavefront)
//          V <- V Z,  W <- W Z           (Ritz pairs, theta descending)
//          stop when ||W_j - theta_j V_j|| <= tol * theta_0 for every j < K
//          V = orth(W)                   (power step)
//
// A warm start (previous factors) runs with a small block p = K + 4; if it
// has not converged after `maxit` steps the block grows to p_max (fresh fill
// columns) for up to another `maxit` steps.  p = L makes the Rayleigh-Ritz
// step a full Jacobi eigen-decomposition (used when L is small).
// orth() is Cholesky-QR applied twice to column-normalised blocks; a column
// whose normalised Cholesky pivot vanishes (rank deficiency) is zeroed.
// Output: the first K Ritz vectors, each with its largest-magnitude entry
// (lowest row on ties) made positive, and their eigenvalues.
//
// The blocks V and W live in LDS when 2 L p_max doubles fit (else in a global
// work area); H, Z and the Jacobi double buffer always live in LDS.  The
// products S V, V^T W, V Z use all 256 threads; Cholesky and the p x p Jacobi
// run on wavefront 0 alone with wavefront-level ordering.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "device.h"
#include "internal.h"
#include "kernels.h"

namespace tk {

constexpr int kEigPMax = 48;
constexpr int kEigThreads = 256;
constexpr int kEigLdsMax = 160 * 1024;

__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

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
  double cs_c[kEigPMax], cs_s[kEigPMax];
  int partner[kEigPMax];
  int perm[kEigPMax];
  int flag;
};

struct EigMem {
  double* H;   // p_max^2 (LDS)
  double* Z;   // p_max^2 (LDS)
  double* H2;  // p_max^2 (LDS)
  double* V;   // L x p, row stride p (LDS or global)
  double* W;
  EigSmall* sm;
};

// Sum over the block of per-thread vectors v[0..n-1] -> out[0..n-1].
__device__ __forceinline__ void block_sum_vec(const double (&v)[kEigPMax], int n, double* red,
                                              double* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < kEigPMax; ++j) {
    if (j < n) {
      double s = wave_sum(v[j]);
      if (lane == 0) red[wave * kEigPMax + j] = s;
    }
  }
  __syncthreads();
  if (threadIdx.x < n) {
    double s = 0.0;
    for (int w = 0; w < 4; ++w) s += red[w * kEigPMax + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// G = V^T V (p x p) with V row-major L x p.
__device__ void gram_small(const double* V, int L, int p, double* G) {
  const int np = p * (p + 1) / 2;
  for (int e = threadIdx.x; e < np; e += kEigThreads) {
    int j1 = 0, rem = e;
    while (rem >= p - j1) {
      rem -= p - j1;
      ++j1;
    }
    const int j2 = j1 + rem;
    double s0 = 0.0, s1 = 0.0;
    int i = 0;
    for (; i + 1 < L; i += 2) {
      s0 = fma(V[i * p + j1], V[i * p + j2], s0);
      s1 = fma(V[(i + 1) * p + j1], V[(i + 1) * p + j2], s1);
    }
    if (i < L) s0 = fma(V[i * p + j1], V[i * p + j2], s0);
    G[j1 * p + j2] = s0 + s1;
    G[j2 * p + j1] = s0 + s1;
  }
}

// One Cholesky-QR pass on V (L x p), in place.
__device__ void cholqr_pass(EigMem& m, int L, int p) {
  double* V = m.V;
  double* H = m.H;
  EigSmall& sh = *m.sm;
  gram_small(V, L, p, H);
  __syncthreads();
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    for (int j = lane; j < p; j += 64) {
      const double d = H[j * p + j];
      sh.dscale[j] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
    }
    wave_fence();
    for (int e = lane; e < p * p; e += 64) {
      const int r = e / p, c = e % p;
      H[e] *= sh.dscale[r] * sh.dscale[c];
    }
    wave_fence();
    for (int j = 0; j < p; ++j) {
      const double piv = H[j * p + j];
      const bool dead = !(piv > 1e-15) || sh.dscale[j] == 0.0;
      const double d = dead ? 0.0 : sqrt(piv);
      wave_fence();
      for (int i = j + 1 + lane; i < p; i += 64) H[i * p + j] = dead ? 0.0 : H[i * p + j] / d;
      if (lane == 0) H[j * p + j] = dead ? 0.0 : d;
      wave_fence();
      const int w = p - j - 1;
      for (int e = lane; e < w * w; e += 64) {
        const int i = j + 1 + e / w;
        const int k = j + 1 + e % w;
        if (k <= i) H[i * p + k] -= H[i * p + j] * H[k * p + j];
      }
      wave_fence();
    }
  }
  __syncthreads();
  // V <- V D R^{-1}; row i solves x R = v D (R upper = transpose of the factor in H)
  for (int i = threadIdx.x; i < L; i += kEigThreads) {
    double x[kEigPMax];
#pragma unroll
    for (int j = 0; j < kEigPMax; ++j) x[j] = (j < p) ? V[i * p + j] * sh.dscale[j] : 0.0;
#pragma unroll
    for (int j = 0; j < kEigPMax; ++j) {
      if (j < p) {
        double s = x[j];
#pragma unroll
        for (int k = 0; k < j; ++k) s -= x[k] * H[j * p + k];
        const double rjj = H[j * p + j];
        x[j] = rjj > 0.0 ? s / rjj : 0.0;
      }
    }
#pragma unroll
    for (int j = 0; j < kEigPMax; ++j)
      if (j < p) V[i * p + j] = x[j];
  }
  __syncthreads();
}

__device__ void orth(EigMem& m, int L, int p) {
  cholqr_pass(m, L, p);
  cholqr_pass(m, L, p);
}

// Cyclic Jacobi (round-robin pairs) on H (p x p) by wavefront 0; Z accumulates
// the rotations.
__device__ void jacobi_wave(EigMem& m, int p, int maxsweep) {
  EigSmall& sh = *m.sm;
  const int lane = threadIdx.x;
  const int pe = p + (p & 1);
  double* Z = m.Z;
  for (int e = lane; e < p * p; e += 64) Z[e] = (e / p == e % p) ? 1.0 : 0.0;
  wave_fence();
  double* Hc = m.H;
  double* Hn = m.H2;
  for (int sweep = 0; sweep < maxsweep; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int e = lane; e < p * p; e += 64) {
      const double v = Hc[e];
      if (e / p == e % p)
        dia += v * v;
      else
        off += v * v;
    }
    off = wave_sum(off);
    dia = wave_sum(dia);
    if (off <= 1e-30 * dia || off == 0.0) break;
    for (int r = 0; r < pe - 1; ++r) {
      if (lane < pe / 2) {
        auto slot = [&](int s) { return s == 0 ? 0 : 1 + (s - 1 + r) % (pe - 1); };
        int a = slot(lane), b = slot(pe - 1 - lane);
        if (a > b) {
          const int t = a;
          a = b;
          b = t;
        }
        double c = 1.0, s = 0.0;
        if (b < p) {
          const double apq = Hc[a * p + b];
          if (apq != 0.0) {
            const double tau = (Hc[b * p + b] - Hc[a * p + a]) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        // rotation J: J[a][a] = c, J[b][a] = -s, J[a][b] = s, J[b][b] = c
        if (a < p) {
          sh.partner[a] = b < p ? b : a;
          sh.cs_c[a] = c;
          sh.cs_s[a] = b < p ? -s : 0.0;
        }
        if (b < p) {
          sh.partner[b] = a;
          sh.cs_c[b] = c;
          sh.cs_s[b] = s;
        }
      }
      wave_fence();
      for (int e = lane; e < p * p; e += 64) {
        const int x = e / p, y = e % p;
        const int xp = sh.partner[x], yp = sh.partner[y];
        const double ax = sh.cs_c[x], bx = sh.cs_s[x], ay = sh.cs_c[y], by = sh.cs_s[y];
        double v = ax * ay * Hc[x * p + y];
        if (yp != y) v += ax * by * Hc[x * p + yp];
        if (xp != x) v += bx * ay * Hc[xp * p + y];
        if (xp != x && yp != y) v += bx * by * Hc[xp * p + yp];
        if (xp == y && x != y) v = 0.0;  // the annihilated pair
        Hn[e] = v;
      }
      for (int e = lane; e < p * p; e += 64) {
        const int i = e / p, y = e % p;
        const int yp = sh.partner[y];
        if (yp < y) continue;
        const double zy = Z[i * p + y];
        if (yp == y) {
          Z[i * p + y] = sh.cs_c[y] * zy;
        } else {
          const double zyp = Z[i * p + yp];
          Z[i * p + y] = sh.cs_c[y] * zy + sh.cs_s[y] * zyp;
          Z[i * p + yp] = sh.cs_c[yp] * zyp + sh.cs_s[yp] * zy;
        }
      }
      wave_fence();
      double* t = Hc;
      Hc = Hn;
      Hn = t;
    }
  }
  if (Hc != m.H) {
    for (int e = lane; e < p * p; e += 64) m.H[e] = Hc[e];
    wave_fence();
  }
}

// Fill columns [j0, p) of V with deterministic pseudo-random values.
__device__ void fill_columns(double* V, int L, int p, int j0, uint64_t seed) {
  for (int e = threadIdx.x; e < L * (p - j0); e += kEigThreads) {
    const int i = e / (p - j0), j = j0 + e % (p - j0);
    V[i * p + j] = hash_unit((seed << 40) ^ ((uint64_t)i << 20) ^ (uint64_t)j);
  }
}

// Re-lay V from row stride p_old to row stride p_new (p_new > p_old), in place.
__device__ void widen_rows(double* V, int L, int p_old, int p_new) {
  // rows move to higher addresses: walk rows from the last one, one row per step
  for (int i = L - 1; i >= 0; --i) {
    double v = 0.0;
    const int j = threadIdx.x;
    if (j < p_old) v = V[i * p_old + j];
    __syncthreads();
    if (j < p_old) V[i * p_new + j] = v;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kEigThreads) void eig_subspace(
    const EigJob* __restrict__ jobs, int job0, const double* __restrict__ S_base,
    const double* __restrict__ V0_base, double* __restrict__ F_base, double* __restrict__ ev_base,
    double* __restrict__ work_base, int* __restrict__ status, int* __restrict__ iters_out,
    int maxit, double tol, int vw_in_lds) {
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

  EigMem m;
  m.H = dyn;
  m.Z = dyn + pmax * pmax;
  m.H2 = dyn + 2 * pmax * pmax;
  if (vw_in_lds) {
    m.V = dyn + 3 * pmax * pmax;
  } else {
    m.V = work_base + job.work_off;
  }
  m.W = m.V + (int64_t)L * pmax;
  m.sm = &small;
  EigSmall& sh = small;

  // start block: p = L (full Jacobi) when L <= p_max; warm: K + 4; cold: p_max
  int p;
  if (pmax == L)
    p = L;
  else if (V0)
    p = min(pmax, K + 4);
  else
    p = pmax;
  bool grown = (p == pmax);
  for (int e = tid; e < L * p; e += kEigThreads) {
    const int i = e / p, j = e % p;
    double v;
    if (p == L)
      v = (i == j) ? 1.0 : 0.0;
    else if (V0 && j < K)
      v = V0[(int64_t)i * K + j];
    else
      v = hash_unit(((uint64_t)mi << 40) ^ ((uint64_t)i << 20) ^ (uint64_t)j);
    m.V[e] = v;
  }
  __syncthreads();
  if (p < L) orth(m, L, p);

  int converged = 0;
  int used = 0;
  for (int it = 0; it < 2 * maxit; ++it) {
    used = it;
    if (it == maxit && !grown) {
      // not converged with the small block: widen to p_max with fresh columns
      widen_rows(m.V, L, p, pmax);
      fill_columns(m.V, L, pmax, p, (uint64_t)mi + 7777);
      p = pmax;
      grown = true;
      __syncthreads();
      orth(m, L, p);
    } else if (it == maxit) {
      break;
    }
    double* V = m.V;
    double* W = m.W;
    // ---- W = S V (S symmetric: threads walk rows i, reading S[l][i] coalesced)
    for (int i = tid; i < L; i += kEigThreads) {
      double acc[kEigPMax];
#pragma unroll
      for (int j = 0; j < kEigPMax; ++j) acc[j] = 0.0;
      // S comes from global memory: 16 loads in flight per step
      constexpr int kPre = 16;
      for (int l0 = 0; l0 < L; l0 += kPre) {
        double sv[kPre];
#pragma unroll
        for (int u = 0; u < kPre; ++u) sv[u] = (l0 + u < L) ? S[(int64_t)(l0 + u) * L + i] : 0.0;
#pragma unroll
        for (int u = 0; u < kPre; ++u) {
          if (l0 + u < L) {
            const double* vr = V + (l0 + u) * p;
#pragma unroll
            for (int j = 0; j < kEigPMax; ++j)
              if (j < p) acc[j] = fma(sv[u], vr[j], acc[j]);
          }
        }
      }
#pragma unroll
      for (int j = 0; j < kEigPMax; ++j)
        if (j < p) W[i * p + j] = acc[j];
    }
    __syncthreads();
    // ---- H = V^T W (symmetrised)
    {
      const int np = p * (p + 1) / 2;
      for (int e = tid; e < np; e += kEigThreads) {
        int j1 = 0, rem = e;
        while (rem >= p - j1) {
          rem -= p - j1;
          ++j1;
        }
        const int j2 = j1 + rem;
        double s12 = 0.0, s21 = 0.0;
        for (int i = 0; i < L; ++i) {
          s12 = fma(V[i * p + j1], W[i * p + j2], s12);
          s21 = fma(V[i * p + j2], W[i * p + j1], s21);
        }
        const double h = 0.5 * (s12 + s21);
        m.H[j1 * p + j2] = h;
        m.H[j2 * p + j1] = h;
      }
    }
    __syncthreads();
    if (tid < 64) {
      jacobi_wave(m, p, 30);
      for (int j = tid; j < p; j += 64) sh.theta[j] = m.H[j * p + j];
      wave_fence();
      for (int j = tid; j < p; j += 64) {
        const double tj = sh.theta[j];
        int rank = 0;
        for (int i = 0; i < p; ++i) {
          const double ti = sh.theta[i];
          rank += (ti > tj) || (ti == tj && i < j);
        }
        sh.perm[rank] = j;
      }
    }
    __syncthreads();
    // ---- Ritz vectors: V <- V Z(:, perm), W <- W Z(:, perm)
    for (int i = tid; i < L; i += kEigThreads) {
      double xv[kEigPMax], xw[kEigPMax];
#pragma unroll
      for (int j = 0; j < kEigPMax; ++j) {
        xv[j] = (j < p) ? V[i * p + j] : 0.0;
        xw[j] = (j < p) ? W[i * p + j] : 0.0;
      }
      for (int c = 0; c < p; ++c) {
        const int src = sh.perm[c];
        double sv = 0.0, sw = 0.0;
#pragma unroll
        for (int j = 0; j < kEigPMax; ++j) {
          if (j < p) {
            const double z = m.Z[j * p + src];
            sv = fma(xv[j], z, sv);
            sw = fma(xw[j], z, sw);
          }
        }
        V[i * p + c] = sv;
        W[i * p + c] = sw;
      }
    }
    __syncthreads();
    // ---- residuals of the leading K Ritz pairs
    {
      double part[kEigPMax];
#pragma unroll
      for (int j = 0; j < kEigPMax; ++j) part[j] = 0.0;
      for (int i = tid; i < L; i += kEigThreads) {
#pragma unroll
        for (int j = 0; j < kEigPMax; ++j) {
          if (j < K) {
            const double r = W[i * p + j] - sh.theta[sh.perm[j]] * V[i * p + j];
            part[j] = fma(r, r, part[j]);
          }
        }
      }
      block_sum_vec(part, K, sh.red, sh.dscale);
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
    for (int e = tid; e < L * p; e += kEigThreads) V[e] = W[e];
    __syncthreads();
    orth(m, L, p);
  }

  // ---- output: first K columns, sign rule, eigenvalues
  const double* V = m.V;
  for (int j = 0; j < K; ++j) {
    double best = -1.0;
    int bi = 0x7fffffff;
    for (int i = tid; i < L; i += kEigThreads) {
      const double a = fabs(V[i * p + j]);
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
      sh.dscale[0] = V[i0 * p + j] < 0.0 ? -1.0 : 1.0;
    }
    __syncthreads();
    const double sg = sh.dscale[0];
    for (int i = tid; i < L; i += kEigThreads) F[(int64_t)i * K + j] = sg * V[i * p + j];
    __syncthreads();
  }
  if (tid < K) ev[tid] = sh.theta[sh.perm[tid]];
  // failures only: callers clear the status array before a sequence of solves
  if (tid == 0 && converged != 1) status[mi] = converged < 0 ? 2 : 1;
  if (tid == 0 && iters_out) iters_out[mi] = used + 1;
}

int eig_block_size(int L, int K, int64_t rank_bound) {
  if (L <= kEigPMax) return L;
  int64_t p = K + 16;
  p = std::min<int64_t>(p, kEigPMax);
  p = std::min<int64_t>(p, L);
  p = std::min<int64_t>(p, std::max<int64_t>(rank_bound, K));
  return (int)std::max<int64_t>(p, K);
}

size_t eig_lds_bytes(int L, int p, bool vw_in_lds) {
  return sizeof(double) * ((size_t)3 * p * p + (vw_in_lds ? (size_t)2 * L * p : 0));
}

static int g_lds_limit = 0;  // dynamic LDS bytes available to one workgroup

bool eig_vw_fits_lds(int L, int p) {
  return eig_lds_bytes(L, p, true) <= (size_t)g_lds_limit;
}

hipError_t launch_eig(int count, const EigJob* jobs_dev, int job0, int Lmax, int pmax,
                      const double* S_base, const double* V0_base, double* F_base,
                      double* ev_base, double* work_base, int* status, int* iters, int maxit,
                      double tol, hipStream_t st) {
  if (count == 0) return hipSuccess;
  if (g_lds_limit == 0) {
    int dev = 0, per_block = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
      e = hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return e;
    int lim = std::min(per_block, kEigLdsMax) - (int)sizeof(EigSmall);
    if (lim > 64 * 1024) {
      e = hipFuncSetAttribute((const void*)eig_subspace,
                              hipFuncAttributeMaxDynamicSharedMemorySize, lim);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        lim = 64 * 1024 - (int)sizeof(EigSmall);
      }
    }
    g_lds_limit = lim;
  }
  const bool in_lds = eig_vw_fits_lds(Lmax, pmax);
  const size_t lds = eig_lds_bytes(Lmax, pmax, in_lds);
  hipLaunchKernelGGL(eig_subspace, dim3(count), dim3(kEigThreads), lds, st, jobs_dev, job0,
                     S_base, V0_base, F_base, ev_base, work_base, status, iters, maxit, tol,
                     in_lds ? 1 : 0);
  return hipGetLastError();
}

int eig_max_K() { return kEigPMax; }

}  // namespace tk
