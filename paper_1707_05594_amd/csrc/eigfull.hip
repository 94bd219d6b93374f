// Leading eigenpairs of a symmetric FP64 matrix without any assumption on the
// eigenvalue gaps (the EVD after the Gram product, Sec. 5; the paper takes
// the leading K_n eigenvectors with an expert driver that tridiagonalises,
// bisects and inverse-iterates).  Used where subspace iteration is not enough:
// K above its block limit, or a solve that did not converge (no gap at K).
//
// Method (one workgroup per matrix for the first kernel):
//   1. Householder tridiagonalisation  Q^T S Q = tridiag(d, e),
//      Q = H_0 H_1 ... H_{L-3},  H_j = I - tau_j v_j v_j^T acting on rows
//      j+1 .. L-1 (v_j stored in row j of the work copy of S, v_j[j+1] = 1).
//   2. L < kInvItMinL: implicit QL iteration with Wilkinson shifts on (d, e),
//      accumulating the plane rotations into Z (eigenvectors of the
//      tridiagonal matrix); one thread chases the bulge and records the
//      rotations, then every thread applies them to its rows of Z; then the
//      ranks of the eigenvalues (descending, lower index first on ties) pick
//      the K largest and their columns of Z.
//   2'. L >= kInvItMinL (as the paper's expert driver does): the K largest
//      eigenvalues by bisection on Sturm counts, one thread per eigenvalue,
//      then their vectors by inverse iteration with the LU factors of
//      T - lambda I (partial pivoting), one thread per vector, then two
//      passes of modified Gram-Schmidt over the K vectors by the whole block
//      (inverse iteration leaves residuals of order eps ||T||; close
//      eigenvalues only cost orthogonality, which the passes restore).  This
//      avoids the L^3 rotation accumulation, which on one CU took most of a
//      large solve.
// A second kernel (a grid of column blocks per matrix) applies Q to the K
// selected columns (reflectors in reverse order, the block in LDS) and the
// sign rule (largest-magnitude entry of each vector positive, lowest row on
// ties).
//
// Work area per matrix (eig_full_work_elems): A (L x L), Zt (L x L, Zt[i][r] =
// Z[r][i], so a rotation of columns i, i+1 of Z reads two rows; the inverse-
// iteration path writes its vectors to rows 0 .. K-1), d, e, tau, the
// selection (as doubles), 4 L, a done flag that the first kernel sets (1:
// solved in this launch) and the second reads, and for L >= kInvItMinL the
// inverse-iteration scratch (6 L doubles per working thread).
//
// Status word of a job: 0 solved, 1 not converged, 2 non-finite values.  A
// job marked only_if_failed runs only when its status word is 1 (the
// subspace solve before it did not converge) and otherwise leaves F alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "device.h"
#include "internal.h"
#include "kernels.h"

namespace tk {

constexpr int kFullThreads = 256;  // back-transform
// reduction, QL / bisection and inverse iteration: 16 waves, so that one CU
// keeps enough loads in flight for the L^3 passes over the work matrix
constexpr int kTqThreads = 1024;
constexpr int kInvItSlots = 512;  // threads that run inverse iteration at once
constexpr int kFullMaxL = 2048;
constexpr int kQlMaxSweeps = 60;  // per eigenvalue

__device__ __forceinline__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kTqThreads / 64; ++w) s += red[w];
  return s;
}

// Smallest value of v over the block (every thread gets it).
__device__ __forceinline__ int block_min(int v, int* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  int r = red[0];
#pragma unroll
  for (int w = 1; w < kTqThreads / 64; ++w) r = min(r, red[w]);
  return r;
}

// ---- leading eigenpairs of the tridiagonal matrix by bisection and inverse
// iteration (the paper's route: the K wanted eigenvalues by Sturm-count
// bisection, their vectors by inverse iteration, then the back-transform),
// for L >= kInvItMinL, where accumulating every QL rotation into an L x L
// matrix on one CU is what the solve spends its time on.
constexpr int kInvItMinL = 192;
constexpr int kInvItIters = 3;
constexpr double kEps = 2.220446049250313e-16;
constexpr double kSafMin = 2.2250738585072014e-308;

// Number of eigenvalues of tridiag(e, d, e) below x (Sturm sequence of the
// LDL^T factorisation of T - x I; pivots below pivmin in magnitude replaced).
__device__ int sturm_count(const double* d, const double* e2, int L, double x, double pivmin) {
  int c = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  c += q < 0.0;
  for (int i = 1; i < L; ++i) {
    q = d[i] - x - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
  }
  return c;
}

// Eigenvalue j (ascending, 0-based) in [lo, hi] by bisection to full precision.
__device__ double bisect_eig(const double* d, const double* e2, int L, int j, double lo,
                             double hi, double pivmin) {
  for (int it = 0; it < 256; ++it) {
    const double mid = 0.5 * (lo + hi);
    const double tol = 2.0 * kEps * fmax(fabs(lo), fabs(hi)) + pivmin;
    if (hi - lo <= tol || mid == lo || mid == hi) break;
    if (sturm_count(d, e2, L, mid, pivmin) <= j)
      lo = mid;
    else
      hi = mid;
  }
  return 0.5 * (lo + hi);
}

// LU factorisation with partial pivoting of T - lam I (U with two
// superdiagonals u0, u1, u2; multipliers m; pv: rows i and i+1 swapped).
// A zero pivot is replaced by eps ||T||.
__device__ void tri_lu(const double* d, const double* e, int L, double lam, double tiny,
                       double* __restrict__ u0, double* __restrict__ u1,
                       double* __restrict__ u2, double* __restrict__ m,
                       double* __restrict__ pv) {
  double a = d[0] - lam;
  double b = L > 1 ? e[0] : 0.0;
  for (int i = 0; i + 1 < L; ++i) {
    const double c = e[i];
    const double an = d[i + 1] - lam;
    const double bn = i + 2 < L ? e[i + 1] : 0.0;
    if (fabs(a) >= fabs(c)) {
      if (a == 0.0) a = tiny;
      const double mu = c / a;
      u0[i] = a;
      u1[i] = b;
      u2[i] = 0.0;
      m[i] = mu;
      pv[i] = 0.0;
      a = an - mu * b;
      b = bn;
    } else {
      const double mu = a / c;
      u0[i] = c;
      u1[i] = an;
      u2[i] = bn;
      m[i] = mu;
      pv[i] = 1.0;
      a = b - mu * an;
      b = -mu * bn;
    }
  }
  u0[L - 1] = a == 0.0 ? tiny : a;
}

// x = (T - lam I)^-1 y through the factors (y is overwritten).
__device__ void tri_solve(int L, const double* __restrict__ u0, const double* __restrict__ u1,
                          const double* __restrict__ u2, const double* __restrict__ m,
                          const double* __restrict__ pv, double* __restrict__ y,
                          double* __restrict__ x) {
  for (int i = 0; i + 1 < L; ++i) {
    if (pv[i] != 0.0) {
      const double t = y[i];
      y[i] = y[i + 1];
      y[i + 1] = t;
    }
    y[i + 1] -= m[i] * y[i];
  }
  double x1 = 0.0, x2 = 0.0;  // x[i + 1], x[i + 2]
  for (int i = L - 1; i >= 0; --i) {
    const double xi = (y[i] - u1[i] * x1 - u2[i] * x2) / u0[i];
    x[i] = xi;
    x2 = x1;
    x1 = xi;
  }
}

// Work area of one matrix: A, Zt, d, e, tau, sel, done; then, for the
// inverse-iteration path, a scratch slot of 6 L doubles per thread that
// works (at most one per thread of the block).
__host__ __device__ inline int64_t eig_full_base_elems(int L) {
  return 2 * (int64_t)L * L + 4 * (int64_t)L + 1;
}
__host__ __device__ inline int invit_slots(int L) { return L < kInvItSlots ? L : kInvItSlots; }

struct FullShared {
  double red[kTqThreads / 64];
  double scal[4];
  int redi[kTqThreads / 64];
  int flag, lo;
};

__global__ __launch_bounds__(kTqThreads) void eig_full_tridiag_ql(
    const EigFullJob* __restrict__ jobs, const double* __restrict__ S_base,
    double* __restrict__ ev_base, double* __restrict__ work_base, int* __restrict__ status) {
  extern __shared__ double lds[];  // v, w (L each), rotation cosines, sines (L each)
  __shared__ FullShared sh;
  const EigFullJob job = jobs[blockIdx.x];
  const int L = job.L, K = job.K, tid = threadIdx.x;
  double* A = work_base + job.work_off;
  double* Zt = A + (int64_t)L * L;
  double* d = Zt + (int64_t)L * L;
  double* e = d + L;
  double* tau = e + L;
  double* sel = tau + L;
  double* done = sel + L;
  if (job.only_if_failed && status[job.status_idx] != 1) {  // nothing to redo
    if (tid == 0) *done = 0.0;
    return;
  }
  const double* S = S_base + job.S_off;
  double* v = lds;
  double* w = lds + L;
  double* cs = lds + 2 * L;
  double* sn = lds + 3 * L;

  for (int64_t i = tid; i < (int64_t)L * L; i += kTqThreads) A[i] = S[i];
  __syncthreads();

  // ---- 1. Householder reduction to tridiagonal form
  for (int j = 0; j + 2 < L; ++j) {
    const int m = L - j - 1;  // length of the column below the diagonal
    double* row = A + (int64_t)j * L + j + 1;  // = that column, by symmetry
    double part = 0.0;
    for (int k = 1 + tid; k < m; k += kTqThreads) part = fma(row[k], row[k], part);
    const double sigma = block_sum(part, sh.red);
    const double alpha = row[0];
    if (tid == 0) {
      double t = 0.0, v0 = 1.0, beta = alpha;
      if (sigma > 0.0) {
        const double mu = sqrt(alpha * alpha + sigma);
        v0 = alpha <= 0.0 ? alpha - mu : -sigma / (alpha + mu);
        t = 2.0 * v0 * v0 / (sigma + v0 * v0);
        beta = mu;
      }
      d[j] = A[(int64_t)j * L + j];
      e[j] = beta;
      tau[j] = t;
      sh.scal[0] = t;
      sh.scal[1] = 1.0 / v0;
    }
    __syncthreads();
    const double t = sh.scal[0];
    if (t == 0.0) {
      if (tid == 0) row[0] = 1.0;  // H_j = I; the stored vector is never used
      __syncthreads();
      continue;
    }
    const double inv = sh.scal[1];
    for (int k = tid; k < m; k += kTqThreads) {
      const double vk = k == 0 ? 1.0 : row[k] * inv;
      v[k] = vk;
    }
    __syncthreads();
    for (int k = tid; k < m; k += kTqThreads) row[k] = v[k];  // kept for the back-transform
    // p = tau * A' v over the trailing block A' (rows/columns j+1 ..), column
    // by column through the symmetric rows, which keeps the loads coalesced
    double* Ap = A + (int64_t)(j + 1) * L + (j + 1);
    for (int i = tid; i < m; i += kTqThreads) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int k = 0;
      for (; k + 4 <= m; k += 4) {
        s0 = fma(Ap[(int64_t)k * L + i], v[k], s0);
        s1 = fma(Ap[(int64_t)(k + 1) * L + i], v[k + 1], s1);
        s2 = fma(Ap[(int64_t)(k + 2) * L + i], v[k + 2], s2);
        s3 = fma(Ap[(int64_t)(k + 3) * L + i], v[k + 3], s3);
      }
      for (; k < m; ++k) s0 = fma(Ap[(int64_t)k * L + i], v[k], s0);
      w[i] = t * ((s0 + s1) + (s2 + s3));
    }
    __syncthreads();
    double pv = 0.0;
    for (int k = tid; k < m; k += kTqThreads) pv = fma(w[k], v[k], pv);
    const double half = 0.5 * t * block_sum(pv, sh.red);
    for (int k = tid; k < m; k += kTqThreads) w[k] = w[k] - half * v[k];
    __syncthreads();
    // A' -= v w^T + w v^T, thread by column: eight rows of its column are
    // loaded together (a row-by-row loop waited one memory latency per row)
    for (int i = tid; i < m; i += kTqThreads) {
      const double wi = w[i], vi = v[i];
      double* col = Ap + i;
      int k = 0;
      for (; k + 8 <= m; k += 8) {
        double a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = col[(int64_t)(k + u) * L];
#pragma unroll
        for (int u = 0; u < 8; ++u) col[(int64_t)(k + u) * L] = a[u] - v[k + u] * wi - w[k + u] * vi;
      }
      for (; k < m; ++k) col[(int64_t)k * L] = col[(int64_t)k * L] - v[k] * wi - w[k] * vi;
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (L >= 2) {
      d[L - 2] = A[(int64_t)(L - 2) * L + (L - 2)];
      e[L - 2] = A[(int64_t)(L - 2) * L + (L - 1)];
    }
    d[L - 1] = A[(int64_t)(L - 1) * L + (L - 1)];
    e[L - 1] = 0.0;
    sh.flag = 0;
    // deflation threshold relative to the matrix norm (max_i |d_i| + |e_i|):
    // a test relative to the two neighbouring diagonal entries stalls when
    // small eigenvalues sit beside large ones (rounding leaves off-diagonal
    // entries of order eps ||S||)
    double tst = 0.0;
    for (int i = 0; i < L; ++i) tst = fmax(tst, fabs(d[i]) + fabs(e[i]));
    sh.scal[3] = tst;
  }
  __syncthreads();
  int bad = 0;
  if (L >= kInvItMinL) {
    // ---- 2'. bisection for the K largest eigenvalues, inverse iteration for
    // their vectors (rows 0 .. K-1 of Zt, largest first; sel[c] = c)
    double* dl = lds;
    double* el = lds + L;
    double* e2 = lds + 2 * L;
    for (int i = tid; i < L; i += kTqThreads) {
      dl[i] = d[i];
      el[i] = e[i];
      e2[i] = e[i] * e[i];
    }
    __syncthreads();
    if (tid == 0) {
      double tn = 0.0, lo = 0.0, hi = 0.0, emax = 0.0;
      for (int i = 0; i < L; ++i) {
        const double r = fabs(el[i]) + (i ? fabs(el[i - 1]) : 0.0);
        tn = fmax(tn, fabs(dl[i]) + r);
        lo = i ? fmin(lo, dl[i] - r) : dl[i] - r;
        hi = i ? fmax(hi, dl[i] + r) : dl[i] + r;
        if (i + 1 < L) emax = fmax(emax, e2[i]);
      }
      if (!(tn > 0.0)) tn = 1.0;  // the zero matrix: any orthonormal basis
      sh.scal[0] = lo - 2.0 * kEps * tn - kSafMin;
      sh.scal[1] = hi + 2.0 * kEps * tn + kSafMin;
      sh.scal[2] = kSafMin * fmax(1.0, emax);
      sh.scal[3] = tn;
    }
    __syncthreads();
    const double lo = sh.scal[0], hi = sh.scal[1], pivmin = sh.scal[2], tn = sh.scal[3];
    for (int t = tid; t < K; t += kTqThreads) {
      const double lam = bisect_eig(dl, e2, L, L - 1 - t, lo, hi, pivmin);
      d[t] = lam;  // d now holds the selected eigenvalues, largest first
      sel[t] = (double)t;
      bad |= !isfinite(lam);
    }
    // inverse iteration, one thread per vector (scratch slots of 6 L doubles);
    // every vector comes out with a residual of order eps ||T||, and close
    // eigenvalues only cost orthogonality, which the block restores below
    const int slots = invit_slots(L);
    double* scr = work_base + job.work_off + eig_full_base_elems(L) + (int64_t)tid * 6 * L;
    const double tiny = kEps * tn;
    for (int t = tid; t < K && tid < slots; t += slots) {
      double* u0 = scr;
      double* u1 = u0 + L;
      double* u2 = u1 + L;
      double* mm = u2 + L;
      double* pv = mm + L;
      double* y = pv + L;
      double* x = Zt + (int64_t)t * L;
      tri_lu(dl, el, L, d[t], tiny, u0, u1, u2, mm, pv);
      // deterministic start vector with entries in [0.5, 1.5)
      for (int i = 0; i < L; ++i)
        x[i] = 0.5 + (double)(((uint64_t)i * 2654435761u + (uint64_t)t * 97u) % 1000u) * 1e-3;
      for (int it = 0; it < kInvItIters; ++it) {
        double nrm = 0.0;
        for (int i = 0; i < L; ++i) nrm = fma(x[i], x[i], nrm);
        const double inv = 1.0 / sqrt(nrm);
        for (int i = 0; i < L; ++i) y[i] = x[i] * inv;
        tri_solve(L, u0, u1, u2, mm, pv, y, x);
      }
    }
    __syncthreads();
    // modified Gram-Schmidt over the K vectors, largest eigenvalue first, twice
    // (the second pass makes exactly repeated eigenvalues orthonormal to
    // rounding): step t removes x_t's direction from every later vector, the
    // four waves taking the later vectors in turn, lanes across the entries
    const int lane = tid & 63, wave = tid >> 6;
    for (int pass = 0; pass < 2; ++pass) {
      for (int t = 0; t < K; ++t) {
        const double* xt = Zt + (int64_t)t * L;
        double nt = 0.0;
        for (int i = lane; i < L; i += 64) nt = fma(xt[i], xt[i], nt);
        nt = wave_sum(nt);
        if (nt > 0.0) {
          for (int u = t + 1 + wave; u < K; u += kTqThreads / 64) {
            double* xu = Zt + (int64_t)u * L;
            double dot = 0.0;
            for (int i = lane; i < L; i += 64) dot = fma(xu[i], xt[i], dot);
            const double cf = wave_sum(dot) / nt;
            for (int i = lane; i < L; i += 64) xu[i] = fma(-cf, xt[i], xu[i]);
          }
        }
        __syncthreads();  // x_{t+1} is final before step t + 1 reads it
      }
    }
    for (int t = wave; t < K; t += kTqThreads / 64) {
      double* x = Zt + (int64_t)t * L;
      double nrm = 0.0;
      for (int i = lane; i < L; i += 64) nrm = fma(x[i], x[i], nrm);
      nrm = wave_sum(nrm);
      bad |= !(nrm > 0.0) || !isfinite(nrm);
      const double inv = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
      for (int i = lane; i < L; i += 64) x[i] *= inv;
    }
  } else {
  for (int64_t i = tid; i < (int64_t)L * L; i += kTqThreads)
    Zt[i] = (i / L == i % L) ? 1.0 : 0.0;
  __syncthreads();

  // ---- 2. implicit QL with Wilkinson shifts; Z accumulates the rotations.
  // The tridiagonal matrix moves to LDS (the reflector buffers v and w are
  // free now): one thread chases the bulge through it, so its every access is
  // on that thread's critical path.
  double* dl = lds;
  double* el = lds + L;
  for (int i = tid; i < L; i += kTqThreads) {
    dl[i] = d[i];
    el[i] = e[i];
  }
  __syncthreads();
  const double thresh = 2.220446049250313e-16 * sh.scal[3];
  for (int l = 0; l < L; ++l) {
    for (int sweep = 0;; ++sweep) {
      // m: the first index >= l whose off-diagonal entry is negligible (L - 1
      // if none), searched by the whole block
      int mloc = L - 1;
      for (int i = l + tid; i < L - 1; i += kTqThreads)
        if (fabs(el[i]) <= thresh) {
          mloc = i;
          break;
        }
      const int m = block_min(mloc, sh.redi);
      if (m == l) break;  // converged (uniform over the block)
      if (tid == 0) {
        int lo = m;  // lowest rotated index
        if (sweep >= kQlMaxSweeps) {
          sh.flag = 1;
        } else {
          double g = (dl[l + 1] - dl[l]) / (2.0 * el[l]);
          double r = hypot(g, 1.0);
          g = dl[m] - dl[l] + el[l] / (g + copysign(r, g));
          double s = 1.0, c = 1.0, p = 0.0;
          bool split = false;
          for (int i = m - 1; i >= l; --i) {
            const double f = s * el[i];
            const double b = c * el[i];
            r = hypot(f, g);
            el[i + 1] = r;
            if (r == 0.0) {  // underflow: the matrix splits here, restart
              dl[i + 1] -= p;
              el[m] = 0.0;
              split = true;
              break;
            }
            s = f / r;
            c = g / r;
            g = dl[i + 1] - p;
            r = (dl[i] - g) * s + 2.0 * c * b;
            p = s * r;
            dl[i + 1] = g + p;
            g = c * r - b;
            cs[i] = c;
            sn[i] = s;
            lo = i;
          }
          if (!split) {
            dl[l] -= p;
            el[l] = g;
            el[m] = 0.0;
          }
        }
        sh.lo = lo;
      }
      __syncthreads();
      if (sh.flag) break;
      const int lo = sh.lo;
      // columns lo .. m of Z: rotation i mixes columns i and i+1, applied for
      // i = m-1 down to lo; each thread carries column i+1 of its rows.  Rows
      // of Zt are read eight rotations ahead (independent loads in flight
      // together; a batch never reads a row it or a later batch writes).
      if (lo < m) {
        for (int r = tid; r < L; r += kTqThreads) {
          double znext = Zt[(int64_t)m * L + r];
          int i = m - 1;
          for (; i - 7 >= lo; i -= 8) {
            double z[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) z[u] = Zt[(int64_t)(i - u) * L + r];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const double c = cs[i - u], s = sn[i - u];
              Zt[(int64_t)(i - u + 1) * L + r] = s * z[u] + c * znext;
              znext = c * z[u] - s * znext;
            }
          }
          for (; i >= lo; --i) {
            const double zi = Zt[(int64_t)i * L + r];
            const double c = cs[i], s = sn[i];
            Zt[(int64_t)(i + 1) * L + r] = s * zi + c * znext;
            znext = c * zi - s * znext;
          }
          Zt[(int64_t)lo * L + r] = znext;
        }
      }
      __syncthreads();
    }
    if (sh.flag) break;
  }
  for (int i = tid; i < L; i += kTqThreads) d[i] = dl[i];
  __syncthreads();

  // ---- 3. the K largest eigenvalues, descending (lower index first on ties)
  for (int j = tid; j < L; j += kTqThreads) {
    const double dj = d[j];
    bad |= !isfinite(dj);
    int rank = 0;
    for (int i = 0; i < L; ++i) {
      const double di = d[i];
      rank += (di > dj) || (di == dj && i < j);
    }
    if (rank < K) sel[rank] = (double)j;
  }
  }  // QL path
  bad = __syncthreads_or(bad);
  __syncthreads();
  double* ev = ev_base + job.ev_off;
  for (int c = tid; c < K; c += kTqThreads) ev[c] = d[(int)sel[c]];
  if (tid == 0) {
    status[job.status_idx] = bad ? 2 : (sh.flag ? 1 : 0);
    *done = (bad || sh.flag) ? 0.0 : 1.0;
  }
}

// Back-transformation of VB selected columns per block: Y = Q Z[:, sel], then
// the sign rule, written to F (L x K row-major).
__global__ __launch_bounds__(kFullThreads) void eig_full_backtransform(
    const EigFullJob* __restrict__ jobs, double* __restrict__ F_base,
    const double* __restrict__ work_base, int VB) {
  extern __shared__ double lds[];
  const EigFullJob job = jobs[blockIdx.x];
  const int L = job.L, K = job.K, tid = threadIdx.x;
  const int c0 = blockIdx.y * VB;
  if (c0 >= K) return;
  const int nc = min(VB, K - c0);
  const double* A = work_base + job.work_off;
  const double* Zt = A + (int64_t)L * L;
  const double* tau = Zt + (int64_t)L * L + 2 * L;
  const double* sel = tau + L;
  if (sel[L] != 1.0) return;  // not solved in this launch
  double* Y = lds;             // L x VB
  double* v = lds + L * VB;    // L
  double* red = v + L;         // kFullThreads
  int* redi = reinterpret_cast<int*>(red + kFullThreads);  // kFullThreads
  for (int e = tid; e < L * VB; e += kFullThreads) {
    const int pos = e / VB, c = e % VB;
    Y[e] = c < nc ? Zt[(int64_t)(int)sel[c0 + c] * L + pos] : 0.0;
  }
  __syncthreads();
  const int nparts = kFullThreads / VB;
  const int cc = tid % VB, part = tid / VB;
  for (int j = L - 3; j >= 0; --j) {
    const double t = tau[j];
    if (t == 0.0) continue;
    const int b = j + 1, m = L - b;
    const double* row = A + (int64_t)j * L + b;
    for (int k = tid; k < m; k += kFullThreads) v[b + k] = row[k];
    __syncthreads();
    double s = 0.0;
    for (int pos = b + part; pos < L; pos += nparts) s = fma(v[pos], Y[pos * VB + cc], s);
    red[tid] = s;
    __syncthreads();
    // thread c < VB sums the parts of column c (entries c, VB + c, ...) and
    // leaves tau * (v^T y_c) in red[c], an entry only it reads
    if (tid < VB) {
      double acc = 0.0;
      for (int q = 0; q < nparts; ++q) acc += red[q * VB + tid];
      red[tid] = t * acc;
    }
    __syncthreads();
    for (int e = tid; e < m * VB; e += kFullThreads) {
      const int pos = b + e / VB, c = e % VB;
      Y[pos * VB + c] -= v[pos] * red[c];
    }
    __syncthreads();
  }
  // sign rule per column
  double best = -1.0;
  int bi = 0x7fffffff;
  for (int pos = part; pos < L; pos += nparts) {
    const double a = fabs(Y[pos * VB + cc]);
    if (a > best || (a == best && pos < bi)) {
      best = a;
      bi = pos;
    }
  }
  red[tid] = best;
  redi[tid] = bi;
  __syncthreads();
  if (tid < VB) {
    double b0 = red[tid];
    int i0 = redi[tid];
    for (int q = 1; q < nparts; ++q) {
      const double ob = red[q * VB + tid];
      const int oi = redi[q * VB + tid];
      if (ob > b0 || (ob == b0 && oi < i0)) {
        b0 = ob;
        i0 = oi;
      }
    }
    red[tid] = Y[i0 * VB + tid] < 0.0 ? -1.0 : 1.0;
  }
  __syncthreads();
  double* F = F_base + job.F_off;
  for (int e = tid; e < L * VB; e += kFullThreads) {
    const int pos = e / VB, c = e % VB;
    if (c < nc) F[(int64_t)pos * K + c0 + c] = red[c] * Y[e];
  }
}

namespace {

int full_vb(int Lmax) {
  // Y (L x VB) + v (L) + the reductions (1.5 kFullThreads) in at most 144 KB
  const int budget = 144 * 1024 / 8 - 2 * kFullThreads - Lmax;
  int vb = 32;
  while (vb > 1 && vb * Lmax > budget) vb /= 2;
  return vb;
}

bool g_full_attr = false;

hipError_t full_attrs() {
  if (g_full_attr) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void*)eig_full_tridiag_ql,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     4 * kFullMaxL * (int)sizeof(double));
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)eig_full_backtransform,
                            hipFuncAttributeMaxDynamicSharedMemorySize, 144 * 1024);
  if (e == hipSuccess) g_full_attr = true;
  return e;
}

}  // namespace

int eig_full_max_L() { return kFullMaxL; }

size_t eig_full_work_elems(int L) {
  return (size_t)eig_full_base_elems(L) +
         (L >= kInvItMinL ? (size_t)6 * L * (size_t)invit_slots(L) : 0);
}

hipError_t launch_eig_full(int count, const EigFullJob* jobs_dev, int Lmax, int Kmax,
                           const double* S_base, double* F_base, double* ev_base,
                           double* work_base, int* status, hipStream_t st) {
  if (count == 0) return hipSuccess;
  if (Lmax < 1 || Lmax > kFullMaxL || Kmax < 1) return hipErrorInvalidValue;
  hipError_t e = full_attrs();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(eig_full_tridiag_ql, dim3(count), dim3(kTqThreads),
                     4 * (size_t)Lmax * sizeof(double), st, jobs_dev, S_base, ev_base, work_base,
                     status);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int vb = full_vb(Lmax);
  const size_t lds = sizeof(double) * ((size_t)Lmax * vb + Lmax + 2 * kFullThreads);
  hipLaunchKernelGGL(eig_full_backtransform, dim3(count, (Kmax + vb - 1) / vb),
                     dim3(kFullThreads), lds, st, jobs_dev, F_base, work_base, vb);
  return hipGetLastError();
}

}  // namespace tk
