// Host-side launchers of the device kernels (all enqueue on `st`).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace tk {

// TTM node: Out[a,k,b] = sum_l F[l,k] In[a,l,b]  (ttm.hip)
// stream_in: the input is read once (streamed past the caches)
// tile: TK_TILE_* kernel choice (FP64 compute ignores it)
hipError_t launch_ttm(int in_dtype, int compute, const void* in, int64_t A, int64_t L, int64_t B,
                      const void* F, int64_t K, void* out, hipStream_t st,
                      bool stream_in = false, int tile = 0);
int ttm_max_L();

// Gram S = Y_(n) Y_(n)^T (gram.hip); `part` holds gram_workspace_elems(L, A*B) doubles
hipError_t launch_gram(int in_dtype, const void* Y, int64_t A, int64_t L, int64_t B, double* S,
                       double* part, hipStream_t st);
size_t gram_workspace_elems(int64_t L, int64_t C);

// Leading eigenpairs (eig.hip).  One job per matrix: S (L x L) at S_base + S_off,
// optional warm start V0 (L x K) at V0_base + V0_off (V0_off < 0: cold start),
// output F (L x K) and eigenvalues (K), and 2 * L * p doubles of work.
struct EigJob {
  int L, K, p, pad_;
  int64_t S_off, V0_off, F_off, ev_off, work_off;
};
// Jobs [job0, job0 + count) of the device table; Lmax / pmax bound their L and p.
// Every job of the launch uses the block width padded(pmax): its work area
// must hold eig_work_elems(L_job, pmax) doubles (not its own p's).
// status[job] is set on failure only (1: no convergence, 2: non-finite);
// iters (nullable) receives the subspace steps each job used.
hipError_t launch_eig(int count, const EigJob* jobs_dev, int job0, int Lmax, int pmax,
                      const double* S_base, const double* V0_base, double* F_base,
                      double* ev_base, double* work_base, int* status, int* iters, int maxit,
                      double tol, hipStream_t st);
int eig_block_size(int L, int K, int64_t rank_bound);
size_t eig_work_elems(int L, int p);  // global work doubles one job may need
int eig_max_K();

// misc.hip
hipError_t launch_sumsq(int dtype, const void* x, int64_t n, double* part, double* out,
                        hipStream_t st);
int sumsq_partials();
hipError_t launch_convert(int from, int to, const void* a, void* b, int64_t n, hipStream_t st);
hipError_t launch_fill(double* a, int64_t n, double v, hipStream_t st);
hipError_t launch_fill_int(int* a, int64_t n, int v, hipStream_t st);
hipError_t launch_residual(int dtype, const void* Tt, const double* Zp, const double* F0, int L0,
                           int K0, int64_t R, double* part, double* out, hipStream_t st);

}  // namespace tk
