// Host-side launchers of the device kernels (all enqueue on `st`).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>
#include <stddef.h>
#include <stdint.h>

namespace tk {

// TTM node: Out[a,k,b] = sum_l F[l,k] In[a,l,b]  (ttm.hip)
// stream_in: the input is read once (streamed past the caches)
// tile: TK_TILE_* kernel choice (FP64 compute ignores it).  out_dtype: TK_F32
// (TK_F64 for FP64 compute), or TK_BF16 for TK_C_BF16 nodes for which
// ttm_bf16_output_ok() holds (the node runs a BF16 kernel).
hipError_t launch_ttm(int in_dtype, int compute, const void* in, int64_t A, int64_t L, int64_t B,
                      const void* F, int64_t K, void* out, hipStream_t st,
                      bool stream_in = false, int tile = 0, int out_dtype = TK_F32);
bool ttm_bf16_output_ok(int in_dtype, int compute, const void* in, int64_t A, int64_t L,
                        int64_t B, const void* out, int tile);
int ttm_max_L();

// Both root TTMs in one pass (ttm2.hip): In viewed as [A, Lp, M, Lq, B],
// Outp = In x_p Fp^T ([A, Kp, M, Lq, B]) and Outq = In x_q Fq^T ([A, Lp, M, Kq, B]).
// FP32 input and compute; applies when ttm_pair_applies() holds.
bool ttm_pair_applies(int in_dtype, int compute, const void* in, int64_t A, int64_t Lp,
                      int64_t M, int64_t Lq, int64_t B, int64_t Kp, int64_t Kq,
                      const void* outp, const void* outq);
// 0: no pair kernel; 1: the general one (lanes over Lq rows, B % 4 == 0);
// 2: the trailing-modes one (M = B = 1, slabs staged in LDS); 3: the
// trailing-modes one for large slabs (M = B = 1, Lq % 4 == 0, Lq <= 256,
// ranks <= 20; slabs streamed through LDS in row chunks).
int ttm_pair_kind(int in_dtype, int compute, const void* in, int64_t A, int64_t Lp, int64_t M,
                  int64_t Lq, int64_t B, int64_t Kp, int64_t Kq, const void* outp,
                  const void* outq);
hipError_t launch_ttm_pair(const float* in, int64_t A, int64_t Lp, int64_t M, int64_t Lq,
                           int64_t B, const float* Fp, int64_t Kp, const float* Fq, int64_t Kq,
                           float* outp, float* outq, hipStream_t st);

// Grouped TTM (batched HOOI): one descriptor per node, FP32 factor and output.
enum {
  kGroupedTile = 0,
  kGroupedWide = 1,
  kGroupedRows = 2,        // B == 1 through LDS, 16-byte loads (L % 4 == 0,
                           // L <= ttm_grouped_row_stage_max_L())
  kGroupedRowsDirect = 3,  // B == 1, direct 16-byte row loads (L % 4 == 0)
  kGroupedRowsScalar = 4,  // B == 1 through LDS, one element per load
                           // (L <= ttm_grouped_row_stage_max_L())
  kGroupedWideScalar = 5   // B >= 32 not readable 16 bytes at a time: 4-byte loads
};
struct TtmNodeDesc {
  const void* in;
  float* out;
  const float* F;  // L x K row-major
  int64_t A, B, nbt;
  int L, K, na, nb;
  int path;   // kGrouped*: the tile body the node's items run
  int lines;  // 1: every run the body reads is whole 128-byte lines (B, or L for
              // rows, times the element size), so streaming loads fetch no
              // line twice; 0: normal loads even for an input read once
};
// Kernel body and item count of a node viewed as [A, L, B] (in_bytes: input
// element size): the wide body (B % 4 == 0, B >= 16, aligned), the LDS row
// body (B == 1, L % 4 == 0; through LDS for L <= 64, direct 16-byte row loads
// above), else the LDS-staged tile body.
void ttm_grouped_geometry(const void* in, const float* out, int in_bytes, int64_t A, int64_t L,
                          int64_t B, TtmNodeDesc* d, int64_t* tiles);
// Dynamic LDS of the grouped kernel for nodes with L <= Lmax.
size_t ttm_grouped_lds(int Lmax);
// Longest rows the grouped kernel stages through LDS.
int ttm_grouped_row_stage_max_L();
// items: (node, tile) pairs, node an index into `nodes` (the whole table);
// counter: zeroed device int (the queue head);
// grid: persistent blocks.  Every node has K <= 16 and L <= Lmax; in_dtype
// TK_F32 or TK_BF16 for all nodes of the launch.
// stream_in: the inputs are read once (non-temporal loads).
hipError_t launch_ttm_grouped(int in_dtype, const TtmNodeDesc* nodes, const int2* items,
                              int n_items, int* counter, int Lmax, int grid, bool stream_in,
                              hipStream_t st);

// The same queue for kGroupedRowsScalar nodes only, with the barrier-free
// single-element row body (a kernel of its own: its registers would lower the
// occupancy of the other bodies).  LDS: ttm_grouped_rows_lds(Lmax).
size_t ttm_grouped_rows_lds(int Lmax);
hipError_t launch_ttm_grouped_rows(int in_dtype, const TtmNodeDesc* nodes, const int2* items,
                                   int n_items, int* counter, int Lmax, int grid, bool stream_in,
                                   hipStream_t st);

// Gram S = Y_(n) Y_(n)^T (gram.hip); `part` holds gram_workspace_elems(L, A*B) doubles
hipError_t launch_gram(int in_dtype, const void* Y, int64_t A, int64_t L, int64_t B, double* S,
                       double* part, hipStream_t st);
size_t gram_workspace_elems(int64_t L, int64_t C);

// Grouped Gram (batched HOOI): one descriptor per matrix; Y viewed as
// [C / B, L, B] (F32 or BF16), partial sums in `part` (nchunks * npairs
// 64 x 64 blocks), result S (L x L).
struct GramDesc {
  const void* Y;
  double* S;
  double* part;
  int64_t B, C, cchunk;
  int L, T, npairs, nchunks;
};
// Fills L, C, T, npairs, cchunk, nchunks; target_blocks > 0 sets the number
// of blocks per matrix the column chunks aim for.
void gram_geometry(int64_t L, int64_t C, int64_t target_blocks, GramDesc* d);
// items: (matrix, chunk, pair, 0); elem_off: n_mats + 1 prefix sums of L_m^2.
hipError_t launch_gram_grouped(int in_dtype, const GramDesc* mats, const int4* items,
                               int n_items, const int64_t* elem_off, int n_mats,
                               int64_t total_elems, hipStream_t st);

// Leading eigenpairs (eig.hip).  One job per matrix: S (L x L) at S_base + S_off,
// optional warm start V0 (L x K) at V0_base + V0_off (V0_off < 0: cold start),
// output F (L x K) and eigenvalues (K), and 2 * L * p doubles of work.
struct EigJob {
  int L, K, p, pad_;
  int64_t S_off, V0_off, F_off, ev_off, work_off;
  // p = L only: the full eigenbasis (L x L row-major) at basis_base +
  // basis_off, or -1.  A warm solve starts from it (re-orthonormalised) and
  // every solve writes its final basis back; any orthonormal basis is a valid
  // start, so callers initialise it to the identity.
  int64_t basis_off = -1;
};
// Jobs [job0, job0 + count) of the device table; Lmax / pmax bound their L and p.
// Every job of the launch uses the block width padded(pmax): its work area
// must hold eig_work_elems(L_job, pmax) doubles (not its own p's).
// status[job] is set on failure only (1: no convergence, 2: non-finite);
// iters (nullable) receives the subspace steps each job used.
hipError_t launch_eig(int count, const EigJob* jobs_dev, int job0, int Lmax, int pmax,
                      const double* S_base, const double* V0_base, double* F_base,
                      double* ev_base, double* work_base, int* status, int* iters, int maxit,
                      double tol, hipStream_t st, double* basis_base = nullptr);
// Identity bases for the p = L jobs of a table (host-built, uploaded by the caller).
void eig_identity_bases(const std::vector<EigJob>& jobs, std::vector<double>* out);
int eig_block_size(int L, int K, int64_t rank_bound);
size_t eig_work_elems(int L, int p);  // global work doubles one job may need
int eig_max_K();

// Gap-free leading eigenpairs (eigfull.hip): Householder tridiagonalisation,
// implicit QL with eigenvector accumulation, back-transformation of the K
// largest, sign rule.  One job per matrix; status[status_idx] receives 0
// (solved), 1 (QL did not converge) or 2 (non-finite); with only_if_failed
// the job runs only when that word is 1 on entry (a subspace solve before it
// failed) and otherwise leaves F and ev untouched.  Work: eig_full_work_elems(L)
// doubles per job at work_base + work_off.  L <= eig_full_max_L().
struct EigFullJob {
  int L, K, status_idx, only_if_failed;
  int64_t S_off, F_off, ev_off, work_off;
};
hipError_t launch_eig_full(int count, const EigFullJob* jobs_dev, int Lmax, int Kmax,
                           const double* S_base, double* F_base, double* ev_base,
                           double* work_base, int* status, hipStream_t st);
size_t eig_full_work_elems(int L);
int eig_full_max_L();

// misc.hip
hipError_t launch_sumsq(int dtype, const void* x, int64_t n, double* part, double* out,
                        hipStream_t st);
int sumsq_partials();
hipError_t launch_convert(int from, int to, const void* a, void* b, int64_t n, hipStream_t st);
hipError_t launch_fill(double* a, int64_t n, double v, hipStream_t st);
hipError_t launch_fill_int(int* a, int64_t n, int v, hipStream_t st);
hipError_t launch_copy_f64(const double* a, double* b, int64_t n, hipStream_t st);  // kernel copy
// out[s] = sum of squares of x[off[s] .. off[s+1]) for s < count (one block each)
hipError_t launch_sumsq_segments(const float* x, const int64_t* off, int count, double* out,
                                 hipStream_t st);
hipError_t launch_residual(int dtype, const void* Tt, const double* Zp, const double* F0, int L0,
                           int K0, int64_t R, double* part, double* out, hipStream_t st);

}  // namespace tk
