/*
 * tucker.h -- C ABI of the MI355X dense Tucker / HOOI library (libtucker.so).
 *
 * The library computes the TTM component of HOOI (Chakaravarthy et al.,
 * "On Optimizing Distributed Tucker Decomposition for Dense Tensors",
 * arXiv 1707.05594) on one AMD Instinct MI355X (gfx950):
 *
 *   for every mode n:  Y_n = T x_{m != n} F_m^T  through a TTM-tree
 *                      (Sec. 3.1 definition; optimal tree by the dynamic
 *                      program of Sec. 3.3),
 *                      F~_n = leading K_n left singular vectors of Y_(n),
 *                      taken from the Gram matrix Y_(n) Y_(n)^T and an FP64
 *                      eigensolver (Sec. 5, Gram + EVD),
 *   then the new core G~ = T x_1 F~_1^T ... x_N F~_N^T and the error
 *   (Fig. 2, "HOOI Procedure"; Sec. 2.2 error).
 *
 * Conventions
 *   - Modes are 0-based (the paper numbers them from 1).
 *   - Tensors are dense, row-major, last mode fastest.  An N-mode tensor with
 *     lengths L_0..L_{N-1} is a contiguous array of prod(L) elements.
 *   - Factor matrices F_n are L_n x K_n, row-major, FP64 on the host side.
 *   - "Device pointer" means memory from hipMalloc (or a torch CUDA tensor) on
 *     the current HIP device; "host pointer" means ordinary process memory.
 *   - Costs are counted in multiply-adds: the paper's FLOP count of a TTM,
 *     K_n |In(u)| (Sec. 3.1), is one multiply-add per term.
 *   - Every function returns TK_OK (0) or a negative error code; the text of
 *     the last error on the calling thread is returned by tk_last_error().
 *     On error no output argument is written unless stated otherwise.
 *   - All device work is enqueued on the stream given to hooi_init (or to the
 *     kernel-level entry points); functions that return host data
 *     synchronise that stream before returning.
 */
#ifndef TUCKER_H
#define TUCKER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---------------------------------------------------------- */
#define TK_OK 0
#define TK_EINVAL (-1)        /* bad argument: sizes, null pointer, mismatch   */
#define TK_ENOMEM (-2)        /* device or host allocation failed              */
#define TK_EDEVICE (-3)       /* a HIP runtime call or kernel launch failed    */
#define TK_ENUMERIC (-4)      /* NaN/Inf met, or the eigensolver did not converge */
#define TK_EUNSUPPORTED (-5)  /* unsupported storage/compute combination       */

#define TK_MAX_MODES 12       /* the planner is O(4^N) (Sec. 3.3)              */

/* storage type of T (and of kernel-level operands) */
#define TK_F64 0
#define TK_F32 1
#define TK_BF16 2
#define TK_F16 3  /* IEEE half; FP32 compute only (each value exact in FP32) */

/* arithmetic of the TTM and Gram kernels.  The eigensolver, the factor
 * orthonormalisation, norms and the error are FP64 in every mode. */
#define TK_C_FP64 0   /* FP64 operands, FP64 accumulation (T stored F64)          */
#define TK_C_FP32 1   /* FP32 operands on FP32 MFMA, FP32 accumulation            */
#define TK_C_BF16 2   /* BF16 operands on BF16 MFMA, FP32 accumulation            */
#define TK_C_BF16X3 3 /* split BF16: a*b ~ ah*bh + ah*bl + al*bh, FP32 accumulation */

/* TTM kernel choice for one node (FP32 / BF16 / bf16x3 compute):
 * AUTO   -- by shape: the wide path (B % 4 == 0, B >= 16; split over L on
 *           grids smaller than the chip; whole slabs per wave for FP32 runs
 *           that are not whole cache lines), the wide path with 4-byte loads
 *           (B >= 32 otherwise), the short-slab path (L <= 32, K <= 32 and
 *           B = 1 or B below the wide paths: whole slabs per wave through
 *           LDS; long aligned rows with K <= L / 2 keep the row path), the
 *           row path (B == 1), else the LDS-staged tile path; the K-group
 *           count from the factor's LDS footprint and the grid size;
 * STAGED -- always the LDS-staged tile path;
 * SPLITK -- AUTO's path with half the K-groups per block (more blocks, the
 *           input re-read from cache). */
#define TK_TILE_AUTO 0
#define TK_TILE_STAGED 1
#define TK_TILE_SPLITK 2
#define TK_TILE_COUNT 3
/* Root nodes only: the tree's two root children run as one pass over T (a
 * kernel for the two trailing modes of an FP32 tensor reads T once for both);
 * set on both root nodes.  hooi_init falls back to TK_TILE_AUTO when no pair
 * kernel takes the shape.  The plain plan never sets it; tk_plan_learned may. */
#define TK_TILE_PAIR 3

/* tree kinds (Sec. 3.2 prior schemes, Sec. 3.3 optimal tree) */
#define TK_TREE_DP 0        /* minimum multiply-add tree, dynamic program         */
#define TK_TREE_CHAIN 1     /* N independent chains, ascending modes (naive)      */
#define TK_TREE_CHAIN_K 2   /* chains in increasing-K_n mode order                */
#define TK_TREE_CHAIN_H 3   /* chains in increasing h_n = K_n/L_n mode order      */
#define TK_TREE_BALANCED 4  /* divide-and-conquer tree, input mode order          */

typedef struct tk_plan tk_plan; /* host-only, owned by the caller (tk_plan_free) */
typedef struct tk_ctx tk_ctx;   /* device state, owned by the caller (hooi_free) */

/* One node of a TTM-tree, in depth-first execution order (parents first). */
typedef struct {
  int32_t parent;    /* index of the parent node; -1 when the parent is the root T */
  int32_t mode;      /* TTM mode of an internal node, or the factor mode of a leaf */
  int32_t is_leaf;   /* 1 for a leaf F~_n, 0 for an internal (TTM) node           */
  int32_t depth;     /* 0 for children of the root                                */
  uint64_t in_card;  /* |In(u)|: elements of the tensor the node reads            */
  uint64_t out_card; /* |Out(u)| = (K_n/L_n)|In(u)| for internal nodes, 0 for leaves */
  uint64_t macs;     /* K_n |In(u)| for internal nodes, 0 for leaves (Sec. 3.1)   */
  uint32_t pre_mask; /* bit j set: mode j already multiplied in In(u)             */
  uint32_t pad_;
} tk_node;

/* ---- planning (host only; Sec. 3.1 cost, Sec. 3.2 heuristics, Sec. 3.3 DP) -- */

/* Build a TTM-tree plan for lengths L[0..N-1] and core lengths K[0..N-1].
 * kind: TK_TREE_*.  topk >= 1: for TK_TREE_DP the plan keeps the topk cheapest
 * distinct trees (rank 0 = the optimum with the documented tie rule); other
 * kinds hold one tree.
 * Requires 2 <= N <= TK_MAX_MODES, 1 <= K_n <= L_n, K_n <= prod_{m != n} K_m
 * (otherwise Y_(n) cannot have rank K_n), prod(L) < 2^62.  TK_EINVAL otherwise.
 * *out receives a new plan owned by the caller. */
int ttm_tree_plan(int N, const int64_t* L, const int64_t* K, int kind, int topk,
                  tk_plan** out);
int tk_plan_count(const tk_plan* plan, int* count);          /* trees held */
int tk_plan_cost(const tk_plan* plan, int rank, uint64_t* macs);
/* Canonical text: leaf "F<n>", node "m<n>(children)", root "T(children)",
 * children sorted as strings.  Writes at most cap bytes including the NUL;
 * TK_EINVAL if cap is too small. */
int tk_plan_string(const tk_plan* plan, int rank, char* buf, size_t cap);
/* Copies up to cap nodes of tree `rank`; *n receives the node count. */
int tk_plan_nodes(const tk_plan* plan, int rank, tk_node* out, int cap, int* n);
/* DP instrumentation: table entries created and table lookups made. */
int tk_plan_stats(const tk_plan* plan, uint64_t* entries, uint64_t* lookups);
/* Largest per-path sum of live intermediate elements of tree `rank` (the DFS
 * workspace bound of Sec. 3.1: at most depth-many intermediates alive). */
int tk_plan_workspace(const tk_plan* plan, int rank, uint64_t* elements);
/* Choose which held tree (rank) hooi_init executes; default rank 0. */
int tk_plan_select(tk_plan* plan, int rank);
void tk_plan_free(tk_plan* plan);

/* ---- processor grids (host only; Sec. 4) ----------------------------------- */

/* Number of N-dimensional grids of P processors, psi(P, N) =
 * prod_i C(e_i + N - 1, N - 1) for P = prod_i p_i^e_i (Sec. 4.2).  TK_EINVAL
 * for P < 1, N < 1 or a count above 2^64. */
int tk_grid_count(int64_t P, int N, uint64_t* count);

#define TK_GRID_STATIC 0   /* one grid for every tensor of the tree (Sec. 4.2)   */
#define TK_GRID_DYNAMIC 1  /* a grid per node, regridding allowed (Sec. 4.3-4.4) */

/* Processor grids for tree `rank` of `plan` on P processors.  A grid
 * <q_1..q_N> (prod q_n = P) is valid when q_n <= K_n for every mode; a TTM
 * along mode n at node u costs (q_n - 1) |Out(u)| words (Sec. 4.1).
 *   TK_GRID_STATIC:  the valid grid with the least total TTM volume;
 *   TK_GRID_DYNAMIC: the optimal scheme of Sec. 4.4: each node keeps its
 *     parent's grid or redistributes its input (|In(u)| words) to a grid of
 *     its own; T is laid out under a grid of free choice.
 * Ties go to the lexicographically first grid, and to keeping the parent's.
 * Out (host, nullable): root_grid[N] (the grid of T), node_grids[cap x N]
 * (the grid of every node of tk_plan_nodes, in that order; leaves repeat
 * their parent's), *volume (words).  Errors: TK_EINVAL (null plan, bad rank,
 * P < 1, cap below the node count, unknown kind, volume above 2^64),
 * TK_EUNSUPPORTED (no valid grid, or more than 2^22 grids to search). */
int tk_plan_grids(const tk_plan* plan, int rank, int64_t P, int kind, int* root_grid,
                  int* node_grids, int cap, uint64_t* volume);

/* ---- HOOI context ---------------------------------------------------------- */

/* Create a context for HOOI on the tensor T.
 *   T_dev: device pointer, row-major prod(L) elements of type tdtype; borrowed
 *          (never written, never freed) and must outlive the context.
 *   plan : tree to execute (NULL: the DP optimum).  Must have been built for
 *          the same (N, L, K); its selected rank is copied, the plan may be freed.
 *   compute: TK_C_*.  Supported: F64 storage with TK_C_FP64; F32 or BF16
 *          storage with TK_C_FP32, TK_C_BF16, TK_C_BF16X3; F16 storage with
 *          TK_C_FP32 only (every half value is exact in FP32, so the tree
 *          runs the FP32 kernels converting on load; else TK_EUNSUPPORTED).  In the BF16
 *          modes the TTMs that form the core (the tree path to the leaf
 *          that folds it, and the direct core chain) run at FP32: the error
 *          is ||T||^2 - ||G||^2, so ||G||^2 needs more than BF16 accuracy.
 *          Intermediates are stored FP32, except in TK_C_BF16 mode where a
 *          node whose children are all TTMs run by a BF16 kernel stores its
 *          output as BF16 (those children round their input to BF16 anyway);
 *          leaf tensors, which the Grams read, stay FP32.
 *   F0_host: NULL to start from HOSVD (F_n = leading K_n left singular vectors
 *          of T_(n)), or host FP64 factors F_0..F_{N-1} concatenated, each
 *          L_n x K_n row-major (checkpoint / resume).  Copied.
 *   stream: hipStream_t (NULL = default stream) used for all device work.
 * Allocates device workspace sized for the tree (TK_ENOMEM on failure). */
int hooi_init(int N, const int64_t* L, const int64_t* K, int tdtype, const void* T_dev,
              const tk_plan* plan, int compute, const double* F0_host, void* stream,
              tk_ctx** out);

/* As hooi_init, starting from the STHOSVD decomposition (Sec. 1 and
 * Sec. 2.2: the initial decomposition is sequentially truncated HOSVD) instead
 * of HOSVD: the modes are processed in `order` (host array of N distinct
 * modes; NULL = ascending), mode n taking the leading K_n eigenvectors of the
 * Gram of the current tensor's mode-n unfolding (FP64, as hooi_init's) and
 * truncating the tensor along n (TTM at FP64 for FP64 storage, else FP32)
 * before the next mode.  Allocates temporary device memory for the truncated
 * tensors (at most |T| K_n / L_n elements, twice), synchronises the stream,
 * then creates the context exactly as hooi_init with these factors.
 * Errors: those of hooi_init, TK_EINVAL for an order that is not a
 * permutation, TK_ENUMERIC from the eigensolver. */
int hooi_init_sthosvd(int N, const int64_t* L, const int64_t* K, int tdtype, const void* T_dev,
                      const tk_plan* plan, int compute, const int* order, void* stream,
                      tk_ctx** out);

/* Run `iters` >= 1 HOOI invocations (Fig. 2, Jacobi form: every chain uses the
 * factors from the start of the invocation).  rel_err: NULL or a host array of
 * `iters` doubles that receives the relative error after each invocation,
 * sqrt(max(||T||^2 - ||G~||^2, 0)) / ||T||.  Each invocation's new core is
 * computed by folding it into the next tree pass (G = Y_n x_n F_n^T); the
 * last one by a direct TTM chain.  Synchronises the stream before returning. */
int hooi_iterate(tk_ctx* ctx, int iters, double* rel_err);

/* Error of the current decomposition: *rel_err as above, *normT = ||T||_F,
 * *normG = ||G||_F (any output may be NULL). */
int tucker_error(tk_ctx* ctx, double* rel_err, double* normT, double* normG);

/* Explicit residual ||T - G x_1 F_1 ... x_N F_N||_F / ||T||_F, accumulated in
 * FP64 on the device without forming the recovered tensor. */
int tucker_error_explicit(tk_ctx* ctx, double* rel_err);

/* Copy out the current FP64 factor F_n (L_n x K_n row-major) / core
 * (prod(K) row-major) to host memory. */
int tk_get_factor(tk_ctx* ctx, int n, double* host);
int tk_get_core(tk_ctx* ctx, double* host);
/* Replace every factor by host FP64 factors (same layout as F0_host). */
int tk_set_factors(tk_ctx* ctx, const double* host);

/* One tree pass with the current factors, no factor update: fills the leaf
 * tensors Y_n and Gram matrices S_n.  Then tk_get_leaf copies Y_n (row-major,
 * lengths K_m for m != n and L_n at mode n, FP64-converted) and tk_get_gram
 * copies S_n (L_n x L_n FP64) to host memory.  Test and inspection aids. */
int tk_tree_pass(tk_ctx* ctx);
int tk_get_leaf(tk_ctx* ctx, int n, double* host);
int tk_get_gram(tk_ctx* ctx, int n, double* host);

/* Per-node device time (ms, HIP events) of one tree pass with the current
 * factors; ms_out has one entry per plan node (leaves: Gram time). */
int tk_profile_tree(tk_ctx* ctx, float* ms_out, int cap, int* n);

/* Subspace steps the FP64 eigensolver used for each mode in the most recent
 * factor update (out: N ints, host).  Observability aid. */
int tk_eig_iterations(tk_ctx* ctx, int* out);

void hooi_free(tk_ctx* ctx);

/* ---- batched HOOI over many independent tensors ---------------------------- */

/* One HOOI invocation (Sec. 2.2, Jacobi form) for `count` tensors at a time,
 * each with its own minimum-cost TTM-tree (Sec. 3.3).  Tree nodes of all
 * tensors are grouped by depth; each depth is one launch of a persistent
 * grouped TTM kernel draining a device queue of (node, tile) items; the
 * leaves' Grams, the eigensolves, the folded cores and their norms are one
 * launch each.  An iteration is captured in a HIP graph and replayed.
 *   N[i]: modes of tensor i; L, K: the lengths concatenated over tensors
 *   (sum of N[i] entries each), 1 <= K <= min(L, 16), L <= 512.
 *   T_dev[i]: device pointer to tensor i (row-major, tdtype TK_F32 or
 *   TK_BF16), borrowed.  compute: TK_C_FP32.  stream: caller's stream,
 *   ordered before and after every call by events.
 * Starts from HOSVD (FP64 eigensolver).  Errors TK_EINVAL, TK_EUNSUPPORTED,
 * TK_ENOMEM, TK_EDEVICE, TK_ENUMERIC (eigensolver failure). */
typedef struct tk_batch tk_batch;
int hooi_batch_init(int count, const int* N, const int64_t* L, const int64_t* K, int tdtype,
                    const void* const* T_dev, int compute, void* stream, tk_batch** out);
/* rel_err: NULL or iters x count doubles; entry (t, i) is the error of tensor
 * i's decomposition entering invocation t (t = 0: the HOSVD start).  After
 * the call the factors are those of invocation iters - 1's output. */
int hooi_batch_iterate(tk_batch* b, int iters, double* rel_err);
/* Error of every tensor's current decomposition (count doubles). */
int hooi_batch_error(tk_batch* b, double* rel_err);
/* FP64 factor F_n of tensor i (L_n x K_n row-major), or all factors
 * concatenated (tensor by tensor, mode by mode). */
int hooi_batch_get_factor(tk_batch* b, int i, int n, double* host);
int hooi_batch_get_factors(tk_batch* b, double* host);
/* Replace every factor (layout as hooi_batch_get_factors; host FP64, copied;
 * TK_ENUMERIC on NaN/Inf).  Solves with p = L (L <= 64) keep their full
 * eigenbasis from one invocation to the next as a warm start; setting the
 * factors resets those bases to the identity, so a resumed batch matches an
 * uninterrupted one to rounding, not bitwise. */
int hooi_batch_set_factors(tk_batch* b, const double* host);
/* on = 0: enqueue every iteration eagerly instead of replaying the graph. */
int hooi_batch_use_graph(tk_batch* b, int on);
/* Autotuner: times a tree pass with 1, 2, 3 and 4 persistent blocks per CU
 * and keeps the fastest; then, at that grid, times the other body for the
 * odd-length row nodes (their own persistent launch with the barrier-free
 * row body, or the shared queue's row body) and keeps the faster; finally
 * re-captures the graph.  ms: NULL or 5 floats (ms per pass: the four grids,
 * then the other row body). */
int hooi_batch_tune(tk_batch* b, int* blocks_per_cu, float* ms);
/* Multiply-adds and algorithmic bytes (inputs read once, outputs written
 * once) of all tree nodes, tree levels and TTM work items. */
int hooi_batch_stats(const tk_batch* b, uint64_t* tree_macs, uint64_t* tree_bytes, int* levels,
                     int* ttm_items);
void hooi_batch_free(tk_batch* b);

/* ---- learned tree and kernel selection ------------------------------------ */

/* Features of one TTM node for the cost model (TK_FEATURES floats):
 * log2 A, log2 L, log2 B, log2 K, log2 input bytes, log2 output bytes,
 * wide kernel applies (0/1), row kernel applies (0/1), input bytes per
 * element / 4, compute class (FP32 0, BF16 0.5, bf16x3 1, FP64 2),
 * tile == STAGED (0/1), tile == SPLITK (0/1), fused root pair (0 here).
 * tile: TK_TILE_AUTO, _STAGED or _SPLITK. */
#define TK_FEATURES 13
int tk_ttm_features(int64_t A, int64_t L, int64_t B, int64_t K, int in_dtype, int compute,
                    int tile, float* out);

/* Features of a fused root pair (both root children in one pass over T
 * viewed as [A, Lp, M, Lq, B]; tk_ttm_pair): log2 A, log2 Lp, log2 (M Lq B),
 * log2 Kp, log2 input bytes, log2 bytes of both outputs, 0, 0, input bytes per
 * element / 4, compute class, 0, 0, 1. */
int tk_pair_features(int64_t A, int64_t Lp, int64_t M, int64_t Lq, int64_t B, int64_t Kp,
                     int64_t Kq, int in_dtype, int compute, float* out);

/* Average time (ms, HIP events on `stream`) of `reps` launches of the TTM
 * node kernel chosen by `tile`, after one untimed launch.  Device buffers as
 * for tk_ttm; their contents only need to be finite. */
int tk_time_ttm(int in_dtype, int compute, const void* in, int64_t A, int64_t L, int64_t B,
                const void* F, int64_t K, void* out, int tile, int reps, void* stream,
                float* ms);

/* Average time (ms) of `reps` launches of tk_ttm_pair, after one untimed
 * launch; buffers as for tk_ttm_pair. */
int tk_time_ttm_pair(int in_dtype, int compute, const void* in, int64_t A, int64_t Lp, int64_t M,
                     int64_t Lq, int64_t B, const void* Fp, int64_t Kp, const void* Fq,
                     int64_t Kq, void* outp, void* outq, int reps, void* stream, float* ms);

/* Per-node kernel choices of tree `rank` (n = its node count; leaf entries
 * are ignored; TK_TILE_PAIR only on both root nodes of a two-child root).
 * hooi_init uses the choices of the selected tree. */
int tk_plan_set_tiles(tk_plan* plan, int rank, const int* tiles, int n);
int tk_plan_get_tiles(const tk_plan* plan, int rank, int* tiles, int cap, int* n);

/* MLP cost model, FP32 on the device: x' = (x - mu)/sigma,
 * h1 = relu(W1 x' + b1), h2 = relu(W2 h1 + b2), y = w3.h2 + b3 (y: log of
 * the node's time in ms).  Parameters flat in the order W1 (hidden x in_dim,
 * row-major), b1, W2 (hidden x hidden), b2, w3, b3; the caller supplies the
 * initial values (tk_mlp_param_count of them), so the library draws no random
 * numbers.  Training: full-batch Adam (beta 0.9 / 0.999, eps 1e-8) on the
 * mean squared error.  Host arrays in and out; errors TK_EINVAL / TK_ENOMEM /
 * TK_EDEVICE. */
typedef struct tk_mlp tk_mlp;
int64_t tk_mlp_param_count(int in_dim, int hidden);
int tk_mlp_create(int in_dim, int hidden, const float* params_host, tk_mlp** out);
int tk_mlp_set_norm(tk_mlp* m, const float* mu, const float* sigma);
/* Standardisation from training data: mu = per-feature mean and sigma =
 * per-feature population standard deviation of the n x in_dim rows of
 * X_host (row-major), in FP64; a feature whose deviation is at most 1e-6
 * keeps sigma = 1.  TK_EINVAL for n < 1 or non-finite features. */
int tk_mlp_fit_norm(tk_mlp* m, const float* X_host, int n);
int tk_mlp_get_params(const tk_mlp* m, float* host);
int tk_mlp_set_params(tk_mlp* m, const float* host); /* also resets Adam's moments */
int tk_mlp_forward(tk_mlp* m, const float* X_host, int n, float* y_host);
int tk_mlp_loss_grad(tk_mlp* m, const float* X_host, const float* y_host, int n,
                     float* loss_host, float* grad_host);
int tk_mlp_train(tk_mlp* m, const float* X_host, const float* y_host, int n, int steps,
                 float lr, float* loss_host /* steps values or NULL */);
void tk_mlp_free(tk_mlp* m);

/* The TTM view of an internal node as the engine runs it: In viewed as
 * [A, L, B] row-major (Sec. 2.1), K outputs, its input and output storage
 * types (TK_F64/F32/BF16/F16) and compute mode (TK_C_*) under the precision
 * rules of hooi_init for the given storage type and compute mode. */
typedef struct {
  int32_t node;      /* index in tk_plan_nodes order                */
  int32_t in_dtype;  /* storage type of In                          */
  int32_t out_dtype; /* storage type of the node's output           */
  int32_t compute;   /* TK_C_* the node's TTM runs at               */
  int64_t A, L, B, K;
} tk_node_view;
/* Views of the internal nodes of tree `rank` (parents first), as
 * tk_plan_learned weighs them and hooi_init runs them (the plan's tiles for
 * that rank, when set, enter the storage-type rules).  out NULL: only *n.
 * Errors: TK_EINVAL (null plan or n, bad rank, dtype or compute, cap below
 * the internal node count). */
int tk_plan_node_views(const tk_plan* plan, int rank, int tdtype, int compute,
                       tk_node_view* out, int cap, int* n);
/* The two root children of tree `rank` when the root has exactly two
 * internal children: view7 = (A, Lp, M, Lq, B, Kp, Kq) with T viewed as
 * [A, Lp, M, Lq, B] for their modes p < q; *fusable = 1 when a pair kernel
 * takes them for this storage type and compute mode (tk_ttm_pair).  Other
 * roots: view7 zeroed and *fusable = 0.  Errors: TK_EINVAL. */
int tk_plan_root_pair(const tk_plan* plan, int rank, int tdtype, int compute, int64_t* view7,
                      int* fusable);

/* Choose among the trees a TK_TREE_DP plan holds (topk > 1) and each
 * internal node's kernel by the model's predicted time (sum over internal
 * nodes, each at its fastest predicted kernel; a tree whose two root
 * children a pair kernel takes may instead run them fused, predicted from
 * tk_pair_features).  The choice replaces the DP optimum with automatic
 * kernels and separate root TTMs only when predicted faster by more than
 * `margin` (fraction); it is stored as the plan's selected rank and tiles.
 * predicted_ms: NULL or tk_plan_count entries (each tree at its best kernels). */
int tk_plan_learned(tk_plan* plan, tk_mlp* model, int tdtype, int compute, double margin,
                    int* chosen, double* predicted_ms);

/* ---- kernel-level entry points (device pointers, enqueued on `stream`) ---- */

/* TTM node (Sec. 2.1): with In viewed as [A, L, B] row-major,
 *   Out[a, k, b] = sum_l F[l, k] * In[a, l, b],  0 <= k < K.
 * in_dtype: TK_F64/TK_F32/TK_BF16/TK_F16 element type of In (TK_F16 with
 * TK_C_FP32 only, else TK_EUNSUPPORTED).  F: device, L x K
 * row-major FP64 when compute == TK_C_FP64, else FP32.  Out: device,
 * [A, K, B] of FP64 (compute FP64) or FP32.  K <= 4096; L <= 512 for
 * TK_C_FP64, L <= 2048 otherwise.  In and Out must not overlap.
 * TK_C_BF16 / TK_C_BF16X3 round (split) In and F to bfloat16 on the fly; a
 * node whose B is not a multiple of 4 (or B == 1 with L not a multiple of 4),
 * or a B % 4 == 0 node of fewer than 256 x 1024 columns (A * B), is computed
 * with FP32 operands instead, which is at least as accurate.  TK_C_FP32 on
 * BF16 input with at least 256 x 1024 such columns runs BF16 MFMAs with the
 * factor split exactly into three bfloat16 terms (FP32 results up to the
 * order of accumulation).
 * Errors: TK_EINVAL (null pointer, size < 1, unknown code), TK_EUNSUPPORTED
 * (dtype/compute pair or size limit), TK_EDEVICE (launch failure). */
int tk_ttm(int in_dtype, int compute, const void* in, int64_t A, int64_t L, int64_t B,
           const void* F, int64_t K, void* out, void* stream);

/* Both children of a TTM-tree root in one pass over the input (Sec. 3.1: a
 * node's output -- here T -- is reused by all its children).  With `in`
 * viewed row-major as [A, Lp, M, Lq, B] (device, FP32):
 *   outp[a, kp, m, lq, b] = sum_lp Fp[lp, kp] in[a, lp, m, lq, b]   ([A, Kp, M, Lq, B])
 *   outq[a, lp, m, kq, b] = sum_lq Fq[lq, kq] in[a, lp, m, lq, b]   ([A, Lp, M, Kq, B])
 * Fp: Lp x Kp, Fq: Lq x Kq row-major FP32, device.  compute: TK_C_FP32.
 * Requirements (else TK_EUNSUPPORTED): 16-byte aligned pointers, Kp, Kq <= 20,
 * and either the two trailing modes (M = B = 1) with Lq % 4 == 0, Lq <= 256,
 * Lp * ceil(Kp / 4) <= 2560 (or Lp * Lq <= 2048, Kp, Kq <= 8, A >= 4096), or
 * B % 4 == 0, Lq <= 256, A * M * B / 4 >= 2048.  Asynchronous on `stream`. */
int tk_ttm_pair(int in_dtype, int compute, const void* in, int64_t A, int64_t Lp, int64_t M,
                int64_t Lq, int64_t B, const void* Fp, int64_t Kp, const void* Fq, int64_t Kq,
                void* outp, void* outq, void* stream);

/* Gram (Sec. 5): with Y viewed as [A, L, B], S[i, j] = sum_{a,b} Y[a,i,b] Y[a,j,b],
 * written as a full symmetric L x L FP64 matrix to device memory S.
 * in_dtype: TK_F64 (FP64 arithmetic), or TK_F32, TK_BF16 or TK_F16 (every
 * entry widened exactly to FP64, FP64 products and sums of fixed-size column
 * blocks in a fixed order: deterministic).  L <= 1024. */
int tk_gram(int in_dtype, const void* Y, int64_t A, int64_t L, int64_t B, double* S,
            void* stream);

/* tk_gram without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same operation, arguments and layouts as tk_gram; the
 * column-chunk partial sums live in a static device array of 4 Mi doubles
 * (32 MiB, held by every GPU the library runs on until the process ends),
 * so the column chunks grow when the partials would not fit (the sums then
 * run in another fixed order: equal to tk_gram within FP64 rounding, still
 * deterministic).  Enqueued on `stream`, no synchronisation.  Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (other streams,
 * other threads) race and must be ordered by the caller.  Errors: those of
 * tk_gram, TK_EUNSUPPORTED when one chunk's partials exceed the array
 * (more than 1024 rows), TK_EDEVICE if the array's address cannot be taken. */
int tk_gram_noalloc(int in_dtype, const void* Y, int64_t A, int64_t L, int64_t B, double* S,
                    void* stream);

/* Leading K eigenpairs of `count` symmetric L x L FP64 matrices (device,
 * contiguous), eigenvalues descending, each eigenvector's largest-magnitude
 * entry (lowest index on ties) made positive (Sec. 2.2: the new factor is the
 * leading K_n left singular vectors of Y_(n), from its Gram matrix, Sec. 5).
 * Subspace iteration (K <= 48, L <= 1024) from V0: NULL (cold start) or
 * device L x K start blocks (warm start, e.g. the previous factors); a matrix
 * whose solve does not converge (no eigen-gap at K), and every matrix when
 * K > 48 or L > 1024, goes through the gap-free solver of tk_eig_full.
 * F: device count x L x K row-major; evals: device count x K.  L <= 2048.
 * Allocates its work areas per call and synchronises the stream.
 * Errors: TK_EINVAL (sizes, null pointers), TK_EUNSUPPORTED (L > 2048),
 * TK_ENUMERIC (non-finite values or no QL convergence), TK_EDEVICE. */
int tk_eig_leading(int count, int L, int K, const double* S, const double* V0, double* F,
                   double* evals, void* stream);

/* The gap-free solver alone (the route the paper's expert eigen-driver takes,
 * Sec. 5): Householder tridiagonalisation of each S, implicit QL with
 * Wilkinson shifts accumulating the eigenvectors of the tridiagonal matrix,
 * the K largest eigenpairs back-transformed, sign rule as tk_eig_leading.
 * Needs no gap at K and no start.  Same layouts, limits and errors as
 * tk_eig_leading (1 <= K <= L <= 2048). */
int tk_eig_full(int count, int L, int K, const double* S, double* F, double* evals,
                void* stream);

const char* tk_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TUCKER_H */
