// HOOI engine: device context, depth-first TTM-tree executor, HOSVD start,
// factor update, core and error (Fig. 2 "HOOI Procedure"; Sec. 3.1 tree
// execution; Sec. 5 Gram + EVD).
//
// Tree execution (Sec. 3.1): nodes run in depth-first order, a node's input is
// its parent's output, and a node's output is reused by all its children.
// Outputs live on a stack: the output of a node at depth d sits right after
// the outputs of its ancestors, so at most one intermediate per depth is alive
// and the workspace is the largest per-path sum of |Out(u)|.
//
// One HOOI invocation (Jacobi form: every chain uses the factors from the
// start of the invocation):
//   tree pass with F^(t): every leaf n gets Y_n, its Gram S_n is formed;
//   the core of decomposition t is folded in, G^(t) = Y_m x_m F_m^(t)T for the
//   leaf m with the smallest Y (all chains agree by commutativity), and
//   ||G^(t)||^2 gives the error of decomposition t;
//   FP64 eigensolver (warm-started from F^(t)) -> F^(t+1).
// The core of the final decomposition comes from a direct TTM chain over T in
// the cheapest order for a single chain (ascending K_j L_j / (L_j - K_j)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"
#include "kernels.h"

using namespace tk;

namespace {

int dalloc(void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(TK_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
  }
  return TK_OK;
}

size_t dtype_size(int dt) { return dt == TK_F64 ? 8 : (dt == TK_F32 ? 4 : 2); }

int64_t align64(int64_t x) { return (x + 63) & ~(int64_t)63; }

// [A, L, B] view of a tensor whose modes in `pre` are already multiplied, along mode n.
}  // namespace

struct tk_ctx {
  Shape s;
  int tdtype = TK_F32;
  int compute = TK_C_FP32;
  // Arithmetic of the core and the error (the folded-core path and the direct
  // core chain).  The error comes from ||T||^2 - ||G||^2, whose absolute
  // error is the relative error of ||G||^2; BF16 operands (2^-8) would make
  // that larger than e^2 itself at the error levels of interest, so the BF16
  // modes form the core at FP32.
  int core_compute = TK_C_FP32;
  std::vector<int> node_compute;  // per tree node: compute, or core_compute on the fold path
  std::vector<int> node_tile;     // per tree node: TK_TILE_* kernel choice from the plan
  // per tree node: storage type of its output.  In TK_C_BF16 mode nodes off the
  // fold path whose kernel is a BF16 one and whose children are all TTMs write
  // BF16 (those consumers round their input to BF16 anyway); everything else,
  // leaf tensors included, is stored in wdtype.
  std::vector<int> node_out_dt;
  // per tree node: its input is read once (T, or a parent with no other
  // child), so the TTM streams it with non-temporal loads
  std::vector<char> node_stream;
  int in_dtype_of(int u) const {
    const int p = tree.nodes[u].parent;
    return p < 0 ? tdtype : node_out_dt[p];
  }
  int wdtype = TK_F32;  // element type of intermediates and compute-precision factors
  const void* T = nullptr;
  hipStream_t st = nullptr;
  Tree tree;
  std::vector<int64_t> node_off;  // element offset of each internal node's output in ws
  std::vector<int> chain_order;   // mode order of the direct core chain
  // Both root children formed by one pass over T (ttm_pair): their indices
  // (pair_u[0] multiplies the lower mode) or -1.  The second child's subtree
  // then sits after the first's in the workspace, since both outputs are live
  // at once.
  int pair_u[2] = {-1, -1};
  int fold_leaf = 0;              // leaf whose Y folds the core
  int64_t ws_elems = 0, chain_a = 0;
  size_t fofs[TK_MAX_MODES + 1] = {};
  size_t sofs[TK_MAX_MODES + 1] = {};
  size_t kofs[TK_MAX_MODES + 1] = {};
  int64_t core_elems = 1;

  void* ws = nullptr;
  double* F64a = nullptr;   // current factors (FP64 master)
  double* F64b = nullptr;   // next factors
  void* Fc = nullptr;       // compute-precision copy of the current factors
  void* Fcb = nullptr;      // compute-precision copy of the next factors
  double* S = nullptr;      // Gram matrices
  double* ev = nullptr;     // eigenvalues
  double* eigwork = nullptr;
  int* status = nullptr;
  EigJob* jobs = nullptr;   // device job table, warm start from F64a
  EigJob* jobs_cold = nullptr;
  std::vector<EigJob> jobs_h;
  // Gap-free solver (eigfull.hip): one job per mode.  A mode whose K exceeds
  // the subspace block limit (full_only) always takes it; every other mode
  // takes it only after a subspace solve that did not converge, so no
  // unconverged factor is ever adopted.
  EigFullJob* fjobs = nullptr;
  double* fwork = nullptr;
  bool full_only[TK_MAX_MODES] = {};
  int fLmax = 0, fKmax = 0;
  double* gpart = nullptr;  // Gram chunk partials
  size_t gpart_elems = 0;
  double* rpart = nullptr;  // reduction partials
  double* scal = nullptr;   // device scalars: [0] ||T||^2, [1..] ||G||^2 history
  int scal_cap = 0;
  void* core = nullptr;     // core of the current decomposition (wdtype)
  std::vector<void*> leaves;  // optional copies of leaf tensors (tk_tree_pass)
  std::vector<int64_t> leaf_elems;

  double normT2 = 0.0;
  double normG2 = 0.0;
  bool core_valid = false;
  int maxit_warm = 20, maxit_cold = 100;
  double eig_tol = 1e-11;
  int Lmax = 0, pmax = 0;

  // Side stream for the per-leaf eigensolves (default priority).  The solve
  // for mode n starts when its Gram is formed (ev_leaf[n]) and signals
  // ev_fac[n] once the new factor (FP64 and compute copy) is written; the main
  // stream waits on ev_fac[n] only before it next uses factor n, so a solve
  // overlaps the rest of its own tree pass and the start of the next one.
  // Up to kMaxSide side streams, mode n's solve on sides[n % count]: the
  // solves of different modes (one workgroup each) run side by side.
  static constexpr int kMaxSide = 4;
  std::vector<hipStream_t> sides;
  hipStream_t side_of(int n) const { return sides[(size_t)n % sides.size()]; }
  // Device work runs on `st`.  With CU partitioning (the default) `st` is an
  // internal stream masked away from a few CUs that only the side stream
  // uses, so the latency-bound eigensolver never shares a CU with the
  // bandwidth-bound tree kernels; `user` is then the caller's stream, joined
  // to `st` by events at every entry point (enter/leave).
  hipStream_t user = nullptr;
  bool own_main = false;
  int side_cus = 0;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipEvent_t ev_leaf[TK_MAX_MODES] = {};
  hipEvent_t ev_fac[TK_MAX_MODES] = {};
  bool pending[TK_MAX_MODES] = {};
  int passes = 0;  // pipelined passes so far (alternates the root-subtree order)

  ~tk_ctx() {
    for (hipStream_t q : sides) (void)hipStreamSynchronize(q);
    if (own_main) (void)hipStreamSynchronize(st);
    void* ptrs[] = {ws, F64a, F64b, wdtype == TK_F64 ? nullptr : Fc,
                    wdtype == TK_F64 ? nullptr : Fcb, S, ev, eigwork, status, jobs,
                    jobs_cold, gpart, rpart, scal, core, fjobs, fwork};
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
    for (void* p : leaves)
      if (p) (void)hipFree(p);
    for (hipEvent_t e : ev_leaf)
      if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : ev_fac)
      if (e) (void)hipEventDestroy(e);
    for (hipStream_t q : sides) (void)hipStreamDestroy(q);
    if (own_main) (void)hipStreamDestroy(st);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
  }

  const void* fc(int n) const {
    return (const char*)Fc + fofs[n] * dtype_size(wdtype);
  }
  void* wsp(int64_t off) const { return (char*)ws + off * dtype_size(wdtype); }
};

namespace {

// Order the context's stream after the caller's work on entry and the
// caller's stream after the context's work on exit (no-ops without an
// internal stream).
struct Handoff {
  tk_ctx* c;
  explicit Handoff(tk_ctx* ctx) : c(ctx) {
    if (c && c->own_main) {
      (void)hipEventRecord(c->ev_in, c->user);
      (void)hipStreamWaitEvent(c->st, c->ev_in, 0);
    }
  }
  ~Handoff() {
    if (c && c->own_main) {
      (void)hipEventRecord(c->ev_out, c->st);
      (void)hipStreamWaitEvent(c->user, c->ev_out, 0);
    }
  }
};

// CUs reserved for the side stream: TK_SIDE_CUS (0 disables the partition),
// default 8.  Mask bit i names the runtime's CU i; the first eight cover one
// CU of each of the eight XCDs (measured: with 1-4 reserved bits the solves
// still ran 3x slower under a concurrent root TTM, with 8 they did not).
int reserved_side_cus() {
  const char* v = getenv("TK_SIDE_CUS");
  if (!v || !*v) return 8;
  const int n = atoi(v);
  return n < 0 ? 0 : std::min(n, 64);
}

// Create the side streams and, when CU partitioning is available, the
// internal main stream; on any failure of the masked variant fall back to
// unmasked side streams and the caller's stream.  One side stream, unless a
// mode goes straight to the gap-free solver (K above the subspace limit):
// those solves take 10-300 ms each, and one stream per mode (at most
// kMaxSide) runs them side by side (HCCI 892 -> 344 ms per invocation).
// Small warm solves stay on one stream: with four, the six-mode tensor's
// invocation went from 4.15 to 5.10 ms.
hipError_t create_streams(tk_ctx* c) {
  const int reserve = reserved_side_cus();
  bool heavy = false;
  for (int n = 0; n < c->s.N; ++n) heavy = heavy || c->full_only[n];
  const int nside = heavy ? std::max(1, std::min(c->s.N, tk_ctx::kMaxSide)) : 1;
  int dev = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  if (reserve > 0 && ncu > 4 * reserve) {
    const int words = (ncu + 31) / 32;
    std::vector<uint32_t> side_mask(words, 0u), main_mask(words, 0u);
    for (int i = 0; i < ncu; ++i) (i < reserve ? side_mask : main_mask)[i / 32] |= 1u << (i % 32);
    std::vector<hipStream_t> sides;
    hipStream_t main = nullptr;
    hipError_t e1 = hipSuccess;
    for (int k = 0; k < nside && e1 == hipSuccess; ++k) {
      hipStream_t q = nullptr;
      e1 = hipExtStreamCreateWithCUMask(&q, (uint32_t)words, side_mask.data());
      if (e1 == hipSuccess) sides.push_back(q);
    }
    hipError_t e2 = e1 == hipSuccess
                        ? hipExtStreamCreateWithCUMask(&main, (uint32_t)words, main_mask.data())
                        : e1;
    hipError_t e3 = e2 == hipSuccess ? hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) : e2;
    hipError_t e4 = e3 == hipSuccess ? hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) : e3;
    if (e4 == hipSuccess) {
      c->sides = sides;
      c->user = c->st;
      c->st = main;
      c->own_main = true;
      c->side_cus = reserve;
      return hipSuccess;
    }
    for (hipStream_t q : sides) (void)hipStreamDestroy(q);
    if (main) (void)hipStreamDestroy(main);
    if (c->ev_in) (void)hipEventDestroy(c->ev_in);
    if (c->ev_out) (void)hipEventDestroy(c->ev_out);
    c->ev_in = c->ev_out = nullptr;
    (void)hipGetLastError();
  }
  for (int k = 0; k < nside; ++k) {
    hipStream_t q = nullptr;
    if ((e = hipStreamCreateWithFlags(&q, hipStreamNonBlocking)) != hipSuccess) return e;
    c->sides.push_back(q);
  }
  return hipSuccess;
}

// Every mode's leading eigenpairs on the main stream: subspace iteration
// (one launch over all modes when every mode takes it), then the gap-free
// solver for the full-only modes and for any solve that did not converge.
int run_eig(tk_ctx* c, bool warm, double* F_out, int maxit) {
  const int N = c->s.N;
  bool any_full = false;
  for (int n = 0; n < N; ++n) any_full = any_full || c->full_only[n];
  if (!any_full) {
    TK_HIP(launch_eig(N, warm ? c->jobs : c->jobs_cold, 0, c->Lmax, c->pmax, c->S, c->F64a,
                      F_out, c->ev, c->eigwork, c->status, c->status + N, maxit, c->eig_tol,
                      c->st));
  } else {
    const std::vector<EigJob>& tab = c->jobs_h;
    for (int n = 0; n < N; ++n) {
      if (c->full_only[n]) continue;
      TK_HIP(launch_eig(1, warm ? c->jobs : c->jobs_cold, n, tab[n].L, c->pmax, c->S, c->F64a,
                        F_out, c->ev, c->eigwork, c->status, c->status + N, maxit, c->eig_tol,
                        c->st));
    }
  }
  TK_HIP(launch_eig_full(N, c->fjobs, c->fLmax, c->fKmax, c->S, F_out, c->ev, c->fwork,
                         c->status, c->st));
  return TK_OK;
}

int refresh_compute_factors(tk_ctx* c) {
  if (c->wdtype == TK_F64) return TK_OK;  // Fc aliases F64a in FP64 mode
  TK_HIP(launch_convert(TK_F64, c->wdtype, c->F64a, c->Fc, (int64_t)c->fofs[c->s.N], c->st));
  return TK_OK;
}

// Make the main stream wait for the pending update of factor n (if any).
int wait_factor(tk_ctx* c, int n) {
  if (!c->pending[n]) return TK_OK;
  TK_HIP(hipStreamWaitEvent(c->st, c->ev_fac[n], 0));
  c->pending[n] = false;
  return TK_OK;
}

// Make the main stream wait for every pending factor update.
int join_factors(tk_ctx* c) {
  for (int n = 0; n < c->s.N; ++n)
    if (int rc = wait_factor(c, n)) return rc;
  return TK_OK;
}

int check_status(tk_ctx* c) {
  if (int rc = join_factors(c)) return rc;
  std::vector<int> st(c->s.N);
  TK_HIP(hipMemcpyAsync(st.data(), c->status, sizeof(int) * c->s.N, hipMemcpyDeviceToHost, c->st));
  TK_HIP(hipStreamSynchronize(c->st));
  for (int n = 0; n < c->s.N; ++n) {
    if (st[n] == 2) return fail(TK_ENUMERIC, "non-finite values in the eigensolver for mode %d", n);
    if (st[n] == 1)
      return fail(TK_ENUMERIC, "eigensolver did not converge for mode %d (no gap at K?)", n);
  }
  return TK_OK;
}

}  // namespace

void tk::tree_precisions(const Shape& s, const std::vector<tk_node>& nodes, int tdtype,
                         int compute, const std::vector<int>& tiles, const void* T,
                         int* fold_leaf, std::vector<int>* node_compute,
                         std::vector<int>* out_dt) {
  const int N = s.N;
  int64_t best = -1;
  for (int n = 0; n < N; ++n) {
    const int64_t y = (int64_t)s.card(((1u << N) - 1) & ~(1u << n));
    if (best < 0 || y < best) {
      best = y;
      *fold_leaf = n;
    }
  }
  const int core_compute =
      (compute == TK_C_BF16 || compute == TK_C_BF16X3) ? TK_C_FP32 : compute;
  node_compute->assign(nodes.size(), compute);
  for (size_t u = 0; u < nodes.size(); ++u)
    if (nodes[u].is_leaf && nodes[u].mode == *fold_leaf)
      for (int v = (int)u; v >= 0; v = nodes[v].parent) (*node_compute)[v] = core_compute;
  auto tile = [&](size_t u) { return u < tiles.size() ? tiles[u] : (int)TK_TILE_AUTO; };
  // intermediates sit at 64-element offsets of the workspace: any 256-byte
  // aligned address stands for them in the kernels' alignment checks
  const void* ws = reinterpret_cast<const void*>((uintptr_t)256);
  const int wdtype = compute == TK_C_FP64 ? TK_F64 : TK_F32;
  std::vector<char> feeds_leaf(nodes.size(), 0);
  for (const tk_node& nd : nodes)
    if (nd.parent >= 0 && nd.is_leaf) feeds_leaf[nd.parent] = 1;
  // parents before children: a child's kernel choice depends on its input's type
  out_dt->assign(nodes.size(), wdtype);
  for (size_t u = 0; u < nodes.size(); ++u) {
    const tk_node& nd = nodes[u];
    if (nd.is_leaf || feeds_leaf[u] || (*node_compute)[u] != TK_C_BF16) continue;
    int64_t A, Lu, B;
    view(s, nd.pre_mask, nd.mode, &A, &Lu, &B);
    const int in_dt = nd.parent < 0 ? tdtype : (*out_dt)[nd.parent];
    bool ok = ttm_bf16_output_ok(in_dt, TK_C_BF16, nd.parent < 0 ? T : ws, A, Lu, B, ws,
                                 tile(u));
    for (size_t v = 0; v < nodes.size() && ok; ++v) {
      if (nodes[v].parent != (int)u) continue;
      int64_t Av, Lv, Bv;
      view(s, nodes[v].pre_mask, nodes[v].mode, &Av, &Lv, &Bv);
      ok = (*node_compute)[v] == TK_C_BF16 &&
           ttm_bf16_output_ok(TK_BF16, TK_C_BF16, ws, Av, Lv, Bv, ws, tile(v));
    }
    if (ok) (*out_dt)[u] = TK_BF16;
  }
}

namespace {

// Execution order of the nodes: depth-first, root subtrees in plan order or,
// with `reverse`, in reverse plan order (each subtree stays depth-first).
std::vector<int> exec_order(const std::vector<tk_node>& nodes, bool reverse) {
  std::vector<int> starts;
  for (size_t u = 0; u < nodes.size(); ++u)
    if (nodes[u].parent < 0) starts.push_back((int)u);
  starts.push_back((int)nodes.size());
  std::vector<int> order;
  const int nsub = (int)starts.size() - 1;
  for (int k = 0; k < nsub; ++k) {
    const int r = reverse ? nsub - 1 - k : k;
    for (int u = starts[r]; u < starts[r + 1]; ++u) order.push_back(u);
  }
  return order;
}

// One tree pass with the compute-precision factors in c->Fc.
//   fold_dst >= 0: fold the core (G = Y_m x_m F_m^T) and store ||G||^2 in scal[fold_dst].
//   keep: copy every leaf tensor to c->leaves.
//   ev_t: optional per-node timing events (2 per node, indexed by node).
//   update: every leaf's warm-started eigensolve runs on the side stream as
//   soon as its Gram is formed, writing the next factors (F64b, Fcb); at the
//   end of the pass next and current factors swap and every factor is marked
//   pending until its solve has finished.  Alternate passes run the root
//   subtrees in reverse order so that a factor finished late in one pass is
//   needed late in the next one.
int tree_pass(tk_ctx* c, int fold_dst, bool keep, hipEvent_t* ev_t, bool update = false) {
  const Shape& s = c->s;
  const auto& nodes = c->tree.nodes;
  const std::vector<int> order = exec_order(nodes, update && (c->passes % 2 == 1));
  bool pair_done = false;
  for (int u : order) {
    const tk_node& nd = nodes[u];
    // the node reads factor nd.mode (a leaf also rewrites Gram buffer nd.mode,
    // which the pending solve of that mode may still read)
    if (int rc = wait_factor(c, nd.mode)) return rc;
    const void* in = nd.parent < 0 ? c->T : c->wsp(c->node_off[nd.parent]);
    const int in_dt = c->in_dtype_of(u);
    int64_t A, L, B;
    view(s, nd.pre_mask, nd.mode, &A, &L, &B);
    if (ev_t) TK_HIP(hipEventRecord(ev_t[2 * u], c->st));
    if (c->pair_u[0] >= 0 && (u == c->pair_u[0] || u == c->pair_u[1])) {
      // both root children in one pass over T (the first of them to run
      // launches it; the other has nothing left to do)
      if (!pair_done) {
        const int up = c->pair_u[0], uq = c->pair_u[1];
        const int p = nodes[up].mode, q = nodes[uq].mode;
        if (int rc = wait_factor(c, p)) return rc;
        if (int rc = wait_factor(c, q)) return rc;
        int64_t Ap, Lp, Bp, Aq, Lq, Bq;
        view(s, 0, p, &Ap, &Lp, &Bp);
        view(s, 0, q, &Aq, &Lq, &Bq);
        TK_HIP(launch_ttm_pair((const float*)c->T, Ap, Lp, Aq / (Ap * Lp), Lq, Bq,
                               (const float*)c->fc(p), s.K[p], (const float*)c->fc(q), s.K[q],
                               (float*)c->wsp(c->node_off[up]), (float*)c->wsp(c->node_off[uq]),
                               c->st));
        pair_done = true;
      }
    } else if (!nd.is_leaf) {
      TK_HIP(launch_ttm(in_dt, c->node_compute[u], in, A, L, B, c->fc(nd.mode), s.K[nd.mode],
                        c->wsp(c->node_off[u]), c->st, c->node_stream[u], c->node_tile[u],
                        c->node_out_dt[u]));
    } else {
      const int n = nd.mode;
      TK_HIP(launch_gram(in_dt, in, A, L, B, c->S + c->sofs[n], c->gpart, c->st));
      if (keep)
        TK_HIP(hipMemcpyAsync(c->leaves[n], in, (size_t)c->leaf_elems[n] * dtype_size(in_dt),
                              hipMemcpyDeviceToDevice, c->st));
      if (update) {
        hipStream_t side = c->side_of(n);
        TK_HIP(hipEventRecord(c->ev_leaf[n], c->st));
        TK_HIP(hipStreamWaitEvent(side, c->ev_leaf[n], 0));
        const EigJob& j = c->jobs_h[n];
        if (!c->full_only[n])
          TK_HIP(launch_eig(1, c->jobs, n, j.L, j.p, c->S, c->F64a, c->F64b, c->ev, c->eigwork,
                            c->status, c->status + s.N, c->maxit_warm, c->eig_tol, side));
        TK_HIP(launch_eig_full(1, c->fjobs + n, j.L, j.K, c->S, c->F64b, c->ev, c->fwork,
                               c->status, side));
        if (c->wdtype != TK_F64)
          TK_HIP(launch_convert(TK_F64, c->wdtype, c->F64b + c->fofs[n],
                                (char*)c->Fcb + c->fofs[n] * dtype_size(c->wdtype),
                                (int64_t)(c->fofs[n + 1] - c->fofs[n]), side));
        TK_HIP(hipEventRecord(c->ev_fac[n], side));
      }
      if (fold_dst >= 0 && n == c->fold_leaf) {
        TK_HIP(launch_ttm(in_dt, c->core_compute, in, A, L, B, c->fc(n), s.K[n], c->core, c->st));
        TK_HIP(launch_sumsq(c->wdtype, c->core, c->core_elems, c->rpart, c->scal + fold_dst,
                            c->st));
      }
    }
    if (ev_t) TK_HIP(hipEventRecord(ev_t[2 * u + 1], c->st));
  }
  if (update) {
    std::swap(c->F64a, c->F64b);
    std::swap(c->Fc, c->Fcb);
    for (int n = 0; n < s.N; ++n) c->pending[n] = true;
    c->passes++;
  }
  return TK_OK;
}

// Core of the current factors by a direct chain over T; ||G||^2 -> scal[dst].
int core_chain(tk_ctx* c, int dst) {
  const Shape& s = c->s;
  uint32_t pre = 0;
  const void* in = c->T;
  int in_dt = c->tdtype;
  const int N = s.N;
  for (int i = 0; i < N; ++i) {
    const int n = c->chain_order[i];
    int64_t A, L, B;
    view(s, pre, n, &A, &L, &B);
    void* out = (i == N - 1) ? c->core : c->wsp((i % 2 == 0) ? 0 : c->chain_a);
    // every input of the chain is read once
    TK_HIP(launch_ttm(in_dt, c->core_compute, in, A, L, B, c->fc(n), s.K[n], out, c->st, true));
    pre |= 1u << n;
    in = out;
    in_dt = c->wdtype;
  }
  TK_HIP(launch_sumsq(c->wdtype, c->core, c->core_elems, c->rpart, c->scal + dst, c->st));
  return TK_OK;
}

double rel_err_of(double normT2, double normG2) {
  return std::sqrt(std::max(normT2 - normG2, 0.0) / normT2);
}

int ensure_scal(tk_ctx* c, int need) {
  if (need <= c->scal_cap) return TK_OK;
  if (c->scal) (void)hipFree(c->scal);
  c->scal = nullptr;
  const int cap = std::max(need, 64);
  if (int rc = dalloc((void**)&c->scal, sizeof(double) * cap)) return rc;
  c->scal_cap = cap;
  return TK_OK;
}

}  // namespace

extern "C" int hooi_init(int N, const int64_t* L, const int64_t* K, int tdtype, const void* T_dev,
                         const tk_plan* plan, int compute, const double* F0_host, void* stream,
                         tk_ctx** out) {
  clear_error();
  if (!out) return fail(TK_EINVAL, "out is null");
  *out = nullptr;
  Shape s;
  if (int rc = make_shape(N, L, K, &s)) return rc;
  if (!T_dev) return fail(TK_EINVAL, "T_dev is null");
  if (tdtype < TK_F64 || tdtype > TK_F16) return fail(TK_EINVAL, "unknown dtype %d", tdtype);
  if (compute < TK_C_FP64 || compute > TK_C_BF16X3)
    return fail(TK_EINVAL, "unknown compute mode %d", compute);
  if ((tdtype == TK_F64) != (compute == TK_C_FP64))
    return fail(TK_EUNSUPPORTED, "FP64 storage pairs with FP64 compute only");
  if (tdtype == TK_F16 && compute != TK_C_FP32)
    return fail(TK_EUNSUPPORTED, "FP16 storage pairs with FP32 compute only");
  const int maxL = std::min(compute == TK_C_FP64 ? 512 : ttm_max_L(), eig_full_max_L());
  for (int j = 0; j < N; ++j)
    if (s.L[j] > maxL) return fail(TK_EUNSUPPORTED, "L[%d]=%lld exceeds %d", j, (long long)s.L[j], maxL);
  if (plan && !plan->shape.same(s)) return fail(TK_EINVAL, "plan was built for another shape");

  tk_ctx* c = new (std::nothrow) tk_ctx;
  if (!c) return fail(TK_ENOMEM, "context allocation failed");
  c->s = s;
  c->tdtype = tdtype;
  c->compute = compute;
  c->wdtype = compute == TK_C_FP64 ? TK_F64 : TK_F32;
  c->T = T_dev;
  c->st = (hipStream_t)stream;
  auto bail = [&](int rc) {
    delete c;
    return rc;
  };

  // ---- plan
  if (plan) {
    const int r = std::min<int>(plan->selected, (int)plan->trees.size() - 1);
    c->tree = plan->trees[r];
    if (r < (int)plan->tiles.size() && !plan->tiles[r].empty()) c->node_tile = plan->tiles[r];
  } else {
    tk_plan* p = nullptr;
    if (int rc = ttm_tree_plan(N, L, K, TK_TREE_DP, 1, &p)) return bail(rc);
    c->tree = p->trees[0];
    tk_plan_free(p);
  }
  const auto& nodes = c->tree.nodes;
  c->node_tile.resize(nodes.size(), TK_TILE_AUTO);
  c->node_off.assign(nodes.size(), 0);
  int64_t ws = 0;
  for (size_t u = 0; u < nodes.size(); ++u) {
    const tk_node& nd = nodes[u];
    // 64-element (>= 256-byte) alignment keeps the kernels' vector loads aligned
    const int64_t base =
        nd.parent < 0 ? 0 : align64(c->node_off[nd.parent] + (int64_t)nodes[nd.parent].out_card);
    c->node_off[u] = base;
    if (!nd.is_leaf) ws = std::max<int64_t>(ws, base + (int64_t)nd.out_card);
  }
  // both root children in one pass over T, when the plan asks for it
  // (TK_TILE_PAIR on both root nodes, as tk_plan_learned or tk_plan_set_tiles
  // set it), with FP32 storage and compute and a shape a pair kernel takes;
  // the second child's subtree moves past the first's in the workspace.
  // Otherwise the root nodes run their own kernels (TK_TILE_AUTO).
  {
    std::vector<int> roots;
    for (size_t u = 0; u < nodes.size(); ++u)
      if (nodes[u].parent < 0) roots.push_back((int)u);
    bool asked = false;
    for (int u : roots) asked = asked || c->node_tile[u] == TK_TILE_PAIR;
    for (int u : roots)
      if (c->node_tile[u] == TK_TILE_PAIR) c->node_tile[u] = TK_TILE_AUTO;
    if (asked && roots.size() == 2 && !nodes[roots[0]].is_leaf &&
        !nodes[roots[1]].is_leaf && tdtype == TK_F32 && compute == TK_C_FP32 &&
        c->node_tile[roots[0]] == TK_TILE_AUTO && c->node_tile[roots[1]] == TK_TILE_AUTO) {
      int up = roots[0], uq = roots[1];
      if (nodes[up].mode > nodes[uq].mode) std::swap(up, uq);
      const int p = nodes[up].mode, q = nodes[uq].mode;
      int64_t Ap, Lp, Bp, Aq, Lq, Bq;
      view(s, 0, p, &Ap, &Lp, &Bp);
      view(s, 0, q, &Aq, &Lq, &Bq);
      // alignment of the outputs is that of the workspace (256 bytes) and its
      // 64-element offsets; checked with representative aligned pointers
      const void* al = (const void*)(uintptr_t)256;
      const int pk = ttm_pair_kind(TK_F32, TK_C_FP32, T_dev, Ap, Lp, Aq / (Ap * Lp), Lq, Bq,
                                   s.K[p], s.K[q], al, al);
      if (pk >= 1) {
        const int second = std::max(roots[0], roots[1]);
        int64_t w1 = 0;
        for (int u = 0; u < second; ++u)
          if (!nodes[u].is_leaf) w1 = std::max<int64_t>(w1, c->node_off[u] + (int64_t)nodes[u].out_card);
        const int64_t shift = align64(w1);
        for (size_t u = second; u < nodes.size(); ++u) {
          c->node_off[u] += shift;
          if (!nodes[u].is_leaf) ws = std::max<int64_t>(ws, c->node_off[u] + (int64_t)nodes[u].out_card);
        }
        c->pair_u[0] = up;
        c->pair_u[1] = uq;
      }
    }
  }
  c->core_compute = (compute == TK_C_BF16 || compute == TK_C_BF16X3) ? TK_C_FP32 : compute;
  tree_precisions(s, nodes, tdtype, compute, c->node_tile, T_dev, &c->fold_leaf,
                  &c->node_compute, &c->node_out_dt);
  // direct core chain order: ascending K L / (L - K), modes with K = L last
  c->chain_order.resize(N);
  for (int j = 0; j < N; ++j) c->chain_order[j] = j;
  std::stable_sort(c->chain_order.begin(), c->chain_order.end(), [&](int a, int b) {
    const bool fa = s.K[a] == s.L[a], fb = s.K[b] == s.L[b];
    if (fa != fb) return !fa;
    if (fa) return false;
    return (__int128)s.K[a] * s.L[a] * (s.L[b] - s.K[b]) <
           (__int128)s.K[b] * s.L[b] * (s.L[a] - s.K[a]);
  });
  {
    const int o0 = c->chain_order[0], o1 = c->chain_order[1];
    const int64_t out1 = (int64_t)(s.card_T() / s.L[o0] * s.K[o0]);
    const int64_t out2 = out1 / s.L[o1] * s.K[o1];
    c->chain_a = align64(out1);
    ws = std::max<int64_t>(ws, c->chain_a + out2);
  }
  c->ws_elems = ws;
  for (int n = 0; n < N; ++n) {
    c->fofs[n + 1] = c->fofs[n] + (size_t)(s.L[n] * s.K[n]);
    c->sofs[n + 1] = c->sofs[n] + (size_t)(s.L[n] * s.L[n]);
    c->kofs[n + 1] = c->kofs[n] + (size_t)s.K[n];
    c->core_elems *= s.K[n];
  }

  // ---- eigensolver jobs
  size_t work = 0;
  c->jobs_h.resize(N);
  std::vector<EigFullJob> fjobs(N);
  size_t fwork = 0;
  for (int n = 0; n < N; ++n) {
    c->full_only[n] = s.K[n] > eig_max_K();
    EigFullJob& f = fjobs[n];
    f.L = (int)s.L[n];
    f.K = (int)s.K[n];
    f.status_idx = n;
    f.only_if_failed = c->full_only[n] ? 0 : 1;
    f.S_off = (int64_t)c->sofs[n];
    f.F_off = (int64_t)c->fofs[n];
    f.ev_off = (int64_t)c->kofs[n];
    f.work_off = (int64_t)fwork;
    fwork += eig_full_work_elems(f.L);
    c->fLmax = std::max(c->fLmax, f.L);
    c->fKmax = std::max(c->fKmax, f.K);
  }
  for (int n = 0; n < N; ++n) {
    EigJob& j = c->jobs_h[n];
    const int64_t rank_bound = (int64_t)(s.card(((1u << N) - 1) & ~(1u << n)) / s.L[n]);
    j.L = (int)s.L[n];
    j.K = (int)s.K[n];
    // full-only modes never run the subspace kernel; a small block keeps the
    // shared block width and work areas of the others unchanged
    j.p = c->full_only[n] ? 8 : eig_block_size(j.L, j.K, rank_bound);
    j.pad_ = 0;
    j.S_off = (int64_t)c->sofs[n];
    j.V0_off = (int64_t)c->fofs[n];
    j.F_off = (int64_t)c->fofs[n];
    j.ev_off = (int64_t)c->kofs[n];
    c->Lmax = std::max(c->Lmax, j.L);
    c->pmax = std::max(c->pmax, j.p);
  }
  // A launch over all modes uses the block width of the widest job for every
  // job, so each work area holds two L_n x padded(pmax) blocks.
  for (int n = 0; n < N; ++n) {
    EigJob& j = c->jobs_h[n];
    j.work_off = (int64_t)work;
    work += eig_work_elems(j.L, c->pmax);
  }
  // cold starts (HOSVD) use the full block; warm starts (previous factors)
  // need only K columns plus a little room to grow, which keeps the blocks in
  // LDS.  This holds for short modes too: a full Jacobi solve of a 64 x 64
  // Gram takes about 1.3 ms on its CU against about 0.1 ms for a K + 4 block,
  // and a solve that does not converge in the small block falls back to the
  // gap-free solver.
  std::vector<EigJob> cold = c->jobs_h;
  for (int n = 0; n < N; ++n) {
    EigJob& j = c->jobs_h[n];
    j.p = std::max(j.K, std::min(j.p, j.K + 4));
  }
  {
    hipError_t e = create_streams(c);
    if (e == hipSuccess && c->own_main) {
      // the caller's stream may still be producing T
      e = hipEventRecord(c->ev_in, c->user);
      if (e == hipSuccess) e = hipStreamWaitEvent(c->st, c->ev_in, 0);
    }
    for (int n = 0; n < N && e == hipSuccess; ++n) {
      e = hipEventCreateWithFlags(&c->ev_leaf[n], hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_fac[n], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
      delete c;
      return fail(TK_EDEVICE, "stream/event creation failed: %s", hipGetErrorString(e));
    }
  }
  for (auto& j : cold) j.V0_off = -1;

  // ---- Gram workspace: leaves and the HOSVD unfoldings of T
  size_t gp = 0;
  for (int n = 0; n < N; ++n) {
    gp = std::max(gp, gram_workspace_elems(s.L[n], (int64_t)(s.card(((1u << N) - 1) & ~(1u << n)) / s.L[n])));
    if (!F0_host) gp = std::max(gp, gram_workspace_elems(s.L[n], (int64_t)(s.card_T() / s.L[n])));
  }
  c->gpart_elems = gp;

  // ---- allocations
  const size_t wsz = dtype_size(c->wdtype);
  int rc = TK_OK;
  if ((rc = dalloc(&c->ws, (size_t)c->ws_elems * wsz))) return bail(rc);
  if ((rc = dalloc((void**)&c->F64a, sizeof(double) * c->fofs[N]))) return bail(rc);
  if ((rc = dalloc((void**)&c->F64b, sizeof(double) * c->fofs[N]))) return bail(rc);
  if (c->wdtype != TK_F64) {
    if ((rc = dalloc(&c->Fc, wsz * c->fofs[N]))) return bail(rc);
    if ((rc = dalloc(&c->Fcb, wsz * c->fofs[N]))) return bail(rc);
  }
  if ((rc = dalloc((void**)&c->S, sizeof(double) * c->sofs[N]))) return bail(rc);
  if ((rc = dalloc((void**)&c->ev, sizeof(double) * c->kofs[N]))) return bail(rc);
  if ((rc = dalloc((void**)&c->eigwork, sizeof(double) * work))) return bail(rc);
  if ((rc = dalloc((void**)&c->status, sizeof(int) * 2 * N))) return bail(rc);
  if ((rc = dalloc((void**)&c->jobs, sizeof(EigJob) * N))) return bail(rc);
  if ((rc = dalloc((void**)&c->jobs_cold, sizeof(EigJob) * N))) return bail(rc);
  if ((rc = dalloc((void**)&c->fjobs, sizeof(EigFullJob) * N))) return bail(rc);
  if ((rc = dalloc((void**)&c->fwork, sizeof(double) * fwork))) return bail(rc);
  if ((rc = dalloc((void**)&c->gpart, sizeof(double) * c->gpart_elems))) return bail(rc);
  if ((rc = dalloc((void**)&c->rpart, sizeof(double) * sumsq_partials()))) return bail(rc);
  if ((rc = ensure_scal(c, 64))) return bail(rc);
  if ((rc = dalloc(&c->core, wsz * (size_t)c->core_elems))) return bail(rc);
  if (c->wdtype == TK_F64) {  // the FP64 masters double as compute copies
    c->Fc = c->F64a;
    c->Fcb = c->F64b;
  }
  // output storage per node, parents before children (a child's kernel choice
  // depends on its input's type).  A node whose output is a leaf tensor keeps
  // it in wdtype: the Gram reads the leaf unrounded.
  std::vector<char> feeds_leaf(nodes.size(), 0);
  std::vector<int> children(nodes.size(), 0);
  for (const tk_node& nd : nodes)
    if (nd.parent >= 0) {
      children[nd.parent]++;
      if (nd.is_leaf) feeds_leaf[nd.parent] = 1;
    }
  // T is streamed by every child of the root (too large to stay in cache
  // between them); an intermediate with one consumer is read once
  c->node_stream.assign(nodes.size(), 0);
  for (size_t u = 0; u < nodes.size(); ++u)
    c->node_stream[u] = nodes[u].parent < 0 || children[nodes[u].parent] == 1;

  {
    hipError_t e = hipMemcpyAsync(c->jobs, c->jobs_h.data(), sizeof(EigJob) * N,
                                  hipMemcpyHostToDevice, c->st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->jobs_cold, cold.data(), sizeof(EigJob) * N, hipMemcpyHostToDevice,
                         c->st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->fjobs, fjobs.data(), sizeof(EigFullJob) * N, hipMemcpyHostToDevice,
                         c->st);
    if (e != hipSuccess) {
      delete c;
      return fail(TK_EDEVICE, "job upload failed: %s", hipGetErrorString(e));
    }
  }

  // ---- ||T||^2
  if (hipError_t e = launch_sumsq(tdtype, T_dev, (int64_t)s.card_T(), c->rpart, c->scal, c->st);
      e != hipSuccess) {
    delete c;
    return fail(TK_EDEVICE, "sum of squares of T failed: %s", hipGetErrorString(e));
  }

  // ---- starting factors
  if (F0_host) {
    for (size_t i = 0; i < c->fofs[N]; ++i)
      if (!std::isfinite(F0_host[i])) return bail(fail(TK_ENUMERIC, "F0 holds NaN/Inf"));
    if (hipError_t e = hipMemcpyAsync(c->F64a, F0_host, sizeof(double) * c->fofs[N],
                                      hipMemcpyHostToDevice, c->st);
        e != hipSuccess) {
      delete c;
      return fail(TK_EDEVICE, "factor upload failed: %s", hipGetErrorString(e));
    }
  } else {
    // HOSVD: F_n = leading K_n left singular vectors of T_(n)
    for (int n = 0; n < N; ++n) {
      int64_t A, Ln, B;
      view(s, 0, n, &A, &Ln, &B);
      if (hipError_t e = launch_gram(tdtype, T_dev, A, Ln, B, c->S + c->sofs[n], c->gpart, c->st);
          e != hipSuccess) {
        delete c;
        return fail(TK_EDEVICE, "HOSVD Gram failed: %s", hipGetErrorString(e));
      }
    }
    if (hipError_t e = launch_fill_int(c->status, N, 0, c->st); e != hipSuccess) {
      delete c;
      return fail(TK_EDEVICE, "status reset failed: %s", hipGetErrorString(e));
    }
    if ((rc = run_eig(c, false, c->F64a, c->maxit_cold))) return bail(rc);
    if ((rc = check_status(c))) return bail(rc);
  }
  if ((rc = refresh_compute_factors(c))) return bail(rc);
  double nt2 = 0.0;
  if (hipError_t e = hipMemcpyAsync(&nt2, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->st);
      e != hipSuccess) {
    delete c;
    return fail(TK_EDEVICE, "readback failed: %s", hipGetErrorString(e));
  }
  if (hipError_t e = hipStreamSynchronize(c->st); e != hipSuccess) {
    delete c;
    return fail(TK_EDEVICE, "hooi_init: %s", hipGetErrorString(e));
  }
  if (!(nt2 > 0.0) || !std::isfinite(nt2)) return bail(fail(TK_ENUMERIC, "||T|| is zero or not finite"));
  c->normT2 = nt2;
  *out = c;
  return TK_OK;
}

namespace {
int eig_solve(int count, int L, int K, const double* S, const double* V0, double* F,
              double* evals, hipStream_t st, bool full_only);
}  // namespace

// STHOSVD start (Sec. 1, Sec. 2.2): modes in `order`, each taking the leading
// K_n eigenvectors of the Gram of the current tensor's mode-n unfolding and
// truncating the tensor along n before the next mode.  The factors then seed
// an ordinary context.
extern "C" int hooi_init_sthosvd(int N, const int64_t* L, const int64_t* K, int tdtype,
                                 const void* T_dev, const tk_plan* plan, int compute,
                                 const int* order, void* stream, tk_ctx** out) {
  clear_error();
  if (!out) return fail(TK_EINVAL, "out is null");
  *out = nullptr;
  Shape s;
  if (int rc = make_shape(N, L, K, &s)) return rc;
  if (!T_dev) return fail(TK_EINVAL, "T_dev is null");
  if (tdtype < TK_F64 || tdtype > TK_F16) return fail(TK_EINVAL, "unknown dtype %d", tdtype);
  if (compute < TK_C_FP64 || compute > TK_C_BF16X3)
    return fail(TK_EINVAL, "unknown compute mode %d", compute);
  if ((tdtype == TK_F64) != (compute == TK_C_FP64))
    return fail(TK_EUNSUPPORTED, "FP64 storage pairs with FP64 compute only");
  if (tdtype == TK_F16 && compute != TK_C_FP32)
    return fail(TK_EUNSUPPORTED, "FP16 storage pairs with FP32 compute only");
  const int maxL = std::min(compute == TK_C_FP64 ? 512 : ttm_max_L(), eig_full_max_L());
  for (int j = 0; j < N; ++j)
    if (s.L[j] > maxL) return fail(TK_EUNSUPPORTED, "L[%d]=%lld exceeds %d", j, (long long)s.L[j], maxL);
  int ord[TK_MAX_MODES];
  bool seen[TK_MAX_MODES] = {};
  for (int i = 0; i < N; ++i) {
    ord[i] = order ? order[i] : i;
    if (ord[i] < 0 || ord[i] >= N || seen[ord[i]])
      return fail(TK_EINVAL, "order is not a permutation of the modes");
    seen[ord[i]] = true;
  }
  hipStream_t st = (hipStream_t)stream;
  // the truncations run at FP64 for FP64 storage, else at FP32 (FP32 or BF16 input)
  const int wdt = tdtype == TK_F64 ? TK_F64 : TK_F32;
  const int tcomp = tdtype == TK_F64 ? TK_C_FP64 : TK_C_FP32;
  const size_t wsz = dtype_size(wdt);
  size_t fofs[TK_MAX_MODES + 1] = {};
  for (int n = 0; n < N; ++n) fofs[n + 1] = fofs[n] + (size_t)(s.L[n] * s.K[n]);
  int64_t Lmax = 0, Kmax = 0;
  size_t gp = 0, ymax = 0;
  uint32_t pre = 0;
  for (int i = 0; i < N; ++i) {
    const int n = ord[i];
    Lmax = std::max(Lmax, s.L[n]);
    Kmax = std::max(Kmax, s.K[n]);
    gp = std::max(gp, gram_workspace_elems(s.L[n], (int64_t)(s.card(pre) / s.L[n])));
    pre |= 1u << n;
    if (i + 1 < N) ymax = std::max(ymax, (size_t)s.card(pre));
  }
  double *F64 = nullptr, *S = nullptr, *ev = nullptr, *part = nullptr;
  void *ya = nullptr, *yb = nullptr, *Fw = nullptr;
  auto cleanup = [&]() {
    for (void* q : {(void*)F64, (void*)S, (void*)ev, (void*)part, ya, yb, Fw})
      if (q) (void)hipFree(q);
  };
  int rc = TK_OK;
  if ((rc = dalloc((void**)&F64, sizeof(double) * fofs[N])) ||
      (rc = dalloc((void**)&S, sizeof(double) * Lmax * Lmax)) ||
      (rc = dalloc((void**)&ev, sizeof(double) * Kmax)) ||
      (rc = dalloc((void**)&part, sizeof(double) * gp)) ||
      (ymax > 0 && ((rc = dalloc(&ya, wsz * ymax)) || (rc = dalloc(&yb, wsz * ymax)))) ||
      (wdt == TK_F32 && (rc = dalloc(&Fw, sizeof(float) * Lmax * Kmax)))) {
    cleanup();
    return rc;
  }
  const void* Y = T_dev;
  int ydt = tdtype;
  pre = 0;
  for (int i = 0; i < N; ++i) {
    const int n = ord[i];
    int64_t A, Ln, B;
    view(s, pre, n, &A, &Ln, &B);
    hipError_t e = launch_gram(ydt, Y, A, Ln, B, S, part, st);
    if (e != hipSuccess) {
      cleanup();
      return fail(TK_EDEVICE, "STHOSVD Gram failed: %s", hipGetErrorString(e));
    }
    // synchronises; subspace iteration first, the gap-free solver if needed
    if ((rc = eig_solve(1, (int)Ln, (int)s.K[n], S, nullptr, F64 + fofs[n], ev, st, false))) {
      cleanup();
      return rc;
    }
    if (i + 1 == N) break;  // the last truncation would only form the core
    const void* Fn = F64 + fofs[n];
    if (wdt == TK_F32) {
      e = launch_convert(TK_F64, TK_F32, F64 + fofs[n], Fw, Ln * s.K[n], st);
      Fn = Fw;
    }
    void* Ynext = (i % 2 == 0) ? ya : yb;
    if (e == hipSuccess)
      e = launch_ttm(ydt, tcomp, Y, A, Ln, B, Fn, s.K[n], Ynext, st, true);
    if (e != hipSuccess) {
      cleanup();
      return fail(TK_EDEVICE, "STHOSVD truncation failed: %s", hipGetErrorString(e));
    }
    Y = Ynext;
    ydt = wdt;
    pre |= 1u << n;
  }
  std::vector<double> Fh(fofs[N]);
  hipError_t e = hipMemcpyAsync(Fh.data(), F64, sizeof(double) * fofs[N], hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  cleanup();
  if (e != hipSuccess) return fail(TK_EDEVICE, "STHOSVD readback failed: %s", hipGetErrorString(e));
  return hooi_init(N, L, K, tdtype, T_dev, plan, compute, Fh.data(), stream, out);
}

extern "C" int hooi_iterate(tk_ctx* c, int iters, double* rel_err) {
  clear_error();
  if (!c) return fail(TK_EINVAL, "ctx is null");
  Handoff handoff(c);
  if (iters < 1) return fail(TK_EINVAL, "iters=%d < 1", iters);
  if (int rc = ensure_scal(c, iters + 2)) return rc;
  // scal[0] = ||T||^2 (kept), scal[1 + t] = ||G^(t)||^2, t = 0..iters
  if (int rc = join_factors(c)) return rc;
  TK_HIP(launch_fill_int(c->status, c->s.N, 0, c->st));
  for (int t = 0; t < iters; ++t)
    if (int rc = tree_pass(c, 1 + t, false, nullptr, true)) return rc;
  if (int rc = join_factors(c)) return rc;
  if (int rc = core_chain(c, 1 + iters)) return rc;
  std::vector<double> g2(iters + 1);
  TK_HIP(hipMemcpyAsync(g2.data(), c->scal + 1, sizeof(double) * (iters + 1), hipMemcpyDeviceToHost,
                        c->st));
  if (int rc = check_status(c)) {  // synchronises
    // keep the factors the last pass started from (each was produced by a
    // converged solve) instead of adopting the failed update; the core of
    // that decomposition is formed again on demand
    std::swap(c->F64a, c->F64b);
    std::swap(c->Fc, c->Fcb);
    c->core_valid = false;
    return rc;
  }
  for (int t = 0; t < iters; ++t)
    if (rel_err) rel_err[t] = rel_err_of(c->normT2, g2[t + 1]);
  c->normG2 = g2[iters];
  c->core_valid = true;
  return TK_OK;
}

extern "C" int tucker_error(tk_ctx* c, double* rel_err, double* normT, double* normG) {
  clear_error();
  if (!c) return fail(TK_EINVAL, "ctx is null");
  Handoff handoff(c);
  if (int rc = join_factors(c)) return rc;
  if (!c->core_valid) {
    if (int rc = core_chain(c, 1)) return rc;
    double g2 = 0.0;
    TK_HIP(hipMemcpyAsync(&g2, c->scal + 1, sizeof(double), hipMemcpyDeviceToHost, c->st));
    TK_HIP(hipStreamSynchronize(c->st));
    c->normG2 = g2;
    c->core_valid = true;
  }
  if (rel_err) *rel_err = rel_err_of(c->normT2, c->normG2);
  if (normT) *normT = std::sqrt(c->normT2);
  if (normG) *normG = std::sqrt(c->normG2);
  return TK_OK;
}

extern "C" int tucker_error_explicit(tk_ctx* c, double* rel_err) {
  clear_error();
  if (!c || !rel_err) return fail(TK_EINVAL, "null argument");
  Handoff handoff(c);
  if (int rc = tucker_error(c, nullptr, nullptr, nullptr)) return rc;
  const Shape& s = c->s;
  const int N = s.N;
  // expand G along modes N-1 .. 1 in FP64: Zp has lengths K0, L1, ..., L_{N-1}
  int64_t big = s.K[0];
  for (int j = 1; j < N; ++j) big *= s.L[j];
  double *bufA = nullptr, *bufB = nullptr, *Ft = nullptr, *part = nullptr;
  int rc = TK_OK;
  if ((rc = dalloc((void**)&bufA, sizeof(double) * big))) return rc;
  if ((rc = dalloc((void**)&bufB, sizeof(double) * big))) {
    (void)hipFree(bufA);
    return rc;
  }
  size_t ftn = 0;
  for (int j = 0; j < N; ++j) ftn = std::max(ftn, (size_t)(s.L[j] * s.K[j]));
  if ((rc = dalloc((void**)&Ft, sizeof(double) * ftn)) ||
      (rc = dalloc((void**)&part, sizeof(double) * (sumsq_partials() + 1)))) {
    (void)hipFree(bufA);
    (void)hipFree(bufB);
    if (Ft) (void)hipFree(Ft);
    return rc;
  }
  auto cleanup = [&]() {
    (void)hipFree(bufA);
    (void)hipFree(bufB);
    (void)hipFree(Ft);
    (void)hipFree(part);
  };
  hipError_t e = launch_convert(c->wdtype, TK_F64, c->core, bufA, c->core_elems, c->st);
  std::vector<double> Fh, Fth;
  uint32_t kmask = (1u << N) - 1;  // modes still at length K
  double* cur = bufA;
  double* nxt = bufB;
  for (int j = N - 1; j >= 1 && e == hipSuccess; --j) {
    Fh.resize((size_t)(s.L[j] * s.K[j]));
    Fth.resize(Fh.size());
    e = hipMemcpyAsync(Fh.data(), c->F64a + c->fofs[j], sizeof(double) * Fh.size(),
                       hipMemcpyDeviceToHost, c->st);
    if (e != hipSuccess) break;
    e = hipStreamSynchronize(c->st);
    if (e != hipSuccess) break;
    // TTM with F_j (L_j x K_j): the kernel's factor argument is F_j^T (K_j x L_j)
    for (int64_t l = 0; l < s.L[j]; ++l)
      for (int64_t k = 0; k < s.K[j]; ++k) Fth[k * s.L[j] + l] = Fh[l * s.K[j] + k];
    e = hipMemcpyAsync(Ft, Fth.data(), sizeof(double) * Fth.size(), hipMemcpyHostToDevice, c->st);
    if (e != hipSuccess) break;
    int64_t A = 1, B = 1;
    for (int m = 0; m < N; ++m) {
      const int64_t d = ((kmask >> m) & 1u) ? s.K[m] : s.L[m];
      if (m < j) A *= d;
      if (m > j) B *= d;
    }
    e = launch_ttm(TK_F64, TK_C_FP64, cur, A, s.K[j], B, Ft, s.L[j], nxt, c->st);
    kmask &= ~(1u << j);
    std::swap(cur, nxt);
  }
  double r2 = 0.0;
  if (e == hipSuccess) {
    const int64_t R = big / s.K[0];
    e = launch_residual(c->tdtype, c->T, cur, c->F64a + c->fofs[0], (int)s.L[0], (int)s.K[0], R,
                        part, part + sumsq_partials(), c->st);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(&r2, part + sumsq_partials(), sizeof(double), hipMemcpyDeviceToHost,
                       c->st);
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  cleanup();
  if (e != hipSuccess) return fail(TK_EDEVICE, "explicit residual failed: %s", hipGetErrorString(e));
  *rel_err = std::sqrt(r2 / c->normT2);
  return TK_OK;
}

extern "C" int tk_get_factor(tk_ctx* c, int n, double* host) {
  clear_error();
  if (!c || !host) return fail(TK_EINVAL, "null argument");
  Handoff handoff(c);
  if (n < 0 || n >= c->s.N) return fail(TK_EINVAL, "mode %d out of range", n);
  if (int rc = join_factors(c)) return rc;
  TK_HIP(hipMemcpyAsync(host, c->F64a + c->fofs[n], sizeof(double) * (c->fofs[n + 1] - c->fofs[n]),
                        hipMemcpyDeviceToHost, c->st));
  TK_HIP(hipStreamSynchronize(c->st));
  return TK_OK;
}

extern "C" int tk_get_core(tk_ctx* c, double* host) {
  clear_error();
  if (!c || !host) return fail(TK_EINVAL, "null argument");
  Handoff handoff(c);
  if (int rc = tucker_error(c, nullptr, nullptr, nullptr)) return rc;
  if (c->wdtype == TK_F64) {
    TK_HIP(hipMemcpyAsync(host, c->core, sizeof(double) * c->core_elems, hipMemcpyDeviceToHost, c->st));
  } else {
    std::vector<float> tmp(c->core_elems);
    TK_HIP(hipMemcpyAsync(tmp.data(), c->core, sizeof(float) * c->core_elems, hipMemcpyDeviceToHost,
                          c->st));
    TK_HIP(hipStreamSynchronize(c->st));
    for (int64_t i = 0; i < c->core_elems; ++i) host[i] = tmp[i];
  }
  TK_HIP(hipStreamSynchronize(c->st));
  return TK_OK;
}

extern "C" int tk_set_factors(tk_ctx* c, const double* host) {
  clear_error();
  if (!c || !host) return fail(TK_EINVAL, "null argument");
  Handoff handoff(c);
  for (size_t i = 0; i < c->fofs[c->s.N]; ++i)
    if (!std::isfinite(host[i])) return fail(TK_ENUMERIC, "factors hold NaN/Inf");
  if (int rc = join_factors(c)) return rc;
  TK_HIP(hipMemcpyAsync(c->F64a, host, sizeof(double) * c->fofs[c->s.N], hipMemcpyHostToDevice, c->st));
  if (int rc = refresh_compute_factors(c)) return rc;
  TK_HIP(hipStreamSynchronize(c->st));
  c->core_valid = false;
  return TK_OK;
}

extern "C" int tk_tree_pass(tk_ctx* c) {
  clear_error();
  if (!c) return fail(TK_EINVAL, "ctx is null");
  Handoff handoff(c);
  const Shape& s = c->s;
  if (c->leaves.empty()) {
    c->leaves.assign(s.N, nullptr);
    c->leaf_elems.assign(s.N, 0);
    for (int n = 0; n < s.N; ++n) {
      c->leaf_elems[n] = (int64_t)s.card(((1u << s.N) - 1) & ~(1u << n));
      if (int rc = dalloc(&c->leaves[n], (size_t)c->leaf_elems[n] * 8)) return rc;
    }
  }
  if (int rc = join_factors(c)) return rc;
  if (int rc = tree_pass(c, -1, true, nullptr)) return rc;
  TK_HIP(hipStreamSynchronize(c->st));
  return TK_OK;
}

extern "C" int tk_get_leaf(tk_ctx* c, int n, double* host) {
  clear_error();
  if (!c || !host) return fail(TK_EINVAL, "null argument");
  Handoff handoff(c);
  if (n < 0 || n >= c->s.N) return fail(TK_EINVAL, "mode %d out of range", n);
  if (c->leaves.empty()) return fail(TK_EINVAL, "call tk_tree_pass first");
  const int64_t m = c->leaf_elems[n];
  // a leaf holds its parent's output type (T's own when it hangs off the root)
  int dt = c->wdtype;
  for (size_t u = 0; u < c->tree.nodes.size(); ++u)
    if (c->tree.nodes[u].is_leaf && c->tree.nodes[u].mode == n) dt = c->in_dtype_of((int)u);
  if (dt == TK_F64) {
    TK_HIP(hipMemcpy(host, c->leaves[n], sizeof(double) * m, hipMemcpyDeviceToHost));
  } else if (dt == TK_F32) {
    std::vector<float> tmp(m);
    TK_HIP(hipMemcpy(tmp.data(), c->leaves[n], sizeof(float) * m, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < m; ++i) host[i] = tmp[i];
  } else {
    std::vector<uint16_t> tmp(m);
    TK_HIP(hipMemcpy(tmp.data(), c->leaves[n], sizeof(uint16_t) * m, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < m; ++i) {
      uint32_t u = (uint32_t)tmp[i] << 16;
      float f;
      memcpy(&f, &u, 4);
      host[i] = f;
    }
  }
  return TK_OK;
}

extern "C" int tk_get_gram(tk_ctx* c, int n, double* host) {
  clear_error();
  if (!c || !host) return fail(TK_EINVAL, "null argument");
  Handoff handoff(c);
  if (n < 0 || n >= c->s.N) return fail(TK_EINVAL, "mode %d out of range", n);
  TK_HIP(hipMemcpyAsync(host, c->S + c->sofs[n], sizeof(double) * (c->sofs[n + 1] - c->sofs[n]),
                        hipMemcpyDeviceToHost, c->st));
  TK_HIP(hipStreamSynchronize(c->st));
  return TK_OK;
}

extern "C" int tk_profile_tree(tk_ctx* c, float* ms_out, int cap, int* n) {
  clear_error();
  if (!c || !n) return fail(TK_EINVAL, "null argument");
  Handoff handoff(c);
  const size_t nn = c->tree.nodes.size();
  *n = (int)nn;
  if (!ms_out) return TK_OK;
  std::vector<hipEvent_t> ev(2 * nn);
  for (auto& e : ev) TK_HIP(hipEventCreate(&e));
  int rc = join_factors(c);
  if (rc == TK_OK) rc = tree_pass(c, -1, false, ev.data());
  if (rc == TK_OK) {
    hipError_t e = hipEventSynchronize(ev.back());
    if (e != hipSuccess) rc = fail(TK_EDEVICE, "profile sync: %s", hipGetErrorString(e));
  }
  for (size_t u = 0; rc == TK_OK && u < nn && (int)u < cap; ++u) {
    float ms = 0.f;
    hipError_t e = hipEventElapsedTime(&ms, ev[2 * u], ev[2 * u + 1]);
    if (e != hipSuccess) rc = fail(TK_EDEVICE, "event time: %s", hipGetErrorString(e));
    ms_out[u] = ms;
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  return rc;
}

extern "C" int tk_eig_iterations(tk_ctx* c, int* out) {
  clear_error();
  if (!c || !out) return fail(TK_EINVAL, "null argument");
  Handoff handoff(c);
  TK_HIP(hipMemcpyAsync(out, c->status + c->s.N, sizeof(int) * c->s.N, hipMemcpyDeviceToHost,
                        c->st));
  TK_HIP(hipStreamSynchronize(c->st));
  return TK_OK;
}

extern "C" void hooi_free(tk_ctx* c) { delete c; }

// ---------------------------------------------------------------- kernel-level entry points --
extern "C" int tk_ttm(int in_dtype, int compute, const void* in, int64_t A, int64_t L, int64_t B,
                      const void* F, int64_t K, void* out, void* stream) {
  clear_error();
  if (!in || !F || !out) return fail(TK_EINVAL, "null pointer");
  if (A < 1 || L < 1 || B < 1 || K < 1) return fail(TK_EINVAL, "sizes must be >= 1");
  if (in_dtype < TK_F64 || in_dtype > TK_F16) return fail(TK_EINVAL, "unknown dtype %d", in_dtype);
  if (compute == TK_C_FP64) {
    if (in_dtype != TK_F64) return fail(TK_EUNSUPPORTED, "FP64 compute needs FP64 input");
    if (L > 512) return fail(TK_EUNSUPPORTED, "FP64 TTM supports L <= 512");
  } else if (compute >= TK_C_FP32 && compute <= TK_C_BF16X3) {
    if (in_dtype == TK_F64)
      return fail(TK_EUNSUPPORTED, "compute mode %d takes F32/BF16/F16 input", compute);
    if (in_dtype == TK_F16 && compute != TK_C_FP32)
      return fail(TK_EUNSUPPORTED, "FP16 input takes FP32 compute only");
    if (L > ttm_max_L()) return fail(TK_EUNSUPPORTED, "L=%lld exceeds %d", (long long)L, ttm_max_L());
  } else {
    return fail(TK_EINVAL, "unknown compute mode %d", compute);
  }
  if (K > 4096) return fail(TK_EUNSUPPORTED, "K > 4096");
  if (A * B > ((int64_t)1 << 40)) return fail(TK_EINVAL, "tensor too large");
  TK_HIP(launch_ttm(in_dtype, compute, in, A, L, B, F, K, out, (hipStream_t)stream));
  return TK_OK;
}

extern "C" int tk_ttm_pair(int in_dtype, int compute, const void* in, int64_t A, int64_t Lp,
                           int64_t M, int64_t Lq, int64_t B, const void* Fp, int64_t Kp,
                           const void* Fq, int64_t Kq, void* outp, void* outq, void* stream) {
  clear_error();
  if (!in || !Fp || !Fq || !outp || !outq) return fail(TK_EINVAL, "null pointer");
  if (A < 1 || Lp < 1 || M < 1 || Lq < 1 || B < 1 || Kp < 1 || Kq < 1 || Kp > Lp || Kq > Lq)
    return fail(TK_EINVAL, "bad sizes");
  if (!ttm_pair_applies(in_dtype, compute, in, A, Lp, M, Lq, B, Kp, Kq, outp, outq))
    return fail(TK_EUNSUPPORTED,
                "fused pair needs FP32 input and compute, 16-byte aligned buffers and "
                "either the two trailing modes (M = B = 1) with Lq %% 4 == 0, Lq <= 256, "
                "K <= 20, or B %% 4 == 0, Lq <= 256, K <= 20 and at least 2048 tiles of "
                "four columns");
  TK_HIP(launch_ttm_pair((const float*)in, A, Lp, M, Lq, B, (const float*)Fp, Kp,
                         (const float*)Fq, Kq, (float*)outp, (float*)outq, (hipStream_t)stream));
  return TK_OK;
}

extern "C" int tk_gram(int in_dtype, const void* Y, int64_t A, int64_t L, int64_t B, double* S,
                       void* stream) {
  clear_error();
  if (!Y || !S) return fail(TK_EINVAL, "null pointer");
  if (A < 1 || L < 1 || B < 1) return fail(TK_EINVAL, "sizes must be >= 1");
  if (L > 1024) return fail(TK_EUNSUPPORTED, "L > 1024");
  if (in_dtype < TK_F64 || in_dtype > TK_F16) return fail(TK_EINVAL, "unknown dtype %d", in_dtype);
  const size_t gp = gram_workspace_elems(L, A * B);
  double* part = nullptr;
  if (int rc = dalloc((void**)&part, sizeof(double) * gp)) return rc;
  hipError_t e = launch_gram(in_dtype, Y, A, L, B, S, part, (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  (void)hipFree(part);
  if (e != hipSuccess) return fail(TK_EDEVICE, "gram: %s", hipGetErrorString(e));
  return TK_OK;
}

namespace {

// count matrices: subspace iteration (unless full_only or K above its block
// limit), then the gap-free solver for every matrix that needs it.
int eig_solve(int count, int L, int K, const double* S, const double* V0, double* F,
              double* evals, hipStream_t st, bool full_only) {
  if (!S || !F || !evals) return fail(TK_EINVAL, "null pointer");
  if (count < 1 || L < 1 || K < 1 || K > L) return fail(TK_EINVAL, "bad sizes");
  if (L > eig_full_max_L()) return fail(TK_EUNSUPPORTED, "L <= %d required", eig_full_max_L());
  const bool subspace = !full_only && K <= eig_max_K() && L <= 1024;
  const int p = eig_block_size(L, K, L);
  std::vector<EigJob> jobs(subspace ? count : 0);
  std::vector<EigFullJob> fjobs(count);
  for (int m = 0; m < count; ++m) {
    if (subspace) {
      EigJob& j = jobs[m];
      j.L = L;
      j.K = K;
      j.p = p;
      j.pad_ = 0;
      j.S_off = (int64_t)m * L * L;
      j.V0_off = V0 ? (int64_t)m * L * K : -1;
      j.F_off = (int64_t)m * L * K;
      j.ev_off = (int64_t)m * K;
      j.work_off = (int64_t)(m * eig_work_elems(L, p));
    }
    EigFullJob& f = fjobs[m];
    f.L = L;
    f.K = K;
    f.status_idx = m;
    f.only_if_failed = subspace ? 1 : 0;
    f.S_off = (int64_t)m * L * L;
    f.F_off = (int64_t)m * L * K;
    f.ev_off = (int64_t)m * K;
    f.work_off = (int64_t)(m * eig_full_work_elems(L));
  }
  EigJob* jd = nullptr;
  EigFullJob* fd = nullptr;
  double *work = nullptr, *fwork = nullptr;
  int* status = nullptr;
  int rc = TK_OK;
  auto cleanup = [&]() {
    for (void* q : {(void*)jd, (void*)fd, (void*)work, (void*)fwork, (void*)status})
      if (q) (void)hipFree(q);
  };
  if ((subspace && ((rc = dalloc((void**)&jd, sizeof(EigJob) * count)) ||
                    (rc = dalloc((void**)&work, sizeof(double) * eig_work_elems(L, p) * count)))) ||
      (rc = dalloc((void**)&fd, sizeof(EigFullJob) * count)) ||
      (rc = dalloc((void**)&fwork, sizeof(double) * eig_full_work_elems(L) * count)) ||
      (rc = dalloc((void**)&status, sizeof(int) * count))) {
    cleanup();
    return rc;
  }
  std::vector<int> sth(count, 0);
  hipError_t e = hipMemcpyAsync(fd, fjobs.data(), sizeof(EigFullJob) * count,
                                hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_fill_int(status, count, 0, st);
  if (subspace) {
    if (e == hipSuccess)
      e = hipMemcpyAsync(jd, jobs.data(), sizeof(EigJob) * count, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = launch_eig(count, jd, 0, L, p, S, V0, F, evals, work, status, nullptr, V0 ? 20 : 100,
                     1e-11, st);
  }
  if (e == hipSuccess) e = launch_eig_full(count, fd, L, K, S, F, evals, fwork, status, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(sth.data(), status, sizeof(int) * count, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  cleanup();
  if (e != hipSuccess) return fail(TK_EDEVICE, "eig: %s", hipGetErrorString(e));
  for (int m = 0; m < count; ++m)
    if (sth[m] != 0) return fail(TK_ENUMERIC, "eigensolver status %d for matrix %d", sth[m], m);
  return TK_OK;
}

}  // namespace

extern "C" int tk_eig_leading(int count, int L, int K, const double* S, const double* V0, double* F,
                              double* evals, void* stream) {
  clear_error();
  return eig_solve(count, L, K, S, V0, F, evals, (hipStream_t)stream, false);
}

extern "C" int tk_eig_full(int count, int L, int K, const double* S, double* F, double* evals,
                           void* stream) {
  clear_error();
  return eig_solve(count, L, K, S, nullptr, F, evals, (hipStream_t)stream, true);
}
