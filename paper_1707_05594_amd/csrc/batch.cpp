// Batched HOOI: one invocation (Sec. 2.2, Jacobi form) over many independent
// tensors at once, each with its own minimum-cost TTM-tree (Sec. 3.3).
//
// The tree nodes of all tensors are grouped by depth.  Each depth is one
// launch of a persistent grouped TTM kernel that drains a device queue of
// (node, tile) items, so thousands of small TTMs cost one launch per tree
// level instead of one per node.  The leaves' Grams (Sec. 5) are one grouped
// launch, all eigensolves one batched launch, the folded cores one grouped
// TTM plus one segmented norm.  One iteration is captured in a HIP graph and
// replayed; the persistent grid size is chosen by timing (hooi_batch_tune).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <new>
#include <vector>

#include "internal.h"
#include "kernels.h"

using namespace tk;

namespace {

int64_t align64(int64_t x) { return (x + 63) & ~(int64_t)63; }

template <typename P>
int dalloc_t(P** p, size_t count) {
  *p = nullptr;
  const size_t bytes = std::max<size_t>(count * sizeof(P), 16);
  if (hipMalloc((void**)p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(TK_ENOMEM, "hipMalloc(%zu bytes) failed", bytes);
  }
  return TK_OK;
}

template <typename P>
int upload(P** dev, const std::vector<P>& host, hipStream_t st) {
  if (int rc = dalloc_t(dev, host.size())) return rc;
  if (!host.empty())
    TK_HIP(hipMemcpyAsync(*dev, host.data(), sizeof(P) * host.size(), hipMemcpyHostToDevice, st));
  return TK_OK;
}

struct Launch {
  int in_dtype = TK_F32;
  int node0 = 0, item0 = 0, n_items = 0;
  int Lmax = 1;
  // items of the odd-L row nodes (kGroupedRowsScalar), right after the others:
  // [ritem0, ritem0 + n_ritems).  The autotuner decides whether they join the
  // shared queue (one launch over both ranges, the shared kernel's row body)
  // or run in a persistent launch of their own (the barrier-free row body).
  int ritem0 = 0, n_ritems = 0, rLmax = 1;
};

}  // namespace

struct tk_batch {
  int count = 0;
  int tdtype = TK_F32;
  std::vector<Shape> shapes;
  std::vector<Tree> trees;
  std::vector<int> fold_leaf;
  std::vector<const void*> T;
  std::vector<double> normT2;
  hipStream_t user = nullptr, st = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // eigensolve classes run concurrently: forked from `st` onto kAux streams
  // (default priority) and joined back before the factor update
  static constexpr int kAux = 4;
  hipStream_t aux[kAux] = {};
  hipEvent_t ev_fork = nullptr, ev_join[kAux] = {};
  int ncu = 256;
  int blocks_per_cu = 4;
  // odd-length row items in a launch of their own (true) or in the shared
  // queue; set by hooi_batch_tune from measured passes.  Untuned default:
  // separate for BF16 storage (the shared body's 2-byte loads are slow).
  bool split_rows = false;

  // factor layout: tensor i, mode n at fofs[i][n] (elements)
  std::vector<std::vector<int64_t>> fofs, sofs, kofs;
  int64_t nF = 0, nS = 0, nK = 0;

  float* ws = nullptr;
  float* Fc = nullptr;
  double* F64a = nullptr;
  double* F64b = nullptr;
  double* S = nullptr;
  double* ev = nullptr;
  double* eigwork = nullptr;
  double* basis = nullptr;  // full eigenbases of the p = L solves (EigJob::basis_off)
  std::vector<EigJob> jobs_h;  // job table (host copy), to restore identity bases
  int* status = nullptr;
  EigJob* jobs_warm = nullptr;
  EigJob* jobs_cold = nullptr;
  int n_jobs = 0, Lmax = 0, pmax = 0;
  // jobs sorted by padded block width: one launch per class, so narrow solves
  // do not run at the widest width (warm and cold tables share the order)
  struct EigClass {
    int job0, count, Lmax, pmax;
  };
  std::vector<EigClass> warm_classes, cold_classes;
  // gap-free solver (eigfull.hip) for the subspace jobs (L > 64) whose solve
  // did not converge: one conditional launch after the eigensolve classes
  EigFullJob* fjobs = nullptr;
  double* fwork = nullptr;
  int n_fjobs = 0, fLmax = 0, fKmax = 0;
  float* core = nullptr;
  int64_t* core_off = nullptr;
  double* normG2 = nullptr;
  double* normT2_dev = nullptr;
  double* sumsq_part = nullptr;

  TtmNodeDesc* ttm_nodes = nullptr;
  int2* ttm_items = nullptr;
  int* counters = nullptr;
  std::vector<Launch> levels;
  Launch fold;

  GramDesc* gram = nullptr;
  int4* gram_items = nullptr;
  int64_t* gram_off = nullptr;
  double* gpart = nullptr;
  int n_gram_items = 0, n_gram = 0;
  int64_t gram_total = 0;

  uint64_t tree_macs = 0, tree_bytes = 0;

  bool use_graph = true;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;

  ~tk_batch() {
    if (st) (void)hipStreamSynchronize(st);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    void* ptrs[] = {ws,        Fc,        F64a,       F64b,     S,          ev,
                    eigwork,   basis,     status,     jobs_warm, jobs_cold, core,
                    core_off,  normG2,    normT2_dev, sumsq_part, ttm_nodes, ttm_items,
                    counters,  gram,      gram_items, gram_off,  gpart,     fjobs,
                    fwork};
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
    if (st) (void)hipStreamDestroy(st);
    for (int k = 0; k < kAux; ++k) {
      if (aux[k]) (void)hipStreamDestroy(aux[k]);
      if (ev_join[k]) (void)hipEventDestroy(ev_join[k]);
    }
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
  }
};

namespace {

struct Handoff {
  tk_batch* b;
  explicit Handoff(tk_batch* bb) : b(bb) {
    (void)hipEventRecord(b->ev_in, b->user);
    (void)hipStreamWaitEvent(b->st, b->ev_in, 0);
  }
  ~Handoff() {
    (void)hipEventRecord(b->ev_out, b->st);
    (void)hipStreamWaitEvent(b->user, b->ev_out, 0);
  }
};

int grid_blocks(const tk_batch* b) { return b->ncu * b->blocks_per_cu; }

// Tree levels, folded cores, their norms and the leaves' Grams (no eigensolve).
int enqueue_pass(tk_batch* b) {
  const int nl = (int)b->levels.size();
  TK_HIP(launch_fill_int(b->counters, 2 * (nl + 1), 0, b->st));
  // items hold indices into the whole node table; each launch has two queue
  // heads (its other items, then its odd-L row items)
  auto run = [&](const Launch& l, int q, bool stream_in) -> hipError_t {
    if (!b->split_rows)  // one queue over both ranges (they are adjacent)
      return launch_ttm_grouped(l.in_dtype, b->ttm_nodes, b->ttm_items + l.item0,
                                l.n_items + l.n_ritems, b->counters + 2 * q,
                                std::max(l.Lmax, l.rLmax), grid_blocks(b), stream_in, b->st);
    hipError_t e = launch_ttm_grouped(l.in_dtype, b->ttm_nodes, b->ttm_items + l.item0,
                                      l.n_items, b->counters + 2 * q, l.Lmax, grid_blocks(b),
                                      stream_in, b->st);
    if (e == hipSuccess)
      e = launch_ttm_grouped_rows(l.in_dtype, b->ttm_nodes, b->ttm_items + l.ritem0, l.n_ritems,
                                  b->counters + 2 * q + 1, l.rLmax, grid_blocks(b), stream_in,
                                  b->st);
    return e;
  };
  for (int d = 0; d < nl; ++d) TK_HIP(run(b->levels[d], d, d == 0));
  TK_HIP(run(b->fold, nl, false));
  TK_HIP(launch_sumsq_segments(b->core, b->core_off, b->count, b->normG2, b->st));
  TK_HIP(launch_gram_grouped(TK_F32, b->gram, b->gram_items, b->n_gram_items, b->gram_off,
                             b->n_gram, b->gram_total, b->st));
  return TK_OK;
}

// One HOOI invocation for every tensor: pass, warm eigensolves, factor update.
int enqueue_iteration(tk_batch* b) {
  if (int rc = enqueue_pass(b)) return rc;
  // classes touch disjoint jobs (S, work areas, bases, outputs): fork them over
  // the auxiliary streams so that small classes share the chip
  const int nc = (int)b->warm_classes.size();
  const int used = std::min(nc, (int)tk_batch::kAux);
  if (used > 0) TK_HIP(hipEventRecord(b->ev_fork, b->st));
  for (int k = 0; k < used; ++k) TK_HIP(hipStreamWaitEvent(b->aux[k], b->ev_fork, 0));
  for (int q = 0; q < nc; ++q) {
    const auto& c = b->warm_classes[q];
    TK_HIP(launch_eig(c.count, b->jobs_warm, c.job0, c.Lmax, c.pmax, b->S, b->F64a, b->F64b,
                      b->ev, b->eigwork, b->status, nullptr, 20, 1e-11,
                      b->aux[q % tk_batch::kAux], b->basis));
  }
  for (int k = 0; k < used; ++k) {
    TK_HIP(hipEventRecord(b->ev_join[k], b->aux[k]));
    TK_HIP(hipStreamWaitEvent(b->st, b->ev_join[k], 0));
  }
  TK_HIP(launch_eig_full(b->n_fjobs, b->fjobs, b->fLmax, b->fKmax, b->S, b->F64b, b->ev,
                         b->fwork, b->status, b->st));
  TK_HIP(launch_copy_f64(b->F64b, b->F64a, b->nF, b->st));
  TK_HIP(launch_convert(TK_F64, TK_F32, b->F64a, b->Fc, b->nF, b->st));
  return TK_OK;
}

int build_graph(tk_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  TK_HIP(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
  int rc = enqueue_iteration(b);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->st, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(TK_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
  b->graph = g;
  TK_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
  return TK_OK;
}

int check_status(tk_batch* b) {
  std::vector<int> st(b->n_jobs);
  TK_HIP(hipMemcpyAsync(st.data(), b->status, sizeof(int) * b->n_jobs, hipMemcpyDeviceToHost, b->st));
  TK_HIP(hipStreamSynchronize(b->st));
  for (int j = 0; j < b->n_jobs; ++j)
    if (st[j] != 0)
      return fail(TK_ENUMERIC, "eigensolver %s for job %d", st[j] == 2 ? "saw NaN/Inf" : "did not converge", j);
  return TK_OK;
}

}  // namespace

extern "C" int hooi_batch_init(int count, const int* N, const int64_t* L, const int64_t* K,
                               int tdtype, const void* const* T_dev, int compute, void* stream,
                               tk_batch** out) {
  clear_error();
  if (!out || !N || !L || !K || !T_dev) return fail(TK_EINVAL, "null pointer");
  *out = nullptr;
  if (count < 1) return fail(TK_EINVAL, "count=%d < 1", count);
  if (tdtype != TK_F32 && tdtype != TK_BF16) return fail(TK_EUNSUPPORTED, "storage must be F32 or BF16");
  if (compute != TK_C_FP32) return fail(TK_EUNSUPPORTED, "batched HOOI computes in FP32");
  tk_batch* b = new (std::nothrow) tk_batch;
  if (!b) return fail(TK_ENOMEM, "batch allocation failed");
  auto bail = [&](int rc) {
    delete b;
    return rc;
  };
  b->count = count;
  b->tdtype = tdtype;
  b->split_rows = tdtype == TK_BF16;
  b->user = (hipStream_t)stream;
  {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      return bail(fail(TK_EDEVICE, "stream/event creation failed"));
    }
    for (int k = 0; k < tk_batch::kAux; ++k)
      if (hipStreamCreateWithFlags(&b->aux[k], hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&b->ev_join[k], hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return bail(fail(TK_EDEVICE, "stream/event creation failed"));
      }
  }
  // ---- shapes and plans (one DP plan per distinct shape)
  std::map<std::vector<int64_t>, Tree> plans;
  int64_t off = 0;
  for (int i = 0; i < count; ++i) {
    Shape s;
    if (N[i] < 2 || N[i] > TK_MAX_MODES) return bail(fail(TK_EINVAL, "tensor %d: N=%d", i, N[i]));
    if (int rc = make_shape(N[i], L + off, K + off, &s)) return bail(rc);
    for (int j = 0; j < s.N; ++j) {
      if (s.K[j] > 16) return bail(fail(TK_EUNSUPPORTED, "tensor %d: K > 16", i));
      if (s.L[j] > 512) return bail(fail(TK_EUNSUPPORTED, "tensor %d: L > 512", i));
    }
    if (!T_dev[i]) return bail(fail(TK_EINVAL, "tensor %d: null pointer", i));
    std::vector<int64_t> key(L + off, L + off + s.N);
    key.insert(key.end(), K + off, K + off + s.N);
    auto it = plans.find(key);
    if (it == plans.end()) {
      tk_plan* p = nullptr;
      if (int rc = ttm_tree_plan(s.N, L + off, K + off, TK_TREE_DP, 1, &p)) return bail(rc);
      it = plans.emplace(key, p->trees[0]).first;
      tk_plan_free(p);
    }
    b->shapes.push_back(s);
    b->trees.push_back(it->second);
    b->T.push_back(T_dev[i]);
    off += s.N;
  }
  hipStream_t st = b->st;
  // the caller's stream may still be producing the tensors (init ends with a
  // synchronisation of st, which orders everything after it)
  if (hipEventRecord(b->ev_in, b->user) != hipSuccess ||
      hipStreamWaitEvent(st, b->ev_in, 0) != hipSuccess) {
    (void)hipGetLastError();
    return bail(fail(TK_EDEVICE, "stream ordering failed"));
  }

  // ---- factor, Gram, eigenvalue layouts
  b->fofs.resize(count);
  b->sofs.resize(count);
  b->kofs.resize(count);
  for (int i = 0; i < count; ++i) {
    const Shape& s = b->shapes[i];
    for (int n = 0; n < s.N; ++n) {
      b->fofs[i].push_back(b->nF);
      b->sofs[i].push_back(b->nS);
      b->kofs[i].push_back(b->nK);
      b->nF += s.L[n] * s.K[n];
      b->nS += s.L[n] * s.L[n];
      b->nK += s.K[n];
    }
  }

  // ---- node outputs (every internal node of every tensor) and cores
  std::vector<std::vector<int64_t>> node_off(count);
  int64_t ws = 0, core_elems = 0;
  std::vector<int64_t> core_off_h(count + 1, 0);
  int depth_max = 0;
  for (int i = 0; i < count; ++i) {
    const auto& nodes = b->trees[i].nodes;
    node_off[i].assign(nodes.size(), -1);
    for (size_t u = 0; u < nodes.size(); ++u) {
      if (nodes[u].is_leaf) continue;
      node_off[i][u] = ws;
      ws = align64(ws + (int64_t)nodes[u].out_card);
      depth_max = std::max(depth_max, (int)nodes[u].depth);
      b->tree_macs += nodes[u].macs;
    }
    const Shape& s = b->shapes[i];
    int best = 0;
    int64_t best_y = -1;
    for (int n = 0; n < s.N; ++n) {
      const int64_t y = (int64_t)s.card(((1u << s.N) - 1) & ~(1u << n));
      if (best_y < 0 || y < best_y) {
        best_y = y;
        best = n;
      }
    }
    b->fold_leaf.push_back(best);
    // cores back to back: core i is the segment [core_off_h[i], core_off_h[i + 1])
    int64_t ce = 1;
    for (int n = 0; n < s.N; ++n) ce *= s.K[n];
    core_off_h[i + 1] = core_off_h[i] + ce;
  }
  core_elems = core_off_h[count];
  int rc = TK_OK;
  if ((rc = dalloc_t(&b->ws, (size_t)ws)) || (rc = dalloc_t(&b->Fc, (size_t)b->nF)) ||
      (rc = dalloc_t(&b->F64a, (size_t)b->nF)) || (rc = dalloc_t(&b->F64b, (size_t)b->nF)) ||
      (rc = dalloc_t(&b->S, (size_t)b->nS)) || (rc = dalloc_t(&b->ev, (size_t)b->nK)) ||
      (rc = dalloc_t(&b->core, (size_t)core_elems)) || (rc = dalloc_t(&b->normG2, (size_t)count)) ||
      (rc = dalloc_t(&b->normT2_dev, (size_t)count)) ||
      (rc = dalloc_t(&b->sumsq_part, (size_t)sumsq_partials() + 1)))
    return bail(rc);

  // ---- grouped TTM tables: tree levels, then the folded cores
  std::vector<TtmNodeDesc> nd_h;
  std::vector<int2> it_h, it_rows;  // it_rows: the current launch's odd-L row items
  std::vector<int64_t> node_tiles;
  auto add_node = [&](const void* in, int in_bytes, float* outp, const float* F, int64_t A,
                      int64_t Ln, int64_t B, int64_t Kn) {
    TtmNodeDesc d;
    d.in = in;
    d.out = outp;
    d.F = F;
    d.A = A;
    d.B = B;
    d.L = (int)Ln;
    d.K = (int)Kn;
    d.lines = 0;
    int64_t tiles = 0;
    ttm_grouped_geometry(in, outp, in_bytes, A, Ln, B, &d, &tiles);
    const int idx = (int)nd_h.size();
    nd_h.push_back(d);
    node_tiles.push_back(tiles);
    auto& dst = d.path == kGroupedRowsScalar ? it_rows : it_h;
    for (int64_t t = 0; t < tiles; ++t) dst.push_back(make_int2(idx, (int)t));
  };
  // close a launch: its odd-L row items go after its other items
  auto close_launch = [&](Launch& l) {
    l.n_items = (int)it_h.size() - l.item0;
    l.ritem0 = (int)it_h.size();
    l.n_ritems = (int)it_rows.size();
    it_h.insert(it_h.end(), it_rows.begin(), it_rows.end());
    it_rows.clear();
  };
  for (int dpt = 0; dpt <= depth_max; ++dpt) {
    Launch l;
    l.in_dtype = dpt == 0 ? tdtype : TK_F32;
    l.node0 = (int)nd_h.size();
    l.item0 = (int)it_h.size();
    for (int i = 0; i < count; ++i) {
      const Shape& s = b->shapes[i];
      const auto& nodes = b->trees[i].nodes;
      for (size_t u = 0; u < nodes.size(); ++u) {
        const tk_node& nd = nodes[u];
        if (nd.is_leaf || (int)nd.depth != dpt) continue;
        int64_t A, Ln, B;
        view(s, nd.pre_mask, nd.mode, &A, &Ln, &B);
        const void* in = nd.parent < 0 ? b->T[i] : (const void*)(b->ws + node_off[i][nd.parent]);
        const int in_bytes = (nd.parent < 0 && tdtype == TK_BF16) ? 2 : 4;
        add_node(in, in_bytes, b->ws + node_off[i][u], b->Fc + b->fofs[i][nd.mode], A, Ln, B,
                 s.K[nd.mode]);
        b->tree_bytes += (uint64_t)nd.in_card * (nd.parent < 0 && tdtype == TK_BF16 ? 2 : 4) +
                         (uint64_t)nd.out_card * 4;
        if (nd_h.back().path == kGroupedRowsScalar)
          l.rLmax = std::max<int>(l.rLmax, (int)Ln);
        else
          l.Lmax = std::max<int>(l.Lmax, (int)Ln);
      }
    }
    close_launch(l);
    b->levels.push_back(l);
  }
  {
    Launch& f = b->fold;
    f.in_dtype = TK_F32;
    f.node0 = (int)nd_h.size();
    f.item0 = (int)it_h.size();
    for (int i = 0; i < count; ++i) {
      const Shape& s = b->shapes[i];
      const auto& nodes = b->trees[i].nodes;
      const int m = b->fold_leaf[i];
      for (size_t u = 0; u < nodes.size(); ++u) {
        const tk_node& nd = nodes[u];
        if (!nd.is_leaf || nd.mode != m) continue;
        int64_t A, Ln, B;
        view(s, nd.pre_mask, m, &A, &Ln, &B);
        add_node(b->ws + node_off[i][nd.parent], 4, b->core + core_off_h[i],
                 b->Fc + b->fofs[i][m], A, Ln, B, s.K[m]);
        if (nd_h.back().path == kGroupedRowsScalar)
          f.rLmax = std::max<int>(f.rLmax, (int)Ln);
        else
          f.Lmax = std::max<int>(f.Lmax, (int)Ln);
      }
    }
    close_launch(f);
  }
  // host check of every descriptor and item against the buffers it names
  {
    auto inside = [](const void* p, int64_t n, int64_t esz, const void* base, int64_t cap) {
      const char* a = (const char*)p;
      const char* lo = (const char*)base;
      return a >= lo && a + n * esz <= lo + cap * esz;
    };
    for (const TtmNodeDesc& d : nd_h) {
      bool in_ok = inside(d.in, d.A * d.L * d.B, 4, b->ws, ws);
      for (int i = 0; i < count && !in_ok; ++i)
        in_ok = inside(d.in, d.A * d.L * d.B, tdtype == TK_BF16 ? 2 : 4, b->T[i],
                       (int64_t)b->shapes[i].card_T());
      const bool out_ok = inside(d.out, d.A * d.K * d.B, 4, b->ws, ws) ||
                          inside(d.out, d.A * d.K * d.B, 4, b->core, core_elems);
      const bool f_ok = inside(d.F, (int64_t)d.L * d.K, 4, b->Fc, b->nF);
      if (!in_ok || !out_ok || !f_ok || d.K > 16 || d.L < 1)
        return bail(fail(TK_EINVAL, "internal: TTM descriptor outside its buffers"));
    }
    for (const int2& w : it_h) {
      if (w.x < 0 || w.x >= (int)nd_h.size()) return bail(fail(TK_EINVAL, "internal: item node"));
      if (w.y < 0 || (int64_t)w.y >= node_tiles[w.x])
        return bail(fail(TK_EINVAL, "internal: item tile"));
    }
    for (const TtmNodeDesc& d : nd_h)
      if ((d.path == kGroupedRows &&
           (d.B != 1 || d.L % 4 != 0 || d.L > ttm_grouped_row_stage_max_L())) ||
          (d.path == kGroupedRowsDirect && (d.B != 1 || d.L % 4 != 0)) ||
          (d.path == kGroupedRowsScalar && (d.B != 1 || d.L > ttm_grouped_row_stage_max_L())) ||
          (d.path == kGroupedWideScalar && d.B < 32))
        return bail(fail(TK_EINVAL, "internal: row body on an unsuitable node"));
  }
  if ((rc = upload(&b->ttm_nodes, nd_h, st)) || (rc = upload(&b->ttm_items, it_h, st)) ||
      (rc = dalloc_t(&b->counters, 2 * (b->levels.size() + 1))))
    return bail(rc);

  // ---- grouped Grams of the leaves
  std::vector<GramDesc> gd;
  std::vector<int4> gi;
  std::vector<int64_t> goff(1, 0);
  int64_t gpart = 0;
  for (int i = 0; i < count; ++i) {
    const Shape& s = b->shapes[i];
    const auto& nodes = b->trees[i].nodes;
    for (int n = 0; n < s.N; ++n) {
      for (size_t u = 0; u < nodes.size(); ++u) {
        const tk_node& nd = nodes[u];
        if (!nd.is_leaf || nd.mode != n) continue;
        int64_t A, Ln, B;
        view(s, nd.pre_mask, n, &A, &Ln, &B);
        GramDesc d;
        gram_geometry(Ln, A * B, 8, &d);
        d.Y = b->ws + node_off[i][nd.parent];
        d.B = B;
        d.S = b->S + b->sofs[i][n];
        d.part = nullptr;  // set after the total is known
        const int m = (int)gd.size();
        gd.push_back(d);
        for (int c = 0; c < d.nchunks; ++c)
          for (int p = 0; p < d.npairs; ++p) gi.push_back(make_int4(m, c, p, 0));
        goff.push_back(goff.back() + Ln * Ln);
        gpart += (int64_t)d.nchunks * d.npairs * 64 * 64;
      }
    }
  }
  if ((rc = dalloc_t(&b->gpart, (size_t)gpart))) return bail(rc);
  {
    int64_t o = 0;
    for (auto& d : gd) {
      d.part = b->gpart + o;
      o += (int64_t)d.nchunks * d.npairs * 64 * 64;
    }
  }
  for (const int4& w : gi) {
    if (w.x < 0 || w.x >= (int)gd.size() || w.y < 0 || w.y >= gd[w.x].nchunks || w.z < 0 ||
        w.z >= gd[w.x].npairs)
      return bail(fail(TK_EINVAL, "internal: Gram item"));
  }
  b->n_gram = (int)gd.size();
  b->n_gram_items = (int)gi.size();
  b->gram_total = goff.back();
  if ((rc = upload(&b->gram, gd, st)) || (rc = upload(&b->gram_items, gi, st)) ||
      (rc = upload(&b->gram_off, goff, st)))
    return bail(rc);

  // ---- eigensolver jobs: warm (previous factors) and cold (HOSVD)
  std::vector<EigJob> jw, jc;
  for (int i = 0; i < count; ++i) {
    const Shape& s = b->shapes[i];
    for (int n = 0; n < s.N; ++n) {
      EigJob j;
      const int64_t rank_bound = (int64_t)(s.card(((1u << s.N) - 1) & ~(1u << n)) / s.L[n]);
      j.L = (int)s.L[n];
      j.K = (int)s.K[n];
      j.p = eig_block_size(j.L, j.K, rank_bound);
      j.pad_ = 0;
      j.S_off = b->sofs[i][n];
      j.V0_off = b->fofs[i][n];
      j.F_off = b->fofs[i][n];
      j.ev_off = b->kofs[i][n];
      j.work_off = 0;
      b->Lmax = std::max(b->Lmax, j.L);
      b->pmax = std::max(b->pmax, j.p);
      jc.push_back(j);
    }
  }
  b->n_jobs = (int)jc.size();
  // full solves (p = L) keep their eigenbasis between invocations
  int64_t nbasis = 0;
  for (auto& j : jc)
    if (j.p == j.L) {
      j.basis_off = nbasis;
      nbasis += (int64_t)j.L * j.L;
    }
  int64_t work = 0;
  for (auto& j : jc) {
    j.work_off = work;
    work += (int64_t)eig_work_elems(j.L, b->pmax);  // the launch's widest block
  }
  // warm solves start from the previous factors with K + 4 columns at any L
  // (a full Jacobi solve of a 64 x 64 Gram costs its CU over a millisecond);
  // one that does not converge there is redone by the gap-free solver
  jw = jc;
  for (auto& j : jw) j.p = std::max(j.K, std::min(j.p, j.K + 4));
  for (auto& j : jc) j.V0_off = -1;
  {
    // order both tables by the warm block width (stable: ties keep tensor order)
    std::vector<int> ord(b->n_jobs);
    for (int q = 0; q < b->n_jobs; ++q) ord[q] = q;
    auto pad = [](int p) { return (p + 7) / 8 * 8; };
    std::stable_sort(ord.begin(), ord.end(),
                     [&](int x, int y) { return pad(jw[x].p) < pad(jw[y].p); });
    std::vector<EigJob> w2, c2;
    for (int q : ord) {
      w2.push_back(jw[q]);
      c2.push_back(jc[q]);
    }
    jw.swap(w2);
    jc.swap(c2);
    auto classes = [&](const std::vector<EigJob>& js, const std::vector<EigJob>& key,
                       std::vector<tk_batch::EigClass>* out) {
      for (int q = 0; q < (int)js.size();) {
        int r = q;
        tk_batch::EigClass c{q, 0, 0, 0};
        while (r < (int)js.size() && pad(key[r].p) == pad(key[q].p)) {
          c.Lmax = std::max(c.Lmax, js[r].L);
          c.pmax = std::max(c.pmax, js[r].p);
          ++r;
        }
        c.count = r - q;
        out->push_back(c);
        q = r;
      }
    };
    classes(jw, jw, &b->warm_classes);
    // cold blocks are wider than warm ones: split the cold table at the same
    // boundaries and take each range's own widest cold block
    classes(jc, jw, &b->cold_classes);
  }
  b->jobs_h = jc;
  // subspace jobs (warm p < L) may fall back to the gap-free solver; job q
  // of the (sorted) tables owns status word q
  std::vector<EigFullJob> fj;
  int64_t fwork = 0;
  for (int q = 0; q < b->n_jobs; ++q) {
    const EigJob& j = jc[q];
    if (jw[q].p == j.L) continue;
    EigFullJob f;
    f.L = j.L;
    f.K = j.K;
    f.status_idx = q;
    f.only_if_failed = 1;
    f.S_off = j.S_off;
    f.F_off = j.F_off;
    f.ev_off = j.ev_off;
    f.work_off = fwork;
    fwork += (int64_t)eig_full_work_elems(j.L);
    b->fLmax = std::max(b->fLmax, j.L);
    b->fKmax = std::max(b->fKmax, j.K);
    fj.push_back(f);
  }
  b->n_fjobs = (int)fj.size();
  if (b->n_fjobs > 0 && ((rc = dalloc_t(&b->fwork, (size_t)fwork)) || (rc = upload(&b->fjobs, fj, st))))
    return bail(rc);
  if (nbasis > 0) {
    std::vector<double> ident;
    eig_identity_bases(jc, &ident);
    if ((rc = dalloc_t(&b->basis, (size_t)nbasis))) return bail(rc);
    if (hipMemcpy(b->basis, ident.data(), sizeof(double) * ident.size(), hipMemcpyHostToDevice) !=
        hipSuccess)
      return bail(fail(TK_EDEVICE, "basis upload failed"));
  }
  if ((rc = dalloc_t(&b->eigwork, (size_t)work)) || (rc = dalloc_t(&b->status, (size_t)b->n_jobs)) ||
      (rc = upload(&b->jobs_warm, jw, st)) || (rc = upload(&b->jobs_cold, jc, st)))
    return bail(rc);
  if ((rc = upload(&b->core_off, core_off_h, st))) return bail(rc);

  // ---- ||T_i||^2 and the HOSVD start (Grams of the unfoldings of T_i)
  b->normT2.assign(count, 0.0);
  size_t gp_hosvd = 0;
  for (int i = 0; i < count; ++i) {
    const Shape& s = b->shapes[i];
    for (int n = 0; n < s.N; ++n)
      gp_hosvd = std::max(gp_hosvd, gram_workspace_elems(s.L[n], (int64_t)(s.card_T() / s.L[n])));
  }
  double* hpart = nullptr;
  if ((rc = dalloc_t(&hpart, gp_hosvd))) return bail(rc);
  hipError_t e = hipSuccess;
  for (int i = 0; i < count && e == hipSuccess; ++i) {
    const Shape& s = b->shapes[i];
    e = launch_sumsq(tdtype, b->T[i], (int64_t)s.card_T(), b->sumsq_part,
                     b->normT2_dev + i, st);
    for (int n = 0; n < s.N && e == hipSuccess; ++n) {
      int64_t A, Ln, B;
      view(s, 0u, n, &A, &Ln, &B);
      e = launch_gram(tdtype, b->T[i], A, Ln, B, b->S + b->sofs[i][n], hpart, st);
    }
  }
  if (e == hipSuccess) e = launch_fill_int(b->status, b->n_jobs, 0, st);
  for (size_t k = 0; k < b->cold_classes.size() && e == hipSuccess; ++k) {
    const auto& c = b->cold_classes[k];
    e = launch_eig(c.count, b->jobs_cold, c.job0, c.Lmax, c.pmax, b->S, b->F64a, b->F64a, b->ev,
                   b->eigwork, b->status, nullptr, 100, 1e-11, st, b->basis);
  }
  if (e == hipSuccess)
    e = launch_eig_full(b->n_fjobs, b->fjobs, b->fLmax, b->fKmax, b->S, b->F64a, b->ev,
                        b->fwork, b->status, st);
  if (e == hipSuccess) e = launch_convert(TK_F64, TK_F32, b->F64a, b->Fc, b->nF, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->normT2.data(), b->normT2_dev, sizeof(double) * count,
                       hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(hpart);
  if (e != hipSuccess) return bail(fail(TK_EDEVICE, "batched HOSVD failed: %s", hipGetErrorString(e)));
  if ((rc = check_status(b))) return bail(rc);
  for (int i = 0; i < count; ++i)
    if (!(b->normT2[i] > 0.0) || !std::isfinite(b->normT2[i]))
      return bail(fail(TK_ENUMERIC, "tensor %d: ||T|| is zero or not finite", i));
  *out = b;
  return TK_OK;
}

extern "C" int hooi_batch_iterate(tk_batch* b, int iters, double* rel_err) {
  clear_error();
  if (!b) return fail(TK_EINVAL, "batch is null");
  if (iters < 1) return fail(TK_EINVAL, "iters=%d < 1", iters);
  Handoff handoff(b);
  if (b->use_graph && !b->exec)
    if (int rc = build_graph(b)) return rc;
  std::vector<double> g2((size_t)iters * b->count);
  TK_HIP(launch_fill_int(b->status, b->n_jobs, 0, b->st));
  for (int t = 0; t < iters; ++t) {
    if (b->use_graph) {
      TK_HIP(hipGraphLaunch(b->exec, b->st));
    } else if (int rc = enqueue_iteration(b)) {
      return rc;
    }
    TK_HIP(hipMemcpyAsync(g2.data() + (size_t)t * b->count, b->normG2, sizeof(double) * b->count,
                          hipMemcpyDeviceToHost, b->st));
  }
  TK_HIP(hipStreamSynchronize(b->st));
  if (int rc = check_status(b)) return rc;
  if (rel_err)
    for (int t = 0; t < iters; ++t)
      for (int i = 0; i < b->count; ++i) {
        const double t2 = b->normT2[i];
        rel_err[(size_t)t * b->count + i] =
            std::sqrt(std::max(t2 - g2[(size_t)t * b->count + i], 0.0) / t2);
      }
  return TK_OK;
}

extern "C" int hooi_batch_error(tk_batch* b, double* rel_err) {
  clear_error();
  if (!b || !rel_err) return fail(TK_EINVAL, "null pointer");
  Handoff handoff(b);
  if (int rc = enqueue_pass(b)) return rc;
  std::vector<double> g2(b->count);
  TK_HIP(hipMemcpyAsync(g2.data(), b->normG2, sizeof(double) * b->count, hipMemcpyDeviceToHost,
                        b->st));
  TK_HIP(hipStreamSynchronize(b->st));
  for (int i = 0; i < b->count; ++i)
    rel_err[i] = std::sqrt(std::max(b->normT2[i] - g2[i], 0.0) / b->normT2[i]);
  return TK_OK;
}

extern "C" int hooi_batch_get_factor(tk_batch* b, int i, int n, double* host) {
  clear_error();
  if (!b || !host) return fail(TK_EINVAL, "null pointer");
  if (i < 0 || i >= b->count) return fail(TK_EINVAL, "tensor %d out of range", i);
  if (n < 0 || n >= b->shapes[i].N) return fail(TK_EINVAL, "mode %d out of range", n);
  Handoff handoff(b);
  const Shape& s = b->shapes[i];
  TK_HIP(hipMemcpyAsync(host, b->F64a + b->fofs[i][n], sizeof(double) * s.L[n] * s.K[n],
                        hipMemcpyDeviceToHost, b->st));
  TK_HIP(hipStreamSynchronize(b->st));
  return TK_OK;
}

extern "C" int hooi_batch_set_factors(tk_batch* b, const double* host) {
  clear_error();
  if (!b || !host) return fail(TK_EINVAL, "null pointer");
  for (int64_t q = 0; q < b->nF; ++q)
    if (!std::isfinite(host[q])) return fail(TK_ENUMERIC, "factors hold NaN/Inf");
  Handoff handoff(b);
  TK_HIP(hipMemcpyAsync(b->F64a, host, sizeof(double) * b->nF, hipMemcpyHostToDevice, b->st));
  TK_HIP(launch_convert(TK_F64, TK_F32, b->F64a, b->Fc, b->nF, b->st));
  std::vector<double> ident;
  if (b->basis) {
    // the full solves restart from identity bases, as after initialisation
    eig_identity_bases(b->jobs_h, &ident);
    TK_HIP(hipMemcpyAsync(b->basis, ident.data(), sizeof(double) * ident.size(),
                          hipMemcpyHostToDevice, b->st));
  }
  TK_HIP(hipStreamSynchronize(b->st));
  return TK_OK;
}

extern "C" int hooi_batch_get_factors(tk_batch* b, double* host) {
  clear_error();
  if (!b || !host) return fail(TK_EINVAL, "null pointer");
  Handoff handoff(b);
  TK_HIP(hipMemcpyAsync(host, b->F64a, sizeof(double) * b->nF, hipMemcpyDeviceToHost, b->st));
  TK_HIP(hipStreamSynchronize(b->st));
  return TK_OK;
}

extern "C" int hooi_batch_use_graph(tk_batch* b, int on) {
  clear_error();
  if (!b) return fail(TK_EINVAL, "batch is null");
  b->use_graph = on != 0;
  return TK_OK;
}

extern "C" int hooi_batch_tune(tk_batch* b, int* blocks_per_cu, float* ms) {
  clear_error();
  if (!b) return fail(TK_EINVAL, "batch is null");
  Handoff handoff(b);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  TK_HIP(hipEventCreate(&e0));
  TK_HIP(hipEventCreate(&e1));
  // average time of three passes in the current configuration (after one
  // untimed pass at it)
  auto time_pass = [&](float* t) -> int {
    int rc = enqueue_pass(b);
    hipError_t e = rc ? hipSuccess : hipEventRecord(e0, b->st);
    for (int r = 0; r < 3 && rc == TK_OK && e == hipSuccess; ++r) rc = enqueue_pass(b);
    if (rc == TK_OK && e == hipSuccess) e = hipEventRecord(e1, b->st);
    if (rc == TK_OK && e == hipSuccess) e = hipEventSynchronize(e1);
    if (rc == TK_OK && e == hipSuccess) e = hipEventElapsedTime(t, e0, e1);
    if (rc == TK_OK && e != hipSuccess) rc = fail(TK_EDEVICE, "tuning failed: %s", hipGetErrorString(e));
    *t /= 3.f;
    return rc;
  };
  // 1. blocks per CU (the grouped kernel holds 3 per CU; 4 oversubscribes)
  static const int cand[4] = {1, 2, 3, 4};
  float best = 0.f;
  int pick = b->blocks_per_cu;
  int rc = TK_OK;
  for (int c = 0; c < 4 && rc == TK_OK; ++c) {
    b->blocks_per_cu = cand[c];
    float t = 0.f;
    rc = time_pass(&t);
    if (rc == TK_OK) {
      if (ms) ms[c] = t;
      if (c == 0 || t < best) {
        best = t;
        pick = cand[c];
      }
    }
  }
  // 2. the odd-length rows' body: the shared queue's or the separate launch's
  bool split_pick = b->split_rows;
  if (rc == TK_OK) {
    b->blocks_per_cu = pick;
    b->split_rows = !b->split_rows;
    float t = 0.f;
    rc = time_pass(&t);
    if (rc == TK_OK && t < best) {
      best = t;
      split_pick = b->split_rows;
    }
    if (ms) ms[4] = t;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->split_rows = split_pick;
  if (rc) return rc;
  b->blocks_per_cu = pick;
  if (blocks_per_cu) *blocks_per_cu = pick;
  if (b->use_graph) return build_graph(b);  // re-capture with the chosen configuration
  return TK_OK;
}

extern "C" int hooi_batch_stats(const tk_batch* b, uint64_t* tree_macs, uint64_t* tree_bytes,
                                int* levels, int* ttm_items) {
  clear_error();
  if (!b) return fail(TK_EINVAL, "batch is null");
  if (tree_macs) *tree_macs = b->tree_macs;
  if (tree_bytes) *tree_bytes = b->tree_bytes;
  if (levels) *levels = (int)b->levels.size();
  if (ttm_items) {
    int n = b->fold.n_items + b->fold.n_ritems;
    for (const auto& l : b->levels) n += l.n_items + l.n_ritems;
    *ttm_items = n;
  }
  return TK_OK;
}

extern "C" void hooi_batch_free(tk_batch* b) { delete b; }
