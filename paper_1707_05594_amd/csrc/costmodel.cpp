// Learned choice among the planner's k best TTM-trees and each node's TTM
// kernel (tile).  The trees the dynamic program of Sec. 3.3 ranks by
// multiply-adds (Sec. 3.1) can differ in run time at equal or near-equal cost:
// a node whose B is a multiple of four runs the wide kernel, an odd B the
// staged one, a small grid benefits from split K.  A small MLP (mlp.hip)
// predicts the log of a node's time from its shape features; a tree's
// predicted time is the sum over its internal nodes, each at its best
// predicted kernel.  The selection falls back to the DP optimum with the
// automatic kernels unless a candidate is predicted faster by a margin.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"
#include "kernels.h"

namespace tk {
int mlp_forward_host(tk_mlp* m, const float* X_host, int n, float* y_host);
}

using namespace tk;

namespace {

int elem_bytes(int dtype) { return dtype == TK_F64 ? 8 : dtype == TK_F32 ? 4 : 2; }

void features(int64_t A, int64_t L, int64_t B, int64_t K, int in_dtype, int compute, int tile,
              float* f) {
  const double lA = std::log2((double)A), lL = std::log2((double)L), lB = std::log2((double)B);
  const double lK = std::log2((double)K);
  const double in_bytes = (double)A * L * B * elem_bytes(in_dtype);
  const double out_bytes = (double)A * K * B * (compute == TK_C_FP64 ? 8 : 4);
  f[0] = (float)lA;
  f[1] = (float)lL;
  f[2] = (float)lB;
  f[3] = (float)lK;
  f[4] = (float)std::log2(in_bytes);
  f[5] = (float)std::log2(out_bytes);
  f[6] = (B % 4 == 0 && B >= 16) ? 1.f : 0.f;  // the wide kernel applies
  f[7] = (B == 1 && L % 4 == 0) ? 1.f : 0.f;   // the row kernel applies
  f[8] = (float)elem_bytes(in_dtype) / 4.f;
  f[9] = compute == TK_C_FP32 ? 0.f : compute == TK_C_BF16 ? 0.5f : compute == TK_C_BF16X3 ? 1.f : 2.f;
  f[10] = tile == TK_TILE_STAGED ? 1.f : 0.f;
  f[11] = tile == TK_TILE_SPLITK ? 1.f : 0.f;
  f[12] = 0.f;
}

void pair_features(int64_t A, int64_t Lp, int64_t M, int64_t Lq, int64_t B, int64_t Kp,
                   int64_t Kq, int in_dtype, int compute, float* f) {
  const double in_bytes = (double)A * Lp * M * Lq * B * elem_bytes(in_dtype);
  const double ob = compute == TK_C_FP64 ? 8 : 4;
  const double out_bytes = ((double)A * Kp * M * Lq * B + (double)A * Lp * M * Kq * B) * ob;
  f[0] = (float)std::log2((double)A);
  f[1] = (float)std::log2((double)Lp);
  f[2] = (float)std::log2((double)M * Lq * B);
  f[3] = (float)std::log2((double)Kp);
  f[4] = (float)std::log2(in_bytes);
  f[5] = (float)std::log2(out_bytes);
  f[6] = 0.f;
  f[7] = 0.f;
  f[8] = (float)elem_bytes(in_dtype) / 4.f;
  f[9] = compute == TK_C_FP32 ? 0.f : compute == TK_C_BF16 ? 0.5f : compute == TK_C_BF16X3 ? 1.f : 2.f;
  f[10] = 0.f;
  f[11] = 0.f;
  f[12] = 1.f;
}

// The tree's root pair (p < q) when the root has exactly two internal
// children and the pair kernel for the two trailing modes takes them.
bool fusable_pair(const Shape& s, const std::vector<tk_node>& nodes, int tdtype, int compute,
                  int* up, int* uq) {
  std::vector<int> roots;
  for (size_t u = 0; u < nodes.size(); ++u)
    if (nodes[u].parent < 0) roots.push_back((int)u);
  if (roots.size() != 2 || nodes[roots[0]].is_leaf || nodes[roots[1]].is_leaf) return false;
  int a = roots[0], b = roots[1];
  if (nodes[a].mode > nodes[b].mode) std::swap(a, b);
  int64_t Ap, Lp, Bp, Aq, Lq, Bq;
  view(s, 0, nodes[a].mode, &Ap, &Lp, &Bp);
  view(s, 0, nodes[b].mode, &Aq, &Lq, &Bq);
  const void* al = (const void*)(uintptr_t)256;
  if (ttm_pair_kind(tdtype, compute, al, Ap, Lp, Aq / (Ap * Lp), Lq, Bq, s.K[nodes[a].mode],
                    s.K[nodes[b].mode], al, al) != 2)
    return false;
  *up = a;
  *uq = b;
  return true;
}

}  // namespace

extern "C" int tk_ttm_features(int64_t A, int64_t L, int64_t B, int64_t K, int in_dtype,
                               int compute, int tile, float* out) {
  clear_error();
  if (!out) return fail(TK_EINVAL, "out is null");
  if (A < 1 || L < 1 || B < 1 || K < 1) return fail(TK_EINVAL, "sizes must be >= 1");
  if (in_dtype < TK_F64 || in_dtype > TK_F16) return fail(TK_EINVAL, "unknown dtype %d", in_dtype);
  if (compute < TK_C_FP64 || compute > TK_C_BF16X3)
    return fail(TK_EINVAL, "unknown compute mode %d", compute);
  if (tile < 0 || tile >= TK_TILE_COUNT) return fail(TK_EINVAL, "unknown tile %d", tile);
  features(A, L, B, K, in_dtype, compute, tile, out);
  return TK_OK;
}

extern "C" int tk_pair_features(int64_t A, int64_t Lp, int64_t M, int64_t Lq, int64_t B,
                                int64_t Kp, int64_t Kq, int in_dtype, int compute, float* out) {
  clear_error();
  if (!out) return fail(TK_EINVAL, "out is null");
  if (A < 1 || Lp < 1 || M < 1 || Lq < 1 || B < 1 || Kp < 1 || Kq < 1)
    return fail(TK_EINVAL, "sizes must be >= 1");
  if (in_dtype < TK_F64 || in_dtype > TK_F16) return fail(TK_EINVAL, "unknown dtype %d", in_dtype);
  if (compute < TK_C_FP64 || compute > TK_C_BF16X3)
    return fail(TK_EINVAL, "unknown compute mode %d", compute);
  pair_features(A, Lp, M, Lq, B, Kp, Kq, in_dtype, compute, out);
  return TK_OK;
}

extern "C" int tk_time_ttm_pair(int in_dtype, int compute, const void* in, int64_t A, int64_t Lp,
                                int64_t M, int64_t Lq, int64_t B, const void* Fp, int64_t Kp,
                                const void* Fq, int64_t Kq, void* outp, void* outq, int reps,
                                void* stream, float* ms) {
  clear_error();
  if (!in || !Fp || !Fq || !outp || !outq || !ms) return fail(TK_EINVAL, "null pointer");
  if (reps < 1) return fail(TK_EINVAL, "reps < 1");
  if (!ttm_pair_applies(in_dtype, compute, in, A, Lp, M, Lq, B, Kp, Kq, outp, outq))
    return fail(TK_EUNSUPPORTED, "no pair kernel takes this shape");
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  TK_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(TK_EDEVICE, "event creation failed");
  }
  auto run = [&]() {
    return launch_ttm_pair((const float*)in, A, Lp, M, Lq, B, (const float*)Fp, Kp,
                           (const float*)Fq, Kq, (float*)outp, (float*)outq, st);
  };
  hipError_t e = run();  // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = run();
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(TK_EDEVICE, "timing failed: %s", hipGetErrorString(e));
  *ms = t / (float)reps;
  return TK_OK;
}

extern "C" int tk_time_ttm(int in_dtype, int compute, const void* in, int64_t A, int64_t L,
                           int64_t B, const void* F, int64_t K, void* out, int tile, int reps,
                           void* stream, float* ms) {
  clear_error();
  if (!in || !F || !out || !ms) return fail(TK_EINVAL, "null pointer");
  if (A < 1 || L < 1 || B < 1 || K < 1 || reps < 1) return fail(TK_EINVAL, "sizes must be >= 1");
  if (tile < 0 || tile >= TK_TILE_COUNT) return fail(TK_EINVAL, "unknown tile %d", tile);
  if (compute == TK_C_FP64 ? (in_dtype != TK_F64 || L > 512)
                           : (in_dtype == TK_F64 || L > ttm_max_L()))
    return fail(TK_EUNSUPPORTED, "dtype/compute pair or L not supported");
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  TK_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(TK_EDEVICE, "event creation failed");
  }
  hipError_t e = launch_ttm(in_dtype, compute, in, A, L, B, F, K, out, st, false, tile);  // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  for (int r = 0; r < reps && e == hipSuccess; ++r)
    e = launch_ttm(in_dtype, compute, in, A, L, B, F, K, out, st, false, tile);
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(TK_EDEVICE, "timing failed: %s", hipGetErrorString(e));
  *ms = t / (float)reps;
  return TK_OK;
}

extern "C" int tk_plan_set_tiles(tk_plan* plan, int rank, const int* tiles, int n) {
  clear_error();
  if (!plan || !tiles) return fail(TK_EINVAL, "null pointer");
  if (rank < 0 || rank >= (int)plan->trees.size()) return fail(TK_EINVAL, "rank %d out of range", rank);
  if (n != (int)plan->trees[rank].nodes.size())
    return fail(TK_EINVAL, "n=%d but the tree has %zu nodes", n, plan->trees[rank].nodes.size());
  const auto& nodes = plan->trees[rank].nodes;
  int npair = 0;
  for (int i = 0; i < n; ++i) {
    if (tiles[i] == TK_TILE_PAIR) {
      if (nodes[i].parent >= 0 || nodes[i].is_leaf)
        return fail(TK_EINVAL, "TK_TILE_PAIR on node %d, which is not a root TTM", i);
      ++npair;
    } else if (tiles[i] < 0 || tiles[i] >= TK_TILE_COUNT) {
      return fail(TK_EINVAL, "unknown tile %d", tiles[i]);
    }
  }
  int nroots = 0;
  for (const tk_node& nd : nodes) nroots += nd.parent < 0;
  if (npair != 0 && !(npair == 2 && nroots == 2))
    return fail(TK_EINVAL, "TK_TILE_PAIR goes on both root nodes of a two-child root");
  plan->tiles.resize(plan->trees.size());
  plan->tiles[rank].assign(tiles, tiles + n);
  return TK_OK;
}

extern "C" int tk_plan_get_tiles(const tk_plan* plan, int rank, int* tiles, int cap, int* n) {
  clear_error();
  if (!plan || !n) return fail(TK_EINVAL, "null pointer");
  if (rank < 0 || rank >= (int)plan->trees.size()) return fail(TK_EINVAL, "rank %d out of range", rank);
  const int nn = (int)plan->trees[rank].nodes.size();
  *n = nn;
  if (tiles) {
    const bool set = rank < (int)plan->tiles.size() && !plan->tiles[rank].empty();
    for (int i = 0; i < std::min(cap, nn); ++i) tiles[i] = set ? plan->tiles[rank][i] : TK_TILE_AUTO;
  }
  return TK_OK;
}

extern "C" int tk_plan_node_views(const tk_plan* plan, int rank, int tdtype, int compute,
                                  tk_node_view* out, int cap, int* n) {
  clear_error();
  if (!plan || !n) return fail(TK_EINVAL, "null pointer");
  if (rank < 0 || rank >= (int)plan->trees.size()) return fail(TK_EINVAL, "rank %d out of range", rank);
  if (tdtype < TK_F64 || tdtype > TK_F16) return fail(TK_EINVAL, "unknown dtype %d", tdtype);
  if (compute < TK_C_FP64 || compute > TK_C_BF16X3)
    return fail(TK_EINVAL, "unknown compute mode %d", compute);
  const Shape& s = plan->shape;
  const auto& nodes = plan->trees[rank].nodes;
  int count = 0;
  for (const tk_node& nd : nodes) count += nd.is_leaf ? 0 : 1;
  *n = count;
  if (!out) return TK_OK;
  if (cap < count) return fail(TK_EINVAL, "cap %d < %d internal nodes", cap, count);
  const bool set = rank < (int)plan->tiles.size() && !plan->tiles[rank].empty();
  const std::vector<int> tiles = set ? plan->tiles[rank] : std::vector<int>();
  int fold_leaf = 0;
  std::vector<int> node_compute, out_dt;
  tree_precisions(s, nodes, tdtype, compute, tiles, reinterpret_cast<const void*>((uintptr_t)256),
                  &fold_leaf, &node_compute, &out_dt);
  int i = 0;
  for (int u = 0; u < (int)nodes.size(); ++u) {
    if (nodes[u].is_leaf) continue;
    tk_node_view& v = out[i++];
    v.node = u;
    v.in_dtype = nodes[u].parent < 0 ? tdtype : out_dt[nodes[u].parent];
    v.compute = node_compute[u];
    v.out_dtype = out_dt[u];
    view(s, nodes[u].pre_mask, nodes[u].mode, &v.A, &v.L, &v.B);
    v.K = s.K[nodes[u].mode];
  }
  return TK_OK;
}

extern "C" int tk_plan_root_pair(const tk_plan* plan, int rank, int tdtype, int compute,
                                 int64_t* view7, int* fusable) {
  clear_error();
  if (!plan || !view7 || !fusable) return fail(TK_EINVAL, "null pointer");
  if (rank < 0 || rank >= (int)plan->trees.size()) return fail(TK_EINVAL, "rank %d out of range", rank);
  if (tdtype < TK_F64 || tdtype > TK_F16) return fail(TK_EINVAL, "unknown dtype %d", tdtype);
  if (compute < TK_C_FP64 || compute > TK_C_BF16X3)
    return fail(TK_EINVAL, "unknown compute mode %d", compute);
  const Shape& s = plan->shape;
  const auto& nodes = plan->trees[rank].nodes;
  std::vector<int> roots;
  for (size_t u = 0; u < nodes.size(); ++u)
    if (nodes[u].parent < 0) roots.push_back((int)u);
  *fusable = 0;
  if (roots.size() != 2 || nodes[roots[0]].is_leaf || nodes[roots[1]].is_leaf) {
    for (int i = 0; i < 7; ++i) view7[i] = 0;
    return TK_OK;
  }
  const int p = std::min(nodes[roots[0]].mode, nodes[roots[1]].mode);
  const int q = std::max(nodes[roots[0]].mode, nodes[roots[1]].mode);
  int64_t Ap, Lp, Bp, Aq, Lq, Bq;
  view(s, 0, p, &Ap, &Lp, &Bp);
  view(s, 0, q, &Aq, &Lq, &Bq);
  view7[0] = Ap;
  view7[1] = Lp;
  view7[2] = Aq / (Ap * Lp);
  view7[3] = Lq;
  view7[4] = Bq;
  view7[5] = s.K[p];
  view7[6] = s.K[q];
  int up, uq;
  *fusable = fusable_pair(s, nodes, tdtype, compute, &up, &uq) ? 1 : 0;
  return TK_OK;
}

extern "C" int tk_plan_learned(tk_plan* plan, tk_mlp* model, int tdtype, int compute,
                               double margin, int* chosen, double* predicted_ms) {
  clear_error();
  if (!plan || !model) return fail(TK_EINVAL, "null pointer");
  if (tdtype < TK_F64 || tdtype > TK_F16) return fail(TK_EINVAL, "unknown dtype %d", tdtype);
  if (compute < TK_C_FP64 || compute > TK_C_BF16X3)
    return fail(TK_EINVAL, "unknown compute mode %d", compute);
  if (!(margin >= 0.0 && margin < 1.0)) return fail(TK_EINVAL, "margin outside [0, 1)");
  const Shape& s = plan->shape;
  const int ntiles = compute == TK_C_FP64 ? 1 : TK_TILE_COUNT;
  // one feature row per (tree, internal node, tile), each node with the
  // input type and compute mode the engine gives it (the core's path at FP32
  // in the BF16 modes; BF16 intermediates where the engine stores them)
  std::vector<float> X;
  struct Row {
    int tree, node, tile;
  };
  std::vector<Row> rows;
  const void* aligned = reinterpret_cast<const void*>((uintptr_t)256);
  for (int r = 0; r < (int)plan->trees.size(); ++r) {
    const auto& nodes = plan->trees[r].nodes;
    int fold_leaf = 0;
    std::vector<int> node_compute, out_dt;
    tree_precisions(s, nodes, tdtype, compute, std::vector<int>(), aligned, &fold_leaf,
                    &node_compute, &out_dt);
    for (int u = 0; u < (int)nodes.size(); ++u) {
      if (nodes[u].is_leaf) continue;
      int64_t A, L, B;
      view(s, nodes[u].pre_mask, nodes[u].mode, &A, &L, &B);
      const int in_dt = nodes[u].parent < 0 ? tdtype : out_dt[nodes[u].parent];
      for (int t = 0; t < ntiles; ++t) {
        float f[TK_FEATURES];
        features(A, L, B, s.K[nodes[u].mode], in_dt, node_compute[u], t, f);
        X.insert(X.end(), f, f + TK_FEATURES);
        rows.push_back({r, u, t});
      }
    }
  }
  // one more row per tree whose root pair a pair kernel takes (FP32 only)
  const int R0 = (int)plan->trees.size();
  std::vector<int> pair_row(R0, -1), pair_p(R0, -1), pair_q(R0, -1);
  if (tdtype == TK_F32 && compute == TK_C_FP32)
    for (int r = 0; r < R0; ++r) {
      int up, uq;
      if (!fusable_pair(s, plan->trees[r].nodes, tdtype, compute, &up, &uq)) continue;
      const int p = plan->trees[r].nodes[up].mode, q = plan->trees[r].nodes[uq].mode;
      int64_t Ap, Lp, Bp, Aq, Lq, Bq;
      view(s, 0, p, &Ap, &Lp, &Bp);
      view(s, 0, q, &Aq, &Lq, &Bq);
      float f[TK_FEATURES];
      pair_features(Ap, Lp, Aq / (Ap * Lp), Lq, Bq, s.K[p], s.K[q], tdtype, compute, f);
      X.insert(X.end(), f, f + TK_FEATURES);
      pair_row[r] = (int)rows.size();
      pair_p[r] = up;
      pair_q[r] = uq;
      rows.push_back({r, -1, TK_TILE_PAIR});
    }
  if (rows.empty()) return fail(TK_EINVAL, "plan holds no internal nodes");
  std::vector<float> y(rows.size());
  if (int rc = mlp_forward_host(model, X.data(), (int)rows.size(), y.data())) return rc;
  const int R = (int)plan->trees.size();
  std::vector<double> best_total(R, 0.0), auto_total(R, 0.0);
  std::vector<std::vector<int>> best_tile(R);
  std::vector<std::vector<double>> best_ms(R);
  for (int r = 0; r < R; ++r) {
    best_tile[r].assign(plan->trees[r].nodes.size(), TK_TILE_AUTO);
    best_ms[r].assign(plan->trees[r].nodes.size(), INFINITY);
  }
  for (size_t i = 0; i < rows.size(); ++i) {
    const double ms = std::exp((double)y[i]);
    const Row& w = rows[i];
    if (w.node < 0) continue;  // pair rows are weighed per tree below
    if (w.tile == TK_TILE_AUTO) auto_total[w.tree] += ms;
    if (ms < best_ms[w.tree][w.node]) {
      best_ms[w.tree][w.node] = ms;
      best_tile[w.tree][w.node] = w.tile;
    }
  }
  int pick = 0;
  for (int r = 0; r < R; ++r) {
    for (size_t u = 0; u < best_ms[r].size(); ++u)
      if (std::isfinite(best_ms[r][u])) best_total[r] += best_ms[r][u];
    if (pair_row[r] >= 0) {
      // fused: the pair launch replaces both root TTMs
      const double fused = best_total[r] - best_ms[r][pair_p[r]] - best_ms[r][pair_q[r]] +
                           std::exp((double)y[pair_row[r]]);
      if (fused < best_total[r]) {
        best_total[r] = fused;
        best_tile[r][pair_p[r]] = TK_TILE_PAIR;
        best_tile[r][pair_q[r]] = TK_TILE_PAIR;
      }
    }
    if (best_total[r] < best_total[pick]) pick = r;
    if (predicted_ms) predicted_ms[r] = best_total[r];
  }
  plan->tiles.assign(R, std::vector<int>());
  if (best_total[pick] < (1.0 - margin) * auto_total[0]) {
    plan->selected = pick;
    plan->tiles[pick] = best_tile[pick];
  } else {
    plan->selected = 0;  // fallback: the DP optimum with the automatic kernels
    pick = 0;
  }
  if (chosen) *chosen = plan->selected;
  return TK_OK;
}
