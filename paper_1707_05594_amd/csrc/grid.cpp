// Processor-grid planning for a TTM-tree (Sec. 4): host only.
//
// P processors form an N-dimensional grid <q_1, ..., q_N>, prod q_n = P, that
// cuts every tensor of the tree into P blocks (Sec. 4.1).  A TTM along mode
// n at node u then reduce-scatters (q_n - 1) |Out(u)| words, and only grids
// with q_n <= K_n for every n are used (valid grids: no empty blocks).
//   * static gridding (Sec. 4.2): one grid for the whole tree, the one with the
//     least total TTM volume, by exhaustive search over the psi(P, N) ordered
//     factorisations of P;
//   * dynamic gridding (Sec. 4.3-4.4): each node u may redistribute its input
//     to a grid of its own at a cost of |In(u)| words; the optimal scheme comes
//     from the bottom-up recurrence over (node, parent grid) pairs.  The grid a
//     regridding node takes minimises its own TTM volume plus its subtrees'
//     optimal volumes; T is laid out under a grid of free choice; ties go to
//     the first grid in lexicographic order, and to keeping the parent's grid.
// Nothing here runs on the GPU: the engine holds T on one device, so the plan
// is what a multi-device execution of the same tree would follow.
#include <algorithm>
#include <cstring>
#include <vector>

#include "internal.h"

namespace tk {
namespace {

typedef unsigned __int128 u128;

// All N-tuples of positive integers with product P, lexicographic order.
void enum_grids(int64_t P, int N, std::vector<int64_t>& cur, std::vector<std::vector<int64_t>>* out,
                size_t cap, bool* over) {
  if (*over) return;
  if ((int)cur.size() == N - 1) {
    cur.push_back(P);
    if (out->size() >= cap) {
      *over = true;
    } else {
      out->push_back(cur);
    }
    cur.pop_back();
    return;
  }
  for (int64_t d = 1; d <= P; ++d) {
    if (P % d) continue;
    cur.push_back(d);
    enum_grids(P / d, N, cur, out, cap, over);
    cur.pop_back();
    if (*over) return;
  }
}

// C(n, k); false when it exceeds 2^64 - 1.  Each partial product
// C(n - k + i, i) is an integer below 2^64 before the next step, so the
// step's product stays below 2^128.
bool binom(uint64_t n, uint64_t k, uint64_t* out) {
  u128 r = 1;
  for (uint64_t i = 1; i <= k; ++i) {
    r = r * (n - k + i) / i;
    if (r > (u128)UINT64_MAX) return false;
  }
  *out = (uint64_t)r;
  return true;
}

}  // namespace
}  // namespace tk

using namespace tk;

extern "C" int tk_grid_count(int64_t P, int N, uint64_t* count) {
  clear_error();
  if (!count) return fail(TK_EINVAL, "count is null");
  if (P < 1 || N < 1) return fail(TK_EINVAL, "P >= 1 and N >= 1 required");
  // r stays below 2^64 after every factor, so each product fits in 128 bits
  u128 r = 1;
  int64_t x = P;
  for (int64_t p = 2; p * p <= x; ++p) {
    int e = 0;
    while (x % p == 0) {
      x /= p;
      ++e;
    }
    if (e) {
      uint64_t c = 0;
      if (!binom((uint64_t)e + (uint64_t)N - 1, (uint64_t)N - 1, &c))
        return fail(TK_EINVAL, "count overflows 64 bits");
      r *= c;
      if (r > (u128)UINT64_MAX) return fail(TK_EINVAL, "count overflows 64 bits");
    }
  }
  if (x > 1) r *= (uint64_t)N;  // one prime to the first power: C(N, N - 1)
  if (r > (u128)UINT64_MAX) return fail(TK_EINVAL, "count overflows 64 bits");
  *count = (uint64_t)r;
  return TK_OK;
}

extern "C" int tk_plan_grids(const tk_plan* plan, int rank, int64_t P, int kind, int* root_grid,
                             int* node_grids, int cap, uint64_t* volume) {
  clear_error();
  if (!plan) return fail(TK_EINVAL, "plan is null");
  if (rank < 0 || rank >= (int)plan->trees.size()) return fail(TK_EINVAL, "rank %d out of range", rank);
  if (P < 1) return fail(TK_EINVAL, "P=%lld < 1", (long long)P);
  if (kind != TK_GRID_STATIC && kind != TK_GRID_DYNAMIC) return fail(TK_EINVAL, "unknown grid kind %d", kind);
  const Shape& s = plan->shape;
  const int N = s.N;
  const auto& nodes = plan->trees[rank].nodes;
  const int nn = (int)nodes.size();
  if (node_grids && cap < nn) return fail(TK_EINVAL, "cap %d < %d nodes", cap, nn);

  // valid grids (q_n <= K_n), lexicographic order
  const size_t kMaxGrids = (size_t)1 << 22;
  std::vector<std::vector<int64_t>> all;
  std::vector<int64_t> cur;
  bool over = false;
  enum_grids(P, N, cur, &all, kMaxGrids, &over);
  if (over) return fail(TK_EUNSUPPORTED, "more than %zu grids of %lld processors", kMaxGrids, (long long)P);
  std::vector<std::vector<int64_t>> G;
  for (auto& g : all) {
    bool ok = true;
    for (int n = 0; n < N; ++n) ok = ok && g[n] <= s.K[n];
    if (ok) G.push_back(g);
  }
  if (G.empty()) return fail(TK_EUNSUPPORTED, "no valid grid: some q_n would exceed K_n");
  const int ng = (int)G.size();
  std::vector<int> chosen(nn, 0);
  int root_g = 0;
  u128 best = 0;

  if (kind == TK_GRID_STATIC) {
    for (int gi = 0; gi < ng; ++gi) {
      u128 v = 0;
      for (const tk_node& u : nodes)
        if (!u.is_leaf) v += (u128)(G[gi][u.mode] - 1) * u.out_card;
      if (gi == 0 || v < best) {
        best = v;
        root_g = gi;
      }
    }
    std::fill(chosen.begin(), chosen.end(), root_g);
  } else {
    // opt[u][g]: optimal volume of u's subtree given its parent's grid g
    // (0 for leaves); dec[u][g]: the grid u takes
    std::vector<std::vector<u128>> below(nn, std::vector<u128>(ng, 0));
    std::vector<std::vector<u128>> opt(nn, std::vector<u128>(ng, 0));
    std::vector<std::vector<int>> dec(nn, std::vector<int>(ng, 0));
    for (int u = nn - 1; u >= 0; --u) {  // children come after their parent
      const tk_node& nd = nodes[u];
      if (nd.is_leaf) {
        for (int g = 0; g < ng; ++g) dec[u][g] = g;
      } else {
        const int n = nd.mode;
        int rg = 0;
        u128 rv = 0;
        for (int g = 0; g < ng; ++g) {
          const u128 v = (u128)(G[g][n] - 1) * nd.out_card + below[u][g];
          if (g == 0 || v < rv) {
            rv = v;
            rg = g;
          }
        }
        const u128 move = (u128)nd.in_card + rv;
        for (int g = 0; g < ng; ++g) {
          const u128 keep = (u128)(G[g][n] - 1) * nd.out_card + below[u][g];
          if (rg == g || keep <= move) {
            opt[u][g] = keep;
            dec[u][g] = g;
          } else {
            opt[u][g] = move;
            dec[u][g] = rg;
          }
        }
      }
      if (nd.parent >= 0)
        for (int g = 0; g < ng; ++g) below[nd.parent][g] += opt[u][g];
    }
    for (int g = 0; g < ng; ++g) {
      u128 v = 0;
      for (int u = 0; u < nn; ++u)
        if (nodes[u].parent < 0) v += opt[u][g];
      if (g == 0 || v < best) {
        best = v;
        root_g = g;
      }
    }
    for (int u = 0; u < nn; ++u) {
      const int pg = nodes[u].parent < 0 ? root_g : chosen[nodes[u].parent];
      chosen[u] = dec[u][pg];
    }
  }
  if (best > (u128)UINT64_MAX) return fail(TK_EINVAL, "volume overflows 64 bits");
  if (volume) *volume = (uint64_t)best;
  if (root_grid)
    for (int n = 0; n < N; ++n) root_grid[n] = (int)G[root_g][n];
  if (node_grids)
    for (int u = 0; u < nn; ++u)
      for (int n = 0; n < N; ++n) node_grids[(size_t)u * N + n] = (int)G[chosen[u]][n];
  return TK_OK;
}
