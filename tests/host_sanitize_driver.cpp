// Host driver for the address/undefined-behaviour sanitizer build of the
// host-only sources of libtucker (the TTM-tree planner, Sec. 3, and the
// processor-grid planner, Sec. 4).  Built with g++ -fsanitize=address,undefined
// by tests/test_host_sanitizers.py; every call goes through the C ABI of
// include/tucker.h, valid arguments and invalid ones, and a few invariants are
// checked on the way.  Prints "host driver ok" and returns 0 on success.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "tucker.h"

namespace {

int failures = 0;

#define CHECK(cond)                                                           \
  do {                                                                        \
    if (!(cond)) {                                                            \
      std::fprintf(stderr, "check failed at line %d: %s (%s)\n", __LINE__,    \
                   #cond, tk_last_error());                                   \
      ++failures;                                                             \
    }                                                                         \
  } while (0)

// Small deterministic generator for test shapes (xorshift64).
struct Gen {
  uint64_t s;
  uint64_t next() {
    s ^= s << 13;
    s ^= s >> 7;
    s ^= s << 17;
    return s;
  }
  int64_t in(int64_t lo, int64_t hi) { return lo + (int64_t)(next() % (uint64_t)(hi - lo + 1)); }
};

void valid_ranks(int N, const int64_t* L, int64_t* K) {
  for (int n = 0; n < N; ++n)
    if (K[n] > L[n]) K[n] = L[n];
  for (int pass = 0; pass < 4; ++pass)
    for (int n = 0; n < N; ++n) {
      int64_t others = 1;
      for (int m = 0; m < N; ++m)
        if (m != n) others *= K[m];
      if (K[n] > others) K[n] = others;
    }
}

void exercise_plan(tk_plan* p, int N, const int64_t* L, const int64_t* K) {
  int count = 0;
  CHECK(tk_plan_count(p, &count) == TK_OK && count >= 1);
  uint64_t prev = 0;
  for (int r = 0; r < count; ++r) {
    uint64_t macs = 0;
    CHECK(tk_plan_cost(p, r, &macs) == TK_OK);
    CHECK(macs >= prev);  // ranks in cost order
    prev = macs;
    // string: exact size, then one byte short (must be rejected, not overrun)
    std::vector<char> buf(1 << 16);
    CHECK(tk_plan_string(p, r, buf.data(), buf.size()) == TK_OK);
    const size_t len = std::strlen(buf.data());
    std::vector<char> exact(len + 1);
    CHECK(tk_plan_string(p, r, exact.data(), exact.size()) == TK_OK);
    CHECK(std::strcmp(exact.data(), buf.data()) == 0);
    std::vector<char> shorter(len);
    CHECK(tk_plan_string(p, r, shorter.data(), shorter.size()) == TK_EINVAL);
    // nodes: count, then a full copy, then a too-small buffer
    int n = 0;
    CHECK(tk_plan_nodes(p, r, nullptr, 0, &n) == TK_OK || n > 0);
    std::vector<tk_node> nodes(n > 0 ? n : 1);
    int n2 = 0;
    CHECK(tk_plan_nodes(p, r, nodes.data(), n, &n2) == TK_OK && n2 == n);
    int leaves = 0;
    for (int i = 0; i < n; ++i) {
      CHECK(nodes[i].parent < i);  // parents first
      CHECK(nodes[i].mode >= 0 && nodes[i].mode < N);
      leaves += nodes[i].is_leaf ? 1 : 0;
    }
    CHECK(leaves == N);
    uint64_t ws = 0;
    CHECK(tk_plan_workspace(p, r, &ws) == TK_OK);
    // grids of 1, 2, 6 and 8 processors, static and dynamic
    for (int64_t P : {1, 2, 6, 8}) {
      for (int kind : {TK_GRID_STATIC, TK_GRID_DYNAMIC}) {
        std::vector<int> root(N), ng((size_t)n * N);
        uint64_t vol = 0;
        const int rc = tk_plan_grids(p, r, P, kind, root.data(), ng.data(), n, &vol);
        CHECK(rc == TK_OK || rc == TK_EUNSUPPORTED);
        if (rc == TK_OK) {
          int64_t prod = 1;
          for (int m = 0; m < N; ++m) {
            prod *= root[m];
            CHECK(root[m] >= 1 && root[m] <= K[m]);
          }
          CHECK(prod == P);
        }
        if (n > 1) CHECK(tk_plan_grids(p, r, P, kind, root.data(), ng.data(), n - 1, &vol) ==
                         TK_EINVAL);
      }
    }
  }
  CHECK(tk_plan_cost(p, count, nullptr) != TK_OK);
  CHECK(tk_plan_select(p, count) == TK_EINVAL);
  CHECK(tk_plan_select(p, count - 1) == TK_OK);
  uint64_t entries = 0, lookups = 0;
  CHECK(tk_plan_stats(p, &entries, &lookups) == TK_OK);
  (void)L;
}

}  // namespace

int main() {
  Gen g{0x9E3779B97F4A7C15ull};
  // seeded random shapes, every tree kind, several topk
  for (int trial = 0; trial < 30; ++trial) {
    const int N = (int)g.in(2, 10);
    int64_t L[TK_MAX_MODES], K[TK_MAX_MODES];
    for (int n = 0; n < N; ++n) {
      L[n] = g.in(1, 60);
      K[n] = g.in(1, L[n]);
    }
    valid_ranks(N, L, K);
    for (int kind = TK_TREE_DP; kind <= TK_TREE_BALANCED; ++kind) {
      tk_plan* p = nullptr;
      // k-best DP planning takes up to 8 modes; the single optimum any number
      const int topk = kind == TK_TREE_DP && N <= 8 ? (int)g.in(1, 12) : 1;
      CHECK(ttm_tree_plan(N, L, K, kind, topk, &p) == TK_OK && p);
      if (kind == TK_TREE_DP && N > 8) {
        tk_plan* q = nullptr;
        CHECK(ttm_tree_plan(N, L, K, kind, 2, &q) != TK_OK && !q);
      }
      if (p) exercise_plan(p, N, L, K);
      tk_plan_free(p);
    }
  }
  // the widest supported mode count
  {
    int64_t L[TK_MAX_MODES], K[TK_MAX_MODES];
    for (int n = 0; n < TK_MAX_MODES; ++n) {
      L[n] = 3 + n % 4;
      K[n] = 2;
    }
    tk_plan* p = nullptr;
    CHECK(ttm_tree_plan(TK_MAX_MODES, L, K, TK_TREE_DP, 1, &p) == TK_OK);
    if (p) exercise_plan(p, TK_MAX_MODES, L, K);
    tk_plan_free(p);
  }
  // invalid arguments: each must fail cleanly and leave *out null
  {
    int64_t L[3] = {8, 9, 10}, K[3] = {2, 3, 4};
    tk_plan* p = nullptr;
    CHECK(ttm_tree_plan(3, L, K, TK_TREE_DP, 1, nullptr) == TK_EINVAL);
    CHECK(ttm_tree_plan(1, L, K, TK_TREE_DP, 1, &p) == TK_EINVAL && !p);
    CHECK(ttm_tree_plan(TK_MAX_MODES + 1, L, K, TK_TREE_DP, 1, &p) == TK_EINVAL && !p);
    CHECK(ttm_tree_plan(3, nullptr, K, TK_TREE_DP, 1, &p) == TK_EINVAL && !p);
    CHECK(ttm_tree_plan(3, L, K, 99, 1, &p) == TK_EINVAL && !p);
    CHECK(ttm_tree_plan(3, L, K, TK_TREE_DP, 0, &p) == TK_EINVAL && !p);
    int64_t Kbig[3] = {2, 3, 11};  // K > L
    CHECK(ttm_tree_plan(3, L, Kbig, TK_TREE_DP, 1, &p) == TK_EINVAL && !p);
    int64_t Kzero[3] = {2, 0, 4};
    CHECK(ttm_tree_plan(3, L, Kzero, TK_TREE_DP, 1, &p) == TK_EINVAL && !p);
    int64_t Krank[3] = {2, 2, 5};  // K_2 > K_0 K_1
    CHECK(ttm_tree_plan(3, L, Krank, TK_TREE_DP, 1, &p) == TK_EINVAL && !p);
    int64_t Lhuge[3] = {INT64_C(1) << 31, INT64_C(1) << 31, 4};  // prod(L) >= 2^62
    CHECK(ttm_tree_plan(3, Lhuge, K, TK_TREE_DP, 1, &p) == TK_EINVAL && !p);
    CHECK(std::strlen(tk_last_error()) > 0);
    CHECK(tk_plan_count(nullptr, nullptr) == TK_EINVAL);
    char buf[8];
    CHECK(tk_plan_string(nullptr, 0, buf, sizeof buf) == TK_EINVAL);
    CHECK(tk_plan_grids(nullptr, 0, 2, TK_GRID_STATIC, nullptr, nullptr, 0, nullptr) ==
          TK_EINVAL);
  }
  // psi(P, N): closed form at prime powers, and the overflow guard
  {
    uint64_t c = 0;
    CHECK(tk_grid_count(32, 7, &c) == TK_OK && c == 462);  // C(5 + 6, 6)
    CHECK(tk_grid_count(1, 5, &c) == TK_OK && c == 1);
    CHECK(tk_grid_count(0, 5, &c) == TK_EINVAL);
    // 2^62 over 64 modes: C(125, 63) > 2^64; over 2 modes: 63
    CHECK(tk_grid_count(INT64_C(1) << 62, 64, &c) == TK_EINVAL);
    CHECK(tk_grid_count(INT64_C(1) << 62, 2, &c) == TK_OK && c == 63);
    // 2^20 3^20 over 40 modes: C(59, 39)^2 > 2^64 while each factor fits
    CHECK(tk_grid_count(INT64_C(3486784401) * INT64_C(1048576), 40, &c) == TK_EINVAL);
    CHECK(tk_grid_count(12, 3, nullptr) == TK_EINVAL);
  }
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("host driver ok\n");
  return 0;
}
