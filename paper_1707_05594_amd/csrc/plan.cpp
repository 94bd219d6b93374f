// TTM-tree planner (host only).
//
// Cost model (Sec. 3.1, computational load): an internal node u labelled n
// costs K_n |In(u)| multiply-adds and outputs |Out(u)| = (K_n/L_n) |In(u)|.
//
// Optimal tree (Sec. 3.3): memoised dynamic program over sub-problems
// (P, Q, R) -- modes already multiplied, factors to produce below the node,
// modes free for reuse.  Splitting Q into Q1, Q2 hands the other half to each
// side as reusable, (P, Q1, R+Q2) and (P, Q2, R+Q1), so R is always the
// complement of P+Q and a state is the pair (P, Q).  Table entries are
// addressed by a base-3 code of (P, Q) (at most 3^N entries).  Ties: reuse
// candidates in ascending mode, then splits Q1 (holding the lowest mode of Q)
// in ascending bitmask order; the first strict minimum wins.
//
// k-best variant: every state keeps its cheapest distinct forests (identified
// by an order-independent 64-bit hash of the canonical tree), built from the
// kept forests of its sub-states; rank 0 is the plain optimum above.
//
// Prior schemes (Sec. 3.2): chain trees (naive, K-ordered, h-ordered) and the
// divide-and-conquer balanced tree.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <limits>
#include <new>
#include <string>
#include <unordered_set>
#include <vector>

#include "internal.h"

namespace tk {

static thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

void clear_error() { g_last_error.clear(); }

int make_shape(int N, const int64_t* L, const int64_t* K, Shape* s) {
  if (!L || !K || !s) return fail(TK_EINVAL, "null pointer argument");
  if (N < 2 || N > TK_MAX_MODES) return fail(TK_EINVAL, "N=%d outside [2, %d]", N, TK_MAX_MODES);
  s->N = N;
  long double prodL = 1;
  for (int j = 0; j < N; ++j) {
    if (L[j] < 1) return fail(TK_EINVAL, "L[%d]=%lld < 1", j, (long long)L[j]);
    if (K[j] < 1 || K[j] > L[j])
      return fail(TK_EINVAL, "K[%d]=%lld outside [1, L[%d]=%lld]", j, (long long)K[j], j,
                  (long long)L[j]);
    s->L[j] = L[j];
    s->K[j] = K[j];
    prodL *= (long double)L[j];
  }
  if (prodL >= 4.611686018427387904e18L) return fail(TK_EINVAL, "prod(L) >= 2^62");
  for (int n = 0; n < N; ++n) {
    long double pk = 1;
    for (int m = 0; m < N; ++m)
      if (m != n) pk *= (long double)K[m];
    if ((long double)K[n] > pk)
      return fail(TK_EINVAL,
                  "K[%d]=%lld exceeds the product of the other core lengths (rank of Y_(n))", n,
                  (long long)K[n]);
  }
  return TK_OK;
}

std::string canonical_string(const std::vector<tk_node>& nodes) {
  std::vector<std::vector<int>> kids(nodes.size());
  std::vector<int> top;
  for (size_t i = 0; i < nodes.size(); ++i) {
    if (nodes[i].parent < 0)
      top.push_back((int)i);
    else
      kids[nodes[i].parent].push_back((int)i);
  }
  std::function<std::string(int)> str = [&](int i) -> std::string {
    if (nodes[i].is_leaf) return "F" + std::to_string(nodes[i].mode);
    std::vector<std::string> cs;
    for (int c : kids[i]) cs.push_back(str(c));
    std::sort(cs.begin(), cs.end());
    std::string s = "m" + std::to_string(nodes[i].mode) + "(";
    for (size_t j = 0; j < cs.size(); ++j) s += (j ? "," : "") + cs[j];
    return s + ")";
  };
  std::vector<std::string> cs;
  for (int c : top) cs.push_back(str(c));
  std::sort(cs.begin(), cs.end());
  std::string s = "T(";
  for (size_t j = 0; j < cs.size(); ++j) s += (j ? "," : "") + cs[j];
  return s + ")";
}

uint64_t workspace_elements(const std::vector<tk_node>& nodes) {
  std::vector<uint64_t> live(nodes.size(), 0);
  uint64_t best = 0;
  for (size_t i = 0; i < nodes.size(); ++i) {
    uint64_t above = nodes[i].parent < 0 ? 0 : live[nodes[i].parent];
    live[i] = above + (nodes[i].is_leaf ? 0 : nodes[i].out_card);
    best = std::max(best, live[i]);
  }
  return best;
}

namespace {

constexpr uint64_t kUnset = std::numeric_limits<uint64_t>::max();
constexpr uint64_t kInf = std::numeric_limits<uint64_t>::max() - 1;

inline uint64_t sat_add(uint64_t a, uint64_t b) { return (a >= kInf - b) ? kInf : a + b; }
inline uint64_t sat_mul(uint64_t a, uint64_t b) {
  if (a == 0 || b == 0) return 0;
  return (a > kInf / b) ? kInf : a * b;
}

// Emits one internal node or leaf into the tree under construction.
struct Emitter {
  const Shape& s;
  std::vector<tk_node>& out;
  int internal(int parent, int depth, uint32_t P, int n) {
    tk_node nd{};
    nd.parent = parent;
    nd.mode = n;
    nd.is_leaf = 0;
    nd.depth = depth;
    nd.in_card = s.card(P);
    nd.out_card = s.card(P | (1u << n));
    nd.macs = (uint64_t)s.K[n] * nd.in_card;
    nd.pre_mask = P;
    out.push_back(nd);
    return (int)out.size() - 1;
  }
  void leaf(int parent, int depth, uint32_t P, int n) {
    tk_node nd{};
    nd.parent = parent;
    nd.mode = n;
    nd.is_leaf = 1;
    nd.depth = depth;
    nd.in_card = s.card(P);
    nd.pre_mask = P;
    out.push_back(nd);
  }
};

inline int lowest_bit(uint32_t x) { return __builtin_ctz(x); }

// ---------------------------------------------------------------- plain DP --
struct DP {
  const Shape& s;
  uint32_t full;
  std::vector<uint64_t> pow3, cost;
  std::vector<int32_t> choice;  // >=0 reuse mode, <0 split with Q1 = -choice-1, kLeaf
  uint64_t entries = 0, lookups = 0;
  static constexpr int32_t kLeaf = std::numeric_limits<int32_t>::min();

  explicit DP(const Shape& sh) : s(sh), full((1u << sh.N) - 1) {
    pow3.resize(s.N + 1);
    pow3[0] = 1;
    for (int j = 1; j <= s.N; ++j) pow3[j] = pow3[j - 1] * 3;
    cost.assign(pow3[s.N], kUnset);
    choice.assign(pow3[s.N], 0);
  }
  uint64_t code(uint32_t P, uint32_t Q) const {
    uint64_t c = 0;
    for (int j = 0; j < s.N; ++j) c += pow3[j] * (((P >> j) & 1u) + 2u * ((Q >> j) & 1u));
    return c;
  }
  uint64_t solve(uint32_t P, uint32_t Q) {
    ++lookups;
    const uint64_t c = code(P, Q);
    if (cost[c] != kUnset) return cost[c];
    ++entries;
    const uint32_t R = full & ~(P | Q);
    if (R == 0 && (Q & (Q - 1)) == 0) {
      cost[c] = 0;
      choice[c] = kLeaf;
      return 0;
    }
    uint64_t best = kUnset;
    int32_t ch = 0;
    const uint64_t size = s.card(P);
    for (int n = 0; n < s.N; ++n) {
      if (!((R >> n) & 1u)) continue;
      uint64_t v = sat_add(sat_mul((uint64_t)s.K[n], size), solve(P | (1u << n), Q));
      if (v < best) {
        best = v;
        ch = n;
      }
    }
    const uint32_t low = Q & (~Q + 1u);
    for (uint32_t Q1 = (0u - Q) & Q; Q1 != 0 && Q1 != Q; Q1 = (Q1 - Q) & Q) {
      if (!(Q1 & low)) continue;
      uint64_t v = sat_add(solve(P, Q1), solve(P, Q ^ Q1));
      if (v < best) {
        best = v;
        ch = -(int32_t)Q1 - 1;
      }
    }
    cost[c] = best;
    choice[c] = ch;
    return best;
  }
  void build(Emitter& em, uint32_t P, uint32_t Q, int parent, int depth) {
    const int32_t ch = choice[code(P, Q)];
    if (ch == kLeaf) {
      em.leaf(parent, depth, P, lowest_bit(Q));
    } else if (ch >= 0) {
      int me = em.internal(parent, depth, P, ch);
      build(em, P | (1u << ch), Q, me, depth + 1);
    } else {
      const uint32_t Q1 = (uint32_t)(-(ch + 1));
      build(em, P, Q1, parent, depth);
      build(em, P, Q ^ Q1, parent, depth);
    }
  }
};

// ---------------------------------------------------------------- k-best DP --
inline uint64_t mix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

struct Cand {
  uint64_t cost;
  uint64_t hash;      // order-independent hash of the forest (sum of top-level node hashes)
  uint32_t top_modes; // labels of internal top-level nodes (to reject repeated sibling labels)
  int32_t kind;       // 0 leaf, 1 reuse, 2 split
  int32_t a, i1, i2;  // reuse: a = mode, i1 = index in child list; split: a = Q1
};

struct KBest {
  const Shape& s;
  uint32_t full;
  int keep;
  std::vector<uint64_t> pow3;
  std::vector<std::vector<Cand>> lists;
  std::vector<uint8_t> done;
  uint64_t entries = 0, lookups = 0;

  KBest(const Shape& sh, int k) : s(sh), full((1u << sh.N) - 1), keep(k) {
    pow3.resize(s.N + 1);
    pow3[0] = 1;
    for (int j = 1; j <= s.N; ++j) pow3[j] = pow3[j - 1] * 3;
    lists.resize(pow3[s.N]);
    done.assign(pow3[s.N], 0);
  }
  uint64_t code(uint32_t P, uint32_t Q) const {
    uint64_t c = 0;
    for (int j = 0; j < s.N; ++j) c += pow3[j] * (((P >> j) & 1u) + 2u * ((Q >> j) & 1u));
    return c;
  }
  const std::vector<Cand>& solve(uint32_t P, uint32_t Q) {
    ++lookups;
    const uint64_t c = code(P, Q);
    if (done[c]) return lists[c];
    ++entries;
    std::vector<Cand> cands;
    const uint32_t R = full & ~(P | Q);
    if (R == 0 && (Q & (Q - 1)) == 0) {
      Cand cd{0, mix64(0x1000 + (uint64_t)lowest_bit(Q)), 0, 0, 0, 0, 0};
      cands.push_back(cd);
    } else {
      const uint64_t size = s.card(P);
      for (int n = 0; n < s.N; ++n) {
        if (!((R >> n) & 1u)) continue;
        const std::vector<Cand>& sub = solve(P | (1u << n), Q);
        const uint64_t own = sat_mul((uint64_t)s.K[n], size);
        for (size_t i = 0; i < sub.size(); ++i) {
          Cand cd{sat_add(own, sub[i].cost), mix64(mix64((uint64_t)n + 77) ^ sub[i].hash),
                  1u << n, 1, n, (int32_t)i, 0};
          cands.push_back(cd);
        }
      }
      const uint32_t low = Q & (~Q + 1u);
      for (uint32_t Q1 = (0u - Q) & Q; Q1 != 0 && Q1 != Q; Q1 = (Q1 - Q) & Q) {
        if (!(Q1 & low)) continue;
        const std::vector<Cand>& l1 = solve(P, Q1);
        const std::vector<Cand>& l2 = solve(P, Q ^ Q1);
        for (size_t i = 0; i < l1.size(); ++i)
          for (size_t j = 0; j < l2.size(); ++j) {
            if (l1[i].top_modes & l2[j].top_modes) continue;  // repeated sibling label
            Cand cd{sat_add(l1[i].cost, l2[j].cost), l1[i].hash + l2[j].hash,
                    l1[i].top_modes | l2[j].top_modes, 2, (int32_t)Q1, (int32_t)i, (int32_t)j};
            cands.push_back(cd);
          }
      }
      std::stable_sort(cands.begin(), cands.end(),
                       [](const Cand& x, const Cand& y) { return x.cost < y.cost; });
    }
    std::vector<Cand>& out = lists[c];
    std::unordered_set<uint64_t> seen;
    for (const Cand& cd : cands) {
      if ((int)out.size() >= keep) break;
      if (!seen.insert(cd.hash).second) continue;
      out.push_back(cd);
    }
    done[c] = 1;
    return out;
  }
  void build(Emitter& em, uint32_t P, uint32_t Q, int idx, int parent, int depth) {
    const Cand& cd = lists[code(P, Q)][idx];
    if (cd.kind == 0) {
      em.leaf(parent, depth, P, lowest_bit(Q));
    } else if (cd.kind == 1) {
      int me = em.internal(parent, depth, P, cd.a);
      build(em, P | (1u << cd.a), Q, cd.i1, me, depth + 1);
    } else {
      const uint32_t Q1 = (uint32_t)cd.a;
      build(em, P, Q1, cd.i1, parent, depth);
      build(em, P, Q ^ Q1, cd.i2, parent, depth);
    }
  }
};

// -------------------------------------------------------------- prior schemes --
void emit_chain(Emitter& em, const std::vector<int>& modes, int parent, int depth, uint32_t P,
                std::function<void(int, int, uint32_t)> below) {
  for (int m : modes) {
    parent = em.internal(parent, depth, P, m);
    P |= 1u << m;
    ++depth;
  }
  below(parent, depth, P);
}

void emit_balanced(Emitter& em, const std::vector<int>& S, int parent, int depth, uint32_t P) {
  if (S.size() == 1) {
    em.leaf(parent, depth, P, S[0]);
    return;
  }
  const size_t m = S.size() / 2;
  std::vector<int> S1(S.begin(), S.begin() + m), S2(S.begin() + m, S.end());
  emit_chain(em, S1, parent, depth, P,
             [&](int p, int d, uint32_t PP) { emit_balanced(em, S2, p, d, PP); });
  emit_chain(em, S2, parent, depth, P,
             [&](int p, int d, uint32_t PP) { emit_balanced(em, S1, p, d, PP); });
}

std::vector<int> mode_order(const Shape& s, int kind) {
  std::vector<int> o(s.N);
  for (int j = 0; j < s.N; ++j) o[j] = j;
  if (kind == TK_TREE_CHAIN_K) {
    std::stable_sort(o.begin(), o.end(), [&](int a, int b) { return s.K[a] < s.K[b]; });
  } else if (kind == TK_TREE_CHAIN_H) {
    // h_a < h_b  <=>  K_a L_b < K_b L_a (exact in 128-bit)
    std::stable_sort(o.begin(), o.end(), [&](int a, int b) {
      return (__int128)s.K[a] * s.L[b] < (__int128)s.K[b] * s.L[a];
    });
  }
  return o;
}

uint64_t sum_cost(const std::vector<tk_node>& nodes) {
  uint64_t c = 0;
  for (const tk_node& nd : nodes) c = sat_add(c, nd.macs);
  return c;
}

}  // namespace
}  // namespace tk

using namespace tk;

extern "C" int ttm_tree_plan(int N, const int64_t* L, const int64_t* K, int kind, int topk,
                             tk_plan** out) {
  clear_error();
  if (!out) return fail(TK_EINVAL, "out is null");
  Shape s;
  int rc = make_shape(N, L, K, &s);
  if (rc) return rc;
  if (topk < 1 || topk > 256) return fail(TK_EINVAL, "topk=%d outside [1, 256]", topk);
  if (kind < TK_TREE_DP || kind > TK_TREE_BALANCED) return fail(TK_EINVAL, "unknown tree kind %d", kind);
  if (kind == TK_TREE_DP && topk > 1 && N > 8)
    return fail(TK_EINVAL, "k-best planning supports N <= 8");
  tk_plan* p = new (std::nothrow) tk_plan;
  if (!p) return fail(TK_ENOMEM, "plan allocation failed");
  p->shape = s;
  p->kind = kind;
  const uint32_t full = (1u << N) - 1;
  try {
    if (kind == TK_TREE_DP && topk == 1) {
      DP dp(s);
      uint64_t c = dp.solve(0, full);
      if (c >= kInf) {
        delete p;
        return fail(TK_EINVAL, "tree cost overflows 64 bits");
      }
      Tree t;
      Emitter em{s, t.nodes};
      dp.build(em, 0, full, -1, 0);
      t.cost = c;
      p->trees.push_back(std::move(t));
      p->entries = dp.entries;
      p->lookups = dp.lookups;
    } else if (kind == TK_TREE_DP) {
      KBest kb(s, std::max(4 * topk, 16));
      const std::vector<Cand>& top = kb.solve(0, full);
      for (size_t i = 0; i < top.size() && (int)i < topk; ++i) {
        if (top[i].cost >= kInf) break;
        Tree t;
        Emitter em{s, t.nodes};
        kb.build(em, 0, full, (int)i, -1, 0);
        t.cost = top[i].cost;
        p->trees.push_back(std::move(t));
      }
      p->entries = kb.entries;
      p->lookups = kb.lookups;
    } else {
      Tree t;
      Emitter em{s, t.nodes};
      if (kind == TK_TREE_BALANCED) {
        std::vector<int> S(N);
        for (int j = 0; j < N; ++j) S[j] = j;
        emit_balanced(em, S, -1, 0, 0);
      } else {
        std::vector<int> order = mode_order(s, kind);
        for (int n = 0; n < N; ++n) {
          std::vector<int> ch;
          for (int j : order)
            if (j != n) ch.push_back(j);
          emit_chain(em, ch, -1, 0, 0,
                     [&](int par, int d, uint32_t PP) { em.leaf(par, d, PP, n); });
        }
      }
      t.cost = sum_cost(t.nodes);
      p->trees.push_back(std::move(t));
    }
  } catch (const std::bad_alloc&) {
    delete p;
    return fail(TK_ENOMEM, "planner ran out of host memory");
  }
  for (Tree& t : p->trees) {
    t.canon = canonical_string(t.nodes);
    if (sum_cost(t.nodes) != t.cost) {
      delete p;
      return fail(TK_EINVAL, "internal planner inconsistency");
    }
  }
  *out = p;
  return TK_OK;
}

extern "C" int tk_plan_count(const tk_plan* plan, int* count) {
  if (!plan || !count) return fail(TK_EINVAL, "null argument");
  *count = (int)plan->trees.size();
  return TK_OK;
}

static int check_rank(const tk_plan* plan, int rank) {
  if (!plan) return fail(TK_EINVAL, "plan is null");
  if (rank < 0 || rank >= (int)plan->trees.size())
    return fail(TK_EINVAL, "rank %d outside [0, %d)", rank, (int)plan->trees.size());
  return TK_OK;
}

extern "C" int tk_plan_cost(const tk_plan* plan, int rank, uint64_t* macs) {
  if (int rc = check_rank(plan, rank)) return rc;
  if (!macs) return fail(TK_EINVAL, "macs is null");
  *macs = plan->trees[rank].cost;
  return TK_OK;
}

extern "C" int tk_plan_string(const tk_plan* plan, int rank, char* buf, size_t cap) {
  if (int rc = check_rank(plan, rank)) return rc;
  const std::string& s = plan->trees[rank].canon;
  if (!buf || cap < s.size() + 1)
    return fail(TK_EINVAL, "buffer of %zu bytes too small for %zu", cap, s.size() + 1);
  memcpy(buf, s.c_str(), s.size() + 1);
  return TK_OK;
}

extern "C" int tk_plan_nodes(const tk_plan* plan, int rank, tk_node* out, int cap, int* n) {
  if (int rc = check_rank(plan, rank)) return rc;
  if (!n) return fail(TK_EINVAL, "n is null");
  const auto& nodes = plan->trees[rank].nodes;
  *n = (int)nodes.size();
  if (out) {
    if (cap < 0) return fail(TK_EINVAL, "cap < 0");
    int m = std::min(cap, (int)nodes.size());
    memcpy(out, nodes.data(), sizeof(tk_node) * (size_t)m);
  }
  return TK_OK;
}

extern "C" int tk_plan_stats(const tk_plan* plan, uint64_t* entries, uint64_t* lookups) {
  if (!plan) return fail(TK_EINVAL, "plan is null");
  if (entries) *entries = plan->entries;
  if (lookups) *lookups = plan->lookups;
  return TK_OK;
}

extern "C" int tk_plan_workspace(const tk_plan* plan, int rank, uint64_t* elements) {
  if (int rc = check_rank(plan, rank)) return rc;
  if (!elements) return fail(TK_EINVAL, "elements is null");
  *elements = workspace_elements(plan->trees[rank].nodes);
  return TK_OK;
}

extern "C" int tk_plan_select(tk_plan* plan, int rank) {
  if (int rc = check_rank(plan, rank)) return rc;
  plan->selected = rank;
  return TK_OK;
}

extern "C" void tk_plan_free(tk_plan* plan) { delete plan; }

extern "C" const char* tk_last_error(void) { return tk::g_last_error.c_str(); }
