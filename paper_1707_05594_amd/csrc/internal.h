// Internal declarations shared by the host-side sources of libtucker.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tucker.h"

namespace tk {

// Record the calling thread's last error and return `code`.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

struct Shape {
  int N = 0;
  int64_t L[TK_MAX_MODES] = {};
  int64_t K[TK_MAX_MODES] = {};
  uint64_t card_T() const {
    uint64_t c = 1;
    for (int j = 0; j < N; ++j) c *= (uint64_t)L[j];
    return c;
  }
  // |T[P]|: T after multiplying along the modes of bitmask P.
  uint64_t card(uint32_t P) const {
    uint64_t c = 1;
    for (int j = 0; j < N; ++j) c *= (uint64_t)(((P >> j) & 1u) ? K[j] : L[j]);
    return c;
  }
  bool same(const Shape& o) const {
    if (N != o.N) return false;
    for (int j = 0; j < N; ++j)
      if (L[j] != o.L[j] || K[j] != o.K[j]) return false;
    return true;
  }
};

// [A, L, B] view of a node's input: In(u) has multiplied the modes in `pre`
// (lengths K there, L elsewhere); the node multiplies along mode n.
inline void view(const Shape& s, uint32_t pre, int n, int64_t* A, int64_t* L, int64_t* B) {
  int64_t a = 1, b = 1;
  for (int j = 0; j < s.N; ++j) {
    const int64_t d = ((pre >> j) & 1u) ? s.K[j] : s.L[j];
    if (j < n) a *= d;
    if (j > n) b *= d;
  }
  *A = a;
  *L = ((pre >> n) & 1u) ? s.K[n] : s.L[n];
  *B = b;
}

// Checks 2 <= N <= TK_MAX_MODES, 1 <= K_n <= L_n, K_n <= prod_{m!=n} K_m,
// prod(L) < 2^62.  Fills `s`.  Returns TK_OK or TK_EINVAL (with message).
int make_shape(int N, const int64_t* L, const int64_t* K, Shape* s);

struct Tree {
  std::vector<tk_node> nodes;  // depth-first execution order, parents first
  uint64_t cost = 0;           // multiply-adds
  std::string canon;           // canonical text
};

std::string canonical_string(const std::vector<tk_node>& nodes);
uint64_t workspace_elements(const std::vector<tk_node>& nodes);

// Precision of every node of a tree as the engine runs it (engine.cpp):
//   fold_leaf: the leaf whose tensor folds the core (smallest Y, lowest mode);
//   node_compute[u]: `compute`, except FP32 on the path from the root to the
//     fold leaf in the BF16 modes (the core is formed at FP32);
//   out_dt[u]: storage of node u's output: BF16 when u runs the BF16 mode, no
//     child of u is a leaf, and u and every child have a BF16 kernel for it
//     (BF16 output and input); else FP32 (FP64 for FP64 compute).
// T: the tensor's device address (its alignment picks kernels); the
// intermediates are taken to sit at the engine's 64-element-aligned offsets.
// tiles: per-node kernel choices (TK_TILE_*), or empty for automatic.
void tree_precisions(const Shape& s, const std::vector<tk_node>& nodes, int tdtype, int compute,
                     const std::vector<int>& tiles, const void* T, int* fold_leaf,
                     std::vector<int>* node_compute, std::vector<int>* out_dt);

}  // namespace tk

struct tk_plan {
  tk::Shape shape;
  int kind = 0;
  int selected = 0;  // rank used by hooi_init
  std::vector<tk::Tree> trees;
  // per tree: TK_TILE_* of every node (empty: TK_TILE_AUTO everywhere)
  std::vector<std::vector<int>> tiles;
  uint64_t entries = 0, lookups = 0;
};

// Return TK_EDEVICE with the HIP error text from a function returning int.
#define TK_HIP(call)                                                          \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess)                                                     \
      return tk::fail(TK_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)
