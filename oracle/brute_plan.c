/*
 * Brute-force enumeration of TTM-trees -- test infrastructure only (oracle).
 *
 * A TTM-tree (Sec. 3.1, definition of TTM-trees) gives every leaf F_n a
 * root-to-leaf path that holds each mode other than n exactly once.  Fix one
 * ordering of the N-1 modes for every leaf (((N-1)!)^N choices, Sec. 3.3
 * Remarks); merging equal path prefixes turns the N chains into a trie, and
 * every TTM-tree that does not repeat a label among siblings is such a trie.
 * (Repeating a label among siblings only adds a TTM, so the minimum over all
 * trees is reached by a trie.)
 *
 * The cost of a tree is the sum over internal nodes u of K_n * |In(u)| with
 * |Out(u)| = (K_n / L_n) |In(u)| (Sec. 3.1, computational load).
 *
 * brute_plan() walks all tries for N <= 6 (N = 6 is only practical for tiny
 * k-best requests on small inputs; the tests use N <= 5), returning the
 * minimum cost, how many tries reach it, and the k cheapest tries with their
 * paths.  Exact 64-bit integer arithmetic throughout.
 */
#include <stdint.h>
#include <string.h>

#define BP_MAXN 6
#define BP_MAXNODES (BP_MAXN * BP_MAXN + 2)
#define BP_MAXK 256

typedef unsigned long long u64;

static int bp_N;
static u64 bp_L[BP_MAXN], bp_K[BP_MAXN];
static int bp_child[BP_MAXNODES][BP_MAXN];
static u64 bp_out[BP_MAXNODES];
static int bp_nnodes;
static int bp_paths[BP_MAXN][BP_MAXN]; /* current path of every leaf */

static int bp_k;
static int bp_nbest;
static u64 bp_best_cost[BP_MAXK];
static int bp_best_paths[BP_MAXK][BP_MAXN][BP_MAXN];
static u64 bp_min_cost, bp_min_count;

static int next_permutation(int *a, int n) {
    int i = n - 2;
    while (i >= 0 && a[i] >= a[i + 1]) i--;
    if (i < 0) return 0;
    int j = n - 1;
    while (a[j] <= a[i]) j--;
    int t = a[i]; a[i] = a[j]; a[j] = t;
    for (int l = i + 1, r = n - 1; l < r; l++, r--) { t = a[l]; a[l] = a[r]; a[r] = t; }
    return 1;
}

static void record(u64 cost) {
    if (cost < bp_min_cost) { bp_min_cost = cost; bp_min_count = 1; }
    else if (cost == bp_min_cost) bp_min_count++;
    if (bp_k <= 0) return;
    int slot = -1;
    if (bp_nbest < bp_k) {
        slot = bp_nbest++;
    } else {
        int worst = 0;
        for (int i = 1; i < bp_nbest; i++)
            if (bp_best_cost[i] > bp_best_cost[worst]) worst = i;
        if (cost < bp_best_cost[worst]) slot = worst;
    }
    if (slot < 0) return;
    bp_best_cost[slot] = cost;
    memcpy(bp_best_paths[slot], bp_paths, sizeof(bp_paths));
}

static void walk(int n, u64 cost) {
    if (n == bp_N) { record(cost); return; }
    int perm[BP_MAXN];
    int m = 0;
    for (int j = 0; j < bp_N; j++) if (j != n) perm[m++] = j;
    do {
        /* insert the path for leaf n, remembering which nodes were created */
        int made_parent[BP_MAXN], made_mode[BP_MAXN], nmade = 0;
        int cur = 0;
        u64 add = 0;
        for (int i = 0; i < m; i++) {
            int md = perm[i];
            if (bp_child[cur][md] < 0) {
                int nu = bp_nnodes++;
                for (int j = 0; j < bp_N; j++) bp_child[nu][j] = -1;
                bp_out[nu] = bp_out[cur] / bp_L[md] * bp_K[md];
                add += bp_K[md] * bp_out[cur];
                bp_child[cur][md] = nu;
                made_parent[nmade] = cur;
                made_mode[nmade] = md;
                nmade++;
            }
            cur = bp_child[cur][md];
        }
        for (int i = 0; i < m; i++) bp_paths[n][i] = perm[i];
        walk(n + 1, cost + add);
        for (int i = nmade - 1; i >= 0; i--) {
            bp_child[made_parent[i]][made_mode[i]] = -1;
            bp_nnodes--;
        }
    } while (next_permutation(perm, m));
}

/* Returns 0 on success, -1 on bad arguments.  paths_out holds, for each of the
 * *nout best tries, N rows of N-1 modes (row n = path of leaf n). */
int brute_plan(int N, const u64 *L, const u64 *K, int k, u64 *min_cost,
               u64 *min_count, u64 *costs_out, int *paths_out, int *nout) {
    if (N < 2 || N > BP_MAXN || k < 0 || k > BP_MAXK) return -1;
    bp_N = N;
    u64 size = 1;
    for (int j = 0; j < N; j++) {
        if (K[j] < 1 || K[j] > L[j]) return -1;
        bp_L[j] = L[j];
        bp_K[j] = K[j];
        size *= L[j];
    }
    bp_nnodes = 1;
    for (int j = 0; j < N; j++) bp_child[0][j] = -1;
    bp_out[0] = size;
    bp_k = k;
    bp_nbest = 0;
    bp_min_cost = ~0ULL;
    bp_min_count = 0;
    walk(0, 0);
    *min_cost = bp_min_cost;
    *min_count = bp_min_count;
    /* sort the kept tries by cost (insertion sort, stable on equal cost) */
    int order[BP_MAXK];
    for (int i = 0; i < bp_nbest; i++) order[i] = i;
    for (int i = 1; i < bp_nbest; i++) {
        int v = order[i], j = i - 1;
        while (j >= 0 && bp_best_cost[order[j]] > bp_best_cost[v]) { order[j + 1] = order[j]; j--; }
        order[j + 1] = v;
    }
    for (int i = 0; i < bp_nbest; i++) {
        costs_out[i] = bp_best_cost[order[i]];
        for (int n = 0; n < N; n++)
            for (int s = 0; s < N - 1; s++)
                paths_out[(i * N + n) * (N - 1) + s] = bp_best_paths[order[i]][n][s];
    }
    *nout = bp_nbest;
    return 0;
}
