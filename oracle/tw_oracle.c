/*
 * CPU oracle for exact treewidth by elimination orderings.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no code, header, table or constant with the
 * HIP path.
 *
 * Everything here is deliberately plain and slow:
 *
 *   - Q(S,v) follows the definition in §2 (Preliminaries): the vertices
 *     outside S, other than v, that v reaches by paths whose internal
 *     vertices all lie in S.  It is computed as a closure on vertex sets:
 *     start from the neighbours of v; whenever a vertex of S is in the set,
 *     add its neighbours; stop when nothing changes; then drop S and v
 *     (reading: v is not a member of Q(S,v)).
 *
 *   - O1, the subset dynamic programme (§1 and §2: eliminating a set S gives
 *     the same intermediate graph whatever the order, so a Held-Karp style
 *     recurrence over subsets works):
 *        TW(empty) = 0,
 *        TW(S) = min over v in S of max(TW(S - v), |Q(S - v, v)|),
 *     and tw(G) = TW(V).
 *
 *   - O2, brute force over all n! orders with the width of each order found by
 *     explicit fill-in (§2, the alternative view: eliminating v removes it and
 *     turns its neighbourhood into a clique; the width is the largest degree
 *     met).  A second, independent definition used to pin O1.
 *
 *   - O4, the level-by-level search of Listing 1 (§3.1) for one bound k: every
 *     set S of the input list is extended by every vertex v outside S whose
 *     degree |Q(S,v)| is at most k; duplicates are removed exactly (sort and
 *     unique, not a Bloom filter).
 *
 *   - O6, per-state minor-min-width pruning (§3.3, applied to the graph that
 *     remains once S is eliminated).  That graph H_S has vertex set V - S and
 *     an edge uw exactly when w lies in Q(S, u) (§2).  MMW repeatedly records
 *     the second-smallest degree, takes the lowest-index vertex of minimum
 *     degree, deletes it if isolated and otherwise contracts it into its
 *     lowest-index minimum-degree neighbour; the bound is the largest
 *     recorded degree.  A state with MMW(H_S) > k cannot be completed within
 *     width k and is not expanded.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC -o libtworacle.so tw_oracle.c
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXN 64

/* Q(S,v) of §2 as a vertex set.  `reach` collects every vertex joined to v
 * by a path whose internal vertices lie in S: the neighbours of v, and the
 * neighbours of every vertex of S already collected.  `spent` marks the
 * vertices of S whose neighbours were added.  v must lie outside S. */
static uint64_t q_set(const uint64_t *rows, uint64_t S, int v)
{
    uint64_t reach = rows[v];
    uint64_t spent = 0;
    for (;;) {
        uint64_t open = reach & S & ~spent;
        if (!open)
            break;
        int u = __builtin_ctzll(open);
        spent |= 1ULL << u;
        reach |= rows[u];
    }
    return reach & ~S & ~(1ULL << v);
}

static int q_degree(const uint64_t *rows, uint64_t S, int v)
{
    return __builtin_popcountll(q_set(rows, S, v));
}

int tworacle_q_degree(int n, const uint64_t *rows, uint64_t S, int v)
{
    if (n < 1 || n > MAXN || v < 0 || v >= n || ((S >> v) & 1ULL))
        return -1;
    return q_degree(rows, S, v);
}

static int popcount64(uint64_t x)
{
    int c = 0;
    while (x) {
        x &= x - 1;
        c++;
    }
    return c;
}

/* O1: fills tw_table[S] = TW(S) for all 2^n subsets S, returns TW(V).
 * Subsets are processed one cardinality at a time; within a cardinality every
 * entry depends only on the previous one, so those entries are independent. */
int tworacle_subset_dp(int n, const uint64_t *rows, uint8_t *tw_table, int nthreads)
{
    if (n < 1 || n > 30)
        return -1;
    const int64_t total = (int64_t)1 << n;
    tw_table[0] = 0;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#endif
    for (int c = 1; c <= n; c++) {
#pragma omp parallel for schedule(dynamic, 4096)
        for (int64_t S = 1; S < total; S++) {
            if (popcount64((uint64_t)S) != c)
                continue;
            int best = 255;
            for (int v = 0; v < n; v++) {
                if (!(((uint64_t)S >> v) & 1ULL))
                    continue;
                uint64_t R = (uint64_t)S & ~(1ULL << v);
                int d = q_degree(rows, R, v);
                int w = tw_table[R] > d ? tw_table[R] : d;
                if (w < best)
                    best = w;
            }
            tw_table[S] = (uint8_t)best;
        }
    }
    return tw_table[total - 1];
}

/* Level i of the bound-k search read off an O1 table: all S with |S| = i and
 * TW(S) <= k, in ascending order.  Returns the count (or -1 if it exceeds cap;
 * out may be NULL to only count). */
int64_t tworacle_frontier_from_table(int n, const uint8_t *tw_table, int i, int k,
                                     uint64_t *out, int64_t cap)
{
    const int64_t total = (int64_t)1 << n;
    int64_t cnt = 0;
    for (int64_t S = 0; S < total; S++) {
        if (popcount64((uint64_t)S) == i && tw_table[S] <= k) {
            if (out) {
                if (cnt >= cap)
                    return -1;
                out[cnt] = (uint64_t)S;
            }
            cnt++;
        }
    }
    return cnt;
}

/* Width of an elimination order by explicit fill-in (§2, alternative view).
 * Returns -1 if order is not a permutation of 0..n-1. */
static int fill_in_width(int n, const unsigned char adj0[MAXN][MAXN], const int *order)
{
    unsigned char adj[MAXN][MAXN];
    unsigned char alive[MAXN];
    memcpy(adj, adj0, sizeof adj);
    for (int u = 0; u < n; u++)
        alive[u] = 1;
    int width = 0;
    for (int t = 0; t < n; t++) {
        int v = order[t];
        int nb[MAXN], d = 0;
        for (int u = 0; u < n; u++)
            if (alive[u] && u != v && adj[v][u])
                nb[d++] = u;
        if (d > width)
            width = d;
        for (int a = 0; a < d; a++)
            for (int b = 0; b < d; b++)
                if (a != b)
                    adj[nb[a]][nb[b]] = 1;
        alive[v] = 0;
    }
    return width;
}

static void build_matrix(int n, const uint64_t *rows, unsigned char adj[MAXN][MAXN])
{
    memset(adj, 0, sizeof(unsigned char) * MAXN * MAXN);
    for (int u = 0; u < n; u++)
        for (int w = 0; w < n; w++)
            adj[u][w] = (unsigned char)((rows[u] >> w) & 1ULL);
}

int tworacle_order_width(int n, const uint64_t *rows, const int32_t *order)
{
    unsigned char adj[MAXN][MAXN];
    unsigned char seen[MAXN];
    int ord[MAXN];
    if (n < 1 || n > MAXN)
        return -1;
    memset(seen, 0, sizeof seen);
    for (int t = 0; t < n; t++) {
        if (order[t] < 0 || order[t] >= n || seen[order[t]])
            return -1;
        seen[order[t]] = 1;
        ord[t] = order[t];
    }
    build_matrix(n, rows, adj);
    return fill_in_width(n, adj, ord);
}

/* O2: minimum fill-in width over all n! orders (lexicographic enumeration).
 * best_order (nullable) receives the first order reaching the minimum. */
int tworacle_brute_force(int n, const uint64_t *rows, int32_t *best_order)
{
    unsigned char adj[MAXN][MAXN];
    int p[MAXN];
    if (n < 1 || n > 10)
        return -1;
    build_matrix(n, rows, adj);
    for (int t = 0; t < n; t++)
        p[t] = t;
    int best = n;
    for (;;) {
        int w = fill_in_width(n, adj, p);
        if (w < best) {
            best = w;
            if (best_order)
                for (int t = 0; t < n; t++)
                    best_order[t] = p[t];
        }
        /* next permutation in lexicographic order */
        int a = n - 2;
        while (a >= 0 && p[a] > p[a + 1])
            a--;
        if (a < 0)
            break;
        int b = n - 1;
        while (p[b] < p[a])
            b--;
        int tmp = p[a];
        p[a] = p[b];
        p[b] = tmp;
        for (int l = a + 1, r = n - 1; l < r; l++, r--) {
            tmp = p[l];
            p[l] = p[r];
            p[r] = tmp;
        }
    }
    return best;
}

/* LSD radix sort of 64-bit keys, 16 bits per pass (tmp has the same size). */
static void radix_sort(uint64_t *a, uint64_t *tmp, int64_t cnt)
{
    static int64_t hist[1 << 16];
    uint64_t all_or = 0;
    for (int64_t t = 0; t < cnt; t++)
        all_or |= a[t];
    for (int shift = 0; shift < 64; shift += 16) {
        if (((all_or >> shift) & 0xFFFFULL) == 0)
            continue;
        memset(hist, 0, sizeof hist);
        for (int64_t t = 0; t < cnt; t++)
            hist[(a[t] >> shift) & 0xFFFF]++;
        int64_t sum = 0;
        for (int d = 0; d < (1 << 16); d++) {
            int64_t h = hist[d];
            hist[d] = sum;
            sum += h;
        }
        for (int64_t t = 0; t < cnt; t++)
            tmp[hist[(a[t] >> shift) & 0xFFFF]++] = a[t];
        memcpy(a, tmp, (size_t)cnt * sizeof(uint64_t));
    }
}

/* Which of `nparts` (a power of two) classes a successor key falls in:
 * three 21-bit pieces of the key folded by xor, low bits taken.  Only used to
 * split one level's successors into groups that are deduplicated one at a
 * time; equal keys always land in the same group. */
static int key_part(uint64_t key, int nparts)
{
    return (int)((key ^ (key >> 21) ^ (key >> 42)) & (uint64_t)(nparts - 1));
}

/* O4, one level of Listing 1 (§3.1) for the bound k: every S of in[] is
 * extended by every v of `allowed` outside S with |Q(S,v)| <= k; the
 * successors are sorted and duplicates removed.  Only vertices in `allowed`
 * may be added (all vertices: the plain search; the complement of a maximum
 * clique: the first optimisation of §3.1, which never picks a clique vertex
 * because some optimal order eliminates the clique last).
 *
 * With nparts > 1 only the successors whose key_part is `part` are produced
 * (and only their pairs counted), so a level too large for memory is built
 * group by group; the groups of one level are disjoint and together give the
 * whole level.
 *
 * *out receives a malloc'd array (free it with tworacle_free) of the distinct
 * successors in ascending order.  Returns their number, or -1 on a bad
 * argument or allocation failure.  *generated (nullable) receives the number
 * of feasible (S,v) pairs, *candidates (nullable) the number of (S,v) pairs
 * tried. */
int64_t tworacle_bfs_level_part(int n, const uint64_t *rows, int k, uint64_t allowed,
                                const uint64_t *in, int64_t in_count, int nparts, int part,
                                uint64_t **out, int64_t *generated, int64_t *candidates, int nthreads)
{
    if (n < 1 || n > MAXN || in_count < 0 || nparts < 1 || (nparts & (nparts - 1)) != 0 ||
        part < 0 || part >= nparts)
        return -1;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
    int nt = omp_get_max_threads();
#else
    int nt = 1;
#endif
    uint64_t **buf = calloc((size_t)nt, sizeof(uint64_t *));
    int64_t *len = calloc((size_t)nt, sizeof(int64_t));
    int64_t *capb = calloc((size_t)nt, sizeof(int64_t));
    int64_t *tried = calloc((size_t)nt, sizeof(int64_t));
    int fail = 0;
#pragma omp parallel
    {
#ifdef _OPENMP
        int tid = omp_get_thread_num();
#else
        int tid = 0;
#endif
#pragma omp for schedule(dynamic, 256)
        for (int64_t s = 0; s < in_count; s++) {
            uint64_t S = in[s];
            for (int v = 0; v < n; v++) {
                if (((S >> v) & 1ULL) || !((allowed >> v) & 1ULL))
                    continue;
                uint64_t key = S | (1ULL << v);
                if (nparts > 1 && key_part(key, nparts) != part)
                    continue;
                tried[tid]++;
                if (q_degree(rows, S, v) <= k) {
                    if (len[tid] == capb[tid]) {
                        int64_t nc = capb[tid] ? capb[tid] + capb[tid] / 2 : 4096;
                        uint64_t *nb = realloc(buf[tid], (size_t)nc * sizeof(uint64_t));
                        if (!nb) {
                            fail = 1;
                            continue;
                        }
                        buf[tid] = nb;
                        capb[tid] = nc;
                    }
                    buf[tid][len[tid]++] = key;
                }
            }
        }
    }
    int64_t total = 0, ntried = 0;
    for (int t = 0; t < nt; t++) {
        total += len[t];
        ntried += tried[t];
    }
    int64_t result = -1;
    uint64_t *all_keys = NULL, *tmp = NULL;
    if (!fail)
        all_keys = malloc((size_t)(total ? total : 1) * sizeof(uint64_t));
    if (all_keys) {
        int64_t pos = 0;
        for (int t = 0; t < nt; t++) {
            if (len[t])
                memcpy(all_keys + pos, buf[t], (size_t)len[t] * sizeof(uint64_t));
            pos += len[t];
            free(buf[t]);
            buf[t] = NULL;
        }
        tmp = malloc((size_t)(total ? total : 1) * sizeof(uint64_t));
    }
    if (all_keys && tmp) {
        radix_sort(all_keys, tmp, total);
        int64_t u = 0;
        for (int64_t t = 0; t < total; t++)
            if (t == 0 || all_keys[t] != all_keys[t - 1])
                all_keys[u++] = all_keys[t];
        *out = all_keys;
        all_keys = NULL;
        result = u;
        if (generated)
            *generated = total;
        if (candidates)
            *candidates = ntried;
    }
    for (int t = 0; t < nt; t++)
        free(buf[t]);
    free(all_keys);
    free(tmp);
    free(buf);
    free(len);
    free(capb);
    free(tried);
    return result;
}

int64_t tworacle_bfs_level_masked(int n, const uint64_t *rows, int k, uint64_t allowed,
                                  const uint64_t *in, int64_t in_count, uint64_t **out,
                                  int64_t *generated, int64_t *candidates, int nthreads)
{
    return tworacle_bfs_level_part(n, rows, k, allowed, in, in_count, 1, 0, out, generated, candidates,
                                   nthreads);
}

int64_t tworacle_bfs_level(int n, const uint64_t *rows, int k, const uint64_t *in,
                           int64_t in_count, uint64_t **out,
                           int64_t *generated, int64_t *candidates, int nthreads)
{
    return tworacle_bfs_level_part(n, rows, k, ~0ULL, in, in_count, 1, 0, out, generated, candidates,
                                   nthreads);
}

void tworacle_free(void *p)
{
    free(p);
}

/* Number of feasible (S,v) pairs over a list of states, without storing them
 * (used to time the oracle on a bounded sample). */
int64_t tworacle_count_feasible(int n, const uint64_t *rows, int k, const uint64_t *in,
                                int64_t in_count, int64_t *candidates, int nthreads)
{
    if (n < 1 || n > MAXN)
        return -1;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#endif
    int64_t feas = 0, tried = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : feas, tried)
    for (int64_t s = 0; s < in_count; s++) {
        uint64_t S = in[s];
        for (int v = 0; v < n; v++) {
            if ((S >> v) & 1ULL)
                continue;
            tried++;
            if (q_degree(rows, S, v) <= k)
                feas++;
        }
    }
    if (candidates)
        *candidates = tried;
    return feas;
}

int tworacle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---- O6: per-state minor-min-width ------------------------------------ */

/* out[u] = Q(S, u) for u outside S, 0 for u in S: the rows of H_S. */
int tworacle_eliminated_graph(int n, const uint64_t *rows, uint64_t S, uint64_t *out)
{
    if (n < 1 || n > MAXN)
        return -1;
    for (int u = 0; u < n; u++)
        out[u] = ((S >> u) & 1ULL) ? 0 : q_set(rows, S, u);
    return 0;
}

/* MMW of the graph on the vertices of `alive` with neighbour sets nb[]
 * (modified in place). */
static int mmw_on(int n, uint64_t *nb, uint64_t alive)
{
    int lb = 0;
    while (popcount64(alive) >= 2) {
        int v = -1, d1 = MAXN + 1;
        for (int u = 0; u < n; u++)
            if (((alive >> u) & 1ULL) && popcount64(nb[u]) < d1) {
                d1 = popcount64(nb[u]);
                v = u;
            }
        int d2 = MAXN + 1;
        for (int u = 0; u < n; u++)
            if (u != v && ((alive >> u) & 1ULL) && popcount64(nb[u]) < d2)
                d2 = popcount64(nb[u]);
        if (d2 > lb)
            lb = d2;
        if (nb[v] == 0) {
            alive &= ~(1ULL << v);
            continue;
        }
        int c = -1, dc = MAXN + 1;
        for (int w = 0; w < n; w++)
            if (((nb[v] >> w) & 1ULL) && popcount64(nb[w]) < dc) {
                dc = popcount64(nb[w]);
                c = w;
            }
        /* contract v into c: c keeps its label and gains v's other neighbours */
        for (int w = 0; w < n; w++) {
            if (!((nb[v] >> w) & 1ULL))
                continue;
            nb[w] &= ~(1ULL << v);
            if (w != c) {
                nb[w] |= 1ULL << c;
                nb[c] |= 1ULL << w;
            }
        }
        nb[v] = 0;
        alive &= ~(1ULL << v);
    }
    return lb;
}

int tworacle_mmw(int n, const uint64_t *rows)
{
    uint64_t nb[MAXN];
    if (n < 1 || n > MAXN)
        return -1;
    memcpy(nb, rows, sizeof(uint64_t) * (size_t)n);
    return mmw_on(n, nb, n == 64 ? ~0ULL : (1ULL << n) - 1);
}

/* MMW(H_S). */
int tworacle_mmw_eliminated(int n, const uint64_t *rows, uint64_t S)
{
    uint64_t nb[MAXN];
    if (tworacle_eliminated_graph(n, rows, S, nb) != 0)
        return -1;
    const uint64_t all = n == 64 ? ~0ULL : (1ULL << n) - 1;
    return mmw_on(n, nb, all & ~S);
}

/* keep[s] = 1 iff MMW(H_S) <= k for S = states[s]; returns how many are kept. */
int64_t tworacle_mmw_keep(int n, const uint64_t *rows, int k, const uint64_t *states, int64_t count,
                          uint8_t *keep, int nthreads)
{
    if (n < 1 || n > MAXN)
        return -1;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#endif
    int64_t kept = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : kept)
    for (int64_t s = 0; s < count; s++) {
        keep[s] = tworacle_mmw_eliminated(n, rows, states[s]) <= k;
        kept += keep[s];
    }
    return kept;
}
