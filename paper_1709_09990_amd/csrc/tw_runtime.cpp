// Host runtime of libtw: the C-ABI of include/tw.h.
//
// decide(k) runs the level loop of Listing 1 (§3.1) on the device: level 0 is
// {empty set}; each level is one expansion launch into an exact hash table and
// a compacted next level.  The next level's size is unknown before the launch,
// so it is estimated from the growth of the previous level; if the launch
// overflows its output capacity (or the table's probe backstop), the level is
// replayed with larger buffers — an exact answer is never traded for memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cmath>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "tw.h"
#include "tw_probe.h"
#include "tw_mmw.h"
#include "tw_batch.h"
#include "tw_internal.h"

namespace {

using twk::LevelCounters;

// First-fit allocator over one caller-given device range (options.workspace,
// or the static scratch of tw_solve_noalloc): host bookkeeping only, blocks of
// 256-byte multiples, neighbours merged on release.
struct Carver {
    uintptr_t base = 0;
    size_t bytes = 0;
    std::vector<std::pair<size_t, size_t>> free_list;  // (offset, size), ascending, merged

    static size_t round_up(size_t n) { return (n + 255) & ~(size_t)255; }
    void reset(void *p, size_t n)
    {
        const uintptr_t b = ((uintptr_t)p + 255) & ~(uintptr_t)255;
        const size_t lost = (size_t)(b - (uintptr_t)p);
        base = b;
        bytes = n > lost ? (n - lost) & ~(size_t)255 : 0;
        free_list.clear();
        if (bytes)
            free_list.emplace_back(0, bytes);
    }
    void *take(size_t n)
    {
        n = round_up(n);
        for (size_t t = 0; t < free_list.size(); ++t) {
            if (free_list[t].second < n)
                continue;
            const size_t off = free_list[t].first;
            free_list[t].first += n;
            free_list[t].second -= n;
            if (!free_list[t].second)
                free_list.erase(free_list.begin() + (long)t);
            return (void *)(base + off);
        }
        return nullptr;
    }
    void put(void *p, size_t n)
    {
        n = round_up(n);
        const size_t off = (size_t)((uintptr_t)p - base);
        size_t i = 0;
        while (i < free_list.size() && free_list[i].first < off)
            ++i;
        free_list.insert(free_list.begin() + (long)i, std::make_pair(off, n));
        if (i + 1 < free_list.size() && free_list[i].first + free_list[i].second == free_list[i + 1].first) {
            free_list[i].second += free_list[i + 1].second;
            free_list.erase(free_list.begin() + (long)i + 1);
        }
        if (i > 0 && free_list[i - 1].first + free_list[i - 1].second == free_list[i].first) {
            free_list[i - 1].second += free_list[i].second;
            free_list.erase(free_list.begin() + (long)i);
        }
    }
    size_t largest() const
    {
        size_t m = 0;
        for (const auto &f : free_list)
            m = std::max(m, f.second);
        return m;
    }
};

struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
    Carver *from = nullptr;  // carved from a caller range (null: hipMalloc)
};

struct Captured;  // an instantiated level loop (below)

struct Level {
    Buf keys;
    Buf lastv;
    uint64_t count = 0;
};

struct Graph {
    int n = 0;
    uint64_t rows[64] = {};
};

}  // namespace

// Device memory of tw_solve_noalloc: one array per GPU, held until the process
// ends.  Host code never passes `scratch` itself to a kernel (on the host the
// name is a stand-in, not a device address): the address of each device's
// copy is looked up once per device with hipGetSymbolAddress and kept in
// g_scratch_ptr.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kNoAllocMaxN = 32;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::atomic<void *> g_scratch_ptr[kMaxDevices];

// With device `device` current: the address of its copy of `scratch`.
hipError_t scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return hipErrorInvalidDevice;
    if (g_scratch_ptr[device].load())
        return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return e != hipSuccess ? e : hipErrorInvalidSymbol;
    g_scratch_ptr[device].store(ptr);
    return hipSuccess;
}

}  // namespace

struct tw_ctx {
    tw_options opt{};
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int cu_count = 256;
    std::string err;
    std::vector<Buf> cache;  // free device buffers kept for reuse
    Buf d_adj, d_ctr, d_find;
    Buf d_adj_wide;          // two words per row (graphs of up to 126 vertices)
    Buf table;               // current hash table (reused between levels)
    Buf bloom;               // Bloom bit array (Bloom variant only)
    Buf parts, part_meta;    // partitioned insert: successor buffer, counters and prefixes
    LevelCounters *h_ctr = nullptr;      // pinned host mirror
    unsigned long long *h_find = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    tw_mpnn *net = nullptr;  // learned start bound (k_policy = TW_K_LEARNED)
    Carver ws;               // options.workspace, when given
    Carver *carve = nullptr; // where device buffers come from (null: hipMalloc)
    uint64_t keep_budget = 1ull << 30;  // bytes of levels tw_solve keeps for the order
    bool no_capture = false; // set while a call must not create graphs or pinned memory
    std::vector<Captured *> captured;  // instantiated level loops, by graph shape
    int batch_leave_blocks = 0; // persistent batch grid: blocks per CU left to concurrent single-graph work
    void *h_cap = nullptr;   // pinned host block for the captured loop's control and counters
};

namespace {

tw_status fail(tw_ctx *c, tw_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c)
        c->err = buf;
    return s;
}

#define HIP_TRY(c, expr)                                                                    \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((c), e_ == hipErrorOutOfMemory ? TW_ENOMEM : TW_EDEVICE, "%s: %s", \
                        #expr, hipGetErrorString(e_));                                      \
    } while (0)

int popc(uint64_t x) { return __builtin_popcountll(x); }

uint64_t binom_sat(int n, int r)
{
    if (r < 0 || r > n)
        return 0;
    r = std::min(r, n - r);
    unsigned __int128 v = 1;
    for (int t = 1; t <= r; ++t) {
        v = v * (unsigned)(n - r + t) / (unsigned)t;
        if (v > (unsigned __int128)UINT64_MAX)
            return UINT64_MAX;
    }
    return (uint64_t)v;
}

uint64_t pow2_at_least(uint64_t x)
{
    uint64_t p = 64;
    while (p < x)
        p <<= 1;
    return p;
}

tw_status validate(tw_ctx *c, const tw_graph *g, Graph &out)
{
    if (!g || !g->adj)
        return fail(c, TW_EINVAL, "graph or adjacency pointer is NULL");
    if (g->n < 1 || g->n > 64)
        return fail(c, TW_EINVAL, "n=%u outside 1..64", g->n);
    out.n = (int)g->n;
    const uint64_t all = out.n == 64 ? ~0ull : ((1ull << out.n) - 1);
    for (int i = 0; i < out.n; ++i) {
        uint64_t r = g->adj[i];
        if (r & ~all)
            return fail(c, TW_EINVAL, "row %d has bits at positions >= n", i);
        if ((r >> i) & 1ull)
            return fail(c, TW_EINVAL, "self-loop at vertex %d", i);
        out.rows[i] = r;
    }
    for (int i = 0; i < out.n; ++i)
        for (int j = 0; j < out.n; ++j)
            if (((out.rows[i] >> j) & 1ull) != ((out.rows[j] >> i) & 1ull))
                return fail(c, TW_EINVAL, "adjacency not symmetric at (%d,%d)", i, j);
    return TW_OK;
}

// ---------------------------------------------------------------------------
// device memory: a small cache of freed buffers, best fit, then hipMalloc
// ---------------------------------------------------------------------------

void release(tw_ctx *c, Buf &b)
{
    if (b.p && b.from)
        b.from->put(b.p, b.bytes);
    else if (b.p)
        c->cache.push_back(b);
    b = Buf{};
}

// Device bytes the next buffers may take: the largest free block of the
// caller's range, else what the device reports free.
size_t free_device_bytes(tw_ctx *c)
{
    if (c->carve)
        return c->carve->largest();
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess)
        free_b = (size_t)16 << 30;
    return free_b;
}

void drop_cache(tw_ctx *c)
{
    for (Buf &b : c->cache)
        (void)hipFree(b.p);
    c->cache.clear();
}

tw_status acquire(tw_ctx *c, Buf &b, size_t bytes)
{
    if (b.p && b.bytes >= bytes)
        return TW_OK;
    release(c, b);
    bytes = std::max<size_t>(bytes, 256);
    if (c->carve) {
        void *p = c->carve->take(bytes);
        if (!p)
            return fail(c, TW_ENOMEM, "%zu bytes do not fit the caller's device range (largest free block %zu)",
                        bytes, c->carve->largest());
        b.p = p;
        b.bytes = bytes;
        b.from = c->carve;
        return TW_OK;
    }
    int best = -1;
    for (size_t t = 0; t < c->cache.size(); ++t)
        if (c->cache[t].bytes >= bytes &&
            (best < 0 || c->cache[t].bytes < c->cache[(size_t)best].bytes))
            best = (int)t;
    // reuse only if not grossly oversized
    if (best >= 0 && c->cache[(size_t)best].bytes <= 4 * bytes + (1u << 20)) {
        b = c->cache[(size_t)best];
        c->cache.erase(c->cache.begin() + best);
        return TW_OK;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(c->stream);
        drop_cache(c);
        e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(c, TW_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes,
                        hipGetErrorString(e));
        }
    }
    b.p = p;
    b.bytes = bytes;
    return TW_OK;
}

// ---------------------------------------------------------------------------
// host algorithms: minor-min-width (§3.3) and fill-in width (§2)
// ---------------------------------------------------------------------------

int mmw_bound(const Graph &g)
{
    uint64_t nb[64];
    uint64_t alive = g.n == 64 ? ~0ull : ((1ull << g.n) - 1);
    for (int v = 0; v < g.n; ++v)
        nb[v] = g.rows[v];
    int lb = 0;
    while (popc(alive) >= 2) {
        int d1 = 1 << 20, d2 = 1 << 20, v = -1;
        for (uint64_t a = alive; a; a &= a - 1) {
            const int x = __builtin_ctzll(a);
            const int d = popc(nb[x]);
            if (d < d1) {
                d2 = d1;
                d1 = d;
                v = x;
            } else if (d < d2) {
                d2 = d;
            }
        }
        lb = std::max(lb, d2);
        if (d1 == 0) {
            alive &= ~(1ull << v);
            continue;
        }
        int u = -1, du = 1 << 20;
        for (uint64_t a = nb[v]; a; a &= a - 1) {
            const int x = __builtin_ctzll(a);
            const int d = popc(nb[x]);
            if (d < du) {
                du = d;
                u = x;
            }
        }
        // contract v into u
        for (uint64_t a = nb[v]; a; a &= a - 1) {
            const int w = __builtin_ctzll(a);
            nb[w] &= ~(1ull << v);
            if (w != u) {
                nb[w] |= 1ull << u;
                nb[u] |= 1ull << w;
            }
        }
        nb[v] = 0;
        alive &= ~(1ull << v);
    }
    return lb;
}

int fill_in_width(const Graph &g, const int32_t *order)
{
    uint64_t adj[64];
    uint64_t seen = 0;
    for (int v = 0; v < g.n; ++v)
        adj[v] = g.rows[v];
    for (int t = 0; t < g.n; ++t) {
        const int v = order[t];
        if (v < 0 || v >= g.n || ((seen >> v) & 1ull))
            return -1;
        seen |= 1ull << v;
    }
    uint64_t alive = seen;
    int width = 0;
    for (int t = 0; t < g.n; ++t) {
        const int v = order[t];
        const uint64_t N = adj[v] & alive & ~(1ull << v);
        width = std::max(width, popc(N));
        for (uint64_t a = N; a; a &= a - 1) {
            const int u = __builtin_ctzll(a);
            adj[u] |= N & ~(1ull << u);
        }
        alive &= ~(1ull << v);
    }
    return width;
}

// ---------------------------------------------------------------------------
// the level loop
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// §3.1, first two optimisations: clique skip and disjoint-path edges
// ---------------------------------------------------------------------------

struct Reduction {
    uint64_t clique = 0;  // a maximum clique: never added to a state
    int clique_size = 0;
    // paths[u * 64 + v]: internally vertex-disjoint u-v paths for non-adjacent
    // u, v (capped at 255); pairs that cannot reach floor + 1 are left at 0
    std::vector<uint8_t> paths = std::vector<uint8_t>(64 * 64, 0);
};

// Bron-Kerbosch with pivoting lists every maximal clique; keep the largest,
// ties to the one whose ascending vertex list is lexicographically smallest
// (the lowest vertex where two equal-size sets differ lies in the smaller).
void clique_search(const Graph &g, uint64_t R, uint64_t P, uint64_t X, uint64_t &best, int &best_size)
{
    if (!P && !X) {
        const int sz = __builtin_popcountll(R);
        const uint64_t d = R ^ best;
        if (sz > best_size || (sz == best_size && d && (R & d & (~d + 1ull)))) {
            best = R;
            best_size = sz;
        }
        return;
    }
    if (__builtin_popcountll(R) + __builtin_popcountll(P) < best_size)
        return;
    int pivot = -1, pivot_deg = -1;
    for (uint64_t m = P | X; m; m &= m - 1) {
        const int u = __builtin_ctzll(m);
        const int d = __builtin_popcountll(P & g.rows[u]);
        if (d > pivot_deg) {
            pivot = u;
            pivot_deg = d;
        }
    }
    for (uint64_t m = P & ~g.rows[pivot]; m; m &= m - 1) {
        const int v = __builtin_ctzll(m);
        const uint64_t bit = 1ull << v;
        clique_search(g, R | bit, P & g.rows[v], X & g.rows[v], best, best_size);
        P &= ~bit;
        X |= bit;
    }
}

// Menger count for non-adjacent s, t by augmenting paths in the split graph:
// vertex w becomes in(w) -> out(w) of capacity 1 (unbounded for s and t), an
// edge {a, b} the arcs out(a) -> in(b) and out(b) -> in(a).  Stops at `cap`.
int vertex_disjoint_paths(const Graph &g, int s, int t, int cap)
{
    const int n = g.n;
    uint8_t fv[64] = {};           // flow through in(w) -> out(w)
    uint64_t fe[64] = {};          // fe[a] bit b: one unit on out(a) -> in(b)
    int flow = 0;
    int prev[128];
    int queue[128];
    while (flow < cap) {
        for (int x = 0; x < 2 * n; ++x)
            prev[x] = -2;
        const int src = 2 * s + 1, snk = 2 * t;
        prev[src] = -1;
        int qh = 0, qt = 0;
        queue[qt++] = src;
        while (qh < qt && prev[snk] == -2) {
            const int x = queue[qh++];
            const int w = x >> 1;
            auto visit = [&](int y) {
                if (prev[y] == -2) {
                    prev[y] = x;
                    queue[qt++] = y;
                }
            };
            if (x & 1) {  // out(w): forward to in(b) for every neighbour; back to in(w) if w carries flow
                for (uint64_t m = g.rows[w]; m; m &= m - 1)
                    visit(2 * __builtin_ctzll(m));
                if (fv[w])
                    visit(2 * w);
            } else {      // in(w): through w if it has room; back along out(a) -> in(w) arcs with flow
                if (w == s || w == t || !fv[w])
                    visit(2 * w + 1);
                for (uint64_t m = g.rows[w]; m; m &= m - 1) {
                    const int a = __builtin_ctzll(m);
                    if ((fe[a] >> w) & 1ull)
                        visit(2 * a + 1);
                }
            }
        }
        if (prev[snk] == -2)
            break;
        for (int y = snk; prev[y] >= 0; y = prev[y]) {
            const int x = prev[y];
            const int wx = x >> 1, wy = y >> 1;
            if (wx == wy) {
                if (wx != s && wx != t)
                    fv[wx] = (x & 1) ? 0 : 1;  // in -> out adds flow, out -> in removes it
            } else if (x & 1) {
                fe[wx] |= 1ull << wy;          // out(a) -> in(b)
            } else {
                fe[wy] &= ~(1ull << wx);       // in(b) -> out(a): cancel a unit on out(a) -> in(b)
            }
        }
        ++flow;
    }
    return flow;
}

// Clique and path counts of g.  With floor >= 0 only bounds k >= floor will
// be searched (and none below |C| - 1), so pairs that cannot have more paths
// than that are skipped; floor < 0 counts every pair.
Reduction reduction_of(const Graph &g, int floor)
{
    Reduction r;
    const uint64_t all = g.n == 64 ? ~0ull : ((1ull << g.n) - 1);
    clique_search(g, 0, all, 0, r.clique, r.clique_size);
    if (floor >= 0)
        floor = std::max(floor, r.clique_size - 1);
    int deg[64];
    for (int v = 0; v < g.n; ++v)
        deg[v] = __builtin_popcountll(g.rows[v]);
    for (int u = 0; u < g.n; ++u)
        for (int v = u + 1; v < g.n; ++v) {
            if ((g.rows[u] >> v) & 1ull)
                continue;
            const int bound = std::min(deg[u], deg[v]);
            if (bound <= floor)
                continue;  // at most `bound` paths: never reaches floor + 1
            const int p = std::min(255, vertex_disjoint_paths(g, u, v, bound));
            r.paths[(size_t)u * 64 + v] = r.paths[(size_t)v * 64 + u] = (uint8_t)p;
        }
    return r;
}

// G plus uv for every pair with >= k + 1 disjoint paths.
Graph augmented(const Graph &g, const Reduction &r, int k)
{
    Graph a = g;
    for (int u = 0; u < g.n; ++u)
        for (int v = 0; v < g.n; ++v)
            if ((int)r.paths[(size_t)u * 64 + v] > k)
                a.rows[u] |= 1ull << v;
    return a;
}

struct RunStats {
    uint64_t states_expanded = 0, expansions = 0, successors = 0, unique = 0, peak = 0;
    uint32_t decisions = 0, levels = 0, retries = 0, launches = 0;
    double kernel_seconds = 0;
    uint64_t run_peak = 0;  // largest level of the last decide run
};

// Per-graph outcome of a search (start bound, certifying run's peak, work).
void add_run_stats(RunStats &into, const RunStats &from)
{
    into.states_expanded += from.states_expanded;
    into.expansions += from.expansions;
    into.successors += from.successors;
    into.unique += from.unique;
    into.peak = std::max(into.peak, from.peak);
    into.decisions += from.decisions;
    into.levels += from.levels;
    into.retries += from.retries;
    into.launches += from.launches;
    into.kernel_seconds += from.kernel_seconds;
}

struct GraphOutcome {
    uint64_t peak_yes = 0, expansions = 0, states = 0;
    uint64_t peak_any = 0;  // largest level met (for a failed search: what the failing level reached)
    int32_t start_k = 0;
    uint32_t decisions = 0;
    int32_t path = 1;
};

void add_stats(tw_stats *st, const RunStats &r, double secs)
{
    if (!st)
        return;
    st->states_expanded = r.states_expanded;
    st->expansions = r.expansions;
    st->successors = r.successors;
    st->unique = r.unique;
    st->peak_frontier = r.peak;
    st->decisions = r.decisions;
    st->levels = r.levels;
    st->retries = r.retries;
    st->launches = r.launches;
    st->seconds = secs;
    st->kernel_seconds = r.kernel_seconds;
}

struct Sink {
    void (*fn)(const tw_level_record *, void *) = nullptr;
    void *user = nullptr;
};

tw_status emit_level(tw_ctx *c, const Sink &sink, int k, int i, const Level &lv, int key_bytes,
                     uint64_t expansions, uint64_t successors)
{
    std::vector<uint64_t> keys(lv.count);
    std::vector<uint8_t> lastv(lv.count, 0);
    if (lv.count) {
        if (key_bytes == 4) {
            std::vector<uint32_t> k32(lv.count);
            HIP_TRY(c, hipMemcpyAsync(k32.data(), lv.keys.p, lv.count * 4, hipMemcpyDeviceToHost,
                                      c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            for (uint64_t t = 0; t < lv.count; ++t)
                keys[t] = k32[t];
        } else {
            HIP_TRY(c, hipMemcpyAsync(keys.data(), lv.keys.p, lv.count * 8, hipMemcpyDeviceToHost,
                                      c->stream));
        }
        if (i > 0)
            HIP_TRY(c, hipMemcpyAsync(lastv.data(), lv.lastv.p, lv.count, hipMemcpyDeviceToHost,
                                      c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    tw_level_record rec{};
    rec.k = k;
    rec.level = i;
    rec.count = lv.count;
    rec.expansions = expansions;
    rec.successors = successors;
    rec.states = keys.data();
    rec.last_v = lastv.data();
    sink.fn(&rec, sink.user);
    return TW_OK;
}

// Per-state minor-min-width pruning (§3.3): level `in` is replaced by its
// states S with MMW(H_S) <= k (creating vertices kept alongside).  A dropped
// state has no completion within width k, so no order is lost.
tw_status prune_level(tw_ctx *c, Level &in, int n, int k, int kb, RunStats &rs)
{
    Buf keys, lastv;
    tw_status s = acquire(c, keys, in.count * (uint64_t)kb);
    if (s == TW_OK && in.lastv.p)
        s = acquire(c, lastv, in.count);
    if (s != TW_OK) {
        release(c, keys);
        return s;
    }
    HIP_TRY(c, twk::launch_zero_counters((LevelCounters *)c->d_ctr.p, c->stream));
    twk::PruneArgs a{};
    a.in = in.keys.p;
    a.in_lastv = (const uint8_t *)in.lastv.p;
    a.in_count = in.count;
    a.out = keys.p;
    a.out_lastv = (uint8_t *)lastv.p;
    a.adj = (const uint64_t *)c->d_adj.p;
    a.kept = &((LevelCounters *)c->d_ctr.p)->out_count;
    a.n = n;
    a.k = k;
    a.key_bytes = kb;
    const uint64_t waves = (in.count + 63) / 64;
    uint64_t blocks = (waves + twk::kWavesPerBlock - 1) / twk::kWavesPerBlock;
    blocks = std::min<uint64_t>(std::max<uint64_t>(blocks, 1), (uint64_t)c->cu_count * 8);
    HIP_TRY(c, twk::launch_mmw_prune(a, (unsigned)blocks, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->h_ctr, c->d_ctr.p, sizeof(LevelCounters), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const uint64_t kept = c->h_ctr->out_count;
    if (kept > in.count)
        return fail(c, TW_EDEVICE, "pruning kept %llu of %llu states", (unsigned long long)kept,
                    (unsigned long long)in.count);
    release(c, in.keys);
    release(c, in.lastv);
    in.keys = keys;
    in.lastv = lastv;
    in.count = kept;
    return TW_OK;
}

// Level retention of run_decide.
enum Keep {
    kKeepPair = 0,     // only the current pair; levels.back() is the last level reached
    kKeepAll = 1,      // levels[0..L] stay on the device, each trimmed to its exact size
    kKeepIfSmall = 2,  // as kKeepAll while the kept levels fit keep_budget bytes, then as kKeepPair
};

// Runs decide(k).  Levels are retained as `keep` says (levels.size() == L + 1
// after a YES means every level was kept, for order reconstruction).  With
// allowed != all, only vertices of `allowed` are ever added: the levels are
// then the full levels restricted to subsets of `allowed` (feasibility of a
// set does not depend on the vertices outside it being allowed).
tw_status run_decide(tw_ctx *c, const Graph &g, int k, int keep, const Sink *sink,
                     std::vector<Level> &levels, int *yes, RunStats &rs, uint64_t allowed = ~0ull)
{
    const int n = g.n;
    const int L = std::max(0, n - k - 1);
    const int kb = n <= 32 ? 4 : 8;
    bool keep_levels = keep != kKeepPair;
    uint64_t kept_bytes = 0;
    rs.decisions++;

    for (Level &lv : levels) {
        release(c, lv.keys);
        release(c, lv.lastv);
    }
    levels.assign(1, Level{});
    // level 0 = {empty set}
    {
        Level &l0 = levels[0];
        tw_status s = acquire(c, l0.keys, 8);
        if (s != TW_OK)
            return s;
        HIP_TRY(c, hipMemsetAsync(l0.keys.p, 0, 8, c->stream));
        l0.count = 1;
    }
    if (sink && sink->fn) {
        tw_status s = emit_level(c, *sink, k, 0, levels[0], kb, 0, 0);
        if (s != TW_OK)
            return s;
    }
    HIP_TRY(c, hipMemcpyAsync(c->d_adj.p, g.rows, sizeof(uint64_t) * 64, hipMemcpyHostToDevice,
                              c->stream));

    const float alpha = (c->opt.load_factor > 0.f && c->opt.load_factor <= 0.9f)
                            ? c->opt.load_factor
                            : 0.25f;
    const size_t dev_free = free_device_bytes(c);
    double growth = (double)n;      // |level 1| <= n
    double pair_ratio = (double)n;  // feasible pairs per state of the previous level
    Buf scratch_keys, scratch_lastv;
    tw_status status = TW_OK;
    uint64_t cur = 1;
    uint64_t run_peak = 1;
    int i = 0;

    for (; i < L; ++i) {
        Level &in = levels.back();
        if (c->opt.mmw_prune == TW_MMW_PRUNE && in.count) {
            status = prune_level(c, in, n, k, kb, rs);
            if (status != TW_OK)
                goto done;
            if (in.count == 0) {
                cur = 0;
                break;
            }
        }
        const uint64_t in_count = in.count;
        const bool bloom = c->opt.dedup == TW_DEDUP_BLOOM || c->opt.dedup == TW_DEDUP_BLOOM_CERTIFIED;
        // every new state comes from a distinct (S, v) pair; exact dedup also
        // never exceeds C(n, i+1), while concurrent Bloom inserts of one state
        // may both report it new
        const uint64_t pairs = in_count > UINT64_MAX / 64 ? UINT64_MAX : in_count * (uint64_t)(n - i);
        const uint64_t bound = bloom ? pairs : std::min<uint64_t>(binom_sat(n, i + 1), pairs);
        // first guess of |level i+1|: the last growth ratio with 30% slack
        uint64_t guess;
        if (c->opt.capacity_override)
            guess = c->opt.capacity_override;
        else
            guess = (uint64_t)std::min<double>((double)in_count * std::max(1.0, growth) * 1.3 + 4096.0,
                                               1.8e19);
        guess = std::max<uint64_t>(std::min(guess, bound), 1);
        // a sparse table (fewer probes) while it takes at most a third of free memory
        float a_eff = std::max(alpha, std::min(0.5f, (float)((double)guess * kb * 3.0 / (double)dev_free)));
        uint64_t part_guess = 0;  // successor-buffer entries (partitioned insert)

        uint64_t out_count = 0, succ = 0;
        bool injected = false;
        for (;;) {
            if (c->opt.max_states && guess > c->opt.max_states)
                guess = std::max<uint64_t>(c->opt.max_states, 1);
            // table of any size (multiply-shift slot mapping), a multiple of 64 slots
            uint64_t slots = ((uint64_t)((double)guess / a_eff) + 64 + 63) / 64 * 64;
            // large tables: partition the insert by hash range into slices of <= 64 MB
            int P = 1;
            uint64_t slice = slots, part_cap = 0;
            if (!bloom && n <= 58 && c->opt.partition != 1) {
                const uint64_t tbytes = slots * (uint64_t)kb;
                const uint64_t limit = 64ull << 20;
                if (c->opt.partition == 2)
                    P = (int)std::min<uint64_t>(twk::kMaxParts, std::max<uint64_t>(2, (tbytes + limit - 1) / limit));
            }
            if (P > 1) {
                slice = ((slots + (uint64_t)P - 1) / (uint64_t)P + 63) / 64 * 64;
                slots = slice * (uint64_t)P;
                if (!part_guess)
                    part_guess = (uint64_t)std::min<double>((double)in_count * pair_ratio * 1.3 + 4096.0 * P,
                                                            (double)pairs + 64.0 * P);
                // entries per sub-region: an equal share of the guess plus slack
                const uint64_t regions = (uint64_t)P * twk::kSubRegions;
                part_cap = (uint64_t)(1.1 * (double)part_guess / (double)regions) + 64;
                tw_status ps = acquire(c, c->parts, part_cap * regions * 8);
                if (ps == TW_OK)
                    ps = acquire(c, c->part_meta, (regions * 3 + 1) * 8);
                if (ps != TW_OK) {
                    // no room for the successor buffer: single-phase insert for this level
                    release(c, c->parts);
                    c->err.clear();
                    P = 1;
                    slice = slots;
                }
            }
            uint64_t out_cap = std::min<uint64_t>(bound, std::max<uint64_t>(guess, (uint64_t)(0.6 * (double)slots)));
            if (c->opt.max_states)
                out_cap = std::min<uint64_t>(out_cap, c->opt.max_states);
            uint64_t bloom_bits = 0;
            if (bloom) {
                bloom_bits = pow2_at_least((uint64_t)twk::kBloomBitsPerState * out_cap + 1);
                status = acquire(c, c->bloom, bloom_bits / 8);
            } else {
                status = acquire(c, c->table, slots * kb);
            }
            if (status == TW_OK)
                status = acquire(c, scratch_keys, out_cap * kb);
            if (status == TW_OK)
                status = acquire(c, scratch_lastv, out_cap);
            if (status == TW_ENOMEM && !bloom && a_eff < 0.8f) {
                // short of memory: a fuller table before giving up
                release(c, scratch_keys);
                release(c, scratch_lastv);
                release(c, c->table);
                drop_cache(c);
                a_eff = 0.8f;
                status = TW_OK;
                c->err.clear();
                continue;
            }
            if (status != TW_OK)
                goto done;

            if (bloom)
                HIP_TRY(c, twk::launch_fill_zero(c->bloom.p, bloom_bits / 8, c->stream));
            else
                HIP_TRY(c, twk::launch_fill_empty(c->table.p, slots * kb, c->stream));
            HIP_TRY(c, twk::launch_zero_counters((LevelCounters *)c->d_ctr.p, c->stream));
            twk::LevelArgs a{};
            a.in = in.keys.p;
            a.in_count = in_count;
            a.out = scratch_keys.p;
            a.out_lastv = (uint8_t *)scratch_lastv.p;
            a.out_cap = out_cap;
            a.table = bloom ? nullptr : c->table.p;
            a.table_slots = slots;
            a.allowed = allowed;
            a.bloom = bloom ? (uint32_t *)c->bloom.p : nullptr;
            a.bloom_mask = bloom ? bloom_bits - 1 : 0;
            a.adj = (const uint64_t *)c->d_adj.p;
            a.n = n;
            a.k = k;
            a.ctr = (LevelCounters *)c->d_ctr.p;
            a.max_probe = (uint32_t)std::min<uint64_t>(slots, 1u << 16);
            a.read_first = c->opt.probe == 1 ? 0 : 1;
            a.key_bytes = kb;
            const uint64_t waves = (in_count + 63) / 64;
            uint64_t blocks = (waves + twk::kWavesPerBlock - 1) / twk::kWavesPerBlock;
            blocks = std::min<uint64_t>(std::max<uint64_t>(blocks, 1), (uint64_t)c->cu_count * 8);
            if (P > 1) {
                // phase 1: expand and scatter every feasible pair into its hash-range partition
                const int R = P * twk::kSubRegions;
                twk::ScatterArgs sc{};
                sc.parts = (uint64_t *)c->parts.p;
                sc.sub_cap = part_cap;
                sc.sub_count = (unsigned long long *)c->part_meta.p;
                sc.P = P;
                HIP_TRY(c, twk::launch_fill_zero(c->part_meta.p, (size_t)R * 8, c->stream));
                if (c->opt.timing)
                    HIP_TRY(c, hipEventRecord(c->ev0, c->stream));
                HIP_TRY(c, twk::launch_scatter(a, sc, (unsigned)blocks, c->stream));
                if (c->opt.timing)
                    HIP_TRY(c, hipEventRecord(c->ev1, c->stream));
                std::vector<uint64_t> cnt((size_t)R);
                HIP_TRY(c, hipMemcpyAsync(cnt.data(), c->part_meta.p, (size_t)R * 8, hipMemcpyDeviceToHost,
                                          c->stream));
                HIP_TRY(c, hipMemcpyAsync(c->h_ctr, c->d_ctr.p, sizeof(LevelCounters), hipMemcpyDeviceToHost,
                                          c->stream));
                HIP_TRY(c, hipStreamSynchronize(c->stream));
                if (c->opt.timing) {
                    float ms = 0.f;
                    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
                    rs.kernel_seconds += ms * 1e-3;
                }
                uint64_t most = 0;
                for (uint64_t x : cnt)
                    most = std::max(most, x);
                if (c->h_ctr->overflow || most > part_cap) {
                    // successor buffer too small: grow it and replay the level
                    rs.retries++;
                    part_guess = std::max<uint64_t>(part_guess * 2, (uint64_t)(1.25 * (double)most * R));
                    continue;
                }
                // phase 2: insert partition by partition (chunk prefix over 64-entry chunks)
                std::vector<uint64_t> meta((size_t)R * 2 + 1);
                uint64_t chunks = 0;
                for (int r = 0; r < R; ++r) {
                    meta[(size_t)r] = chunks;
                    chunks += (cnt[(size_t)r] + 63) / 64;
                }
                meta[(size_t)R] = chunks;
                for (int r = 0; r < R; ++r)
                    meta[(size_t)R + 1 + (size_t)r] = cnt[(size_t)r];
                uint64_t *dmeta = (uint64_t *)c->part_meta.p + R;
                HIP_TRY(c, hipMemcpyAsync(dmeta, meta.data(), meta.size() * 8, hipMemcpyHostToDevice, c->stream));
                twk::GatherArgs ga{};
                ga.parts = (const uint64_t *)c->parts.p;
                ga.sub_cap = part_cap;
                ga.chunk_prefix = dmeta;
                ga.count = dmeta + R + 1;
                ga.P = P;
                ga.slice = slice;
                const uint64_t gblocks = std::min<uint64_t>(
                    std::max<uint64_t>((chunks + twk::kWavesPerBlock - 1) / twk::kWavesPerBlock, 1),
                    (uint64_t)c->cu_count * 8);
                if (c->opt.timing)
                    HIP_TRY(c, hipEventRecord(c->ev0, c->stream));
                HIP_TRY(c, twk::launch_gather(a, ga, (unsigned)gblocks, c->stream));
                if (c->opt.timing)
                    HIP_TRY(c, hipEventRecord(c->ev1, c->stream));
            } else {
                if (c->opt.timing)
                    HIP_TRY(c, hipEventRecord(c->ev0, c->stream));
                HIP_TRY(c, twk::launch_expand(a, (unsigned)blocks, c->stream));
                if (c->opt.timing)
                    HIP_TRY(c, hipEventRecord(c->ev1, c->stream));
            }
            HIP_TRY(c, hipMemcpyAsync(c->h_ctr, c->d_ctr.p, sizeof(LevelCounters),
                                      hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            rs.launches++;
            if (c->opt.timing) {
                float ms = 0.f;
                HIP_TRY(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
                rs.kernel_seconds += ms * 1e-3;
            }
            LevelCounters h = *c->h_ctr;
            if (c->opt.fault_inject_level == i + 1 && !injected) {
                // test hook: this level's first build counts as an overflow
                injected = true;
                h.overflow = 1;
            }
            if (!h.overflow) {
                out_count = h.out_count;
                succ = h.successors;
                break;
            }
            // overflow: regrow and replay the level (h.out_count is a lower bound)
            rs.retries++;
            if (c->opt.max_states && out_cap >= c->opt.max_states) {
                run_peak = std::max<uint64_t>(run_peak, h.out_count);
                status = fail(c, TW_ECAPACITY, "level %d needs more than max_states=%llu states",
                              i + 1, (unsigned long long)c->opt.max_states);
                goto done;
            }
            if (!bloom && !injected && out_cap >= bound && (double)slots * 0.8 >= (double)bound) {
                status = fail(c, TW_EDEVICE, "overflow at level %d with capacity at its bound", i + 1);
                goto done;
            }
            guess = std::min<uint64_t>(bound, std::max<uint64_t>(guess * 2, (uint64_t)(1.3 * (double)h.out_count)));
        }

        rs.states_expanded += in_count;
        rs.expansions += in_count * (uint64_t)(n - i);
        rs.successors += succ;
        rs.unique += out_count;
        rs.levels++;
        rs.peak = std::max(rs.peak, std::max(out_count, in_count));
        run_peak = std::max(run_peak, out_count);
        growth = in_count ? (double)out_count / (double)in_count : 1.0;
        pair_ratio = in_count ? (double)succ / (double)in_count : (double)n;

        if (keep_levels && keep == kKeepIfSmall) {
            kept_bytes += out_count * (uint64_t)(kb + 1);
            if (kept_bytes > c->keep_budget) {
                // too large to keep every level: continue with the current pair only
                keep_levels = false;
                for (size_t t = 0; t + 1 < levels.size(); ++t) {
                    release(c, levels[t].keys);
                    release(c, levels[t].lastv);
                }
                levels.erase(levels.begin(), levels.end() - 1);
            }
        }
        // the new level: an exact-size copy when levels are kept, else the scratch pair itself
        Level nl;
        nl.count = out_count;
        if (keep_levels || sink) {
            status = acquire(c, nl.keys, std::max<uint64_t>(out_count, 1) * kb);
            if (status == TW_OK)
                status = acquire(c, nl.lastv, std::max<uint64_t>(out_count, 1));
            if (status != TW_OK)
                goto done;
            if (out_count) {
                HIP_TRY(c, hipMemcpyAsync(nl.keys.p, scratch_keys.p, out_count * kb,
                                          hipMemcpyDeviceToDevice, c->stream));
                HIP_TRY(c, hipMemcpyAsync(nl.lastv.p, scratch_lastv.p, out_count,
                                          hipMemcpyDeviceToDevice, c->stream));
            }
        } else {
            nl.keys = scratch_keys;
            nl.lastv = scratch_lastv;
            scratch_keys = Buf{};
            scratch_lastv = Buf{};
        }
        if (sink && sink->fn) {
            status = emit_level(c, *sink, k, i + 1, nl, kb, in_count * (uint64_t)(n - i), succ);
            if (status != TW_OK) {
                release(c, nl.keys);
                release(c, nl.lastv);
                goto done;
            }
        }
        if (!keep_levels) {
            Level &old = levels.back();
            // the old input becomes the next scratch output
            if (!sink) {
                scratch_keys = old.keys;
                scratch_lastv = old.lastv;
                old.keys = Buf{};
                old.lastv = Buf{};
            } else {
                release(c, old.keys);
                release(c, old.lastv);
            }
            levels.back() = nl;
        } else {
            levels.push_back(nl);
        }
        cur = out_count;
        if (out_count == 0)
            break;
    }
done:
    release(c, scratch_keys);
    release(c, scratch_lastv);
    rs.run_peak = run_peak;
    if (status != TW_OK)
        return status;
    *yes = (i >= L && cur > 0) ? 1 : 0;
    if (L == 0)
        *yes = 1;
    return TW_OK;
}

tw_status ensure_ctx_buffers(tw_ctx *c)
{
    tw_status s = acquire(c, c->d_adj, 64 * sizeof(uint64_t));
    if (s == TW_OK)
        s = acquire(c, c->d_ctr, sizeof(LevelCounters));
    if (s == TW_OK)
        s = acquire(c, c->d_find, sizeof(unsigned long long));
    return s;
}

// Follow last_v back from a state of the last level to the empty set.
tw_status reconstruct(tw_ctx *c, const Graph &g, int k, const std::vector<Level> &levels,
                      int32_t *order)
{
    const int n = g.n;
    const int L = (int)levels.size() - 1;
    const int kb = n <= 32 ? 4 : 8;
    std::vector<int> rev;
    uint64_t S = 0;
    uint64_t idx = 0;
    if (L > 0) {
        uint64_t key = 0;
        HIP_TRY(c, hipMemcpyAsync(&key, levels[L].keys.p, kb, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        S = key;
        const uint64_t SL = S;
        for (int i = L; i >= 1; --i) {
            uint8_t v = 0;
            HIP_TRY(c, hipMemcpyAsync(&v, (const uint8_t *)levels[i].lastv.p + idx, 1,
                                      hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            if (v >= n || !((S >> v) & 1ull))
                return fail(c, TW_EDEVICE, "reconstruction: bad last vertex %d at level %d", v, i);
            rev.push_back(v);
            S &= ~(1ull << v);
            if (i == 1)
                break;
            *c->h_find = ~0ull;
            HIP_TRY(c, hipMemcpyAsync(c->d_find.p, c->h_find, 8, hipMemcpyHostToDevice, c->stream));
            HIP_TRY(c, twk::launch_find(levels[i - 1].keys.p, levels[i - 1].count, S, kb,
                                        (unsigned long long *)c->d_find.p, c->stream));
            HIP_TRY(c, hipMemcpyAsync(c->h_find, c->d_find.p, 8, hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            idx = *c->h_find;
            if (idx == ~0ull)
                return fail(c, TW_EDEVICE, "reconstruction: predecessor missing at level %d", i - 1);
        }
        S = SL;
    }
    int t = 0;
    for (int r = (int)rev.size() - 1; r >= 0; --r)
        order[t++] = rev[(size_t)r];
    for (int v = 0; v < n; ++v)
        if (!((S >> v) & 1ull))
            order[t++] = v;
    if (t != n)
        return fail(c, TW_EDEVICE, "reconstruction produced %d of %d vertices", t, n);
    const int w = fill_in_width(g, order);
    if (w < 0 || w > k)
        return fail(c, TW_EDEVICE, "reconstructed order has width %d > %d", w, k);
    return TW_OK;
}

void free_levels(tw_ctx *c, std::vector<Level> &levels)
{
    for (Level &lv : levels) {
        release(c, lv.keys);
        release(c, lv.lastv);
    }
    levels.clear();
}

// decide(k) with the reductions of §3.1 when red is set: NO without a search
// below the clique bound, else the search on G_k+ never adding a clique vertex.
tw_status run_decide_reduced(tw_ctx *c, const Graph &g, const Reduction *red, int k, int keep,
                             const Sink *sink, std::vector<Level> &levels, int *yes, RunStats &rs,
                             uint64_t allowed = ~0ull)
{
    if (!red)
        return run_decide(c, g, k, keep, sink, levels, yes, rs, allowed);
    if (k < red->clique_size - 1) {
        free_levels(c, levels);
        rs.decisions++;
        *yes = 0;
        return TW_OK;
    }
    return run_decide(c, augmented(g, *red, k), k, keep, sink, levels, yes, rs, allowed & ~red->clique);
}

// decide(k) as run_decide_reduced; under TW_DEDUP_BLOOM_CERTIFIED a NO of the
// Bloom search is decided again by the exact search (a false positive of the
// filter only drops states, so only a NO can be wrong).
tw_status decide_checked(tw_ctx *c, const Graph &g, const Reduction *red, int k, int keep,
                         std::vector<Level> &levels, int *yes, RunStats &rs)
{
    tw_status s = run_decide_reduced(c, g, red, k, keep, nullptr, levels, yes, rs);
    if (s == TW_OK && !*yes && c->opt.dedup == TW_DEDUP_BLOOM_CERTIFIED) {
        c->opt.dedup = TW_DEDUP_EXACT;
        s = run_decide_reduced(c, g, red, k, keep, nullptr, levels, yes, rs);
        c->opt.dedup = TW_DEDUP_BLOOM_CERTIFIED;
    }
    return s;
}

// ---------------------------------------------------------------------------
// Captured level loop.  For graphs whose every level fits its binomial bound
// in a modest budget, the level loop of a bound (Listing 1) is a fixed
// sequence of launches — per level one clearing launch and one expansion —
// whose sizes and bound come from device memory, captured once per graph
// shape in a HIP graph and replayed for every bound (and every later graph of
// that shape): one launch and one readback per bound instead of a launch
// sequence and a host wait per level.  Level i has room for C(m, i) states (m
// vertices may be added), which no exact level exceeds, so a replay cannot
// overflow its capacity; a table overflow (probe backstop) sends the bound to
// the host-driven loop.
// ---------------------------------------------------------------------------
struct Captured {
    int n = 0, levels = 0;
    std::vector<uint64_t> off;       // level offsets in states (levels + 1 entries)
    Buf keys, lastv, table, ctr, ctl, off_dev, out;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

constexpr uint64_t kCaptureBudget = 256ull << 20;
constexpr float kCaptureLoad = 0.25f;
// internal status (beside the public 0..4): run this bound on the host-driven loop
constexpr tw_status kNotCaptured = static_cast<tw_status>(7);

struct CapHost {
    twk::CaptureCtl ctl;
    LevelCounters ctr[64];
    int32_t order[64];
    uint64_t last_state;
    int32_t err;
    int32_t pad2;
};

void destroy_captured(tw_ctx *c, Captured *cp)
{
    if (cp->exec)
        (void)hipGraphExecDestroy(cp->exec);
    if (cp->graph)
        (void)hipGraphDestroy(cp->graph);
    release(c, cp->keys);
    release(c, cp->lastv);
    release(c, cp->table);
    release(c, cp->ctr);
    release(c, cp->ctl);
    release(c, cp->off_dev);
    release(c, cp->out);
    delete cp;
}

// The instantiated loop for graphs on n vertices, built on first use (the
// context keeps the last kCaptureKeep); null when the path does not apply.
// Level i has room for C(n, i) states: every level of any bound, with any set
// of vertices allowed, fits.
constexpr size_t kCaptureKeep = 4;

Captured *capture_for(tw_ctx *c, const Graph &g)
{
    if (c->opt.capture == TW_CAPTURE_OFF || c->no_capture || !c->h_cap || c->opt.dedup != TW_DEDUP_EXACT ||
        c->opt.mmw_prune != TW_MMW_NONE || c->opt.partition == 2 || c->opt.fault_inject_level ||
        c->opt.capacity_override || g.n > 32 || g.n < 2)
        return nullptr;
    const int n = g.n;
    for (Captured *cp : c->captured)
        if (cp->n == n)
            return cp->exec ? cp : nullptr;
    const int levels = n - 1;  // bounds k >= 0 run at most n - 1 levels
    std::vector<uint64_t> off((size_t)levels + 2, 0);
    uint64_t widest = 1;
    for (int i = 0; i <= levels; ++i) {
        const uint64_t cap = std::max<uint64_t>(binom_sat(n, i), 1);
        off[(size_t)i + 1] = off[(size_t)i] + cap;
        widest = std::max(widest, cap);
    }
    const uint64_t states = off[(size_t)levels + 1];
    const uint64_t slots_max = ((uint64_t)((double)widest / kCaptureLoad) + 64 + 63) / 64 * 64;
    const uint64_t bytes = states * 5 + slots_max * 4;
    if (bytes > kCaptureBudget || bytes > free_device_bytes(c) / 4)
        return nullptr;
    Captured *cp = new (std::nothrow) Captured();
    if (!cp)
        return nullptr;
    cp->n = n;
    cp->levels = levels;
    cp->off = off;
    if (c->captured.size() >= kCaptureKeep) {
        (void)hipStreamSynchronize(c->stream);
        destroy_captured(c, c->captured.front());
        c->captured.erase(c->captured.begin());
    }
    c->captured.push_back(cp);  // cached even when unusable (exec stays null)
    tw_status s = acquire(c, cp->keys, states * 4);
    if (s == TW_OK)
        s = acquire(c, cp->lastv, states);
    if (s == TW_OK)
        s = acquire(c, cp->table, slots_max * 4);
    if (s == TW_OK)
        s = acquire(c, cp->ctr, sizeof(LevelCounters) * 64);
    if (s == TW_OK)
        s = acquire(c, cp->ctl, sizeof(twk::CaptureCtl));
    if (s == TW_OK)
        s = acquire(c, cp->off_dev, off.size() * 8);
    if (s == TW_OK)
        s = acquire(c, cp->out, 64 * 4 + 32);  // order, last state, error flag (cleared as 24 bytes)
    if (s != TW_OK) {
        c->err.clear();
        return nullptr;
    }
    // level 0 is the empty set, at keys[off[0]]; the replays never write there
    if (hipMemcpyAsync(cp->off_dev.p, off.data(), off.size() * 8, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        twk::launch_fill_zero(cp->keys.p, 16, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return nullptr;
    auto *ctl = (const twk::CaptureCtl *)cp->ctl.p;
    auto *ctr = (LevelCounters *)cp->ctr.p;
    if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed) != hipSuccess)
        return nullptr;
    hipError_t e = hipSuccess;
    for (int i = 0; i < levels && e == hipSuccess; ++i) {
        twk::GateArgs ga{ctl, ctr, i};
        const uint64_t next_cap = off[(size_t)i + 2] - off[(size_t)i + 1];
        const uint64_t slots = ((uint64_t)((double)next_cap / kCaptureLoad) + 64 + 63) / 64 * 64;
        e = twk::launch_prep_gated(ga, cp->table.p, slots * 4, c->stream);
        if (e != hipSuccess)
            break;
        twk::LevelArgs a{};
        a.in = (const uint32_t *)cp->keys.p + off[(size_t)i];
        a.out = (uint32_t *)cp->keys.p + off[(size_t)i + 1];
        a.out_lastv = (uint8_t *)cp->lastv.p + off[(size_t)i + 1];
        a.out_cap = next_cap;
        a.table = cp->table.p;
        a.table_slots = slots;
        a.allowed = ~0ull;  // the replay takes it from the control block
        a.adj = (const uint64_t *)c->d_adj.p;
        a.n = n;
        a.ctr = ctr + i;
        a.max_probe = (uint32_t)std::min<uint64_t>(slots, 1u << 16);
        a.read_first = c->opt.probe == 1 ? 0 : 1;
        a.key_bytes = 4;
        const uint64_t this_cap = off[(size_t)i + 1] - off[(size_t)i];
        const uint64_t waves = (this_cap + 63) / 64;
        uint64_t blocks = (waves + twk::kWavesPerBlock - 1) / twk::kWavesPerBlock;
        blocks = std::min<uint64_t>(std::max<uint64_t>(blocks, 1), (uint64_t)c->cu_count * 8);
        e = twk::launch_expand_gated(a, ga, (unsigned)blocks, c->stream);
    }
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(c->stream, &graph);
    if (e != hipSuccess || e2 != hipSuccess || !graph) {
        if (graph)
            (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        return nullptr;
    }
    cp->graph = graph;
    if (hipGraphInstantiate(&cp->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        cp->exec = nullptr;
        (void)hipGetLastError();
        return nullptr;
    }
    return cp;
}

// decide(k) by one replay of the captured loop; counters as run_decide's.
tw_status captured_decide(tw_ctx *c, Captured &cp, const Graph &g, int k, uint64_t allowed, int *yes,
                          RunStats &rs)
{
    const int n = g.n;
    const int L = std::max(0, n - k - 1);
    rs.decisions++;
    if (L == 0) {
        *yes = 1;
        rs.run_peak = 1;
        return TW_OK;
    }
    CapHost *h = (CapHost *)c->h_cap;
    h->ctl.k = k;
    h->ctl.L = L;
    h->ctl.allowed = allowed;
    HIP_TRY(c, hipMemcpyAsync(c->d_adj.p, g.rows, sizeof(uint64_t) * 64, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(cp.ctl.p, &h->ctl, sizeof h->ctl, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipGraphLaunch(cp.exec, c->stream));
    HIP_TRY(c, hipMemcpyAsync(h->ctr, cp.ctr.p, sizeof(LevelCounters) * (size_t)L, hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    rs.launches++;
    // a table overflow, or a level above max_states (whose slot held it all):
    // the bound runs on the host-driven loop, which reports the cap
    for (int j = 0; j < L; ++j) {
        const LevelCounters &lc = h->ctr[j];
        if (lc.overflow || (c->opt.max_states && lc.out_count > c->opt.max_states))
            return kNotCaptured;
        if (lc.out_count == 0)
            break;
    }
    uint64_t cur = 1, run_peak = 1;
    int i = 0;
    for (; i < L; ++i) {
        const LevelCounters &lc = h->ctr[i];
        const uint64_t in_count = cur, out_count = lc.out_count;
        rs.states_expanded += in_count;
        rs.expansions += in_count * (uint64_t)(n - i);
        rs.successors += lc.successors;
        rs.unique += out_count;
        rs.levels++;
        rs.peak = std::max(rs.peak, std::max(out_count, in_count));
        run_peak = std::max(run_peak, out_count);
        cur = out_count;
        if (out_count == 0)
            break;
    }
    rs.run_peak = run_peak;
    *yes = (i >= L && cur > 0) ? 1 : 0;
    return TW_OK;
}

// The order of the YES replay just run at bound k on (possibly augmented) g.
tw_status captured_order(tw_ctx *c, Captured &cp, const Graph &g, int k, int32_t *order)
{
    const int n = g.n;
    const int L = std::max(0, n - k - 1);
    CapHost *h = (CapHost *)c->h_cap;
    uint64_t SL = 0;
    if (L > 0) {
        twk::BacktrackArgs b{};
        b.keys = cp.keys.p;
        b.lastv = (const uint8_t *)cp.lastv.p;
        b.off = (const uint64_t *)cp.off_dev.p;
        b.ctl = (const twk::CaptureCtl *)cp.ctl.p;
        b.ctr = (const LevelCounters *)cp.ctr.p;
        b.order = (int32_t *)cp.out.p;
        b.last_state = (uint64_t *)((char *)cp.out.p + 256);
        b.err = (int32_t *)((char *)cp.out.p + 264);
        HIP_TRY(c, twk::launch_zero_counters((LevelCounters *)((char *)cp.out.p + 256), c->stream));
        HIP_TRY(c, twk::launch_backtrack(b, 4, c->stream));
        HIP_TRY(c, hipMemcpyAsync(h->order, cp.out.p, 256 + 16, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if (h->err)
            return fail(c, TW_EDEVICE, "captured backtrack: a predecessor is missing");
        SL = h->last_state;
    }
    int t = 0;
    for (; t < L; ++t) {
        const int v = h->order[t];
        if (v < 0 || v >= n || !((SL >> v) & 1ull))
            return fail(c, TW_EDEVICE, "captured backtrack: bad vertex %d at step %d", v, t);
        order[t] = v;
    }
    for (int v = 0; v < n; ++v)
        if (!((SL >> v) & 1ull))
            order[t++] = v;
    if (t != n || popc(SL) != L)
        return fail(c, TW_EDEVICE, "captured backtrack produced %d of %d vertices", t, n);
    const int w = fill_in_width(g, order);
    if (w < 0 || w > k)
        return fail(c, TW_EDEVICE, "captured order has width %d > %d", w, k);
    return TW_OK;
}

// ---------------------------------------------------------------------------
// Graphs of up to 126 vertices: states of two words (vertices 0..63, 64..125).
// The level loop, duplicate removal, overflow replay and order rebuild are
// those of the 64-vertex path (exact duplicate removal only); the table slot
// layout that limits n to 126 is described with the kernel.
// ---------------------------------------------------------------------------
constexpr int kWideMaxN = 126;

struct V2 {
    uint64_t w[2] = {0, 0};
    bool has(int v) const { return (w[v >> 6] >> (v & 63)) & 1ull; }
    void set(int v) { w[v >> 6] |= 1ull << (v & 63); }
    void clear(int v) { w[v >> 6] &= ~(1ull << (v & 63)); }
    int count() const { return popc(w[0]) + popc(w[1]); }
    bool any() const { return (w[0] | w[1]) != 0; }
    V2 operator&(const V2 &o) const { V2 r; r.w[0] = w[0] & o.w[0]; r.w[1] = w[1] & o.w[1]; return r; }
    V2 operator|(const V2 &o) const { V2 r; r.w[0] = w[0] | o.w[0]; r.w[1] = w[1] | o.w[1]; return r; }
    V2 operator~() const { V2 r; r.w[0] = ~w[0]; r.w[1] = ~w[1]; return r; }
    int lowest() const { return w[0] ? __builtin_ctzll(w[0]) : 64 + __builtin_ctzll(w[1]); }
};

struct GraphW {
    int n = 0;
    V2 rows[128];
};

V2 all_of(int n)
{
    V2 a;
    for (int v = 0; v < n; ++v)
        a.set(v);
    return a;
}

tw_status validate_wide(tw_ctx *c, const tw_graph128 *g, GraphW &out)
{
    if (!g || !g->adj)
        return fail(c, TW_EINVAL, "graph or adjacency pointer is NULL");
    if (g->n < 1 || g->n > kWideMaxN)
        return fail(c, TW_EINVAL, "n=%u outside 1..%d", g->n, kWideMaxN);
    out.n = (int)g->n;
    const V2 all = all_of(out.n);
    for (int i = 0; i < out.n; ++i) {
        V2 r;
        r.w[0] = g->adj[2 * i];
        r.w[1] = g->adj[2 * i + 1];
        if ((r & ~all).any())
            return fail(c, TW_EINVAL, "row %d has bits at positions >= n", i);
        if (r.has(i))
            return fail(c, TW_EINVAL, "self-loop at vertex %d", i);
        out.rows[i] = r;
    }
    for (int i = 0; i < out.n; ++i)
        for (int j = 0; j < out.n; ++j)
            if (out.rows[i].has(j) != out.rows[j].has(i))
                return fail(c, TW_EINVAL, "adjacency not symmetric at (%d,%d)", i, j);
    return TW_OK;
}

// Minor-min-width (§3.3) with the tie-breaks of mmw_bound.
int mmw_bound_wide(const GraphW &g)
{
    V2 nb[128];
    V2 alive = all_of(g.n);
    for (int v = 0; v < g.n; ++v)
        nb[v] = g.rows[v];
    int lb = 0;
    while (alive.count() >= 2) {
        int d1 = 1 << 20, d2 = 1 << 20, v = -1;
        for (int x = 0; x < g.n; ++x) {
            if (!alive.has(x))
                continue;
            const int d = nb[x].count();
            if (d < d1) {
                d2 = d1;
                d1 = d;
                v = x;
            } else if (d < d2) {
                d2 = d;
            }
        }
        lb = std::max(lb, d2);
        if (d1 == 0) {
            alive.clear(v);
            continue;
        }
        int u = -1, du = 1 << 20;
        for (int x = 0; x < g.n; ++x)
            if (nb[v].has(x) && nb[x].count() < du) {
                du = nb[x].count();
                u = x;
            }
        for (int w = 0; w < g.n; ++w) {
            if (!nb[v].has(w))
                continue;
            nb[w].clear(v);
            if (w != u) {
                nb[w].set(u);
                nb[u].set(w);
            }
        }
        nb[v] = V2{};
        alive.clear(v);
    }
    return lb;
}

int fill_in_width_wide(const GraphW &g, const int32_t *order)
{
    V2 adj[128], seen;
    for (int v = 0; v < g.n; ++v)
        adj[v] = g.rows[v];
    for (int t = 0; t < g.n; ++t) {
        const int v = order[t];
        if (v < 0 || v >= g.n || seen.has(v))
            return -1;
        seen.set(v);
    }
    V2 alive = seen;
    int width = 0;
    for (int t = 0; t < g.n; ++t) {
        const int v = order[t];
        V2 N = adj[v] & alive;
        N.clear(v);
        width = std::max(width, N.count());
        for (int u = 0; u < g.n; ++u)
            if (N.has(u)) {
                V2 add = N;
                add.clear(u);
                adj[u] = adj[u] | add;
            }
        alive.clear(v);
    }
    return width;
}

tw_status emit_level_wide(tw_ctx *c, const Sink &sink, int k, int i, const Level &lv, uint64_t expansions,
                          uint64_t successors)
{
    std::vector<uint64_t> keys(2 * lv.count);
    std::vector<uint8_t> lastv(lv.count, 0);
    if (lv.count) {
        HIP_TRY(c, hipMemcpyAsync(keys.data(), lv.keys.p, lv.count * 16, hipMemcpyDeviceToHost, c->stream));
        if (i > 0)
            HIP_TRY(c, hipMemcpyAsync(lastv.data(), lv.lastv.p, lv.count, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    tw_level_record rec{};
    rec.k = k;
    rec.level = i;
    rec.count = lv.count;
    rec.expansions = expansions;
    rec.successors = successors;
    rec.states = keys.data();
    rec.last_v = lastv.data();
    sink.fn(&rec, sink.user);
    return TW_OK;
}

// decide(k) for a graph of up to 126 vertices (Listing 1, exact duplicate
// removal).  keep_all: every level stays on the device, trimmed to its size.
tw_status run_decide_wide(tw_ctx *c, const GraphW &g, int k, bool keep_all, const Sink *sink,
                          std::vector<Level> &levels, int *yes, RunStats &rs, V2 allowed)
{
    const int n = g.n;
    const int L = std::max(0, n - k - 1);
    rs.decisions++;
    free_levels(c, levels);
    levels.assign(1, Level{});
    {
        Level &l0 = levels[0];
        tw_status s = acquire(c, l0.keys, 16);
        if (s != TW_OK)
            return s;
        HIP_TRY(c, twk::launch_fill_zero(l0.keys.p, 16, c->stream));
        l0.count = 1;
    }
    if (sink && sink->fn) {
        tw_status s = emit_level_wide(c, *sink, k, 0, levels[0], 0, 0);
        if (s != TW_OK)
            return s;
    }
    {
        tw_status s = acquire(c, c->d_adj_wide, 128 * 16);
        if (s != TW_OK)
            return s;
        std::vector<uint64_t> rows(256, 0);
        for (int v = 0; v < n; ++v) {
            rows[2 * v] = g.rows[v].w[0];
            rows[2 * v + 1] = g.rows[v].w[1];
        }
        HIP_TRY(c, hipMemcpyAsync(c->d_adj_wide.p, rows.data(), rows.size() * 8, hipMemcpyHostToDevice,
                                  c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    const float alpha = (c->opt.load_factor > 0.f && c->opt.load_factor <= 0.9f) ? c->opt.load_factor : 0.25f;
    const size_t dev_free = free_device_bytes(c);
    double growth = (double)n;
    Buf scratch_keys, scratch_lastv;
    tw_status status = TW_OK;
    uint64_t cur = 1, run_peak = 1;
    int i = 0;
    for (; i < L; ++i) {
        Level &in = levels.back();
        const uint64_t in_count = in.count;
        const uint64_t pairs = in_count > UINT64_MAX / 128 ? UINT64_MAX : in_count * (uint64_t)(n - i);
        const uint64_t bound = std::min<uint64_t>(binom_sat(n, i + 1), pairs);
        uint64_t guess = c->opt.capacity_override
                             ? c->opt.capacity_override
                             : (uint64_t)std::min<double>((double)in_count * std::max(1.0, growth) * 1.3 + 4096.0,
                                                          1.8e19);
        guess = std::max<uint64_t>(std::min(guess, bound), 1);
        float a_eff = std::max(alpha, std::min(0.5f, (float)((double)guess * 16 * 3.0 / (double)dev_free)));
        uint64_t out_count = 0, succ = 0;
        bool injected = false;
        for (;;) {
            if (c->opt.max_states && guess > c->opt.max_states)
                guess = std::max<uint64_t>(c->opt.max_states, 1);
            const uint64_t slots = ((uint64_t)((double)guess / a_eff) + 64 + 63) / 64 * 64;
            uint64_t out_cap = std::min<uint64_t>(bound, std::max<uint64_t>(guess, (uint64_t)(0.6 * (double)slots)));
            if (c->opt.max_states)
                out_cap = std::min<uint64_t>(out_cap, c->opt.max_states);
            status = acquire(c, c->table, slots * 16);
            if (status == TW_OK)
                status = acquire(c, scratch_keys, out_cap * 16);
            if (status == TW_OK)
                status = acquire(c, scratch_lastv, out_cap);
            if (status == TW_ENOMEM && a_eff < 0.8f) {
                release(c, scratch_keys);
                release(c, scratch_lastv);
                release(c, c->table);
                drop_cache(c);
                a_eff = 0.8f;
                status = TW_OK;
                c->err.clear();
                continue;
            }
            if (status != TW_OK)
                goto done;
            HIP_TRY(c, twk::launch_fill_empty(c->table.p, slots * 16, c->stream));
            HIP_TRY(c, twk::launch_zero_counters((LevelCounters *)c->d_ctr.p, c->stream));
            twk::LevelArgs a{};
            a.in = in.keys.p;
            a.in_count = in_count;
            a.out = scratch_keys.p;
            a.out_lastv = (uint8_t *)scratch_lastv.p;
            a.out_cap = out_cap;
            a.table = c->table.p;
            a.table_slots = slots;
            a.allowed = allowed.w[0];
            a.adj = (const uint64_t *)c->d_adj_wide.p;
            a.n = n;
            a.k = k;
            a.ctr = (LevelCounters *)c->d_ctr.p;
            a.max_probe = (uint32_t)std::min<uint64_t>(slots, 1u << 16);
            a.key_bytes = 16;
            const uint64_t waves = (in_count + 63) / 64;
            uint64_t blocks = (waves + twk::kWavesPerBlock - 1) / twk::kWavesPerBlock;
            blocks = std::min<uint64_t>(std::max<uint64_t>(blocks, 1), (uint64_t)c->cu_count * 8);
            if (c->opt.timing)
                HIP_TRY(c, hipEventRecord(c->ev0, c->stream));
            HIP_TRY(c, twk::launch_expand_wide(a, allowed.w[1], (unsigned)blocks, c->stream));
            if (c->opt.timing)
                HIP_TRY(c, hipEventRecord(c->ev1, c->stream));
            HIP_TRY(c, hipMemcpyAsync(c->h_ctr, c->d_ctr.p, sizeof(LevelCounters), hipMemcpyDeviceToHost,
                                      c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            rs.launches++;
            if (c->opt.timing) {
                float ms = 0.f;
                HIP_TRY(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
                rs.kernel_seconds += ms * 1e-3;
            }
            LevelCounters h = *c->h_ctr;
            if (c->opt.fault_inject_level == i + 1 && !injected) {
                injected = true;
                h.overflow = 1;
            }
            if (!h.overflow) {
                out_count = h.out_count;
                succ = h.successors;
                break;
            }
            rs.retries++;
            if (c->opt.max_states && out_cap >= c->opt.max_states) {
                status = fail(c, TW_ECAPACITY, "level %d needs more than max_states=%llu states", i + 1,
                              (unsigned long long)c->opt.max_states);
                goto done;
            }
            if (out_cap >= bound && (double)slots * 0.8 >= (double)bound && !injected) {
                status = fail(c, TW_EDEVICE, "overflow at level %d with capacity at its bound", i + 1);
                goto done;
            }
            guess = std::min<uint64_t>(bound, std::max<uint64_t>(guess * 2, (uint64_t)(1.3 * (double)h.out_count)));
            a_eff = std::max(a_eff * 0.75f, 0.1f);
        }
        rs.states_expanded += in_count;
        rs.expansions += in_count * (uint64_t)(n - i);
        rs.successors += succ;
        rs.unique += out_count;
        rs.levels++;
        rs.peak = std::max(rs.peak, std::max(out_count, in_count));
        run_peak = std::max(run_peak, out_count);
        growth = in_count ? (double)out_count / (double)in_count : 1.0;
        {
            Level nl;
            nl.count = out_count;
            if (keep_all || sink) {
                status = acquire(c, nl.keys, std::max<uint64_t>(out_count, 1) * 16);
                if (status == TW_OK)
                    status = acquire(c, nl.lastv, std::max<uint64_t>(out_count, 1));
                if (status != TW_OK)
                    goto done;
                if (out_count) {
                    HIP_TRY(c, hipMemcpyAsync(nl.keys.p, scratch_keys.p, out_count * 16, hipMemcpyDeviceToDevice,
                                              c->stream));
                    HIP_TRY(c, hipMemcpyAsync(nl.lastv.p, scratch_lastv.p, out_count, hipMemcpyDeviceToDevice,
                                              c->stream));
                }
            } else {
                nl.keys = scratch_keys;
                nl.lastv = scratch_lastv;
                scratch_keys = Buf{};
                scratch_lastv = Buf{};
            }
            if (sink && sink->fn) {
                status = emit_level_wide(c, *sink, k, i + 1, nl, in_count * (uint64_t)(n - i), succ);
                if (status != TW_OK) {
                    release(c, nl.keys);
                    release(c, nl.lastv);
                    goto done;
                }
            }
            if (!keep_all) {
                Level &old = levels.back();
                if (!sink) {
                    scratch_keys = old.keys;
                    scratch_lastv = old.lastv;
                    old.keys = Buf{};
                    old.lastv = Buf{};
                } else {
                    release(c, old.keys);
                    release(c, old.lastv);
                }
                levels.back() = nl;
            } else {
                levels.push_back(nl);
            }
        }
        cur = out_count;
        if (out_count == 0)
            break;
    }
done:
    release(c, scratch_keys);
    release(c, scratch_lastv);
    rs.run_peak = run_peak;
    if (status != TW_OK)
        return status;
    *yes = (L == 0 || (i >= L && cur > 0)) ? 1 : 0;
    return TW_OK;
}

// The order of a YES run whose levels were all kept: follow the creating
// vertex back from the first state of the last level.
tw_status reconstruct_wide(tw_ctx *c, const GraphW &g, int k, const std::vector<Level> &levels, int32_t *order)
{
    const int n = g.n;
    const int L = (int)levels.size() - 1;
    std::vector<int> rev;
    V2 S, SL;
    if (L > 0) {
        uint64_t key[2] = {0, 0};
        HIP_TRY(c, hipMemcpyAsync(key, levels[L].keys.p, 16, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        S.w[0] = key[0];
        S.w[1] = key[1];
        SL = S;
        uint64_t idx = 0;
        for (int i = L; i >= 1; --i) {
            uint8_t v = 0;
            HIP_TRY(c, hipMemcpyAsync(&v, (const uint8_t *)levels[i].lastv.p + idx, 1, hipMemcpyDeviceToHost,
                                      c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            if (v >= n || !S.has(v))
                return fail(c, TW_EDEVICE, "reconstruction: bad last vertex %d at level %d", v, i);
            rev.push_back(v);
            S.clear(v);
            if (i == 1)
                break;
            *c->h_find = ~0ull;
            HIP_TRY(c, hipMemcpyAsync(c->d_find.p, c->h_find, 8, hipMemcpyHostToDevice, c->stream));
            HIP_TRY(c, twk::launch_find_wide(levels[i - 1].keys.p, levels[i - 1].count, S.w[0], S.w[1],
                                             (unsigned long long *)c->d_find.p, c->stream));
            HIP_TRY(c, hipMemcpyAsync(c->h_find, c->d_find.p, 8, hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            idx = *c->h_find;
            if (idx == ~0ull)
                return fail(c, TW_EDEVICE, "reconstruction: predecessor missing at level %d", i - 1);
        }
    }
    int t = 0;
    for (int r = (int)rev.size() - 1; r >= 0; --r)
        order[t++] = rev[(size_t)r];
    for (int v = 0; v < n; ++v)
        if (!SL.has(v))
            order[t++] = v;
    if (t != n)
        return fail(c, TW_EDEVICE, "reconstruction produced %d of %d vertices", t, n);
    const int w = fill_in_width_wide(g, order);
    if (w < 0 || w > k)
        return fail(c, TW_EDEVICE, "reconstructed order has width %d > %d", w, k);
    return TW_OK;
}

// tw and an order: ascending bounds from the minor-min-width bound; each YES
// keeps its levels while they fit the keep budget, else the search is run
// again restricted to the subsets of one last-level state.
tw_status solve_wide(tw_ctx *c, const GraphW &g, int32_t *out_tw, int32_t *out_order, RunStats &rs)
{
    const int n = g.n;
    const V2 all = all_of(n);
    for (int k = mmw_bound_wide(g); k < n; ++k) {
        std::vector<Level> levels;
        int yes = 0;
        const int L = std::max(0, n - k - 1);
        // a YES needs its levels for the order; keep them unless they outgrow the budget
        tw_status s = run_decide_wide(c, g, k, false, nullptr, levels, &yes, rs, all);
        if (s != TW_OK) {
            free_levels(c, levels);
            return s;
        }
        if (!yes) {
            free_levels(c, levels);
            continue;
        }
        V2 SL;
        if (L > 0) {
            uint64_t key[2] = {0, 0};
            HIP_TRY(c, hipMemcpyAsync(key, levels.back().keys.p, 16, hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            SL.w[0] = key[0];
            SL.w[1] = key[1];
        }
        free_levels(c, levels);
        // the levels restricted to subsets of one last-level state are small: keep them all
        int yes2 = 0;
        s = run_decide_wide(c, g, k, true, nullptr, levels, &yes2, rs, L > 0 ? SL : all);
        if (s == TW_OK && !yes2)
            s = fail(c, TW_EDEVICE, "restricted search lost the state it started from");
        if (s == TW_OK)
            s = reconstruct_wide(c, g, k, levels, out_order);
        free_levels(c, levels);
        if (s != TW_OK)
            return s;
        *out_tw = k;
        return TW_OK;
    }
    return fail(c, TW_EDEVICE, "no bound below n gave YES");
}

// Search from bound k0 (lb <= k0 <= n-1): after a YES at k (its order kept)
// move down, after a NO move up, until a YES at t meets a NO at t-1 or t = lb.
// With k0 = lb this is the ascending search of Listing 1 started at the
// minor-min-width bound.
tw_status solve_one(tw_ctx *c, const Graph &g, const Reduction *red, int lb, int k0, int32_t *out_tw,
                    int32_t *out_order, RunStats &rs, GraphOutcome *oc)
{
    const int n = g.n;
    const uint64_t e0 = rs.expansions, s0 = rs.states_expanded;
    const uint32_t d0 = rs.decisions;
    int known_no = lb - 1;
    int best_yes = n - 1;
    uint64_t peak_yes = 1;
    for (int v = 0; v < n; ++v)
        out_order[v] = v;  // any order has width <= n - 1
    int k = std::min(std::max(k0, lb), n - 1);
    if (oc)
        oc->start_k = k;
    std::vector<int32_t> order((size_t)n);
    std::vector<Level> levels;
    Captured *cap = capture_for(c, g);
    while (best_yes > known_no + 1) {
        int yes = 0;
        if (oc && rs.decisions > d0)
            oc->peak_any = std::max(oc->peak_any, rs.run_peak);
        if (cap) {
            // the level loop as one graph replay per bound
            tw_status s = TW_OK;
            if (red && k < red->clique_size - 1)
                rs.decisions++;  // NO without a search below the clique bound
            else
                s = captured_decide(c, *cap, red ? augmented(g, *red, k) : g, k, red ? ~red->clique : ~0ull,
                                    &yes, rs);
            if (s == kNotCaptured) {
                rs.decisions--;
                cap = nullptr;  // this bound (and the rest) on the host-driven loop
                continue;
            }
            if (s == TW_OK && yes)
                s = captured_order(c, *cap, red ? augmented(g, *red, k) : g, k, order.data());
            if (s != TW_OK)
                return s;
            if (yes) {
                best_yes = k;
                peak_yes = rs.run_peak;
                std::copy(order.begin(), order.end(), out_order);
                k = best_yes - 1;
            } else {
                known_no = std::max(known_no, k);
                k = known_no + 1;
            }
            if (k >= best_yes || k <= known_no)
                break;
            continue;
        }
        tw_status s = decide_checked(c, g, red, k, kKeepIfSmall, levels, &yes, rs);
        if (oc)
            oc->peak_any = std::max(oc->peak_any, rs.run_peak);
        if ((s == TW_ECAPACITY || s == TW_ENOMEM) && k > known_no + 1) {
            // a bound above the ascending frontier (a learned start) outgrew the
            // state cap or memory: continue upwards from the frontier instead
            free_levels(c, levels);
            c->err.clear();
            k = known_no + 1;
            continue;
        }
        if (s != TW_OK) {
            free_levels(c, levels);
            return s;
        }
        if (yes) {
            const uint64_t peak = rs.run_peak;
            // the order: from the kept levels, or, when they were too large to
            // keep, pick one state S_L of the last level and search again over
            // subsets of S_L only (small), keeping those levels
            uint64_t SL = 0;
            const int L = std::max(0, n - k - 1);
            if (L > 0 && (int)levels.size() != L + 1) {
                const int kb = n <= 32 ? 4 : 8;
                HIP_TRY(c, hipMemcpyAsync(&SL, levels.back().keys.p, kb, hipMemcpyDeviceToHost, c->stream));
                HIP_TRY(c, hipStreamSynchronize(c->stream));
                free_levels(c, levels);
                int yes2 = 0;
                const int dedup = c->opt.dedup;
                c->opt.dedup = TW_DEDUP_EXACT;  // the small restricted search is always exact
                s = run_decide_reduced(c, g, red, k, kKeepAll, nullptr, levels, &yes2, rs, SL);
                c->opt.dedup = dedup;
                if (s == TW_OK && !yes2)
                    s = fail(c, TW_EDEVICE, "restricted search lost the state it started from");
                if (s != TW_OK) {
                    free_levels(c, levels);
                    return s;
                }
            }
            s = reconstruct(c, red ? augmented(g, *red, k) : g, k, levels, order.data());
            free_levels(c, levels);
            rs.run_peak = peak;
            if (s != TW_OK)
                return s;
            const int w = fill_in_width(g, order.data());
            best_yes = (c->opt.dedup != TW_DEDUP_EXACT && w >= lb && w < k) ? w : k;
            peak_yes = rs.run_peak;
            std::copy(order.begin(), order.end(), out_order);
            k = best_yes - 1;
        } else {
            free_levels(c, levels);
            known_no = std::max(known_no, k);
            k = known_no + 1;
        }
        if (k >= best_yes || k <= known_no)
            break;
    }
    const int w = fill_in_width(g, out_order);
    if (w != best_yes)
        return fail(c, TW_EDEVICE, "order width %d differs from treewidth %d", w, best_yes);
    *out_tw = best_yes;
    if (oc) {
        oc->peak_any = std::max(oc->peak_any, rs.run_peak);
        oc->peak_yes = peak_yes;
        oc->expansions = rs.expansions - e0;
        oc->states = rs.states_expanded - s0;
        oc->decisions = rs.decisions - d0;
        oc->path = 1;
    }
    return TW_OK;
}

// Trace mode of the batched search (tw_trace_batch): per graph, up to
// max_records level records; nrecords[t] is what graph t's last batched
// attempt wrote (or wanted, when above max_records).
struct BatchTrace {
    uint32_t max_records = 0;
    uint64_t first_arena = 0;     // arena of the first attempt (0: as tw_solve_batch)
    tw_batch_level *records = nullptr;
    uint32_t *nrecords = nullptr;
};

// One batched solve (level rounds or one persistent launch) over the graphs ids[0..B): start bound k0s[t] and
// arena of arena[t] states for graph ids[t].  Graphs that finish get their
// tw, order and outcome; graphs whose arena or table filled up are appended
// to single_ids for the tw_solve path.

// The batch schedule a call runs: TW_BATCH_AUTO takes the persistent queue,
// or level rounds with the reductions (their small levels favour the rounds).
int batch_schedule_of(const tw_ctx *c)
{
    if (c->opt.batch_schedule != TW_BATCH_AUTO)
        return c->opt.batch_schedule;
    return c->opt.reductions == TW_REDUCE_CLIQUE_PATHS ? TW_BATCH_ROUNDS : TW_BATCH_PERSISTENT;
}

tw_status batch_launch(tw_ctx *c, const std::vector<Graph> &graphs, const std::vector<Reduction> *reds,
                       const std::vector<int> &lbs,
                       const std::vector<int> &k0s, const std::vector<uint64_t> &arenas,
                       const std::vector<int> &ids, int32_t *out_tw, int32_t *out_orders,
                       const std::vector<size_t> &offs, tw_status *out_status, std::vector<int> &single_ids,
                       std::vector<GraphOutcome> &outcomes, RunStats &rs, const BatchTrace *trace)
{
    const size_t B = ids.size();
    if (!B)
        return TW_OK;
    uint32_t chunk = c->opt.batch_chunk ? c->opt.batch_chunk : 256u;
    chunk = std::max<uint32_t>(64u, (chunk + 63u) / 64u * 64u);
    const float alpha = (c->opt.load_factor > 0.f && c->opt.load_factor <= 0.9f) ? c->opt.load_factor : 0.5f;
    uint64_t job_cap = 0, arena_total = 0, slot_total = 0;
    std::vector<uint64_t> aoff(B), soff(B), slots(B);
    for (size_t b = 0; b < B; ++b) {
        const int n = graphs[(size_t)ids[b]].n;
        job_cap += (uint64_t)n * (uint64_t)n + 1;
        aoff[b] = arena_total;
        arena_total += arenas[b];
        // table sized for the arena at the target load (a level holds well under the whole arena)
        slots[b] = ((uint64_t)((double)arenas[b] * 0.5 / alpha) + 64 + 63) / 64 * 64;
        soff[b] = slot_total;
        slot_total += slots[b];
    }
    const size_t job_bytes = (job_cap * sizeof(twk::BatchJob) + 15) / 16 * 16;
    Buf d_graphs, d_jobs, d_q, d_keys, d_lastv, d_parent, d_table, d_paths, d_trace;
    auto cleanup = [&]() {
        release(c, d_trace);
        release(c, d_paths);
        release(c, d_parent);
        release(c, d_graphs);
        release(c, d_jobs);
        release(c, d_q);
        release(c, d_keys);
        release(c, d_lastv);
        release(c, d_table);
    };
    tw_status s = acquire(c, d_graphs, B * sizeof(twk::BatchGraph));
    if (s == TW_OK)
        s = acquire(c, d_jobs, job_bytes);
    if (s == TW_OK)
        s = acquire(c, d_q, sizeof(twk::BatchQueue));
    if (s == TW_OK)
        s = acquire(c, d_keys, arena_total * sizeof(uint64_t));
    if (s == TW_OK)
        s = acquire(c, d_lastv, arena_total);
    if (s == TW_OK)
        s = acquire(c, d_parent, arena_total * sizeof(uint32_t));
    if (s == TW_OK)
        s = acquire(c, d_table, slot_total * sizeof(uint64_t));
    if (s == TW_OK && reds)
        s = acquire(c, d_paths, B * 64 * 64);
    const uint64_t tcap = trace ? trace->max_records : 0;
    if (s == TW_OK && tcap)
        s = acquire(c, d_trace, B * tcap * sizeof(twk::BatchTraceRec));
    if (s != TW_OK) {
        cleanup();
        return s;
    }
    std::vector<uint8_t> hpaths(reds ? B * 64 * 64 : 0);
    std::vector<twk::BatchGraph> hg(B);
    std::vector<twk::BatchJob> hj(B);
    for (size_t b = 0; b < B; ++b) {
        const int t = ids[b];
        const Graph &g = graphs[(size_t)t];
        twk::BatchGraph &G = hg[b];
        std::memset(&G, 0, sizeof G);
        for (int j = 0; j < g.n; ++j)
            G.adj[j] = g.rows[j];
        G.keys = (uint64_t *)d_keys.p + aoff[b];
        G.lastv = (uint8_t *)d_lastv.p + aoff[b];
        G.parent = (uint32_t *)d_parent.p + aoff[b];
        G.arena_cap = arenas[b];
        G.table = (uint64_t *)d_table.p + soff[b];
        G.table_slots = slots[b];
        G.level_off[0] = 0;
        G.level_off[1] = 1;
        G.status = twk::kBatchRunning;
        G.n = g.n;
        G.k = k0s[(size_t)t];
        G.level = 0;
        G.L = g.n - G.k - 1;
        G.tw = -1;
        G.known_no = lbs[(size_t)t] - 1;
        G.best_yes = g.n - 1;
        G.tag = 1;
        G.decisions = 1;
        G.peak_k = 1;
        G.peak_yes = 1;
        for (int v = 0; v < 64; ++v)
            G.order[v] = v < g.n ? v : -1;
        G.allowed = ~0ull;
        G.paths = nullptr;
        G.fault_level = c->opt.fault_inject_level;
        if (tcap) {
            G.trace = (twk::BatchTraceRec *)d_trace.p + b * tcap;
            G.trace_cap = (uint32_t)tcap;
        }
        for (int j = 0; j < g.n; ++j)
            G.adjk[j] = g.rows[j];
        if (reds) {
            const Reduction &r = (*reds)[(size_t)t];
            G.allowed = ~r.clique;
            std::memcpy(hpaths.data() + b * 64 * 64, r.paths.data(), 64 * 64);
            G.paths = (const uint8_t *)d_paths.p + b * 64 * 64;
            // the first bound's rows; later bounds set theirs on the device
            for (int j = 0; j < g.n; ++j)
                for (int u = 0; u < g.n; ++u)
                    if ((int)r.paths[(size_t)j * 64 + u] > G.k)
                        G.adjk[j] |= 1ull << u;
        }
        twk::BatchJob &J = hj[b];
        std::memset(&J, 0, sizeof J);
        J.graph = (int32_t)b;
        J.count = 1;
        J.out_base = 1;
        J.k = G.k;
        J.tag = G.tag;
        J.chunk = chunk;
        J.ready = 1;  // one chunk: the empty set
    }
    twk::BatchQueue hq{};
    hq.tail = B;
    hq.capacity = job_cap;
    hq.active = (uint32_t)B;
    // tables start with tag 0 (never a live tag); jobs beyond the first B are not ready
    HIP_TRY(c, twk::launch_fill_zero(d_table.p, slot_total * sizeof(uint64_t), c->stream));
    HIP_TRY(c, twk::launch_fill_zero(d_jobs.p, job_bytes, c->stream));
    HIP_TRY(c, hipMemcpyAsync(d_graphs.p, hg.data(), B * sizeof(twk::BatchGraph), hipMemcpyHostToDevice,
                              c->stream));
    if (reds)
        HIP_TRY(c, hipMemcpyAsync(d_paths.p, hpaths.data(), B * 64 * 64, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(d_jobs.p, hj.data(), B * sizeof(twk::BatchJob), hipMemcpyHostToDevice,
                              c->stream));
    HIP_TRY(c, hipMemcpyAsync(d_q.p, &hq, sizeof hq, hipMemcpyHostToDevice, c->stream));

    twk::BatchArgs a{};
    a.graphs = (twk::BatchGraph *)d_graphs.p;
    a.jobs = (twk::BatchJob *)d_jobs.p;
    a.q = (twk::BatchQueue *)d_q.p;
    a.chunk = chunk;
    a.max_probe = 1u << 14;
    a.max_load = 0.85f;
    a.spin_limit = 8u * 1000u * 1000u;  // idle polls of up to ~4 us each: about half a minute
    a.nb = (uint32_t)B;
    int per_cu = twk::batch_blocks_per_cu();
    if (batch_schedule_of(c) == TW_BATCH_PERSISTENT && c->batch_leave_blocks)
        per_cu = std::max(1, per_cu - c->batch_leave_blocks);  // a resident grid would leave no room
    const unsigned grid = (unsigned)(c->cu_count * per_cu);
    a.nwaves = grid * (unsigned)twk::kBatchWavesPerBlock;
    if (c->opt.timing)
        HIP_TRY(c, hipEventRecord(c->ev0, c->stream));
    if (batch_schedule_of(c) == TW_BATCH_PERSISTENT) {
        HIP_TRY(c, twk::launch_batch(a, grid, c->stream));
    } else {
        // level rounds until no graph runs; the host looks every 8 rounds
        a.jobs = nullptr;
        Buf d_tasks;
        tw_status ts = acquire(c, d_tasks, (B + 1) * sizeof(uint32_t));
        if (ts != TW_OK) {
            cleanup();
            return ts;
        }
        // every graph's search ends within n bounds of n levels each
        const int max_rounds = 64 * 64 + 64;
        bool finished = false;
        for (int round = 0; round < max_rounds && !finished; ++round) {
            hipError_t e = twk::launch_batch_round(a, (uint32_t)B, (uint32_t *)d_tasks.p, grid, c->stream);
            if (e == hipSuccess && (round & 7) == 7)
                e = hipMemcpyAsync(&hq, d_q.p, sizeof hq, hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess && (round & 7) == 7)
                e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) {
                release(c, d_tasks);
                cleanup();
                return fail(c, TW_EDEVICE, "batch round %d: %s", round, hipGetErrorString(e));
            }
            if ((round & 7) == 7)
                finished = hq.active == 0 || hq.abort;
        }
        release(c, d_tasks);
        if (!finished) {
            cleanup();
            return fail(c, TW_EDEVICE, "batch rounds did not finish within %d rounds", max_rounds);
        }
    }
    if (c->opt.timing)
        HIP_TRY(c, hipEventRecord(c->ev1, c->stream));
    HIP_TRY(c, hipMemcpyAsync(hg.data(), d_graphs.p, B * sizeof(twk::BatchGraph), hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipMemcpyAsync(&hq, d_q.p, sizeof hq, hipMemcpyDeviceToHost, c->stream));
    std::vector<twk::BatchTraceRec> hrec(B * tcap);
    if (tcap)
        HIP_TRY(c, hipMemcpyAsync(hrec.data(), d_trace.p, hrec.size() * sizeof(twk::BatchTraceRec),
                                  hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    static_assert(sizeof(twk::BatchTraceRec) == sizeof(tw_batch_level), "trace record layout");
    if (tcap)
        for (size_t b = 0; b < B; ++b) {
            const int t = ids[b];
            trace->nrecords[t] = hg[b].status == twk::kBatchDone ? hg[b].trace_len : 0;
            std::memcpy(trace->records + (size_t)t * tcap, hrec.data() + b * tcap,
                        std::min<uint64_t>(hg[b].trace_len, tcap) * sizeof(twk::BatchTraceRec));
        }
    rs.launches++;
    if (c->opt.timing) {
        float ms = 0.f;
        HIP_TRY(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
        rs.kernel_seconds += ms * 1e-3;
    }
    cleanup();
    if (hq.abort)
        return fail(c, TW_EDEVICE, "batch kernel aborted (work-queue wait bound or job capacity)");
    for (size_t b = 0; b < B; ++b) {
        const twk::BatchGraph &G = hg[b];
        const int t = ids[b];
        rs.states_expanded += G.states;
        rs.expansions += G.expansions;
        rs.successors += G.successors;
        rs.levels += G.levels_run;
        rs.decisions += G.decisions;
        rs.unique += G.unique;
        rs.peak = std::max<uint64_t>(rs.peak, G.peak);
        if (G.status != twk::kBatchDone) {
            single_ids.push_back(t);
            continue;
        }
        const Graph &g = graphs[(size_t)t];
        int32_t *o = out_orders + offs[(size_t)t];
        for (int v = 0; v < g.n; ++v)
            o[v] = G.order[v];
        const int w = fill_in_width(g, o);
        if (w != G.tw) {
            out_status[t] = fail(c, TW_EDEVICE, "batch graph %d: order width %d != treewidth %d", t, w, G.tw);
            continue;
        }
        out_tw[t] = G.tw;
        out_status[t] = TW_OK;
        GraphOutcome &oc = outcomes[(size_t)t];
        oc.peak_yes = G.peak_yes;
        oc.peak_any = G.peak;
        oc.expansions = G.expansions;
        oc.states = G.states;
        oc.start_k = k0s[(size_t)t];
        oc.decisions = G.decisions;
        oc.path = 0;
    }
    return TW_OK;
}

// Splits the batchable graphs into launches that fit a device-memory budget.
tw_status batch_run(tw_ctx *c, const std::vector<Graph> &graphs, const std::vector<Reduction> *reds,
                    const std::vector<int> &lbs,
                    const std::vector<int> &k0s, const std::vector<uint64_t> &arena_of,
                    const std::vector<int> &ids, int32_t *out_tw, int32_t *out_orders,
                    const std::vector<size_t> &offs, tw_status *out_status, std::vector<int> &single_ids,
                    std::vector<GraphOutcome> &outcomes, RunStats &rs, const BatchTrace *trace)
{
    const size_t free_b = free_device_bytes(c);
    const uint64_t budget = c->carve ? (uint64_t)(free_b * 0.9)
                                     : std::max<uint64_t>((uint64_t)(free_b / 2), (uint64_t)1 << 30);
    std::vector<int> group;
    std::vector<uint64_t> arenas;
    uint64_t used = 0;
    for (size_t q = 0; q <= ids.size(); ++q) {
        uint64_t need = 0;
        if (q < ids.size())
            need = arena_of[(size_t)ids[q]] * 13 + arena_of[(size_t)ids[q]] * 8 + 4096;
        if (q == ids.size() || (!group.empty() && used + need > budget)) {
            tw_status s = batch_launch(c, graphs, reds, lbs, k0s, arenas, group, out_tw, out_orders, offs,
                                       out_status, single_ids, outcomes, rs, trace);
            if (s == TW_ENOMEM) {
                // device memory taken meanwhile (the single-graph workers run
                // concurrently on their own streams): these graphs go that way too
                single_ids.insert(single_ids.end(), group.begin(), group.end());
                c->err.clear();
            } else if (s != TW_OK) {
                return s;
            }
            group.clear();
            arenas.clear();
            used = 0;
        }
        if (q < ids.size()) {
            group.push_back(ids[q]);
            arenas.push_back(arena_of[(size_t)ids[q]]);
            used += need;
        }
    }
    return TW_OK;
}

bool read_weights(const char *path, std::vector<float> &params)
{
    if (!path)
        return false;
    FILE *f = std::fopen(path, "rb");
    if (!f)
        return false;
    char magic[8];
    uint32_t count = 0;
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "TWMPNN01", 8) == 0 &&
              std::fread(&count, 4, 1, f) == 1 && count == tw_mpnn_param_count();
    if (ok) {
        params.resize(count);
        ok = std::fread(params.data(), 4, count, f) == count;
    }
    std::fclose(f);
    return ok;
}

// Learned start bounds and admission for graphs ids (network outputs: tw/n
// and log2(peak + 1)/32).
//  - Start bound: one below the prediction rounded down, clamped to [lb, n-2].
//    Starting at tw-1 costs nothing extra (the NO at tw-1 certifies the answer
//    anyway), while starting above tw adds a YES run at a larger bound, the
//    most expensive kind (and one whose levels may not fit); so errors are
//    pushed downwards.
//  - Graphs larger than any the network was trained on (kLearnedMaxN) keep
//    the ascending search's start and arena: predictions there overshoot.
//  - Admission: the arena of a batched graph is 16 x the predicted peak level
//    (never below the default); a graph whose arena would exceed kArenaMax is
//    sent to the single-graph path at once (where the worker contexts run it
//    beside the batch) instead of overflowing in the batch.
constexpr uint64_t kArenaMax = 1ull << 23;
// largest graphs whose learned start is used (the committed networks were
// trained on graphs of 16..30 and 16..40 vertices)
constexpr int kLearnedMaxN = 40;
// arena of the second batched attempt for graphs that outgrew the first
constexpr uint64_t kArenaRetry = 1ull << 24;
constexpr int kSingleWorkers = 4;  // worker contexts of the single-graph path in tw_solve_batch

tw_status predict_starts(tw_ctx *c, const std::vector<Graph> &graphs, const std::vector<int> &lbs,
                         const std::vector<int> &ids, std::vector<int> &k0s, std::vector<uint64_t> &arena_of,
                         std::vector<char> *too_big = nullptr)
{
    if (!c->net || ids.empty())
        return TW_OK;
    std::vector<tw_graph> gs(ids.size());
    for (size_t q = 0; q < ids.size(); ++q) {
        gs[q].n = (uint32_t)graphs[(size_t)ids[q]].n;
        gs[q].adj = graphs[(size_t)ids[q]].rows;
    }
    std::vector<float> pred(ids.size() * 2);
    tw_status s = tw_mpnn_predict(c->net, gs.data(), (uint32_t)ids.size(), pred.data());
    if (s != TW_OK)
        return fail(c, s, "network prediction failed");
    // states a level may hold: the cap, else what a table and two levels of
    // 8-byte keys at load 0.5 leave of the device memory (about 34 bytes each)
    const double fit = c->opt.max_states ? (double)c->opt.max_states : (double)free_device_bytes(c) / 34.0;
    for (size_t q = 0; q < ids.size(); ++q) {
        const int t = ids[q];
        const int n = graphs[(size_t)t].n;
        if (n > kLearnedMaxN)
            continue;  // beyond the trained sizes: the ascending search's start and arena
        const double tw_pred = (double)pred[2 * q] * n;
        const double peak = std::exp2(std::min(40.0, std::max(0.0, 32.0 * (double)pred[2 * q + 1]))) - 1.0;
        int k0 = (int)std::floor(tw_pred) - 1;
        k0 = std::max(lbs[(size_t)t], std::min(k0, n - 2));
        // a start above the ascending frontier pays off only when its levels
        // fit: a predicted peak beyond half of what fits starts at the frontier
        if (peak > 0.5 * fit)
            k0 = lbs[(size_t)t];
        k0s[(size_t)t] = k0;
        const double want = 16.0 * peak;
        if (too_big && want > (double)kArenaMax)
            (*too_big)[(size_t)t] = 1;
        arena_of[(size_t)t] = std::max<uint64_t>(arena_of[(size_t)t],
                                                 pow2_at_least((uint64_t)std::min(want, (double)kArenaMax)));
    }
    return TW_OK;
}

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" {

const char *tw_status_str(tw_status s)
{
    switch (s) {
    case TW_OK: return "ok";
    case TW_EINVAL: return "invalid argument";
    case TW_ENOMEM: return "out of memory";
    case TW_EDEVICE: return "device error";
    case TW_ECAPACITY: return "capacity limit reached";
    }
    return "unknown status";
}

const char *tw_last_error(const tw_ctx *ctx) { return ctx ? ctx->err.c_str() : ""; }

tw_status tw_ctx_create(const tw_options *options, tw_ctx **out)
{
    if (!out)
        return TW_EINVAL;
    *out = nullptr;
    tw_ctx *c = new (std::nothrow) tw_ctx();
    if (!c)
        return TW_ENOMEM;
    if (options) {
        size_t sz = options->struct_size ? std::min(options->struct_size, sizeof(tw_options))
                                         : sizeof(tw_options);
        std::memcpy(&c->opt, options, sz);
    }
    c->opt.struct_size = sizeof(tw_options);
    if ((c->opt.dedup != TW_DEDUP_EXACT && c->opt.dedup != TW_DEDUP_BLOOM &&
         c->opt.dedup != TW_DEDUP_BLOOM_CERTIFIED) ||
        (c->opt.reductions != TW_REDUCE_NONE && c->opt.reductions != TW_REDUCE_CLIQUE_PATHS) ||
        (c->opt.batch_schedule != TW_BATCH_AUTO && c->opt.batch_schedule != TW_BATCH_ROUNDS &&
         c->opt.batch_schedule != TW_BATCH_PERSISTENT) ||
        (c->opt.mmw_prune != TW_MMW_NONE && c->opt.mmw_prune != TW_MMW_PRUNE)) {
        delete c;
        return TW_EINVAL;
    }
    if (c->opt.workspace && c->opt.workspace_bytes) {
        c->ws.reset(c->opt.workspace, c->opt.workspace_bytes);
        c->carve = &c->ws;
    }
    if (c->opt.fault_inject_level < 0) {
        delete c;
        return TW_EINVAL;
    }
    c->device = c->opt.device;
    auto bad = [&](hipError_t e) {
        (void)e;
        delete c;
        return TW_EDEVICE;
    };
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess)
        return bad(e);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess && prop.multiProcessorCount > 0)
        c->cu_count = prop.multiProcessorCount;
    if (c->opt.stream) {
        c->stream = (hipStream_t)c->opt.stream;
    } else {
        e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (e != hipSuccess)
            return bad(e);
        c->own_stream = true;
    }
    if (scratch_setup(c->device) != hipSuccess) {
        tw_ctx_destroy(c);
        return TW_EDEVICE;
    }
    if (hipHostMalloc((void **)&c->h_ctr, sizeof(LevelCounters), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&c->h_find, sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess) {
        tw_ctx_destroy(c);
        return TW_ENOMEM;
    }
    if (c->opt.capture != TW_CAPTURE_AUTO && c->opt.capture != TW_CAPTURE_OFF) {
        tw_ctx_destroy(c);
        return TW_EINVAL;
    }
    if (c->opt.capture == TW_CAPTURE_AUTO &&
        hipHostMalloc(&c->h_cap, sizeof(CapHost), hipHostMallocDefault) != hipSuccess) {
        tw_ctx_destroy(c);
        return TW_ENOMEM;
    }
    if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
        tw_ctx_destroy(c);
        return TW_EDEVICE;
    }
    if (ensure_ctx_buffers(c) != TW_OK) {
        tw_ctx_destroy(c);
        return TW_ENOMEM;
    }
    if (c->opt.k_policy == TW_K_LEARNED) {
        std::vector<float> params;
        if (!read_weights(c->opt.weights_path, params) ||
            tw_mpnn_create(c->device, c->stream, params.data(), &c->net) != TW_OK) {
            tw_ctx_destroy(c);
            return TW_EINVAL;
        }
    } else if (c->opt.k_policy != TW_K_ASCENDING) {
        tw_ctx_destroy(c);
        return TW_EINVAL;
    }
    *out = c;
    return TW_OK;
}

void tw_ctx_destroy(tw_ctx *c)
{
    if (!c)
        return;
    (void)hipSetDevice(c->device);
    if (c->net)
        tw_mpnn_destroy(c->net);
    if (c->stream)
        (void)hipStreamSynchronize(c->stream);
    for (Captured *cp : c->captured)
        destroy_captured(c, cp);
    c->captured.clear();
    if (c->h_cap)
        (void)hipHostFree(c->h_cap);
    release(c, c->d_adj);
    release(c, c->d_adj_wide);
    release(c, c->d_ctr);
    release(c, c->d_find);
    release(c, c->table);
    release(c, c->bloom);
    release(c, c->parts);
    release(c, c->part_meta);
    drop_cache(c);
    if (c->h_ctr)
        (void)hipHostFree(c->h_ctr);
    if (c->h_find)
        (void)hipHostFree(c->h_find);
    if (c->ev0)
        (void)hipEventDestroy(c->ev0);
    if (c->ev1)
        (void)hipEventDestroy(c->ev1);
    if (c->own_stream && c->stream)
        (void)hipStreamDestroy(c->stream);
    delete c;
}

tw_status tw_decide(tw_ctx *c, const tw_graph *gr, int32_t k, int32_t *out_yes, tw_stats *stats)
{
    if (!c || !out_yes)
        return TW_EINVAL;
    c->err.clear();
    Graph g;
    tw_status s = validate(c, gr, g);
    if (s != TW_OK)
        return s;
    if (k < 0)
        return fail(c, TW_EINVAL, "k=%d < 0", k);
    if (hipSetDevice(c->device) != hipSuccess)
        return fail(c, TW_EDEVICE, "hipSetDevice failed");
    const double t0 = now_s();
    RunStats rs;
    std::vector<Level> levels;
    int yes = 0;
    Reduction red;
    if (c->opt.reductions)
        red = reduction_of(g, -1);
    s = kNotCaptured;
    if (Captured *cap = capture_for(c, g)) {
        // the level loop as one graph replay (NO without a search below the clique bound)
        if (c->opt.reductions && k < red.clique_size - 1) {
            rs.decisions++;
            s = TW_OK;
        } else {
            s = captured_decide(c, *cap, c->opt.reductions ? augmented(g, red, k) : g, k,
                                c->opt.reductions ? ~red.clique : ~0ull, &yes, rs);
        }
        if (s == kNotCaptured) {
            rs = RunStats{};
            c->err.clear();
        }
    }
    if (s == kNotCaptured)
        s = decide_checked(c, g, c->opt.reductions ? &red : nullptr, k, kKeepPair, levels, &yes, rs);
    free_levels(c, levels);
    add_stats(stats, rs, now_s() - t0);  // the work done, also when the call fails
    if (s != TW_OK)
        return s;
    *out_yes = yes;
    return TW_OK;
}

tw_status tw_trace_decide(tw_ctx *c, const tw_graph *gr, int32_t k,
                          void (*sink)(const tw_level_record *, void *), void *user, int32_t *out_yes)
{
    if (!c || !sink)
        return TW_EINVAL;
    c->err.clear();
    Graph g;
    tw_status s = validate(c, gr, g);
    if (s != TW_OK)
        return s;
    if (k < 0)
        return fail(c, TW_EINVAL, "k=%d < 0", k);
    if (hipSetDevice(c->device) != hipSuccess)
        return fail(c, TW_EDEVICE, "hipSetDevice failed");
    RunStats rs;
    std::vector<Level> levels;
    Sink sk;
    sk.fn = sink;
    sk.user = user;
    int yes = 0;
    Reduction red;
    if (c->opt.reductions)
        red = reduction_of(g, -1);
    s = run_decide_reduced(c, g, c->opt.reductions ? &red : nullptr, k, kKeepPair, &sk, levels, &yes, rs);
    free_levels(c, levels);
    if (s != TW_OK)
        return s;
    if (out_yes)
        *out_yes = yes;
    return TW_OK;
}

tw_status tw_solve(tw_ctx *c, const tw_graph *gr, int32_t *out_tw, int32_t *out_order, tw_stats *stats)
{
    if (!c || !out_tw || !out_order)
        return TW_EINVAL;
    c->err.clear();
    Graph g;
    tw_status s = validate(c, gr, g);
    if (s != TW_OK)
        return s;
    if (hipSetDevice(c->device) != hipSuccess)
        return fail(c, TW_EDEVICE, "hipSetDevice failed");
    const double t0 = now_s();
    RunStats rs;
    int lb = mmw_bound(g);
    Reduction red;
    if (c->opt.reductions) {
        red = reduction_of(g, lb);
        lb = std::max(lb, red.clique_size - 1);
    }
    std::vector<Graph> one(1, g);
    std::vector<int> lbs(1, lb), k0s(1, lb), ids(1, 0);
    std::vector<uint64_t> arena(1, 0);
    if (lb < g.n - 1) {
        s = predict_starts(c, one, lbs, ids, k0s, arena);
        if (s != TW_OK)
            return s;
    }
    s = solve_one(c, g, c->opt.reductions ? &red : nullptr, lb, k0s[0], out_tw, out_order, rs, nullptr);
    if (s != TW_OK)
        return s;
    add_stats(stats, rs, now_s() - t0);
    return TW_OK;
}

tw_status tw_decide128(tw_ctx *c, const tw_graph128 *gr, int32_t k, int32_t *out_yes, tw_stats *stats)
{
    if (!c || !out_yes)
        return TW_EINVAL;
    c->err.clear();
    GraphW g;
    tw_status s = validate_wide(c, gr, g);
    if (s != TW_OK)
        return s;
    if (k < 0)
        return fail(c, TW_EINVAL, "k=%d < 0", k);
    if (hipSetDevice(c->device) != hipSuccess)
        return fail(c, TW_EDEVICE, "hipSetDevice failed");
    const double t0 = now_s();
    RunStats rs;
    std::vector<Level> levels;
    int yes = 0;
    s = run_decide_wide(c, g, k, false, nullptr, levels, &yes, rs, all_of(g.n));
    free_levels(c, levels);
    if (s != TW_OK)
        return s;
    *out_yes = yes;
    add_stats(stats, rs, now_s() - t0);
    return TW_OK;
}

tw_status tw_trace_decide128(tw_ctx *c, const tw_graph128 *gr, int32_t k,
                             void (*sink)(const tw_level_record *, void *), void *user, int32_t *out_yes)
{
    if (!c || !sink)
        return TW_EINVAL;
    c->err.clear();
    GraphW g;
    tw_status s = validate_wide(c, gr, g);
    if (s != TW_OK)
        return s;
    if (k < 0)
        return fail(c, TW_EINVAL, "k=%d < 0", k);
    if (hipSetDevice(c->device) != hipSuccess)
        return fail(c, TW_EDEVICE, "hipSetDevice failed");
    RunStats rs;
    std::vector<Level> levels;
    Sink sk;
    sk.fn = sink;
    sk.user = user;
    int yes = 0;
    s = run_decide_wide(c, g, k, false, &sk, levels, &yes, rs, all_of(g.n));
    free_levels(c, levels);
    if (s != TW_OK)
        return s;
    if (out_yes)
        *out_yes = yes;
    return TW_OK;
}

tw_status tw_solve128(tw_ctx *c, const tw_graph128 *gr, int32_t *out_tw, int32_t *out_order, tw_stats *stats)
{
    if (!c || !out_tw || !out_order)
        return TW_EINVAL;
    c->err.clear();
    GraphW g;
    tw_status s = validate_wide(c, gr, g);
    if (s != TW_OK)
        return s;
    if (hipSetDevice(c->device) != hipSuccess)
        return fail(c, TW_EDEVICE, "hipSetDevice failed");
    const double t0 = now_s();
    RunStats rs;
    s = solve_wide(c, g, out_tw, out_order, rs);
    if (s != TW_OK)
        return s;
    const int w = fill_in_width_wide(g, out_order);
    if (w != *out_tw)
        return fail(c, TW_EDEVICE, "order width %d differs from treewidth %d", w, *out_tw);
    add_stats(stats, rs, now_s() - t0);
    return TW_OK;
}

tw_status tw_mmw128(const tw_graph128 *gr, int32_t *out_lb)
{
    if (!out_lb)
        return TW_EINVAL;
    GraphW g;
    tw_status s = validate_wide(nullptr, gr, g);
    if (s != TW_OK)
        return s;
    *out_lb = mmw_bound_wide(g);
    return TW_OK;
}

tw_status tw_order_width128(const tw_graph128 *gr, const int32_t *order, int32_t *out_width)
{
    if (!order || !out_width)
        return TW_EINVAL;
    GraphW g;
    tw_status s = validate_wide(nullptr, gr, g);
    if (s != TW_OK)
        return s;
    *out_width = fill_in_width_wide(g, order);
    return TW_OK;
}

tw_status tw_solve_noalloc(tw_ctx *c, const tw_graph *gr, int32_t *out_tw, int32_t *out_order, tw_stats *stats)
{
    if (!c || !out_tw || !out_order)
        return TW_EINVAL;
    c->err.clear();
    Graph g;
    tw_status s = validate(c, gr, g);
    if (s != TW_OK)
        return s;
    if (g.n > kNoAllocMaxN)
        return fail(c, TW_EINVAL, "tw_solve_noalloc takes n <= %d (n=%d)", kNoAllocMaxN, g.n);
    if (hipSetDevice(c->device) != hipSuccess)
        return fail(c, TW_EDEVICE, "hipSetDevice failed");
    void *base = c->device >= 0 && c->device < kMaxDevices ? g_scratch_ptr[c->device].load() : nullptr;
    if (!base)
        return fail(c, TW_EDEVICE, "static scratch of device %d not set up", c->device);
    const double t0 = now_s();
    RunStats rs;
    int lb = mmw_bound(g);
    Reduction red;
    if (c->opt.reductions) {
        red = reduction_of(g, lb);
        lb = std::max(lb, red.clique_size - 1);
    }
    // every device buffer of this call comes from the scratch: the context's
    // own buffers and cache are set aside and put back afterwards
    Carver scr;
    scr.reset(base, kScratchBytes);
    Buf saved_adj = c->d_adj, saved_ctr = c->d_ctr, saved_find = c->d_find, saved_table = c->table,
        saved_bloom = c->bloom, saved_parts = c->parts, saved_meta = c->part_meta;
    std::vector<Buf> saved_cache;
    saved_cache.swap(c->cache);
    Carver *saved_carve = c->carve;
    const uint64_t saved_budget = c->keep_budget;
    c->d_adj = c->d_ctr = c->d_find = c->table = c->bloom = c->parts = c->part_meta = Buf{};
    c->carve = &scr;
    c->keep_budget = kScratchBytes / 4;
    c->no_capture = true;
    s = ensure_ctx_buffers(c);
    if (s == TW_OK)
        s = solve_one(c, g, c->opt.reductions ? &red : nullptr, lb, lb, out_tw, out_order, rs, nullptr);
    if (s == TW_ENOMEM)
        s = fail(c, TW_ECAPACITY, "the search needs more than the %zu-byte static scratch (%s)", kScratchBytes,
                 c->err.c_str());
    // the carved buffers are dropped with the scratch's bookkeeping
    c->d_adj = saved_adj;
    c->d_ctr = saved_ctr;
    c->d_find = saved_find;
    c->table = saved_table;
    c->bloom = saved_bloom;
    c->parts = saved_parts;
    c->part_meta = saved_meta;
    c->cache.swap(saved_cache);
    c->carve = saved_carve;
    c->keep_budget = saved_budget;
    c->no_capture = false;
    if (s != TW_OK)
        return s;
    add_stats(stats, rs, now_s() - t0);
    return TW_OK;
}

namespace {

tw_status solve_batch(tw_ctx *c, const tw_graph *gs, uint32_t count, int32_t *out_tw, int32_t *out_orders,
                      tw_status *out_status, tw_graph_stats *out_graph_stats, tw_stats *stats,
                      const BatchTrace *trace)
{
    if (!c || (count && (!gs || !out_tw || !out_orders || !out_status)))
        return TW_EINVAL;
    c->err.clear();
    if (hipSetDevice(c->device) != hipSuccess)
        return fail(c, TW_EDEVICE, "hipSetDevice failed");
    const double t0 = now_s();
    RunStats rs;
    std::vector<Graph> graphs(count);
    std::vector<size_t> offs(count);
    std::vector<int> lbs(count, 0), k0s(count, 0);
    std::vector<uint64_t> arena_of(count, 0);
    std::vector<GraphOutcome> outcomes(count);
    std::vector<int> batch_ids;   // graphs solved together on the device
    std::vector<int> single_ids;  // graphs solved one at a time
    // default arena: as large as half of free device memory allows over the
    // batch (21 bytes per state: key, creator byte, parent index, table slot), 2^16..2^22
    uint64_t default_arena = c->opt.batch_graph_states;
    if (!default_arena) {
        const size_t free_b = free_device_bytes(c);
        const uint64_t per = (uint64_t)(free_b / 2) / std::max<uint64_t>(1, count) / 21;
        default_arena = 1ull << 16;
        while (default_arena < (1ull << 22) && default_arena * 2 <= per)
            default_arena *= 2;
    }
    size_t off = 0;
    for (uint32_t t = 0; t < count; ++t) {
        offs[t] = off;
        off += gs[t].n;
        out_tw[t] = -1;
        out_status[t] = validate(c, &gs[t], graphs[t]);
        if (out_status[t] == TW_OK)
            lbs[t] = mmw_bound(graphs[t]);
    }
    // §3.1 reductions: clique and path counts per graph, on the host's cores
    std::vector<Reduction> reds;
    if (c->opt.reductions) {
        reds.resize(count);
        const unsigned nth = std::max(1u, std::min<unsigned>(std::thread::hardware_concurrency(), 16u));
        std::vector<std::thread> pool;
        std::atomic<uint32_t> next{0};
        for (unsigned w = 0; w < nth; ++w)
            pool.emplace_back([&]() {
                for (uint32_t t; (t = next.fetch_add(1)) < count;)
                    if (out_status[t] == TW_OK)
                        reds[t] = reduction_of(graphs[t], lbs[t]);
            });
        for (std::thread &th : pool)
            th.join();
        for (uint32_t t = 0; t < count; ++t)
            if (out_status[t] == TW_OK)
                lbs[t] = std::max(lbs[t], reds[t].clique_size - 1);
    }
    for (uint32_t t = 0; t < count; ++t) {
        if (out_status[t] != TW_OK)
            continue;
        const Graph &g = graphs[t];
        k0s[t] = lbs[t];
        // an arena never needs more than every subset of V (minus V itself)
        arena_of[t] = g.n < 20 ? std::min<uint64_t>(default_arena, 1ull << g.n) : default_arena;
        if (lbs[t] >= g.n - 1) {
            // tw = n - 1: decide(n - 1) needs no level; any order has width n - 1
            out_tw[t] = g.n - 1;
            for (int v = 0; v < g.n; ++v)
                out_orders[offs[t] + v] = v;
            outcomes[t].start_k = g.n - 1;
            outcomes[t].path = 2;
        } else if (g.n <= twk::kBatchMaxN && c->opt.dedup == TW_DEDUP_EXACT && c->opt.mmw_prune == TW_MMW_NONE) {
            batch_ids.push_back((int)t);
        } else {
            single_ids.push_back((int)t);
        }
    }
    std::vector<int> learned_ids = batch_ids;
    learned_ids.insert(learned_ids.end(), single_ids.begin(), single_ids.end());
    std::vector<char> too_big(count, 0);
    tw_status st = predict_starts(c, graphs, lbs, learned_ids, k0s, arena_of, &too_big);
    if (st != TW_OK)
        return st;
    const bool library_arena = !c->opt.batch_graph_states || (trace && trace->first_arena);
    if (trace && trace->first_arena)
        for (int t : batch_ids)
            arena_of[(size_t)t] = trace->first_arena;
    else if (c->opt.batch_graph_states)
        for (int t : batch_ids)
            arena_of[(size_t)t] = c->opt.batch_graph_states;
    else if (c->net) {
        // admission: graphs predicted to outgrow any arena skip the batch
        std::vector<int> keep;
        for (int t : batch_ids) {
            if (too_big[(size_t)t])
                single_ids.push_back(t);
            else
                keep.push_back(t);
        }
        batch_ids.swap(keep);
    }
    const std::vector<Reduction> *rp = c->opt.reductions ? &reds : nullptr;

    // Graphs for the single-graph path run on a pool of worker contexts, each
    // with its own stream and host thread (one per hardware queue): those known
    // before the batch starts (above the batched size, Bloom dedup, or predicted
    // too large for an arena) beside the batched search, those that outgrow
    // their arena after it, largest first.  One graph's small levels leave most
    // of the GPU idle; several graphs at once fill it.  A graph that runs out of
    // memory beside the others is solved again alone at the end.  With a
    // caller's workspace they run one at a time on this context.
    struct Pool {
        std::vector<tw_ctx *> ctxs;
        std::vector<RunStats> rs;
        std::vector<std::thread> th;
        std::mutex m;
        std::condition_variable cv;
        std::deque<int> q;
        bool closed = false;
        tw_status status = TW_OK;
        std::string err;
        void finish()
        {
            {
                std::lock_guard<std::mutex> g(m);
                closed = true;
            }
            cv.notify_all();
            for (std::thread &t : th)
                if (t.joinable())
                    t.join();
        }
        ~Pool()
        {
            {
                std::lock_guard<std::mutex> g(m);
                q.clear();  // an early return: the queued graphs are not needed
            }
            finish();
            for (tw_ctx *x : ctxs)
                tw_ctx_destroy(x);
        }
    } pool;
    auto worker = [&](size_t w) {
        if (hipSetDevice(c->device) != hipSuccess) {
            std::lock_guard<std::mutex> g(pool.m);
            if (pool.status == TW_OK) {
                pool.status = TW_EDEVICE;
                pool.err = "hipSetDevice failed on a worker context";
            }
            return;
        }
        for (;;) {
            int t;
            {
                std::unique_lock<std::mutex> lk(pool.m);
                pool.cv.wait(lk, [&]() { return pool.closed || !pool.q.empty(); });
                if (pool.q.empty())
                    return;
                t = pool.q.front();
                pool.q.pop_front();
            }
            GraphOutcome oc;
            tw_status s = solve_one(pool.ctxs[w], graphs[(size_t)t], rp ? &reds[(size_t)t] : nullptr,
                                    lbs[(size_t)t], k0s[(size_t)t], &out_tw[t], out_orders + offs[(size_t)t],
                                    pool.rs[w], &oc);
            out_status[t] = s;
            outcomes[(size_t)t] = oc;
            if (s != TW_OK)
                out_tw[t] = -1;
            if (s == TW_EDEVICE) {
                std::lock_guard<std::mutex> g(pool.m);
                if (pool.status == TW_OK) {
                    pool.status = s;
                    pool.err = pool.ctxs[w]->err;
                }
                pool.q.clear();
                pool.closed = true;
                pool.cv.notify_all();
                return;
            }
        }
    };
    // the workers, on first need (none with a caller's workspace, or if no
    // context can be made: the graphs then run below on this context)
    auto start_pool = [&]() {
        if (!pool.ctxs.empty() || c->carve)
            return;
        tw_options o = c->opt;
        o.stream = nullptr;
        o.k_policy = TW_K_ASCENDING;  // starts are already chosen
        o.weights_path = nullptr;
        for (int w = 0; w < kSingleWorkers; ++w) {
            tw_ctx *x = nullptr;
            if (tw_ctx_create(&o, &x) != TW_OK)
                break;
            pool.ctxs.push_back(x);
        }
        pool.rs.resize(pool.ctxs.size());
        for (size_t w = 0; w < pool.ctxs.size(); ++w) {
            try {
                pool.th.emplace_back(worker, w);
            } catch (...) {
                break;  // no more threads: the workers started so far serve the queue
            }
        }
        // a context without a thread is not kept (with none, this context
        // solves the graphs itself)
        while (pool.ctxs.size() > pool.th.size()) {
            tw_ctx_destroy(pool.ctxs.back());
            pool.ctxs.pop_back();
        }
    };
    auto enqueue = [&](std::vector<int> &ids) {
        if (ids.empty())
            return;
        start_pool();
        if (pool.ctxs.empty())
            return;  // they stay in ids, for this context
        std::stable_sort(ids.begin(), ids.end(), [&](int x, int y) { return graphs[(size_t)x].n > graphs[(size_t)y].n; });
        {
            std::lock_guard<std::mutex> g(pool.m);
            pool.q.insert(pool.q.end(), ids.begin(), ids.end());
        }
        pool.cv.notify_all();
        ids.clear();
    };
    const bool early = !single_ids.empty();
    enqueue(single_ids);
    // single-graph work running beside the batch: the persistent grid leaves
    // each CU room for two blocks of it (its waves stay resident otherwise)
    struct LeaveRoom {
        tw_ctx *c;
        ~LeaveRoom() { c->batch_leave_blocks = 0; }
    } leave_room{c};
    c->batch_leave_blocks = early && !pool.ctxs.empty() ? 2 : 0;

    const size_t before = single_ids.size();
    st = batch_run(c, graphs, rp, lbs, k0s, arena_of, batch_ids, out_tw, out_orders, offs, out_status,
                   single_ids, outcomes, rs, trace);
    if (st != TW_OK)
        return st;
    // graphs whose levels outgrew their arena: once more together, with 4x the
    // arena (up to kArenaRetry states), before the one-at-a-time path
    if (library_arena && single_ids.size() > before) {
        std::vector<int> retry(single_ids.begin() + (long)before, single_ids.end());
        single_ids.resize(before);
        std::vector<int> again;
        for (int t : retry) {
            if (arena_of[(size_t)t] < kArenaRetry) {
                arena_of[(size_t)t] = std::min<uint64_t>(arena_of[(size_t)t] * 4, kArenaRetry);
                again.push_back(t);
            } else {
                single_ids.push_back(t);
            }
        }
        st = batch_run(c, graphs, rp, lbs, k0s, arena_of, again, out_tw, out_orders, offs, out_status,
                       single_ids, outcomes, rs, trace);
        if (st != TW_OK)
            return st;
    }
    c->batch_leave_blocks = 0;
    enqueue(single_ids);
    for (int t : single_ids) {
        GraphOutcome oc;
        tw_status s = solve_one(c, graphs[(size_t)t], rp ? &reds[(size_t)t] : nullptr, lbs[(size_t)t],
                                k0s[(size_t)t], &out_tw[t],
                                out_orders + offs[(size_t)t], rs, &oc);
        out_status[t] = s;
        outcomes[(size_t)t] = oc;
        if (s != TW_OK)
            out_tw[t] = -1;
        if (s == TW_EDEVICE)
            return s;
    }
    pool.finish();
    for (const RunStats &w : pool.rs)
        add_run_stats(rs, w);
    if (pool.status != TW_OK)
        return fail(c, pool.status, "%s", pool.err.c_str());
    // graphs a worker could not fit beside the batched search or the other
    // workers: once more here, alone
    for (uint32_t t = 0; t < count; ++t) {
        if (out_status[t] != TW_ENOMEM || graphs[t].n == 0)
            continue;
        GraphOutcome oc;
        tw_status s = solve_one(c, graphs[t], rp ? &reds[t] : nullptr, lbs[t], k0s[t], &out_tw[t],
                                out_orders + offs[t], rs, &oc);
        out_status[t] = s;
        outcomes[t] = oc;
        if (s != TW_OK)
            out_tw[t] = -1;
        if (s == TW_EDEVICE)
            return s;
    }
    if (out_graph_stats)
        for (uint32_t t = 0; t < count; ++t) {
            tw_graph_stats &o = out_graph_stats[t];
            std::memset(&o, 0, sizeof o);
            o.peak_yes = outcomes[t].peak_yes;
            o.expansions = outcomes[t].expansions;
            o.states_expanded = outcomes[t].states;
            o.start_k = outcomes[t].start_k;
            o.decisions = outcomes[t].decisions;
            o.path = outcomes[t].path;
            o.peak_any = outcomes[t].peak_any;
        }
    add_stats(stats, rs, now_s() - t0);
    return TW_OK;
}

}  // namespace

tw_status tw_solve_batch(tw_ctx *c, const tw_graph *gs, uint32_t count, int32_t *out_tw,
                         int32_t *out_orders, tw_status *out_status, tw_graph_stats *out_graph_stats,
                         tw_stats *stats)
{
    return solve_batch(c, gs, count, out_tw, out_orders, out_status, out_graph_stats, stats, nullptr);
}

tw_status tw_trace_batch(tw_ctx *c, const tw_graph *gs, uint32_t count, uint64_t first_arena_states,
                         uint32_t max_records, tw_batch_level *out_records, uint32_t *out_nrecords,
                         int32_t *out_tw, int32_t *out_orders, tw_status *out_status,
                         tw_graph_stats *out_graph_stats)
{
    if (!c || (count && (!out_records || !out_nrecords)) || max_records == 0)
        return TW_EINVAL;
    for (uint32_t t = 0; t < count; ++t)
        out_nrecords[t] = 0;
    BatchTrace tr;
    tr.max_records = max_records;
    tr.first_arena = first_arena_states;
    tr.records = out_records;
    tr.nrecords = out_nrecords;
    return solve_batch(c, gs, count, out_tw, out_orders, out_status, out_graph_stats, nullptr, &tr);
}

tw_status tw_probe_rate(int device, uint64_t bytes, uint64_t count, int mode, double *out_seconds)
{
    if (!out_seconds || mode < 0 || mode > 5 || bytes < 4096 || count == 0)
        return TW_EINVAL;
    *out_seconds = 0.0;
    if (hipSetDevice(device) != hipSuccess)
        return TW_EDEVICE;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
        return TW_EDEVICE;
    const unsigned blocks = (unsigned)cus * 8u;
    const uint64_t threads = (uint64_t)blocks * twk::kProbeBlock;
    uint64_t per_thread = (count + threads - 1) / threads;
    if (mode == 2)
        per_thread = (per_thread + 7) / 8 * 8;
    void *buf = nullptr;
    uint32_t *sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    tw_status st = TW_OK;
    float ms = 0.f;
    if (hipMalloc(&buf, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return TW_ENOMEM;
    }
    if (hipMalloc((void **)&sink, 4) != hipSuccess || hipMemset(buf, 0xFF, bytes) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        st = TW_EDEVICE;
        goto out;
    }
    // one untimed pass so the timed one meets warm TLBs
    if (twk::launch_probe_rate(buf, bytes, per_thread, mode, blocks, sink, nullptr) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess || hipMemset(buf, 0xFF, bytes) != hipSuccess ||
        hipEventRecord(e0, nullptr) != hipSuccess ||
        twk::launch_probe_rate(buf, bytes, per_thread, mode, blocks, sink, nullptr) != hipSuccess ||
        hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        st = TW_EDEVICE;
        goto out;
    }
    *out_seconds = (double)ms * 1e-3 * (double)count / (double)(per_thread * threads);
out:
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    if (sink)
        (void)hipFree(sink);
    (void)hipFree(buf);
    return st;
}

tw_status tw_reductions(const tw_graph *gr, uint64_t *out_clique, uint8_t *out_paths)
{
    if (!out_clique)
        return TW_EINVAL;
    Graph g;
    tw_status s = validate(nullptr, gr, g);
    if (s != TW_OK)
        return s;
    const Reduction r = reduction_of(g, -1);
    *out_clique = r.clique;
    if (out_paths)
        for (int u = 0; u < g.n; ++u)
            for (int v = 0; v < g.n; ++v)
                out_paths[u * g.n + v] = r.paths[(size_t)u * 64 + v];
    return TW_OK;
}

tw_status tw_mmw(const tw_graph *gr, int32_t *out_lb)
{
    if (!out_lb)
        return TW_EINVAL;
    Graph g;
    tw_status s = validate(nullptr, gr, g);
    if (s != TW_OK)
        return s;
    *out_lb = mmw_bound(g);
    return TW_OK;
}

tw_status tw_tree_decomposition(const tw_graph *gr, const int32_t *order, uint64_t *out_bags,
                                int32_t *out_parent, int32_t *out_width)
{
    if (!order || !out_bags || !out_parent || !out_width)
        return TW_EINVAL;
    Graph g;
    tw_status s = validate(nullptr, gr, g);
    if (s != TW_OK)
        return s;
    int pos[64];
    uint64_t seen = 0;
    for (int t = 0; t < g.n; ++t) {
        const int v = order[t];
        if (v < 0 || v >= g.n || ((seen >> v) & 1ull))
            return TW_EINVAL;
        seen |= 1ull << v;
        pos[v] = t;
    }
    // eliminate in order; bag(v) = v plus its neighbours still present, which
    // become a clique (fill-in); the parent is the one of them eliminated first
    uint64_t adj[64];
    for (int v = 0; v < g.n; ++v)
        adj[v] = g.rows[v];
    uint64_t alive = seen;
    int width = 0;
    for (int t = 0; t < g.n; ++t) {
        const int v = order[t];
        const uint64_t N = adj[v] & alive & ~(1ull << v);
        width = std::max(width, popc(N));
        out_bags[v] = N | (1ull << v);
        int parent = -1;
        for (uint64_t a = N; a; a &= a - 1) {
            const int u = __builtin_ctzll(a);
            adj[u] |= N & ~(1ull << u);
            if (parent < 0 || pos[u] < pos[parent])
                parent = u;
        }
        out_parent[v] = parent;
        alive &= ~(1ull << v);
    }
    *out_width = width;
    return TW_OK;
}

tw_status tw_order_width(const tw_graph *gr, const int32_t *order, int32_t *out_width)
{
    if (!order || !out_width)
        return TW_EINVAL;
    Graph g;
    tw_status s = validate(nullptr, gr, g);
    if (s != TW_OK)
        return s;
    *out_width = fill_in_width(g, order);
    return TW_OK;
}

}  // extern "C"
