// Batched search: every graph of a batch runs its own level loop (§3.1,
// Listing 1), from the bound the host gives it (lower bound or prediction),
// moving until a YES at t meets a NO at t-1 (or t = lower bound); the order of
// each YES is captured before the arena is reused.  Each graph has its own
// arena (all levels of its current bound, back to back, with each state's
// creating vertex and parent index for the order) and its own hash table.
// Table slots carry a 16-bit tag above the 48-bit state; a slot whose tag is
// not the level's tag counts as empty, so tables are never cleared.
//
// Two schedules share the per-chunk expansion (process_chunk) and the
// per-graph advance (finish_level):
//  * level rounds (round_kernel and friends, at the end of this file): one
//    launch per level of every running graph, then one that advances them;
//  * one persistent launch (batch_kernel): a device queue of jobs, one per
//    (graph, level), cut into chunks that every wave of the grid takes; the
//    wave finishing a level's last chunk advances that graph alone.  Exit:
//    every wave leaves once no graph is running, or after spin_limit
//    consecutive sleeps without work (abort flag; the host reports an error).
//
// Hand-over between waves of the persistent launch.  On this part each XCD
// has its own L2, so an agent-scope acquire invalidates the fetching XCD's
// L2 and a release writes it back (buffer_inv / buffer_wbl2), which would be
// paid per task and per poll.  That maintenance exists to make plain
// accesses coherent.  Here every value one wave hands to another (arena
// states, job and per-graph fields) is instead stored and loaded with
// device-scope relaxed atomics, which the compiler emits as single sc1
// accesses, each coherent across the XCDs by itself.  What remains is order:
// a writer drains its memory counters (s_waitcnt 0: every earlier access,
// stores included, complete at device scope; the same wait a release makes)
// before the atomic that publishes the data, and a reader issues its loads
// only after the atomic that shows the data published.  Compiler barriers
// keep the compiler from moving accesses across either point.  Counters stay
// read-modify-write atomics.  Idle waves poll two words and rescan the job
// window only when it changed, so that waiting takes little from the memory
// system the working waves probe.  Level rounds use plain accesses: the
// kernel boundaries order their levels.
#include "tw_batch.h"
#include "tw_wave.h"

namespace twk {
namespace {

constexpr int kBatchWaves = kBatchWavesPerBlock;
constexpr int kBatchBlock = 64 * kBatchWaves;
constexpr int kBatchStage = 384;  // 13 bytes per staged winner: 8 blocks of 4 waves fit a CU
constexpr uint64_t kKeyMask = (1ull << kBatchKeyBits) - 1;
constexpr uint64_t kMaxTask = 1024;  // states per task, largest (unless the caller asks for more)

template <typename T>
__device__ __forceinline__ T ld_relaxed(T *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Plain or device-coherent access (C: the persistent launch).
template <bool C, typename T>
__device__ __forceinline__ T ldc(const T *p)
{
    if constexpr (C)
        return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        return *p;
}

template <bool C, typename T>
__device__ __forceinline__ void stc(T *p, T v)
{
    if constexpr (C)
        __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        *p = v;
}

// Every memory access the wave has issued completes (stores acknowledged)
// before any later one issues; the compiler moves no access across it.
__device__ __forceinline__ void drain()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Digests of trace mode: two published 64-bit mixers, summed and xored over a
// level's states so the result does not depend on the order states are won.
__device__ __forceinline__ uint64_t splitmix64_out(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t fmix64(uint64_t z)
{
    z = (z ^ (z >> 33)) * 0xFF51AFD7ED558CCDull;
    z = (z ^ (z >> 33)) * 0xC4CEB9FE1A85EC53ull;
    return z ^ (z >> 33);
}

// Called by one lane: append a job for (g, level).  In the persistent launch
// the calling wave keeps the job's first chunk for itself (the cursor starts
// at 1), so a level of one chunk goes on without waiting for another wave to
// find it; returns the job's index + 1, or 0 when no job was made.
template <bool C>
__device__ uint64_t push_job(const BatchArgs &a, int g, int level, uint64_t begin, uint64_t count, int k,
                             uint32_t tag, uint64_t out_base)
{
    if (!a.jobs)
        return 0;  // level rounds: the graph's level fields are the next round's work
    const unsigned long long idx = atomicAdd(&a.q->tail, 1ull);
    if (idx >= a.q->capacity) {
        atomicOr(&a.q->abort, 1u);
        return 0;
    }
    BatchJob *j = &a.jobs[idx];
    stc<C>(&j->graph, (int32_t)g);
    stc<C>(&j->level, (int32_t)level);
    stc<C>(&j->begin, begin);
    stc<C>(&j->count, count);
    stc<C>(&j->out_base, out_base);
    stc<C>(&j->k, (int32_t)k);
    stc<C>(&j->tag, tag);
    // about 64 tasks for a large level (up to kMaxTask states each), so that
    // the graphs running together give every wave work in large pieces;
    // never below the task size the caller chose
    uint64_t per = (count + 63) / 64;
    per = (per + 63) / 64 * 64;
    per = per < a.chunk ? a.chunk : (per > kMaxTask ? (a.chunk > kMaxTask ? a.chunk : kMaxTask) : per);
    stc<C>(&j->chunk, (uint32_t)per);
    const uint32_t nchunks = (uint32_t)((count + per - 1) / per);
    stc<C>(&j->cursor, 1u);  // chunk 0 is the caller's
    // this job's fields, and the graph fields written before it, are complete
    // before ready shows
    drain();
    __hip_atomic_store(&j->ready, nchunks, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return (uint64_t)idx + 1;
}

// Whole wave, after a YES at bound G->k with G->L levels in the arena: follow
// the vertex that created each state and the index of the state it came from
// (both stored per state) back to the empty set, then the k+1 vertices never
// eliminated, ascending.  Each step is checked: the predecessor must be the
// state minus that vertex (else the host's width check rejects the order).
template <bool C>
__device__ void capture_order(BatchGraph *G, int lane)
{
    const int L = (int)first_lane32((uint32_t)ldc<C>(&G->L));
    const int n = G->n;
    const uint64_t cap = G->arena_cap;
    uint64_t at = L > 0 ? read_lane64(ldc<C>(&G->level_off[L]), 0) : 0ull;
    const uint64_t SL = L > 0 && at < cap ? read_lane64(ldc<C>(&G->keys[at]), 0) : 0ull;
    uint64_t S = SL;
    for (int i = L; i >= 1 && at < cap; --i) {
        const int v = (int)first_lane32(ldc<C>(&G->lastv[at]));
        if (lane == 0)
            stc<C>(&G->order[i - 1], (int32_t)v);
        S &= ~(1ull << v);
        if (i == 1)
            break;
        at = read_lane64(ldc<C>(&G->level_off[i - 1]), 0) + (uint64_t)first_lane32(ldc<C>(&G->parent[at]));
        if (at >= cap || read_lane64(ldc<C>(&G->keys[at]), 0) != S)
            break;
    }
    if (lane == 0) {
        int t = L;
        for (int v = 0; v < n && t < 64; ++v)
            if (!((SL >> v) & 1ull))
                stc<C>(&G->order[t++], (int32_t)v);
    }
}

template <bool C>
__device__ void graph_done(const BatchArgs &a, BatchGraph *G, uint32_t status, int lane)
{
    if (lane == 0) {
        stc<C>(&G->status, status);
        if (C)
            drain();  // the graph's fields are complete before it stops counting as active
        atomicSub(&a.q->active, 1u);
    }
}

// Restart graph G at level 0 of bound k (lane 0 writes, then publishes the job).
// Whole wave: lane j's row of the adjacency bound k expands with.
template <bool C>
__device__ void set_bound_rows(BatchGraph *G, int k, int lane)
{
    const int n = G->n;
    const uint8_t *paths = G->paths;
    if (!paths || lane >= n)
        return;
    // edges of G_k+: pairs joined by more than k disjoint paths (§3.1)
    uint64_t row = G->adj[lane];
    const uint8_t *cnt = paths + lane * 64;
    for (int u = 0; u < n; ++u)
        if ((int)cnt[u] > k)
            row |= 1ull << u;
    stc<C>(&G->adjk[lane], row);
}

template <bool C>
__device__ uint64_t start_bound(const BatchArgs &a, BatchGraph *G, int g, int k, int lane)
{
    set_bound_rows<C>(G, k, lane);
    uint64_t pushed = 0;
    if (lane == 0) {
        const uint32_t tag = ldc<C>(&G->tag) + 1u;
        stc<C>(&G->k, (int32_t)k);
        stc<C>(&G->decisions, ldc<C>(&G->decisions) + 1u);
        stc<C>(&G->L, (int32_t)(G->n - k - 1));
        stc<C>(&G->level, 0);
        stc<C>(&G->tag, tag);
        stc<C>(&G->out_count, 0ull);
        stc<C>(&G->peak_k, 1ull);
        stc<C>(&G->level_off[0], (uint64_t)0);
        stc<C>(&G->level_off[1], (uint64_t)1);  // level 0 is the empty set (never read from the arena)
        // the job is published after every lane's row (the drain waits for the whole wave)
        pushed = push_job<C>(a, g, 0, 0, 1, k, tag, 1);
    }
    return read_lane64(pushed, 0);
}

// Whole wave, after every chunk of (g, level) has finished.  Advances the
// graph's search: a NO raises the lower side, a YES (with its order captured)
// lowers the upper side; the graph is done when they meet.  The starting
// bound may be the minor-min-width bound (ascending search) or a prediction
// (the search then moves down after a YES and up after a NO).
// Returns the index + 1 of the job it published with its first chunk kept
// (persistent launch), else 0.
template <bool C>
__device__ uint64_t finish_level(const BatchArgs &a, int g, int level, uint64_t in_count, int lane)
{
    BatchGraph *G = &a.graphs[g];
    // the fields the whole wave needs, loaded back to back (one memory round
    // trip in the persistent launch, where each is a device-scope load)
    const uint64_t cnt = read_lane64(ld_relaxed(&G->out_count), 0);
    const uint32_t ovf = first_lane32(ld_relaxed(&G->overflow));
    const int k = (int)first_lane32((uint32_t)ldc<C>(&G->k));
    const uint32_t tag = first_lane32(ldc<C>(&G->tag));
    const int known = (int)first_lane32((uint32_t)ldc<C>(&G->known_no));
    const int best = (int)first_lane32((uint32_t)ldc<C>(&G->best_yes));
    const int L = (int)first_lane32((uint32_t)ldc<C>(&G->L));
    const int next = level + 1;
    const uint64_t next_off = read_lane64(ldc<C>(&G->level_off[next]), 0);
    const int n = G->n;
    if (lane == 0) {
        // counters the host reads after the launch (and peak_k, which this
        // wave reads back at a YES): atomics that return nothing, so no wait
        atomicAdd(&G->states, (unsigned long long)in_count);
        atomicAdd(&G->expansions, (unsigned long long)(in_count * (uint64_t)(n - level)));
        atomicAdd(&G->levels_run, 1u);
        atomicAdd(&G->unique, (unsigned long long)cnt);
        atomicMax(&G->peak, (unsigned long long)cnt);
        atomicMax(&G->peak_k, (unsigned long long)cnt);
        if (G->trace) {
            // record level+1 of bound k, then start the next level's digests
            // (every chunk of the level is done and no job of its next level
            // is published yet, so nothing else touches them now)
            const uint32_t len = atomicAdd(&G->trace_len, 1u);
            const unsigned long long dsum = atomicExch(&G->digest_sum, 0ull);
            const unsigned long long dxor = atomicExch(&G->digest_xor, 0ull);
            const unsigned long long succ = ldc<C>(&G->successors);
            const unsigned long long mark = ldc<C>(&G->succ_mark);
            if (len < G->trace_cap) {
                BatchTraceRec *r = &G->trace[len];
                stc<C>(&r->k, (int32_t)k);
                stc<C>(&r->level, (int32_t)next);
                stc<C>(&r->count, cnt);
                stc<C>(&r->successors, (uint64_t)(succ - mark));
                stc<C>(&r->digest_sum, (uint64_t)dsum);
                stc<C>(&r->digest_xor, (uint64_t)dxor);
            }
            stc<C>(&G->succ_mark, succ);
        }
    }
    if (ovf || tag >= 0xFFFEu || next == G->fault_level) {
        graph_done<C>(a, G, kBatchFallback, lane);
        return 0;
    }
    if (cnt == 0) {
        // NO at bound k
        const int known_no = k > known ? k : known;
        if (lane == 0)
            stc<C>(&G->known_no, (int32_t)known_no);
        if (best <= known_no + 1) {
            if (lane == 0)
                stc<C>(&G->tw, (int32_t)best);
            graph_done<C>(a, G, kBatchDone, lane);
            return 0;
        }
        return start_bound<C>(a, G, g, known_no + 1, lane);
    }
    if (lane == 0)
        stc<C>(&G->level_off[next + 1], next_off + cnt);
    if (next < L) {
        uint64_t pushed = 0;
        if (lane == 0) {
            stc<C>(&G->level, (int32_t)next);
            stc<C>(&G->tag, tag + 1u);
            stc<C>(&G->out_count, 0ull);
            pushed = push_job<C>(a, g, next, next_off, cnt, k, tag + 1u, next_off + cnt);
        }
        return read_lane64(pushed, 0);
    }
    // YES at bound k: keep its order, then certify or move down
    if (lane == 0)
        stc<C>(&G->level, (int32_t)next);
    capture_order<C>(G, lane);
    if (lane == 0) {
        stc<C>(&G->best_yes, (int32_t)k);
        stc<C>(&G->peak_yes, ldc<C>(&G->peak_k));  // stored by this lane above
    }
    if (k - 1 <= known) {
        if (lane == 0)
            stc<C>(&G->tw, (int32_t)k);
        graph_done<C>(a, G, kBatchDone, lane);
        return 0;
    }
    return start_bound<C>(a, G, g, k - 1, lane);
}

// States [lo, hi) of level `level` of graph g (the level starts at arena
// offset `begin`): expand every state, insert feasible successors into the
// graph's tagged table, append the new ones to its next level.  Whole wave.
template <bool C>
__device__ void process_chunk(const BatchArgs &a, int g, int level, uint64_t begin, uint64_t lo, uint64_t hi,
                              int k, uint32_t tag32, uint64_t out_base, int lane, uint64_t *stage_key,
                              uint8_t *stage_v, uint32_t *stage_p)
{
    BatchGraph *G = &a.graphs[g];
    const int n = (int)first_lane32((uint32_t)G->n);
    const uint64_t tag = (uint64_t)tag32 << kBatchKeyBits;
    const uint64_t tslots = read_lane64(G->table_slots, 0);
    const uint64_t arena_cap = read_lane64(G->arena_cap, 0);
    const uint64_t max_fill = (uint64_t)((double)tslots * a.max_load);
    // reads stay inside the arena whatever the level fields hold
    if (begin > arena_cap)
        return;
    if (hi > arena_cap - begin)
        hi = arena_cap - begin;
    uint64_t *keys = G->keys;
    uint8_t *lastv = G->lastv;
    uint32_t *parent = G->parent;
    uint64_t *table = G->table;
    const uint64_t Aj = lane < n ? ldc<C>(&G->adjk[lane]) : 0ull;
    const bool lane_allowed = ((G->allowed >> lane) & 1ull) != 0ull;
    const uint64_t lanebit = 1ull << lane;
    const bool tracing = G->trace != nullptr;

    uint32_t staged = 0;
    uint64_t feasible = 0;
    bool overflow = false;
    auto flush = [&]() {
        if (staged == 0)
            return;
        wave_lds_sync();
        uint64_t base = 0;
        if (lane == 0)
            base = atomicAdd(&G->out_count, (unsigned long long)staged);
        base = read_lane64(base, 0);
        if (base + staged > max_fill || out_base + base + staged > arena_cap) {
            overflow = true;
        } else {
            for (uint32_t q = (uint32_t)lane; q < staged; q += 64) {
                stc<C>(&keys[out_base + base + q], stage_key[q]);
                stc<C>(&lastv[out_base + base + q], stage_v[q]);
                stc<C>(&parent[out_base + base + q], stage_p[q]);
            }
        }
        wave_lds_sync();
        staged = 0;
    };

    for (uint64_t chunk = lo; chunk < hi && !overflow; chunk += 64) {
        const uint64_t idx = chunk + (uint64_t)lane;
        const uint64_t mine = (idx < hi && level > 0) ? ldc<C>(&keys[begin + idx]) : 0ull;
        const int cnt = hi - chunk < 64 ? (int)(hi - chunk) : 64;
        for (int s = 0; s < cnt; ++s) {
            const uint64_t S = read_lane64(mine, s);
            const bool feas = lane_feasible(S, Aj, lane, n, k) && lane_allowed;
            const uint64_t fmask = ballot(feas);
            feasible += (uint64_t)__popcll(fmask);
            if (fmask == 0)
                continue;
            const uint64_t key = S | lanebit;
            bool won = false;
            if (feas) {
                const uint64_t want = tag | key;
                uint64_t slot = slot_in(key, tslots);
                uint64_t cur = ld_relaxed(&table[slot]);
                for (uint32_t p = 0;;) {
                    if ((cur & ~kKeyMask) == tag) {
                        if (cur == want)
                            break;  // already claimed this level
                        if (++p > a.max_probe) {
                            overflow = true;
                            break;
                        }
                        slot = slot + 1 == tslots ? 0 : slot + 1;
                        cur = ld_relaxed(&table[slot]);
                        continue;
                    }
                    // stale slot (older tag or never used): claim it
                    const uint64_t prev = (uint64_t)atomicCAS((unsigned long long *)&table[slot],
                                                              (unsigned long long)cur,
                                                              (unsigned long long)want);
                    if (prev == cur) {
                        won = true;
                        break;
                    }
                    cur = prev;
                }
            }
            if (tracing && won) {
                atomicAdd(&G->digest_sum, (unsigned long long)splitmix64_out(key));
                atomicXor(&G->digest_xor, (unsigned long long)fmix64(key));
            }
            overflow = ballot(overflow) != 0ull;
            const uint64_t winners = ballot(won);
            const uint32_t nw = (uint32_t)__popcll(winners);
            if (nw == 0)
                continue;
            if (staged + nw > (uint32_t)kBatchStage)
                flush();
            if (won) {
                const uint32_t pos = staged + (uint32_t)lanes_below(winners);
                stage_key[pos] = key;
                stage_v[pos] = (uint8_t)lane;
                stage_p[pos] = (uint32_t)(chunk + (uint64_t)s);
            }
            staged += nw;
        }
    }
    if (!overflow)
        flush();
    if (lane == 0) {
        if (overflow)
            atomicOr(&G->overflow, 1u);
        if (feasible)
            atomicAdd(&G->successors, (unsigned long long)feasible);
    }
}

// Jobs from the queue's head that a wave looks at for a chunk.  Waves start
// at different offsets, so a level of a few chunks is not contended by every
// idle wave of the grid, and an exhausted job is skipped after one load
// rather than one atomic per wave.  A wave that found nothing looks again
// only once the head or the tail has moved (a job's chunks, once all handed
// out, stay so), or when a job it saw was not yet published; meanwhile its
// polls read two words, so idle waves take little from the memory system
// the working ones probe.
constexpr uint32_t kJobWindow = 64;

__global__ __launch_bounds__(kBatchBlock) void batch_kernel(BatchArgs a)
{
    __shared__ uint64_t stage_key[kBatchWaves][kBatchStage];
    __shared__ uint32_t stage_p[kBatchWaves][kBatchStage];
    __shared__ uint8_t stage_v[kBatchWaves][kBatchStage];
    const int lane = (int)(threadIdx.x & 63);
    const int wv = (int)(threadIdx.x >> 6);
    const uint32_t gw = blockIdx.x * kBatchWaves + (uint32_t)wv;
    uint32_t spins = 0;
    uint64_t seen_h = ~0ull, seen_t = ~0ull;
    uint64_t kept = 0;  // job whose first chunk this wave kept when it published it (index + 1)

    for (;;) {
        BatchJob *J = nullptr;
        uint32_t c = 0, nchunks = 0;
        if (kept) {
            J = &a.jobs[kept - 1];
            nchunks = first_lane32(ld_relaxed(&J->ready));
            kept = 0;
        } else {
            const uint64_t h = read_lane64(ld_relaxed(&a.q->head), 0);
            uint64_t t = read_lane64(ld_relaxed(&a.q->tail), 0);
            if (t > a.q->capacity)
                t = a.q->capacity;
            if (h != seen_h || t != seen_t) {
                const uint32_t span = t > h ? (uint32_t)(t - h < kJobWindow ? t - h : kJobWindow) : 0u;
                bool unpublished = false;
                for (uint32_t q = 0; q < span; ++q) {
                    const uint64_t jid = h + (gw + q) % span;
                    BatchJob *cand = &a.jobs[jid];
                    const uint32_t nc = first_lane32(ld_relaxed(&cand->ready));  // chunks, once published
                    if (nc == 0) {
                        unpublished = true;
                        continue;
                    }
                    // the job's fields are read only after it was seen published
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                    if (first_lane32(ld_relaxed(&cand->cursor)) < nc) {
                        uint32_t got = 0;
                        if (lane == 0)
                            got = atomicAdd(&cand->cursor, 1u);
                        got = (uint32_t)__builtin_amdgcn_readlane((int)got, 0);
                        if (got < nc) {
                            J = cand;
                            c = got;
                            nchunks = nc;
                            break;
                        }
                    }
                    // every chunk handed out: the head moves past it
                    if (jid == h && lane == 0)
                        atomicCAS(&a.q->head, (unsigned long long)h, (unsigned long long)(h + 1));
                }
                if (!J && !unpublished) {
                    seen_h = h;
                    seen_t = t;
                }
            }
        }
        if (!J) {
            // the exit words on every eighth idle poll (they sit on a line of their own)
            if ((spins & 7u) == 0u &&
                (first_lane32(ld_relaxed(&a.q->abort)) || first_lane32(ld_relaxed(&a.q->active)) == 0))
                break;
            if (++spins > a.spin_limit) {
                if (lane == 0)
                    atomicOr(&a.q->abort, 1u);
                break;
            }
            // back off while there is no work: about 0.05, 0.9 and 3.4 us per poll
            if (spins < 16)
                __builtin_amdgcn_s_sleep(2);
            else if (spins < 256)
                __builtin_amdgcn_s_sleep(32);
            else
                __builtin_amdgcn_s_sleep(127);
            continue;
        }
        spins = 0;
        const int g = (int)first_lane32((uint32_t)ldc<true>(&J->graph));
        const int level = (int)first_lane32((uint32_t)ldc<true>(&J->level));
        const uint64_t begin = read_lane64(ldc<true>(&J->begin), 0);
        const uint64_t count = read_lane64(ldc<true>(&J->count), 0);
        const uint64_t out_base = read_lane64(ldc<true>(&J->out_base), 0);
        const int k = (int)first_lane32((uint32_t)ldc<true>(&J->k));
        const uint32_t tag = first_lane32(ldc<true>(&J->tag));
        if ((uint32_t)g >= a.nb || level < 0 || level > 63) {
            if (lane == 0)
                atomicOr(&a.q->abort, 1u);  // a job that names no graph: stop, the host reports it
            break;
        }
        const uint64_t per = (uint64_t)first_lane32(ldc<true>(&J->chunk));
        const uint64_t lo = (uint64_t)c * per;
        const uint64_t hi = lo + per < count ? lo + per : count;
        process_chunk<true>(a, g, level, begin, lo, hi, k, tag, out_base, lane, stage_key[wv], stage_v[wv],
                            stage_p[wv]);
        drain();  // this chunk's states and counters are complete before it counts as done
        uint32_t d = 0;
        if (lane == 0)
            d = atomicAdd(&J->done, 1u) + 1;
        d = (uint32_t)__builtin_amdgcn_readlane((int)d, 0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (d == nchunks)
            kept = finish_level<true>(a, g, level, count, lane);
    }
}

// ---------------------------------------------------------------------------
// Level rounds.  One launch expands the current level of every running graph,
// its chunks laid out by a prefix sum over the graphs; a second launch
// advances every graph that ran a level (next level, next bound, or done).
// The kernel boundaries order the levels, so no wave waits on another and
// every access is a plain one; the price is a launch pair and a small plan
// launch per round, which the persistent queue does without.
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t level_count(const BatchArgs &a, uint32_t g)
{
    const BatchGraph *G = &a.graphs[g];
    if (G->status != kBatchRunning)
        return 0;
    return G->level_off[G->level + 1] - G->level_off[G->level];
}

// One workgroup: this round's states per task (about two tasks per wave,
// 64..1024, a multiple of 64) and the first task of every graph.
__global__ __launch_bounds__(1024) void plan_kernel(BatchArgs a, uint32_t B, uint32_t *task_start, uint32_t nwaves)
{
    __shared__ unsigned long long part[1024];
    __shared__ uint32_t scan[1024];
    const uint32_t t = threadIdx.x;
    unsigned long long sum = 0;
    for (uint32_t g = t; g < B; g += 1024)
        sum += level_count(a, g);
    part[t] = sum;
    __syncthreads();
    for (uint32_t off = 512; off; off >>= 1) {
        if (t < off)
            part[t] += part[t + off];
        __syncthreads();
    }
    const unsigned long long total = part[0];
    uint64_t c = (total + 2ull * nwaves - 1) / (2ull * nwaves);
    c = (c + 63) / 64 * 64;
    c = c < 64 ? 64 : (c > 1024 ? 1024 : c);
    uint32_t carry = 0;
    for (uint32_t base = 0; base < B; base += 1024) {
        const uint32_t g = base + t;
        const uint32_t cnt = g < B ? (uint32_t)((level_count(a, g) + c - 1) / c) : 0u;
        scan[t] = cnt;
        __syncthreads();
        for (uint32_t off = 1; off < 1024; off <<= 1) {
            const uint32_t v = t >= off ? scan[t - off] : 0u;
            __syncthreads();
            scan[t] += v;
            __syncthreads();
        }
        if (g < B)
            task_start[g] = carry + scan[t] - cnt;
        carry += scan[1023];
        __syncthreads();
    }
    if (t == 0) {
        task_start[B] = carry;
        a.q->head = c;  // the queue's head word carries the round's task size
    }
}

__global__ __launch_bounds__(kBatchBlock) void round_kernel(BatchArgs a, uint32_t B, const uint32_t *task_start)
{
    __shared__ uint64_t stage_key[kBatchWaves][kBatchStage];
    __shared__ uint32_t stage_p[kBatchWaves][kBatchStage];
    __shared__ uint8_t stage_v[kBatchWaves][kBatchStage];
    const int lane = (int)(threadIdx.x & 63);
    const int wv = (int)(threadIdx.x >> 6);
    const uint32_t total = task_start[B];
    const uint64_t c = a.q->head;
    const uint32_t nw = gridDim.x * kBatchWaves;
    for (uint32_t t = blockIdx.x * kBatchWaves + wv; t < total; t += nw) {
        // graph of task t: the last g with task_start[g] <= t
        uint32_t lo = 0, hi = B;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (task_start[mid] <= t)
                lo = mid;
            else
                hi = mid;
        }
        const BatchGraph *G = &a.graphs[lo];
        const int level = (int)first_lane32((uint32_t)G->level);
        const uint64_t begin = read_lane64(G->level_off[level], 0);
        const uint64_t count = read_lane64(G->level_off[level + 1], 0) - begin;
        const uint64_t first = (uint64_t)(t - task_start[lo]) * c;
        const uint64_t last = first + c < count ? first + c : count;
        const int k = (int)first_lane32((uint32_t)G->k);
        const uint32_t tag = first_lane32(G->tag);
        const uint64_t out_base = read_lane64(G->level_off[level + 1], 0);
        process_chunk<false>(a, (int)lo, level, begin, first, last, k, tag, out_base, lane, stage_key[wv],
                             stage_v[wv], stage_p[wv]);
    }
}

// One wave per graph: close the level it ran this round.
__global__ __launch_bounds__(kBatchBlock) void advance_kernel(BatchArgs a, uint32_t B)
{
    const int lane = (int)(threadIdx.x & 63);
    const uint32_t g = blockIdx.x * kBatchWaves + (threadIdx.x >> 6);
    if (g >= B)
        return;
    const BatchGraph *G = &a.graphs[g];
    if (first_lane32(G->status) != kBatchRunning)
        return;
    const int level = (int)first_lane32((uint32_t)G->level);
    const uint64_t count = read_lane64(G->level_off[level + 1], 0) - read_lane64(G->level_off[level], 0);
    finish_level<false>(a, (int)g, level, count, lane);
}

}  // namespace

hipError_t launch_batch_round(const BatchArgs &a, uint32_t B, uint32_t *task_start, unsigned grid_blocks,
                              hipStream_t s)
{
    hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(1024), 0, s, a, B, task_start,
                       (uint32_t)(grid_blocks * kBatchWaves));
    hipLaunchKernelGGL(round_kernel, dim3(grid_blocks), dim3(kBatchBlock), 0, s, a, B,
                       (const uint32_t *)task_start);
    hipLaunchKernelGGL(advance_kernel, dim3((B + kBatchWaves - 1) / kBatchWaves), dim3(kBatchBlock), 0, s, a, B);
    return hipGetLastError();
}

int batch_blocks_per_cu()
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batch_kernel, kBatchBlock, 0) != hipSuccess ||
        blocks < 1)
        blocks = 1;
    return blocks;
}

hipError_t launch_batch(const BatchArgs &a, unsigned grid_blocks, hipStream_t s)
{
    hipLaunchKernelGGL(batch_kernel, dim3(grid_blocks), dim3(kBatchBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace twk
