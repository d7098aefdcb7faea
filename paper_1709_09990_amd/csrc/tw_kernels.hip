// gfx950 kernels of the level-synchronous treewidth search (§3.1, Listing 1)
// with exact duplicate removal (§3.2 replaced by an exact hash table).
//
// One wavefront expands one state S at a time.  Lane j holds adjacency row j,
// so one ballot over "lane j is in S and touches the current set" is one
// breadth-first step inside G[S].  For each component K of G[S] a second
// ballot gives N_out(K), the vertices outside S adjacent to K.  For v outside
// S, Q(S,v) (§2) is N(v) minus S together with N_out(K) for every component K
// that v touches, minus v itself; v is feasible iff |Q(S,v)| <= k.  Feasible
// successors S + {v} are inserted into an open-addressing table by atomic
// compare-and-swap; the lane that claims an empty slot owns the new state,
// stages it in LDS and the wave appends its staged winners to the next level
// with one atomic per batch (stream compaction).  The Bloom-filter variant of
// §3.2 replaces the table insert with 17 double-hashed bit probes.
#include "tw_internal.h"
#include "tw_wave.h"

namespace twk {
namespace {

constexpr int kStage = 384;  // winners a wave stages in LDS before appending (8 blocks fit a CU)

__device__ __forceinline__ uint64_t rotl64(uint64_t x, int r)
{
    return (x << r) | (x >> (64 - r));
}

__device__ __forceinline__ uint64_t murmur_fmix64(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

// MurmurHash3_x64_128 (Appleby, public domain description) of one 8-byte
// little-endian key with seed 0: a key shorter than a 16-byte block goes
// through the tail step only.  Returns the two 64-bit halves.
__device__ __forceinline__ void murmur3_x64_128_u64(uint64_t key, uint64_t &h1, uint64_t &h2)
{
    const uint64_t c1 = 0x87c37b91114253d5ull, c2 = 0x4cf5ad432745937full;
    h1 = 0;
    h2 = 0;
    uint64_t k1 = key;
    k1 *= c1;
    k1 = rotl64(k1, 31);
    k1 *= c2;
    h1 ^= k1;
    h1 ^= 8ull;
    h2 ^= 8ull;
    h1 += h2;
    h2 += h1;
    h1 = murmur_fmix64(h1);
    h2 = murmur_fmix64(h2);
    h1 += h2;
    h2 += h1;
}

// Bloom insert (§3.2): positions H_i = h1 + i*h2 (i = 1..17) mod m.  A bit
// already seen set is never cleared within a level, so a plain load that reads
// 1 is final; only bits read as 0 are set with an atomic OR.  The state is new
// iff some OR found its bit clear.
__device__ __forceinline__ bool bloom_insert(uint32_t *bits, uint64_t mask, uint64_t key)
{
    uint64_t h1, h2;
    murmur3_x64_128_u64(key, h1, h2);
    bool fresh = false;
#pragma unroll
    for (int i = 1; i <= kBloomProbes; ++i) {
        const uint64_t pos = (h1 + (uint64_t)i * h2) & mask;
        uint32_t *w = bits + (pos >> 5);
        const uint32_t b = 1u << (pos & 31);
        const uint32_t seen = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!(seen & b)) {
            const uint32_t old = atomicOr(w, b);
            if (!(old & b))
                fresh = true;
        }
    }
    return fresh;
}

template <typename K>
__device__ __forceinline__ K cas(K *p, K expected, K desired);

template <>
__device__ __forceinline__ uint32_t cas<uint32_t>(uint32_t *p, uint32_t e, uint32_t d)
{
    return atomicCAS(p, e, d);
}

template <>
__device__ __forceinline__ uint64_t cas<uint64_t>(uint64_t *p, uint64_t e, uint64_t d)
{
    return (uint64_t)atomicCAS((unsigned long long *)p, (unsigned long long)e,
                               (unsigned long long)d);
}

// Inserts `key` into the exact table; true iff this call stored it.
// read_first: linear probing over 16-byte buckets of W = 16 / sizeof(K) slots,
// each read with one load.  Within a level a slot only goes from EMPTY to a
// key, so a key seen in the copy is final; an EMPTY in the copy may be stale
// and is claimed with a CAS, whose returned value replaces it in the copy.
// Slots are taken in bucket order, so a key is never placed after a slot that
// was EMPTY.  Otherwise: one CAS per slot, slot by slot.
template <typename K>
__device__ __forceinline__ bool table_insert(const LevelArgs &a, K *table, K key)
{
    const K EMPTY = (K)~(K)0;
    bool won = false;
    if (a.read_first) {
        constexpr int W = 16 / (int)sizeof(K);
        using Vec = unsigned __attribute__((ext_vector_type(4)));
        const uint64_t nb = a.table_slots / W;
        uint64_t b = __umul64hi(slot_hash((uint64_t)key), nb);
        for (uint32_t p = 0;; ++p) {
            const Vec raw = *(const Vec *)(table + b * W);
            K slot[W];
            __builtin_memcpy(slot, &raw, 16);
            bool done = false;
#pragma unroll
            for (int j = 0; j < W; ++j) {
                if (!done && slot[j] == EMPTY) {
                    const K old = cas<K>(&table[b * W + j], EMPTY, key);
                    won = old == EMPTY;
                    slot[j] = won ? key : old;
                }
                done |= slot[j] == key;
            }
            if (done)
                break;
            if (p >= a.max_probe) {
                atomicOr(&a.ctr->overflow, 1u);
                break;
            }
            b = b + 1 == nb ? 0 : b + 1;
        }
    } else {
        uint64_t h = slot_in((uint64_t)key, a.table_slots);
        for (uint32_t p = 0;; ++p) {
            const K old = cas<K>(&table[h], EMPTY, key);
            if (old == EMPTY) {
                won = true;
                break;
            }
            if (old == key)
                break;
            if (p >= a.max_probe) {
                atomicOr(&a.ctr->overflow, 1u);
                break;
            }
            h = h + 1 == a.table_slots ? 0 : h + 1;
        }
    }
    return won;
}

// Expansion of one level.  Each wave walks chunks of 64 input states; per
// state it finds the feasible lanes and appends their successors to a
// per-wave LDS queue.  Whenever 64 are queued the wave inserts them with all
// 64 lanes at once, so the probes of a wave run at full width and one memory
// round trip serves 64 successors rather than the few of one state.
template <typename K, bool kBloom>
__device__ __forceinline__ void expand_level(const LevelArgs &a)
{
    constexpr uint32_t kQueue = 128;  // ring of pending successors per wave
    __shared__ K stage_key[kWavesPerBlock][kStage];
    __shared__ uint8_t stage_v[kWavesPerBlock][kStage];
    __shared__ K queue_key[kWavesPerBlock][kQueue];
    __shared__ uint8_t queue_v[kWavesPerBlock][kQueue];

    const int lane = (int)(threadIdx.x & 63);
    const int wv = (int)(threadIdx.x >> 6);
    const K *in = (const K *)a.in;
    K *out = (K *)a.out;
    K *table = (K *)a.table;
    const uint64_t Aj = lane < a.n ? a.adj[lane] : 0ull;
    const bool lane_allowed = ((a.allowed >> lane) & 1ull) != 0ull;

    const uint64_t wave_id = (uint64_t)blockIdx.x * kWavesPerBlock + wv;
    const uint64_t n_waves = (uint64_t)gridDim.x * kWavesPerBlock;

    uint32_t staged = 0;       // wave-uniform
    uint32_t qhead = 0;        // wave-uniform ring position of the oldest queued successor
    uint32_t qcount = 0;       // wave-uniform
    uint64_t feasible = 0;     // wave-uniform count of feasible pairs

    // Append the staged winners to the next level (one atomic per batch).
    auto flush = [&]() {
        if (staged == 0)
            return;
        wave_lds_sync();
        uint64_t base = 0;
        if (lane == 0)
            base = atomicAdd(&a.ctr->out_count, (unsigned long long)staged);
        base = read_lane64(base, 0);
        if (base + staged > a.out_cap) {
            if (lane == 0)
                atomicOr(&a.ctr->overflow, 1u);
        } else {
            for (uint32_t t = (uint32_t)lane; t < staged; t += 64) {
                out[base + t] = stage_key[wv][t];
                a.out_lastv[base + t] = stage_v[wv][t];
            }
        }
        wave_lds_sync();
        staged = 0;
    };

    // Insert the m (<= 64) oldest queued successors, one per lane.
    auto drain = [&](uint32_t m) {
        wave_lds_sync();
        const bool have = (uint32_t)lane < m;
        K key = 0;
        uint8_t v = 0;
        if (have) {
            const uint32_t at = (qhead + (uint32_t)lane) & (kQueue - 1);
            key = queue_key[wv][at];
            v = queue_v[wv][at];
        }
        wave_lds_sync();
        qhead = (qhead + m) & (kQueue - 1);
        qcount -= m;
        bool won = false;
        if (have) {
            if (kBloom)
                won = bloom_insert(a.bloom, a.bloom_mask, (uint64_t)key);
            else
                won = table_insert<K>(a, table, key);
        }
        const uint64_t winners = ballot(won);
        const uint32_t nw = (uint32_t)__popcll(winners);
        if (nw == 0)
            return;
        if (staged + nw > (uint32_t)kStage)
            flush();
        if (won) {
            const uint32_t pos = staged + (uint32_t)lanes_below(winners);
            stage_key[wv][pos] = key;
            stage_v[wv][pos] = v;
        }
        staged += nw;
    };

    for (uint64_t chunk = wave_id * 64; chunk < a.in_count; chunk += n_waves * 64) {
        unsigned int ovf = __hip_atomic_load(&a.ctr->overflow, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        if (__builtin_amdgcn_readfirstlane(ovf))
            break;
        const uint64_t idx = chunk + (uint64_t)lane;
        const uint64_t mine = idx < a.in_count ? (uint64_t)in[idx] : 0ull;
        const uint64_t left = a.in_count - chunk;
        const int cnt = left < 64 ? (int)left : 64;

        for (int s = 0; s < cnt; ++s) {
            const uint64_t S = read_lane64(mine, s);
            const bool feas = lane_feasible(S, Aj, lane, a.n, a.k) && lane_allowed;
            const uint64_t feas_mask = ballot(feas);
            const uint32_t nf = (uint32_t)__popcll(feas_mask);
            feasible += nf;
            if (nf == 0)
                continue;
            // qcount < 64 here and nf <= 64, so the ring of 128 never overruns
            if (feas) {
                const uint32_t at = (qhead + qcount + (uint32_t)lanes_below(feas_mask)) & (kQueue - 1);
                queue_key[wv][at] = (K)(S | (1ull << lane));
                queue_v[wv][at] = (uint8_t)lane;
            }
            qcount += nf;
            if (qcount >= 64)
                drain(64);
        }
    }
    while (qcount)
        drain(qcount < 64 ? qcount : 64);
    flush();
    if (lane == 0 && feasible)
        atomicAdd(&a.ctr->successors, (unsigned long long)feasible);
}

template <typename K, bool kBloom>
__global__ __launch_bounds__(kBlock) void expand_kernel(LevelArgs a)
{
    expand_level<K, kBloom>(a);
}

// ---------------------------------------------------------------------------
// Level loop of one bound as a fixed sequence of launches (captured once in a
// HIP graph and replayed for every bound and graph of the same shape): level
// i reads its size from the counters the launch for level i-1 left in device
// memory, and its bound from the control block, and does nothing when it lies
// beyond L(k), follows an empty level, or follows an overflow.
// ---------------------------------------------------------------------------

// Size of level `level`, or 0 when the level is not run for this bound.
__device__ __forceinline__ uint64_t gated_count(const GateArgs &g)
{
    if (g.level >= g.ctl->L)
        return 0;
    if (g.level == 0)
        return 1;
    const LevelCounters &prev = g.ctr[g.level - 1];
    return prev.overflow ? 0 : prev.out_count;
}

// Clears level `level`'s counters, and its table when the level runs.
__global__ void prep_gated_kernel(GateArgs g, uint4 *table, uint64_t n16)
{
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid == 0) {
        LevelCounters *c = &g.ctr[g.level];
        c->out_count = 0;
        c->successors = 0;
        c->overflow = 0;
        c->pad = 0;
    }
    if (gated_count(g) == 0)
        return;
    const uint4 v = make_uint4(~0u, ~0u, ~0u, ~0u);
    for (uint64_t i = gid; i < n16; i += (uint64_t)gridDim.x * blockDim.x)
        table[i] = v;
}

template <typename K>
__global__ __launch_bounds__(kBlock) void expand_gated_kernel(LevelArgs a, GateArgs g)
{
    const uint64_t cnt = gated_count(g);
    if (cnt == 0)
        return;
    a.in_count = cnt;
    a.k = g.ctl->k;
    a.allowed = g.ctl->allowed;
    expand_level<K, false>(a);
}

// One workgroup: the order of a YES run of the gated loop.  From the first
// state of level L, each step reads the vertex that created the state, takes
// it out, and finds the remaining set in the level below (every thread scans
// a strided share; the lowest index found wins).  Writes order[0..L) and the
// last state; *err = 1 if a predecessor is missing.
template <typename K>
__global__ __launch_bounds__(1024) void backtrack_kernel(BacktrackArgs b)
{
    __shared__ unsigned long long found;
    const K *keys = (const K *)b.keys;
    const int L = b.ctl->L;
    if (L <= 0) {
        if (threadIdx.x == 0)
            *b.last_state = 0;
        return;
    }
    uint64_t idx = 0;
    uint64_t S = (uint64_t)keys[b.off[L]];
    if (threadIdx.x == 0)
        *b.last_state = S;
    for (int i = L; i >= 1; --i) {
        const int v = b.lastv[b.off[i] + idx];
        if (threadIdx.x == 0)
            b.order[i - 1] = v;
        S &= ~(1ull << v);
        if (i == 1)
            break;
        const uint64_t cnt = i - 1 == 0 ? 1 : b.ctr[i - 2].out_count;
        if (threadIdx.x == 0)
            found = ~0ull;
        __syncthreads();
        const K *lv = keys + b.off[i - 1];
        for (uint64_t t = threadIdx.x; t < cnt; t += blockDim.x)
            if ((uint64_t)lv[t] == S)
                atomicMin(&found, (unsigned long long)t);
        __syncthreads();
        idx = found;
        __syncthreads();
        if (idx == ~0ull) {
            if (threadIdx.x == 0)
                *b.err = 1;
            return;
        }
    }
}

// ---------------------------------------------------------------------------
// Partitioned insert for large levels.  The random probes of a single-phase
// insert each pull a whole cache line from HBM when the table is larger than
// the caches.  Phase 1 (scatter_kernel) expands as above but writes each
// feasible (S, v) as one entry into partition p (hash range) of a successor
// buffer, through per-wave LDS buckets flushed 8 entries (64 bytes) at a time.
// Phase 2 (gather_kernel) walks the partitions in order, so at any moment the
// waves probe one table slice small enough to stay in the Infinity Cache.
// ---------------------------------------------------------------------------

constexpr int kBucket = 8;

template <typename K>
__global__ __launch_bounds__(kBlock) void scatter_kernel(LevelArgs a, ScatterArgs sc)
{
    __shared__ uint64_t bucket[kWavesPerBlock][kMaxParts][kBucket];
    __shared__ uint32_t bcount[kWavesPerBlock][kMaxParts];
    const int lane = (int)(threadIdx.x & 63);
    const int wv = (int)(threadIdx.x >> 6);
    const K *in = (const K *)a.in;
    const uint64_t lanebit = 1ull << lane;
    const uint64_t Aj = lane < a.n ? a.adj[lane] : 0ull;
    const uint64_t wave_id = (uint64_t)blockIdx.x * kWavesPerBlock + wv;
    const uint64_t n_waves = (uint64_t)gridDim.x * kWavesPerBlock;
    bcount[wv][lane] = 0;
    wave_lds_sync();

    uint64_t feasible = 0;
    bool overflow = false;  // wave-uniform
    const uint64_t sub = wave_id % kSubRegions;
    auto region = [&](int p) { return (uint64_t)p * kSubRegions + sub; };
    auto flush_bucket = [&](int p, uint32_t cnt) {
        uint64_t base = 0;
        if (lane == 0)
            base = atomicAdd(&sc.sub_count[region(p)], (unsigned long long)cnt);
        base = read_lane64(base, 0);
        if (base + cnt > sc.sub_cap)
            overflow = true;
        else if ((uint32_t)lane < cnt)
            sc.parts[region(p) * sc.sub_cap + base + (uint64_t)lane] = bucket[wv][p][lane];
    };

    for (uint64_t chunk = wave_id * 64; chunk < a.in_count && !overflow; chunk += n_waves * 64) {
        unsigned int ovf = __hip_atomic_load(&a.ctr->overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (__builtin_amdgcn_readfirstlane(ovf))
            break;
        const uint64_t idx = chunk + (uint64_t)lane;
        const uint64_t mine = idx < a.in_count ? (uint64_t)in[idx] : 0ull;
        const uint64_t left = a.in_count - chunk;
        const int cnt = left < 64 ? (int)left : 64;
        for (int s = 0; s < cnt; ++s) {
            const uint64_t S = read_lane64(mine, s);
            const bool feas = lane_feasible(S, Aj, lane, a.n, a.k) && ((a.allowed >> lane) & 1ull);
            const uint64_t fmask = ballot(feas);
            feasible += (uint64_t)__popcll(fmask);
            if (fmask == 0ull)
                continue;
            int p = 0;
            uint32_t pos = kBucket;
            bool lane_ovf = false;
            if (feas) {
                const uint64_t key = S | lanebit;
                const uint64_t entry = key | ((uint64_t)lane << kEntryVShift);
                p = (int)(((slot_hash(key) >> 32) * (uint64_t)sc.P) >> 32);
                pos = atomicAdd(&bcount[wv][p], 1u);
                if (pos < (uint32_t)kBucket) {
                    bucket[wv][p][pos] = entry;
                } else {
                    // bucket filled earlier in this step: write straight through
                    const uint64_t at = atomicAdd(&sc.sub_count[region(p)], 1ull);
                    if (at < sc.sub_cap)
                        sc.parts[region(p) * sc.sub_cap + at] = entry;
                    else
                        lane_ovf = true;
                }
            }
            if (ballot(lane_ovf))
                overflow = true;
            uint64_t full = ballot(feas && pos == (uint32_t)kBucket - 1);
            if (full) {
                wave_lds_sync();
                while (full) {
                    const int l = __builtin_ctzll(full);
                    full &= full - 1;
                    const int pf = __builtin_amdgcn_readlane(p, l);
                    flush_bucket(pf, kBucket);
                    if (lane == 0)
                        bcount[wv][pf] = 0;
                }
                wave_lds_sync();
            }
        }
    }
    wave_lds_sync();
    for (int p = 0; p < sc.P && !overflow; ++p) {
        uint32_t c = first_lane32(bcount[wv][p]);
        c = c > (uint32_t)kBucket ? (uint32_t)kBucket : c;
        if (c)
            flush_bucket(p, c);
    }
    if (lane == 0) {
        if (overflow)
            atomicOr(&a.ctr->overflow, 1u);
        if (feasible)
            atomicAdd(&a.ctr->successors, (unsigned long long)feasible);
    }
}

template <typename K>
__global__ __launch_bounds__(kBlock) void gather_kernel(LevelArgs a, GatherArgs ga)
{
    __shared__ K stage_key[kWavesPerBlock][kStage];
    __shared__ uint8_t stage_v[kWavesPerBlock][kStage];
    const K EMPTY = (K)~(K)0;
    const int lane = (int)(threadIdx.x & 63);
    const int wv = (int)(threadIdx.x >> 6);
    K *out = (K *)a.out;
    K *table = (K *)a.table;
    const uint64_t wave_id = (uint64_t)blockIdx.x * kWavesPerBlock + wv;
    const uint64_t n_waves = (uint64_t)gridDim.x * kWavesPerBlock;
    const uint64_t total = ga.chunk_prefix[(uint64_t)ga.P * kSubRegions];
    const uint64_t vmask = (1ull << kEntryVShift) - 1;
    uint32_t staged = 0;

    auto flush = [&]() {
        if (staged == 0)
            return;
        wave_lds_sync();
        uint64_t base = 0;
        if (lane == 0)
            base = atomicAdd(&a.ctr->out_count, (unsigned long long)staged);
        base = read_lane64(base, 0);
        if (base + staged > a.out_cap) {
            if (lane == 0)
                atomicOr(&a.ctr->overflow, 1u);
        } else {
            for (uint32_t t = (uint32_t)lane; t < staged; t += 64) {
                out[base + t] = stage_key[wv][t];
                a.out_lastv[base + t] = stage_v[wv][t];
            }
        }
        wave_lds_sync();
        staged = 0;
    };

    for (uint64_t c = wave_id; c < total; c += n_waves) {
        unsigned int ovf = __hip_atomic_load(&a.ctr->overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (__builtin_amdgcn_readfirstlane(ovf))
            break;
        // region of chunk c: the last r with chunk_prefix[r] <= c (uniform search)
        int lo = 0, hi = ga.P * kSubRegions;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (ga.chunk_prefix[mid] <= c)
                lo = mid;
            else
                hi = mid;
        }
        const int r = lo;
        const int p = r / kSubRegions;
        const uint64_t off = (c - ga.chunk_prefix[r]) * 64 + (uint64_t)lane;
        const bool valid = off < ga.count[r];
        const uint64_t entry = valid ? ga.parts[(uint64_t)r * ga.sub_cap + off] : 0ull;
        const K key = (K)(entry & vmask);
        const int v = (int)(entry >> kEntryVShift);
        bool won = false;
        if (valid) {
            const uint64_t lo_slot = (uint64_t)p * ga.slice;
            uint64_t h = lo_slot + (((slot_hash((uint64_t)key) & 0xFFFFFFFFull) * ga.slice) >> 32);
            const uint64_t hi_slot = lo_slot + ga.slice;
            for (uint32_t q = 0;; ++q) {
                K old = __hip_atomic_load(&table[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (old == EMPTY) {
                    old = cas<K>(&table[h], EMPTY, key);
                    if (old == EMPTY) {
                        won = true;
                        break;
                    }
                }
                if (old == key)
                    break;
                if (q >= a.max_probe) {
                    atomicOr(&a.ctr->overflow, 1u);
                    break;
                }
                h = h + 1 == hi_slot ? lo_slot : h + 1;
            }
        }
        const uint64_t winners = ballot(won);
        const uint32_t nw = (uint32_t)__popcll(winners);
        if (nw == 0)
            continue;
        if (staged + nw > (uint32_t)kStage)
            flush();
        if (won) {
            const uint32_t pos = staged + (uint32_t)lanes_below(winners);
            stage_key[wv][pos] = key;
            stage_v[wv][pos] = (uint8_t)v;
        }
        staged += nw;
    }
    flush();
}

__global__ void fill_empty_kernel(uint4 *p, uint64_t n16)
{
    const uint4 v = make_uint4(~0u, ~0u, ~0u, ~0u);
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void fill_zero_kernel(uint4 *p, uint64_t n16)
{
    const uint4 v = make_uint4(0u, 0u, 0u, 0u);
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void zero_counters_kernel(LevelCounters *c)
{
    if (threadIdx.x == 0) {
        c->out_count = 0;
        c->successors = 0;
        c->overflow = 0;
        c->pad = 0;
    }
}

template <typename K>
__global__ void find_kernel(const K *keys, uint64_t count, K target, unsigned long long *result)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        if (keys[i] == target)
            atomicMin(result, (unsigned long long)i);
}

unsigned blocks_for(uint64_t items, unsigned per_block, unsigned cap)
{
    uint64_t b = (items + per_block - 1) / per_block;
    if (b < 1)
        b = 1;
    if (b > cap)
        b = cap;
    return (unsigned)b;
}

}  // namespace

hipError_t launch_fill_empty(void *table, uint64_t bytes, hipStream_t s)
{
    const uint64_t n16 = bytes / 16;
    if (n16 == 0)
        return hipSuccess;
    hipLaunchKernelGGL(fill_empty_kernel, dim3(blocks_for(n16, 256, 8192)), dim3(256), 0, s,
                       (uint4 *)table, n16);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void *p, uint64_t bytes, hipStream_t s)
{
    const uint64_t n16 = bytes / 16;
    if (n16 == 0)
        return hipSuccess;
    hipLaunchKernelGGL(fill_zero_kernel, dim3(blocks_for(n16, 256, 8192)), dim3(256), 0, s,
                       (uint4 *)p, n16);
    return hipGetLastError();
}

hipError_t launch_zero_counters(LevelCounters *c, hipStream_t s)
{
    hipLaunchKernelGGL(zero_counters_kernel, dim3(1), dim3(64), 0, s, c);
    return hipGetLastError();
}

hipError_t launch_expand(const LevelArgs &a, unsigned grid_blocks, hipStream_t s)
{
    if (a.in_count == 0)
        return hipSuccess;
    const bool bloom = a.bloom != nullptr;
    if (a.key_bytes == 4) {
        if (bloom)
            hipLaunchKernelGGL((expand_kernel<uint32_t, true>), dim3(grid_blocks), dim3(kBlock), 0, s, a);
        else
            hipLaunchKernelGGL((expand_kernel<uint32_t, false>), dim3(grid_blocks), dim3(kBlock), 0, s, a);
    } else {
        if (bloom)
            hipLaunchKernelGGL((expand_kernel<uint64_t, true>), dim3(grid_blocks), dim3(kBlock), 0, s, a);
        else
            hipLaunchKernelGGL((expand_kernel<uint64_t, false>), dim3(grid_blocks), dim3(kBlock), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_prep_gated(const GateArgs &g, void *table, uint64_t bytes, hipStream_t s)
{
    const uint64_t n16 = bytes / 16;
    hipLaunchKernelGGL(prep_gated_kernel, dim3(blocks_for(n16 ? n16 : 1, 256, 8192)), dim3(256), 0, s, g,
                       (uint4 *)table, n16);
    return hipGetLastError();
}

hipError_t launch_expand_gated(const LevelArgs &a, const GateArgs &g, unsigned grid_blocks, hipStream_t s)
{
    if (a.key_bytes == 4)
        hipLaunchKernelGGL(expand_gated_kernel<uint32_t>, dim3(grid_blocks), dim3(kBlock), 0, s, a, g);
    else
        hipLaunchKernelGGL(expand_gated_kernel<uint64_t>, dim3(grid_blocks), dim3(kBlock), 0, s, a, g);
    return hipGetLastError();
}

hipError_t launch_backtrack(const BacktrackArgs &b, int key_bytes, hipStream_t s)
{
    if (key_bytes == 4)
        hipLaunchKernelGGL(backtrack_kernel<uint32_t>, dim3(1), dim3(1024), 0, s, b);
    else
        hipLaunchKernelGGL(backtrack_kernel<uint64_t>, dim3(1), dim3(1024), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_scatter(const LevelArgs &a, const ScatterArgs &sc, unsigned grid_blocks, hipStream_t s)
{
    if (a.in_count == 0)
        return hipSuccess;
    if (a.key_bytes == 4)
        hipLaunchKernelGGL(scatter_kernel<uint32_t>, dim3(grid_blocks), dim3(kBlock), 0, s, a, sc);
    else
        hipLaunchKernelGGL(scatter_kernel<uint64_t>, dim3(grid_blocks), dim3(kBlock), 0, s, a, sc);
    return hipGetLastError();
}

hipError_t launch_gather(const LevelArgs &a, const GatherArgs &ga, unsigned grid_blocks, hipStream_t s)
{
    if (a.key_bytes == 4)
        hipLaunchKernelGGL(gather_kernel<uint32_t>, dim3(grid_blocks), dim3(kBlock), 0, s, a, ga);
    else
        hipLaunchKernelGGL(gather_kernel<uint64_t>, dim3(grid_blocks), dim3(kBlock), 0, s, a, ga);
    return hipGetLastError();
}

hipError_t launch_find(const void *keys, uint64_t count, uint64_t target, int key_bytes,
                       unsigned long long *result, hipStream_t s)
{
    if (count == 0)
        return hipSuccess;
    const unsigned g = blocks_for(count, 256, 4096);
    if (key_bytes == 4)
        hipLaunchKernelGGL(find_kernel<uint32_t>, dim3(g), dim3(256), 0, s, (const uint32_t *)keys,
                           count, (uint32_t)target, result);
    else
        hipLaunchKernelGGL(find_kernel<uint64_t>, dim3(g), dim3(256), 0, s, (const uint64_t *)keys,
                           count, target, result);
    return hipGetLastError();
}

}  // namespace twk
