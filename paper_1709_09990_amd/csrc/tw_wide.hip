// Level expansion for graphs of up to 126 vertices: states of two 64-bit
// words (vertices 0..63 in the low word, 64..125 in the high word).
//
// The search is the one of Listing 1 (§3.1): every S of level i and every v
// outside S with |Q(S, v)| <= k (§2) gives the successor S + {v}; duplicates
// are removed exactly.  The wave layout widens the 64-vertex kernel's: lane j
// holds the adjacency rows of vertex j and of vertex j + 64, so one breadth-
// first step inside G[S] is two ballots (one per half of the vertex set), and
// each lane decides two candidate vertices per state.
//
// Duplicate removal without a 16-byte compare-and-swap (gfx950's widest is 64
// bits): a table slot is two words, w0 = state bits 0..62 and w1 = bits
// 63..125, each with bit 63 clear; EMPTY is all ones.  A state claims a slot
// with one 64-bit compare-and-swap on w0 and then publishes w1.  A reader that
// finds w0 equal to its own low part and w1 still EMPTY waits (reloading the
// slot at the next step of its probe loop) until w1 appears; the wait is
// bounded, past the bound the level overflows and the host replays it.
#include "tw_internal.h"
#include "tw_wave.h"

namespace twk {
namespace {

constexpr uint64_t kLow63 = (1ull << 63) - 1;
constexpr uint64_t kEmpty = ~0ull;
constexpr uint32_t kWideWait = 1u << 20;  // probe-loop steps a reader may wait for a publication
constexpr int kWideStage = 192;           // winners a wave stages in LDS (17 bytes each)
constexpr uint32_t kWideQueue = 256;      // pending successors per wave (a state adds at most 126)

__device__ __forceinline__ uint64_t ld_agent(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_agent(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Slot of a 126-bit state (w0, w1) in a table of `slots` two-word slots.
__device__ __forceinline__ uint64_t wide_slot(uint64_t w0, uint64_t w1, uint64_t slots)
{
    return __umul64hi(slot_hash(w0 ^ slot_hash(w1 + 0x632BE59BD9B4E019ull)), slots);
}

// Inserts the state (w0, w1) (bit 63 of both clear); true iff this call
// stored it.  Sets *ovf when the probe or wait bound is exceeded.
__device__ __forceinline__ bool wide_insert(uint64_t *table, uint64_t slots, uint64_t w0k, uint64_t w1k,
                                            uint32_t max_probe, bool &ovf)
{
    uint64_t s = wide_slot(w0k, w1k, slots);
    uint32_t probes = 0, waits = 0;
    for (;;) {
        uint64_t *slot = table + 2 * s;
        uint64_t w0 = ld_agent(slot);
        if (w0 == kEmpty) {
            const uint64_t old = (uint64_t)atomicCAS((unsigned long long *)slot, (unsigned long long)kEmpty,
                                                     (unsigned long long)w0k);
            if (old == kEmpty) {
                st_agent(slot + 1, w1k);
                return true;
            }
            w0 = old;
        }
        if (w0 == w0k) {
            const uint64_t w1 = ld_agent(slot + 1);
            if (w1 == kEmpty) {
                // claimed by an equal low part, high part not yet published
                if (++waits > kWideWait) {
                    ovf = true;
                    return false;
                }
                continue;
            }
            if (w1 == w1k)
                return false;
        }
        if (++probes > max_probe) {
            ovf = true;
            return false;
        }
        s = s + 1 == slots ? 0 : s + 1;
    }
}

// |Q(S, v)| <= k for this lane's two vertices, v = lane (rows A) and
// v = lane + 64 (rows B).  Components of G[S] are grown by ballots: bit j of
// the low ballot is "vertex j's row meets the component", of the high ballot
// the same for vertex j + 64.  The vertices outside S adjacent to a component
// join Q of every candidate adjacent to it (§2).
__device__ __forceinline__ void wide_feasible(uint64_t Slo, uint64_t Shi, uint64_t Alo, uint64_t Ahi,
                                              uint64_t Blo, uint64_t Bhi, int lane, int n, int k, bool &fa,
                                              bool &fb)
{
    const uint64_t lb = 1ull << lane;
    uint64_t qa_lo = 0, qa_hi = 0, qb_lo = 0, qb_hi = 0;
    uint64_t rem_lo = Slo, rem_hi = Shi;
    while (rem_lo | rem_hi) {
        uint64_t c_lo = 0, c_hi = 0;
        if (rem_lo)
            c_lo = rem_lo & (~rem_lo + 1ull);
        else
            c_hi = rem_hi & (~rem_hi + 1ull);
        uint64_t t_lo, t_hi;
        for (;;) {
            t_lo = ballot(((Alo & c_lo) | (Ahi & c_hi)) != 0ull);
            t_hi = ballot(((Blo & c_lo) | (Bhi & c_hi)) != 0ull);
            const uint64_t n_lo = c_lo | (t_lo & Slo), n_hi = c_hi | (t_hi & Shi);
            if (n_lo == c_lo && n_hi == c_hi)
                break;
            c_lo = n_lo;
            c_hi = n_hi;
        }
        rem_lo &= ~c_lo;
        rem_hi &= ~c_hi;
        const uint64_t o_lo = t_lo & ~Slo, o_hi = t_hi & ~Shi;
        if (o_lo & lb) {
            qa_lo |= o_lo;
            qa_hi |= o_hi;
        }
        if (o_hi & lb) {
            qb_lo |= o_lo;
            qb_hi |= o_hi;
        }
    }
    const uint64_t QAlo = (Alo | qa_lo) & ~Slo & ~lb, QAhi = (Ahi | qa_hi) & ~Shi;
    const uint64_t QBlo = (Blo | qb_lo) & ~Slo, QBhi = (Bhi | qb_hi) & ~Shi & ~lb;
    fa = lane < n && !((Slo >> lane) & 1ull) && __popcll(QAlo) + __popcll(QAhi) <= k;
    fb = lane + 64 < n && !((Shi >> lane) & 1ull) && __popcll(QBlo) + __popcll(QBhi) <= k;
}

// One level: in/out keys are (lo, hi) pairs; a.adj holds 2n words (row v at
// adj[2v], adj[2v+1]); a.allowed / allowed_hi the vertices that may be added.
__global__ __launch_bounds__(kBlock) void expand_wide_kernel(LevelArgs a, uint64_t allowed_hi)
{
    __shared__ uint64_t stage_lo[kWavesPerBlock][kWideStage];
    __shared__ uint64_t stage_hi[kWavesPerBlock][kWideStage];
    __shared__ uint8_t stage_v[kWavesPerBlock][kWideStage];
    __shared__ uint64_t queue_lo[kWavesPerBlock][kWideQueue];
    __shared__ uint64_t queue_hi[kWavesPerBlock][kWideQueue];
    __shared__ uint8_t queue_v[kWavesPerBlock][kWideQueue];

    const int lane = (int)(threadIdx.x & 63);
    const int wv = (int)(threadIdx.x >> 6);
    const uint64_t *in = (const uint64_t *)a.in;
    uint64_t *out = (uint64_t *)a.out;
    uint64_t *table = (uint64_t *)a.table;
    const int n = a.n;
    const uint64_t Alo = lane < n ? a.adj[2 * lane] : 0ull, Ahi = lane < n ? a.adj[2 * lane + 1] : 0ull;
    const uint64_t Blo = lane + 64 < n ? a.adj[2 * (lane + 64)] : 0ull;
    const uint64_t Bhi = lane + 64 < n ? a.adj[2 * (lane + 64) + 1] : 0ull;
    const bool allow_a = ((a.allowed >> lane) & 1ull) != 0ull;
    const bool allow_b = ((allowed_hi >> lane) & 1ull) != 0ull;

    const uint64_t wave_id = (uint64_t)blockIdx.x * kWavesPerBlock + wv;
    const uint64_t n_waves = (uint64_t)gridDim.x * kWavesPerBlock;
    uint32_t staged = 0, qhead = 0, qcount = 0;
    uint64_t feasible = 0;
    bool ovf = false;

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
                out[2 * (base + t)] = stage_lo[wv][t];
                out[2 * (base + t) + 1] = stage_hi[wv][t];
                a.out_lastv[base + t] = stage_v[wv][t];
            }
        }
        wave_lds_sync();
        staged = 0;
    };

    auto drain = [&](uint32_t m) {
        wave_lds_sync();
        const bool have = (uint32_t)lane < m;
        uint64_t lo = 0, hi = 0;
        uint8_t v = 0;
        if (have) {
            const uint32_t at = (qhead + (uint32_t)lane) & (kWideQueue - 1);
            lo = queue_lo[wv][at];
            hi = queue_hi[wv][at];
            v = queue_v[wv][at];
        }
        wave_lds_sync();
        qhead = (qhead + m) & (kWideQueue - 1);
        qcount -= m;
        bool won = false;
        if (have)
            won = wide_insert(table, a.table_slots, lo & kLow63, (lo >> 63) | (hi << 1), a.max_probe, ovf);
        const uint64_t winners = ballot(won);
        const uint32_t nw = (uint32_t)__popcll(winners);
        if (nw == 0)
            return;
        if (staged + nw > (uint32_t)kWideStage)
            flush();
        if (won) {
            const uint32_t pos = staged + (uint32_t)lanes_below(winners);
            stage_lo[wv][pos] = lo;
            stage_hi[wv][pos] = hi;
            stage_v[wv][pos] = v;
        }
        staged += nw;
    };

    for (uint64_t chunk = wave_id * 64; chunk < a.in_count; chunk += n_waves * 64) {
        const unsigned int o = __hip_atomic_load(&a.ctr->overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (__builtin_amdgcn_readfirstlane(o))
            break;
        const uint64_t idx = chunk + (uint64_t)lane;
        const uint64_t my_lo = idx < a.in_count ? in[2 * idx] : 0ull;
        const uint64_t my_hi = idx < a.in_count ? in[2 * idx + 1] : 0ull;
        const uint64_t left = a.in_count - chunk;
        const int cnt = left < 64 ? (int)left : 64;
        for (int s = 0; s < cnt; ++s) {
            const uint64_t Slo = read_lane64(my_lo, s), Shi = read_lane64(my_hi, s);
            bool fa, fb;
            wide_feasible(Slo, Shi, Alo, Ahi, Blo, Bhi, lane, n, a.k, fa, fb);
            fa = fa && allow_a;
            fb = fb && allow_b;
            const uint64_t ma = ballot(fa), mb = ballot(fb);
            const uint32_t na = (uint32_t)__popcll(ma), nb = (uint32_t)__popcll(mb);
            feasible += na + nb;
            if (na + nb == 0)
                continue;
            // qcount < 64 here and na + nb <= 126, so the ring of 256 never overruns
            if (fa) {
                const uint32_t at = (qhead + qcount + (uint32_t)lanes_below(ma)) & (kWideQueue - 1);
                queue_lo[wv][at] = Slo | (1ull << lane);
                queue_hi[wv][at] = Shi;
                queue_v[wv][at] = (uint8_t)lane;
            }
            if (fb) {
                const uint32_t at = (qhead + qcount + na + (uint32_t)lanes_below(mb)) & (kWideQueue - 1);
                queue_lo[wv][at] = Slo;
                queue_hi[wv][at] = Shi | (1ull << lane);
                queue_v[wv][at] = (uint8_t)(lane + 64);
            }
            qcount += na + nb;
            while (qcount >= 64)
                drain(64);
        }
    }
    while (qcount)
        drain(qcount < 64 ? qcount : 64);
    flush();
    if (ballot(ovf) != 0ull && lane == 0)
        atomicOr(&a.ctr->overflow, 1u);
    if (lane == 0 && feasible)
        atomicAdd(&a.ctr->successors, (unsigned long long)feasible);
}

__global__ void find_wide_kernel(const uint64_t *keys, uint64_t count, uint64_t lo, uint64_t hi,
                                 unsigned long long *result)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        if (keys[2 * i] == lo && keys[2 * i + 1] == hi)
            atomicMin(result, (unsigned long long)i);
}

}  // namespace

hipError_t launch_expand_wide(const LevelArgs &a, uint64_t allowed_hi, unsigned grid_blocks, hipStream_t s)
{
    if (a.in_count == 0)
        return hipSuccess;
    hipLaunchKernelGGL(expand_wide_kernel, dim3(grid_blocks), dim3(kBlock), 0, s, a, allowed_hi);
    return hipGetLastError();
}

hipError_t launch_find_wide(const void *keys, uint64_t count, uint64_t lo, uint64_t hi, unsigned long long *result,
                            hipStream_t s)
{
    if (count == 0)
        return hipSuccess;
    uint64_t b = (count + 255) / 256;
    b = b < 1 ? 1 : (b > 4096 ? 4096 : b);
    hipLaunchKernelGGL(find_wide_kernel, dim3((unsigned)b), dim3(256), 0, s, (const uint64_t *)keys, count, lo, hi,
                       result);
    return hipGetLastError();
}

}  // namespace twk
