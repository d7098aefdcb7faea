// Per-state minor-min-width pruning for gfx950 (§3.3).
//
// The paper computes MMW of the graph left after eliminating S without
// storing that graph (a disjoint-set structure and two graph searches per
// contraction), to fit the per-thread memory of its GPU.  Here one wave
// handles one state and the graph is stored after all: lane u holds row u of
// H_S, the set Q(S, u), as a 64-bit mask in registers.  The rows come from the
// same ballot breadth-first search over the components of G[S] that the
// expansion uses; each contraction is then a few wave-wide minimum
// reductions and per-lane mask updates, with no memory traffic at all.
//
// MMW rounds (as the oracle's O6): test the second-smallest degree; take
// the lowest-index vertex v of minimum degree; delete it if isolated, else
// contract it into its lowest-index minimum-degree neighbour u (u keeps its
// label and gains v's other neighbours).  A state is dropped as soon as a
// round's second-smallest degree exceeds k; rounds stop once at most k + 1
// vertices remain, since no degree there can exceed k.
#include "tw_mmw.h"
#include "tw_wave.h"

namespace twk {
namespace {

// Row u of H_S for this lane's vertex u (0 for lanes in S or >= n): the
// vertices outside S and other than u that u reaches through S (§2).
__device__ __forceinline__ uint64_t eliminated_row(uint64_t S, uint64_t Aj, int lane, int n)
{
    const uint64_t lanebit = 1ull << lane;
    uint64_t qacc = 0;
    uint64_t rem = S;
    while (rem) {
        uint64_t comp = rem & (~rem + 1ull);
        uint64_t touch;
        for (;;) {
            touch = ballot((Aj & comp) != 0ull);
            const uint64_t nxt = comp | (touch & S);
            if (nxt == comp)
                break;
            comp = nxt;
        }
        rem &= ~comp;
        const uint64_t nout = touch & ~S;
        if (nout & lanebit)
            qacc |= nout;
    }
    const bool live = lane < n && !((S >> lane) & 1ull);
    return live ? (Aj | qacc) & ~S & ~lanebit : 0ull;
}

// Minimum over the 64 lanes (every lane active), returned uniformly: DPP
// swaps within quads (lane ^ 1, lane ^ 2) and rotations by 4 and 8 within
// each row of 16 give every lane its row's minimum; the four row minima are
// read into scalars.  No LDS traffic, unlike a shuffle through ds_bpermute.
__device__ __forceinline__ uint32_t wave_min(uint32_t x)
{
    // every source lane exists for these patterns, so bound_ctrl does not
    // matter; setting it lets the compiler fold each move into the min
    x = min(x, (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, true));   // quad_perm 1,0,3,2
    x = min(x, (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, true));   // quad_perm 2,3,0,1
    x = min(x, (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x124, 0xF, 0xF, true));  // row_ror 4
    x = min(x, (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x128, 0xF, 0xF, true));  // row_ror 8
    const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)x, 0);
    const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)x, 16);
    const uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int)x, 32);
    const uint32_t r3 = (uint32_t)__builtin_amdgcn_readlane((int)x, 48);
    return min(min(r0, r1), min(r2, r3));
}

// True when MMW of the graph (rows `row`, vertex set `alive`, uniform) exceeds k.
__device__ __forceinline__ bool mmw_exceeds(uint64_t row, uint64_t alive, int lane, int k)
{
    const uint32_t none = 0xFFFFFFFFu;
    while (__popcll(alive) >= k + 2) {
        const bool live = (alive >> lane) & 1ull;
        const int deg = __popcll(row);
        // the second-smallest degree exceeds k exactly when at most one
        // vertex has degree <= k
        if (__popcll(ballot(live && deg <= k)) <= 1)
            return true;
        const uint32_t key = live ? ((uint32_t)deg << 6) | (uint32_t)lane : none;
        const int v = (int)(wave_min(key) & 63u);
        const uint64_t vb = 1ull << v;
        const uint64_t rv = read_lane64(row, v);
        if (rv) {
            const uint32_t m3 = wave_min(((rv >> lane) & 1ull) ? key : none);
            const int u = (int)(m3 & 63u);
            const uint64_t ub = 1ull << u;
            if (row & vb) {
                row &= ~vb;
                if (lane != u)
                    row |= ub;
            }
            if (lane == u)
                row = (row | rv) & ~(ub | vb);
            if (lane == v)
                row = 0;
        }
        alive &= ~vb;
    }
    return false;
}

template <typename Key>
__device__ __forceinline__ uint64_t key_of_lane(Key x, int t)
{
    if constexpr (sizeof(Key) == 4)
        return (uint32_t)__builtin_amdgcn_readlane((int)x, t);
    else
        return read_lane64(x, t);
}

// Each wave takes chunks of 64 consecutive states; lane t loads state t of the
// chunk, the wave then decides the states one at a time and writes the kept
// ones with one counter update per chunk.
template <typename Key>
__global__ __launch_bounds__(256) void mmw_prune_kernel(PruneArgs a)
{
    const int lane = (int)(threadIdx.x & 63u);
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    const Key *in = (const Key *)a.in;
    Key *out = (Key *)a.out;
    const uint64_t Aj = lane < a.n ? a.adj[lane] : 0ull;
    const uint64_t nmask = a.n == 64 ? ~0ull : (1ull << a.n) - 1ull;
    const uint64_t chunks = (a.in_count + 63) / 64;
    for (uint64_t c = wave; c < chunks; c += waves) {
        const uint64_t idx = c * 64 + (uint64_t)lane;
        const bool have = idx < a.in_count;
        const Key mine = have ? in[idx] : (Key)0;
        const uint8_t mine_v = (have && a.in_lastv) ? a.in_lastv[idx] : 0;
        const int m = (int)min<uint64_t>(64, a.in_count - c * 64);
        uint64_t keep = 0;
        for (int t = 0; t < m; ++t) {
            const uint64_t S = key_of_lane<Key>(mine, t);
            const uint64_t row = eliminated_row(S, Aj, lane, a.n);
            if (!mmw_exceeds(row, nmask & ~S, lane, a.k))
                keep |= 1ull << t;
        }
        unsigned long long base = 0;
        if (lane == 0 && keep)
            base = atomicAdd(a.kept, (unsigned long long)__popcll(keep));
        base = ((unsigned long long)(uint32_t)__shfl((int)(uint32_t)(base >> 32), 0, 64) << 32) |
               (uint32_t)__shfl((int)(uint32_t)base, 0, 64);
        if ((keep >> lane) & 1ull) {
            const uint64_t pos = base + (uint64_t)lanes_below(keep);
            out[pos] = mine;
            if (a.in_lastv)
                a.out_lastv[pos] = mine_v;
        }
    }
}

}  // namespace

hipError_t launch_mmw_prune(const PruneArgs &a, unsigned grid_blocks, hipStream_t s)
{
    if (a.in_count == 0)
        return hipSuccess;
    if (!a.in || !a.out || !a.adj || !a.kept || a.n < 1 || a.n > 64 || (a.in_lastv && !a.out_lastv) ||
        (a.key_bytes == 4 && a.n > 32) || (a.key_bytes != 4 && a.key_bytes != 8))
        return hipErrorInvalidValue;
    if (a.key_bytes == 4)
        hipLaunchKernelGGL(mmw_prune_kernel<uint32_t>, dim3(grid_blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(mmw_prune_kernel<uint64_t>, dim3(grid_blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace twk
