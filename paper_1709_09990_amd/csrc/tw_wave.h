// Wave64 helpers shared by the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace twk {

__device__ __forceinline__ uint64_t read_lane64(uint64_t x, int lane)
{
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, lane);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t first_lane32(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}

__device__ __forceinline__ uint64_t ballot(bool p)
{
    return __builtin_amdgcn_ballot_w64(p);
}

// Number of set bits of mask below this lane.
__device__ __forceinline__ int lanes_below(uint64_t mask)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Orders this wave's LDS writes before its later LDS reads by other lanes.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Slot hash of a state: two multiply-xorshift rounds.
__device__ __forceinline__ uint64_t slot_hash(uint64_t key)
{
    uint64_t h = key * 0xD6E8FEB86659FD93ull;
    h ^= h >> 32;
    h *= 0xD6E8FEB86659FD93ull;
    h ^= h >> 32;
    return h;
}

// |Q(S, v)| <= k for this lane's vertex v (§2): components of G[S] by ballot
// breadth-first search; N_out(K) of each component by one more ballot; lane v
// unions N_out(K) for the components it touches.  Aj is this lane's adjacency
// row (0 for lanes >= n).  Returns whether lane v is a feasible successor.
__device__ __forceinline__ bool lane_feasible(uint64_t S, uint64_t Aj, int lane, int n, int k)
{
    const uint64_t lanebit = 1ull << lane;
    const bool inS = (S >> lane) & 1ull;
    uint64_t qacc = 0;
    uint64_t rem = S;
    while (rem) {
        uint64_t comp = rem & (~rem + 1ull);
        for (;;) {
            const uint64_t nxt = comp | ballot(inS && (Aj & comp) != 0ull);
            if (nxt == comp)
                break;
            comp = nxt;
        }
        rem &= ~comp;
        const uint64_t nout = ballot(!inS && (Aj & comp) != 0ull);
        if (nout & lanebit)
            qacc |= nout;
    }
    const uint64_t Q = (Aj | qacc) & ~S & ~lanebit;
    return lane < n && !inS && __popcll(Q) <= k;
}

}  // namespace twk
