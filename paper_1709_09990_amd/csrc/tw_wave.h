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

// Hash of a state: one xorshift, one multiply by an odd constant (the high
// bits are used: a range reduction takes the top of hash * size).
__device__ __forceinline__ uint64_t slot_hash(uint64_t key)
{
    return (key ^ (key >> 29)) * 0x9E3779B97F4A7C15ull;
}

// |Q(S, v)| <= k for this lane's vertex v (§2).  Components of G[S] by ballot
// breadth-first search: lane j reports whether its row A[j] meets the current
// set; the lanes of S among them extend the component, and once it stops
// growing the lanes outside S among them are N_out(K), the outside vertices
// adjacent to K.  Lane v unions N_out(K) for the components it touches.  Aj is
// this lane's adjacency row (0 for lanes >= n).  Returns whether lane v is a
// feasible successor.
__device__ __forceinline__ bool lane_feasible(uint64_t S, uint64_t Aj, int lane, int n, int k)
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
    const uint64_t Q = (Aj | qacc) & ~S & ~lanebit;
    return lane < n && !((S >> lane) & 1ull) && __popcll(Q) <= k;
}

// Slot of a key in a table of `slots` entries (any size): the high half of
// hash * slots (multiply-shift range reduction).
__device__ __forceinline__ uint64_t slot_in(uint64_t key, uint64_t slots)
{
    return __umul64hi(slot_hash(key), slots);
}

}  // namespace twk
