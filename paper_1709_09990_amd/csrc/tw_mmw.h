// Per-state minor-min-width pruning (§3.3): declarations shared by the host
// runtime and the gfx950 kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace twk {

// One prune launch over level i: every state S with MMW(H_S) <= k is copied
// (with its creating vertex) to out; the others are dropped.  H_S is the graph
// left after eliminating S: vertices V - S, an edge uw when w lies in Q(S, u).
struct PruneArgs {
    const void *in;             // level i keys (uint32 when key_bytes = 4, else uint64)
    const uint8_t *in_lastv;    // creating vertex of each key, or nullptr (level 0)
    uint64_t in_count;
    void *out;                  // kept keys, room for in_count
    uint8_t *out_lastv;         // kept creating vertices (unused when in_lastv is nullptr)
    const uint64_t *adj;        // n adjacency rows (device)
    unsigned long long *kept;   // zero on entry; number of kept states on exit
    int n;
    int k;
    int key_bytes;
};

hipError_t launch_mmw_prune(const PruneArgs &a, unsigned grid_blocks, hipStream_t s);

}  // namespace twk
