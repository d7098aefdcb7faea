// Declarations shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace twk {

// Device-resident counters of one level launch (zeroed before it).
struct LevelCounters {
    unsigned long long out_count;   // distinct successors claimed so far
    unsigned long long successors;  // feasible (S, v) pairs, duplicates included
    unsigned int overflow;          // 1: output capacity or probe limit exceeded
    unsigned int pad;
};

// Arguments of one expansion launch (level i -> level i+1).
struct LevelArgs {
    const void *in;         // level i keys (uint32 or uint64)
    uint64_t in_count;
    void *out;              // level i+1 keys, capacity out_cap
    uint8_t *out_lastv;     // vertex that created each level i+1 key
    uint64_t out_cap;
    void *table;            // open-addressing table of table_slots entries, all EMPTY on entry
    uint64_t table_slots;
    uint64_t allowed;       // vertices that may be added (all for a full search)
    const uint64_t *adj;    // n adjacency rows (device)
    int n;
    int k;
    LevelCounters *ctr;
    uint32_t max_probe;     // probe-length backstop
    int read_first;         // 1: plain load before the compare-and-swap (slots only go EMPTY -> key)
    int key_bytes;          // 4 (n <= 32) or 8
    // Bloom-filter variant (§3.2): used instead of the table when bloom != nullptr
    uint32_t *bloom;        // bit array of bloom_mask+1 bits, all zero on entry
    uint64_t bloom_mask;
};

// Partitioned insert (large levels): phase 1 writes every feasible (S, v) as
// one 64-bit entry (state | v << 58) into partition p of the successor buffer;
// phase 2 inserts partition by partition into that partition's table slice.
// Each partition is split into kSubRegions regions with their own counters
// (wave w appends to region w mod kSubRegions), so the flush atomics spread
// over P * kSubRegions addresses instead of P.
struct ScatterArgs {
    uint64_t *parts;        // P * kSubRegions regions of sub_cap entries
    uint64_t sub_cap;
    unsigned long long *sub_count;   // [P * kSubRegions] entries claimed (may exceed sub_cap: overflow)
    int P;
};

struct GatherArgs {
    const uint64_t *parts;
    uint64_t sub_cap;
    const uint64_t *chunk_prefix;    // [P*kSubRegions+1] exclusive prefix of 64-entry chunks per region
    const uint64_t *count;           // [P*kSubRegions] entries per region
    int P;
    uint64_t slice;                  // table slots per partition
};

// Gated level loop (one bound as a fixed launch sequence, for HIP graphs).
struct CaptureCtl {
    int k;                  // the bound
    int L;                  // levels run: max(0, n - k - 1)
    uint64_t allowed;       // vertices that may be added to a state
};

struct GateArgs {
    const CaptureCtl *ctl;
    LevelCounters *ctr;     // ctr[i]: the launch that builds level i+1 from level i
    int level;              // i
};

struct BacktrackArgs {
    const void *keys;       // every level, level i at keys + off[i] (key_bytes each)
    const uint8_t *lastv;   // creating vertex, same offsets
    const uint64_t *off;    // device: level offsets
    const CaptureCtl *ctl;
    const LevelCounters *ctr;
    int32_t *order;         // out: order[0..L)
    uint64_t *last_state;   // out: the level-L state the order ends in
    int32_t *err;           // out: 1 if a predecessor was not found
};

constexpr int kMaxParts = 64;
constexpr int kSubRegions = 64;
constexpr int kEntryVShift = 58;     // entries carry v above bit 58 (n <= 58)

constexpr int kBloomProbes = 17;     // hash functions per state (§3.2)
constexpr int kBloomBitsPerState = 24;  // m / n lower bound (§3.2)

constexpr int kBlock = 256;          // 4 waves of 64
constexpr int kWavesPerBlock = kBlock / 64;

hipError_t launch_fill_empty(void *table, uint64_t bytes, hipStream_t s);
hipError_t launch_fill_zero(void *p, uint64_t bytes, hipStream_t s);
hipError_t launch_expand(const LevelArgs &a, unsigned grid_blocks, hipStream_t s);
hipError_t launch_scatter(const LevelArgs &a, const ScatterArgs &sc, unsigned grid_blocks, hipStream_t s);
hipError_t launch_gather(const LevelArgs &a, const GatherArgs &ga, unsigned grid_blocks, hipStream_t s);
hipError_t launch_find(const void *keys, uint64_t count, uint64_t target, int key_bytes,
                       unsigned long long *result, hipStream_t s);
hipError_t launch_zero_counters(LevelCounters *c, hipStream_t s);
// Graphs of up to 126 vertices: keys are (low word, high word) pairs, a.adj
// holds two words per row, a.allowed the low half of the allowed vertices.
hipError_t launch_expand_wide(const LevelArgs &a, uint64_t allowed_hi, unsigned grid_blocks, hipStream_t s);
hipError_t launch_find_wide(const void *keys, uint64_t count, uint64_t lo, uint64_t hi, unsigned long long *result,
                            hipStream_t s);
hipError_t launch_prep_gated(const GateArgs &g, void *table, uint64_t bytes, hipStream_t s);
hipError_t launch_expand_gated(const LevelArgs &a, const GateArgs &g, unsigned grid_blocks, hipStream_t s);
hipError_t launch_backtrack(const BacktrackArgs &b, int key_bytes, hipStream_t s);

}  // namespace twk
