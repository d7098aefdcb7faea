// Device structures of the batched search (many graphs solved together: level
// rounds, or one persistent launch with a work queue).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace twk {

// Graph status in a batch.
enum : uint32_t {
    kBatchRunning = 0,
    kBatchDone = 1,      // YES at bound k; the levels of that run are in the arena
    kBatchFallback = 2,  // arena or table too small: solve it alone on the host path
};

constexpr int kBatchKeyBits = 48;   // keys below bit 48, table tag above
constexpr int kBatchWavesPerBlock = 4;
constexpr int kBatchMaxN = 48;

// One level of one graph's batched search, recorded in trace mode (a test
// hook): the level's size, the feasible pairs that built it, and two
// order-independent digests of its states (sum of the splitmix64 output
// function, xor of MurmurHash3's fmix64).  Layout shared with tw_batch_level.
struct BatchTraceRec {
    int32_t k;
    int32_t level;
    uint64_t count;
    uint64_t successors;
    uint64_t digest_sum;
    uint64_t digest_xor;
};

// Per-graph state, device resident.  Written by the host before the launch;
// afterwards only by the wave that finishes a level of this graph (counters
// by atomics; in the persistent launch every field that changes is stored and
// loaded with device-scope atomics).
struct BatchGraph {
    uint64_t adj[64];
    uint64_t adjk[64];       // adjacency the current bound expands with: adj, plus with paths the
                             // pairs joined by more than k disjoint paths (set per bound)
    uint64_t *keys;          // arena: the levels of the current bound, back to back
    uint8_t *lastv;
    uint32_t *parent;        // per state: index of the state it came from, within the level below
    uint64_t arena_cap;      // states the arena holds
    uint64_t *table;         // tagged open-addressing table (tag << 48 | key), zero-initialised
    uint64_t table_slots;
    uint64_t level_off[66];  // arena offset of level i (current bound)
    unsigned long long out_count;   // states claimed for the level being built
    unsigned long long successors;  // feasible pairs over the whole solve
    unsigned long long expansions;  // (S, v) pairs over the whole solve
    unsigned long long states;      // states expanded over the whole solve
    unsigned long long peak;        // largest level
    unsigned long long unique;      // states written over the whole solve
    unsigned long long peak_k;      // largest level of the current bound
    unsigned long long peak_yes;    // largest level of the best YES run
    uint32_t overflow;
    uint32_t status;
    int32_t n, k, level, L;
    int32_t tw;
    int32_t known_no;        // largest bound known to be NO (lower bound - 1 at start)
    int32_t best_yes;        // smallest bound known to be YES (n - 1 at start)
    uint32_t tag;
    uint32_t decisions, levels_run;
    int32_t order[64];       // elimination order of the best YES run (width best_yes)
    uint64_t allowed;        // vertices that may be added to a state (all, or all but a maximum clique)
    const uint8_t *paths;    // 64 x 64 disjoint-path counts: bound k adds uv when > k (null: none)
    // trace mode (null trace: off): one record per level built, up to trace_cap
    BatchTraceRec *trace;
    uint32_t trace_cap;
    uint32_t trace_len;      // records written, or wanted when above trace_cap
    unsigned long long digest_sum;  // digests of the level being built
    unsigned long long digest_xor;
    unsigned long long succ_mark;   // successors when the level being built started
    int32_t fault_level;     // test hook: building this level counts as an overflow (0: off)
    int32_t pad_;
};

// One level of one graph: ready tasks of up to chunk states.  It carries
// the graph fields every task needs (bound, table tag, where the next level
// starts), so a task reads them with the job.
struct BatchJob {
    int32_t graph;
    int32_t level;
    uint64_t begin;          // arena offset of the level's first state
    uint64_t count;
    uint64_t out_base;       // arena offset of the next level
    int32_t k;
    uint32_t tag;
    uint32_t chunk;          // states per chunk
    uint32_t cursor;         // next chunk to hand out (atomic)
    uint32_t done;           // chunks finished (atomic)
    uint32_t ready;          // 0, then the number of chunks once the fields above are written
                             // (stored after they completed): one load tells both
    uint32_t pad_[2];
};

// The words every wave polls (head, tail) and the exit words (active,
// abort) sit on separate 128-byte lines.
struct BatchQueue {
    unsigned long long head;      // persistent queue: first job not yet exhausted; level rounds: the round's task size
    unsigned long long tail;      // jobs reserved
    unsigned long long capacity;
    unsigned long long pad0_[13];
    uint32_t active;              // graphs still running
    uint32_t abort;               // set if a wait exceeded its bound or the job array filled
    uint32_t pad1_[30];
};
static_assert(sizeof(BatchQueue) == 256, "queue lines");

struct BatchArgs {
    BatchGraph *graphs;
    BatchJob *jobs;
    BatchQueue *q;
    uint32_t chunk;          // states per task (multiple of 64); the persistent queue's smallest task
    uint32_t max_probe;
    float max_load;          // a level above this fraction of the table overflows
    uint32_t spin_limit;     // sleeps a wave may spend waiting for work before aborting
    uint32_t nb;             // graphs in the batch
    uint32_t nwaves;         // waves of the persistent grid
};

hipError_t launch_batch(const BatchArgs &a, unsigned grid_blocks, hipStream_t s);
// One level round (a.jobs == nullptr): plan the tasks of every running graph's
// current level into task_start[0..B], expand them, advance the graphs.
hipError_t launch_batch_round(const BatchArgs &a, uint32_t B, uint32_t *task_start, unsigned grid_blocks,
                              hipStream_t s);
int batch_blocks_per_cu();

}  // namespace twk
