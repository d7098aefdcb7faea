/*
 * tw.h — exact treewidth on AMD MI355X (gfx950): the level-synchronous search
 * over elimination-ordering states of van der Zanden & Bodlaender,
 * "Computing Treewidth on the GPU" (arXiv 1709.09990).
 *
 * Definitions used throughout (paper §2 and §3.1):
 *   - A graph has n <= 64 vertices 0..n-1, given as n adjacency rows: bit j of
 *     adj[i] is set iff {i, j} is an edge.  Rows must be symmetric with no
 *     self-loops and no bits at positions >= n.
 *   - A state is a vertex set S, stored as a bitmask (32-bit keys on the device
 *     when n <= 32, 64-bit otherwise; always uint64_t across this interface).
 *   - Q(S, v), for v outside S, is the set of vertices outside S and other than
 *     v that v reaches by paths whose internal vertices all lie in S (§2).
 *     |Q(S, v)| is the degree of v once S has been eliminated.
 *   - For a bound k, level 0 is {empty set}; level i+1 holds every S + {v}
 *     with S in level i, v not in S and |Q(S, v)| <= k, each set once
 *     (Listing 1, §3.1; duplicates removed exactly, §3.2).
 *   - decide(k) is YES iff level L(k) = max(0, n-k-1) is non-empty: the last
 *     k+1 vertices can go in any order (third optimisation of §3.1).
 *   - tw(G) = the smallest k with decide(k) = YES.
 *
 * All functions are extern "C" and never throw.  Every array argument is a
 * host pointer owned by the caller unless stated otherwise; the library copies
 * what it needs during the call and holds no caller pointer afterwards.
 * Device memory (frontiers, hash tables) belongs to the context and persists
 * between calls until tw_ctx_destroy.  A context serves one host thread at a
 * time; calls return after every output has been written.
 *
 * Errors are returned, never hidden: no answer is ever truncated.  If the
 * device memory needed by a level cannot be obtained even after regrowing, the
 * call fails with TW_ENOMEM (or TW_ECAPACITY when a caller-imposed limit is
 * hit), and the message is available from tw_last_error.
 */
#ifndef TW_H
#define TW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TW_OK = 0,
    TW_EINVAL = 1,    /* bad argument: graph not simple/symmetric, n outside 1..64, k < 0, NULL output */
    TW_ENOMEM = 2,    /* device or host memory could not be obtained */
    TW_EDEVICE = 3,   /* HIP runtime error, or an internal consistency check failed */
    TW_ECAPACITY = 4  /* a level needs more states than options.max_states allows */
} tw_status;

/* Duplicate removal between levels (§3.2). */
enum {
    TW_DEDUP_EXACT = 0, /* open-addressing hash table in HBM, atomic compare-and-swap (default) */
    TW_DEDUP_BLOOM = 1, /* Bloom filter, 17 probes by double hashing (§3.2); a NO answer is then not certified */
    TW_DEDUP_BLOOM_CERTIFIED = 2 /* Bloom search, and every NO of tw_decide / tw_solve decided again by the
                                    exact search (a false positive only drops states, so only a NO can be
                                    wrong; a YES is certified by its order's width) */
};

/* Choice of the bounds k tried by tw_solve / tw_solve_batch (§3.1). */
enum {
    TW_K_ASCENDING = 0, /* k = minor-min-width lower bound (§3.3), then k+1, ... until YES */
    TW_K_LEARNED = 1    /* start from a predicted k; YES at t is certified by NO at t-1 or t = lower bound; a
                           graph whose predicted largest level exceeds half of what fits (max_states, else
                           device memory), or with more than 40 vertices (beyond the sizes the networks were
                           trained on), starts at the lower bound */
};

/* A graph: n rows, host pointer, caller-owned. */
typedef struct {
    uint32_t n;
    const uint64_t *adj;
} tw_graph;

/* Context options.  Zero-initialise, set struct_size = sizeof(tw_options),
 * then change what you need. */
typedef struct {
    size_t struct_size;
    int device;               /* HIP device ordinal */
    void *stream;             /* hipStream_t to launch on, or NULL for a stream the context creates */
    int dedup;                /* TW_DEDUP_EXACT, TW_DEDUP_BLOOM or TW_DEDUP_BLOOM_CERTIFIED */
    float load_factor;        /* target hash-table load in (0, 0.9]; 0 picks the default 0.25 (raised
                                 towards 0.5 when the table would take over a third of free memory) */
    int k_policy;             /* TW_K_ASCENDING or TW_K_LEARNED */
    const char *weights_path; /* TW_K_LEARNED: file of network parameters: 8 bytes "TWMPNN01", a
                                 uint32 count (= tw_mpnn_param_count()), then count float32 values,
                                 little-endian; read at tw_ctx_create (TW_EINVAL if absent or bad) */
    uint64_t max_states;      /* cap on states per level (0 = limited only by device memory) */
    uint64_t capacity_override; /* test hook: first guess of every level's size (0 = estimate); a
                                   small value forces the overflow -> regrow -> replay path */
    int timing;               /* 1: time every expansion launch with HIP events (tw_stats.kernel_*) */
    int probe;                /* exact table probe: 0 = default, 1 = compare-and-swap only,
                                 2 = plain load first, CAS only on an empty slot */
    int partition;            /* exact insert: 0 or 1 = single phase (default), 2 = two phases: expand
                                 and scatter the feasible pairs into hash-range partitions, then insert
                                 partition by partition into table slices of <= 64 MB (n <= 58).  The
                                 two-phase form keeps the probes in the Infinity Cache but pays a
                                 second pass; it measured slower on MI355X for the levels tried */
    /* tw_solve_batch: graphs with n <= 48 run together on the device, each with
       its own state arena (all levels of its current bound) and hash table. */
    uint64_t batch_graph_states; /* arena states per graph (0 = as many as half the free device memory
                                    allows, 2^16..2^22); a graph that outgrows its arena or table is
                                    re-solved alone by the tw_solve path */
    uint32_t batch_chunk;     /* smallest work-queue task in states, multiple of 64 (0 = 256); a large level is cut
                                 into about two tasks per wave of the grid, up to 1024 states each */
    int batch_schedule;       /* tw_solve_batch: TW_BATCH_AUTO (default) takes the persistent queue, or level
                                 rounds when options.reductions is on (its levels are small, and small
                                 levels favour the rounds); TW_BATCH_PERSISTENT: one persistent launch
                                 with a device work queue of (graph, level) jobs cut into tasks of at
                                 least batch_chunk states; TW_BATCH_ROUNDS: level rounds — per round one
                                 launch expands the current level of every running graph (tasks sized
                                 for about two per wave) and a second advances each graph */
    int reductions;           /* TW_REDUCE_NONE (default): the levels are those of Listing 1.
                                 TW_REDUCE_CLIQUE_PATHS: the first two optimisations of §3.1 — the
                                 vertices of a maximum clique C are never added to a state (some optimal
                                 order ends with C; C is the maximum clique whose ascending vertex list is
                                 lexicographically smallest), decide(k) is NO without a search when
                                 k < |C| - 1, and the search for bound k runs on G plus an edge uv for
                                 every non-adjacent pair joined by >= k + 1 internally vertex-disjoint
                                 paths in G (counts taken once per graph).  Answers are unchanged; levels
                                 become {S outside C : |S| = i, S has width <= k in that graph}. */
    int mmw_prune;            /* TW_MMW_NONE (default), or TW_MMW_PRUNE: per-state minor-min-width (§3.3)
                                 — before a level is expanded, every state S whose eliminated graph H_S
                                 (vertices outside S, an edge uw when w lies in Q(S, u)) has minor-min-width
                                 above k is dropped, since the remaining vertices cannot then be eliminated
                                 within width k.  MMW as tw_mmw, on H_S.  Answers are unchanged; level i+1
                                 holds the successors of the kept states of level i (levels handed to a
                                 trace sink are the unpruned ones; the kept-state counts go to
                                 tw_stats.states_expanded).  tw_solve_batch then solves every graph on the
                                 tw_solve path. */
    /* Device memory from the caller (it owns it; a torch tensor, say):
       when workspace is non-NULL, every device buffer of the context (levels, hash tables, counters,
       batch arenas) is carved from [workspace, workspace + workspace_bytes) and the library calls
       no hipMalloc for them; a level that does not fit fails with TW_ENOMEM.  The range must stay
       valid and unused by the caller until tw_ctx_destroy.  tw_solve_batch then solves the graphs
       bound for the single-graph path on this context, after the batched ones.  The learned start
       bound's network (TW_K_LEARNED) keeps its own small allocation. */
    void *workspace;
    size_t workspace_bytes;
    int fault_inject_level;   /* test hook (0 = off): the first build of level i = fault_inject_level of
                                 every bound is treated as an overflow, so the regrow -> replay path
                                 runs (tw_stats.retries counts it) and the level is built again; in
                                 the batched search the graph reaching that level leaves the batch
                                 for the single-graph path.  Answers and levels are unchanged; with
                                 max_states at that level's size the replay fails with TW_ECAPACITY */
    int capture;              /* TW_CAPTURE_AUTO (default): tw_decide, tw_solve (and tw_solve_batch's
                                 single-graph path) run a bound's whole level loop (Listing 1, §3.1) as one replay of
                                 a HIP graph when every level fits its binomial bound C(m, i) within
                                 256 MiB (n <= 25 or so; exact dedup, no MMW pruning, no test hooks): the
                                 launches read each level's size and the bound from device memory and do
                                 nothing past an empty level, so the host waits once per bound instead of
                                 once per level.  The graph is captured once per graph shape and kept by
                                 the context.  TW_CAPTURE_OFF: the host-driven level loop always */
} tw_options;

enum { TW_CAPTURE_AUTO = 0, TW_CAPTURE_OFF = 1 };

enum { TW_REDUCE_NONE = 0, TW_REDUCE_CLIQUE_PATHS = 1 };
enum { TW_BATCH_AUTO = 0, TW_BATCH_ROUNDS = 1, TW_BATCH_PERSISTENT = 2 };
enum { TW_MMW_NONE = 0, TW_MMW_PRUNE = 1 };

/* Counters of one call (summed over every bound k and level it ran). */
typedef struct {
    uint64_t states_expanded; /* sum of |level i| over the levels expanded */
    uint64_t expansions;      /* candidate (S, v) pairs: sum of |level i| * (n - i) */
    uint64_t successors;      /* feasible (S, v) pairs generated (before duplicate removal) */
    uint64_t unique;          /* distinct states written: sum of |level i+1| */
    uint64_t peak_frontier;   /* largest level met */
    uint32_t decisions;       /* bounds k tried */
    uint32_t levels;          /* levels expanded */
    uint32_t retries;         /* levels replayed after an overflow */
    uint32_t launches;        /* expansion kernel launches (replays included) */
    double seconds;           /* wall time of the call */
    double kernel_seconds;    /* summed duration of the expansion launches (options.timing = 1) */
} tw_stats;

typedef struct tw_ctx tw_ctx;

/* Create a context on options->device (options may be NULL for defaults). */
tw_status tw_ctx_create(const tw_options *options, tw_ctx **out);
void tw_ctx_destroy(tw_ctx *ctx);

/* decide(k) of Listing 1 (§3.1): *out_yes = 1 iff tw(G) <= k.  k >= n-1 is
 * YES without a level.  stats may be NULL; it receives the counters of the
 * levels built also when the call fails (TW_ECAPACITY or TW_ENOMEM at some
 * level: the counters of the levels before it). */
tw_status tw_decide(tw_ctx *ctx, const tw_graph *g, int32_t k, int32_t *out_yes, tw_stats *stats);

/* tw(G) and an elimination order of that width (§2): ascending k from the
 * minor-min-width bound (§3.3), or from the learned start bound (moving down
 * after a YES, up after a NO) with options.k_policy = TW_K_LEARNED.  out_order[t] is the t-th vertex eliminated;
 * it must hold n entries.  The order is rebuilt from the last level by
 * following, for each state, the vertex that created it back to the empty
 * set (from the kept levels, or, when they were too large to keep, from a
 * search restricted to the subsets of one last-level state), then the k+1
 * remaining vertices in ascending index; its width is checked to equal
 * *out_tw before returning. */
tw_status tw_solve(tw_ctx *ctx, const tw_graph *g, int32_t *out_tw, int32_t *out_order, tw_stats *stats);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): tw_solve with
 * ascending bounds from the minor-min-width lower bound (options.k_policy is
 * ignored), where every device buffer of the call (levels, hash table,
 * counters) lies in the library's static scratch of 64 MiB per GPU instead
 * of memory the call allocates.  The call makes no hipMalloc or hipFree.
 * n must be at most 32 (else TW_EINVAL); a search whose levels do not fit
 * the scratch fails with TW_ECAPACITY.  Every call on one GPU shares that
 * GPU's scratch, which keeps the last call's contents: calls that overlap on
 * one GPU (from several threads or contexts) race and must not be made. */
tw_status tw_solve_noalloc(tw_ctx *ctx, const tw_graph *g, int32_t *out_tw, int32_t *out_order, tw_stats *stats);

/* tw_solve for count graphs of uneven size.  out_tw[count], out_status[count];
 * out_orders holds the orders back to back (sum of n entries, graph order).
 * Graphs with n <= 48 are solved together on the device, each with its own
 * arena (every level of its current bound) and tagged hash table, by one
 * persistent kernel with a device work queue or by level rounds (one launch
 * expands the current level of every running graph, a second advances each
 * graph's level or bound); options.batch_schedule chooses.  Graphs whose
 * levels outgrow their arena get one more batched attempt with four times the
 * arena, and then, like the others, the tw_solve path, which runs on up to
 * four worker contexts of its own (each with its own stream and host thread;
 * none when options.workspace is given): those bound there from the start
 * beside the batched search, the rest after it.  The treewidths equal
 * tw_solve's; each order is checked by fill-in to have exactly that width
 * (several orders may qualify).
 * With options.k_policy = TW_K_LEARNED each graph starts at the bound the
 * network predicts (clamped to [lower bound, n-2]) and gets an arena sized
 * from the predicted peak level; the search then certifies the answer exactly
 * (YES at t and NO at t-1, or t = lower bound).  A start above the ascending
 * frontier whose levels exceed max_states or memory continues upwards from
 * the frontier instead.  out_graph_stats (nullable,
 * [count]) receives per-graph outcomes.  A graph that fails gets its own
 * status; the others still complete.  The return value is TW_OK unless an
 * argument is invalid or the device failed. */
typedef struct {
    uint64_t peak_yes;        /* largest level of the run that certified the answer (YES at tw) */
    uint64_t expansions;      /* (S, v) pairs over this graph's whole search */
    uint64_t states_expanded; /* states expanded over this graph's whole search */
    int32_t start_k;          /* first bound tried (lower bound, or the learned prediction) */
    uint32_t decisions;       /* bounds tried */
    int32_t path;             /* 0: batched on the device, 1: single-graph path, 2: trivial (tw = n-1) */
    int32_t reserved;
    uint64_t peak_any;        /* largest level met over the graph's search; for a graph that failed with
                                 TW_ECAPACITY, at least max_states (the size the failing level reached) */
} tw_graph_stats;

tw_status tw_solve_batch(tw_ctx *ctx, const tw_graph *gs, uint32_t count, int32_t *out_tw,
                         int32_t *out_orders, tw_status *out_status, tw_graph_stats *out_graph_stats,
                         tw_stats *stats);

/* Test hook for the batched search: one record per level a graph's batched
 * search built (Listing 1's level loop, §3.1, run for many graphs at once),
 * in the order built.  digest_sum is the sum mod 2^64 of the splitmix64
 * output function (Steele, Lea and Flood) over the level's states, digest_xor
 * the xor of MurmurHash3's fmix64 over them: equal sets give equal digests
 * whatever order the states were found in. */
typedef struct {
    int32_t k;
    int32_t level;        /* i >= 1: the record describes level i of bound k */
    uint64_t count;       /* |level i| */
    uint64_t successors;  /* feasible (S, v) pairs from level i-1 (duplicates included) */
    uint64_t digest_sum;
    uint64_t digest_xor;
} tw_batch_level;

/* tw_solve_batch with every batched graph's levels recorded.  Up to
 * max_records records per graph go to out_records[t * max_records ...];
 * out_nrecords[t] is the number the graph's successful batched attempt made
 * (above max_records: only the first max_records were kept), 0 for graphs
 * solved on the single-graph path or trivially.  first_arena_states (0: as
 * tw_solve_batch) sets the arena of the first batched attempt; graphs that
 * outgrow it get the retry with four times the arena (level rounds), whose
 * records replace the first attempt's.  Other arguments and outcomes as
 * tw_solve_batch.  TW_EINVAL if max_records is 0 or an output is NULL. */
tw_status tw_trace_batch(tw_ctx *ctx, const tw_graph *gs, uint32_t count, uint64_t first_arena_states,
                         uint32_t max_records, tw_batch_level *out_records, uint32_t *out_nrecords,
                         int32_t *out_tw, int32_t *out_orders, tw_status *out_status,
                         tw_graph_stats *out_graph_stats);

/* One level of a bound-k search, as handed to a trace sink. */
typedef struct {
    int32_t k;
    int32_t level;        /* i: this record describes level i (sets of size i) */
    uint64_t count;       /* |level i| */
    uint64_t expansions;  /* (S, v) pairs tried to build it: |level i-1| * (n - i + 1) */
    uint64_t successors;  /* feasible pairs among them */
    const uint64_t *states; /* the |level i| states, unordered; valid during the callback only */
    const uint8_t *last_v;  /* for each state, a vertex v with state - {v} in level i-1 */
} tw_level_record;

/* Test hook: decide(k) with every level copied to the host and handed to
 * sink (levels 0..L(k), or up to the first empty one). */
tw_status tw_trace_decide(tw_ctx *ctx, const tw_graph *g, int32_t k,
                          void (*sink)(const tw_level_record *rec, void *user), void *user,
                          int32_t *out_yes);

/* ---------------------------------------------------------------------------
 * Graphs of up to 126 vertices.  The paper keeps states as bitsets and notes
 * that wider bitsets extend the method (§3.1, §4.2); here a state is two
 * 64-bit words (vertices 0..63, then 64..125).  The limit of 126 comes from
 * the exact table: gfx950's widest compare-and-swap is 64 bits, so a slot
 * holds the state as two 63-bit halves, each word keeping one bit to tell a
 * free or unpublished half from a written one.  Same search as tw_decide /
 * tw_solve with exact duplicate removal (options.dedup, reductions, mmw_prune
 * and partition do not apply; the learned start bound is not used).
 * ------------------------------------------------------------------------- */
typedef struct {
    uint32_t n;          /* 1 <= n <= 126 */
    const uint64_t *adj; /* 2n words: row i is adj[2i] (vertices 0..63) and adj[2i+1] (64..125);
                            symmetric, no self-loops, no bits at positions >= n; caller-owned */
} tw_graph128;

/* decide(k) of Listing 1 (§3.1) on a graph of up to 126 vertices. */
tw_status tw_decide128(tw_ctx *ctx, const tw_graph128 *g, int32_t k, int32_t *out_yes, tw_stats *stats);
/* tw(G) and an order of that width (out_order: n entries), ascending bounds
 * from the minor-min-width bound; after the first YES the order is rebuilt
 * from the search restricted to the subsets of one last-level state. */
tw_status tw_solve128(tw_ctx *ctx, const tw_graph128 *g, int32_t *out_tw, int32_t *out_order, tw_stats *stats);
/* Test hook as tw_trace_decide; each record's states array holds 2 words per
 * state (low, high), count states. */
tw_status tw_trace_decide128(tw_ctx *ctx, const tw_graph128 *g, int32_t k,
                             void (*sink)(const tw_level_record *rec, void *user), void *user, int32_t *out_yes);
/* Host only: tw_mmw and tw_order_width for graphs of up to 126 vertices. */
tw_status tw_mmw128(const tw_graph128 *g, int32_t *out_lb);
tw_status tw_order_width128(const tw_graph128 *g, const int32_t *order, int32_t *out_width);

/* Minor-min-width lower bound with the second-smallest-degree improvement
 * (§3.3): each round takes the lowest-index vertex of minimum degree, deletes
 * it if isolated, otherwise contracts it into its lowest-index minimum-degree
 * neighbour; the bound is the largest second-smallest degree met. Host only. */
tw_status tw_mmw(const tw_graph *g, int32_t *out_lb);

/* Host only: what TW_REDUCE_CLIQUE_PATHS uses for g (§3.1).  *out_clique =
 * the maximum clique it never adds to a state (vertex mask; the one whose
 * ascending vertex list is lexicographically smallest); out_paths (n*n bytes,
 * may be NULL) row-major: internally vertex-disjoint u-v path counts for
 * non-adjacent u != v, capped at 255, 0 on the diagonal and for edges. */
tw_status tw_reductions(const tw_graph *g, uint64_t *out_clique, uint8_t *out_paths);

/* Tree decomposition from an elimination order (§1 states the goal is a
 * decomposition; §2 gives the order view).  Eliminating the vertices in order
 * with fill-in, bag(v) = v plus its neighbours not yet eliminated at that time;
 * out_bags[v] (n masks) holds it, and out_parent[v] (n entries) is the vertex
 * of bag(v) minus v that is eliminated first, or -1 when that set is empty
 * (one root per connected component).  These bags on that forest satisfy the
 * three conditions of a tree decomposition, and *out_width = max |bag| - 1 is
 * the order's width.  TW_EINVAL if order is not a permutation of 0..n-1.
 * Host only; all arrays caller-owned. */
tw_status tw_tree_decomposition(const tw_graph *g, const int32_t *order, uint64_t *out_bags,
                                int32_t *out_parent, int32_t *out_width);

/* Width of an elimination order by fill-in (§2); -1 in *out_width if order is
 * not a permutation of 0..n-1.  Host only. */
tw_status tw_order_width(const tw_graph *g, const int32_t *order, int32_t *out_width);

/* ---------------------------------------------------------------------------
 * Learned start bound: a small message-passing network (not from the paper)
 * that predicts a graph's treewidth and the size of the largest level of its
 * certifying search.  The exact search always decides the answer; the network
 * only picks where the search starts and how much memory a graph gets.
 *
 *   node features   [1, deg(v)/8, core(v)/8, n/64]     (core = core number)
 *   3 layers        H' = ReLU(H Ws^T + (A H) Wn^T + b), hidden width 64
 *   readout         [sum_v H_v ; max_v H_v] -> y = Wo r + bo, two outputs:
 *                   y0 ~ tw / n,  y1 ~ log2(peak level + 1) / 32
 *
 * Parameters are tw_mpnn_param_count() floats, in this order: for each layer
 * Ws [64][64] (row = output), Wn [64][64], b [64]; then Wo [2][128], bo [2].
 * Products run as bfloat16 MFMA with float32 accumulation (operands H, A H,
 * Ws, Wn, and in the backward pass dZ and dZ Wn, rounded to bfloat16, ties
 * to even); the master parameters and Adam moments stay float32.
 * ------------------------------------------------------------------------- */
typedef struct tw_mpnn tw_mpnn;

uint32_t tw_mpnn_param_count(void);
/* Host only: the 64 x 4 node features of g (rows beyond n are zero). */
tw_status tw_mpnn_features(const tw_graph *g, float *out);
/* A network on device with the given host parameters (copied); stream may be NULL. */
tw_status tw_mpnn_create(int device, void *stream, const float *params, tw_mpnn **out);
void tw_mpnn_destroy(tw_mpnn *m);
/* Replace the parameters (resets the Adam moments); read them back. */
tw_status tw_mpnn_set_params(tw_mpnn *m, const float *params);
tw_status tw_mpnn_get_params(tw_mpnn *m, float *params);
/* out[2*t + j] = output j for graph t. */
tw_status tw_mpnn_predict(tw_mpnn *m, const tw_graph *gs, uint32_t count, float *out);
/* Mean squared error over graphs and both outputs against targets[2*t + j],
 * and its gradient (out_grads: tw_mpnn_param_count() floats).  Per-graph
 * gradients are summed in graph order (deterministic). */
tw_status tw_mpnn_gradients(tw_mpnn *m, const tw_graph *gs, uint32_t count, const float *targets,
                            float *out_loss, float *out_grads);
/* Test hook: one graph's forward and backward pass (loss: the mean of the two
 * outputs' squared errors against target[2]) with the float32 values of the
 * kernels recorded before each bfloat16 rounding, so every product can be
 * checked on its own against the same bfloat16 operands.  out_trace holds
 * tw_mpnn_trace_floats() floats, each 64 x 64 block row-major [node][feature]:
 *   [0, 3*4096)        A H_l, l = 0..2
 *   [3*4096, 6*4096)   H_l Ws_l^T + (A H_l) Wn_l^T + b_l before the ReLU, l = 0..2
 *   then 256 floats    r[128] (sum and max readout), y[2]
 *   then 4096          dL/dH_3
 *   then 3*4096        dL/dZ_l, l = 0..2
 *   then 2*4096        dL/dZ_l Wn_l, l = 1, 2
 *   then 2*4096        dL/dH_l, l = 1, 2
 * out_grads (tw_mpnn_param_count() floats): the gradient of that loss. */
uint32_t tw_mpnn_trace_floats(void);
tw_status tw_mpnn_trace(tw_mpnn *m, const tw_graph *g, const float *target, float *out_trace, float *out_grads);

/* One AdamW step (beta 0.9 / 0.999, eps 1e-8; weight decay on the matrices
 * only) on the loss above; *out_loss (nullable) is the loss before the step. */
tw_status tw_mpnn_train_step(tw_mpnn *m, const tw_graph *gs, uint32_t count, const float *targets, float lr,
                             float weight_decay, float *out_loss);

/* Machine reference for the table insert (a diagnostic, not part of the
 * search): times random operations on a fresh device buffer of `bytes` bytes
 * (>= 4096, allocated and freed by the call) on `device`, with eight
 * 256-thread workgroups per compute unit like the expansion kernel.  mode 0:
 * one 16-byte load per operation, one in flight per lane (the probe of the
 * exact table); 1: one 64-bit compare-and-swap; 2: 16-byte loads, eight in
 * flight per lane; 3: as 0 with the nontemporal hint; 4: one 8-byte load;
 * 5: one 8-byte relaxed atomic load at system scope.  *out_seconds is the kernel time (HIP events) scaled to
 * exactly `count` operations.  TW_EINVAL on a bad argument, TW_ENOMEM if the
 * buffer does not fit, TW_EDEVICE on a HIP error. */
tw_status tw_probe_rate(int device, uint64_t bytes, uint64_t count, int mode, double *out_seconds);

const char *tw_status_str(tw_status s);
/* Message of the last failure on ctx (empty string if none); valid until the next call. */
const char *tw_last_error(const tw_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* TW_H */
