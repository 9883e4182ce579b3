/*
 * hipscc -- strongly connected components on one MI355X (gfx950) by the
 * BGSS randomized algorithm with vertical granularity control (VGC) and a
 * parallel hash-bag frontier.
 *
 * Paper: Wang, Dong, Gu, Sun, "Parallel Strong Connectivity Based on Faster
 * Reachability", SIGMOD 2023 (arXiv 2303.04934).
 *
 * C ABI.  Plain integers and pointers only.  Every pointer documented as
 * "device" must point to memory of the device the context was created on;
 * the caller owns it and the library never frees it.  "host" pointers are
 * ordinary CPU memory.  Calls are synchronous: they enqueue work on the
 * context's stream and wait for it before returning, so outputs are ready on
 * return.  Inputs are never modified.  A context is not thread safe; use one
 * per host thread.  No C++ exception crosses this interface.
 *
 * Errors: every call returns an scc_status; on failure scc_last_error(ctx)
 * returns a message that stays valid until the next call on that context.
 */
#ifndef HIPSCC_H
#define HIPSCC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t scc_status;
enum {
    SCC_OK = 0,
    SCC_EINVAL = -1,     /* bad argument (null pointer, bad size, bad option) */
    SCC_EGRAPH = -2,     /* the CSR failed validation */
    SCC_ENOMEM = -3,     /* device allocation failed */
    SCC_ECAPACITY = -4,  /* caller-provided output buffer too small */
    SCC_EHIP = -5,       /* a HIP runtime call failed */
    SCC_EPOLICY = -6,    /* malformed policy weights */
    SCC_EINTERNAL = -7   /* an internal invariant failed (a bug) */
};

typedef struct scc_ctx scc_ctx_t;

/* A directed graph G = (V, E), |V| = n, |E| = m (Section 2, notation), as a
 * CSR of out-arcs and the CSR of the transpose graph G^T (the backward search
 * runs on G^T, Section 2, "Reachability Search").  All four arrays are device
 * int32:
 *   out_off[n+1]: out_off[0] = 0, nondecreasing, out_off[n] = m;
 *   out_adj[m]:   targets in [0, n);
 *   in_off/in_adj: the same arc multiset, grouped by target.
 * 0 <= n < 2^31 and 0 <= m < 2^31.  Self loops and parallel arcs are allowed
 * (neither changes the SCCs). */
typedef struct {
    int32_t n;
    int32_t m;
    const int32_t *out_off;
    const int32_t *out_adj;
    const int32_t *in_off;
    const int32_t *in_adj;
} scc_graph_t;

/* Tunables.  Fill with scc_default_options() and change fields; passing NULL
 * means the defaults.  None of them changes a result, only work and rounds.
 *   tau          VGC budget: arcs a local search examines before it stops and
 *                hands its queue to the next frontier (Section 3.2).  Default
 *                2048: Section 3.2 ties the budget to the cost of scheduling a
 *                task, and a GPU round (launches plus host check) costs more
 *                than a multicore one, so the default sits above the paper's
 *                2^9, inside the range it finds insensitive (2^6..2^12).
 *                tau <= 1 disables local search (plain frontier BFS,
 *                Algorithm 2).
 *   beta         prefix-doubling multiplier for the source batches
 *                (Algorithm 1 doubles; Table 1 uses 1.5; any constant > 1
 *                keeps the bounds).  Default 2: fewer, larger batches mean
 *                fewer latency-bound rounds on the GPU.  Must be > 1.
 *   lambda_log2  log2 of the hash bag's first chunk (Table 1: 10 for tens of
 *                threads).  0 (default) = automatic: up to 2^20 slots, so that
 *                thousands of inserting wavefronts spread over many stripes.
 *   sigma        samples that trigger a hash bag chunk advance (Table 1: 50).
 *   kappa        stripe probes before an insert forces a chunk advance (each
 *                probe tries another random stripe of the current chunk;
 *                default 32, so that the sampled load estimate, not the probe
 *                limit, moves the chunk, as Section 3.3 intends).
 *   alpha        target load factor of a bag chunk (0 < alpha < 1).
 *   seed         seed of the random vertex permutation.
 *   policy       0 = fixed schedule, 1 = learned per-round policy (needs
 *                scc_policy_load; falls back to the fixed schedule otherwise),
 *                2 = exploration: a random budget class per round (for
 *                collecting training traces).
 *   dense        single-source search direction mode: -1 automatic,
 *                0 never pull, 1 always pull (Section 4.2).
 *   validate     1 = check the CSR (O(n + m)) before running.
 *   trim         1 = remove vertices of zero in- or out-degree first (4.1).
 *   table_init   reach table slots for the first multi-source batch (power of
 *                two); 0 = the sizing heuristic of Section 4.5.
 *   table_floor  the heuristic's floor as a fraction of the active vertices
 *                (Section 4.5 uses 0.3); the other term is 1.5 x the previous
 *                batch's pairs x the batch growth.  Default 1.2: a sparser
 *                table means fewer linear-probing steps, each a dependent
 *                load and CAS on the GPU, and HBM is plentiful; a smaller
 *                floor risks restarts on a larger table.  With first-source
 *                slots the table holds only a vertex's later pairs: the
 *                floor is halved, the pair term counts (g - 1) x the previous
 *                pairs + its table pairs (g the batch growth), a full table
 *                restarts four times as large, and each batch that restarted
 *                doubles the floor of the call's later batches (up to 16x).
 *   seeds_per_wave frontier entries a wavefront takes per fetch (1..64);
 *                0 = chosen from the frontier size.
 *   timing       bit mask over SCC_KERNEL_*: bit k brackets every launch of
 *                frontier kernel k with HIP events and reports its time and
 *                algorithmic bytes in the stats (each timed launch costs a
 *                little overhead, so time only what is needed; 0 = off).
 *   trace        1 = record one row per search round (read back with
 *                scc_trace_read); the host then checks every round.
 *   arcs_per_lane  arcs each lane of a wavefront has in flight per pass of
 *                a local-search step: 1, 2 or 4 (0 = default 1).  More arcs
 *                per lane shorten the chain of dependent memory accesses of a
 *                step but cost registers, hence resident wavefronts.
 *   beta_fast    batches grow by beta_fast instead of beta after a cheap
 *                batch: its frontiers (degree sums seen at host checks)
 *                never reached a sixteenth of the expand grid's lanes, or
 *                its sources reached fewer than 4 vertices each (per
 *                direction) and its frontiers never exceeded the lanes.  Its
 *                rounds were latency bound, so a larger batch costs little.
 *                After a batch that was also short (at most 4 rounds per
 *                direction) and cheap in pairs (fewer than 4 reached vertices
 *                per source and direction), the next batch grows by
 *                max(beta_fast, 64).  Any growth factor above 1 keeps
 *                Algorithm 1 correct.  A batch grown this way that overflows
 *                its reach table or frontier buffers is abandoned and taken
 *                again at beta growth.  Default 4; <= beta turns both off.
 *   vgc_fill     local search runs in rounds whose frontier has fewer arcs
 *                (entries x average degree) than vgc_fill x the lanes of the
 *                expand grid; a frontier above that keeps the GPU busy on its
 *                own and runs as a plain round (0 = default 2; < 0 = cut at
 *                one entry per wavefront).
 *   union_arcs_max  scc_labels_batched: most arcs one disjoint union of
 *                consecutive graphs may hold (0 = default 2^31 - 1, the int32
 *                arc-index limit).  A smaller value splits a batch into more
 *                unions; used to exercise the split on small batches.
 *   first_slot   1 (default) = multi-source searches claim each vertex's
 *                first pair in a per-vertex slot (4 bytes at the vertex, next
 *                to its label) and only later pairs in the reach table; 0 =
 *                every pair in the table (Section 4.3).  The slot replaces
 *                most random table probes with an access at the vertex
 *                itself (grid 10^4 x 10^4: 782 -> 722 ms per call).
 *   vgc_measure  what the VGC budget tau counts (Section 3.2 names
 *                alternatives to examined arcs): 0 = examined arcs (default),
 *                1 = new claims (generated reachability pairs, or visited
 *                vertices for a single source).
 *   ldd_beta     scc_cc: growth of the centre batches of the low-diameter
 *                decomposition per round (Section 5.1 uses 1.2; default).
 *   packed       with first_slot: 1 = the multi-source searches read packed
 *                per-vertex records {first arc, degree, label, first-source
 *                slot} of 16 bytes (one memory sector per claim instead of
 *                three), built once per call; 0 = separate arrays; -1
 *                (default) = records when more than half the vertices
 *                survive trimming (the build pass is then worth it).
 *   graph_rounds 1 = a block of sparse rounds between two host checks runs
 *                as one captured HIP graph, replayed when a block with the
 *                same round count and launch arguments comes again (cached
 *                per context); 0 (default) = one launch per kernel.  Not
 *                with timing, trace or the learned policy, and ignored by
 *                scc_labels_static.
 *   union_streams  scc_labels_batched: the batch is split into at least this
 *                many disjoint unions of consecutive graphs (balanced by
 *                arcs), run concurrently, each on a stream of its own driven
 *                by a host thread of its own (its state kept in a worker
 *                context that the calling context owns); long-diameter
 *                graphs leave most of the GPU idle in their latency-bound
 *                rounds, which the other unions' rounds then use.  1 = the
 *                unions run one after another on the context's stream; 0
 *                (default) = automatic (2).
 *   tau_single   VGC budget of single-source searches (the first SCC's
 *                search): 0 (default) = 4 x tau, or tau itself when tau <= 1.
 *                A single source has one narrow search to run, so a longer
 *                local search saves rounds without idling other work
 *                (measured: SQR 44.6 -> 40.9 ms, the 1000^2 torus 20.8 ->
 *                19.7 ms at 8192 against 2048). */
typedef struct {
    int32_t tau;
    float beta;
    int32_t lambda_log2;
    int32_t sigma;
    int32_t kappa;
    float alpha;
    uint64_t seed;
    int32_t policy;
    int32_t dense;
    int32_t validate;
    int32_t trim;
    int64_t table_init;
    int32_t seeds_per_wave;
    int32_t timing;
    int32_t trace;
    int32_t arcs_per_lane;
    float vgc_fill;
    float beta_fast;
    float table_floor;
    int32_t union_arcs_max;
    int32_t first_slot;
    int32_t vgc_measure;
    float ldd_beta;
    int32_t graph_rounds;
    int32_t packed;
    int32_t union_streams;
    int32_t tau_single;
} scc_options_t;

/* Frontier kernels timed with options.timing. */
#define SCC_KERNEL_EXPAND_SINGLE 0  /* sparse single-source expand round */
#define SCC_KERNEL_EXPAND_MULTI 1   /* multi-source expand round */
#define SCC_KERNEL_PULL 2           /* dense pull round */
#define SCC_KERNEL_HEAVY_SINGLE 3   /* edge-parallel pass, single-source lanes */
#define SCC_KERNEL_HEAVY_MULTI 4    /* edge-parallel pass, multi-source lanes */
#define SCC_KERNEL_EXTRACT 5        /* ExtractAll */
#define SCC_KERNEL_UNION 6          /* scc_cc: the union-find pass over the arcs */
#define SCC_KERNELS 7

/* Per-call statistics (host struct, written when non-NULL).  Times are
 * milliseconds measured with HIP events on the context's stream.  The five
 * phases follow the paper's breakdown (Section 4 / Figure 8): trimming,
 * first SCC (single-source searches), multi-search, hash table resizing and
 * labeling (relabel + canonicalisation). */
typedef struct {
    double ms_total, ms_trim, ms_first, ms_multi, ms_resize, ms_label;
    int64_t n, m;
    int64_t batches;          /* source batches that ran a search */
    int64_t rounds_first;     /* frontier rounds of the single-source search (both directions) */
    int64_t rounds_multi;     /* frontier rounds of all multi-source searches */
    int64_t dense_rounds;     /* rounds that ran in pull mode */
    int64_t entries_expanded; /* frontier / local-queue entries expanded */
    int64_t arcs_scanned;     /* adjacency slots read by searches */
    int64_t claim_attempts;   /* label-equal targets that were tried */
    int64_t claims;           /* successful claims = reachability pairs found */
    int64_t claims_table;     /* of those (first-source slots on), the pairs that went to the reach table */
    int64_t bag_inserts;      /* hash bag inserts */
    int64_t bag_chunk_advances;
    int64_t table_restarts;   /* searches re-run with a larger table */
    int64_t restart_rounds;   /* rounds of the attempts those restarts abandoned */
    int64_t trimmed;          /* vertices finished by trimming */
    int64_t n_scc;            /* number of SCCs (scc_labels only) */
    int64_t policy_calls;     /* rounds decided by the learned policy */
    int64_t policy_fallbacks; /* rounds where the policy output was unusable */
    int64_t bytes_alg;        /* algorithmic HBM bytes of the whole call */
    /* with options.timing: for the frontier kernels (SCC_KERNEL_*) the summed
     * event time of their launches, the number of launches and their
     * algorithmic bytes.  Expand and edge-parallel: frontier entry 8,
     * offsets 8 per expanded entry, per scanned arc 8 (multi: target id and
     * its label) or 4 (single: target id), per claim attempt 8 (multi: a
     * reach-record probe) or 4 (single: a visited word), per claim 8 or 4,
     * 8 per bag insert.  Pull: visited and
     * next words (n/4), offsets 8 per unvisited vertex, 8 per scanned arc
     * (target id + frontier word).  ExtractAll: 24 per extracted entry (bag
     * slot read, frontier write, the entry's offsets for the degree sum).
     * Union pass: 8 per arc (target id + its cluster), 12 per vertex
     * (offsets, cluster), 16 per link attempt (two finds' first parents). */
    double ms_kernel[SCC_KERNELS];
    int64_t launches_kernel[SCC_KERNELS];
    int64_t bytes_kernel[SCC_KERNELS];
} scc_stats_t;

/* Library version string (static storage). */
const char *scc_version(void);

/* Default options (the paper's Table 1 values where it gives one). */
scc_status scc_default_options(scc_options_t *opt);

/* Create a context on HIP device `device`.  `stream` is a hipStream_t to run
 * on (NULL: the context creates and owns one).  The context owns all scratch
 * memory; it grows on demand and is freed by scc_destroy. */
scc_status scc_create(scc_ctx_t **ctx, int device, void *stream);
void scc_destroy(scc_ctx_t *ctx);
const char *scc_last_error(const scc_ctx_t *ctx);

/* SCC labels (Algorithm 1 with Section 4's implementation details).
 * labels_out: device int32[n]; on return labels_out[v] is the minimum vertex
 * id of v's strongly connected component (the output of Section 2's problem
 * statement, made canonical).  Stats may be NULL. */
scc_status scc_labels(scc_ctx_t *ctx, const scc_graph_t *g, int32_t *labels_out, const scc_options_t *opt,
                      scc_stats_t *stats);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments and result as scc_labels, but every scratch buffer of the call
 * (per-vertex state, visited bitmaps, both reach tables, frontiers, hash
 * bags) is carved from one fixed device array of 512 MiB that the library
 * holds per device from load until the process ends; the call itself makes
 * no hipMalloc, hipFree or other allocating call (the context's own control
 * block and pinned host mirror were allocated by scc_create).
 * Limits:
 *   - about 1.5 million vertices with the default options (the carve takes
 *     roughly 340 bytes per vertex, rounded up to powers of two); a larger
 *     graph returns SCC_ECAPACITY before any work is queued;
 *   - reach tables stop at next_pow2(max(1024, 4n)) slots and frontiers at
 *     2n entries per round: a search that outgrows them returns
 *     SCC_ECAPACITY (scc_labels would grow them);
 *   - options.timing and options.trace must be 0 (they create events), and
 *     the stats carry no phase times.
 * Every call on a device shares that device's array and keeps the previous
 * call's contents: each call clears what must start empty, so calls in
 * sequence are independent, but calls that overlap on one GPU (from other
 * contexts, streams or threads) race and give undefined results. */
scc_status scc_labels_static(scc_ctx_t *ctx, const scc_graph_t *g, int32_t *labels_out, const scc_options_t *opt,
                             scc_stats_t *stats);

/* Reachability pairs (Section 2, "Reachability Search"; the MultiReach of
 * Algorithm 1).  dir = 0 searches G (out_*), dir = 1 searches G^T (in_*).
 * sources: device int32[k], distinct, with labels[s] >= 0.  labels: device
 * int32[n]; an arc (u, w) is used only if labels[u] == labels[w] (Algorithm 1
 * skips arcs whose endpoints have different labels); vertices with a negative
 * label are excluded.  Output: every pair (v, j) with sources[j] ~> v,
 * including (sources[j], j), exactly once, sorted ascending by (j, v) (the
 * sort runs on the device), written as pairs_out[2*i] = v,
 * pairs_out[2*i+1] = j (device int32[2 * capacity]).
 * *n_pairs (host) always receives the number of pairs; if it exceeds
 * capacity the call returns SCC_ECAPACITY and pairs_out is unspecified.
 * With k == 1 the single-source (visited-flag) search is used. */
scc_status scc_reach(scc_ctx_t *ctx, const scc_graph_t *g, int32_t dir, const int32_t *sources, int32_t k,
                     const int32_t *labels, int32_t *pairs_out, int64_t capacity, int64_t *n_pairs,
                     const scc_options_t *opt, scc_stats_t *stats);

/* SCC labels of G independent graphs in one pass (their disjoint union is
 * searched by the same kernels).  vtx_base and arc_base are host int64[G+1]
 * prefix sums of the graphs' vertex and arc counts.  Device arrays, graph g's
 * part stored contiguously:
 *   out_off/in_off: int32[vtx_base[G] + G]; graph g's n_g + 1 LOCAL offsets
 *                   start at index vtx_base[g] + g;
 *   out_adj/in_adj: int32[arc_base[G]]; graph g's arcs start at arc_base[g]
 *                   and hold LOCAL vertex ids in [0, n_g).
 * labels_out: device int32[vtx_base[G]]; graph g's labels start at
 * vtx_base[g] and are LOCAL ids (min local id of the SCC).  The total vertex
 * count must stay below 2^31; the total arc count may exceed it. */
scc_status scc_labels_batched(scc_ctx_t *ctx, int32_t G, const int64_t *vtx_base, const int64_t *arc_base,
                              const int32_t *out_off, const int32_t *out_adj, const int32_t *in_off,
                              const int32_t *in_adj, int32_t *labels_out, const scc_options_t *opt,
                              scc_stats_t *stats);

/* Connected components (Section 5.1, Algorithm 4, LDD-UF-JTB).  Only the
 * out-CSR of g is read (in_off / in_adj may be NULL).  A low-diameter
 * decomposition assigns every vertex to a cluster centre: centres are added
 * in random order in batches growing by options.ldd_beta per round, and
 * every round searches out from the frontier with VGC (budget options.tau)
 * and the hash bag; a concurrent union-find then merges the clusters joined
 * by an arc.  labels_out: device int32[n]; on return labels_out[v] is the
 * smallest vertex id of v's weakly connected component, i.e. of its
 * connected component when g is symmetric (every arc has its reverse), the
 * undirected graphs the paper runs this on.  Stats: ms_first = the
 * decomposition, ms_label = union-find and labels, rounds_first = its
 * search rounds, n_scc = the number of components, arcs_scanned and
 * claim_attempts include the union pass's arcs and link attempts. */
scc_status scc_cc(scc_ctx_t *ctx, const scc_graph_t *g, int32_t *labels_out, const scc_options_t *opt,
                  scc_stats_t *stats);

/* Least-element lists (Section 5.2, Algorithm 5).  Only the out-CSR of g is
 * read.  The vertices take a random total order (from options.seed); the
 * list of u holds every s with d(s, u) < d(k, u) for all k before s in the
 * order, d the distance along arcs from s to u (the undirected distance when
 * g is symmetric, the graphs the paper uses).  The order is processed in
 * batches of sizes 1, beta, beta^2, ... (options.beta; Algorithm 5 doubles);
 * each batch runs a multi-source BFS from its sources that claims pairs in a
 * reach table and keeps its frontier in the hash bag, and enters a vertex
 * only at a distance below the best one of earlier batches (no local search:
 * the BFS order is part of the result).  Outputs (device):
 *   order_out  int32[n] (may be NULL): order_out[i] = the vertex at position i;
 *   loff       int64[n+1]: u's entries are [loff[u], loff[u+1]);
 *   src_out, dist_out  int32[capacity]: entry i = (source vertex, distance),
 *              each list in order of the sources' positions, so its distances
 *              decrease and it ends with (u, 0).
 * *n_entries (host) always receives the total; above capacity the call
 * returns SCC_ECAPACITY (loff, src_out, dist_out unspecified).  Stats:
 * batches, rounds_multi = BFS rounds, table_restarts = batches re-run on a
 * larger table, ms_multi = the batches, ms_label = the final lists. */
scc_status scc_le_lists(scc_ctx_t *ctx, const scc_graph_t *g, int32_t *order_out, int64_t *loff, int32_t *src_out,
                        int32_t *dist_out, int64_t capacity, int64_t *n_entries, const scc_options_t *opt,
                        scc_stats_t *stats);

/* Load the learned round policy: a float32 MLP 5 -> 32 -> 32 -> 8 with ReLU,
 * weights as one host blob [W1(32x5), b1(32), W2(32x32), b2(32), W3(8x32),
 * b3(8)] (row-major, out x in), n_floats = 1512.  The 8 outputs score
 * 4 VGC budgets x 2 frontier modes for the next round.  The blob is copied.
 * Non-finite weights are rejected with SCC_EPOLICY. */
scc_status scc_policy_load(scc_ctx_t *ctx, const float *weights, int64_t n_floats);

/* Evaluate the loaded policy on host features (float32[rows*5]) with the
 * device inference kernel; writes float32[rows*8] scores to host `scores`.
 * Test hook for parity with a CPU forward pass. */
scc_status scc_policy_eval(scc_ctx_t *ctx, const float *feats, int32_t rows, float *scores);

/* Per-round trace of the last call made with options.trace = 1: one row of
 * SCC_TRACE_FIELDS floats per round and search lane:
 *   0 kind (0 single-source sparse, 1 single-source dense, 2 multi-source)
 *   1..5 the policy features before the round (log2(1 + frontier size),
 *        log2(1 + frontier degree sum), visited fraction, log2(1 + round),
 *        log2(1 + deepest local search of the previous round))
 *   6 VGC budget used, 7 round time in ms (events), 8 entries claimed in
 *   the round, 9 frontier size after the round, 10 batch index, 11 n.
 * out: host float[cap * SCC_TRACE_FIELDS]; *n_rows receives the row count
 * (rows beyond cap are dropped). */
#define SCC_TRACE_FIELDS 12
scc_status scc_trace_read(scc_ctx_t *ctx, float *out, int64_t cap, int64_t *n_rows);

/* Hash bag self test (Section 3.3).  keys: device uint64[n] (any values);
 * every key is inserted by a concurrent wave-aggregated Insert in `rounds`
 * rounds of the round-robin split keys[i] -> round i % rounds; after each
 * round ExtractAll appends the bag's content to out (device uint64[n]).
 * *n_out (host) receives the number extracted, which equals n when the
 * structure is correct.  Stats report chunk advances.  Test hook. */
scc_status scc_bag_selftest(scc_ctx_t *ctx, const uint64_t *keys, int64_t n, int32_t rounds, uint64_t *out,
                            int64_t *n_out, const scc_options_t *opt, scc_stats_t *stats);

/* Statistics of the last scc_bag_selftest on this context, for the bounds of
 * Theorem 1 (Section 3.3, Appendix A): with alpha = 1/2 a chunk is left at a
 * load within [1/4, 3/4] w.h.p., and s elements occupy a prefix of
 * O(s + lambda) slots.  rows: host double[4 * cap], one row (round, chunk,
 * load, cause) per chunk that was left during a round, load = its filled
 * slots / its size when that round's ExtractAll ran (late inserts of waves
 * that read the old chunk included), cause = 0 when its samples reached
 * sigma, 1 when an insert exceeded kappa stripe probes; *n_rows receives the
 * row count.  prefix: host
 * int64[prefix_cap], the used prefix (tail of the current chunk) at each
 * round's ExtractAll; *n_rounds receives the round count.  Test hook. */
scc_status scc_bag_stats(scc_ctx_t *ctx, double *rows, int64_t cap, int64_t *n_rows, int64_t *prefix,
                         int64_t prefix_cap, int64_t *n_rounds);

#ifdef __cplusplus
}
#endif

#endif /* HIPSCC_H */
