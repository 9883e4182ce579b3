// hipscc kernels (gfx950).  All kernels are launched by runtime.hip.
#pragma once

#include "bag.h"
#include "device.h"
#include "policy.h"

namespace hipscc {

enum { kCtrSeeds = 0, kCtrExpanded, kCtrArcs, kCtrAttempts, kCtrClaims, kCtrInserts, kNumCtr };
constexpr int kCtrStripes = 32;
// Counter kinds: the work of each frontier kernel (expand single-source,
// expand multi-source, pull, edge-parallel single- and multi-source).
enum { kKindExpandSingle = 0, kKindExpandMulti = 1, kKindPull = 2, kKindHeavySingle = 3, kKindHeavyMulti = 4,
       kKindUnion = 5, kNumKinds = 6 };

// Round control of one search lane (one direction of a search), in device
// memory.  Rounds alternate between parity 0 and 1 so that one round's
// counters can be reset while the next round's are in use.
struct RoundCtl {
    uint32_t nF[2];        // frontier sizes
    uint32_t heavy_n[2];   // items deferred to the edge-parallel kernel
    uint32_t err;          // kErr* bits
    uint32_t rounds;       // rounds with a non-empty frontier
    uint32_t listpos;      // bitmap -> list conversion cursor
    uint32_t pad;
    unsigned long long fdeg[2]; // summed degree of the frontier of each parity (0: not known)
    unsigned long long claims;  // pairs (or vertices) claimed by this lane's search (folded at round end)
    uint32_t lsdepth[2];        // deepest local search (steps) of the round of each parity (folded)
    uint32_t tau_cur;           // VGC budget of the next round when a policy sets it
    uint32_t mode_pref;         // policy's preferred mode for the next round (0 sparse, 1 dense)
    uint32_t policy_calls;
    uint32_t policy_fallbacks;
    uint32_t snap_rounds, snap_depth;  // trace snapshot of the round's inputs
    unsigned long long snap_nf, snap_fdeg, snap_claims;
    uint32_t pad2;
    unsigned long long tclaims;  // of the claims, those that went to the reach table (first-source slots on)
};

// Striped round counters of one lane.  Atomics on one address from many
// blocks serialise in the L2, so blocks spread them over kStripes cache
// lines (block b uses line b % kStripes); one thread folds the lines into
// RoundCtl when the round ends.
constexpr int kStripes = 16;
struct alignas(128) StripeLine {
    unsigned long long claims;  // cumulative over the search
    uint32_t depth;             // this round's deepest local search
    uint32_t nf;                // this round's next-frontier size (dense rounds)
    uint32_t work[2];           // dynamic group counters of the expand kernel, per parity
    unsigned long long tclaims; // cumulative claims that went to the reach table
    uint32_t pad[24];
};
static_assert(sizeof(StripeLine) == 128, "one cache line per stripe");
struct LaneStripes {
    StripeLine s[kStripes];
};

// Zeroes every stripe (all threads of one block take part).
__device__ __forceinline__ void stripes_clear(LaneStripes *ls) {
    uint32_t *w = reinterpret_cast<uint32_t *>(ls);
    for (uint32_t i = threadIdx.x; i < sizeof(LaneStripes) / 4; i += blockDim.x) w[i] = 0u;
}

// Round-end fold (one thread): claims and the round's local-search depth
// into RoundCtl; this parity's work counters and the depth lines restart.
__device__ __forceinline__ void stripes_fold(RoundCtl *rc, LaneStripes *ls, int par) {
    unsigned long long c = 0, tc = 0;
    uint32_t d = 0;
    for (int i = 0; i < kStripes; i++) {
        StripeLine &L = ls->s[i];
        c += L.claims;
        tc += L.tclaims;
        d = L.depth > d ? L.depth : d;
        L.depth = 0;
        L.work[par] = 0;
    }
    rc->claims = c;
    rc->tclaims = tc;
    rc->lsdepth[par] = d;
}

// Call-level values shared by all lanes.
struct Shared {
    uint32_t k;            // sources selected for the batch
    uint32_t first;        // first active permutation position (batch 1)
    uint32_t emit;         // pairs emitted by scc_reach (entries logged by a LE-lists batch)
    uint32_t bad;          // validation flags
    uint32_t max_deg;      // largest out- or in-degree of the graph (0: not known yet)
    unsigned long long cursor;  // LE-lists: entries in the list log
};

// Call-level counts that whole grids add to, striped like LaneStripes (block
// b adds to line b % kStripes); the host sums the lines.
struct alignas(128) CountLine {
    uint32_t fin;          // vertices finished so far (all batches)
    uint32_t trimmed;      // vertices finished by trimming
    uint32_t nscc;         // canonical representatives
    uint32_t pad[29];
};
static_assert(sizeof(CountLine) == 128, "one cache line per stripe");
struct CountStripes {
    CountLine s[kStripes];
};

// Work counters, striped over kCtrStripes slots to spread the atomics.
struct Counters {
    unsigned long long c[kCtrStripes][kNumKinds][8];
};

constexpr uint32_t kErrTable = 1u;      // reach table probe limit exceeded
constexpr uint32_t kErrCapacity = 2u;   // frontier / heavy list capacity exceeded
constexpr uint32_t kErrUnfinished = 4u; // a vertex had no SCC key at the end

constexpr int kQcap = 256;  // local queue entries per wave (LDS)
// First-source slot claims flag their vertex's granule of 2^kDirtyLog2
// vertices (a plain byte store, nothing waits for it), so the per-vertex
// relabel visits only granules that a batch touched: a vertex has table pairs
// only if its slot is taken, and sums and finish marks only if it has pairs.
constexpr int kDirtyLog2 = 12;
constexpr int kQmask = kQcap - 1;
constexpr int kStepArcs = 256;  // arcs a wave commits to per local-search step
constexpr int kHeavyChunk = 4096;  // arcs per edge-parallel work item

enum { kSingle = 0, kMulti = 1, kMultiFirst = 2, kLdd = 3, kLe = 4, kMultiRec = 5 };

// One reachability search (one direction).  kSingle claims vertices in a
// visited bitmap whose bits were pre-set for every vertex outside the search's
// subproblem; kMulti claims (vertex, source) pairs in the reach table;
// kMultiFirst claims the first pair of each vertex in a per-vertex slot
// (first[v] = source index) and only later pairs in the reach table.  kLdd
// kMultiRec is kMultiFirst on packed per-vertex records {first arc, degree,
// label, first-source slot} (16 bytes, one memory sector per claim instead
// of the label, slot and offsets arrays).  kLdd
// is kSingle for the low-diameter decomposition of Algorithm 4: an entry
// carries its cluster centre in place of the source index, and a claim also
// records owner[w] = centre.  kLe is the pruned multi-BFS of Algorithm 5 (LE
// lists): pairs in the table, but an arc (u, w) is followed at distance
// level + 1 only while that beats delta(w) (label holds delta), and there is
// no local search (the BFS order matters).
struct Search {
    const int32_t *off;
    const int32_t *adj;
    const int32_t *label;   // kMulti: arc (u, w) is used iff label[w] == label of the source
    uint32_t *vis;          // kSingle
    uint64_t *table;        // kMulti
    int32_t *first;         // kMultiFirst: per-vertex first-source slot (-1 = empty)
    int4 *rec;              // kMultiRec: per-vertex {first arc, degree, label, first-source slot}
    uint8_t *dirty;         // first-source slots: granule flags (null: none kept)
    int32_t *owner;         // kLdd: cluster centre of each claimed vertex
    int32_t level;          // kLe: distance of the entries this round expands
    // kLe: ExtractAll also logs each new frontier entry (pair key, level + 1)
    // at position emit + its frontier index (null: not logged)
    uint64_t *lkeys;
    int32_t *ldist;
    uint64_t lcap;
    uint32_t lkbits;
    Shared *lsh;
    uint64_t tmask;
    uint32_t probe_limit;
    const int32_t *srclab;  // kMulti: label of source j
    uint64_t *F;            // packed frontier (read by expand, rewritten by extract)
    uint64_t *heavy;        // deferred high-degree items (entry, chunk) pairs
    uint64_t fcap;          // capacity of F (entries)
    uint64_t hcap;          // capacity of heavy (items)
    Bag bag;
    RoundCtl *rc;
    LaneStripes *ls;
    Counters *cn;
    int32_t kind;           // counter kind of the expand kernel
    int32_t par;
    int32_t tau;            // <= 1: plain frontier BFS
    int32_t seeds;          // 0: automatic
    int32_t heavy_deg;
    uint32_t vgc_cut;       // local search only while the frontier has fewer entries than this ...
    unsigned long long vgc_arcs;  // ... or, when its degree sum is known, fewer arcs than this
    uint32_t tau_from_rc;   // 1: the budget of each round is rc->tau_cur (set by the policy)
    const float *policy_w;  // non-null: ExtractAll's last block runs the policy for the next round
    float nsub;             // subproblem size (policy feature)
    uint32_t fallback_tau;  // budget when the policy's scores are unusable
    int32_t measure;        // what the budget counts: 0 examined arcs, 1 new claims (pairs / visited vertices)
};

// ------------------------------------------------------------- utilities ----
__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u64(uint64_t *p, uint64_t n, uint64_t v) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Block-wide sum of per-thread counts, one atomic per block.  Every thread
// of the block must call it.
__device__ __forceinline__ void block_add_u32(uint32_t *ctr, uint32_t x) {
    __shared__ uint32_t part[kWavesPerBlock];
    x = wave_sum_u32(x);
    if (lane_id() == 0) part[threadIdx.x / kWave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kWavesPerBlock; w++) t += part[w];
        if (t) atomicAdd(ctr, t);
    }
}

// Block-wide maximum of per-thread values, one atomic per block.  Every
// thread of the block must call it.
__device__ __forceinline__ void block_max_u32(uint32_t *ctr, uint32_t x) {
    __shared__ uint32_t m;
    if (threadIdx.x == 0) m = 0;
    __syncthreads();
    if (x) atomicMax(&m, x);
    __syncthreads();
    if (threadIdx.x == 0 && m) atomicMax(ctr, m);
}

// Block-wide reservation: wave w of the block asks for cnt slots (the value
// of lane 0 counts) and gets the first of its own range; one atomic per
// block.  Every thread of the block must call it.
__device__ __forceinline__ uint32_t block_reserve(uint32_t *ctr, uint32_t cnt) {
    __shared__ uint32_t want[kWavesPerBlock];
    __shared__ uint32_t base_s;
    const int wv = threadIdx.x / kWave;
    if (lane_id() == 0) want[wv] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kWavesPerBlock; w++) t += want[w];
        base_s = t ? atomicAdd(ctr, t) : 0u;
    }
    __syncthreads();
    uint32_t b = base_s;
    for (int w = 0; w < wv; w++) b += want[w];
    __syncthreads();  // want/base_s are rewritten by the next call
    return b;
}

// Block-wide flush of the kNumCtr work counters into one stripe.  Returns, on
// thread i < kNumCtr, the block's total of counter i.
__device__ __forceinline__ unsigned long long block_flush_ctr(unsigned long long *dst, unsigned long long (&c)[kNumCtr]) {
    __shared__ unsigned long long part[kWavesPerBlock][kNumCtr];
    // a lane's own counts stay far below 2^32 within one launch
#pragma unroll
    for (int i = 0; i < kNumCtr; i++) c[i] = wave_sum_u32((uint32_t)c[i]);
    if (lane_id() == 0)
        for (int i = 0; i < kNumCtr; i++) part[threadIdx.x / kWave][i] = c[i];
    __syncthreads();
    unsigned long long t = 0;
    if (threadIdx.x < kNumCtr) {
        for (int w = 0; w < kWavesPerBlock; w++) t += part[w][threadIdx.x];
        if (t) atomicAdd(&dst[threadIdx.x], t);
    }
    return t;
}

// ------------------------------------------------------------------ trim ----
// Section 4.1: a vertex with zero in- or out-degree is a singleton SCC.
// Finished vertices store ~key (negative); key = v here.
// It also writes the first search's visited bitmaps (both directions): the
// trimmed vertices are the ones outside its subproblem (label 0), so they are
// pre-set; the source's own bit is set when it is seeded.  A wave covers 64
// consecutive vertices, i.e. two bitmap words.
__global__ void k_trim(int32_t n, const int32_t *out_off, const int32_t *in_off, int32_t *label, int32_t do_trim,
                       uint32_t *vis0, uint32_t *vis1, CountStripes *cs, Shared *sh) {
    uint32_t cnt = 0, dmax = 0;
    const int lane = lane_id();
    for (int64_t v0 = blockIdx.x * (int64_t)blockDim.x; v0 < n; v0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = v0 + threadIdx.x;
        bool t = true;  // past the end: blocked
        if (v < n) {
            const int32_t dout = out_off[v + 1] - out_off[v], din = in_off[v + 1] - in_off[v];
            dmax = max(dmax, (uint32_t)max(dout, din));
            t = do_trim && (dout == 0 || din == 0);
            label[v] = t ? ~(int32_t)v : 0;
            cnt += t;
        }
        const uint64_t m = ballot(t);
        if ((lane == 0 || lane == 32) && v < n) {
            const uint32_t bits = lane == 0 ? (uint32_t)m : (uint32_t)(m >> 32);
            vis0[v >> 5] = bits;
            vis1[v >> 5] = bits;
        }
    }
    block_add_u32(&cs->s[blockIdx.x % kStripes].trimmed, cnt);
    block_max_u32(&sh->max_deg, dmax);
}

// Largest out-degree (one atomic per block), for searches that skip trimming.
__global__ void k_max_deg(int32_t n, const int32_t *off, Shared *sh) {
    uint32_t dmax = 0;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        dmax = max(dmax, (uint32_t)(off[v + 1] - off[v]));
    block_max_u32(&sh->max_deg, dmax);
}

// ----------------------------------------------------- source selection ----
// Batch 1 of Algorithm 1 is one random vertex; among active vertices, take the
// first one in permutation order.  Scans positions [p0, p1); one atomic per
// block after a block-wide minimum.
__global__ void k_first_active(Perm P, uint32_t p0, uint32_t p1, const int32_t *label, Shared *sh) {
    __shared__ uint32_t part[kWavesPerBlock];
    if (p0 > 0 && ld_relaxed(&sh->first) < p0) return;  // an earlier range already found one
    uint32_t best = 0xffffffffu;
    for (uint64_t j = p0 + blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < p1; j += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t v = perm_apply(P, (uint32_t)j);
        if (label[v] >= 0) {
            best = (uint32_t)j;
            break;  // later positions of this thread are larger
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const uint32_t o = (uint32_t)__shfl_xor((int)best, d, kWave);
        best = o < best ? o : best;
    }
    if (lane_id() == 0) part[threadIdx.x / kWave] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t b = part[0];
        for (int w = 1; w < kWavesPerBlock; w++) b = part[w] < b ? part[w] : b;
        if (b != 0xffffffffu) atomicMin(&sh->first, b);
    }
}

// The same selection for a long range, by a coalesced scan over the vertices:
// an active vertex is a source when its permutation position (perm_invert)
// falls in [p0, p1).  Reading every label in order costs 4n bytes, less than
// gathering the range's labels in random order once the range exceeds about
// n/16 positions (one cache sector per position).
// The inverse permutation is computed once per call: the first scan (build)
// inverts every active vertex and stores its position in invp, later scans
// read them.  A finished vertex never becomes active again, so the vertices a
// later scan asks for are a subset of those the build stored.
// Output slots come from one counter (the batch's source count), and
// same-address atomics serialise (about 11 ns each on MI355X), so a block
// reserves once per kScanPer x 256 vertices: each thread keeps the labels of
// its kScanPer vertices in registers until the block's reservation is made.
constexpr int kScanPer = 16;
__global__ __launch_bounds__(kBlock) void k_select_scan(Perm P, uint32_t p0, uint32_t p1, int32_t n,
                                                        const int32_t *label, int32_t *srcvert, int32_t *srclab,
                                                        Shared *sh, uint32_t *invp, bool build) {
    __shared__ uint32_t part[kWavesPerBlock];
    __shared__ uint32_t base_s;
    const int lane = lane_id();
    const int wv = threadIdx.x / kWave;
    const int64_t tile = (int64_t)kBlock * kScanPer;
    for (int64_t t0 = (int64_t)blockIdx.x * tile; t0 < n; t0 += (int64_t)gridDim.x * tile) {
        int32_t lab[kScanPer];
        uint32_t act = 0;
#pragma unroll
        for (int r = 0; r < kScanPer; r++) {
            const int64_t v = t0 + (int64_t)r * kBlock + threadIdx.x;
            int32_t l = -1;
            if (v < n) {
                l = label[v];
                if (l >= 0) {
                    uint32_t j;
                    if (build) {
                        j = perm_invert(P, (uint32_t)v);
                        invp[v] = j;
                    } else {
                        j = invp[v];
                    }
                    if (j < p0 || j >= p1) l = -1;
                }
            }
            lab[r] = l;
            act |= (l >= 0 ? 1u : 0u) << r;
        }
        const int cnt = __popc(act);
        const int incl = wave_incl_scan(cnt);
        if (lane == kWave - 1) part[wv] = (uint32_t)incl;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t tsum = 0;
            for (int w = 0; w < kWavesPerBlock; w++) tsum += part[w];
            base_s = tsum ? atomicAdd(&sh->k, tsum) : 0u;
        }
        __syncthreads();
        uint32_t pos = base_s + (uint32_t)(incl - cnt);
        for (int w = 0; w < wv; w++) pos += part[w];
        __syncthreads();  // part/base_s are rewritten next iteration
#pragma unroll
        for (int r = 0; r < kScanPer; r++) {
            if ((act >> r) & 1u) {
                srcvert[pos] = (int32_t)(t0 + (int64_t)r * kBlock + threadIdx.x);
                srclab[pos] = lab[r];
                pos++;
            }
        }
    }
}

// Sources of one batch: the active vertices among permutation positions
// [p0, p1) (Algorithm 1: F = P_i intersect V').  Reserves output slots like
// k_select_scan, once per kScanPer x 256 positions.
__global__ __launch_bounds__(kBlock) void k_select_sources(Perm P, uint32_t p0, uint32_t p1, const int32_t *label,
                                                           int32_t *srcvert, int32_t *srclab, Shared *sh) {
    __shared__ uint32_t part[kWavesPerBlock];
    __shared__ uint32_t base_s;
    const int lane = lane_id();
    const int wv = threadIdx.x / kWave;
    const int64_t tile = (int64_t)kBlock * kScanPer;
    for (int64_t t0 = (int64_t)p0 + (int64_t)blockIdx.x * tile; t0 < (int64_t)p1; t0 += (int64_t)gridDim.x * tile) {
        int32_t vs[kScanPer], lab[kScanPer];
        uint32_t act = 0;
#pragma unroll
        for (int r = 0; r < kScanPer; r++) {
            const int64_t j = t0 + (int64_t)r * kBlock + threadIdx.x;
            vs[r] = -1;
            lab[r] = -1;
            if (j < (int64_t)p1) {
                vs[r] = (int32_t)perm_apply(P, (uint32_t)j);
                lab[r] = label[vs[r]];
            }
            act |= (lab[r] >= 0 ? 1u : 0u) << r;
        }
        const int cnt = __popc(act);
        const int incl = wave_incl_scan(cnt);
        if (lane == kWave - 1) part[wv] = (uint32_t)incl;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t tsum = 0;
            for (int w = 0; w < kWavesPerBlock; w++) tsum += part[w];
            base_s = tsum ? atomicAdd(&sh->k, tsum) : 0u;
        }
        __syncthreads();
        uint32_t pos = base_s + (uint32_t)(incl - cnt);
        for (int w = 0; w < wv; w++) pos += part[w];
        __syncthreads();  // part/base_s are rewritten next iteration
#pragma unroll
        for (int r = 0; r < kScanPer; r++) {
            if ((act >> r) & 1u) {
                srcvert[pos] = vs[r];
                srclab[pos] = lab[r];
                pos++;
            }
        }
    }
}

// ---------------------------------------------------------- reach claims ----
__device__ __forceinline__ bool claim_bit(uint32_t *vis, int32_t w) {
    uint32_t bit = 1u << (w & 31);
    uint32_t *p = vis + (w >> 5);
    if (ld_relaxed(p) & bit) return false;
    return (atomicOr(p, bit) & bit) == 0;
}

// 1: new pair claimed; 0: pair already present; -1: probe limit exceeded.
__device__ __forceinline__ int claim_pair(uint64_t *T, uint64_t mask, uint32_t limit, uint64_t key) {
    uint64_t h = mix64(key) & mask;
    for (uint32_t p = 0; p <= limit; p++) {
        uint64_t cur = ld_relaxed64(T + h);
        if (cur == key) return 0;
        if (cur == kEmpty64) {
            unsigned long long old = atomicCAS((unsigned long long *)(T + h), (unsigned long long)kEmpty64,
                                               (unsigned long long)key);
            if (old == kEmpty64) return 1;
            if (old == key) return 0;
        }
        h = (h + 1) & mask;
    }
    return -1;
}

// A pair claim with the inline first-source slot: the slot of w holds the
// first source that reached w; a pair of any other source goes to the table.
// Returns like claim_pair, except that a new pair claimed in the table
// returns 2.
__device__ __forceinline__ int claim_pair_slot(int32_t *slot, uint64_t *T, uint64_t mask, uint32_t limit, int32_t w,
                                               uint32_t src) {
    const int32_t f = (int32_t)ld_relaxed(reinterpret_cast<const uint32_t *>(slot));
    if (f == (int32_t)src) return 0;
    if (f == -1) {
        const int32_t old = atomicCAS(slot, -1, (int32_t)src);
        if (old == -1) return 1;
        if (old == (int32_t)src) return 0;
    }
    const int c = claim_pair(T, mask, limit, pair_key(w, src));
    return c == 1 ? 2 : c;
}
__device__ __forceinline__ int claim_pair_first(int32_t *first, uint64_t *T, uint64_t mask, uint32_t limit, int32_t w,
                                                uint32_t src) {
    return claim_pair_slot(first + w, T, mask, limit, w, src);
}
// The first-source slot of vertex v in a slot array of the given stride
// (1: plain slots; 4: the last field of packed records).
__device__ __forceinline__ int32_t *slot_of(int32_t *base, int32_t stride, int64_t v) { return base + stride * v; }

__device__ __forceinline__ bool table_contains(const uint64_t *T, uint64_t mask, uint32_t limit, uint64_t key) {
    uint64_t h = mix64(key) & mask;
    for (uint32_t p = 0; p <= limit; p++) {
        uint64_t cur = T[h];
        if (cur == key) return true;
        if (cur == kEmpty64) return false;
        h = (h + 1) & mask;
    }
    return false;
}

// The single source of a search: s_fixed if >= 0, else the vertex at the
// first active permutation position (or -1 when there is none).
__device__ __forceinline__ int32_t single_source(int32_t s_fixed, const Shared *sh, Perm P) {
    if (s_fixed >= 0) return s_fixed;
    const uint32_t j = sh->first;
    return j < P.n ? (int32_t)perm_apply(P, j) : -1;
}

// Seed the search: single source.  Bit v of vis = "not available" (outside the
// subproblem L), plus the source itself, which is claimed up front.
__global__ void k_premark(int32_t n, const int32_t *label, int32_t L, int32_t s_fixed, const Shared *sh, Perm P,
                          uint32_t *vis) {
    const int32_t s = single_source(s_fixed, sh, P);
    for (int64_t v0 = blockIdx.x * (int64_t)blockDim.x; v0 < n; v0 += (int64_t)gridDim.x * blockDim.x) {
        int64_t v = v0 + threadIdx.x;
        bool blocked = v >= n || label[v] != L || v == s;
        uint64_t m = ballot(blocked);
        int l = lane_id();
        // lanes 0 and 32 write the two 32-bit words covering this wave's 64 vertices
        int64_t wbase = (v0 + (threadIdx.x & ~63)) >> 5;
        if (l == 0 && (wbase << 5) < n) vis[wbase] = (uint32_t)m;
        if (l == 32 && ((wbase + 1) << 5) < n) vis[wbase + 1] = (uint32_t)(m >> 32);
    }
}

__global__ void k_seed_single(int32_t s_fixed, const Shared *sh, Perm P, uint64_t *F, RoundCtl *rc,
                              LaneStripes *ls, uint32_t *vis) {
    if (blockIdx.x == 0) stripes_clear(ls);
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int32_t s = single_source(s_fixed, sh, P);
        if (s >= 0) {
            F[0] = pair_key(s, 0);
            vis[s >> 5] |= 1u << (s & 31);  // the source is claimed up front
        }
        rc->nF[0] = s >= 0 ? 1u : 0u;
        rc->nF[1] = 0;
        rc->heavy_n[0] = rc->heavy_n[1] = 0;
        rc->fdeg[0] = rc->fdeg[1] = 0;
        rc->claims = 0;
        rc->rounds = 0;
        rc->err = 0;
    }
}

// Multi-source seed of one or two lanes (blockIdx.y = lane): claim (s_j, j)
// in the lane's reach table and put it in its frontier.
struct SeedArgs {
    uint64_t *T[2];
    int32_t *first[2];      // non-null: the lane claims first pairs in per-vertex slots
    int32_t fstride[2];     // their stride in int32 (1 plain slots, 4 packed records)
    uint8_t *dirty;         // granule flags of claimed slots (may be null)
    uint64_t mask[2];
    uint64_t *F[2];
    RoundCtl *rc[2];
    LaneStripes *ls[2];
};

__global__ void k_seed_multi(const int32_t *srcvert, const Shared *sh, SeedArgs A, uint32_t limit) {
    const int l = blockIdx.y;
    RoundCtl *rc = A.rc[l];
    if (blockIdx.x == 0) stripes_clear(A.ls[l]);
    const uint32_t k = sh->k;
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < k; j += gridDim.x * blockDim.x) {
        uint64_t key = pair_key(srcvert[j], j);
        const int c = A.first[l] ? claim_pair_slot(slot_of(A.first[l], A.fstride[l], srcvert[j]), A.T[l], A.mask[l],
                                                   limit, srcvert[j], j)
                                 : claim_pair(A.T[l], A.mask[l], limit, key);
        if (c < 0) atomicOr(&rc->err, kErrTable);
        if (c == 1 && A.first[l] && A.dirty) A.dirty[srcvert[j] >> kDirtyLog2] = 1;
        A.F[l][j] = key;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        rc->nF[0] = k;
        rc->nF[1] = 0;
        rc->heavy_n[0] = rc->heavy_n[1] = 0;
        rc->fdeg[0] = rc->fdeg[1] = 0;
        rc->rounds = 0;
    }
}

// Start of a multi-source batch: both lanes' round state and the batch's
// source count back to zero (one small launch).
__global__ void k_batch_reset(Shared *sh, RoundCtl *rc0, RoundCtl *rc1) {
    uint32_t *a = reinterpret_cast<uint32_t *>(rc0);
    uint32_t *b = reinterpret_cast<uint32_t *>(rc1);
    for (uint32_t i = threadIdx.x; i < sizeof(RoundCtl) / 4; i += blockDim.x) {
        a[i] = 0u;
        b[i] = 0u;
    }
    if (threadIdx.x == 0) sh->k = 0;
}

// ---------------------------------------------------------------- expand ----
// One frontier round with vertical granularity control (Section 3.1-3.2).
//
// Each wavefront is one task: it takes a group of frontier entries and runs
// one bounded local search seeded with all of them.  Its FIFO local queue
// lives in LDS; each step the wave takes whole entries from the queue head
// (as many as fit in kStepArcs arcs), spreads their arcs over its 64 lanes,
// and claims the targets.  Every examined arc counts against the task's
// budget tau, successful or not (Section 3.2).  Newly claimed entries go to
// the local queue while it has room, otherwise straight to the hash bag.
// When the budget is spent or the queue is empty, what is left in the queue
// is inserted into the bag, i.e. the next frontier (Section 3.2).  With
// tau <= 1, or when the frontier's arcs already keep every lane busy, nothing
// is searched locally and this is one plain round (Algorithm 2/3).  Entries
// with more than heavy_deg arcs are deferred to k_expand_heavy, which spreads
// one adjacency list over the whole grid (Section 3.2: vertices with more
// than tau neighbours are processed edge-parallel).
//
// A local search is a chain of dependent memory accesses, one level per step,
// so its latency is the critical path of a round.  Queue entries therefore
// carry their adjacency range and label, fetched when the entry is claimed
// in parallel with the claim itself, and a claim issues the target's label,
// its first reach-table probe and its offsets together.
template <int MODE, int ILP>
__device__ __forceinline__ void expand_round(const Search &S, uint32_t bid, uint32_t nblk) {
    constexpr bool PAIRS = MODE == kMulti || MODE == kMultiFirst || MODE == kLe || MODE == kMultiRec;
    constexpr bool FIRST = MODE == kMultiFirst || MODE == kMultiRec;
    constexpr bool REC = MODE == kMultiRec;
    __shared__ uint64_t Qk[kWavesPerBlock][kQcap];                 // (vertex, source) keys
    __shared__ int2 Qr[kWavesPerBlock][kQcap];                     // (first arc, degree)
    __shared__ int32_t Ql[kWavesPerBlock][PAIRS ? kQcap : 1];      // entry's label (multi-source)
    __shared__ int32_t Sx[kWavesPerBlock][4][kWave];
    const int wv = threadIdx.x / kWave;
    const int lane = lane_id();
    uint64_t *Q = Qk[wv];
    int2 *R = Qr[wv];
    int32_t *QL = Ql[wv];
    int32_t *sexcl = Sx[wv][0];
    int32_t *sbeg = Sx[wv][1];
    int32_t *ssrc = Sx[wv][2];
    int32_t *slab = Sx[wv][3];
    RoundCtl *rc = S.rc;
    uint32_t nF = ld_relaxed(&rc->nF[S.par]);
    if (nF == 0) return;
    if (nF > S.fcap) nF = (uint32_t)S.fcap;  // overflow was flagged by ExtractAll
    const int32_t tau = S.tau_from_rc ? (int32_t)ld_relaxed(&rc->tau_cur) : S.tau;
    if (bid == 0 && threadIdx.x == 0) rc->rounds += 1;
    const uint32_t nwaves = nblk * kWavesPerBlock;
    const uint32_t wave_gid = bid * kWavesPerBlock + wv;
    // Seeds per wave: one group per wave when the frontier fits, so a round
    // lasts one local search rather than several in sequence.
    uint32_t G = (uint32_t)S.seeds;
    if (G == 0) {
        G = (nF + nwaves - 1) / nwaves;
        if (G > 64) G = 64;
        if (G < 1) G = 1;
    }
    const uint32_t ngroups = (nF + G - 1) / G;
    // Local search exists to give each task enough work when the frontier is
    // too small to keep the machine busy (Section 3.1); a frontier that
    // already fills every wavefront runs as a plain round.
    const unsigned long long fd = ld_relaxed64(reinterpret_cast<const uint64_t *>(&rc->fdeg[S.par]));
    const bool vgc = tau > 1 && ((fd > 0 && S.vgc_arcs > 0) ? fd < S.vgc_arcs : nF < S.vgc_cut);
    uint32_t depth = 0;
    uint32_t wseq = 0;
    unsigned long long c_seeds = 0, c_exp = 0, c_arcs = 0, c_att = 0, c_claims = 0, c_ins = 0, c_tclaims = 0;

    // Groups: wave w first takes group w; the groups past the wave count are
    // dealt out through per-stripe counters (wave w draws from stripe
    // w % kStripes: group nwaves + stripe + kStripes * draw).
    const uint32_t wstripe = wave_gid % kStripes;
    uint32_t grp = wave_gid;
    while (grp < ngroups) {
        const uint32_t start = grp * G;
        const int cnt = (int)((nF - start) < G ? (nF - start) : G);
        if (lane < cnt) {
            const uint64_t e = S.F[start + lane];
            const int32_t u = key_vertex(e);
            Q[lane] = e;
            // an entry (u, j) was claimed because label[u] equals source j's
            // label, so the entry carries the label its arcs are tested against
            if (REC) {
                const int4 r = S.rec[u];
                R[lane] = make_int2(r.x, r.y);
                QL[lane] = r.z;
            } else {
                const int32_t b0 = S.off[u];
                R[lane] = make_int2(b0, S.off[u + 1] - b0);
                if (PAIRS) QL[lane] = S.label[u];
            }
        }
        c_seeds += (unsigned long long)cnt;
        int head = 0, tail = cnt;
        long long t = 0;
        // the wave is the task whose size tau bounds (Section 3.2): its
        // seeds share one local search of budget tau
        const long long budget = vgc ? (long long)tau : 0;
        wave_lds_sync();
        uint32_t steps = 0;
        while (head < tail && (!vgc || t < budget)) {
            steps++;
            const int avail = tail - head;
            const int k = avail < kWave ? avail : kWave;
            uint64_t e = 0;
            int32_t d = 0, beg = 0, lab = 0;
            uint32_t s = 0;
            if (lane < k) {
                e = Q[(head + lane) & kQmask];
                const int2 r2 = R[(head + lane) & kQmask];
                beg = r2.x;
                d = r2.y;
                s = key_source(e);
                if (PAIRS) lab = QL[(head + lane) & kQmask];
            }
            // candidate heavy entries (deferred to the edge-parallel kernel)
            bool hv = lane < k && d > S.heavy_deg;
            const int nch = hv ? (d + kHeavyChunk - 1) / kHeavyChunk : 0;
            // whole entries whose arcs start within the step's arc window
            const int incl0 = wave_incl_scan(hv ? 0 : d);
            const int excl0 = incl0 - (hv ? 0 : d);
            const uint64_t cm = ballot(lane < k && excl0 < kStepArcs);
            const int kk = popc64(cm);
            const bool mine = lane < kk;
            hv = hv && mine;
            const int nchm = hv ? nch : 0;
            const int hincl = wave_incl_scan(nchm);
            const int htot = wave_bcast(hincl, kWave - 1);
            if (htot > 0) {
                uint32_t hb = 0;
                if (lane == 0) hb = atomicAdd(&rc->heavy_n[S.par], (uint32_t)htot);
                hb = wave_bcast_u(hb, 0);
                const bool fits = (uint64_t)hb + (uint64_t)htot <= S.hcap;
                if (fits) {
                    for (int c = 0; c < nchm; c++) {
                        const uint64_t pos = (uint64_t)hb + (uint64_t)(hincl - nchm + c);
                        S.heavy[2 * pos] = e;
                        S.heavy[2 * pos + 1] = (uint64_t)c;
                    }
                } else {
                    // no room: blank the reserved items below capacity and
                    // expand these entries here instead
                    for (int c = 0; c < nchm; c++) {
                        const uint64_t pos = (uint64_t)hb + (uint64_t)(hincl - nchm + c);
                        if (pos < S.hcap) S.heavy[2 * pos] = kEmpty64;
                    }
                    hv = false;
                }
            }
            const int dd = hv ? 0 : d;
            const int incl = wave_incl_scan(mine ? dd : 0);
            const int excl = incl - (mine ? dd : 0);
            const int D = wave_bcast(incl, kk - 1);
            if (mine) {
                sexcl[lane] = excl;
                sbeg[lane] = beg;
                ssrc[lane] = (int32_t)s;
                slab[lane] = lab;
            }
            head += kk;
            if (S.measure == 0) t += D;
            c_exp += (mine && !hv) ? 1 : 0;
            wave_lds_sync();
            // The step's arcs, ILP per lane: every phase issues the memory
            // operations of all of a lane's arcs before it uses any result,
            // so a step costs one chain of dependent accesses, not ILP.
            for (int base = 0; base < D; base += kWave * ILP) {
                bool va[ILP], claimed[ILP];
                int32_t w[ILP], lo_[ILP];
                uint64_t ne[ILP];
                int2 nr[ILP];
                int32_t nlab[ILP];
#pragma unroll
                for (int j = 0; j < ILP; j++) {
                    const int a = base + j * kWave + lane;
                    va[j] = a < D;
                    claimed[j] = false;
                    ne[j] = 0;
                    nr[j] = make_int2(0, 0);
                    nlab[j] = 0;
                    int lo = 0;
                    if (va[j]) {
                        int hi = kk - 1;
                        while (lo < hi) {
                            const int mid = (lo + hi + 1) >> 1;
                            if (sexcl[mid] <= a) lo = mid; else hi = mid - 1;
                        }
                    }
                    lo_[j] = lo;
                    w[j] = 0;
                    if (va[j]) w[j] = S.adj[sbeg[lo] + (a - sexcl[lo])];
                }
#pragma unroll
                for (int j = 0; j < ILP; j++)
                    if (va[j]) {
                        ne[j] = pair_key(w[j], (uint32_t)ssrc[lo_[j]]);
                        c_arcs++;
                    }
                if (!PAIRS) {
                    uint32_t old[ILP];
                    int32_t o0[ILP], o1[ILP];
                    if (vgc) {
                        // latency-bound regime: one atomic, offsets fetched alongside
#pragma unroll
                        for (int j = 0; j < ILP; j++) {
                            old[j] = 0xffffffffu;
                            o0[j] = o1[j] = 0;
                            if (va[j]) {
                                o0[j] = S.off[w[j]];
                                o1[j] = S.off[w[j] + 1];
                                old[j] = atomicOr(S.vis + (w[j] >> 5), 1u << (w[j] & 31));
                            }
                        }
#pragma unroll
                        for (int j = 0; j < ILP; j++) {
                            claimed[j] = va[j] && !((old[j] >> (w[j] & 31)) & 1u);
                            nr[j] = make_int2(o0[j], o1[j] - o0[j]);
                        }
                    } else {
                        // throughput regime: skip the atomic for visited targets
#pragma unroll
                        for (int j = 0; j < ILP; j++) old[j] = va[j] ? ld_relaxed(S.vis + (w[j] >> 5)) : 0xffffffffu;
#pragma unroll
                        for (int j = 0; j < ILP; j++)
                            if (!((old[j] >> (w[j] & 31)) & 1u)) old[j] = atomicOr(S.vis + (w[j] >> 5), 1u << (w[j] & 31));
                            else old[j] = 0xffffffffu;
#pragma unroll
                        for (int j = 0; j < ILP; j++) claimed[j] = va[j] && !((old[j] >> (w[j] & 31)) & 1u);
                    }
#pragma unroll
                    for (int j = 0; j < ILP; j++) c_att += va[j] ? 1 : 0;
                    if (MODE == kLdd) {
#pragma unroll
                        for (int j = 0; j < ILP; j++)
                            if (claimed[j]) S.owner[w[j]] = (int32_t)key_source(ne[j]);
                    }
                } else {
                    uint64_t h[ILP], cur[ILP];
                    int32_t o0[ILP], o1[ILP], fs[ILP];
                    int st[ILP];  // 2: claim pending, 1: claimed, 0: present or skipped
#pragma unroll
                    for (int j = 0; j < ILP; j++) {
                        h[j] = 0;
                        cur[j] = 0;
                        o0[j] = o1[j] = 0;
                        fs[j] = -1;
                        nlab[j] = -1;
                        if (va[j] && REC) {
                            // one 16-byte record: offsets, label and slot together
                            const int4 r = S.rec[w[j]];
                            o0[j] = r.x;
                            o1[j] = r.x + r.y;
                            nlab[j] = r.z;
                            fs[j] = r.w;
                        } else if (va[j]) {
                            nlab[j] = S.label[w[j]];
                            if (FIRST) {
                                fs[j] = (int32_t)ld_relaxed(reinterpret_cast<const uint32_t *>(S.first + w[j]));
                            } else {
                                h[j] = mix64(ne[j]) & S.tmask;
                                cur[j] = ld_relaxed64(S.table + h[j]);
                            }
                            if (vgc) {
                                o0[j] = S.off[w[j]];
                                o1[j] = S.off[w[j] + 1];
                            }
                        }
                    }
#pragma unroll
                    for (int j = 0; j < ILP; j++) {
                        const bool admit = MODE == kLe ? S.level + 1 < nlab[j] : nlab[j] == slab[lo_[j]];
                        st[j] = (va[j] && admit) ? 2 : 0;
                        c_att += st[j] == 2 ? 1 : 0;
                        nr[j] = make_int2(o0[j], o1[j] - o0[j]);
                    }
                    bool tab[ILP];
#pragma unroll
                    for (int j = 0; j < ILP; j++) tab[j] = false;
                    if (FIRST) {
                        // the inline slot first: already this source's, free
                        // (claim it), or another source's (the pair goes to the table)
#pragma unroll
                        for (int j = 0; j < ILP; j++) {
                            tab[j] = false;
                            if (st[j] != 2) continue;
                            const int32_t src = (int32_t)key_source(ne[j]);
                            if (fs[j] == src) {
                                st[j] = 0;
                            } else if (fs[j] == -1) {
                                int32_t *sl = REC ? reinterpret_cast<int32_t *>(S.rec + w[j]) + 3 : S.first + w[j];
                                const int32_t old = atomicCAS(sl, -1, src);
                                if (old == -1) {
                                    st[j] = 1;
                                    if (S.dirty) S.dirty[w[j] >> kDirtyLog2] = 1;
                                }
                                else if (old == src) st[j] = 0;
                                else tab[j] = true;
                            } else {
                                tab[j] = true;
                            }
                        }
#pragma unroll
                        for (int j = 0; j < ILP; j++)
                            if (tab[j]) {
                                h[j] = mix64(ne[j]) & S.tmask;
                                cur[j] = ld_relaxed64(S.table + h[j]);
                            }
                    }
                    // linear probing from the first slot (already loaded);
                    // every round of the loop is one load + one CAS per lane
                    for (uint32_t p = 0;; p++) {
                        unsigned long long old[ILP];
                        bool cas[ILP];
#pragma unroll
                        for (int j = 0; j < ILP; j++) {
                            cas[j] = false;
                            old[j] = 0;
                            if (st[j] == 2) {
                                if (cur[j] == ne[j]) {
                                    st[j] = 0;
                                } else if (cur[j] == kEmpty64) {
                                    old[j] = atomicCAS((unsigned long long *)(S.table + h[j]),
                                                       (unsigned long long)kEmpty64, (unsigned long long)ne[j]);
                                    cas[j] = true;
                                }
                            }
                        }
                        bool more = false;
#pragma unroll
                        for (int j = 0; j < ILP; j++) {
                            if (cas[j] && old[j] == kEmpty64) st[j] = 1;
                            else if (cas[j] && old[j] == ne[j]) st[j] = 0;
                            if (st[j] == 2) {
                                h[j] = (h[j] + 1) & S.tmask;
                                more = true;
                            }
                        }
                        if (!more) break;
                        if (p >= S.probe_limit) {
#pragma unroll
                            for (int j = 0; j < ILP; j++) st[j] = st[j] == 2 ? 0 : st[j];
                            atomicOr(&rc->err, kErrTable);
                            break;
                        }
#pragma unroll
                        for (int j = 0; j < ILP; j++)
                            if (st[j] == 2) cur[j] = ld_relaxed64(S.table + h[j]);
                    }
#pragma unroll
                    for (int j = 0; j < ILP; j++) {
                        claimed[j] = st[j] == 1;
                        c_tclaims += (FIRST && tab[j] && claimed[j]) ? 1 : 0;
                    }
                }
                // new entries: the local queue while it has room, else the bag
                int tot = 0, rk[ILP];
#pragma unroll
                for (int j = 0; j < ILP; j++) {
                    const uint64_t m = ballot(claimed[j]);
                    rk[j] = tot + rank_below(m);
                    tot += popc64(m);
                    c_claims += claimed[j] ? 1 : 0;
                }
                if (S.measure == 1) t += tot;
                if (tot == 0) continue;
                const int room = vgc ? kQcap - (tail - head) : 0;
                bool tobag[ILP];
#pragma unroll
                for (int j = 0; j < ILP; j++) {
                    if (claimed[j] && rk[j] < room) {
                        const int qi = (tail + rk[j]) & kQmask;
                        Q[qi] = ne[j];
                        R[qi] = nr[j];
                        if (PAIRS) QL[qi] = nlab[j];
                    }
                    tobag[j] = claimed[j] && rk[j] >= room;
                }
                tail += tot < room ? tot : room;
                c_ins += (unsigned long long)bag_insert_wave_n<ILP>(S.bag, tobag, ne, wave_gid, wseq);
            }
            wave_lds_sync();
        }
        depth = steps > depth ? steps : depth;
        // flush the rest of the local queue into the next frontier
        for (int i = head; i < tail; i += kWave) {
            const bool h = i + lane < tail;
            const uint64_t e = h ? Q[(i + lane) & kQmask] : 0;
            c_ins += (unsigned long long)bag_insert_wave(S.bag, h, e, wave_gid, wseq);
        }
        wave_lds_sync();
        if (ngroups <= nwaves) break;
        uint32_t nxt = 0;
        if (lane == 0) nxt = nwaves + wstripe + kStripes * atomicAdd(&S.ls->s[wstripe].work[S.par], 1u);
        grp = wave_bcast_u(nxt, 0);
    }
    __shared__ uint32_t dmax[kWavesPerBlock];
    if (lane == 0) dmax[wv] = depth;
    unsigned long long c[kNumCtr] = {c_seeds, c_exp, c_arcs, c_att, c_claims, c_ins};
    const unsigned long long t = block_flush_ctr(S.cn->c[bid % kCtrStripes][S.kind], c);  // has a barrier
    StripeLine &sl = S.ls->s[bid % kStripes];
    if (threadIdx.x == kCtrClaims && t) atomicAdd(&sl.claims, t);
    if (FIRST) {
        // table claims: a block-wide sum, one atomic per block
        __shared__ unsigned long long tpart[kWavesPerBlock];
        const unsigned long long tw = wave_sum_u64(c_tclaims);
        if (lane == 0) tpart[wv] = tw;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long tt = 0;
            for (int w = 0; w < kWavesPerBlock; w++) tt += tpart[w];
            if (tt) atomicAdd(&sl.tclaims, tt);
        }
    }
    if (threadIdx.x == kNumCtr) {
        uint32_t d = 0;
        for (int w = 0; w < kWavesPerBlock; w++) d = dmax[w] > d ? dmax[w] : d;
        if (d) atomicMax(&sl.depth, d);
    }
}

// A launch serves one or two search lanes (the forward and the backward
// search of a batch): with two, the first `split` blocks take lane 0 and the
// rest lane 1, so the two searches' rounds run side by side.
struct LanePair {
    Search S[2];
    int32_t nl;      // lanes in this launch (1 or 2)
    uint32_t split;  // blocks of lane 0 when nl == 2
};

__device__ __forceinline__ int pair_lane(const LanePair &P, uint32_t &bid, uint32_t &nblk) {
    if (P.nl < 2) return 0;
    if (bid < P.split) {
        nblk = P.split;
        return 0;
    }
    bid -= P.split;
    nblk -= P.split;
    return 1;
}

template <int MODE, int ILP>
__global__ __launch_bounds__(kBlock) void k_expand(LanePair P) {
    uint32_t bid = blockIdx.x, nblk = gridDim.x;
    const int l = pair_lane(P, bid, nblk);
    expand_round<MODE, ILP>(P.S[l], bid, nblk);
}

// Edge-parallel expansion of the deferred high-degree entries.  Each item is
// one kHeavyChunk-arc slice of an adjacency list; a block takes an item and
// its four waves stride over the slice; claims go to the bag.
template <int MODE>
__device__ __forceinline__ void heavy_round(const Search &S, uint32_t bid, uint32_t nblk) {
    constexpr bool PAIRS = MODE == kMulti || MODE == kMultiFirst || MODE == kLe || MODE == kMultiRec;
    constexpr bool REC = MODE == kMultiRec;
    RoundCtl *rc = S.rc;
    uint32_t nh = ld_relaxed(&rc->heavy_n[S.par]);
    if (nh == 0) return;
    if (nh > S.hcap) nh = (uint32_t)S.hcap;
    const int lane = lane_id();
    const int wv = threadIdx.x / kWave;
    const uint32_t wave_gid = bid * kWavesPerBlock + wv;
    uint32_t wseq = 0x8000u;
    unsigned long long c_exp = 0, c_arcs = 0, c_att = 0, c_claims = 0, c_ins = 0, c_tclaims = 0;
    for (uint32_t h = bid; h < nh; h += nblk) {
        const uint64_t e = S.heavy[2 * (uint64_t)h];
        if (e == kEmpty64) continue;  // block-uniform
        const uint32_t chunk = (uint32_t)S.heavy[2 * (uint64_t)h + 1];
        const int32_t u = key_vertex(e);
        const uint32_t src = key_source(e);
        const int32_t beg0 = REC ? S.rec[u].x : S.off[u];
        const int64_t d = REC ? (int64_t)S.rec[u].y : (int64_t)S.off[u + 1] - beg0;
        const int64_t lo = (int64_t)chunk * kHeavyChunk;
        const int64_t len = (d - lo) < kHeavyChunk ? (d - lo) : kHeavyChunk;
        const int32_t lab = (MODE == kMulti || MODE == kMultiFirst || REC) ? S.srclab[src] : 0;
        if (chunk == 0 && threadIdx.x == 0) c_exp++;
        for (int64_t base = (int64_t)wv * kWave; base < len; base += kBlock) {
            const int64_t a = base + lane;
            bool claimed = false;
            uint64_t ne = 0;
            if (a < len) {
                const int32_t w = S.adj[beg0 + lo + a];
                c_arcs++;
                if (!PAIRS) {
                    c_att++;
                    claimed = claim_bit(S.vis, w);
                    if (MODE == kLdd && claimed) S.owner[w] = (int32_t)src;
                } else if (MODE == kLe ? S.level + 1 < S.label[w] : (REC ? S.rec[w].z : S.label[w]) == lab) {
                    c_att++;
                    const int c = REC ? claim_pair_slot(reinterpret_cast<int32_t *>(S.rec + w) + 3, S.table, S.tmask,
                                                        S.probe_limit, w, src)
                                  : MODE == kMultiFirst
                                      ? claim_pair_first(S.first, S.table, S.tmask, S.probe_limit, w, src)
                                      : claim_pair(S.table, S.tmask, S.probe_limit, pair_key(w, src));
                    if (c < 0) atomicOr(&rc->err, kErrTable);
                    claimed = c >= 1;
                    c_tclaims += c == 2 ? 1 : 0;
                    if (c == 1 && S.dirty) S.dirty[w >> kDirtyLog2] = 1;
                }
                ne = pair_key(w, src);
            }
            c_claims += claimed ? 1 : 0;
            c_ins += (unsigned long long)bag_insert_wave(S.bag, claimed, ne, wave_gid, wseq);
        }
    }
    unsigned long long c[kNumCtr] = {0, c_exp, c_arcs, c_att, c_claims, c_ins};
    const unsigned long long t =
        block_flush_ctr(S.cn->c[bid % kCtrStripes][PAIRS ? kKindHeavyMulti : kKindHeavySingle], c);
    if (threadIdx.x == kCtrClaims && t) atomicAdd(&S.ls->s[bid % kStripes].claims, t);
    if (MODE == kMultiFirst || REC) {
        __shared__ unsigned long long tpart[kWavesPerBlock];
        const unsigned long long tw = wave_sum_u64(c_tclaims);
        if (lane == 0) tpart[wv] = tw;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long tt = 0;
            for (int w = 0; w < kWavesPerBlock; w++) tt += tpart[w];
            if (tt) atomicAdd(&S.ls->s[bid % kStripes].tclaims, tt);
        }
    }
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_expand_heavy(LanePair P) {
    uint32_t bid = blockIdx.x, nblk = gridDim.x;
    const int l = pair_lane(P, bid, nblk);
    heavy_round<MODE>(P.S[l], bid, nblk);
}

// ------------------------------------------------------------ dense mode ----
// Dense round of a single-source search (Section 4.2, the dense-backward
// optimisation): every vertex of the subproblem that is not yet visited scans
// its predecessors (in-arcs for a forward search, out-arcs for a backward
// one) and joins the next frontier at the first predecessor found in the
// current frontier, skipping its remaining arcs.  A wave owns 64 consecutive
// vertices, i.e. two bitmap words, so it updates visited/next words with plain
// stores.  next is written for every word, so it needs no clearing.
__global__ __launch_bounds__(kBlock) void k_pull(int32_t n, const int32_t *off, const int32_t *adj, uint32_t *vis,
                                                 const uint32_t *front, uint32_t *next, LaneStripes *ls, Counters *cn) {
    const int lane = lane_id();
    uint32_t found_cnt = 0;
    unsigned long long c_exp = 0, c_arcs = 0;
    for (int64_t v0 = blockIdx.x * (int64_t)blockDim.x + (threadIdx.x & ~(kWave - 1)); v0 < n;
         v0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = v0 + lane;
        const int64_t wi = v >> 5;
        const uint32_t word = v < n ? vis[wi] : 0xffffffffu;
        bool found = false;
        if (v < n && !((word >> (v & 31)) & 1u)) {
            c_exp++;
            const int32_t e1 = off[v + 1];
            // four predecessors per iteration: their ids, then their frontier
            // words, are loaded together (one chain of two accesses per four arcs)
            for (int32_t e = off[v]; e < e1 && !found; e += 4) {
                int32_t u[4];
#pragma unroll
                for (int i = 0; i < 4; i++) u[i] = e + i < e1 ? adj[e + i] : -1;
                uint32_t f[4];
#pragma unroll
                for (int i = 0; i < 4; i++) f[i] = u[i] >= 0 ? front[u[i] >> 5] : 0u;
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    if (u[i] < 0 || found) continue;
                    c_arcs++;
                    found = (f[i] >> (u[i] & 31)) & 1u;
                }
            }
        }
        const uint64_t m = ballot(found);
        found_cnt += found ? 1 : 0;
        if ((lane == 0 || lane == 32) && v < n) {
            const uint32_t bits = lane == 0 ? (uint32_t)m : (uint32_t)(m >> 32);
            next[wi] = bits;
            if (bits) vis[wi] = word | bits;
        }
    }
    // the next frontier's size and the claims go to the lane's stripes;
    // k_round_end folds them (pull claims count as the lane's claims)
    unsigned long long c[kNumCtr] = {0, c_exp, c_arcs, 0, (unsigned long long)found_cnt, 0};
    const unsigned long long t = block_flush_ctr(cn->c[blockIdx.x % kCtrStripes][kKindPull], c);
    StripeLine &sl = ls->s[blockIdx.x % kStripes];
    if (threadIdx.x == kCtrClaims && t) {
        atomicAdd(&sl.claims, t);
        atomicAdd(&sl.nf, (uint32_t)t);
    }
}

// Trace mode: snapshot the inputs of the coming round (the policy features);
// par is the coming round's parity, so the previous round's depth is at par ^ 1.
__global__ void k_trace_snap(RoundCtl *rc, int par) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        rc->snap_nf = (unsigned long long)rc->nF[0] + rc->nF[1];
        rc->snap_fdeg = rc->fdeg[par];
        rc->snap_claims = rc->claims;
        rc->snap_rounds = rc->rounds;
        rc->snap_depth = rc->lsdepth[par ^ 1];
    }
}

// End of a dense round: the next frontier's size and the claims from the
// stripes, this round's counters cleared.
__global__ void k_round_end(RoundCtl *rc, LaneStripes *ls, int par) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        uint32_t nf = 0;
        for (int i = 0; i < kStripes; i++) {
            nf += ls->s[i].nf;
            ls->s[i].nf = 0;
        }
        stripes_fold(rc, ls, par);
        rc->nF[par ^ 1] = nf;
        rc->nF[par] = 0;
        rc->fdeg[0] = rc->fdeg[1] = 0;  // a pull round does not sum degrees
        rc->heavy_n[par] = 0;
        rc->rounds += 1;
    }
}

// Frontier list (entries (v, 0)) -> bitmap; bits must be clear on entry.
__global__ void k_list_to_bitmap(const uint64_t *F, const RoundCtl *rc, int par, uint64_t fcap, uint32_t *bits) {
    uint64_t nf = rc->nF[par];
    if (nf > fcap) nf = fcap;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < nf; i += (uint64_t)gridDim.x * blockDim.x) {
        const int32_t v = key_vertex(F[i]);
        atomicOr(&bits[v >> 5], 1u << (v & 31));
    }
}

// Bitmap -> frontier list (order unspecified).  Each block owns a contiguous
// range of words: it counts their bits, reserves its output range with one
// atomic, and each thread writes the entries of its own sub-range.
__global__ __launch_bounds__(kBlock) void k_bitmap_to_list(int32_t n, const uint32_t *bits, uint64_t *F, uint64_t fcap,
                                                           RoundCtl *rc) {
    __shared__ uint32_t part[kWavesPerBlock];
    __shared__ uint32_t base_s;
    const uint64_t nwords = ((uint64_t)n + 31) >> 5;
    const uint64_t per_block = (nwords + gridDim.x - 1) / gridDim.x;
    const uint64_t w0 = (uint64_t)blockIdx.x * per_block;
    const uint64_t w1 = w0 + per_block < nwords ? w0 + per_block : nwords;
    const uint64_t per_thread = (per_block + kBlock - 1) / kBlock;
    const uint64_t t0 = w0 + threadIdx.x * per_thread;
    const uint64_t t1 = t0 + per_thread < w1 ? t0 + per_thread : w1;
    uint32_t cnt = 0;
    for (uint64_t w = t0; w < t1; w++) cnt += (uint32_t)__popc(bits[w]);
    // block exclusive scan of the per-thread counts
    const int lane = lane_id();
    int incl = wave_incl_scan((int)cnt);
    if (lane == kWave - 1) part[threadIdx.x / kWave] = (uint32_t)incl;
    __syncthreads();
    uint32_t wave_off = 0, total = 0;
    for (int w = 0; w < kWavesPerBlock; w++) {
        if (w < (int)(threadIdx.x / kWave)) wave_off += part[w];
        total += part[w];
    }
    if (threadIdx.x == 0) base_s = total ? atomicAdd(&rc->listpos, total) : 0u;
    __syncthreads();
    uint64_t pos = (uint64_t)base_s + wave_off + (uint32_t)(incl - (int)cnt);
    for (uint64_t w = t0; w < t1; w++) {
        uint32_t x = bits[w];
        while (x) {
            const int b = __ffs(x) - 1;
            x &= x - 1;
            const int64_t v = (int64_t)(w << 5) + b;
            if (v < n && pos < fcap) F[pos] = pair_key((int32_t)v, 0);
            pos++;
        }
    }
}

// --------------------------------------------------------- ExtractAll ----
// Packs the bag's used prefix [0, tail[r]) into the frontier array F and
// clears it (Section 3.3: ExtractAll emits and removes all elements).  A wave
// handles 64 stripes: a prefix sum of their counts gives each stripe's output
// offset; a block reserves its four waves' ranges with one atomic.  With
// S.fdeg_on it also sums the degrees of the extracted entries (the frontier's
// arc count, used to choose the next round's mode).  The last block to finish
// resets the bag's chunk state and this round's counters.
__device__ __forceinline__ void extract_round(const Search &S, int par, uint32_t bid, uint32_t nblk) {
    __shared__ uint32_t part[kWavesPerBlock];
    __shared__ uint32_t base_s;
    const Bag &B = S.bag;
    RoundCtl *rc = S.rc;
    const int lane = lane_id();
    const int wv = threadIdx.x / kWave;
    uint32_t r = ld_relaxed(&B.ctl->r);
    if (r >= B.nchunks) r = B.nchunks - 1;
    const uint64_t nst = bag_chunk_hi(B, r) >> kStripeLog2;
    unsigned long long fdeg = 0;
    // the log's first position for this round (the lane's last block moves
    // emit past the round's entries once every block has read it)
    const uint64_t lbase = S.lkeys ? (uint64_t)ld_relaxed(&S.lsh->emit) : 0;
    for (uint64_t sb0 = (uint64_t)bid * kBlock; sb0 < nst; sb0 += (uint64_t)nblk * kBlock) {
        const uint64_t sb = sb0 + (uint64_t)wv * kWave;
        const uint64_t st = sb + lane;
        uint32_t c = 0;
        if (st < nst) {
            c = B.cnt[st];
            if (c > (uint32_t)kStripe) c = kStripe;
        }
        const int incl = wave_incl_scan((int)c);
        const int tot = wave_bcast(incl, kWave - 1);
        if (lane == 0) part[wv] = (uint32_t)tot;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t t = 0;
            for (int w = 0; w < kWavesPerBlock; w++) t += part[w];
            base_s = t ? atomicAdd(&rc->nF[par ^ 1], t) : 0u;
        }
        __syncthreads();
        uint32_t base = base_s;
        for (int w = 0; w < wv; w++) base += part[w];
        __syncthreads();  // part/base_s are rewritten next iteration
        if (tot == 0) continue;
        const int excl = incl - (int)c;
        for (int j = 0; j < kWave; j++) {
            const int cj = wave_bcast((int)c, j);
            if (cj == 0) continue;
            const uint64_t oj = (uint64_t)base + (uint64_t)wave_bcast(excl, j);
            if (lane < cj) {
                const uint64_t v = B.slots[((sb + j) << kStripeLog2) + lane];
                if (oj + lane < S.fcap) {
                    S.F[oj + lane] = v;
                    if (S.lkeys && lbase + oj + lane < S.lcap) {
                        S.lkeys[lbase + oj + lane] = ((uint64_t)(uint32_t)key_vertex(v) << S.lkbits) | key_source(v);
                        S.ldist[lbase + oj + lane] = S.level + 1;
                    }
                } else {
                    atomicOr(&rc->err, kErrCapacity);
                }
                if (S.off) {  // the bag self-test extracts keys of no graph
                    const int32_t u = key_vertex(v);
                    fdeg += (unsigned long long)(S.off[u + 1] - S.off[u]);
                }
            }
        }
        if (st < nst && c) {
            B.cnt[st] = 0;
            if (B.track) atomicAdd(&B.ctl->fill[bag_chunk_of_stripe(B, st)], c);
        }
    }
    {
        // the new frontier's degree sum (its offsets are read anyway by the
        // next round, so this mostly warms the cache for it)
        __shared__ unsigned long long fpart[kWavesPerBlock];
        fdeg = wave_sum_u64(fdeg);
        if (lane == 0) fpart[wv] = fdeg;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long t = 0;
            for (int w = 0; w < kWavesPerBlock; w++) t += fpart[w];
            if (t) atomicAdd(&rc->fdeg[par ^ 1], t);
        }
    }
}

// The reset ExtractAll ends with (one thread, once every block has read r):
// chunk state and this round's counters.
__device__ __forceinline__ void extract_reset(const Search &S, int par) {
    const Bag &B = S.bag;
    for (uint32_t i = 0; i < B.nchunks && i < (uint32_t)kMaxChunks; i++) B.ctl->sample[i] = 0;
    B.ctl->last_r = B.ctl->r;
    B.ctl->r = 0;
    B.ctl->done_blocks = 0;
    S.rc->nF[par] = 0;
    S.rc->fdeg[par] = 0;
    S.rc->heavy_n[par] = 0;
    stripes_fold(S.rc, S.ls, par);
    if (S.lkeys) {
        const uint64_t nf = S.rc->nF[par ^ 1];
        S.lsh->emit += (uint32_t)(nf < S.fcap ? nf : S.fcap);
    }
}

// ExtractAll of one or two lanes (split as in k_expand); each lane's frontier
// parity is in its Search.
__global__ __launch_bounds__(kBlock) void k_bag_extract(LanePair P) {
    __shared__ bool last;
    uint32_t bid = blockIdx.x, nblk = gridDim.x;
    const int l = pair_lane(P, bid, nblk);
    const Search &S = P.S[l];
    extract_round(S, S.par, bid, nblk);
    // ExtractAll also clears the chunk state: the lane's last block does it
    // once every block of the lane has finished reading r.
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        last = atomicAdd(&S.bag.ctl->done_blocks, 1u) == nblk - 1;
    }
    __syncthreads();
    if (!last) return;  // block-uniform
    if (threadIdx.x == 0) {
        __threadfence();
        extract_reset(S, S.par);
    }
    if (S.policy_w) {
        // the learned policy picks the next round's budget here, where the new
        // frontier's statistics are complete, instead of in a launch of its own
        __shared__ float x[kPolicyIn], h1[kPolicyHidden], h2[kPolicyHidden], y[kPolicyOut];
        __shared__ uint32_t nf;
        RoundCtl *rc = S.rc;
        const int np = S.par ^ 1;
        __syncthreads();
        if (threadIdx.x == 0) {
            nf = rc->nF[np];
            policy_features((float)nf, (float)rc->fdeg[np], (float)rc->claims, S.nsub, (float)rc->rounds,
                            (float)rc->lsdepth[S.par], x);
        }
        __syncthreads();
        if (nf == 0) return;  // block-uniform: no next round
        if (threadIdx.x < kWave) policy_forward_wave(S.policy_w, x, y, h1, h2);
        __syncthreads();
        if (threadIdx.x == 0)
            // single-source lanes may also pick the dense (pull) mode of Section 4.2
            policy_pick(y, S.kind == kKindExpandSingle ? 3u : 1u, S.fallback_tau, &rc->tau_cur, &rc->mode_pref,
                        &rc->policy_calls, &rc->policy_fallbacks);
    }
}

// -------------------------------------------------------------- relabel ----
// Single source (the first SCC, Section 4.2): vertices reached both ways are
// finished with key s; vertices reached one way move to a new subproblem
// labelled by the hash of (old label, R_in, R_out) (Algorithm 1).
__global__ void k_finish_single(int32_t n, int32_t *label, int32_t L, const Shared *shc, Perm P, const uint32_t *visF,
                                const uint32_t *visB, CountStripes *cs) {
    const int32_t s = single_source(-1, shc, P);
    if (s < 0) return;
    uint32_t cnt = 0;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        if (label[v] != L) continue;
        const bool f = (visF[v >> 5] >> (v & 31)) & 1u;
        const bool b = (visB[v >> 5] >> (v & 31)) & 1u;
        if (f && b) {
            label[v] = ~s;
            cnt++;
        } else if (f || b) {
            label[v] = relabel_hash(L, b ? sig_term_in(s) : 0ull, f ? sig_term_out(s) : 0ull);
        }
    }
    block_add_u32(&cs->s[blockIdx.x % kStripes].fin, cnt);
}

// Multi source, pass 1: accumulate the per-vertex set hashes of R_out (pairs
// of the forward table) and R_in (backward table), and detect vertices that
// share a source in both directions (Algorithm 1: R_1 and R_2 intersect).
// With clear_in the backward table's slots are emptied as they are read (no
// thread of this pass probes that table; the dense relabel that follows does
// not read it).
__global__ void k_accumulate(const uint64_t *Tout, uint64_t mout, uint64_t *Tin, uint64_t min_,
                             uint32_t limit, const int32_t *srcvert, unsigned long long *sig_out,
                             unsigned long long *sig_in, int32_t *fin, bool clear_in, const int32_t *firstF,
                             const int32_t *firstB, int32_t fstride) {
    // with first-source slots a vertex's pairs are its slot plus its table
    // keys, per direction; the slots themselves are summed by the per-vertex
    // relabel, and a shared source is found here for every combination that
    // involves a table key (slot/slot is the relabel's test)
    const uint64_t n_out = mout + 1, n_tot = n_out + min_ + 1;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n_tot; i += (uint64_t)gridDim.x * blockDim.x) {
        if (i < n_out) {
            const uint64_t key = Tout[i];
            if (key == kEmpty64) continue;
            const int32_t v = key_vertex(key);
            atomicAdd(&sig_out[v], (unsigned long long)sig_term_out(srcvert[key_source(key)]));
            if (firstB && firstB[(int64_t)fstride * v] == (int32_t)key_source(key))
                atomicMin(&fin[v], (int32_t)key_source(key));
        } else {
            const uint64_t key = Tin[i - n_out];
            if (key == kEmpty64) continue;
            if (clear_in) Tin[i - n_out] = kEmpty64;
            const int32_t v = key_vertex(key);
            atomicAdd(&sig_in[v], (unsigned long long)sig_term_in(srcvert[key_source(key)]));
            if ((firstF && firstF[(int64_t)fstride * v] == (int32_t)key_source(key)) ||
                table_contains(Tout, mout, limit, key))
                atomicMin(&fin[v], (int32_t)key_source(key));
        }
    }
}

// Multi source, pass 2: one owner per touched vertex (first to stamp it with
// this batch's epoch) writes its new label and resets its accumulators; every
// table slot is cleared for the next batch.
__global__ void k_relabel_multi(uint64_t *Tout, uint64_t mout, uint64_t *Tin, uint64_t min_, const int32_t *srcvert,
                                unsigned long long *sig_out, unsigned long long *sig_in, int32_t *fin,
                                int32_t *stamp, int32_t epoch, int32_t *label, CountStripes *cs) {
    const uint64_t n_out = mout + 1, n_tot = n_out + min_ + 1;
    uint32_t cnt = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n_tot; i += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t *slot = i < n_out ? Tout + i : Tin + (i - n_out);
        const uint64_t key = *slot;
        if (key == kEmpty64) continue;
        *slot = kEmpty64;
        const int32_t v = key_vertex(key);
        if (atomicExch(&stamp[v], epoch) == epoch) continue;
        const int32_t f = fin[v];
        if (f != kInf32) {
            label[v] = ~srcvert[f];
            cnt++;
        } else {
            label[v] = relabel_hash(label[v], sig_in[v], sig_out[v]);
        }
        sig_in[v] = 0;
        sig_out[v] = 0;
        fin[v] = kInf32;
    }
    block_add_u32(&cs->s[blockIdx.x % kStripes].fin, cnt);
}

// Multi source, pass 2 for batches whose pairs are a sizeable fraction of the
// vertices: the same relabelling as k_relabel_multi, taken per vertex in one
// coalesced pass instead of per table slot with an owner election (a vertex
// was touched iff its accumulators are set; finished vertices are never
// claimed).  The forward table is cleared here, the backward one was cleared
// by k_accumulate.
__device__ __forceinline__ uint32_t relabel_vertex(uint64_t v, const int32_t *srcvert, unsigned long long *sig_out,
                                                   unsigned long long *sig_in, int32_t *fin, int32_t *label,
                                                   int32_t *firstF, int32_t *firstB, int32_t fstride, int4 *recF,
                                                   int4 *recB) {
    const int32_t l = label[v];
    if (l < 0) return 0;
    int32_t f = kInf32;
    unsigned long long si = 0, so = 0;
    if (firstF) {
        // the first-source slots: their pairs join the signatures, a source
        // in both slots finishes the vertex, and the slots empty; a vertex
        // with both slots empty has no pairs at all (table pairs need a
        // taken slot), so its accumulators are not read
        int32_t *pa = firstF + (int64_t)fstride * v, *pb = firstB + (int64_t)fstride * v;
        const int32_t a = *pa, b = *pb;
        if (a < 0 && b < 0) return 0;
        f = fin[v];
        si = sig_in[v];
        so = sig_out[v];
        if (a >= 0) {
            so += sig_term_out(srcvert[a]);
            *pa = -1;
        }
        if (b >= 0) {
            si += sig_term_in(srcvert[b]);
            *pb = -1;
        }
        if (a >= 0 && a == b && a < f) f = a;
    } else {
        f = fin[v];
        si = sig_in[v];
        so = sig_out[v];
    }
    int32_t nl;
    uint32_t fin_cnt = 0;
    if (f != kInf32) {
        nl = ~srcvert[f];
        fin_cnt = 1;
    } else if ((si | so) != 0ull) {
        nl = relabel_hash(l, si, so);
    } else {
        return 0;
    }
    label[v] = nl;
    if (recF) {  // the packed records carry a copy of the label
        recF[v].z = nl;
        recB[v].z = nl;
    }
    sig_in[v] = 0;
    sig_out[v] = 0;
    fin[v] = kInf32;
    return fin_cnt;
}

// Multi source, pass 2 for batches whose pairs are a sizeable fraction of the
// vertices: the same relabelling as k_relabel_multi, taken per vertex in one
// coalesced pass instead of per table slot with an owner election (a vertex
// was touched iff its accumulators are set; finished vertices are never
// claimed).  With granule flags (first-source slots), only flagged granules
// are visited, and their flags are cleared.  The forward table is cleared
// here, the backward one was cleared by k_accumulate.
__global__ void k_relabel_dense(int32_t n, uint64_t *Tout, uint64_t mout, const int32_t *srcvert,
                                unsigned long long *sig_out, unsigned long long *sig_in, int32_t *fin, int32_t *label,
                                CountStripes *cs, int32_t *firstF, int32_t *firstB, int32_t fstride, int4 *recF,
                                int4 *recB, uint8_t *dirty) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i <= mout; i += stride) Tout[i] = kEmpty64;
    uint32_t cnt = 0;
    if (!dirty) {
        for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < (uint64_t)n; v += stride)
            cnt += relabel_vertex(v, srcvert, sig_out, sig_in, fin, label, firstF, firstB, fstride, recF, recB);
    } else {
        const uint64_t ng = ((uint64_t)n + (1u << kDirtyLog2) - 1) >> kDirtyLog2;
        for (uint64_t g = blockIdx.x; g < ng; g += gridDim.x) {
            const uint8_t d = dirty[g];
            __syncthreads();  // every thread has read the flag before it is cleared
            if (!d) continue;
            if (threadIdx.x == 0) dirty[g] = 0;
            const uint64_t v1 = min((g + 1) << kDirtyLog2, (uint64_t)n);
            for (uint64_t v = (g << kDirtyLog2) + threadIdx.x; v < v1; v += blockDim.x)
                cnt += relabel_vertex(v, srcvert, sig_out, sig_in, fin, label, firstF, firstB, fstride, recF, recB);
        }
    }
    block_add_u32(&cs->s[blockIdx.x % kStripes].fin, cnt);
}

// Packed records of both directions for the multi-source batches: {first
// arc, degree, label, empty first-source slot}.
__global__ void k_build_rec(int32_t n, const int32_t *out_off, const int32_t *in_off, const int32_t *label, int4 *recF,
                            int4 *recB) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t l = label[v];
        const int32_t a = out_off[v], b = in_off[v];
        recF[v] = make_int4(a, out_off[v + 1] - a, l, -1);
        recB[v] = make_int4(b, in_off[v + 1] - b, l, -1);
    }
}

// Empties the first-source slots of one direction's records.
__global__ void k_clear_rec_slots(int32_t n, int4 *rec) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        rec[v].w = -1;
}

// ---------------------------------------------------------- canonical ----
// labels_out[v] = min vertex id of v's SCC: every finished vertex holds ~key
// with key a member of its SCC; a min-reduction per key then a gather.
// aux[k] starts at k: every SCC key is a member of its SCC, so a member v with
// v >= key cannot lower the minimum.  The rest is first reduced per block in a
// small LDS hash table (one global atomic per block and key), which keeps the
// atomics on the key of a giant SCC from serialising.
__global__ void k_iota(int32_t n, int32_t *a) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        a[v] = (int32_t)v;
}

__global__ __launch_bounds__(kBlock) void k_canon_min(int32_t n, const int32_t *label, int32_t *aux, uint32_t *err) {
    constexpr int H = 2 * kBlock;
    __shared__ int32_t hk[H], hv[H];
    for (int i = threadIdx.x; i < H; i += blockDim.x) {
        hk[i] = -1;
        hv[i] = kInf32;
    }
    __syncthreads();
    const int lane = lane_id();
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t l = label[v];
        const bool bad = l >= 0 || ~l >= n;
        if (bad) atomicOr(err, kErrUnfinished);
        const int32_t key = ~l;
        const bool want = !bad && v < key;
        // a wave's vertices are consecutive, so among its lanes with the key
        // of its lowest wanting lane, that lane holds the smallest id: the
        // others have nothing to add (the members of a giant SCC often fill
        // much of a wave)
        const uint64_t wm = ballot(want);
        if (!want) continue;
        const int L0 = __builtin_ctzll(wm);
        if (lane != L0 && key == wave_bcast(key, L0)) continue;
        const int slot = (int)(mix64((uint64_t)key) & (H - 1));
        const int32_t prev = atomicCAS(&hk[slot], -1, key);
        if (prev == -1 || prev == key) atomicMin(&hv[slot], (int32_t)v);
        else atomicMin(&aux[key], (int32_t)v);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < H; i += blockDim.x)
        if (hk[i] >= 0) atomicMin(&aux[hk[i]], hv[i]);
}

__global__ void k_canon_write(int32_t n, const int32_t *label, const int32_t *aux, int32_t *out, CountStripes *cs) {
    uint32_t cnt = 0;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t l = label[v];
        const int32_t r = (l < 0 && ~l < n) ? aux[~l] : -1;
        out[v] = r;
        cnt += (r == v);
    }
    block_add_u32(&cs->s[blockIdx.x % kStripes].nscc, cnt);
}

// ---------------------------------------------------------- reach output ----
// The pairs of a search as sort keys (j << vbits) | v, so that an ascending
// sort orders them by (source index, vertex).  Slots come from one block
// reservation each; keys past `cap` are counted but not written.
__global__ void k_emit_single(int32_t n, const int32_t *label, int32_t L, const uint32_t *vis, uint64_t *keys,
                              uint64_t cap, Shared *sh) {
    for (int64_t v0 = blockIdx.x * (int64_t)blockDim.x; v0 < n; v0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = v0 + threadIdx.x;
        const bool hit = v < n && label[v] == L && ((vis[v >> 5] >> (v & 31)) & 1u);
        const uint64_t m = ballot(hit);
        const uint32_t base = block_reserve(&sh->emit, (uint32_t)popc64(m));
        if (hit) {
            const uint64_t pos = (uint64_t)base + rank_below(m);
            if (pos < cap) keys[pos] = (uint64_t)v;
        }
    }
}

__global__ void k_emit_table(const uint64_t *T, uint64_t mask, uint32_t vbits, uint64_t *keys, uint64_t cap,
                             Shared *sh) {
    const uint64_t nt = mask + 1;
    for (uint64_t i0 = blockIdx.x * (uint64_t)blockDim.x; i0 < nt; i0 += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t i = i0 + threadIdx.x;
        const uint64_t key = i < nt ? T[i] : kEmpty64;
        const bool hit = key != kEmpty64;
        const uint64_t m = ballot(hit);
        const uint32_t base = block_reserve(&sh->emit, (uint32_t)popc64(m));
        if (hit) {
            const uint64_t pos = (uint64_t)base + rank_below(m);
            if (pos < cap) keys[pos] = ((uint64_t)key_source(key) << vbits) | (uint64_t)(uint32_t)key_vertex(key);
        }
    }
}

// Sorted keys -> output pairs (vertex, source index).
__global__ void k_unpack_pairs(const uint64_t *keys, uint64_t cnt, uint32_t vbits, int32_t *pairs) {
    const uint64_t vmask = (1ull << vbits) - 1;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < cnt; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t k = keys[i];
        pairs[2 * i] = (int32_t)(k & vmask);
        pairs[2 * i + 1] = (int32_t)(k >> vbits);
    }
}

// ------------------------------------------------------- connectivity ----
// Connected components by LDD-UF-JTB (Algorithm 4): a low-diameter
// decomposition grows clusters from randomly ordered centres added in
// batches of growing size, each round searching out from the frontier
// (Section 5.1 runs these searches with VGC and the hash bag); every vertex
// ends with owner[v], the centre of its cluster.  A union-find over the arcs
// whose endpoints have different owners then merges clusters.

// Adds batch [p0, p1) of the centre order to the frontier: a vertex not yet
// claimed by any cluster becomes a centre (its own owner) and a frontier
// entry (v, v).  The frontier grows at rc->nF[par]; its degree sum too.
__global__ __launch_bounds__(kBlock) void k_ldd_add(Perm P, uint32_t p0, uint32_t p1, const int32_t *off, uint32_t *vis,
                                                    int32_t *owner, uint64_t *F, uint64_t fcap, RoundCtl *rc, int par) {
    __shared__ unsigned long long dpart[kWavesPerBlock];
    unsigned long long deg = 0;
    for (uint64_t j0 = p0 + (uint64_t)blockIdx.x * blockDim.x; j0 < p1; j0 += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t j = j0 + threadIdx.x;
        bool mine = false;
        int32_t v = 0;
        if (j < p1) {
            v = (int32_t)perm_apply(P, (uint32_t)j);
            mine = claim_bit(vis, v);
        }
        const uint64_t m = ballot(mine);
        const uint32_t base = block_reserve(&rc->nF[par], (uint32_t)popc64(m));
        if (mine) {
            owner[v] = v;
            const uint64_t pos = (uint64_t)base + rank_below(m);
            if (pos < fcap) F[pos] = pair_key(v, (uint32_t)v);
            else atomicOr(&rc->err, kErrCapacity);
            deg += (unsigned long long)(off[v + 1] - off[v]);
        }
    }
    deg = wave_sum_u64(deg);
    if (lane_id() == 0) dpart[threadIdx.x / kWave] = deg;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kWavesPerBlock; w++) t += dpart[w];
        if (t) atomicAdd(&rc->fdeg[par], t);
    }
}

// Union-find with randomized linking (the root of lower priority is linked
// under the other; priority = a hash of the id, ties by id) and path
// splitting in find (Jayanti, Tarjan and Boix-Adsera's concurrent
// union-find, the "UF-JTB" of Algorithm 4).
__device__ __forceinline__ int32_t uf_find(int32_t *parent, int32_t x) {
    for (;;) {
        const int32_t p = (int32_t)ld_relaxed(reinterpret_cast<const uint32_t *>(parent + x));
        if (p == x) return x;
        const int32_t g = (int32_t)ld_relaxed(reinterpret_cast<const uint32_t *>(parent + p));
        if (g == p) return p;
        // x's parent moves up to its grandparent (still an ancestor of x)
        __hip_atomic_store(parent + x, g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = g;
    }
}

__device__ __forceinline__ bool uf_higher(int32_t a, int32_t b) {
    const uint64_t ha = mix64((uint64_t)(uint32_t)a ^ 0x7F4A7C15ull), hb = mix64((uint64_t)(uint32_t)b ^ 0x7F4A7C15ull);
    return ha != hb ? ha > hb : a > b;
}

__device__ __forceinline__ void uf_union(int32_t *parent, int32_t a, int32_t b) {
    for (;;) {
        a = uf_find(parent, a);
        b = uf_find(parent, b);
        if (a == b) return;
        if (uf_higher(b, a)) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        // b (the lower priority root) goes under a, unless b stopped being a root
        if (atomicCAS(parent + b, b, a) == b) return;
    }
}

// bstart[b] = the vertex whose adjacency holds arc b * A (the arc blocks of
// k_cc_union start from it).
__global__ void k_arc_block_starts(int32_t n, const int32_t *off, int64_t A, int32_t *bstart) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        const int64_t lo = off[u], hi = off[u + 1];
        for (int64_t b = (lo + A - 1) / A; b * A < hi; b++) bstart[b] = (int32_t)u;
    }
}

// The union pass: block b owns arcs [b A, (b + 1) A), thread t the run of
// A / kBlock arcs at b A + t A / kBlock; its first arc's vertex is found by a
// binary search between the vertices that start this block and the next.
constexpr int64_t kUnionArcs = 4096;
__global__ __launch_bounds__(kBlock) void k_cc_union(int32_t n, int64_t m, const int32_t *off, const int32_t *adj,
                                                     const int32_t *owner, int32_t *parent, const int32_t *bstart,
                                                     Counters *cn) {
    constexpr int64_t per = kUnionArcs / kBlock;
    const int64_t nb = (m + kUnionArcs - 1) / kUnionArcs;
    unsigned long long c_arcs = 0, c_unions = 0;
    for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
        const int64_t e0 = b * kUnionArcs + (int64_t)threadIdx.x * per;
        if (e0 >= m) continue;
        int32_t lo = bstart[b], hi = b + 1 < nb ? bstart[b + 1] : n - 1;
        while (lo < hi) {  // the largest u with off[u] <= e0
            const int32_t mid = lo + (hi - lo + 1) / 2;
            if (off[mid] <= e0) lo = mid; else hi = mid - 1;
        }
        int32_t u = lo;
        int32_t ou = owner[u];
        int64_t next = off[u + 1];
        const int64_t e1 = e0 + per < m ? e0 + per : m;
        for (int64_t e = e0; e < e1; e++) {
            if (e >= next) {
                do {
                    u++;
                    next = off[u + 1];
                } while (e >= next);
                ou = owner[u];
            }
            const int32_t ow = owner[adj[e]];
            c_arcs++;
            if (ow != ou) {
                c_unions++;
                uf_union(parent, ou, ow);
            }
        }
    }
    unsigned long long c[kNumCtr] = {0, 0, c_arcs, c_unions, 0, 0};
    block_flush_ctr(cn->c[blockIdx.x % kCtrStripes][kKindUnion], c);
}

// Final component of every vertex as a finished SCC-style key (~root), so
// that the canonical-minimum kernels turn it into the component's smallest id.
__global__ void k_cc_finish(int32_t n, const int32_t *owner, int32_t *parent, int32_t *label) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        label[v] = ~uf_find(parent, owner[v]);
}

// ------------------------------------------------------------ LE-lists ----
// Least-element lists by the BGSS batches of Algorithm 5: the vertices in a
// random order, batch i = the next 2^(i-1) of them; each batch runs a pruned
// multi-BFS (kLe rounds) from its sources, every pair (w, j) it claims at
// distance d < delta(w) is logged, and afterwards, per vertex, the pairs of
// the batch are filtered against the batch's earlier sources, delta drops to
// the best distance, and the survivors join the lists.

// Sources of a batch: srcvert[j] = the vertex at position p0 + j.
__global__ void k_le_sources(Perm P, uint32_t p0, uint32_t k, int32_t *srcvert) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < k; j += gridDim.x * blockDim.x)
        srcvert[j] = (int32_t)perm_apply(P, p0 + j);
}

__global__ void k_perm_write(Perm P, int32_t n, int32_t *order) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        order[i] = (int32_t)perm_apply(P, (uint32_t)i);
}

// Appends the frontier (the pairs first reached at distance `level`) to the
// batch log: key (w << kbits) | j, value level.  Slots from one counter, one
// reservation per block.
__global__ __launch_bounds__(kBlock) void k_le_log(const uint64_t *F, const RoundCtl *rc, int par, uint64_t fcap,
                                                   int32_t level, uint32_t kbits, uint64_t *keys, int32_t *dist,
                                                   uint64_t cap, Shared *sh) {
    uint64_t nf = rc->nF[par];
    if (nf > fcap) nf = fcap;
    for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x; i0 < nf; i0 += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t i = i0 + threadIdx.x;
        const bool h = i < nf;
        const uint64_t m = ballot(h);
        const uint32_t base = block_reserve(&sh->emit, (uint32_t)popc64(m));
        if (h) {
            const uint64_t pos = (uint64_t)base + rank_below(m);
            if (pos < cap) {
                const uint64_t e = F[i];
                keys[pos] = ((uint64_t)(uint32_t)key_vertex(e) << kbits) | key_source(e);
                dist[pos] = level;
            }
        }
    }
}

// The batch log sorted by (w, j): within a vertex's run of entries (sources
// in order), an entry survives iff its distance beats every earlier entry of
// the run (Algorithm 5 filters the triples that violate the list's order);
// the last survivor carries the new delta(w).  One thread walks each run.
__global__ void k_le_filter(const uint64_t *keys, const int32_t *dist, uint64_t cnt, uint32_t kbits, uint8_t *keep,
                            int32_t *delta) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < cnt; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t w = keys[i] >> kbits;
        if (i > 0 && (keys[i - 1] >> kbits) == w) continue;  // not the start of a run
        int32_t best = kInf32;
        uint64_t r = i;
        for (; r < cnt && (keys[r] >> kbits) == w; r++) {
            const bool k = dist[r] < best;
            keep[r] = k ? 1 : 0;
            if (k) best = dist[r];
        }
        if (best < delta[w]) delta[w] = best;
    }
}

// Survivors of a batch -> the list log: key (w << pbits) | position of the
// source, value distance.
__global__ __launch_bounds__(kBlock) void k_le_append(const uint64_t *keys, const int32_t *dist, const uint8_t *keep,
                                                      uint64_t cnt, uint32_t kbits, uint32_t p0, uint32_t pbits,
                                                      uint64_t *lkeys, int32_t *ldist, uint64_t cap,
                                                      unsigned long long *cursor) {
    __shared__ uint32_t part[kWavesPerBlock];
    __shared__ unsigned long long base_s;
    for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x; i0 < cnt; i0 += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t i = i0 + threadIdx.x;
        const bool h = i < cnt && keep[i];
        const uint64_t m = ballot(h);
        if (lane_id() == 0) part[threadIdx.x / kWave] = (uint32_t)popc64(m);
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long t = 0;
            for (int w = 0; w < kWavesPerBlock; w++) t += part[w];
            base_s = t ? atomicAdd(cursor, t) : 0ull;
        }
        __syncthreads();
        unsigned long long b = base_s;
        for (int w = 0; w < (int)(threadIdx.x / kWave); w++) b += part[w];
        __syncthreads();
        if (h) {
            const uint64_t pos = b + rank_below(m);
            if (pos < cap) {
                const uint64_t w = keys[i] >> kbits;
                const uint64_t j = keys[i] & ((1ull << kbits) - 1);
                lkeys[pos] = (w << pbits) | (p0 + j);
                ldist[pos] = dist[i];
            }
        }
    }
}

// The sorted list log -> CSR: loff[w] = first entry of w; sources recovered
// from their positions.
__global__ void k_le_csr(const uint64_t *lkeys, const int32_t *ldist, uint64_t cnt, uint32_t pbits, int32_t n, Perm P,
                         int64_t *loff, int32_t *src, int32_t *dist) {
    const uint64_t pmask = (1ull << pbits) - 1;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i <= cnt; i += (uint64_t)gridDim.x * blockDim.x) {
        const int64_t w = i < cnt ? (int64_t)(lkeys[i] >> pbits) : (int64_t)n;
        const int64_t wp = i > 0 ? (int64_t)(lkeys[i - 1] >> pbits) : -1;
        for (int64_t x = wp + 1; x <= w; x++) loff[x] = (int64_t)i;  // vertices without entries in between
        if (i < cnt) {
            src[i] = (int32_t)perm_apply(P, (uint32_t)(lkeys[i] & pmask));
            dist[i] = ldist[i];
        }
    }
}

// ------------------------------------------------------------ bag test ----
// Inserts keys[i] for i with i % rounds == rr, one element per lane.
__global__ __launch_bounds__(kBlock) void k_bag_insert_test(const uint64_t *keys, int64_t n, int32_t rounds,
                                                             int32_t rr, Bag B, Counters *cn) {
    const uint32_t nwaves = gridDim.x * kWavesPerBlock;
    const uint32_t wave_gid = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    uint32_t wseq = 0;
    const int64_t cnt = (n - rr + rounds - 1) / rounds;  // elements of this round
    unsigned long long ins = 0;
    for (int64_t b = (int64_t)wave_gid * kWave; b < cnt; b += (int64_t)nwaves * kWave) {
        const int64_t i = b + lane_id();
        const bool h = i < cnt;
        const uint64_t e = h ? keys[i * rounds + rr] : 0;
        ins += (unsigned long long)bag_insert_wave(B, h, e, wave_gid, wseq);
    }
    ins = wave_sum_u64(ins);
    if (lane_id() == 0 && ins) atomicAdd(&cn->c[blockIdx.x % kCtrStripes][kKindExpandSingle][kCtrInserts], ins);
}

__global__ void k_copy_u64(const uint64_t *src, uint64_t *dst, const RoundCtl *rc, int par, uint64_t cap) {
    const uint32_t n = rc->nF[par];
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n && i < cap; i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

}  // namespace hipscc
