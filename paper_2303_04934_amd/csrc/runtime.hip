// hipscc host runtime: the C ABI of include/hipscc.h.
//
// Algorithm 1 (BGSS) is driven from the host one source batch at a time.  The
// forward and the backward search of a batch run as two "lanes" whose rounds
// (expand -> edge-parallel -> ExtractAll, or a dense pull round) are launched
// interleaved on one stream; the host looks at the frontier sizes only between
// blocks of rounds.  Everything a batch needs (its source, its sources' count)
// is resolved on the device, so consecutive batches do not wait for the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <type_traits>
#include <utility>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>

#include "hipscc.h"
#include "kernels.h"

using namespace hipscc;

namespace {

// Device control block: the part before `cn` is copied to the host at every
// check; the counters only when statistics are gathered.
struct DevCtl {
    RoundCtl lane[2];
    BagCtl bag[2];
    Shared sh;
    CountStripes cs;
    Counters cn;
    LaneStripes ls[2];
};
constexpr size_t kCtlHead = offsetof(DevCtl, cn);

template <typename T>
struct DevBuf {
    T *p = nullptr;
    uint64_t cap = 0;  // elements
};

struct Fail {
    scc_status code;
};

constexpr int kMaxSlots = 64;   // rounds per launch block
constexpr int kTimedMax = 4 * kMaxSlots;  // timed launches between host checks
constexpr int kPhases = 5;      // trim, first, multi, resize, label
constexpr uint32_t kProbeLimit = 128;
constexpr uint64_t kCheapPairs = 4;  // reach pairs per source of a batch that counts as cheap
constexpr uint64_t kDenseLabelDiv = 8;
constexpr int64_t kShortRounds = 4;      // a batch of at most this many rounds per direction is short ...
constexpr double kShortGrowth = 64.0;
constexpr int kMaxUnionStreams = 8;      // concurrent unions of scc_labels_batched
constexpr int kAutoUnionStreams = 2;    // ... and the next one grows by this factor  // relabel per vertex once a batch has n / 8 pairs

}  // namespace

struct scc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int num_cu = 256;
    uint64_t table_slots_max = 1ull << 24;  // cap of the estimated reach-table size (set from device memory)
    int expand_blocks = 2048;
    int expand_grid[6][3] = {};     // resident-grid size per (mode, log2 arcs per lane)
    int arcs_per_lane = 1;          // options.arcs_per_lane of the current call
    double vgc_fill = 2.0;          // options.vgc_fill of the current call
    std::string err;

    DevBuf<int32_t> label, aux, stamp, srcvert, srclab, fin;
    DevBuf<uint32_t> invp;          // inverse vertex permutation (large source batches)
    DevBuf<unsigned long long> sig_out, sig_in;
    DevBuf<uint32_t> vis[2];        // visited bitmaps of the two single-source lanes
    DevBuf<uint32_t> bm[2][2];      // front/next bitmaps per lane (dense mode)
    DevBuf<uint64_t> Tout, Tin;     // reach tables (forward, backward)
    DevBuf<int32_t> firstS[2];      // first-source slots per direction (options.first_slot)
    DevBuf<int4> rec[2];            // packed per-vertex records per direction (options.packed)
    DevBuf<uint8_t> dirty;          // granules with a claimed first-source slot (kept all clear between batches)
    int64_t first_clean_n = 0;      // the slots are known empty (-1) on [0, first_clean_n)
    DevBuf<uint64_t> F[2], heavy[2];
    DevBuf<uint64_t> bag_slots[2];
    DevBuf<uint32_t> bag_cnt[2];
    uint32_t bag_nchunks[2] = {0, 0};
    uint32_t bag_lam_log2[2] = {0, 0};  // each lane's first-chunk size (log2)
    DevCtl *dctl = nullptr;
    DevCtl *hctl = nullptr;         // pinned
    DevBuf<int32_t> ubuf;           // batched: union CSR scratch
    DevBuf<uint64_t> rkeys[2];      // scc_reach: pair sort keys (double buffer)
    DevBuf<uint8_t> rtemp;          // scc_reach: radix sort scratch
    DevBuf<int32_t> bstart;         // scc_cc: first vertex of each arc block
    // scc_le_lists: a batch's pair log and its sorted copy, the keep flags,
    // the list log and its sorted copy
    DevBuf<uint64_t> lk[2], gk[2];
    DevBuf<int32_t> ld[2], gd[2];
    DevBuf<uint8_t> lkeep;
    uint32_t salt = 1;
    bool tables_dirty = false;      // a failed call may leave claims behind
    // stamp/fin/sig_in/sig_out are known clean on [0, vclean_n) (zero sums,
    // no finish mark, stamps below stamp_next): each batch's relabel leaves
    // them so, and a call that ends normally starts the next one clean
    int64_t vclean_n = 0;
    int32_t stamp_next = 1;
    // options.timing: events around frontier-kernel launches
    uint32_t timing = 0;            // options.timing: bit k times kernel k (SCC_KERNEL_*)
    hipEvent_t tev[kTimedMax][2] = {};  // timed launches since the last host check
    int tev_kind[kTimedMax] = {};
    int tev_n = 0;
    double tm_ms[SCC_KERNELS] = {};
    int64_t tm_launches[SCC_KERNELS] = {};
    int64_t dense_rounds = 0;
    // options.trace rows and the round events that time them
    bool tracing = false;
    std::vector<float> trace;
    hipEvent_t rev[2][2] = {};
    int32_t epoch = 0;
    uint64_t explore_state = 0;
    // phase events (statistics)
    std::vector<hipEvent_t> pev;
    size_t pev_used = 0;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> plog;
    Policy policy;
    // scc_labels_batched with concurrent unions: one context per stream,
    // owned by this one (created on first use, destroyed with it)
    std::vector<scc_ctx *> workers;
    size_t worker_groups = 0;       // unions of the workers' last batch
    // scc_labels_static: this device's copy of the static scratch array, and
    // whether the current call must not allocate (buffers are carved views)
    uint8_t *scratch = nullptr;
    bool noalloc = false;
    // options.graph_rounds: captured blocks of sparse rounds, keyed by the
    // block's round count and its lanes' launch arguments
    bool graph_rounds = false;
    std::vector<std::pair<std::vector<uint8_t>, hipGraphExec_t>> gcache;
    // statistics of the last scc_bag_selftest: (round, chunk, load, cause) for
    // every chunk left before its round's ExtractAll, and each round's used
    // prefix
    std::vector<double> bag_rows;
    std::vector<int64_t> bag_prefix;
};

namespace {

void set_err(scc_ctx *c, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
}

#define HIPCHK(call)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) {                                                                   \
            set_err(c, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
            throw Fail{SCC_EHIP};                                                                 \
        }                                                                                         \
    } while (0)

#define LAUNCHCHK(name)                                                                          \
    do {                                                                                         \
        hipError_t e_ = hipGetLastError();                                                       \
        if (e_ != hipSuccess) {                                                                  \
            set_err(c, "launch of %s failed: %s", name, hipGetErrorString(e_));                  \
            throw Fail{SCC_EHIP};                                                                \
        }                                                                                        \
    } while (0)

template <typename T>
void ensure(scc_ctx *c, DevBuf<T> &b, uint64_t n, bool *grew = nullptr) {
    if (grew) *grew = false;
    if (n == 0) n = 1;
    if (b.cap >= n) return;
    if (c->noalloc) {
        set_err(c, "a buffer of %llu elements exceeds its part of the static scratch (%llu)", (unsigned long long)n,
                (unsigned long long)b.cap);
        throw Fail{SCC_ECAPACITY};
    }
    if (b.p) {
        HIPCHK(hipStreamSynchronize(c->stream));
        HIPCHK(hipFree(b.p));
        b.p = nullptr;
        b.cap = 0;
    }
    uint64_t want = n + n / 8 + 64;
    hipError_t e = hipMalloc((void **)&b.p, want * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        set_err(c, "hipMalloc of %llu bytes failed: %s", (unsigned long long)(want * sizeof(T)), hipGetErrorString(e));
        throw Fail{SCC_ENOMEM};
    }
    b.cap = want;
    if (grew) *grew = true;
}

// Grows b to at least n elements keeping its first `keep` elements.
template <typename T>
void grow_keep(scc_ctx *c, DevBuf<T> &b, uint64_t n, uint64_t keep) {
    if (b.cap >= n) return;
    DevBuf<T> nb;
    ensure(c, nb, n);
    if (keep > 0 && b.p)
        HIPCHK(hipMemcpyAsync(nb.p, b.p, sizeof(T) * std::min<uint64_t>(keep, b.cap), hipMemcpyDeviceToDevice,
                              c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (b.p) HIPCHK(hipFree(b.p));
    b = nb;
}

template <typename T>
void release(DevBuf<T> &b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

inline unsigned grid_for(scc_ctx *c, uint64_t n, unsigned per_cu = 16) {
    uint64_t g = (n + kBlock - 1) / kBlock;
    uint64_t mx = (uint64_t)c->num_cu * per_cu;
    if (g > mx) g = mx;
    if (g < 1) g = 1;
    return (unsigned)g;
}

void fill_u32(scc_ctx *c, uint32_t *p, uint64_t n, uint32_t v) {
    if (!n) return;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(c, n)), dim3(kBlock), 0, c->stream, p, n, v);
    LAUNCHCHK("k_fill_u32");
}
void fill_u64(scc_ctx *c, uint64_t *p, uint64_t n, uint64_t v) {
    if (!n) return;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(c, n)), dim3(kBlock), 0, c->stream, p, n, v);
    LAUNCHCHK("k_fill_u64");
}

// Copies the control head (lanes, bags, shared values) to the host and waits.
void sync_ctl(scc_ctx *c, bool with_counters = false) {
    HIPCHK(hipMemcpyAsync(c->hctl, c->dctl, with_counters ? sizeof(DevCtl) : kCtlHead, hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
}

// Sums of the striped call-level counts (host copy, after sync_ctl).
int64_t count_sum(const scc_ctx *c, uint32_t CountLine::*f) {
    int64_t t = 0;
    for (int i = 0; i < kStripes; i++) t += c->hctl->cs.s[i].*f;
    return t;
}

// Zeroes the whole control block inside the stream (a fill kernel, no memset).
// (the host mirror's degree maximum is cleared too: until a check copies the
// new call's value, a stale one would let a launch skip a needed pass)
void reset_ctl(scc_ctx *c) {
    fill_u32(c, (uint32_t *)c->dctl, sizeof(DevCtl) / 4, 0u);
    c->hctl->sh.max_deg = 0;
}
void reset_lane_ctl(scc_ctx *c, int id) { fill_u32(c, (uint32_t *)&c->dctl->lane[id], sizeof(RoundCtl) / 4, 0u); }

uint64_t next_pow2(uint64_t x) {
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

// ------------------------------------------------------------- phase log --
void phase_begin(scc_ctx *c, int phase, bool on) {
    if (!on) return;
    if (c->pev_used + 2 > c->pev.size()) {
        for (int i = 0; i < 64; i++) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            c->pev.push_back(e);
        }
    }
    hipEvent_t a = c->pev[c->pev_used++], b = c->pev[c->pev_used++];
    HIPCHK(hipEventRecord(a, c->stream));
    c->plog.push_back({phase, {a, b}});
}
void phase_end(scc_ctx *c, bool on) {
    if (!on || c->plog.empty()) return;
    HIPCHK(hipEventRecord(c->plog.back().second.second, c->stream));
}
// After a final sync: sums the logged phase intervals into ms[kPhases].
void phase_collect(scc_ctx *c, double *ms) {
    for (auto &e : c->plog) {
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, e.second.first, e.second.second));
        ms[e.first] += t;
    }
    c->plog.clear();
    c->pev_used = 0;
}

scc_options_t defaults() {
    scc_options_t o;
    memset(&o, 0, sizeof o);
    o.tau = 2048;
    o.beta = 2.0f;
    o.beta_fast = 4.0f;
    o.table_floor = 1.2f;
    o.lambda_log2 = 0;
    o.sigma = 50;
    o.kappa = 32;
    o.alpha = 0.5f;
    o.seed = 0x5EEDull;
    o.policy = 0;
    o.dense = -1;
    o.validate = 1;
    o.trim = 1;
    o.table_init = 0;
    o.seeds_per_wave = 0;
    o.timing = 0;
    o.ldd_beta = 1.2f;
    o.first_slot = 1;
    o.packed = -1;
    o.union_streams = 0;
    o.tau_single = 0;
    return o;
}

int32_t single_tau(const scc_options_t &o) {
    if (o.tau_single > 0) return o.tau_single;
    if (o.tau <= 1) return o.tau;
    return (int32_t)std::min<int64_t>(4 * (int64_t)o.tau, 1 << 30);
}

// log2 of the hash bag's first chunk for searches of up to `entries` entries
// per round.  options.lambda_log2 = 0 picks it: every wavefront that inserts
// reserves room in one random 64-slot stripe of the current chunk, so the
// first chunk needs many stripes to keep thousands of wavefronts' atomics
// apart: 2^20 slots, or less for small searches (at least 2^10, the paper's
// value for tens of threads).
uint32_t lam_log2_for(const scc_options_t &o, uint64_t entries) {
    if (o.lambda_log2 > 0) return (uint32_t)o.lambda_log2;
    uint32_t l = 10;
    while (l < 20 && (1ull << l) < entries) l++;
    return l;
}

void check_opts(scc_ctx *c, const scc_options_t &o) {
    if (!(o.table_floor >= 0.f) || !(o.table_floor <= 16.f)) {
        set_err(c, "table_floor must be in [0, 16]");
        throw Fail{SCC_EINVAL};
    }
    if (!(o.vgc_fill >= -1e6f && o.vgc_fill <= 1e6f) || !(o.beta_fast >= 0.f && o.beta_fast <= 1e6f)) {
        set_err(c, "vgc_fill / beta_fast out of range");
        throw Fail{SCC_EINVAL};
    }
    if (o.arcs_per_lane != 0 && o.arcs_per_lane != 1 && o.arcs_per_lane != 2 && o.arcs_per_lane != 4) {
        set_err(c, "arcs_per_lane must be 0, 1, 2 or 4");
        throw Fail{SCC_EINVAL};
    }
    if (!(o.beta > 1.0f) || !(o.beta < 1e6f)) { set_err(c, "beta must be > 1"); throw Fail{SCC_EINVAL}; }
    if (o.lambda_log2 != 0 && (o.lambda_log2 < kStripeLog2 || o.lambda_log2 > 24)) {
        set_err(c, "lambda_log2 must be 0 (automatic) or in [%d, 24]", kStripeLog2);
        throw Fail{SCC_EINVAL};
    }
    if (o.sigma < 1 || o.kappa < 0 || !(o.alpha > 0.f && o.alpha < 1.f)) {
        set_err(c, "sigma >= 1, kappa >= 0 and 0 < alpha < 1 required");
        throw Fail{SCC_EINVAL};
    }
    if (o.seeds_per_wave < 0 || o.seeds_per_wave > 64) { set_err(c, "seeds_per_wave in [0, 64]"); throw Fail{SCC_EINVAL}; }
    if (o.table_init < 0 || (o.table_init & (o.table_init - 1))) {
        set_err(c, "table_init must be 0 or a power of two");
        throw Fail{SCC_EINVAL};
    }
    if (o.policy < 0 || o.policy > 2) { set_err(c, "policy must be 0, 1 or 2"); throw Fail{SCC_EINVAL}; }
    if (o.dense < -1 || o.dense > 1) { set_err(c, "dense must be -1, 0 or 1"); throw Fail{SCC_EINVAL}; }
    if (o.union_arcs_max < 0) { set_err(c, "union_arcs_max must be >= 0"); throw Fail{SCC_EINVAL}; }
    if (o.first_slot < 0 || o.first_slot > 1) { set_err(c, "first_slot must be 0 or 1"); throw Fail{SCC_EINVAL}; }
    if (o.vgc_measure < 0 || o.vgc_measure > 1) { set_err(c, "vgc_measure must be 0 or 1"); throw Fail{SCC_EINVAL}; }
    if (o.packed < -1 || o.packed > 1) { set_err(c, "packed must be -1, 0 or 1"); throw Fail{SCC_EINVAL}; }
    if (o.tau_single < 0) {
        set_err(c, "tau_single must be >= 0");
        throw Fail{SCC_EINVAL};
    }
    if (o.union_streams < 0 || o.union_streams > kMaxUnionStreams) {
        set_err(c, "union_streams must be in [0, %d]", kMaxUnionStreams);
        throw Fail{SCC_EINVAL};
    }
    if (!(o.ldd_beta > 1.0f) || !(o.ldd_beta < 1e6f)) { set_err(c, "ldd_beta must be > 1"); throw Fail{SCC_EINVAL}; }
}

// Buffers of lane `id` sized for up to `entries` frontier entries per round.
// The hash bag's capacity is the smallest lambda * 2^j >= 2 (entries + lambda)
// (reading of Section 3.3 with alpha = 1/2: the last chunk alone then holds
// every element).
void ensure_lane(scc_ctx *c, int id, uint64_t entries, uint32_t lam_log2) {
    const uint64_t lam = 1ull << lam_log2;
    uint32_t nch = 1;
    while ((lam << (nch - 1)) < 2 * (entries + lam)) nch++;
    if (nch > (uint32_t)kMaxChunks) { set_err(c, "hash bag too large"); throw Fail{SCC_ENOMEM}; }
    const uint64_t cap = lam << (nch - 1);
    bool g2 = false;
    ensure(c, c->bag_slots[id], cap);
    ensure(c, c->bag_cnt[id], cap >> kStripeLog2, &g2);
    // the chunk count belongs to the lane's own lambda: it is recomputed
    // whenever that lambda changes, and only grows while it stays
    const bool lam_changed = lam_log2 != c->bag_lam_log2[id];
    if (g2 || lam_changed) fill_u32(c, c->bag_cnt[id].p, c->bag_cnt[id].cap, 0u);
    if (nch > c->bag_nchunks[id] || lam_changed) c->bag_nchunks[id] = nch;
    c->bag_lam_log2[id] = lam_log2;
    ensure(c, c->F[id], entries + kWave);
    ensure(c, c->heavy[id], 2 * (entries + kWave));
}

// Clears lane id's bag (its stripe counters and chunk state).
void reset_bag(scc_ctx *c, int id) {
    fill_u32(c, c->bag_cnt[id].p, c->bag_cnt[id].cap, 0u);
    fill_u32(c, (uint32_t *)&c->dctl->bag[id], sizeof(BagCtl) / 4, 0u);
}

Search make_search(scc_ctx *c, int id, const scc_options_t &o, int mode) {
    Search S;
    memset(&S, 0, sizeof S);
    S.F = c->F[id].p;
    S.heavy = c->heavy[id].p;
    S.fcap = c->F[id].cap;
    S.hcap = c->heavy[id].cap / 2;
    S.bag.slots = c->bag_slots[id].p;
    S.bag.cnt = c->bag_cnt[id].p;
    S.bag.ctl = &c->dctl->bag[id];
    S.bag.lam_log2 = c->bag_lam_log2[id];
    S.bag.nchunks = c->bag_nchunks[id];
    // every chunk the kernels may use lies inside the lane's slot and
    // stripe-counter buffers
    const uint64_t used = (1ull << S.bag.lam_log2) << (S.bag.nchunks ? S.bag.nchunks - 1 : 0);
    if (S.bag.nchunks < 1 || S.bag.nchunks > (uint32_t)kMaxChunks || used > c->bag_slots[id].cap ||
        (used >> kStripeLog2) > c->bag_cnt[id].cap) {
        set_err(c, "internal: hash bag of lane %d (lambda 2^%u, %u chunks) exceeds its buffers", id,
                S.bag.lam_log2, S.bag.nchunks);
        throw Fail{SCC_EINTERNAL};
    }
    S.bag.sigma = (uint32_t)o.sigma;
    S.bag.kappa = (uint32_t)o.kappa;
    S.bag.alpha = o.alpha;
    S.rc = &c->dctl->lane[id];
    S.ls = &c->dctl->ls[id];
    S.cn = &c->dctl->cn;
    S.kind = (mode == kMulti || mode == kMultiFirst || mode == kLe || mode == kMultiRec) ? kKindExpandMulti
                                                                                        : kKindExpandSingle;
    // a single-source search gets the longer budget of tau_single
    S.tau = mode == kSingle ? single_tau(o) : o.tau;
    S.seeds = o.seeds_per_wave;
    S.heavy_deg = 1024;
    S.probe_limit = kProbeLimit;
    S.vgc_cut = (uint32_t)c->expand_blocks * kWavesPerBlock;
    S.measure = o.vgc_measure;
    return S;
}

// ------------------------------------------------------------------ lanes --
struct Lane {
    int id = 0;
    int mode = kSingle;
    Search S;
    bool live = false;
    int par = 0;
    uint64_t nf = 0;
    double growth = 1.0;     // frontier growth per round (host estimate)
    int64_t rounds = 0;
    // state before the round, for trace rows
    uint64_t fdeg = 0, claims = 0;
    uint32_t tau_used = 0;
    int64_t nsub = 1;
    double avg_deg = 1.0;    // arcs per vertex of the graph (local-search cut)
    bool policy_primed = false;  // the learned policy has picked this search's first budget
    // single source
    bool dense = false, have_list = true;
    const int32_t *roff = nullptr, *radj = nullptr;
    int32_t n = 0;
    // multi source
    DevBuf<uint64_t> *T = nullptr;
    uint64_t *tslots = nullptr;
    uint64_t *fslots = nullptr;  // frontier entries its buffers hold (null: from tslots)
};

struct DriveParams {
    const scc_options_t *o = nullptr;
    int64_t n = 0;           // vertices of the graph
    int64_t m = 0;           // arcs of the graph
    int64_t nsub = 0;        // active vertices (upper bound)
    scc_stats_t *st = nullptr;
    double *resize_ms = nullptr;
    uint64_t peak_fdeg = 0;  // out: largest frontier degree sum seen at a host check
    uint32_t table_full = 0; // out: restarts caused by a full reach table
    bool abandon_on_overflow = false;  // a multi-source overflow abandons the batch instead of restarting
    bool abandoned = false;  // out: the batch was abandoned (every lane stopped, nothing cleared yet)
};

// ExtractAll grid: each block walks 256 stripes (16K slots) per step, and the
// last-block ticket costs one atomic per block, so a modest grid suffices.
unsigned extract_blocks(scc_ctx *c) { return (unsigned)std::max(c->num_cu / 2, 1); }

// Before a round: the learned policy picks each sparse lane's budget on the
// device (one launch for the round's lanes), and for a single-source lane
// also the frontier mode of the next round, which the host applies at its
// checks; exploration draws a random budget class per lane.
void launch_policy(scc_ctx *c, Lane **ls, int nl, const scc_options_t &o) {
    if (nl == 0) return;
    if (o.policy == 1 && c->policy.loaded) {
        // a search's first round gets its budget from a launch of its own;
        // later rounds get it from the previous round's ExtractAll (traced
        // runs keep the launch, so that a row records the budget it used)
        PolicyLane P[2];
        memset(P, 0, sizeof P);
        int np = 0;
        for (int j = 0; j < nl; j++) {
            Lane &L = *ls[j];
            L.S.tau_from_rc = 1;
            L.S.policy_w = c->tracing ? nullptr : c->policy.w;
            L.S.nsub = (float)L.nsub;
            L.S.fallback_tau = (uint32_t)std::max(o.tau, 0);
            if (L.policy_primed && !c->tracing) continue;
            RoundCtl *rc = L.S.rc;
            P[np++] = PolicyLane{rc->nF, &rc->fdeg[L.par], &rc->claims, &rc->rounds, &rc->lsdepth[L.par ^ 1],
                                 (float)L.nsub, &rc->tau_cur, &rc->mode_pref, &rc->policy_calls, &rc->policy_fallbacks,
                                 L.mode == kSingle ? 3u : 1u};
            L.policy_primed = true;
        }
        if (np) {
            hipLaunchKernelGGL(k_policy_round, dim3(np), dim3(64), 0, c->stream, c->policy.w, P[0], P[np > 1 ? 1 : 0],
                               (uint32_t)std::max(o.tau, 0));
            LAUNCHCHK("k_policy_round");
        }
    } else if (o.policy == 2) {
        for (int j = 0; j < nl; j++) {
            c->explore_state = mix64(c->explore_state + 0x9E3779B97F4A7C15ull);
            ls[j]->S.tau = (int32_t)policy_tau((int)(c->explore_state >> 62));
            ls[j]->S.tau_from_rc = 0;
        }
    }
}

// options.timing: HIP events around one frontier-kernel launch of `kind`;
// the host adds them up at its next check (timed_collect).
int timed_begin(scc_ctx *c, int kind) {
    if (!((c->timing >> kind) & 1) || c->tev_n >= kTimedMax) return -1;
    const int i = c->tev_n++;
    c->tev_kind[i] = kind;
    HIPCHK(hipEventRecord(c->tev[i][0], c->stream));
    return i;
}
void timed_end(scc_ctx *c, int i) {
    if (i >= 0) HIPCHK(hipEventRecord(c->tev[i][1], c->stream));
}
void timed_collect(scc_ctx *c) {
    for (int i = 0; i < c->tev_n; i++) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, c->tev[i][0], c->tev[i][1]));
        c->tm_ms[c->tev_kind[i]] += ms;
        c->tm_launches[c->tev_kind[i]] += 1;
    }
    c->tev_n = 0;
}

// The expand kernel of a search mode and arcs-per-lane setting.
const void *expand_kernel(int mode, int apl) {
    if (mode == kMultiRec) {
        if (apl == 1) return reinterpret_cast<const void *>(&k_expand<kMultiRec, 1>);
        if (apl == 2) return reinterpret_cast<const void *>(&k_expand<kMultiRec, 2>);
        return reinterpret_cast<const void *>(&k_expand<kMultiRec, 4>);
    }
    if (mode == kLe) {
        if (apl == 1) return reinterpret_cast<const void *>(&k_expand<kLe, 1>);
        if (apl == 2) return reinterpret_cast<const void *>(&k_expand<kLe, 2>);
        return reinterpret_cast<const void *>(&k_expand<kLe, 4>);
    }
    if (mode == kLdd) {
        if (apl == 1) return reinterpret_cast<const void *>(&k_expand<kLdd, 1>);
        if (apl == 2) return reinterpret_cast<const void *>(&k_expand<kLdd, 2>);
        return reinterpret_cast<const void *>(&k_expand<kLdd, 4>);
    }
    if (mode == kMultiFirst) {
        if (apl == 1) return reinterpret_cast<const void *>(&k_expand<kMultiFirst, 1>);
        if (apl == 2) return reinterpret_cast<const void *>(&k_expand<kMultiFirst, 2>);
        return reinterpret_cast<const void *>(&k_expand<kMultiFirst, 4>);
    }
    if (mode == kMulti) {
        if (apl == 1) return reinterpret_cast<const void *>(&k_expand<kMulti, 1>);
        if (apl == 2) return reinterpret_cast<const void *>(&k_expand<kMulti, 2>);
        return reinterpret_cast<const void *>(&k_expand<kMulti, 4>);
    }
    if (apl == 1) return reinterpret_cast<const void *>(&k_expand<kSingle, 1>);
    if (apl == 2) return reinterpret_cast<const void *>(&k_expand<kSingle, 2>);
    return reinterpret_cast<const void *>(&k_expand<kSingle, 4>);
}

// One sparse round of one or two lanes of the same mode: expand, the
// edge-parallel pass over deferred heavy entries, and ExtractAll, each one
// launch for both lanes (the grid split between them).
void launch_sparse(scc_ctx *c, Lane **ls, int nl) {
    LanePair P;
    memset(&P, 0, sizeof P);
    P.nl = nl;
    const int mode = ls[0]->mode;
    const int ai = c->arcs_per_lane == 1 ? 0 : (c->arcs_per_lane == 2 ? 1 : 2);
    const unsigned eb = (unsigned)c->expand_grid[mode][ai];
    const unsigned hb = (unsigned)c->num_cu * 4;
    const unsigned xb = extract_blocks(c) * (unsigned)nl;
    for (int j = 0; j < nl; j++) {
        Search &S = ls[j]->S;
        S.par = ls[j]->par;
        S.bag.salt = c->salt++;
        const unsigned mine = nl == 2 ? (j == 0 ? eb / 2 : eb - eb / 2) : eb;
        // local search while the frontier's arcs leave the lanes short of work
        const double waves = (double)mine * kWavesPerBlock;
        const double arcs = c->vgc_fill > 0 ? c->vgc_fill * (double)mine * kBlock : 0.0;
        S.vgc_cut = (uint32_t)std::min(std::max(waves, arcs / ls[j]->avg_deg), 2147483647.0);
        S.vgc_arcs = c->vgc_fill > 0 ? (unsigned long long)arcs : 0ull;
        P.S[j] = S;
    }
    P.split = eb / 2;
    const int t = timed_begin(c, P.S[0].kind);
    const void *fn = expand_kernel(mode, c->arcs_per_lane);
    void *args[] = {&P};
    HIPCHK(hipLaunchKernel(fn, dim3(eb), dim3(kBlock), args, 0, c->stream));
    timed_end(c, t);
    P.split = hb / 2;
    // no vertex of the graph has more arcs than the heavy threshold (known
    // once a host check has seen the degree maximum): no entry can be
    // deferred, and the edge-parallel pass has nothing to do
    const uint32_t dmax = c->hctl->sh.max_deg;
    const bool no_heavy = dmax > 0 && dmax <= (uint32_t)ls[0]->S.heavy_deg &&
                          (nl < 2 || dmax <= (uint32_t)ls[1]->S.heavy_deg);
    const bool pairs = mode == kMulti || mode == kMultiFirst || mode == kLe || mode == kMultiRec;
    if (!no_heavy) {
        const int th = timed_begin(c, pairs ? SCC_KERNEL_HEAVY_MULTI : SCC_KERNEL_HEAVY_SINGLE);
        if (mode == kMultiRec) hipLaunchKernelGGL(k_expand_heavy<kMultiRec>, dim3(hb), dim3(kBlock), 0, c->stream, P);
        else if (mode == kLe) hipLaunchKernelGGL(k_expand_heavy<kLe>, dim3(hb), dim3(kBlock), 0, c->stream, P);
        else if (mode == kLdd) hipLaunchKernelGGL(k_expand_heavy<kLdd>, dim3(hb), dim3(kBlock), 0, c->stream, P);
        else if (mode == kMultiFirst)
            hipLaunchKernelGGL(k_expand_heavy<kMultiFirst>, dim3(hb), dim3(kBlock), 0, c->stream, P);
        else if (mode == kMulti) hipLaunchKernelGGL(k_expand_heavy<kMulti>, dim3(hb), dim3(kBlock), 0, c->stream, P);
        else hipLaunchKernelGGL(k_expand_heavy<kSingle>, dim3(hb), dim3(kBlock), 0, c->stream, P);
        LAUNCHCHK("k_expand_heavy");
        timed_end(c, th);
    }
    P.split = xb / 2;
    const int tx = timed_begin(c, SCC_KERNEL_EXTRACT);
    hipLaunchKernelGGL(k_bag_extract, dim3(xb), dim3(kBlock), 0, c->stream, P);
    LAUNCHCHK("k_bag_extract");
    timed_end(c, tx);
    for (int j = 0; j < nl; j++) ls[j]->par ^= 1;
}

void launch_dense(scc_ctx *c, Lane &L) {
    Search &S = L.S;
    uint32_t *front = c->bm[L.id][0].p;
    uint32_t *next = c->bm[L.id][1].p;
    const uint64_t words = (uint64_t)L.n / 32 + 2;
    if (L.have_list) {
        fill_u32(c, front, words, 0u);
        hipLaunchKernelGGL(k_list_to_bitmap, dim3(grid_for(c, L.nf)), dim3(kBlock), 0, c->stream, S.F, S.rc, L.par,
                           S.fcap, front);
        LAUNCHCHK("k_list_to_bitmap");
        L.have_list = false;
    }
    const int t = timed_begin(c, kKindPull);
    hipLaunchKernelGGL(k_pull, dim3(grid_for(c, (uint64_t)L.n)), dim3(kBlock), 0, c->stream, L.n, L.roff, L.radj, S.vis,
                       front, next, S.ls, S.cn);
    LAUNCHCHK("k_pull");
    timed_end(c, t);
    hipLaunchKernelGGL(k_round_end, dim3(1), dim3(64), 0, c->stream, S.rc, S.ls, L.par);
    LAUNCHCHK("k_round_end");
    std::swap(c->bm[L.id][0], c->bm[L.id][1]);
    L.par ^= 1;
}

// options.graph_rounds: k sparse rounds of the lanes sp as one HIP graph.
// The block is captured the first time (the launches are exactly those of
// launch_sparse) and replayed whenever a block with the same round count,
// lanes and launch arguments comes again (the bag's per-round salt, which
// only decorrelates stripe choices, repeats with the graph).
void run_graph_block(scc_ctx *c, Lane **sp, int nsp, int k) {
    // (the degree maximum decides whether the block holds edge-parallel passes)
    const uint32_t dmax = c->hctl->sh.max_deg;
    std::vector<uint8_t> key(2 * sizeof(int) + sizeof(uint32_t) + (size_t)nsp * (sizeof(Search) + sizeof(int)));
    uint8_t *q = key.data();
    memcpy(q, &k, sizeof(int));
    memcpy(q + sizeof(int), &nsp, sizeof(int));
    memcpy(q + 2 * sizeof(int), &dmax, sizeof(uint32_t));
    q += 2 * sizeof(int) + sizeof(uint32_t);
    for (int j = 0; j < nsp; j++) {
        Search s = sp[j]->S;
        s.bag.salt = 0;
        s.par = sp[j]->par;
        memcpy(q, &s, sizeof(Search));
        memcpy(q + sizeof(Search), &sp[j]->mode, sizeof(int));
        q += sizeof(Search) + sizeof(int);
    }
    for (auto &e : c->gcache)
        if (e.first == key) {
            HIPCHK(hipGraphLaunch(e.second, c->stream));
            for (int j = 0; j < nsp; j++) sp[j]->par ^= (k & 1);
            return;
        }
    if (c->gcache.size() >= 64) {
        HIPCHK(hipStreamSynchronize(c->stream));
        for (auto &e : c->gcache) (void)hipGraphExecDestroy(e.second);
        c->gcache.clear();
    }
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
    for (int r = 0; r < k; r++) launch_sparse(c, sp, nsp);
    HIPCHK(hipStreamEndCapture(c->stream, &g));
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        set_err(c, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
        throw Fail{SCC_EHIP};
    }
    c->gcache.push_back({std::move(key), ex});
    HIPCHK(hipGraphLaunch(ex, c->stream));
}

// A multi-source lane whose reach table or frontier buffers overflowed
// restarts with the one that ran out larger (Section 4.5 resizes once an
// insertion probes too often; the table cannot grow while claims are in
// flight).  A full table grows fourfold: the abandoned attempt's work is
// lost, and reach counts are heavy tailed, so a second restart costs more than
// the larger table.  A lane without its own frontier size sizes the buffers
// from the table.
void restart_multi(scc_ctx *c, Lane &L, DriveParams &P, bool table_full, bool lane_full) {
    auto t0 = std::chrono::steady_clock::now();
    uint64_t &ts = *L.tslots;
    if (table_full) {
        ts *= 4;
        P.table_full++;
    } else if (!L.fslots) {
        ts *= 2;
    }
    if (lane_full && L.fslots) *L.fslots *= 2;
    bool grew = false;
    ensure(c, *L.T, ts, &grew);
    fill_u64(c, L.T->p, grew ? L.T->cap : ts, kEmpty64);
    ensure_lane(c, L.id, L.fslots ? *L.fslots : std::max<uint64_t>(ts, (uint64_t)P.n), c->bag_lam_log2[L.id]);
    reset_bag(c, L.id);
    reset_lane_ctl(c, L.id);
    Search S = make_search(c, L.id, *P.o, L.mode);
    S.off = L.S.off;
    S.adj = L.S.adj;
    S.label = L.S.label;
    S.srclab = L.S.srclab;
    S.first = L.S.first;
    S.rec = L.S.rec;
    S.dirty = L.S.dirty;
    S.table = L.T->p;
    S.tmask = ts - 1;
    L.S = S;
    // the abandoned attempt's first-source claims go too
    if (S.first) fill_u32(c, (uint32_t *)S.first, (uint64_t)P.n, 0xffffffffu);
    if (S.rec) {
        hipLaunchKernelGGL(k_clear_rec_slots, dim3(grid_for(c, (uint64_t)P.n)), dim3(kBlock), 0, c->stream,
                           (int32_t)P.n, S.rec);
        LAUNCHCHK("k_clear_rec_slots");
    }
    SeedArgs A;
    memset(&A, 0, sizeof A);
    A.dirty = S.dirty;
    A.first[0] = S.rec ? reinterpret_cast<int32_t *>(S.rec) + 3 : S.first;
    A.fstride[0] = S.rec ? 4 : 1;
    A.T[0] = S.table;
    A.mask[0] = S.tmask;
    A.F[0] = S.F;
    A.rc[0] = S.rc;
    A.ls[0] = S.ls;
    hipLaunchKernelGGL(k_seed_multi, dim3(grid_for(c, (uint64_t)P.n), 1), dim3(kBlock), 0, c->stream, c->srcvert.p,
                       &c->dctl->sh, A, kProbeLimit);
    LAUNCHCHK("k_seed_multi");
    L.par = 0;
    L.nf = 1;
    if (P.st) P.st->table_restarts++;
    if (P.resize_ms) *P.resize_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// Clears what an abandoned multi-source search left behind: its reach table,
// its first-source slots, its bag and its round state.
void abandon_multi(scc_ctx *c, Lane &L, int64_t n) {
    fill_u64(c, L.T->p, *L.tslots, kEmpty64);
    if (L.S.first) fill_u32(c, (uint32_t *)L.S.first, (uint64_t)n, 0xffffffffu);
    if (L.S.rec) {
        hipLaunchKernelGGL(k_clear_rec_slots, dim3(grid_for(c, (uint64_t)n)), dim3(kBlock), 0, c->stream, (int32_t)n,
                           L.S.rec);
        LAUNCHCHK("k_clear_rec_slots");
    }
    reset_bag(c, L.id);
    reset_lane_ctl(c, L.id);
}

// Runs seeded lanes until every frontier is empty.
//
// Single-source lanes switch between sparse and dense rounds (Section 4.2)
// by Beamer's rule: dense once the frontier's arcs exceed m / 28, sparse again
// once the frontier has fewer than nsub / 24 vertices (options.dense forces
// either mode).  A lane near the switch is checked every round; otherwise
// rounds go in blocks of K (doubling up to 64) between checks.  Each round
// expands entries claimed in the previous round, so a search has at most
// (claimable entries + 1) rounds; the launch count guards the loop.
void drive(scc_ctx *c, Lane *lanes, int nl, DriveParams &P) {
    const scc_options_t &o = *P.o;
    const int dense_opt = o.dense;
    const bool use_policy = o.policy == 1 && c->policy.loaded;
    for (int i = 0; i < nl; i++) {
        Lane &L = lanes[i];
        L.live = true;
        L.par = 0;
        L.nf = 1;
        L.growth = 64.0;
        L.dense = dense_opt == 1 && L.mode == kSingle;
        L.have_list = true;
        L.fdeg = L.claims = 0;
        L.rounds = 0;
        L.nsub = std::max<int64_t>(P.nsub, 1);
        L.avg_deg = P.n > 0 ? std::max(1.0, (double)P.m / (double)P.n) : 1.0;
        L.policy_primed = false;
    }
    // direction-optimising switch (single-source searches): dense once the
    // frontier's arcs exceed m / 28 (a pull round is a coalesced pass, so the
    // switch comes earlier than the CPU rule's m / 14), sparse again below
    // |V'| / 24 frontier vertices
    const uint64_t arcs_on = (uint64_t)std::max<int64_t>(P.m / 28, 1);
    const int64_t back_off = std::max<int64_t>(P.nsub / 24, 1);
    // rounds between host checks: they double while nothing needs watching.
    // Multi-source searches start at 2, which saves a check on the many
    // two-round searches of low-diameter graphs (a spare round on an empty
    // frontier is a few microseconds of empty launches); single-source
    // searches start at 1 so that the dense switch is seen in time.
    bool all_multi = true;
    for (int i = 0; i < nl; i++) all_multi = all_multi && lanes[i].mode != kSingle;
    int K = all_multi ? 2 : 1;
    uint64_t launched = 0;
    uint64_t limit = (uint64_t)P.n + 64;
    for (int i = 0; i < nl; i++)
        if (lanes[i].mode != kSingle) limit = std::max<uint64_t>(limit, (uint64_t)P.n + 2 * *lanes[i].tslots + 64);
    bool was_dense[2] = {false, false};
    for (;;) {
        bool any = false, watch = false;
        for (int i = 0; i < nl; i++) {
            const Lane &L = lanes[i];
            if (!L.live) continue;
            any = true;
            // watch a lane whose frontier may reach the switch soon: fast
            // growing frontiers are projected a few rounds ahead
            const double proj = L.growth >= 2.0 ? std::pow(L.growth, (double)std::min(K, 3)) : 1.0;
            if (L.mode == kSingle && dense_opt != 0 && (L.dense || (double)L.nf * proj * 16.0 > (double)back_off))
                watch = true;
        }
        if (!any) break;
        const int k = (watch || c->tracing) ? 1 : K;
        bool graphed = false;
        if (c->graph_rounds && !c->tracing && !c->timing && !use_policy && k >= 2) {
            // a block of plain sparse rounds (no pull round, no host-side
            // policy step) runs as one captured graph
            Lane *gl[2];
            int ng = 0;
            bool ok = true;
            for (int i = 0; i < nl; i++) {
                if (!lanes[i].live) continue;
                if (lanes[i].dense) ok = false;
                gl[ng++] = &lanes[i];
            }
            if (ok && ng > 0 && !(ng == 2 && gl[0]->mode != gl[1]->mode)) {
                run_graph_block(c, gl, ng, k);
                graphed = true;
            }
        }
        for (int r = 0; r < (graphed ? 0 : k); r++) {
            // sparse lanes of this round share their launches (traced rounds
            // are timed per lane, so they launch alone)
            Lane *sp[2];
            int nsp = 0;
            for (int i = 0; i < nl; i++) {
                Lane &L = lanes[i];
                if (!L.live) continue;
                if (c->tracing) {
                    hipLaunchKernelGGL(k_trace_snap, dim3(1), dim3(64), 0, c->stream, L.S.rc, L.par);
                    LAUNCHCHK("k_trace_snap");
                    if (!L.dense) {
                        Lane *one = &L;
                        launch_policy(c, &one, 1, o);
                    }
                }
                if (c->tracing) HIPCHK(hipEventRecord(c->rev[L.id][0], c->stream));
                was_dense[L.id] = L.dense;
                if (L.dense) {
                    launch_dense(c, L);
                    c->dense_rounds++;
                    if (use_policy && !c->tracing) {
                        // a pull round has no ExtractAll: the policy runs in a
                        // launch of its own for the next round's mode
                        L.policy_primed = false;
                        Lane *one = &L;
                        launch_policy(c, &one, 1, o);
                    }
                } else if (c->tracing) {
                    Lane *one = &L;
                    launch_sparse(c, &one, 1);
                } else {
                    sp[nsp++] = &L;
                }
                if (c->tracing) HIPCHK(hipEventRecord(c->rev[L.id][1], c->stream));
            }
            launch_policy(c, sp, nsp, o);
            if (nsp == 2 && sp[0]->mode != sp[1]->mode) {
                launch_sparse(c, &sp[0], 1);
                launch_sparse(c, &sp[1], 1);
            } else if (nsp) {
                launch_sparse(c, sp, nsp);
            }
        }
        launched += (uint64_t)k;
        sync_ctl(c);
        timed_collect(c);
        bool switched = false;
        for (int i = 0; i < nl; i++) {
            Lane &L = lanes[i];
            if (!L.live) continue;
            const RoundCtl &rc = c->hctl->lane[L.id];
            const bool lane_full = (rc.err & kErrCapacity) || c->hctl->bag[L.id].overflow;
            if (lane_full && L.mode == kSingle) {
                // a single-source frontier holds each vertex at most once
                set_err(c, "frontier capacity exceeded (err=%u, bag overflow=%u)", rc.err, c->hctl->bag[L.id].overflow);
                throw Fail{SCC_EINTERNAL};
            }
            const uint64_t nf_new = (uint64_t)rc.nF[0] + rc.nF[1];
            if (c->tracing && rc.rounds > L.rounds) {
                float x[kPolicyIn];
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, c->rev[L.id][0], c->rev[L.id][1]));
                hipscc::policy_features_host((float)rc.snap_nf, (float)rc.snap_fdeg, (float)rc.snap_claims,
                                             (float)L.nsub, (float)rc.snap_rounds, (float)rc.snap_depth, x);
                const float tau = (float)(use_policy ? rc.tau_cur : (uint32_t)std::max(L.S.tau, 0));
                const float row[SCC_TRACE_FIELDS] = {
                    (float)(L.mode != kSingle ? 2 : (was_dense[L.id] ? 1 : 0)), x[0], x[1], x[2], x[3], x[4], tau, ms,
                    (float)(rc.claims - rc.snap_claims), (float)nf_new, (float)c->epoch, (float)P.n};
                c->trace.insert(c->trace.end(), row, row + SCC_TRACE_FIELDS);
            }
            // a multi-source search whose reach table or frontier buffers ran
            // out restarts with the one that ran out larger, or stops the
            // whole batch when its caller would rather shrink it
            if (L.mode != kSingle && ((rc.err & kErrTable) || lane_full)) {
                if (P.st) {
                    P.st->rounds_multi += rc.rounds;  // rounds of the abandoned attempt
                    P.st->restart_rounds += rc.rounds;
                }
                if (P.abandon_on_overflow) {
                    P.abandoned = true;
                    if (P.st) P.st->table_restarts++;
                    break;
                }
                restart_multi(c, L, P, (rc.err & kErrTable) != 0, lane_full);
                L.fdeg = L.claims = 0;
                L.rounds = 0;
                L.policy_primed = false;
                continue;
            }
            L.fdeg = rc.fdeg[rc.nF[0] ? 0 : 1];
            P.peak_fdeg = std::max<uint64_t>(P.peak_fdeg, L.fdeg);
            L.claims = rc.claims;
            if (L.nf > 0 && nf_new > 0)
                L.growth = std::pow((double)nf_new / (double)L.nf, 1.0 / (double)(L.dense ? 1 : k));
            L.nf = nf_new;
            L.rounds = rc.rounds;
            if (L.nf == 0) {
                L.live = false;
                continue;
            }
            L.par = rc.nF[0] ? 0 : 1;
            if (L.mode != kSingle || dense_opt == 0) continue;
            bool to_dense, to_sparse;
            if (o.policy == 2 && dense_opt == -1 && c->tracing) {
                // exploration: a coin decides the mode once the frontier is not tiny
                c->explore_state = mix64(c->explore_state + 0x632BE59BD9B4E019ull);
                const bool want_dense = (int64_t)L.nf * 256 > L.nsub && (c->explore_state >> 63);
                to_dense = !L.dense && want_dense;
                to_sparse = L.dense && !want_dense;
            } else if (use_policy && dense_opt == -1 && !c->tracing) {
                // the policy's mode for the next round (Section 4.2 dense
                // mode): 1 lets the direction rule switch to pull rounds,
                // 0 keeps (or brings) the search sparse
                const bool allow = rc.mode_pref == 1;
                to_dense = !L.dense && allow && L.fdeg > arcs_on;
                to_sparse = L.dense && (!allow || (int64_t)L.nf < back_off);
            } else {
                to_dense = !L.dense && (dense_opt == 1 || L.fdeg > arcs_on);
                to_sparse = L.dense && dense_opt == -1 && (int64_t)L.nf < back_off;
            }
            if (to_dense) {
                L.dense = true;
                L.have_list = true;
                switched = true;
            } else if (to_sparse) {
                // back to sparse: the bitmap frontier becomes the list F
                fill_u32(c, &L.S.rc->listpos, 1, 0u);
                hipLaunchKernelGGL(k_bitmap_to_list, dim3((unsigned)c->num_cu * 4), dim3(kBlock), 0, c->stream, L.n,
                                   c->bm[L.id][0].p, L.S.F, L.S.fcap, L.S.rc);
                LAUNCHCHK("k_bitmap_to_list");
                L.dense = false;
                L.have_list = true;
                L.policy_primed = false;
                switched = true;
            }
        }
        if (P.abandoned) {
            for (int i = 0; i < nl; i++) lanes[i].live = false;
            break;
        }
        if (launched > limit) {
            set_err(c, "internal: search did not finish after %llu rounds", (unsigned long long)launched);
            throw Fail{SCC_EINTERNAL};
        }
        K = switched || watch ? 1 : std::min(K * 2, kMaxSlots);
    }
    if (P.st) {
        for (int i = 0; i < nl; i++) {
            P.st->policy_calls += c->hctl->lane[lanes[i].id].policy_calls;
            P.st->policy_fallbacks += c->hctl->lane[lanes[i].id].policy_fallbacks;
        }
        if (o.policy == 1 && !c->policy.loaded) P.st->policy_fallbacks += (int64_t)launched;
    }
}

// ------------------------------------------------------------------ graph --
struct GraphDev {
    int32_t n, m;
    const int32_t *out_off, *out_adj, *in_off, *in_adj;
};

// O(n + m) checks: offsets start at 0, end at m, never decrease; targets in
// range; the transposed CSR has the in-degree histogram of the out-arcs.
__global__ void k_validate_off(int32_t n, int32_t m, const int32_t *off, uint32_t *bad) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v <= n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t o = off[v];
        if (v == 0 && o != 0) atomicOr(bad, 1u);
        if (v == n && o != m) atomicOr(bad, 1u);
        if (v < n && off[v + 1] < o) atomicOr(bad, 1u);
    }
}
__global__ void k_validate_adj(int32_t n, int32_t m, const int32_t *adj, int32_t *hist, uint32_t *bad) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t w = adj[e];
        if (w < 0 || w >= n) atomicOr(bad, 2u);
        else if (hist) atomicAdd(&hist[w], 1);
    }
}
__global__ void k_validate_hist(int32_t n, const int32_t *in_off, const int32_t *hist, uint32_t *bad) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        if (in_off[v + 1] - in_off[v] != hist[v]) atomicOr(bad, 4u);
}

void validate_graph(scc_ctx *c, const GraphDev &g) {
    uint32_t *bad = &c->dctl->sh.bad;
    fill_u32(c, bad, 1, 0u);
    hipLaunchKernelGGL(k_validate_off, dim3(grid_for(c, (uint64_t)g.n + 1)), dim3(kBlock), 0, c->stream, g.n, g.m,
                       g.out_off, bad);
    hipLaunchKernelGGL(k_validate_off, dim3(grid_for(c, (uint64_t)g.n + 1)), dim3(kBlock), 0, c->stream, g.n, g.m,
                       g.in_off, bad);
    LAUNCHCHK("k_validate_off");
    sync_ctl(c);
    if (c->hctl->sh.bad) {
        set_err(c, "invalid CSR offsets (must start at 0, end at m, never decrease)");
        throw Fail{SCC_EGRAPH};
    }
    fill_u32(c, (uint32_t *)c->aux.p, (uint64_t)g.n, 0u);
    hipLaunchKernelGGL(k_validate_adj, dim3(grid_for(c, (uint64_t)g.m)), dim3(kBlock), 0, c->stream, g.n, g.m,
                       g.out_adj, c->aux.p, bad);
    hipLaunchKernelGGL(k_validate_adj, dim3(grid_for(c, (uint64_t)g.m)), dim3(kBlock), 0, c->stream, g.n, g.m,
                       g.in_adj, (int32_t *)nullptr, bad);
    LAUNCHCHK("k_validate_adj");
    sync_ctl(c);
    if (c->hctl->sh.bad) {
        set_err(c, "arc target out of range [0, n)");
        throw Fail{SCC_EGRAPH};
    }
    hipLaunchKernelGGL(k_validate_hist, dim3(grid_for(c, (uint64_t)g.n)), dim3(kBlock), 0, c->stream, g.n, g.in_off,
                       c->aux.p, bad);
    LAUNCHCHK("k_validate_hist");
    sync_ctl(c);
    if (c->hctl->sh.bad) {
        set_err(c, "in-CSR is not the transpose of the out-CSR (in-degree mismatch)");
        throw Fail{SCC_EGRAPH};
    }
}

// ------------------------------------------------------------ call setup --
void init_call(scc_ctx *c, scc_stats_t *st, int64_t n, int64_t m, const scc_options_t *o = nullptr) {
    HIPCHK(hipSetDevice(c->device));
    c->err.clear();
    c->timing = o ? (uint32_t)o->timing : 0u;
    c->graph_rounds = o && o->graph_rounds == 1 && !c->noalloc;
    c->arcs_per_lane = (o && o->arcs_per_lane > 0) ? o->arcs_per_lane : 1;
    c->vgc_fill = (o && o->vgc_fill != 0.f) ? (double)o->vgc_fill : 2.0;
    if (c->timing && !c->tev[0][0])
        for (auto &a : c->tev)
            for (auto &e : a) HIPCHK(hipEventCreate(&e));
    c->tev_n = 0;
    for (int i = 0; i < SCC_KERNELS; i++) {
        c->tm_ms[i] = 0;
        c->tm_launches[i] = 0;
    }
    c->dense_rounds = 0;
    c->tracing = o && o->trace;
    c->trace.clear();
    c->epoch = 0;
    c->explore_state = o ? o->seed * 0x2545F4914F6CDD1Dull + 7 : 7;
    if (c->tracing && !c->rev[0][0])
        for (auto &a : c->rev)
            for (auto &e : a) HIPCHK(hipEventCreate(&e));
    c->plog.clear();
    c->pev_used = 0;
    if (st) {
        memset(st, 0, sizeof *st);
        st->n = n;
        st->m = m;
    }
    reset_ctl(c);
    if (c->tables_dirty) {
        if (c->Tout.p) fill_u64(c, c->Tout.p, c->Tout.cap, kEmpty64);
        if (c->Tin.p) fill_u64(c, c->Tin.p, c->Tin.cap, kEmpty64);
        c->tables_dirty = false;
    }
}

void check_graph_args(scc_ctx *c, const scc_graph_t *g) {
    if (!g) { set_err(c, "graph is NULL"); throw Fail{SCC_EINVAL}; }
    if (g->n < 0 || g->m < 0) { set_err(c, "negative n or m"); throw Fail{SCC_EINVAL}; }
    if (!g->out_off || !g->in_off || (g->m > 0 && (!g->out_adj || !g->in_adj))) {
        set_err(c, "graph has a NULL array");
        throw Fail{SCC_EINVAL};
    }
}

// Per-vertex device state sized for n vertices.
void ensure_vertex_state(scc_ctx *c, int64_t n) {
    bool g[4] = {false, false, false, false};
    ensure(c, c->label, (uint64_t)n);
    ensure(c, c->aux, (uint64_t)n);
    ensure(c, c->stamp, (uint64_t)n, &g[0]);
    ensure(c, c->fin, (uint64_t)n, &g[1]);
    ensure(c, c->srcvert, (uint64_t)n);
    ensure(c, c->srclab, (uint64_t)n);
    ensure(c, c->sig_out, (uint64_t)n, &g[2]);
    ensure(c, c->sig_in, (uint64_t)n, &g[3]);
    if (g[0] || g[1] || g[2] || g[3]) c->vclean_n = 0;  // new memory holds anything
    for (int i = 0; i < 2; i++) {
        ensure(c, c->vis[i], (uint64_t)n / 32 + 2);
        ensure(c, c->bm[i][0], (uint64_t)n / 32 + 2);
        ensure(c, c->bm[i][1], (uint64_t)n / 32 + 2);
    }
}

unsigned long long ctr_kind(const Counters &cn, int kind, int i) {
    unsigned long long t = 0;
    for (int s = 0; s < kCtrStripes; s++) t += cn.c[s][kind][i];
    return t;
}

// Fills the work counters, per-kernel timing and algorithmic bytes (see
// hipscc.h for the per-event byte counts).  Needs a sync with counters.
void fill_counters(scc_ctx *c, scc_stats_t *st, int64_t n) {
    if (!st) return;
    const Counters &cn = c->hctl->cn;
    auto sum = [&](int i) {
        unsigned long long t = 0;
        for (int k = 0; k < kNumKinds; k++) t += ctr_kind(cn, k, i);
        return (int64_t)t;
    };
    st->entries_expanded = sum(kCtrExpanded);
    st->arcs_scanned = sum(kCtrArcs);
    st->claim_attempts = sum(kCtrAttempts);
    st->claims = sum(kCtrClaims);
    st->bag_inserts = sum(kCtrInserts);
    for (int k = 0; k < SCC_KERNELS; k++) {
        st->ms_kernel[k] = c->tm_ms[k];
        st->launches_kernel[k] = c->tm_launches[k];
    }
    // multi-source: every scanned arc reads its target and the target's
    // label, every claim attempt probes 8 bytes and a claim writes 8;
    // single-source: the visited bitmap word stands in for label and probe
    auto search_bytes = [&](int k, bool multi) {
        return (int64_t)(ctr_kind(cn, k, kCtrSeeds) * 8 + ctr_kind(cn, k, kCtrExpanded) * 8 +
                         ctr_kind(cn, k, kCtrArcs) * (multi ? 8 : 4) + ctr_kind(cn, k, kCtrAttempts) * (multi ? 8 : 4) +
                         ctr_kind(cn, k, kCtrClaims) * (multi ? 8 : 4) + ctr_kind(cn, k, kCtrInserts) * 8);
    };
    st->bytes_kernel[SCC_KERNEL_EXPAND_SINGLE] = search_bytes(kKindExpandSingle, false);
    st->bytes_kernel[SCC_KERNEL_EXPAND_MULTI] = search_bytes(kKindExpandMulti, true);
    st->bytes_kernel[SCC_KERNEL_HEAVY_SINGLE] = search_bytes(kKindHeavySingle, false);
    st->bytes_kernel[SCC_KERNEL_HEAVY_MULTI] = search_bytes(kKindHeavyMulti, true);
    // every sparse-round insert is extracted once
    st->bytes_kernel[SCC_KERNEL_EXTRACT] =
        (int64_t)(ctr_kind(cn, kKindExpandSingle, kCtrInserts) + ctr_kind(cn, kKindExpandMulti, kCtrInserts) +
                  ctr_kind(cn, kKindHeavySingle, kCtrInserts) + ctr_kind(cn, kKindHeavyMulti, kCtrInserts)) * 24;
    st->bytes_kernel[SCC_KERNEL_UNION] = (int64_t)(ctr_kind(cn, kKindUnion, kCtrArcs) * 8 +
                                                   ctr_kind(cn, kKindUnion, kCtrAttempts) * 16) +
                                         (ctr_kind(cn, kKindUnion, kCtrArcs) ? 12 * n : 0);
    st->bytes_kernel[2] = (int64_t)(ctr_kind(cn, kKindPull, kCtrExpanded) * 8 + ctr_kind(cn, kKindPull, kCtrArcs) * 8) +
                          c->dense_rounds * (n / 4);
    // whole call: searches (expand, edge-parallel, pull), bag traffic
    // (insert + ExtractAll read + frontier write + frontier read = 32 B per
    // inserted entry), trimming (12 n) and canonical labels (16 n)
    st->bytes_alg = st->entries_expanded * 8 + st->arcs_scanned * 4 + st->claim_attempts * 4 + st->claims * 8 +
                    st->bag_inserts * 32 + 28 * n;
}

// ------------------------------------------------------------------ SCC --
void run_scc(scc_ctx *c, const GraphDev &g, int32_t *labels_out, const scc_options_t &o, scc_stats_t *st) {
    const int32_t n = g.n;
    if (n == 0) return;
    const bool ph = st != nullptr && !c->noalloc;  // phase events are created on first use
    ensure_vertex_state(c, n);
    if (o.validate) validate_graph(c, g);
    // per-call state: the relabel accumulators and stamps are cleared only
    // when the previous call did not leave them clean on [0, n)
    phase_begin(c, 4, ph);
    int64_t clean_after = std::max<int64_t>(c->vclean_n, n);
    if (c->vclean_n < n || c->stamp_next > (1 << 30)) {
        fill_u32(c, (uint32_t *)c->stamp.p, (uint64_t)n, 0u);
        fill_u32(c, (uint32_t *)c->fin.p, (uint64_t)n, (uint32_t)kInf32);
        fill_u64(c, (uint64_t *)c->sig_out.p, (uint64_t)n, 0ull);
        fill_u64(c, (uint64_t *)c->sig_in.p, (uint64_t)n, 0ull);
        c->stamp_next = 1;
        clean_after = n;
    }
    c->vclean_n = 0;  // until this call ends normally
    for (int i = 0; i < 2; i++) {
        ensure_lane(c, i, (uint64_t)n, lam_log2_for(o, (uint64_t)n));
        reset_bag(c, i);
    }
    // first-source slots: empty unless the previous call left them so
    const bool use_first = o.first_slot == 1;
    int64_t first_clean_after = c->first_clean_n;
    if (use_first) {
        for (int d = 0; d < 2; d++) {
            bool grew = false;
            ensure(c, c->firstS[d], (uint64_t)n, &grew);
            if (grew) c->first_clean_n = 0;
        }
        if (c->first_clean_n < n) {
            for (int d = 0; d < 2; d++) fill_u32(c, (uint32_t *)c->firstS[d].p, (uint64_t)n, 0xffffffffu);
            first_clean_after = n;
        }
        c->first_clean_n = 0;  // until this call ends normally
    }
    phase_end(c, ph);

    // ---- trimming (Section 4.1) and the random permutation (Algorithm 1)
    phase_begin(c, 0, ph);
    Shared *sh = &c->dctl->sh;
    hipLaunchKernelGGL(k_trim, dim3(grid_for(c, (uint64_t)n)), dim3(kBlock), 0, c->stream, n, g.out_off, g.in_off,
                       c->label.p, o.trim ? 1 : 0, c->vis[0].p, c->vis[1].p, &c->dctl->cs, sh);
    LAUNCHCHK("k_trim");
    Perm P;
    P.n = (uint32_t)n;
    uint32_t bits = 1;
    while ((1ull << (2 * bits)) < (uint64_t)n) bits++;
    P.half_bits = bits;
    P.key = mix64(o.seed ^ 0x243F6A8885A308D3ull);
    // batch 1 is the first active vertex in permutation order: look at a
    // short prefix first; the scan of the rest returns at once if it found one
    fill_u32(c, &sh->first, 1, 0xffffffffu);
    const uint32_t pre = (uint32_t)std::min<int64_t>(n, 65536);
    hipLaunchKernelGGL(k_first_active, dim3(grid_for(c, pre)), dim3(kBlock), 0, c->stream, P, 0u, pre, c->label.p, sh);
    LAUNCHCHK("k_first_active");
    if (pre < (uint32_t)n) {
        hipLaunchKernelGGL(k_first_active, dim3(grid_for(c, (uint64_t)n)), dim3(kBlock), 0, c->stream, P, pre,
                           (uint32_t)n, c->label.p, sh);
        LAUNCHCHK("k_first_active");
    }
    phase_end(c, ph);

    // ---- first SCC: forward and backward single-source searches (4.2), as
    // two lanes.  The source is read on the device.
    phase_begin(c, 1, ph);
    Lane L[2];
    for (int d = 0; d < 2; d++) {
        // the visited bitmaps were pre-set by the trimming pass
        hipLaunchKernelGGL(k_seed_single, dim3(1), dim3(64), 0, c->stream, -1, sh, P, c->F[d].p, &c->dctl->lane[d],
                           &c->dctl->ls[d], c->vis[d].p);
        LAUNCHCHK("k_seed_single");
        L[d].id = d;
        L[d].mode = kSingle;
        L[d].n = n;
        L[d].S = make_search(c, d, o, kSingle);
        L[d].S.off = d ? g.in_off : g.out_off;
        L[d].S.adj = d ? g.in_adj : g.out_adj;
        L[d].S.label = c->label.p;
        L[d].S.vis = c->vis[d].p;
        L[d].roff = d ? g.out_off : g.in_off;
        L[d].radj = d ? g.out_adj : g.in_adj;
    }
    DriveParams DP;
    DP.o = &o;
    DP.n = n;
    DP.m = g.m;
    DP.nsub = n;
    DP.st = st;
    double resize_ms = 0;
    DP.resize_ms = &resize_ms;
    drive(c, L, 2, DP);
    if (st) st->rounds_first = L[0].rounds + L[1].rounds;
    phase_end(c, ph);
    const uint32_t j1 = c->hctl->sh.first;
    const int64_t trimmed = count_sum(c, &CountLine::trimmed);
    phase_begin(c, 4, ph);
    hipLaunchKernelGGL(k_finish_single, dim3(grid_for(c, (uint64_t)n)), dim3(kBlock), 0, c->stream, n, c->label.p, 0,
                       sh, P, c->vis[0].p, c->vis[1].p, &c->dctl->cs);
    LAUNCHCHK("k_finish_single");
    phase_end(c, ph);
    if (st && j1 < (uint32_t)n) st->batches = 1;
    // packed records for the multi-source batches (first-source slots on):
    // worth their build pass (32 bytes per vertex written) when most
    // vertices survived trimming; not in the allocation-free path
    const bool use_rec = use_first && !c->noalloc &&
                         (o.packed == 1 || (o.packed == -1 && 2 * ((int64_t)n - trimmed) > (int64_t)n));
    if (use_rec) {
        phase_begin(c, 4, ph);
        ensure(c, c->rec[0], (uint64_t)n);
        ensure(c, c->rec[1], (uint64_t)n);
        hipLaunchKernelGGL(k_build_rec, dim3(grid_for(c, (uint64_t)n)), dim3(kBlock), 0, c->stream, n, g.out_off,
                           g.in_off, c->label.p, c->rec[0].p, c->rec[1].p);
        LAUNCHCHK("k_build_rec");
        phase_end(c, ph);
    }

    // granule flags of claimed first-source slots (all clear between batches)
    uint8_t *dirty = nullptr;
    if (use_first && !c->noalloc) {
        bool grew = false;
        const uint64_t ng = (((uint64_t)n + (1u << kDirtyLog2) - 1) >> kDirtyLog2) + 4;
        ensure(c, c->dirty, ng, &grew);
        if (grew) fill_u32(c, reinterpret_cast<uint32_t *>(c->dirty.p), c->dirty.cap / 4, 0u);
        dirty = c->dirty.p;
    }

    // ---- multi-source batches (Algorithm 1, prefix doubling with beta).  The
    // host's view of |V'| lags one batch behind (it is read at the next
    // check); it is only used as an upper bound.
    uint64_t pos = j1 < (uint32_t)n ? (uint64_t)j1 + 1 : (uint64_t)n;
    double bsize = 1.0, prev_bsize = 1.0;
    bool fast_next = false, short_next = false;
    const uint64_t lanes_all = (uint64_t)c->expand_grid[kMulti][0] * kBlock;
    int32_t epoch = 1;
    int32_t stamp_ep = c->stamp_next;  // owner-election stamp of the current batch
    bool invp_built = false;  // the inverse permutation of this call's P is stored
    uint64_t a_out = 0, a_in = 0, ts_out = 0, ts_in = 0, at_out = 0, at_in = 0, fs[2] = {0, 0};
    double floor_boost = 1.0;
    int64_t active = (int64_t)n - trimmed;  // upper bound
    while (active > 0 && pos < (uint64_t)n) {
        // Batches grow by beta (Algorithm 1), or by beta_fast after a batch
        // whose frontiers never filled the GPU's lanes: its rounds were
        // latency bound, so a larger batch costs few extra rounds' time.  A
        // batch whose searches ended within a few rounds and whose sources
        // reached few vertices each cost little more than its fixed launches
        // and checks, so the next one grows by kShortGrowth.
        const double g_fast = short_next ? std::max((double)o.beta_fast, kShortGrowth) : (double)o.beta_fast;
        const bool grew_fast = g_fast > o.beta && fast_next;
        const double bsize0 = bsize, prev_bsize0 = prev_bsize;
        const uint64_t pos0 = pos;
        bsize *= grew_fast ? g_fast : (double)o.beta;
        const uint64_t sz = std::max<uint64_t>((uint64_t)std::ceil(bsize - 1e-9), 1);
        const uint64_t p1 = std::min<uint64_t>((uint64_t)n, pos + sz);
        const uint64_t kmax = std::min<uint64_t>(p1 - pos, (uint64_t)active);
        phase_begin(c, 2, ph);
        hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(kBlock), 0, c->stream, sh, &c->dctl->lane[0], &c->dctl->lane[1]);
        LAUNCHCHK("k_batch_reset");
        if ((p1 - pos) * 16 > (uint64_t)n) {
            const bool build = !invp_built;
            if (build) ensure(c, c->invp, (uint64_t)n);
            hipLaunchKernelGGL(k_select_scan, dim3(grid_for(c, ((uint64_t)n + kScanPer - 1) / kScanPer)), dim3(kBlock),
                               0, c->stream, P,
                               (uint32_t)pos, (uint32_t)p1, n, c->label.p, c->srcvert.p, c->srclab.p, sh, c->invp.p,
                               build);
            LAUNCHCHK("k_select_scan");
            invp_built = true;
        } else {
            hipLaunchKernelGGL(k_select_sources, dim3(grid_for(c, (p1 - pos + kScanPer - 1) / kScanPer)), dim3(kBlock),
                               0, c->stream, P,
                               (uint32_t)pos, (uint32_t)p1, c->label.p, c->srcvert.p, c->srclab.p, sh);
            LAUNCHCHK("k_select_sources");
        }
        pos = p1;
        // Section 4.5: next table size = nextpow2(max(0.3 b, 1.5 a)), b = |V'|,
        // a = pairs found by the previous search in the same direction.
        // (the pairs of the previous batch scale with the batch's growth)
        const double growth = bsize / std::max(prev_bsize, 1.0);
        prev_bsize = bsize;
        // The table stops at eight times the active vertices plus the
        // sources (and at a fixed share of device memory): a batch that finds
        // more pairs restarts on a larger table, instead of every batch
        // reserving tables (and the frontier bags sized from them) for the
        // worst case.
        // With first-source slots a vertex's first pair sits in its slot and
        // only the others go to the table.  A batch g times larger finds about
        // g times the pairs, on at least the vertices the previous batch
        // reached (a - at of them, at = its table pairs), so the table is
        // sized for (g - 1) a + at pairs, and the floor is half (the
        // vertices' first pairs need no room).  Each batch whose table filled
        // up doubles the floor of the call's later batches: one source
        // reaching much more than the earlier ones did shows that the
        // estimate is low for this graph.
        auto size_for = [&](uint64_t a, uint64_t at) {
            const double floor = (double)o.table_floor * (double)active * floor_boost / (use_first ? 2.0 : 1.0);
            const double pairs = use_first ? std::max(growth - 1.0, 0.0) * (double)a + (double)at
                                           : growth * (double)a;
            uint64_t want = (uint64_t)std::max(floor, 1.5 * pairs);
            want = std::min<uint64_t>(want, 8 * (uint64_t)std::max<int64_t>(active, 0) + 2 * kmax);
            want = std::max<uint64_t>(want, 2 * kmax);
            want = std::min<uint64_t>(want, c->table_slots_max);
            want = std::max<uint64_t>(want, 1024);
            if (o.table_init > 0 && epoch == 1) want = (uint64_t)o.table_init;
            return next_pow2(want);
        };
        auto t_rs = std::chrono::steady_clock::now();
        ts_out = size_for(a_out, at_out);
        ts_in = size_for(a_in, at_in);
        // frontier buffers for one round's pairs: sized from all the pairs
        // the batch is expected to find (a table with first-source slots
        // holds only some of them), at least n and at most 2n (a search that
        // needs more restarts with larger ones)
        for (int d = 0; d < 2; d++) {
            const double full = std::max((double)o.table_floor * (double)active,
                                         1.5 * growth * (double)(d ? a_in : a_out));
            const uint64_t want = use_first ? next_pow2((uint64_t)std::max(full, 1024.0)) : (d ? ts_in : ts_out);
            fs[d] = std::max<uint64_t>(std::min<uint64_t>(want, 2 * (uint64_t)n), (uint64_t)n);
        }
        bool grew = false;
        ensure(c, c->Tout, ts_out, &grew);
        if (grew) fill_u64(c, c->Tout.p, c->Tout.cap, kEmpty64);
        ensure(c, c->Tin, ts_in, &grew);
        if (grew) fill_u64(c, c->Tin.p, c->Tin.cap, kEmpty64);
        c->tables_dirty = true;
        for (int d = 0; d < 2; d++) ensure_lane(c, d, fs[d], c->bag_lam_log2[d]);
        resize_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_rs).count();
        SeedArgs SA;
        memset(&SA, 0, sizeof SA);
        for (int d = 0; d < 2; d++) {
            DevBuf<uint64_t> &T = d ? c->Tin : c->Tout;
            uint64_t &ts = d ? ts_in : ts_out;
            L[d] = Lane();
            L[d].id = d;
            L[d].mode = use_rec ? kMultiRec : (use_first ? kMultiFirst : kMulti);
            L[d].n = n;
            L[d].T = &T;
            L[d].tslots = &ts;
            L[d].fslots = &fs[d];
            L[d].S = make_search(c, d, o, L[d].mode);
            L[d].S.first = (use_first && !use_rec) ? c->firstS[d].p : nullptr;
            L[d].S.rec = use_rec ? c->rec[d].p : nullptr;
            L[d].S.dirty = dirty;
            SA.first[d] = use_rec ? reinterpret_cast<int32_t *>(c->rec[d].p) + 3 : L[d].S.first;
            SA.fstride[d] = use_rec ? 4 : 1;
            SA.dirty = dirty;
            L[d].S.off = d ? g.in_off : g.out_off;
            L[d].S.adj = d ? g.in_adj : g.out_adj;
            L[d].S.label = c->label.p;
            L[d].S.srclab = c->srclab.p;
            L[d].S.table = T.p;
            L[d].S.tmask = ts - 1;
            SA.T[d] = T.p;
            SA.mask[d] = ts - 1;
            SA.F[d] = c->F[d].p;
            SA.rc[d] = &c->dctl->lane[d];
            SA.ls[d] = &c->dctl->ls[d];
        }
        hipLaunchKernelGGL(k_seed_multi, dim3(grid_for(c, kmax), 2), dim3(kBlock), 0, c->stream, c->srcvert.p, sh, SA,
                           kProbeLimit);
        LAUNCHCHK("k_seed_multi");
        DP.nsub = active;
        DP.peak_fdeg = 0;
        DP.table_full = 0;
        DP.abandon_on_overflow = grew_fast;
        DP.abandoned = false;
        c->epoch = epoch;
        drive(c, L, 2, DP);
        if (DP.table_full) floor_boost = std::min(floor_boost * 2.0, 16.0);
        if (DP.abandoned) {
            // A batch that grew faster than beta (its predecessors were
            // cheap) found more pairs than its tables or frontiers hold: its
            // sources' reach is larger than the cheap batches suggested, and
            // pairs grow with the batch, so instead of restarting on larger
            // buffers the searches are dropped and the batch is taken again
            // from the same position at the size beta growth gives.
            for (int d = 0; d < 2; d++) abandon_multi(c, L[d], n);
            phase_end(c, ph);
            pos = pos0;
            bsize = bsize0;
            prev_bsize = prev_bsize0;
            fast_next = short_next = false;
            continue;
        }
        phase_end(c, ph);
        const uint32_t k = c->hctl->sh.k;
        a_out = c->hctl->lane[0].claims + k;
        a_in = c->hctl->lane[1].claims + k;
        // with first-source slots the tables hold only the later pairs of a
        // vertex: the next tables are sized from those
        at_out = c->hctl->lane[0].tclaims;
        at_in = c->hctl->lane[1].tclaims;
        if (st) st->claims_table += (int64_t)(at_out + at_in);
        // a cheap batch: its frontiers never used a sixteenth of the GPU's
        // lanes (its rounds were latency bound), or its sources reached few
        // vertices each and its frontiers never filled the GPU; the next
        // batch may grow faster
        fast_next = DP.peak_fdeg < lanes_all / 16 ||
                    (DP.peak_fdeg < lanes_all && k > 0 && (a_out + a_in) < (uint64_t)kCheapPairs * 2 * k);
        short_next = o.beta_fast > o.beta && std::max(L[0].rounds, L[1].rounds) <= kShortRounds &&
                     (a_out + a_in) < (uint64_t)kCheapPairs * 2 * std::max<uint64_t>(k, 1);
        active = (int64_t)n - trimmed - count_sum(c, &CountLine::fin);
        if (k == 0) continue;  // nothing was claimed; the tables are still clean
        if (st) {
            st->batches += 1;
            st->rounds_multi += L[0].rounds + L[1].rounds;
        }
        phase_begin(c, 4, ph);
        const uint64_t tot = ts_out + ts_in;
        // a batch with many pairs relabels per vertex (one coalesced pass),
        // a small one per table slot (random accesses to the touched vertices)
        // (first-source slots are read per vertex, so such batches always
        // take the per-vertex relabel)
        const bool dense_label = use_first || (a_out + a_in) * kDenseLabelDiv >= (uint64_t)n;
        int32_t *fF = nullptr, *fB = nullptr;
        const int32_t fstride = use_rec ? 4 : 1;
        if (use_rec) {
            fF = reinterpret_cast<int32_t *>(c->rec[0].p) + 3;
            fB = reinterpret_cast<int32_t *>(c->rec[1].p) + 3;
        } else if (use_first) {
            fF = c->firstS[0].p;
            fB = c->firstS[1].p;
        }
        hipLaunchKernelGGL(k_accumulate, dim3(grid_for(c, tot)), dim3(kBlock), 0, c->stream, c->Tout.p, ts_out - 1,
                           c->Tin.p, ts_in - 1, kProbeLimit, c->srcvert.p, c->sig_out.p, c->sig_in.p, c->fin.p,
                           dense_label, fF, fB, fstride);
        LAUNCHCHK("k_accumulate");
        if (dense_label) {
            hipLaunchKernelGGL(k_relabel_dense, dim3(grid_for(c, std::max<uint64_t>(ts_out, (uint64_t)n))), dim3(kBlock),
                               0, c->stream, n, c->Tout.p, ts_out - 1, c->srcvert.p, c->sig_out.p, c->sig_in.p,
                               c->fin.p, c->label.p, &c->dctl->cs, fF, fB, fstride, use_rec ? c->rec[0].p : nullptr,
                               use_rec ? c->rec[1].p : nullptr, dirty);
            LAUNCHCHK("k_relabel_dense");
        } else {
            hipLaunchKernelGGL(k_relabel_multi, dim3(grid_for(c, tot)), dim3(kBlock), 0, c->stream, c->Tout.p,
                               ts_out - 1, c->Tin.p, ts_in - 1, c->srcvert.p, c->sig_out.p, c->sig_in.p, c->fin.p,
                               c->stamp.p, stamp_ep, c->label.p, &c->dctl->cs);
            LAUNCHCHK("k_relabel_multi");
        }
        phase_end(c, ph);
        epoch++;
        stamp_ep++;
    }
    c->stamp_next = stamp_ep;
    // ---- canonical labels: min vertex id per SCC
    phase_begin(c, 4, ph);
    hipLaunchKernelGGL(k_iota, dim3(grid_for(c, (uint64_t)n)), dim3(kBlock), 0, c->stream, n, c->aux.p);
    LAUNCHCHK("k_iota");
    hipLaunchKernelGGL(k_canon_min, dim3(grid_for(c, (uint64_t)n, 4)), dim3(kBlock), 0, c->stream, n, c->label.p,
                       c->aux.p, &sh->bad);
    LAUNCHCHK("k_canon_min");
    hipLaunchKernelGGL(k_canon_write, dim3(grid_for(c, (uint64_t)n)), dim3(kBlock), 0, c->stream, n, c->label.p,
                       c->aux.p, labels_out, &c->dctl->cs);
    LAUNCHCHK("k_canon_write");
    phase_end(c, ph);
    sync_ctl(c, st != nullptr);
    const int64_t fin_all = count_sum(c, &CountLine::fin) + count_sum(c, &CountLine::trimmed);
    if ((c->hctl->sh.bad & kErrUnfinished) || fin_all != (int64_t)n) {
        set_err(c, "internal: %lld of %d vertices ended without an SCC key", (long long)((int64_t)n - fin_all), n);
        throw Fail{SCC_EINTERNAL};
    }
    if (st) {
        double ms[kPhases] = {0, 0, 0, 0, 0};
        phase_collect(c, ms);
        st->ms_trim += ms[0];
        st->ms_first += ms[1];
        st->ms_multi += ms[2];
        st->ms_resize += resize_ms;
        st->ms_label += ms[4];
        st->trimmed = count_sum(c, &CountLine::trimmed);
        st->n_scc = count_sum(c, &CountLine::nscc);
        st->dense_rounds = c->dense_rounds;
        fill_counters(c, st, n);
    }
    c->tables_dirty = false;
    c->vclean_n = clean_after;
    if (use_first) c->first_clean_n = first_clean_after;
}

// sources check for scc_reach: in range, label >= 0, distinct (stamp epoch)
__global__ void k_check_sources(int32_t n, int32_t k, const int32_t *sources, const int32_t *labels, int32_t *srcvert,
                                int32_t *srclab, int32_t *stamp, int32_t epoch, uint32_t *bad) {
    for (int32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < k; j += gridDim.x * blockDim.x) {
        const int32_t s = sources[j];
        if (s < 0 || s >= n) {
            atomicOr(bad, 1u);
            continue;
        }
        const int32_t l = labels[s];
        if (l < 0) atomicOr(bad, 2u);
        if (atomicExch(&stamp[s], epoch) == epoch) atomicOr(bad, 4u);
        srcvert[j] = s;
        srclab[j] = l;
    }
}

// Union CSR of a batch of graphs: global id = vtx_base[g] + local id.  The
// element range is cut into tiles of kUnionTile; one thread finds the graph
// of the tile's first element by binary search over the bases, and every
// thread then walks forward from it (a tile spans few graphs), so the pass
// streams the arrays instead of searching per element.
constexpr int64_t kUnionTile = 4096;

// The graph of element x among graphs [g0, g0 + G): the last one whose base
// (bases = vb or ab) is <= x.  One thread of the block; the result in LDS.
__device__ __forceinline__ int32_t tile_graph(const int64_t *bases, int32_t g0, int32_t G, int64_t x) {
    __shared__ int32_t gs;
    if (threadIdx.x == 0) {
        int32_t lo = g0, hi = g0 + G - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (bases[mid] <= x) lo = mid; else hi = mid - 1;
        }
        gs = lo;
    }
    __syncthreads();
    const int32_t g = gs;
    __syncthreads();  // gs is rewritten by the next tile
    return g;
}

__global__ void k_union_off(int32_t G, const int64_t *vb, const int64_t *ab, const int32_t *off_in, int32_t *off_out,
                            int64_t arc0, int32_t g0) {
    const int64_t v0 = vb[g0];
    const int64_t nv = vb[g0 + G] - v0;
    for (int64_t t0 = (int64_t)blockIdx.x * kUnionTile; t0 <= nv; t0 += (int64_t)gridDim.x * kUnionTile) {
        int32_t g = tile_graph(vb, g0, G, v0 + (t0 < nv ? t0 : nv - 1));
        const int64_t t1 = t0 + kUnionTile < nv + 1 ? t0 + kUnionTile : nv + 1;
        for (int64_t i = t0 + threadIdx.x; i < t1; i += blockDim.x) {
            if (i == nv) {
                off_out[i] = (int32_t)(ab[g0 + G] - arc0);
                continue;
            }
            const int64_t gv = v0 + i;
            while (vb[g + 1] <= gv) g++;
            off_out[i] = (int32_t)(ab[g] - arc0 + off_in[vb[g] + g + (gv - vb[g])]);
        }
    }
}
__global__ void k_union_adj(int32_t G, const int64_t *vb, const int64_t *ab, const int32_t *adj_in, int32_t *adj_out,
                            int32_t g0) {
    const int64_t a0 = ab[g0];
    const int64_t na = ab[g0 + G] - a0;
    for (int64_t t0 = (int64_t)blockIdx.x * kUnionTile; t0 < na; t0 += (int64_t)gridDim.x * kUnionTile) {
        int32_t g = tile_graph(ab, g0, G, a0 + t0);
        const int64_t t1 = t0 + kUnionTile < na ? t0 + kUnionTile : na;
        for (int64_t e = t0 + threadIdx.x; e < t1; e += blockDim.x) {
            const int64_t ge = a0 + e;
            while (ab[g + 1] <= ge) g++;
            adj_out[e] = (int32_t)(vb[g] - vb[g0] + adj_in[ge]);
        }
    }
}
__global__ void k_union_labels(int32_t G, const int64_t *vb, const int32_t *lab_in, int32_t *lab_out, int32_t g0) {
    const int64_t v0 = vb[g0];
    const int64_t nv = vb[g0 + G] - v0;
    for (int64_t t0 = (int64_t)blockIdx.x * kUnionTile; t0 < nv; t0 += (int64_t)gridDim.x * kUnionTile) {
        int32_t g = tile_graph(vb, g0, G, v0 + t0);
        const int64_t t1 = t0 + kUnionTile < nv ? t0 + kUnionTile : nv;
        for (int64_t i = t0 + threadIdx.x; i < t1; i += blockDim.x) {
            const int64_t gv = v0 + i;
            while (vb[g + 1] <= gv) g++;
            lab_out[gv] = (int32_t)(lab_in[i] + v0 - vb[g]);
        }
    }
}

template <typename Fn>
scc_status guard(scc_ctx *c, Fn &&fn) {
    if (!c) return SCC_EINVAL;
    try {
        fn();
        return SCC_OK;
    } catch (const Fail &f) {
        return f.code;
    } catch (const std::bad_alloc &) {
        set_err(c, "host allocation failed");
        return SCC_ENOMEM;
    } catch (...) {
        set_err(c, "unexpected exception");
        return SCC_EINTERNAL;
    }
}

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

void accumulate_stats(scc_stats_t &acc, const scc_stats_t &st) {
    acc.ms_trim += st.ms_trim;
    acc.ms_first += st.ms_first;
    acc.ms_multi += st.ms_multi;
    acc.ms_resize += st.ms_resize;
    acc.ms_label += st.ms_label;
    acc.batches += st.batches;
    acc.rounds_first += st.rounds_first;
    acc.rounds_multi += st.rounds_multi;
    acc.dense_rounds += st.dense_rounds;
    acc.entries_expanded += st.entries_expanded;
    acc.arcs_scanned += st.arcs_scanned;
    acc.claim_attempts += st.claim_attempts;
    acc.claims += st.claims;
    acc.claims_table += st.claims_table;
    acc.bag_inserts += st.bag_inserts;
    acc.bag_chunk_advances += st.bag_chunk_advances;
    acc.table_restarts += st.table_restarts;
    acc.restart_rounds += st.restart_rounds;
    acc.trimmed += st.trimmed;
    acc.n_scc += st.n_scc;
    acc.policy_calls += st.policy_calls;
    acc.policy_fallbacks += st.policy_fallbacks;
    acc.bytes_alg += st.bytes_alg;
    for (int k = 0; k < SCC_KERNELS; k++) {
        acc.ms_kernel[k] += st.ms_kernel[k];
        acc.launches_kernel[k] += st.launches_kernel[k];
        acc.bytes_kernel[k] += st.bytes_kernel[k];
    }
}

// ------------------------------------------------------ static scratch --
// scc_labels_static carves every per-call buffer of scc_labels from one fixed
// device array instead of allocating.  The array is file-scope device memory:
// each device the library runs on holds its own copy from module load until
// the process ends.  Host code must not pass the symbol itself to a kernel
// (on the host it only names the array); scc_create looks up this device's
// address with hipGetSymbolAddress and every use goes through that address.
constexpr uint64_t kStaticScratchBytes = 512ull << 20;
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch[kMaxDevices] = {};

// This device's address of the scratch array (looked up once per device,
// with the device current).
uint8_t *scratch_address(scc_ctx *c) {
    if (c->device < 0 || c->device >= kMaxDevices) {
        set_err(c, "device %d beyond the static scratch table", c->device);
        throw Fail{SCC_EINVAL};
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[c->device]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_err(c, "hipGetSymbolAddress returned no address for the static scratch");
            throw Fail{SCC_EHIP};
        }
        g_scratch[c->device] = (uint8_t *)p;
    }
    return g_scratch[c->device];
}

// Everything run_scc allocates or keeps between calls, swapped out while a
// static call runs on carved views.
struct BufSet {
    DevBuf<int32_t> label, aux, stamp, srcvert, srclab, fin;
    DevBuf<uint32_t> invp;
    DevBuf<unsigned long long> sig_out, sig_in;
    DevBuf<uint32_t> vis[2], bm[2][2];
    DevBuf<uint64_t> Tout, Tin, F[2], heavy[2], bag_slots[2];
    DevBuf<uint32_t> bag_cnt[2];
    DevBuf<int32_t> firstS[2];
    uint32_t bag_nchunks[2], bag_lam_log2[2];
    bool tables_dirty;
    int64_t vclean_n, first_clean_n;
    int32_t stamp_next;
    uint64_t table_slots_max;
};

void bufs_save(const scc_ctx *c, BufSet &b) {
    b.label = c->label; b.aux = c->aux; b.stamp = c->stamp; b.srcvert = c->srcvert; b.srclab = c->srclab;
    b.fin = c->fin; b.invp = c->invp; b.sig_out = c->sig_out; b.sig_in = c->sig_in;
    for (int i = 0; i < 2; i++) {
        b.vis[i] = c->vis[i]; b.bm[i][0] = c->bm[i][0]; b.bm[i][1] = c->bm[i][1];
        b.F[i] = c->F[i]; b.heavy[i] = c->heavy[i]; b.bag_slots[i] = c->bag_slots[i]; b.bag_cnt[i] = c->bag_cnt[i];
        b.bag_nchunks[i] = c->bag_nchunks[i]; b.bag_lam_log2[i] = c->bag_lam_log2[i];
        b.firstS[i] = c->firstS[i];
    }
    b.Tout = c->Tout; b.Tin = c->Tin;
    b.tables_dirty = c->tables_dirty; b.vclean_n = c->vclean_n; b.stamp_next = c->stamp_next;
    b.first_clean_n = c->first_clean_n;
    b.table_slots_max = c->table_slots_max;
}

void bufs_load(scc_ctx *c, const BufSet &b) {
    c->label = b.label; c->aux = b.aux; c->stamp = b.stamp; c->srcvert = b.srcvert; c->srclab = b.srclab;
    c->fin = b.fin; c->invp = b.invp; c->sig_out = b.sig_out; c->sig_in = b.sig_in;
    for (int i = 0; i < 2; i++) {
        c->vis[i] = b.vis[i]; c->bm[i][0] = b.bm[i][0]; c->bm[i][1] = b.bm[i][1];
        c->F[i] = b.F[i]; c->heavy[i] = b.heavy[i]; c->bag_slots[i] = b.bag_slots[i]; c->bag_cnt[i] = b.bag_cnt[i];
        c->bag_nchunks[i] = b.bag_nchunks[i]; c->bag_lam_log2[i] = b.bag_lam_log2[i];
        c->firstS[i] = b.firstS[i];
    }
    c->Tout = b.Tout; c->Tin = b.Tin;
    c->tables_dirty = b.tables_dirty; c->vclean_n = b.vclean_n; c->stamp_next = b.stamp_next;
    c->first_clean_n = b.first_clean_n;
    c->table_slots_max = b.table_slots_max;
}

// The carve of the static scratch for an n-vertex graph: the buffers
// scc_labels sizes for it (per-vertex state, bitmaps, two reach tables of
// next_pow2(max(1024, 4n)) slots, and per lane a frontier, a heavy list and
// a hash bag for 2n entries per round).  With base == nullptr only the size
// is computed.  Returns the bytes used.
uint64_t static_carve(const scc_options_t &o, int64_t n, uint8_t *base, BufSet *out) {
    uint64_t at = 0;
    auto take = [&](auto &buf, uint64_t elems) {
        using T = typename std::remove_reference<decltype(*buf.p)>::type;
        elems = std::max<uint64_t>(elems, 1);
        at = (at + 255) & ~255ull;
        if (base) {
            buf.p = reinterpret_cast<T *>(base + at);
            buf.cap = elems;
        }
        at += elems * sizeof(T);
    };
    BufSet tmp;
    BufSet &b = out ? *out : tmp;
    const uint64_t nv = (uint64_t)n;
    take(b.label, nv); take(b.aux, nv); take(b.stamp, nv); take(b.fin, nv); take(b.srcvert, nv);
    take(b.srclab, nv); take(b.invp, nv); take(b.sig_out, nv); take(b.sig_in, nv);
    for (int i = 0; i < 2; i++) {
        take(b.vis[i], nv / 32 + 2);
        take(b.bm[i][0], nv / 32 + 2);
        take(b.bm[i][1], nv / 32 + 2);
    }
    const uint64_t T = next_pow2(std::max<uint64_t>(1024, 4 * nv));
    take(b.Tout, T);
    take(b.Tin, T);
    take(b.firstS[0], nv);
    take(b.firstS[1], nv);
    const uint64_t E = 2 * nv;
    const uint32_t lam = lam_log2_for(o, nv);
    uint32_t nch = 1;
    while (((1ull << lam) << (nch - 1)) < 2 * (E + (1ull << lam))) nch++;
    const uint64_t bag = (1ull << lam) << (nch - 1);
    for (int i = 0; i < 2; i++) {
        take(b.F[i], E + kWave);
        take(b.heavy[i], 2 * (E + kWave));
        take(b.bag_slots[i], bag);
        take(b.bag_cnt[i], bag >> kStripeLog2);
        b.bag_nchunks[i] = 0;
        b.bag_lam_log2[i] = 0xffffffffu;  // no lambda yet: the first sizing clears the counters
    }
    b.table_slots_max = T;
    b.tables_dirty = true;  // the array keeps whatever the last call on this device left
    b.vclean_n = 0;
    b.first_clean_n = 0;
    b.stamp_next = 1;
    return (at + 255) & ~255ull;
}

}  // namespace

extern "C" {

const char *scc_version(void) { return "hipscc 0.2 (gfx950)"; }

scc_status scc_default_options(scc_options_t *opt) {
    if (!opt) return SCC_EINVAL;
    *opt = defaults();
    return SCC_OK;
}

scc_status scc_create(scc_ctx_t **ctx, int device, void *stream) {
    if (!ctx) return SCC_EINVAL;
    *ctx = nullptr;
    scc_ctx *c = new (std::nothrow) scc_ctx();
    if (!c) return SCC_ENOMEM;
    scc_status s = guard(c, [&] {
        int ndev = 0;
        HIPCHK(hipGetDeviceCount(&ndev));
        if (device < 0 || device >= ndev) {
            set_err(c, "device %d out of range (%d devices)", device, ndev);
            throw Fail{SCC_EINVAL};
        }
        c->device = device;
        HIPCHK(hipSetDevice(device));
        hipDeviceProp_t prop;
        HIPCHK(hipGetDeviceProperties(&prop, device));
        c->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
        // a reach table's estimated size stops at the largest power of two
        // within 1/16 of device memory (2^31 slots, 16 GiB, on a 288 GB
        // device); a search that needs more grows it by restarting
        {
            uint64_t slots = 1024;
            while (slots * 2 * sizeof(uint64_t) * 16 <= (uint64_t)prop.totalGlobalMem) slots *= 2;
            c->table_slots_max = slots;
        }
        int nb = 0;
        HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_expand<kMulti, 1>, kBlock, 0));
        if (nb < 1) nb = 1;
        c->expand_blocks = c->num_cu * nb;
        // one resident wave of blocks per expand variant: its waves take the
        // frontier's groups statically, so blocks beyond the resident set
        // would run a second, serial local search
        for (int m = 0; m < 6; m++)
            for (int ai = 0; ai < 3; ai++) {
                int b = 0;
                HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, expand_kernel(m, 1 << ai), kBlock, 0));
                c->expand_grid[m][ai] = c->num_cu * std::max(b, 1);
            }
        if (stream) {
            c->stream = (hipStream_t)stream;
        } else {
            HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
            c->own_stream = true;
        }
        HIPCHK(hipMalloc((void **)&c->dctl, sizeof(DevCtl)));
        HIPCHK(hipHostMalloc((void **)&c->hctl, sizeof(DevCtl), hipHostMallocDefault));
        memset(c->hctl, 0, sizeof(DevCtl));
        c->scratch = scratch_address(c);
        reset_ctl(c);
        HIPCHK(hipStreamSynchronize(c->stream));
    });
    if (s != SCC_OK) {
        scc_destroy(c);
        return s;
    }
    *ctx = c;
    return SCC_OK;
}

// Frees every per-graph device buffer of a context (the next call allocates
// what it needs again); the caller has synchronised its stream.
void release_work_buffers(scc_ctx *c) {
    release(c->label); release(c->aux); release(c->stamp); release(c->invp); release(c->srcvert); release(c->srclab);
    release(c->fin); release(c->sig_out); release(c->sig_in);
    for (int i = 0; i < 2; i++) {
        release(c->vis[i]); release(c->bm[i][0]); release(c->bm[i][1]);
        release(c->F[i]); release(c->heavy[i]); release(c->bag_slots[i]); release(c->bag_cnt[i]);
        c->bag_nchunks[i] = 0;
        c->bag_lam_log2[i] = 0;
    }
    release(c->Tout); release(c->Tin); release(c->ubuf);
    release(c->firstS[0]); release(c->firstS[1]); release(c->rec[0]); release(c->rec[1]); release(c->dirty);
    c->first_clean_n = 0;
    release(c->rkeys[0]); release(c->rkeys[1]); release(c->rtemp); release(c->bstart);
    for (int i = 0; i < 2; i++) { release(c->lk[i]); release(c->gk[i]); release(c->ld[i]); release(c->gd[i]); }
    release(c->lkeep);
    c->tables_dirty = false;
    c->vclean_n = 0;
    for (auto &e : c->gcache) (void)hipGraphExecDestroy(e.second);
    c->gcache.clear();
}

void scc_destroy(scc_ctx_t *c) {
    if (!c) return;
    for (scc_ctx *w : c->workers) scc_destroy(w);
    c->workers.clear();
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    release_work_buffers(c);
    policy_release(c->policy);
    if (c->dctl) (void)hipFree(c->dctl);
    if (c->hctl) (void)hipHostFree(c->hctl);
    for (auto &a : c->tev)
        for (auto &e : a)
            if (e) (void)hipEventDestroy(e);
    for (auto e : c->pev) (void)hipEventDestroy(e);
    for (auto &a : c->rev)
        for (auto &e : a)
            if (e) (void)hipEventDestroy(e);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char *scc_last_error(const scc_ctx_t *c) { return c ? c->err.c_str() : "null context"; }

scc_status scc_labels(scc_ctx_t *c, const scc_graph_t *g, int32_t *labels_out, const scc_options_t *opt,
                      scc_stats_t *stats) {
    return guard(c, [&] {
        check_graph_args(c, g);
        if (g->n > 0 && !labels_out) { set_err(c, "labels_out is NULL"); throw Fail{SCC_EINVAL}; }
        scc_options_t o = opt ? *opt : defaults();
        check_opts(c, o);
        const double t0 = now_ms();
        init_call(c, stats, g->n, g->m, &o);
        GraphDev gd{g->n, g->m, g->out_off, g->out_adj, g->in_off, g->in_adj};
        run_scc(c, gd, labels_out, o, stats);
        HIPCHK(hipStreamSynchronize(c->stream));
        if (stats) stats->ms_total = now_ms() - t0;
    });
}

scc_status scc_labels_static(scc_ctx_t *c, const scc_graph_t *g, int32_t *labels_out, const scc_options_t *opt,
                             scc_stats_t *stats) {
    return guard(c, [&] {
        check_graph_args(c, g);
        if (g->n > 0 && !labels_out) { set_err(c, "labels_out is NULL"); throw Fail{SCC_EINVAL}; }
        scc_options_t o = opt ? *opt : defaults();
        check_opts(c, o);
        if (o.timing || o.trace) {
            set_err(c, "scc_labels_static records no events: options.timing and options.trace must be 0");
            throw Fail{SCC_EINVAL};
        }
        if (!c->scratch) { set_err(c, "internal: static scratch address not set"); throw Fail{SCC_EINTERNAL}; }
        const uint64_t need = static_carve(o, g->n, nullptr, nullptr);
        if (need > kStaticScratchBytes) {
            set_err(c, "graph with n = %d needs %llu bytes of static scratch, more than its %llu", g->n,
                    (unsigned long long)need, (unsigned long long)kStaticScratchBytes);
            throw Fail{SCC_ECAPACITY};
        }
        const double t0 = now_ms();
        BufSet heap;
        bufs_save(c, heap);
        struct Restore {
            scc_ctx *c;
            BufSet &heap;
            ~Restore() {
                c->noalloc = false;
                bufs_load(c, heap);
            }
        } restore{c, heap};
        BufSet carved;
        static_carve(o, g->n, c->scratch, &carved);
        bufs_load(c, carved);
        c->noalloc = true;
        init_call(c, stats, g->n, g->m, &o);
        GraphDev gd{g->n, g->m, g->out_off, g->out_adj, g->in_off, g->in_adj};
        run_scc(c, gd, labels_out, o, stats);
        HIPCHK(hipStreamSynchronize(c->stream));
        if (stats) stats->ms_total = now_ms() - t0;
    });
}

scc_status scc_reach(scc_ctx_t *c, const scc_graph_t *g, int32_t dir, const int32_t *sources, int32_t k,
                     const int32_t *labels, int32_t *pairs_out, int64_t capacity, int64_t *n_pairs,
                     const scc_options_t *opt, scc_stats_t *stats) {
    return guard(c, [&] {
        if (n_pairs) *n_pairs = 0;
        check_graph_args(c, g);
        if (!n_pairs || k < 0 || capacity < 0 || (dir != 0 && dir != 1)) {
            set_err(c, "bad argument (n_pairs NULL, k < 0, capacity < 0 or dir not 0/1)");
            throw Fail{SCC_EINVAL};
        }
        if (k > 0 && (!sources || !labels)) { set_err(c, "sources/labels NULL"); throw Fail{SCC_EINVAL}; }
        if (capacity > 0 && !pairs_out) { set_err(c, "pairs_out NULL"); throw Fail{SCC_EINVAL}; }
        scc_options_t o = opt ? *opt : defaults();
        check_opts(c, o);
        const double t0 = now_ms();
        init_call(c, stats, g->n, g->m, &o);
        if (k == 0) return;
        if (k > g->n) { set_err(c, "more sources than vertices"); throw Fail{SCC_EINVAL}; }
        const int32_t n = g->n;
        GraphDev gd{g->n, g->m, g->out_off, g->out_adj, g->in_off, g->in_adj};
        ensure_vertex_state(c, n);
        if (o.validate) validate_graph(c, gd);
        // the source check stamps with its own epochs: the next labelling
        // call clears the vertex state again
        c->vclean_n = 0;
        fill_u32(c, (uint32_t *)c->stamp.p, (uint64_t)n, 0u);
        Shared *sh = &c->dctl->sh;
        fill_u32(c, &sh->bad, 1, 0u);
        hipLaunchKernelGGL(k_check_sources, dim3(grid_for(c, (uint64_t)k)), dim3(kBlock), 0, c->stream, n, k, sources,
                           labels, c->srcvert.p, c->srclab.p, c->stamp.p, 1, &sh->bad);
        LAUNCHCHK("k_check_sources");
        fill_u32(c, &sh->k, 1, (uint32_t)k);
        sync_ctl(c);
        if (c->hctl->sh.bad) {
            set_err(c, "sources must be in range, distinct and not excluded (label >= 0); code %u", c->hctl->sh.bad);
            throw Fail{SCC_EINVAL};
        }
        DriveParams DP;
        DP.o = &o;
        DP.n = n;
        DP.m = g->m;
        DP.nsub = n;
        DP.st = stats;
        double rs = 0;
        DP.resize_ms = &rs;
        Lane L;
        L.id = 0;
        L.n = n;
        uint64_t ts = 0;
        // sort keys (j << vbits) | v: vbits covers the vertex ids, kbits the
        // source indices
        uint32_t vbits = 1, kbits = 0;
        while ((1ll << vbits) < (int64_t)n) vbits++;
        while ((1ll << kbits) < (int64_t)k) kbits++;
        if (k == 1) {
            int32_t s = 0, lab = 0;
            HIPCHK(hipMemcpyAsync(&s, sources, 4, hipMemcpyDeviceToHost, c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
            HIPCHK(hipMemcpyAsync(&lab, labels + s, 4, hipMemcpyDeviceToHost, c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
            ensure_lane(c, 0, (uint64_t)n, lam_log2_for(o, (uint64_t)n));
            reset_bag(c, 0);
            Perm P0{(uint32_t)n, 1, 0};
            hipLaunchKernelGGL(k_premark, dim3(grid_for(c, (uint64_t)n)), dim3(kBlock), 0, c->stream, n, labels, lab, s,
                               sh, P0, c->vis[0].p);
            hipLaunchKernelGGL(k_seed_single, dim3(1), dim3(64), 0, c->stream, s, sh, P0, c->F[0].p, &c->dctl->lane[0],
                               &c->dctl->ls[0], c->vis[0].p);
            LAUNCHCHK("k_seed_single");
            L.mode = kSingle;
            L.S = make_search(c, 0, o, kSingle);
            L.S.off = dir ? g->in_off : g->out_off;
            L.S.adj = dir ? g->in_adj : g->out_adj;
            L.S.label = labels;
            L.S.vis = c->vis[0].p;
            L.roff = dir ? g->out_off : g->in_off;
            L.radj = dir ? g->out_adj : g->in_adj;
            drive(c, &L, 1, DP);
            fill_u32(c, &sh->emit, 1, 0u);
            ensure(c, c->rkeys[0], (uint64_t)n);
            hipLaunchKernelGGL(k_emit_single, dim3(grid_for(c, (uint64_t)n)), dim3(kBlock), 0, c->stream, n, labels, lab,
                               c->vis[0].p, c->rkeys[0].p, c->rkeys[0].cap, sh);
            LAUNCHCHK("k_emit_single");
        } else {
            ts = next_pow2(std::max<uint64_t>(std::max<uint64_t>(1024, 4ull * (uint64_t)k),
                                              o.table_init > 0 ? (uint64_t)o.table_init : (uint64_t)n / 4));
            bool grew = false;
            ensure(c, c->Tout, ts, &grew);
            fill_u64(c, c->Tout.p, grew ? c->Tout.cap : ts, kEmpty64);
            c->tables_dirty = true;
            ensure_lane(c, 0, std::max<uint64_t>(ts, (uint64_t)n), lam_log2_for(o, std::max<uint64_t>(ts, (uint64_t)n)));
            reset_bag(c, 0);
            SeedArgs SA;
            memset(&SA, 0, sizeof SA);
            SA.T[0] = c->Tout.p;
            SA.mask[0] = ts - 1;
            SA.F[0] = c->F[0].p;
            SA.rc[0] = &c->dctl->lane[0];
            SA.ls[0] = &c->dctl->ls[0];
            hipLaunchKernelGGL(k_seed_multi, dim3(grid_for(c, (uint64_t)k), 1), dim3(kBlock), 0, c->stream, c->srcvert.p,
                               sh, SA, kProbeLimit);
            LAUNCHCHK("k_seed_multi");
            L.mode = kMulti;
            L.T = &c->Tout;
            L.tslots = &ts;
            L.S = make_search(c, 0, o, kMulti);
            L.S.off = dir ? g->in_off : g->out_off;
            L.S.adj = dir ? g->in_adj : g->out_adj;
            L.S.label = labels;
            L.S.srclab = c->srclab.p;
            L.S.table = c->Tout.p;
            L.S.tmask = ts - 1;
            drive(c, &L, 1, DP);
            fill_u32(c, &sh->emit, 1, 0u);
            ensure(c, c->rkeys[0], ts);
            hipLaunchKernelGGL(k_emit_table, dim3(grid_for(c, ts)), dim3(kBlock), 0, c->stream, c->Tout.p, ts - 1,
                               vbits, c->rkeys[0].p, c->rkeys[0].cap, sh);
            LAUNCHCHK("k_emit_table");
            // leave the table clean for the next call
            fill_u64(c, c->Tout.p, ts, kEmpty64);
        }
        sync_ctl(c, stats != nullptr);
        c->tables_dirty = false;
        *n_pairs = (int64_t)c->hctl->sh.emit;
        if (*n_pairs > (int64_t)c->rkeys[0].cap) {
            set_err(c, "internal: %lld pairs exceed the key buffer", (long long)*n_pairs);
            throw Fail{SCC_EINTERNAL};
        }
        if (*n_pairs > 0 && *n_pairs <= capacity) {
            // ascending (source index, vertex) order, sorted on the device
            const uint64_t cnt = (uint64_t)*n_pairs;
            ensure(c, c->rkeys[1], cnt);
            size_t tb = 0;
            HIPCHK(rocprim::radix_sort_keys(nullptr, tb, c->rkeys[0].p, c->rkeys[1].p, cnt, 0u, vbits + kbits,
                                            c->stream));
            ensure(c, c->rtemp, (uint64_t)tb);
            HIPCHK(rocprim::radix_sort_keys((void *)c->rtemp.p, tb, c->rkeys[0].p, c->rkeys[1].p, cnt, 0u,
                                            vbits + kbits, c->stream));
            hipLaunchKernelGGL(k_unpack_pairs, dim3(grid_for(c, cnt)), dim3(kBlock), 0, c->stream, c->rkeys[1].p, cnt,
                               vbits, pairs_out);
            LAUNCHCHK("k_unpack_pairs");
            HIPCHK(hipStreamSynchronize(c->stream));
        }
        if (stats) {
            stats->ms_total = now_ms() - t0;
            if (k == 1) stats->rounds_first = L.rounds; else stats->rounds_multi = L.rounds;
            stats->ms_resize = rs;
            stats->dense_rounds = c->dense_rounds;
            fill_counters(c, stats, 0);
        }
        if (*n_pairs > capacity) {
            set_err(c, "%lld pairs exceed capacity %lld", (long long)*n_pairs, (long long)capacity);
            throw Fail{SCC_ECAPACITY};
        }
    });
}

scc_status scc_labels_batched(scc_ctx_t *c, int32_t G, const int64_t *vtx_base, const int64_t *arc_base,
                              const int32_t *out_off, const int32_t *out_adj, const int32_t *in_off,
                              const int32_t *in_adj, int32_t *labels_out, const scc_options_t *opt,
                              scc_stats_t *stats) {
    return guard(c, [&] {
        if (G < 0 || (G > 0 && (!vtx_base || !arc_base || !out_off || !in_off || !labels_out))) {
            set_err(c, "bad batched arguments");
            throw Fail{SCC_EINVAL};
        }
        scc_options_t o = opt ? *opt : defaults();
        check_opts(c, o);
        const double t0 = now_ms();
        init_call(c, stats, G ? vtx_base[G] : 0, G ? arc_base[G] : 0, &o);
        if (G == 0) return;
        if (vtx_base[0] != 0 || arc_base[0] != 0) {
            set_err(c, "vtx_base/arc_base must start at 0");
            throw Fail{SCC_EINVAL};
        }
        for (int32_t i = 0; i < G; i++) {
            if (vtx_base[i + 1] < vtx_base[i] || arc_base[i + 1] < arc_base[i]) {
                set_err(c, "vtx_base/arc_base must never decrease");
                throw Fail{SCC_EINVAL};
            }
            if (arc_base[i + 1] - arc_base[i] >= (1ll << 31)) { set_err(c, "graph %d has >= 2^31 arcs", i); throw Fail{SCC_EINVAL}; }
        }
        if (vtx_base[G] >= (1ll << 31)) { set_err(c, "total vertex count must be < 2^31"); throw Fail{SCC_EINVAL}; }
        if (arc_base[G] > 0 && (!out_adj || !in_adj)) { set_err(c, "adjacency NULL"); throw Fail{SCC_EINVAL}; }
        DevBuf<int64_t> dvb, dab;
        struct Free {
            DevBuf<int64_t> &a, &b;
            ~Free() { release(a); release(b); }
        } fr{dvb, dab};
        ensure(c, dvb, (uint64_t)G + 1);
        ensure(c, dab, (uint64_t)G + 1);
        HIPCHK(hipMemcpyAsync(dvb.p, vtx_base, 8 * ((size_t)G + 1), hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(dab.p, arc_base, 8 * ((size_t)G + 1), hipMemcpyHostToDevice, c->stream));
        // groups of consecutive graphs whose union has < 2^31 arcs; the
        // disjoint union of a group is one digraph whose SCCs are the graphs'
        const int64_t lim = o.union_arcs_max > 0 ? (int64_t)o.union_arcs_max : (1ll << 31) - 1;
        const int nstreams = o.union_streams > 0 ? o.union_streams : kAutoUnionStreams;
        std::vector<std::pair<int32_t, int32_t>> groups;
        {
            // at least nstreams groups (when there are that many graphs),
            // each closed once it holds its share of the arcs
            int64_t parts = std::max<int64_t>((arc_base[G] + lim - 1) / lim, nstreams);
            parts = std::min<int64_t>(parts, G);
            const int64_t share = (arc_base[G] + parts - 1) / std::max<int64_t>(parts, 1);
            int32_t g0 = 0;
            while (g0 < G) {
                int32_t g1 = g0 + 1;
                while (g1 < G && arc_base[g1 + 1] - arc_base[g0] < lim && arc_base[g1] - arc_base[g0] < share &&
                       (int64_t)groups.size() + 1 < parts)
                    g1++;
                if ((int64_t)groups.size() + 1 >= parts)  // the last part takes the rest, up to the arc limit
                    while (g1 < G && arc_base[g1 + 1] - arc_base[g0] < lim) g1++;
                groups.push_back({g0, g1});
                g0 = g1;
            }
        }
        // one union on context c (its stream, its buffers; the parameter
        // hides the calling context, so errors are reported on c)
        auto run_union = [&](scc_ctx *c, int32_t g0, int32_t g1, scc_stats_t *acc) {
            const int32_t cnt = g1 - g0;
            const int64_t nv = vtx_base[g1] - vtx_base[g0];
            const int64_t na = arc_base[g1] - arc_base[g0];
            // union CSR scratch: 2 (nv + 1) offsets + 2 na arcs + nv labels
            const uint64_t need = 2 * ((uint64_t)nv + 1) + 2 * (uint64_t)na + (uint64_t)nv;
            ensure(c, c->ubuf, need);
            int32_t *uo = c->ubuf.p, *ui = uo + nv + 1, *ua = ui + nv + 1, *uia = ua + na, *ul = uia + na;
            auto tiles = [&](uint64_t x) {
                return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((x + kUnionTile - 1) / kUnionTile,
                                                                         (uint64_t)c->num_cu * 8));
            };
            const unsigned gv = tiles((uint64_t)nv + 1), ga = tiles((uint64_t)std::max<int64_t>(na, 1));
            hipLaunchKernelGGL(k_union_off, dim3(gv), dim3(kBlock), 0, c->stream, cnt, dvb.p, dab.p, out_off, uo,
                               arc_base[g0], g0);
            hipLaunchKernelGGL(k_union_off, dim3(gv), dim3(kBlock), 0, c->stream, cnt, dvb.p, dab.p, in_off, ui,
                               arc_base[g0], g0);
            if (na > 0) {
                hipLaunchKernelGGL(k_union_adj, dim3(ga), dim3(kBlock), 0, c->stream, cnt, dvb.p, dab.p, out_adj, ua,
                                   g0);
                hipLaunchKernelGGL(k_union_adj, dim3(ga), dim3(kBlock), 0, c->stream, cnt, dvb.p, dab.p, in_adj, uia,
                                   g0);
            }
            LAUNCHCHK("k_union_*");
            GraphDev gd{(int32_t)nv, (int32_t)na, uo, ua, ui, uia};
            scc_stats_t st;
            init_call(c, acc ? &st : nullptr, nv, na, &o);
            run_scc(c, gd, ul, o, acc ? &st : nullptr);
            hipLaunchKernelGGL(k_union_labels, dim3(tiles((uint64_t)nv)), dim3(kBlock), 0, c->stream, cnt, dvb.p, ul,
                               labels_out, g0);
            LAUNCHCHK("k_union_labels");
            HIPCHK(hipStreamSynchronize(c->stream));
            if (acc) accumulate_stats(*acc, st);
        };
        scc_stats_t acc;
        memset(&acc, 0, sizeof acc);
        const int nw = (int)std::min<size_t>((size_t)nstreams, groups.size());
        if (nw <= 1) {
            // the workers' buffers of earlier concurrent calls go first
            for (scc_ctx *w : c->workers) scc_destroy(w);
            c->workers.clear();
            for (auto &gr : groups) run_union(c, gr.first, gr.second, stats ? &acc : nullptr);
        } else {
            // so do this context's own per-graph buffers and any workers
            // beyond this call's count: each union's state lives in one place
            HIPCHK(hipStreamSynchronize(c->stream));
            release_work_buffers(c);
            while ((int)c->workers.size() > nw) {
                scc_destroy(c->workers.back());
                c->workers.pop_back();
            }
            // a different split sizes every union differently: buffers sized
            // for the old unions go before the new ones are allocated
            if ((int)c->workers.size() != nw || c->worker_groups != groups.size()) {
                for (scc_ctx *w : c->workers) {
                    HIPCHK(hipStreamSynchronize(w->stream));
                    release_work_buffers(w);
                }
                c->worker_groups = groups.size();
            }
            // worker contexts, each with its own stream and buffers; they
            // start once the bases are on the device (the inputs were written
            // on the calling context's stream before this call)
            while ((int)c->workers.size() < nw) {
                scc_ctx_t *w = nullptr;
                const scc_status cs = scc_create(&w, c->device, nullptr);
                if (cs != SCC_OK) {
                    set_err(c, "creating a union worker context failed (%d)", (int)cs);
                    throw Fail{cs};
                }
                c->workers.push_back(w);
            }
            std::vector<float> pw;
            if (c->policy.loaded) {
                pw.resize(kPolicyFloats);
                HIPCHK(hipMemcpyAsync(pw.data(), c->policy.w, sizeof(float) * kPolicyFloats, hipMemcpyDeviceToHost,
                                      c->stream));
            }
            HIPCHK(hipStreamSynchronize(c->stream));
            for (int w = 0; w < nw; w++) {
                scc_ctx *wc = c->workers[w];
                if (c->policy.loaded) {
                    if (policy_load(wc->policy, pw.data(), kPolicyFloats, wc->stream) != 0) {
                        set_err(c, "policy upload to a union worker failed");
                        throw Fail{SCC_EHIP};
                    }
                } else {
                    policy_release(wc->policy);
                }
            }
            std::vector<scc_status> rc(nw, SCC_OK);
            std::vector<std::string> msg(nw);
            std::vector<scc_stats_t> wacc(nw);
            for (auto &a : wacc) memset(&a, 0, sizeof a);
            std::vector<std::thread> th;
            for (int w = 0; w < nw; w++)
                th.emplace_back([&, w] {
                    scc_ctx *wc = c->workers[w];
                    rc[w] = guard(wc, [&] {
                        const hipError_t e = hipSetDevice(wc->device);
                        if (e != hipSuccess) {
                            set_err(wc, "hipSetDevice failed: %s", hipGetErrorString(e));
                            throw Fail{SCC_EHIP};
                        }
                        for (size_t i = (size_t)w; i < groups.size(); i += (size_t)nw)
                            run_union(wc, groups[i].first, groups[i].second, stats ? &wacc[w] : nullptr);
                    });
                    if (rc[w] != SCC_OK) msg[w] = wc->err;
                });
            for (auto &t : th) t.join();
            for (int w = 0; w < nw; w++)
                if (rc[w] != SCC_OK) {
                    set_err(c, "union worker %d: %s", w, msg[w].c_str());
                    throw Fail{rc[w]};
                }
            if (stats)
                for (int w = 0; w < nw; w++) accumulate_stats(acc, wacc[w]);
        }
        if (stats) {
            acc.n = vtx_base[G];
            acc.m = arc_base[G];
            acc.ms_total = now_ms() - t0;
            *stats = acc;
        }
    });
}

scc_status scc_cc(scc_ctx_t *c, const scc_graph_t *g, int32_t *labels_out, const scc_options_t *opt,
                  scc_stats_t *stats) {
    return guard(c, [&] {
        if (!g) { set_err(c, "graph is NULL"); throw Fail{SCC_EINVAL}; }
        if (g->n < 0 || g->m < 0) { set_err(c, "negative n or m"); throw Fail{SCC_EINVAL}; }
        if (!g->out_off || (g->m > 0 && !g->out_adj)) { set_err(c, "graph has a NULL out array"); throw Fail{SCC_EINVAL}; }
        if (g->n > 0 && !labels_out) { set_err(c, "labels_out is NULL"); throw Fail{SCC_EINVAL}; }
        scc_options_t o = opt ? *opt : defaults();
        check_opts(c, o);
        const double t0 = now_ms();
        init_call(c, stats, g->n, g->m, &o);
        const int32_t n = g->n;
        const int64_t m = g->m;
        if (n == 0) return;
        const bool ph = stats != nullptr;
        ensure_vertex_state(c, n);
        if (o.validate) {
            uint32_t *bad = &c->dctl->sh.bad;
            fill_u32(c, bad, 1, 0u);
            hipLaunchKernelGGL(k_validate_off, dim3(grid_for(c, (uint64_t)n + 1)), dim3(kBlock), 0, c->stream, n,
                               g->m, g->out_off, bad);
            if (m > 0)
                hipLaunchKernelGGL(k_validate_adj, dim3(grid_for(c, (uint64_t)m)), dim3(kBlock), 0, c->stream, n, g->m,
                                   g->out_adj, (int32_t *)nullptr, bad);
            LAUNCHCHK("k_validate_*");
            sync_ctl(c);
            if (c->hctl->sh.bad) { set_err(c, "invalid CSR (offsets or arc targets)"); throw Fail{SCC_EGRAPH}; }
        }
        int32_t *owner = c->srcvert.p, *parent = c->srclab.p;
        // the degree maximum (the edge-parallel pass is skipped without heavy vertices)
        hipLaunchKernelGGL(k_max_deg, dim3(grid_for(c, (uint64_t)n)), dim3(kBlock), 0, c->stream, n, g->out_off,
                           &c->dctl->sh);
        LAUNCHCHK("k_max_deg");
        // ---- low-diameter decomposition (Algorithm 4, LDD): one search
        // lane, a centre batch added before every round
        phase_begin(c, 1, ph);
        ensure_lane(c, 0, (uint64_t)n, lam_log2_for(o, (uint64_t)n));
        reset_bag(c, 0);
        reset_lane_ctl(c, 0);
        fill_u32(c, (uint32_t *)&c->dctl->ls[0], sizeof(LaneStripes) / 4, 0u);
        fill_u32(c, c->vis[0].p, (uint64_t)n / 32 + 2, 0u);
        hipLaunchKernelGGL(k_iota, dim3(grid_for(c, (uint64_t)n)), dim3(kBlock), 0, c->stream, n, parent);
        LAUNCHCHK("k_iota");
        Perm P;
        P.n = (uint32_t)n;
        uint32_t bits = 1;
        while ((1ull << (2 * bits)) < (uint64_t)n) bits++;
        P.half_bits = bits;
        P.key = mix64(o.seed ^ 0x452821E638D01377ull);
        Lane L;
        L.id = 0;
        L.mode = kLdd;
        L.n = n;
        L.S = make_search(c, 0, o, kLdd);
        L.S.off = g->out_off;
        L.S.adj = g->out_adj;
        L.S.vis = c->vis[0].p;
        L.S.owner = owner;
        L.avg_deg = std::max(1.0, (double)m / (double)n);
        L.par = 0;
        uint64_t pos = 0;
        double bsize = 1.0;
        int64_t rounds = 0;
        while (pos < (uint64_t)n) {
            // every vertex of the batch that no cluster has reached yet
            // becomes a centre (Algorithm 4 adds B_i to the frontier)
            const uint64_t sz = std::max<uint64_t>((uint64_t)std::ceil(bsize - 1e-9), 1);
            const uint64_t p1 = std::min<uint64_t>((uint64_t)n, pos + sz);
            hipLaunchKernelGGL(k_ldd_add, dim3(grid_for(c, p1 - pos)), dim3(kBlock), 0, c->stream, P, (uint32_t)pos,
                               (uint32_t)p1, g->out_off, c->vis[0].p, owner, L.S.F, L.S.fcap, L.S.rc, L.par);
            LAUNCHCHK("k_ldd_add");
            pos = p1;
            bsize *= (double)o.ldd_beta;
            // once every vertex has a cluster the remaining frontier could
            // only find claimed vertices: the decomposition is complete
            if (pos >= (uint64_t)n) break;
            launch_sparse(c, std::array<Lane *, 1>{&L}.data(), 1);
            rounds++;
            if (rounds % kMaxSlots == 0) {
                sync_ctl(c);
                timed_collect(c);
                if ((c->hctl->lane[0].err & kErrCapacity) || c->hctl->bag[0].overflow) {
                    set_err(c, "internal: LDD frontier capacity exceeded");
                    throw Fail{SCC_EINTERNAL};
                }
            }
        }
        sync_ctl(c);
        timed_collect(c);
        if ((c->hctl->lane[0].err & kErrCapacity) || c->hctl->bag[0].overflow) {
            set_err(c, "internal: LDD frontier capacity exceeded");
            throw Fail{SCC_EINTERNAL};
        }
        phase_end(c, ph);
        // ---- union-find over the arcs between clusters, then the canonical
        // smallest vertex id per component
        phase_begin(c, 4, ph);
        if (m > 0) {
            const int64_t nb = (m + kUnionArcs - 1) / kUnionArcs;
            ensure(c, c->bstart, (uint64_t)nb + 1);
            hipLaunchKernelGGL(k_arc_block_starts, dim3(grid_for(c, (uint64_t)n)), dim3(kBlock), 0, c->stream, n,
                               g->out_off, (int64_t)kUnionArcs, c->bstart.p);
            const int tu = timed_begin(c, SCC_KERNEL_UNION);
            hipLaunchKernelGGL(k_cc_union, dim3((unsigned)std::min<int64_t>(nb, (int64_t)c->num_cu * 16)), dim3(kBlock),
                               0, c->stream, n, m, g->out_off, g->out_adj, owner, parent, c->bstart.p, &c->dctl->cn);
            LAUNCHCHK("k_cc_union");
            timed_end(c, tu);
        }
        hipLaunchKernelGGL(k_cc_finish, dim3(grid_for(c, (uint64_t)n)), dim3(kBlock), 0, c->stream, n, owner, parent,
                           c->label.p);
        hipLaunchKernelGGL(k_iota, dim3(grid_for(c, (uint64_t)n)), dim3(kBlock), 0, c->stream, n, c->aux.p);
        hipLaunchKernelGGL(k_canon_min, dim3(grid_for(c, (uint64_t)n, 4)), dim3(kBlock), 0, c->stream, n, c->label.p,
                           c->aux.p, &c->dctl->sh.bad);
        hipLaunchKernelGGL(k_canon_write, dim3(grid_for(c, (uint64_t)n)), dim3(kBlock), 0, c->stream, n, c->label.p,
                           c->aux.p, labels_out, &c->dctl->cs);
        LAUNCHCHK("k_cc_finish / canonical");
        phase_end(c, ph);
        sync_ctl(c, stats != nullptr);
        timed_collect(c);
        if (c->hctl->sh.bad & kErrUnfinished) { set_err(c, "internal: a vertex ended without a component"); throw Fail{SCC_EINTERNAL}; }
        if (stats) {
            double ms[kPhases] = {0, 0, 0, 0, 0};
            phase_collect(c, ms);
            stats->ms_first = ms[1];
            stats->ms_label = ms[4];
            stats->rounds_first = rounds;
            stats->batches = rounds + 1;
            stats->n_scc = count_sum(c, &CountLine::nscc);
            fill_counters(c, stats, n);
            stats->ms_total = now_ms() - t0;
        }
    });
}

scc_status scc_le_lists(scc_ctx_t *c, const scc_graph_t *g, int32_t *order_out, int64_t *loff, int32_t *src_out,
                        int32_t *dist_out, int64_t capacity, int64_t *n_entries, const scc_options_t *opt,
                        scc_stats_t *stats) {
    return guard(c, [&] {
        if (n_entries) *n_entries = 0;
        if (!g || !n_entries) { set_err(c, "graph or n_entries is NULL"); throw Fail{SCC_EINVAL}; }
        if (g->n < 0 || g->m < 0 || capacity < 0) { set_err(c, "negative n, m or capacity"); throw Fail{SCC_EINVAL}; }
        if (!g->out_off || (g->m > 0 && !g->out_adj)) { set_err(c, "graph has a NULL out array"); throw Fail{SCC_EINVAL}; }
        if (!loff || (capacity > 0 && (!src_out || !dist_out))) { set_err(c, "output array is NULL"); throw Fail{SCC_EINVAL}; }
        scc_options_t o = opt ? *opt : defaults();
        check_opts(c, o);
        const double t0 = now_ms();
        init_call(c, stats, g->n, g->m, &o);
        const int32_t n = g->n;
        if (n == 0) {
            fill_u32(c, (uint32_t *)loff, 2, 0u);
            HIPCHK(hipStreamSynchronize(c->stream));
            return;
        }
        const bool ph = stats != nullptr;
        ensure_vertex_state(c, n);
        c->tables_dirty = true;  // the batches leave their pairs in the table
        if (o.validate) {
            uint32_t *bad = &c->dctl->sh.bad;
            fill_u32(c, bad, 1, 0u);
            hipLaunchKernelGGL(k_validate_off, dim3(grid_for(c, (uint64_t)n + 1)), dim3(kBlock), 0, c->stream, n,
                               g->m, g->out_off, bad);
            if (g->m > 0)
                hipLaunchKernelGGL(k_validate_adj, dim3(grid_for(c, (uint64_t)g->m)), dim3(kBlock), 0, c->stream, n,
                                   g->m, g->out_adj, (int32_t *)nullptr, bad);
            LAUNCHCHK("k_validate_*");
            sync_ctl(c);
            if (c->hctl->sh.bad) { set_err(c, "invalid CSR (offsets or arc targets)"); throw Fail{SCC_EGRAPH}; }
        }
        // delta(v): the best distance to v from the sources of earlier batches
        int32_t *delta = c->label.p;
        fill_u32(c, (uint32_t *)delta, (uint64_t)n, (uint32_t)kInf32);
        Perm P;
        P.n = (uint32_t)n;
        uint32_t bits = 1;
        while ((1ull << (2 * bits)) < (uint64_t)n) bits++;
        P.half_bits = bits;
        P.key = mix64(o.seed ^ 0x13198A2E03707344ull);
        if (order_out) {
            hipLaunchKernelGGL(k_perm_write, dim3(grid_for(c, (uint64_t)n)), dim3(kBlock), 0, c->stream, P, n, order_out);
            LAUNCHCHK("k_perm_write");
        }
        uint32_t pbits = 1;
        while ((1ll << pbits) < (int64_t)n) pbits++;
        Shared *sh = &c->dctl->sh;
        // the degree maximum (the edge-parallel pass is skipped without heavy vertices)
        hipLaunchKernelGGL(k_max_deg, dim3(grid_for(c, (uint64_t)n)), dim3(kBlock), 0, c->stream, n, g->out_off, sh);
        LAUNCHCHK("k_max_deg");
        uint64_t gcap = 4 * (uint64_t)n + 1024;  // the list log: about n H_n entries expected
        ensure(c, c->gk[0], gcap);
        ensure(c, c->gd[0], gcap);
        gcap = std::min<uint64_t>(c->gk[0].cap, c->gd[0].cap);
        fill_u32(c, (uint32_t *)&sh->cursor, 2, 0u);
        uint64_t total = 0;
        uint64_t pos = 0;
        double bsize = 1.0;
        uint64_t prev_pairs = 0, prev_k = 1;
        int64_t levels = 0, batches = 0, restarts = 0;
        phase_begin(c, 2, ph);
        while (pos < (uint64_t)n) {
            const uint64_t k = std::min<uint64_t>((uint64_t)n - pos, std::max<uint64_t>((uint64_t)std::ceil(bsize - 1e-9), 1));
            uint32_t kbits = 0;
            while ((1ull << kbits) < k) kbits++;
            hipLaunchKernelGGL(k_le_sources, dim3(grid_for(c, k)), dim3(kBlock), 0, c->stream, P, (uint32_t)pos,
                               (uint32_t)k, c->srcvert.p);
            LAUNCHCHK("k_le_sources");
            // table for the batch's pairs: the previous batch's pairs scaled by
            // the growth (a larger table on overflow)
            uint64_t ts = next_pow2(std::min<uint64_t>(
                std::max<uint64_t>({1024, 4 * k, 2 * prev_pairs * ((k + prev_k - 1) / prev_k)}), c->table_slots_max));
            uint64_t logged = 0;
            for (;;) {
                bool grew = false;
                ensure(c, c->Tout, ts, &grew);
                fill_u64(c, c->Tout.p, grew ? c->Tout.cap : ts, kEmpty64);
                ensure_lane(c, 0, std::max<uint64_t>(ts, (uint64_t)n), lam_log2_for(o, (uint64_t)n));
                reset_bag(c, 0);
                reset_lane_ctl(c, 0);
                ensure(c, c->lk[0], ts);
                ensure(c, c->ld[0], ts);
                const uint64_t lcap = std::min<uint64_t>(c->lk[0].cap, c->ld[0].cap);
                fill_u32(c, &sh->emit, 1, 0u);
                fill_u32(c, &sh->k, 1, (uint32_t)k);
                Lane L;
                L.id = 0;
                L.mode = kLe;
                L.n = n;
                L.S = make_search(c, 0, o, kLe);
                L.S.off = g->out_off;
                L.S.adj = g->out_adj;
                L.S.label = delta;
                L.S.table = c->Tout.p;
                L.S.tmask = ts - 1;
                L.S.tau = 0;  // BFS order: no local search
                // ExtractAll logs every level's new entries (pair key, distance)
                L.S.lkeys = c->lk[0].p;
                L.S.ldist = c->ld[0].p;
                L.S.lcap = lcap;
                L.S.lkbits = kbits;
                L.S.lsh = sh;
                L.avg_deg = std::max(1.0, (double)g->m / (double)n);
                L.par = 0;
                SeedArgs SA;
                memset(&SA, 0, sizeof SA);
                SA.T[0] = c->Tout.p;
                SA.mask[0] = ts - 1;
                SA.F[0] = c->F[0].p;
                SA.rc[0] = &c->dctl->lane[0];
                SA.ls[0] = &c->dctl->ls[0];
                hipLaunchKernelGGL(k_seed_multi, dim3(grid_for(c, k), 1), dim3(kBlock), 0, c->stream, c->srcvert.p, sh,
                                   SA, kProbeLimit);
                LAUNCHCHK("k_seed_multi");
                hipLaunchKernelGGL(k_le_log, dim3(grid_for(c, k)), dim3(kBlock), 0, c->stream, L.S.F, L.S.rc, 0,
                                   L.S.fcap, 0, kbits, c->lk[0].p, c->ld[0].p, lcap, sh);
                LAUNCHCHK("k_le_log");
                int32_t level = 0;
                int K = 1;
                bool failed = false;
                for (;;) {
                    for (int r = 0; r < K; r++) {
                        L.S.level = level;
                        Lane *one = &L;
                        launch_sparse(c, &one, 1);
                        level++;
                    }
                    sync_ctl(c);
                    timed_collect(c);
                    const RoundCtl &rc = c->hctl->lane[0];
                    if ((rc.err & (kErrTable | kErrCapacity)) || c->hctl->bag[0].overflow ||
                        (uint64_t)c->hctl->sh.emit > lcap) {
                        failed = true;
                        break;
                    }
                    if (rc.nF[0] + rc.nF[1] == 0) break;
                    K = std::min(K * 2, kMaxSlots);
                }
                levels += c->hctl->lane[0].rounds;
                if (!failed) {
                    logged = c->hctl->sh.emit;
                    break;
                }
                // the batch restarts on a table (and log) twice as large; delta
                // has not changed yet
                restarts++;
                ts *= 2;
            }
            // per vertex: sort the batch's pairs by (w, j), keep those that beat
            // every earlier source of the batch, lower delta, append to the lists
            if (logged > 0) {
                ensure(c, c->lk[1], logged);
                ensure(c, c->ld[1], logged);
                ensure(c, c->lkeep, logged);
                const uint32_t wbits = pbits + 1;
                size_t tb = 0;
                HIPCHK(rocprim::radix_sort_pairs(nullptr, tb, c->lk[0].p, c->lk[1].p, c->ld[0].p, c->ld[1].p, logged, 0u,
                                                 kbits + wbits, c->stream));
                ensure(c, c->rtemp, (uint64_t)tb);
                HIPCHK(rocprim::radix_sort_pairs((void *)c->rtemp.p, tb, c->lk[0].p, c->lk[1].p, c->ld[0].p, c->ld[1].p,
                                                 logged, 0u, kbits + wbits, c->stream));
                hipLaunchKernelGGL(k_le_filter, dim3(grid_for(c, logged)), dim3(kBlock), 0, c->stream, c->lk[1].p,
                                   c->ld[1].p, logged, kbits, c->lkeep.p, delta);
                LAUNCHCHK("k_le_filter");
                // room for every survivor of this batch in the list log
                if (total + logged > gcap) {
                    const uint64_t want = std::max<uint64_t>(2 * gcap, total + logged);
                    grow_keep(c, c->gk[0], want, total);
                    grow_keep(c, c->gd[0], want, total);
                    gcap = std::min<uint64_t>(c->gk[0].cap, c->gd[0].cap);
                }
                hipLaunchKernelGGL(k_le_append, dim3(grid_for(c, logged)), dim3(kBlock), 0, c->stream, c->lk[1].p,
                                   c->ld[1].p, c->lkeep.p, logged, kbits, (uint32_t)pos, pbits, c->gk[0].p, c->gd[0].p,
                                   gcap, &sh->cursor);
                LAUNCHCHK("k_le_append");
                sync_ctl(c);
                total = c->hctl->sh.cursor;
            }
            prev_pairs = logged;
            prev_k = k;
            pos += k;
            bsize *= (double)o.beta;
            batches++;
        }
        phase_end(c, ph);
        *n_entries = (int64_t)total;
        if ((int64_t)total > capacity) {
            set_err(c, "%llu list entries exceed capacity %lld", (unsigned long long)total, (long long)capacity);
            throw Fail{SCC_ECAPACITY};
        }
        // the lists: sort the log by (vertex, source position), then CSR
        phase_begin(c, 4, ph);
        ensure(c, c->gk[1], std::max<uint64_t>(total, 1));
        ensure(c, c->gd[1], std::max<uint64_t>(total, 1));
        if (total > 0) {
            size_t tb = 0;
            HIPCHK(rocprim::radix_sort_pairs(nullptr, tb, c->gk[0].p, c->gk[1].p, c->gd[0].p, c->gd[1].p, total, 0u,
                                             2 * pbits + 1, c->stream));
            ensure(c, c->rtemp, (uint64_t)tb);
            HIPCHK(rocprim::radix_sort_pairs((void *)c->rtemp.p, tb, c->gk[0].p, c->gk[1].p, c->gd[0].p, c->gd[1].p,
                                             total, 0u, 2 * pbits + 1, c->stream));
        }
        hipLaunchKernelGGL(k_le_csr, dim3(grid_for(c, total + 1)), dim3(kBlock), 0, c->stream, c->gk[1].p, c->gd[1].p,
                           total, pbits, n, P, loff, src_out, dist_out);
        LAUNCHCHK("k_le_csr");
        phase_end(c, ph);
        sync_ctl(c, stats != nullptr);
        if (stats) {
            double ms[kPhases] = {0, 0, 0, 0, 0};
            phase_collect(c, ms);
            stats->ms_multi = ms[2];
            stats->ms_label = ms[4];
            stats->batches = batches;
            stats->rounds_multi = levels;
            stats->table_restarts = restarts;
            fill_counters(c, stats, n);
            stats->ms_total = now_ms() - t0;
        }
    });
}

scc_status scc_policy_load(scc_ctx_t *c, const float *weights, int64_t n_floats) {
    return guard(c, [&] {
        HIPCHK(hipSetDevice(c->device));
        int rc = policy_load(c->policy, weights, n_floats, c->stream);
        if (rc == 1) { set_err(c, "policy needs %d floats, got %lld", kPolicyFloats, (long long)n_floats); throw Fail{SCC_EPOLICY}; }
        if (rc == 2) { set_err(c, "policy weights must be finite"); throw Fail{SCC_EPOLICY}; }
        if (rc != 0) { set_err(c, "policy upload failed"); throw Fail{SCC_EHIP}; }
    });
}

scc_status scc_policy_eval(scc_ctx_t *c, const float *feats, int32_t rows, float *scores) {
    return guard(c, [&] {
        HIPCHK(hipSetDevice(c->device));
        if (rows < 0 || (rows > 0 && (!feats || !scores))) { set_err(c, "bad arguments"); throw Fail{SCC_EINVAL}; }
        if (!c->policy.loaded) { set_err(c, "no policy loaded"); throw Fail{SCC_EPOLICY}; }
        if (rows == 0) return;
        int rc = policy_eval_host(c->policy, feats, rows, scores, c->stream);
        if (rc != 0) { set_err(c, "policy evaluation failed (%d)", rc); throw Fail{SCC_EHIP}; }
    });
}

scc_status scc_trace_read(scc_ctx_t *c, float *out, int64_t cap, int64_t *n_rows) {
    return guard(c, [&] {
        if (!n_rows || cap < 0 || (cap > 0 && !out)) { set_err(c, "bad arguments"); throw Fail{SCC_EINVAL}; }
        const int64_t rows = (int64_t)(c->trace.size() / SCC_TRACE_FIELDS);
        *n_rows = rows;
        const int64_t k = std::min(rows, cap);
        if (k > 0) memcpy(out, c->trace.data(), sizeof(float) * (size_t)k * SCC_TRACE_FIELDS);
    });
}

scc_status scc_bag_selftest(scc_ctx_t *c, const uint64_t *keys, int64_t n, int32_t rounds, uint64_t *out,
                            int64_t *n_out, const scc_options_t *opt, scc_stats_t *stats) {
    return guard(c, [&] {
        if (n < 0 || rounds < 1 || !n_out || (n > 0 && (!keys || !out)) || n >= (1ll << 31)) {
            set_err(c, "bad arguments");
            throw Fail{SCC_EINVAL};
        }
        *n_out = 0;
        scc_options_t o = opt ? *opt : defaults();
        check_opts(c, o);
        init_call(c, stats, n, 0, &o);
        const uint64_t per_round = (uint64_t)((n + rounds - 1) / rounds);
        ensure_lane(c, 0, std::max<uint64_t>(per_round, 1), lam_log2_for(o, std::max<uint64_t>(per_round, 1)));
        ensure(c, c->F[0], (uint64_t)n + kWave);
        reset_bag(c, 0);
        Search S = make_search(c, 0, o, kSingle);
        S.bag.track = 1;
        c->bag_rows.clear();
        c->bag_prefix.clear();
        uint64_t adv = 0;
        for (int32_t rr = 0; rr < rounds; rr++) {
            S.bag.salt = c->salt++;
            fill_u32(c, c->dctl->bag[0].fill, kMaxChunks, 0u);
            fill_u32(c, (uint32_t *)&c->dctl->bag[0].forced, 2, 0u);
            hipLaunchKernelGGL(k_bag_insert_test, dim3((unsigned)c->num_cu * 4), dim3(kBlock), 0, c->stream, keys, n,
                               rounds, rr, S.bag, S.cn);
            LAUNCHCHK("k_bag_insert_test");
            sync_ctl(c);
            adv += c->hctl->bag[0].advances;
            if (c->hctl->bag[0].overflow) { set_err(c, "bag overflow"); throw Fail{SCC_EINTERNAL}; }
            // par = 1: ExtractAll appends to nF[0], which accumulates over rounds
            LanePair LP;
            memset(&LP, 0, sizeof LP);
            LP.S[0] = S;
            LP.S[0].par = 1;
            LP.nl = 1;
            hipLaunchKernelGGL(k_bag_extract, dim3(extract_blocks(c)), dim3(kBlock), 0, c->stream, LP);
            LAUNCHCHK("k_bag_extract");
            fill_u32(c, &c->dctl->bag[0].advances, 1, 0u);
            // chunks below the one current at ExtractAll were left during the
            // round: their fill is the load at the move (plus late inserts)
            sync_ctl(c);
            const BagCtl &bc = c->hctl->bag[0];
            for (uint32_t i = 0; i < bc.last_r && i < (uint32_t)kMaxChunks; i++) {
                const double size = (double)(bag_chunk_hi(S.bag, i) - bag_chunk_lo(S.bag, i));
                c->bag_rows.push_back((double)rr);
                c->bag_rows.push_back((double)i);
                c->bag_rows.push_back((double)bc.fill[i] / size);
                c->bag_rows.push_back((double)((bc.forced >> i) & 1ull));
            }
            c->bag_prefix.push_back((int64_t)bag_chunk_hi(S.bag, bc.last_r));
        }
        sync_ctl(c, true);
        const uint64_t got = c->hctl->lane[0].nF[0];
        if (got > 0)
            HIPCHK(hipMemcpyAsync(out, c->F[0].p, 8 * std::min<uint64_t>(got, (uint64_t)n), hipMemcpyDeviceToDevice,
                                  c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        *n_out = (int64_t)got;
        if (stats) {
            stats->bag_inserts = (int64_t)ctr_kind(c->hctl->cn, kKindExpandSingle, kCtrInserts);
            stats->bag_chunk_advances = (int64_t)adv;
        }
    });
}

scc_status scc_bag_stats(scc_ctx_t *c, double *rows, int64_t cap, int64_t *n_rows, int64_t *prefix,
                         int64_t prefix_cap, int64_t *n_rounds) {
    return guard(c, [&] {
        if (!n_rows || !n_rounds || cap < 0 || prefix_cap < 0 || (cap > 0 && !rows) || (prefix_cap > 0 && !prefix)) {
            set_err(c, "bad arguments");
            throw Fail{SCC_EINVAL};
        }
        const int64_t nr = (int64_t)(c->bag_rows.size() / 4);
        *n_rows = nr;
        if (std::min(nr, cap) > 0) memcpy(rows, c->bag_rows.data(), sizeof(double) * 4 * (size_t)std::min(nr, cap));
        *n_rounds = (int64_t)c->bag_prefix.size();
        const int64_t np = std::min(*n_rounds, prefix_cap);
        if (np > 0) memcpy(prefix, c->bag_prefix.data(), sizeof(int64_t) * (size_t)np);
    });
}

}  // extern "C"
