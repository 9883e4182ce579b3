// hipscc host runtime: the C ABI of include/hipscc.h.
//
// Algorithm 1 (BGSS) driven from the host one source batch at a time; each
// reachability search runs as device-resident rounds (expand -> heavy ->
// ExtractAll), launched in blocks of rounds between host checks of the
// frontier size.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "hipscc.h"
#include "kernels.h"
#include "policy.h"

using namespace hipscc;

namespace {

struct DevCtl {
    RoundCtl rc;
    BagCtl bc;
};

template <typename T>
struct DevBuf {
    T *p = nullptr;
    uint64_t cap = 0;  // elements
};

struct Fail {
    scc_status code;
};

}  // namespace

struct scc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int num_cu = 256;
    int expand_blocks = 2048;
    std::string err;

    DevBuf<int32_t> label, aux, stamp, srcvert, srclab, fin;
    DevBuf<unsigned long long> sig_out, sig_in;
    DevBuf<uint32_t> visF, visB;
    DevBuf<uint64_t> Tout, Tin;
    DevBuf<uint64_t> F, heavy;
    DevBuf<uint64_t> bag_slots;
    DevBuf<uint32_t> bag_cnt;
    uint32_t bag_nchunks = 0;
    uint32_t bag_lam_log2 = 0;
    DevCtl *dctl = nullptr;
    DevCtl *hctl = nullptr;  // pinned
    DevBuf<int32_t> ubuf;    // batched: union CSR scratch
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    uint32_t salt = 1;
    bool tables_dirty = false;  // a failed call may leave claims behind
    Policy policy;
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

void sync_ctl(scc_ctx *c) {
    HIPCHK(hipMemcpyAsync(c->hctl, c->dctl, sizeof(DevCtl), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
}

void reset_ctl(scc_ctx *c) {
    // a tiny fill keeps the reset inside the stream (no memset nodes)
    fill_u32(c, (uint32_t *)c->dctl, sizeof(DevCtl) / 4, 0u);
}

uint64_t next_pow2(uint64_t x) {
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

struct Opts {
    scc_options_t o;
};

scc_options_t defaults() {
    scc_options_t o;
    memset(&o, 0, sizeof o);
    o.tau = 512;
    o.beta = 1.5f;
    o.lambda_log2 = 10;
    o.sigma = 50;
    o.kappa = 8;
    o.alpha = 0.5f;
    o.seed = 0x5EEDull;
    o.policy = 0;
    o.dense = -1;
    o.validate = 1;
    o.trim = 1;
    o.table_init = 0;
    o.seeds_per_wave = 0;
    return o;
}

void check_opts(scc_ctx *c, const scc_options_t &o) {
    if (!(o.beta > 1.0f) || !(o.beta < 1e6f)) { set_err(c, "beta must be > 1"); throw Fail{SCC_EINVAL}; }
    if (o.lambda_log2 < kStripeLog2 || o.lambda_log2 > 24) {
        set_err(c, "lambda_log2 must be in [%d, 24]", kStripeLog2);
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
    if (o.policy != 0 && o.policy != 1) { set_err(c, "policy must be 0 or 1"); throw Fail{SCC_EINVAL}; }
}

// Hash bag sized for up to `entries` elements per round: capacity is the
// smallest lambda * 2^j >= 2 (entries + lambda) (reading of Section 3.3 with
// alpha = 1/2: the last chunk alone then holds every element).
void ensure_bag(scc_ctx *c, uint64_t entries, uint32_t lam_log2) {
    const uint64_t lam = 1ull << lam_log2;
    uint32_t nch = 1;
    while ((lam << (nch - 1)) < 2 * (entries + lam)) nch++;
    if (nch > (uint32_t)kMaxChunks) { set_err(c, "hash bag too large"); throw Fail{SCC_ENOMEM}; }
    const uint64_t cap = lam << (nch - 1);
    bool g1 = false, g2 = false;
    ensure(c, c->bag_slots, cap, &g1);
    ensure(c, c->bag_cnt, cap >> kStripeLog2, &g2);
    if (g2 || lam_log2 != c->bag_lam_log2 || nch > c->bag_nchunks) fill_u32(c, c->bag_cnt.p, c->bag_cnt.cap, 0u);
    c->bag_nchunks = nch;
    c->bag_lam_log2 = lam_log2;
    ensure(c, c->F, entries + kWave);
    ensure(c, c->heavy, entries + kWave);
}

Bag make_bag(scc_ctx *c, const scc_options_t &o) {
    Bag B;
    B.slots = c->bag_slots.p;
    B.cnt = c->bag_cnt.p;
    B.ctl = &c->dctl->bc;
    B.lam_log2 = c->bag_lam_log2;
    B.nchunks = c->bag_nchunks;
    B.sigma = (uint32_t)o.sigma;
    B.kappa = (uint32_t)o.kappa;
    B.alpha = o.alpha;
    B.salt = c->salt;
    return B;
}

// Clears a bag whose state may be inconsistent (after an aborted search).
void reset_bag(scc_ctx *c) {
    fill_u32(c, c->bag_cnt.p, c->bag_cnt.cap, 0u);
    fill_u32(c, (uint32_t *)&c->dctl->bc, sizeof(BagCtl) / 4, 0u);
}

struct Counters {
    unsigned long long expanded, arcs, attempts, claims, inserts;
};

Counters read_counters(const RoundCtl &r) { return {r.expanded, r.arcs, r.attempts, r.claims, r.inserts}; }

enum SearchResult { kDone = 0, kTableOverflow = 1 };

// Runs the frontier rounds of one search until the frontier is empty.  The
// search must already be seeded (frontier in F, nF[0] set).
// Every round expands entries claimed in the previous round, so a search has
// at most (claimable entries + 1) rounds; max_rounds guards the host loop.
template <int MODE>
SearchResult run_rounds(scc_ctx *c, Search S, int64_t *rounds, uint64_t max_rounds) {
    int par = 0;
    int K = 1;
    uint64_t launched = 0;
    const unsigned heavy_blocks = (unsigned)c->num_cu * 4;
    const unsigned extract_blocks = (unsigned)c->num_cu * 2;
    for (;;) {
        for (int i = 0; i < K; i++) {
            S.par = par;
            S.bag.salt = c->salt++;
            hipLaunchKernelGGL(k_expand<MODE>, dim3(c->expand_blocks), dim3(kBlock), 0, c->stream, S);
            LAUNCHCHK("k_expand");
            hipLaunchKernelGGL(k_expand_heavy<MODE>, dim3(heavy_blocks), dim3(kBlock), 0, c->stream, S);
            LAUNCHCHK("k_expand_heavy");
            hipLaunchKernelGGL(k_bag_extract, dim3(extract_blocks), dim3(kBlock), 0, c->stream, S.bag, S.F, S.fcap,
                               S.rc, par);
            LAUNCHCHK("k_bag_extract");
            par ^= 1;
        }
        launched += (uint64_t)K;
        sync_ctl(c);
        const RoundCtl &r = c->hctl->rc;
        if (r.err & kErrTable) return kTableOverflow;
        if ((r.err & kErrCapacity) || c->hctl->bc.overflow) {
            set_err(c, "frontier capacity exceeded (err=%u, bag overflow=%u)", r.err, c->hctl->bc.overflow);
            throw Fail{SCC_EINTERNAL};
        }
        if (r.nF[0] + r.nF[1] == 0) break;
        if (launched > max_rounds + 64) {
            set_err(c, "internal: search did not finish after %llu rounds", (unsigned long long)launched);
            throw Fail{SCC_EINTERNAL};
        }
        K = std::min(K * 2, 64);
    }
    if (rounds) *rounds = c->hctl->rc.rounds;
    return kDone;
}

struct GraphDev {
    int32_t n, m;
    const int32_t *out_off, *out_adj, *in_off, *in_adj;
};

void validate_graph(scc_ctx *c, const GraphDev &g);

struct PhaseClock {
    scc_ctx *c;
    std::chrono::steady_clock::time_point t0;
    explicit PhaseClock(scc_ctx *cc) : c(cc) {
        (void)hipStreamSynchronize(c->stream);
        t0 = std::chrono::steady_clock::now();
    }
    double lap() {
        HIPCHK(hipStreamSynchronize(c->stream));
        auto t1 = std::chrono::steady_clock::now();
        double ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        t0 = t1;
        return ms;
    }
};

Search base_search(scc_ctx *c, const scc_options_t &o, int tau) {
    Search S;
    memset(&S, 0, sizeof S);
    S.F = c->F.p;
    S.heavy = c->heavy.p;
    S.fcap = std::min(c->F.cap, c->heavy.cap);
    S.bag = make_bag(c, o);
    S.rc = &c->dctl->rc;
    S.tau = tau;
    S.seeds = o.seeds_per_wave;
    S.heavy_deg = 1024;
    S.probe_limit = 128;
    return S;
}

void add_counters(scc_stats_t *st, const RoundCtl &r) {
    if (!st) return;
    st->entries_expanded = (int64_t)r.expanded;
    st->arcs_scanned = (int64_t)r.arcs;
    st->claim_attempts = (int64_t)r.attempts;
    st->claims = (int64_t)r.claims;
    st->bag_inserts = (int64_t)r.inserts;
}

// Single-source search from s inside subproblem L (labels), direction dir.
int64_t single_search(scc_ctx *c, const scc_options_t &o, const GraphDev &g, const int32_t *labels, int dir, int32_t L,
                      int32_t s, uint32_t *vis, int tau) {
    const int32_t n = g.n;
    hipLaunchKernelGGL(k_premark, dim3(grid_for(c, (uint64_t)n)), dim3(kBlock), 0, c->stream, n, labels, L, s, vis);
    LAUNCHCHK("k_premark");
    hipLaunchKernelGGL(k_seed_single, dim3(1), dim3(64), 0, c->stream, s, c->F.p, &c->dctl->rc);
    LAUNCHCHK("k_seed_single");
    Search S = base_search(c, o, tau);
    S.off = dir ? g.in_off : g.out_off;
    S.adj = dir ? g.in_adj : g.out_adj;
    S.label = labels;
    S.vis = vis;
    int64_t rounds = 0;
    run_rounds<kSingle>(c, S, &rounds, (uint64_t)n + 1);
    return rounds;
}

// Multi-source search of the k sources in srcvert/srclab (rc.k set) into the
// table T (all EMPTY on entry).  Grows the table and restarts on overflow.
int64_t multi_search(scc_ctx *c, const scc_options_t &o, const GraphDev &g, const int32_t *labels, int dir,
                     DevBuf<uint64_t> &T, uint64_t &tslots, int tau, scc_stats_t *st, double *resize_ms) {
    for (;;) {
        hipLaunchKernelGGL(k_seed_multi, dim3(grid_for(c, c->hctl->rc.k)), dim3(kBlock), 0, c->stream, c->srcvert.p,
                           T.p, tslots - 1, 128u, c->F.p, &c->dctl->rc);
        LAUNCHCHK("k_seed_multi");
        Search S = base_search(c, o, tau);
        S.off = dir ? g.in_off : g.out_off;
        S.adj = dir ? g.in_adj : g.out_adj;
        S.label = labels;
        S.table = T.p;
        S.tmask = tslots - 1;
        S.srclab = c->srclab.p;
        int64_t rounds = 0;
        if (run_rounds<kMulti>(c, S, &rounds, tslots + 1) == kDone) return rounds;
        // Section 4.5: resize once an insertion probes too often.  The table
        // cannot grow while claims are in flight, so the search restarts on a
        // table twice as large.
        auto t0 = std::chrono::steady_clock::now();
        tslots *= 2;
        bool grew = false;
        ensure(c, T, tslots, &grew);
        fill_u64(c, T.p, grew ? T.cap : tslots, kEmpty64);
        ensure_bag(c, tslots, c->bag_lam_log2);
        reset_bag(c);
        // clear the error bit, keep the counters
        fill_u32(c, &c->dctl->rc.err, 1, 0u);
        HIPCHK(hipStreamSynchronize(c->stream));
        if (st) st->table_restarts++;
        if (resize_ms) *resize_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
}

void init_call(scc_ctx *c, scc_stats_t *st, int64_t n, int64_t m) {
    HIPCHK(hipSetDevice(c->device));
    c->err.clear();
    if (st) {
        memset(st, 0, sizeof *st);
        st->n = n;
        st->m = m;
    }
    if (!c->dctl) {
        HIPCHK(hipMalloc((void **)&c->dctl, sizeof(DevCtl)));
        HIPCHK(hipHostMalloc((void **)&c->hctl, sizeof(DevCtl), hipHostMallocDefault));
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
    bool g1, g2, g3;
    ensure(c, c->label, (uint64_t)n);
    ensure(c, c->aux, (uint64_t)n);
    ensure(c, c->stamp, (uint64_t)n, &g1);
    ensure(c, c->fin, (uint64_t)n, &g2);
    ensure(c, c->srcvert, (uint64_t)n);
    ensure(c, c->srclab, (uint64_t)n);
    ensure(c, c->sig_out, (uint64_t)n, &g3);
    ensure(c, c->sig_in, (uint64_t)n);
    ensure(c, c->visF, (uint64_t)n / 32 + 2);
    ensure(c, c->visB, (uint64_t)n / 32 + 2);
    (void)g1;
    (void)g2;
    (void)g3;
}

void fill_algbytes(scc_stats_t *st, int64_t n) {
    if (!st) return;
    // Algorithmic bytes: offsets per expanded entry (8), target id per scanned
    // arc (4), target label / visited word per claim attempt (4), table or
    // bitmap update per claim (8), bag insert + ExtractAll read + frontier
    // write + frontier read (32 per inserted entry), trim (12 n), canonical
    // labels (16 n).
    st->bytes_alg = st->entries_expanded * 8 + st->arcs_scanned * 4 + st->claim_attempts * 4 + st->claims * 8 +
                    st->bag_inserts * 32 + 28 * n;
}

void run_scc(scc_ctx *c, const GraphDev &g, int32_t *labels_out, const scc_options_t &o, scc_stats_t *st) {
    const int32_t n = g.n;
    PhaseClock clk(c);
    if (n == 0) {
        if (st) st->ms_total = 0;
        return;
    }
    ensure_vertex_state(c, n);
    if (o.validate) validate_graph(c, g);
    const int tau = o.tau;
    // per-call state
    fill_u32(c, (uint32_t *)c->stamp.p, (uint64_t)n, 0u);
    fill_u32(c, (uint32_t *)c->fin.p, (uint64_t)n, (uint32_t)kInf32);
    fill_u64(c, (uint64_t *)c->sig_out.p, (uint64_t)n, 0ull);
    fill_u64(c, (uint64_t *)c->sig_in.p, (uint64_t)n, 0ull);
    ensure_bag(c, (uint64_t)n, (uint32_t)o.lambda_log2);
    reset_bag(c);
    if (st) st->ms_label += clk.lap();

    // ---- trimming (Section 4.1)
    hipLaunchKernelGGL(k_trim, dim3(grid_for(c, (uint64_t)n)), dim3(kBlock), 0, c->stream, n, g.out_off, g.in_off,
                       c->label.p, o.trim ? 1 : 0, &c->dctl->rc);
    LAUNCHCHK("k_trim");
    // ---- random permutation (Algorithm 1) and batch 1
    Perm P;
    P.n = (uint32_t)n;
    uint32_t bits = 1;
    while ((1ull << (2 * bits)) < (uint64_t)n) bits++;
    P.half_bits = bits;
    P.key = mix64(o.seed ^ 0x243F6A8885A308D3ull);
    fill_u32(c, &c->dctl->rc.first, 1, 0xffffffffu);
    hipLaunchKernelGGL(k_first_active, dim3(grid_for(c, (uint64_t)n)), dim3(kBlock), 0, c->stream, P, c->label.p,
                       &c->dctl->rc);
    LAUNCHCHK("k_first_active");
    sync_ctl(c);
    int64_t active = (int64_t)n - (int64_t)c->hctl->rc.trimmed;
    if (st) {
        st->trimmed = c->hctl->rc.trimmed;
        st->ms_trim += clk.lap();
    }
    uint64_t pos = n;
    if (active > 0) {
        const uint32_t j1 = c->hctl->rc.first;
        if (j1 >= (uint32_t)n) { set_err(c, "no active vertex found"); throw Fail{SCC_EINTERNAL}; }
        const int32_t s0 = (int32_t)perm_apply(P, j1);
        // first SCC: single-source searches forward and backward (Section 4.2)
        int64_t r1 = single_search(c, o, g, c->label.p, 0, 0, s0, c->visF.p, tau);
        int64_t r2 = single_search(c, o, g, c->label.p, 1, 0, s0, c->visB.p, tau);
        fill_u32(c, &c->dctl->rc.fin, 1, 0u);
        if (st) {
            st->rounds_first = r1 + r2;
            st->batches = 1;
            st->ms_first += clk.lap();
        }
        hipLaunchKernelGGL(k_finish_single, dim3(grid_for(c, (uint64_t)n)), dim3(kBlock), 0, c->stream, n, c->label.p, 0,
                           s0, c->visF.p, c->visB.p, &c->dctl->rc);
        LAUNCHCHK("k_finish_single");
        sync_ctl(c);
        active -= c->hctl->rc.fin;
        if (st) st->ms_label += clk.lap();
        pos = (uint64_t)j1 + 1;
    }
    // ---- multi-source batches (Algorithm 1, prefix doubling with beta)
    double bsize = 1.0;
    int32_t epoch = 1;
    uint64_t a_out = 0, a_in = 0;
    uint64_t ts_out = 0, ts_in = 0;
    while (active > 0 && pos < (uint64_t)n) {
        bsize *= (double)o.beta;
        uint64_t sz = (uint64_t)std::ceil(bsize - 1e-9);
        uint64_t p1 = std::min<uint64_t>((uint64_t)n, pos + std::max<uint64_t>(sz, 1));
        fill_u32(c, &c->dctl->rc.k, 1, 0u);
        hipLaunchKernelGGL(k_select_sources, dim3(grid_for(c, p1 - pos)), dim3(kBlock), 0, c->stream, P, (uint32_t)pos,
                           (uint32_t)p1, c->label.p, c->srcvert.p, c->srclab.p, &c->dctl->rc);
        LAUNCHCHK("k_select_sources");
        sync_ctl(c);
        pos = p1;
        const uint32_t k = c->hctl->rc.k;
        if (k == 0) continue;
        // Section 4.5: next table size = nextpow2(max(0.3 b, 1.5 a)), b = |V'|,
        // a = pairs found by the previous search in the same direction.
        auto size_for = [&](uint64_t a) {
            uint64_t want = (uint64_t)std::max(0.3 * (double)active, 1.5 * (double)a);
            want = std::max<uint64_t>(want, 2ull * k);
            want = std::max<uint64_t>(want, 1024);
            if (o.table_init > 0 && epoch == 1) want = (uint64_t)o.table_init;
            return next_pow2(want);
        };
        auto t_rs = std::chrono::steady_clock::now();
        uint64_t want_out = size_for(a_out), want_in = size_for(a_in);
        bool grew = false;
        ts_out = want_out;
        ensure(c, c->Tout, ts_out, &grew);
        if (grew) fill_u64(c, c->Tout.p, c->Tout.cap, kEmpty64);
        ts_in = want_in;
        ensure(c, c->Tin, ts_in, &grew);
        if (grew) fill_u64(c, c->Tin.p, c->Tin.cap, kEmpty64);
        c->tables_dirty = true;
        ensure_bag(c, std::max<uint64_t>(std::max(ts_out, ts_in), (uint64_t)n), c->bag_lam_log2);
        if (st) st->ms_resize += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_rs).count();
        (void)clk.lap();
        const RoundCtl before = c->hctl->rc;
        double rs = 0;
        int64_t r1 = multi_search(c, o, g, c->label.p, 0, c->Tout, ts_out, tau, st, &rs);
        const uint64_t claims_mid = c->hctl->rc.claims;
        int64_t r2 = multi_search(c, o, g, c->label.p, 1, c->Tin, ts_in, tau, st, &rs);
        a_out = claims_mid - before.claims + k;
        a_in = c->hctl->rc.claims - claims_mid + k;
        if (st) {
            st->rounds_multi += r1 + r2;
            st->batches += 1;
            st->ms_multi += clk.lap() - rs;
            st->ms_resize += rs;
        }
        fill_u32(c, &c->dctl->rc.fin, 1, 0u);
        const uint64_t tot = ts_out + ts_in;
        hipLaunchKernelGGL(k_accumulate, dim3(grid_for(c, tot)), dim3(kBlock), 0, c->stream, c->Tout.p, ts_out - 1,
                           c->Tin.p, ts_in - 1, 128u, c->srcvert.p, c->sig_out.p, c->sig_in.p, c->fin.p);
        LAUNCHCHK("k_accumulate");
        hipLaunchKernelGGL(k_relabel_multi, dim3(grid_for(c, tot)), dim3(kBlock), 0, c->stream, c->Tout.p, ts_out - 1,
                           c->Tin.p, ts_in - 1, c->srcvert.p, c->sig_out.p, c->sig_in.p, c->fin.p, c->stamp.p, epoch,
                           c->label.p, &c->dctl->rc);
        LAUNCHCHK("k_relabel_multi");
        epoch++;
        sync_ctl(c);
        active -= c->hctl->rc.fin;
        if (st) st->ms_label += clk.lap();
    }
    if (active != 0) {
        set_err(c, "internal: %lld vertices left unfinished", (long long)active);
        throw Fail{SCC_EINTERNAL};
    }
    // ---- canonical labels: min vertex id per SCC
    fill_u32(c, (uint32_t *)c->aux.p, (uint64_t)n, (uint32_t)kInf32);
    hipLaunchKernelGGL(k_canon_min, dim3(grid_for(c, (uint64_t)n)), dim3(kBlock), 0, c->stream, n, c->label.p, c->aux.p,
                       &c->dctl->rc);
    LAUNCHCHK("k_canon_min");
    hipLaunchKernelGGL(k_canon_write, dim3(grid_for(c, (uint64_t)n)), dim3(kBlock), 0, c->stream, n, c->label.p,
                       c->aux.p, labels_out, &c->dctl->rc);
    LAUNCHCHK("k_canon_write");
    sync_ctl(c);
    if (c->hctl->rc.err & kErrUnfinished) {
        set_err(c, "internal: a vertex ended without an SCC key");
        throw Fail{SCC_EINTERNAL};
    }
    if (st) {
        st->ms_label += clk.lap();
        st->n_scc = c->hctl->rc.nscc;
        add_counters(st, c->hctl->rc);
        st->ms_total = st->ms_trim + st->ms_first + st->ms_multi + st->ms_resize + st->ms_label;
        fill_algbytes(st, n);
    }
    c->tables_dirty = false;
}

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
    uint32_t *bad = &c->dctl->rc.pad[0];
    fill_u32(c, bad, 1, 0u);
    hipLaunchKernelGGL(k_validate_off, dim3(grid_for(c, (uint64_t)g.n + 1)), dim3(kBlock), 0, c->stream, g.n, g.m,
                       g.out_off, bad);
    hipLaunchKernelGGL(k_validate_off, dim3(grid_for(c, (uint64_t)g.n + 1)), dim3(kBlock), 0, c->stream, g.n, g.m,
                       g.in_off, bad);
    LAUNCHCHK("k_validate_off");
    sync_ctl(c);
    if (c->hctl->rc.pad[0]) {
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
    if (c->hctl->rc.pad[0]) {
        set_err(c, "arc target out of range [0, n)");
        throw Fail{SCC_EGRAPH};
    }
    hipLaunchKernelGGL(k_validate_hist, dim3(grid_for(c, (uint64_t)g.n)), dim3(kBlock), 0, c->stream, g.n, g.in_off,
                       c->aux.p, bad);
    LAUNCHCHK("k_validate_hist");
    sync_ctl(c);
    if (c->hctl->rc.pad[0]) {
        set_err(c, "in-CSR is not the transpose of the out-CSR (in-degree mismatch)");
        throw Fail{SCC_EGRAPH};
    }
    c->hctl->rc.pad[0] = 0;
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

// Union CSR of a batch of graphs: global id = vtx_base[g] + local id.
__global__ void k_union_off(int32_t G, const int64_t *vb, const int64_t *ab, const int32_t *off_in, int32_t *off_out,
                            int64_t arc0, int32_t g0) {
    // one thread per global vertex of the group, plus the end offset
    const int64_t v0 = vb[g0];
    const int64_t nv = vb[g0 + G] - v0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= nv; i += (int64_t)gridDim.x * blockDim.x) {
        if (i == nv) {
            off_out[i] = (int32_t)(ab[g0 + G] - arc0);
            continue;
        }
        // graph of vertex i: binary search in vb
        int lo = g0, hi = g0 + G - 1;
        const int64_t gv = v0 + i;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (vb[mid] <= gv) lo = mid; else hi = mid - 1;
        }
        const int64_t local = gv - vb[lo];
        off_out[i] = (int32_t)(ab[lo] - arc0 + off_in[vb[lo] + lo + local]);
    }
}
__global__ void k_union_adj(int32_t G, const int64_t *vb, const int64_t *ab, const int32_t *adj_in, int32_t *adj_out,
                            int32_t g0) {
    const int64_t a0 = ab[g0];
    const int64_t na = ab[g0 + G] - a0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < na; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t ge = a0 + e;
        int lo = g0, hi = g0 + G - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (ab[mid] <= ge) lo = mid; else hi = mid - 1;
        }
        adj_out[e] = (int32_t)(vb[lo] - vb[g0] + adj_in[ge]);
    }
}
__global__ void k_union_labels(int32_t G, const int64_t *vb, const int32_t *lab_in, int32_t *lab_out, int32_t g0) {
    const int64_t v0 = vb[g0];
    const int64_t nv = vb[g0 + G] - v0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x) {
        int lo = g0, hi = g0 + G - 1;
        const int64_t gv = v0 + i;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (vb[mid] <= gv) lo = mid; else hi = mid - 1;
        }
        lab_out[gv] = (int32_t)(lab_in[i] + v0 - vb[lo]);
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

}  // namespace

extern "C" {

const char *scc_version(void) { return "hipscc 0.1 (gfx950)"; }

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
        int nb = 0;
        HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_expand<kMulti>, kBlock, 0));
        if (nb < 1) nb = 1;
        c->expand_blocks = c->num_cu * nb;
        if (stream) {
            c->stream = (hipStream_t)stream;
        } else {
            HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
            c->own_stream = true;
        }
        HIPCHK(hipMalloc((void **)&c->dctl, sizeof(DevCtl)));
        HIPCHK(hipHostMalloc((void **)&c->hctl, sizeof(DevCtl), hipHostMallocDefault));
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

void scc_destroy(scc_ctx_t *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    release(c->label); release(c->aux); release(c->stamp); release(c->srcvert); release(c->srclab);
    release(c->fin); release(c->sig_out); release(c->sig_in); release(c->visF); release(c->visB);
    release(c->Tout); release(c->Tin); release(c->F); release(c->heavy); release(c->bag_slots);
    release(c->bag_cnt); release(c->ubuf);
    policy_release(c->policy);
    if (c->dctl) (void)hipFree(c->dctl);
    if (c->hctl) (void)hipHostFree(c->hctl);
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
        init_call(c, stats, g->n, g->m);
        GraphDev gd{g->n, g->m, g->out_off, g->out_adj, g->in_off, g->in_adj};
        run_scc(c, gd, labels_out, o, stats);
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
        init_call(c, stats, g->n, g->m);
        if (k == 0) return;
        if (k > g->n) { set_err(c, "more sources than vertices"); throw Fail{SCC_EINVAL}; }
        GraphDev gd{g->n, g->m, g->out_off, g->out_adj, g->in_off, g->in_adj};
        ensure_vertex_state(c, g->n);
        if (o.validate) validate_graph(c, gd);
        PhaseClock clk(c);
        fill_u32(c, (uint32_t *)c->stamp.p, (uint64_t)g->n, 0u);
        uint32_t *bad = &c->dctl->rc.pad[1];
        fill_u32(c, bad, 1, 0u);
        hipLaunchKernelGGL(k_check_sources, dim3(grid_for(c, (uint64_t)k)), dim3(kBlock), 0, c->stream, g->n, k, sources,
                           labels, c->srcvert.p, c->srclab.p, c->stamp.p, 1, bad);
        LAUNCHCHK("k_check_sources");
        fill_u32(c, &c->dctl->rc.k, 1, (uint32_t)k);
        sync_ctl(c);
        if (c->hctl->rc.pad[1]) {
            set_err(c, "sources must be in range, distinct and not excluded (label >= 0); code %u", c->hctl->rc.pad[1]);
            throw Fail{SCC_EINVAL};
        }
        int64_t rounds = 0;
        if (k == 1) {
            int32_t s = 0, L = 0;
            HIPCHK(hipMemcpyAsync(&s, sources, 4, hipMemcpyDeviceToHost, c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
            HIPCHK(hipMemcpyAsync(&L, labels + s, 4, hipMemcpyDeviceToHost, c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
            ensure_bag(c, (uint64_t)g->n, (uint32_t)o.lambda_log2);
            reset_bag(c);
            rounds = single_search(c, o, gd, labels, dir, L, s, c->visF.p, o.tau);
            fill_u32(c, &c->dctl->rc.emit, 1, 0u);
            hipLaunchKernelGGL(k_emit_single, dim3(grid_for(c, (uint64_t)g->n)), dim3(kBlock), 0, c->stream, g->n, labels,
                               L, c->visF.p, s, pairs_out, (uint64_t)capacity, &c->dctl->rc);
            LAUNCHCHK("k_emit_single");
        } else {
            uint64_t ts = next_pow2(std::max<uint64_t>(std::max<uint64_t>(1024, 4ull * (uint64_t)k),
                                                       o.table_init > 0 ? (uint64_t)o.table_init : (uint64_t)g->n / 4));
            bool grew = false;
            ensure(c, c->Tout, ts, &grew);
            fill_u64(c, c->Tout.p, grew ? c->Tout.cap : ts, kEmpty64);
            c->tables_dirty = true;
            ensure_bag(c, std::max<uint64_t>(ts, (uint64_t)g->n), (uint32_t)o.lambda_log2);
            reset_bag(c);
            double rs = 0;
            rounds = multi_search(c, o, gd, labels, dir, c->Tout, ts, o.tau, stats, &rs);
            fill_u32(c, &c->dctl->rc.emit, 1, 0u);
            hipLaunchKernelGGL(k_emit_table, dim3(grid_for(c, ts)), dim3(kBlock), 0, c->stream, c->Tout.p, ts - 1,
                               pairs_out, (uint64_t)capacity, &c->dctl->rc);
            LAUNCHCHK("k_emit_table");
            // leave the table clean for the next call
            fill_u64(c, c->Tout.p, ts, kEmpty64);
            c->tables_dirty = false;
        }
        sync_ctl(c);
        *n_pairs = (int64_t)c->hctl->rc.emit;
        if (stats) {
            stats->ms_total = clk.lap();
            if (k == 1) stats->rounds_first = rounds; else stats->rounds_multi = rounds;
            add_counters(stats, c->hctl->rc);
            fill_algbytes(stats, 0);
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
        init_call(c, stats, G ? vtx_base[G] : 0, G ? arc_base[G] : 0);
        if (G == 0) return;
        for (int32_t i = 0; i < G; i++) {
            if (vtx_base[i + 1] < vtx_base[i] || arc_base[i + 1] < arc_base[i] || vtx_base[0] != 0 || arc_base[0] != 0) {
                set_err(c, "vtx_base/arc_base must start at 0 and never decrease");
                throw Fail{SCC_EINVAL};
            }
            if (arc_base[i + 1] - arc_base[i] >= (1ll << 31)) { set_err(c, "graph %d has >= 2^31 arcs", i); throw Fail{SCC_EINVAL}; }
        }
        if (vtx_base[G] >= (1ll << 31)) { set_err(c, "total vertex count must be < 2^31"); throw Fail{SCC_EINVAL}; }
        if (arc_base[G] > 0 && (!out_adj || !in_adj)) { set_err(c, "adjacency NULL"); throw Fail{SCC_EINVAL}; }
        // device copies of the bases
        DevBuf<int64_t> dvb, dab;
        struct Free {
            DevBuf<int64_t> &a, &b;
            ~Free() { release(a); release(b); }
        } fr{dvb, dab};
        ensure(c, dvb, (uint64_t)G + 1);
        ensure(c, dab, (uint64_t)G + 1);
        HIPCHK(hipMemcpyAsync(dvb.p, vtx_base, 8 * ((size_t)G + 1), hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(dab.p, arc_base, 8 * ((size_t)G + 1), hipMemcpyHostToDevice, c->stream));
        // groups of consecutive graphs whose union has < 2^31 arcs
        scc_stats_t acc;
        memset(&acc, 0, sizeof acc);
        int32_t g0 = 0;
        const int64_t lim = (1ll << 31) - 1;
        while (g0 < G) {
            int32_t g1 = g0 + 1;
            while (g1 < G && arc_base[g1 + 1] - arc_base[g0] < lim) g1++;
            const int32_t cnt = g1 - g0;
            const int64_t nv = vtx_base[g1] - vtx_base[g0];
            const int64_t na = arc_base[g1] - arc_base[g0];
            // union CSR scratch: 2 (nv + 1) offsets + 2 na arcs + nv labels
            const uint64_t need = 2 * ((uint64_t)nv + 1) + 2 * (uint64_t)na + (uint64_t)nv;
            ensure(c, c->ubuf, need);
            int32_t *uo = c->ubuf.p, *ui = uo + nv + 1, *ua = ui + nv + 1, *uia = ua + na, *ul = uia + na;
            const unsigned gv = grid_for(c, (uint64_t)nv + 1), ga = grid_for(c, (uint64_t)std::max<int64_t>(na, 1));
            hipLaunchKernelGGL(k_union_off, dim3(gv), dim3(kBlock), 0, c->stream, cnt, dvb.p, dab.p, out_off, uo,
                               arc_base[g0], g0);
            hipLaunchKernelGGL(k_union_off, dim3(gv), dim3(kBlock), 0, c->stream, cnt, dvb.p, dab.p, in_off, ui,
                               arc_base[g0], g0);
            if (na > 0) {
                hipLaunchKernelGGL(k_union_adj, dim3(ga), dim3(kBlock), 0, c->stream, cnt, dvb.p, dab.p, out_adj, ua, g0);
                hipLaunchKernelGGL(k_union_adj, dim3(ga), dim3(kBlock), 0, c->stream, cnt, dvb.p, dab.p, in_adj, uia, g0);
            }
            LAUNCHCHK("k_union_*");
            GraphDev gd{(int32_t)nv, (int32_t)na, uo, ua, ui, uia};
            scc_stats_t st;
            memset(&st, 0, sizeof st);
            reset_ctl(c);
            run_scc(c, gd, ul, o, stats ? &st : nullptr);
            hipLaunchKernelGGL(k_union_labels, dim3(grid_for(c, (uint64_t)nv)), dim3(kBlock), 0, c->stream, cnt, dvb.p, ul,
                               labels_out, g0);
            LAUNCHCHK("k_union_labels");
            HIPCHK(hipStreamSynchronize(c->stream));
            if (stats) {
                acc.ms_total += st.ms_total; acc.ms_trim += st.ms_trim; acc.ms_first += st.ms_first;
                acc.ms_multi += st.ms_multi; acc.ms_resize += st.ms_resize; acc.ms_label += st.ms_label;
                acc.batches += st.batches; acc.rounds_first += st.rounds_first; acc.rounds_multi += st.rounds_multi;
                acc.dense_rounds += st.dense_rounds; acc.entries_expanded += st.entries_expanded;
                acc.arcs_scanned += st.arcs_scanned; acc.claim_attempts += st.claim_attempts; acc.claims += st.claims;
                acc.bag_inserts += st.bag_inserts; acc.bag_chunk_advances += st.bag_chunk_advances;
                acc.table_restarts += st.table_restarts; acc.trimmed += st.trimmed; acc.n_scc += st.n_scc;
                acc.policy_calls += st.policy_calls; acc.policy_fallbacks += st.policy_fallbacks;
                acc.bytes_alg += st.bytes_alg;
            }
            g0 = g1;
        }
        if (stats) {
            acc.n = vtx_base[G];
            acc.m = arc_base[G];
            *stats = acc;
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
        init_call(c, stats, n, 0);
        const uint64_t per_round = (uint64_t)((n + rounds - 1) / rounds);
        ensure_bag(c, std::max<uint64_t>(per_round, 1), (uint32_t)o.lambda_log2);
        ensure(c, c->F, (uint64_t)n + kWave);
        reset_bag(c);
        Bag B = make_bag(c, o);
        uint64_t adv = 0;
        for (int32_t rr = 0; rr < rounds; rr++) {
            B.salt = c->salt++;
            hipLaunchKernelGGL(k_bag_insert_test, dim3((unsigned)c->num_cu * 4), dim3(kBlock), 0, c->stream, keys, n,
                               rounds, rr, B, &c->dctl->rc);
            LAUNCHCHK("k_bag_insert_test");
            sync_ctl(c);
            adv += c->hctl->bc.advances;
            if (c->hctl->bc.overflow) { set_err(c, "bag overflow"); throw Fail{SCC_EINTERNAL}; }
            // par = 1: ExtractAll appends to nF[0], which accumulates over rounds
            hipLaunchKernelGGL(k_bag_extract, dim3((unsigned)c->num_cu * 2), dim3(kBlock), 0, c->stream, B, c->F.p,
                               (uint64_t)c->F.cap, &c->dctl->rc, 1);
            LAUNCHCHK("k_bag_extract");
            fill_u32(c, &c->dctl->bc.advances, 1, 0u);
        }
        sync_ctl(c);
        const uint64_t got = c->hctl->rc.nF[0];
        if (got > 0) HIPCHK(hipMemcpyAsync(out, c->F.p, 8 * std::min<uint64_t>(got, (uint64_t)n), hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        *n_out = (int64_t)got;
        if (stats) {
            stats->bag_inserts = (int64_t)c->hctl->rc.inserts;
            stats->bag_chunk_advances = (int64_t)adv;
        }
    });
}

}  // extern "C"
