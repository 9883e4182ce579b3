// Parallel hash bag (Section 3.3, Figure 5 / Figure 6), wavefront edition.
//
// The bag is a preallocated array split into chunks of doubling size: chunk 0
// holds [0, lambda), chunk i >= 1 holds [lambda * 2^(i-1), lambda * 2^i).  The
// current chunk r only grows.  Inserts land in chunk r; a sampled estimate of
// its load moves r forward (Section 3.3: each insert is sampled with
// probability sigma / (alpha * chunk size); when a chunk has collected sigma
// samples, a CAS advances r).  ExtractAll packs the used prefix [0, tail[r])
// and clears it, so its cost is proportional to the bag's content plus lambda
// (Theorem 1).
//
// GPU form.  The paper's insert CASes a random slot and probes linearly.  Here
// a wavefront inserts its elements together: each chunk is cut into stripes
// of kStripe slots with one fill counter each; the wave picks a random stripe
// of chunk r and reserves room for all its elements with one fetch-and-add on
// that counter, spilling the remainder to another random stripe (the probe).
// After kappa probes the insert forces a chunk advance, as the paper's probe
// limit does.  A stripe's valid slots are exactly [0, min(count, kStripe)), so
// ExtractAll reads counters instead of scanning for empty slots, and clearing
// resets counters only.  Random stripe choice spreads the atomics over many
// addresses; sampling keeps the chunk advance off the common path.
#pragma once

#include "device.h"

namespace hipscc {

constexpr int kStripeLog2 = 6;
constexpr int kStripe = 1 << kStripeLog2;
constexpr int kMaxChunks = 40;

// Control words of one bag, in device memory.
struct BagCtl {
    uint32_t r;                    // current chunk
    uint32_t done_blocks;          // ExtractAll's last-block ticket
    uint32_t overflow;             // set when the last chunk is full
    uint32_t advances;             // chunk advances (statistics)
    uint32_t sample[kMaxChunks];   // samples taken per chunk
    // statistics of the bag self test (Bag::track): slots filled per chunk,
    // counted by ExtractAll, and the chunk that was current when it ran
    uint32_t fill[kMaxChunks];
    uint32_t last_r;
    uint64_t forced;               // bit i: chunk i was left by the probe limit, not by samples
};

struct Bag {
    uint64_t *slots;     // capacity = lambda << (nchunks - 1) entries
    uint32_t *cnt;       // one fill counter per stripe
    BagCtl *ctl;
    uint32_t lam_log2;   // log2(lambda), lambda >= kStripe
    uint32_t nchunks;
    uint32_t sigma;
    uint32_t kappa;
    float alpha;
    uint32_t salt;       // varies per round: decorrelates stripe choice and sampling
    uint32_t track;      // 1: ExtractAll also counts the filled slots of each chunk (self test)
};

// Chunk that holds stripe st (stripe st covers slots [64 st, 64 st + 64)).
__host__ __device__ __forceinline__ uint32_t bag_chunk_of_stripe(const Bag &B, uint64_t st) {
    const uint64_t q = (st << kStripeLog2) >> B.lam_log2;
    return q == 0 ? 0u : 64u - (uint32_t)__builtin_clzll(q);
}

__host__ __device__ __forceinline__ uint64_t bag_chunk_lo(const Bag &B, uint32_t i) {
    return i == 0 ? 0ull : (1ull << (B.lam_log2 + i - 1));
}
__host__ __device__ __forceinline__ uint64_t bag_chunk_hi(const Bag &B, uint32_t i) {
    return 1ull << (B.lam_log2 + i);
}

// Wave-cooperative Insert of up to A elements per lane.  Every lane of the
// wave must call it (uniform control flow); element j of a lane is present
// when has[j].  The wave's elements are ranked (slot j, then lane) and
// reserved together: one fetch-and-add on a random stripe of chunk r claims
// room for all of them, the remainder spills to the next stripe (the probe).
// `wseq` is a per-wave sequence number (wave-uniform) used to draw the stripe.
// Returns the number of this lane's elements that were inserted.
template <int A>
__device__ __forceinline__ int bag_insert_wave_n(const Bag &B, const bool (&has)[A], const uint64_t (&e)[A],
                                                 uint32_t wave_gid, uint32_t &wseq) {
    bool pending[A];
    int inserted = 0;
#pragma unroll
    for (int j = 0; j < A; j++) {
        pending[j] = has[j];
        inserted += has[j] ? 1 : 0;
    }
    for (;;) {
        // rank of each pending element in (slot, lane) order
        int my[A];
        int k = 0;
#pragma unroll
        for (int j = 0; j < A; j++) {
            const uint64_t m = ballot(pending[j]);
            my[j] = k + rank_below(m);
            k += popc64(m);
        }
        if (k == 0) break;
        uint32_t r = ld_relaxed(&B.ctl->r);
        if (r >= B.nchunks) r = B.nchunks - 1;
        const bool last = (r + 1 >= B.nchunks);
        const uint64_t lo = bag_chunk_lo(B, r), hi = bag_chunk_hi(B, r);
        const uint64_t size = hi - lo;
        // Sampling (Section 3.3): rate sigma / (alpha * size).
        bool advanced = false;
        if (!last) {
            const double rate = (double)B.sigma / ((double)B.alpha * (double)size);
            const uint32_t thr = rate >= 1.0 ? 0xffffffffu : (uint32_t)(rate * 4294967296.0);
            int ns = 0;
#pragma unroll
            for (int j = 0; j < A; j++) {
                const uint32_t coin = (uint32_t)mix64(e[j] ^ ((uint64_t)B.salt << 32) ^ 0x5851F42D4C957F2Dull);
                ns += popc64(ballot(pending[j] && coin < thr));
            }
            if (ns > 0) {
                uint32_t adv = 0;
                if (lane_id() == 0) {
                    const uint32_t old = atomicAdd(&B.ctl->sample[r], (uint32_t)ns);
                    if (old + (uint32_t)ns >= B.sigma) {
                        // try_resize: only one CAS from r wins
                        if (atomicCAS(&B.ctl->r, r, r + 1) == r) atomicAdd(&B.ctl->advances, 1u);
                        adv = 1;
                    }
                }
                advanced = wave_bcast_u(adv, 0) != 0;
            }
        }
        if (advanced) continue;  // insert again into the new chunk
        const uint32_t nst = (uint32_t)(size >> kStripeLog2);
        const uint32_t st0 = (uint32_t)(lo >> kStripeLog2);
        uint32_t st = (uint32_t)(mix64(((uint64_t)wave_gid << 32) ^ (uint64_t)(wseq++) ^ ((uint64_t)B.salt << 20)) % nst);
        int placed = 0;
        uint32_t probes = 0;
        bool spill = false, lost = false;
        while (placed < k) {
            uint32_t o = 0;
            if (lane_id() == 0) o = atomicAdd(&B.cnt[st0 + st], (uint32_t)(k - placed));
            o = wave_bcast_u(o, 0);
            int avail = o < (uint32_t)kStripe ? (int)((uint32_t)kStripe - o) : 0;
            if (avail > k - placed) avail = k - placed;
#pragma unroll
            for (int j = 0; j < A; j++)
                if (pending[j] && my[j] >= placed && my[j] < placed + avail)
                    B.slots[((uint64_t)(st0 + st) << kStripeLog2) + o + (uint32_t)(my[j] - placed)] = e[j];
            placed += avail;
            if (placed < k) {
                // the next probe: a fresh random stripe (no primary clustering,
                // so a long run of full stripes stays as unlikely as the load
                // makes it), except in the last chunk, which never advances
                // and walks its stripes in order until every one was tried
                if (last) st = (st + 1 == nst) ? 0 : st + 1;
                else st = (uint32_t)(mix64(((uint64_t)wave_gid << 32) ^ (uint64_t)(wseq++) ^ ((uint64_t)B.salt << 20) ^
                                           0xD1B54A32D192ED03ull) % nst);
                probes++;
                if (!last && probes > B.kappa) {
                    if (lane_id() == 0) {
                        if (atomicCAS(&B.ctl->r, r, r + 1) == r) {
                            atomicAdd(&B.ctl->advances, 1u);
                            atomicOr((unsigned long long *)&B.ctl->forced, 1ull << r);
                        }
                    }
                    spill = true;
                    break;
                }
                if (last && probes >= nst) {
                    if (lane_id() == 0) atomicOr(&B.ctl->overflow, 1u);
                    lost = true;  // give up: the host sees the overflow flag
                    break;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < A; j++) {
            if (!pending[j]) continue;
            if (lost && my[j] >= placed) inserted--;
            if (my[j] < placed || !spill) pending[j] = false;
        }
        if (!spill) break;
    }
    return inserted;
}

// One element per lane.
__device__ __forceinline__ int bag_insert_wave(const Bag &B, bool has, uint64_t e, uint32_t wave_gid,
                                               uint32_t &wseq) {
    const bool h[1] = {has};
    const uint64_t x[1] = {e};
    return bag_insert_wave_n<1>(B, h, x, wave_gid, wseq);
}

}  // namespace hipscc
