// Device-side helpers shared by the hipscc kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hipscc {

constexpr int kWave = 64;
constexpr int kBlock = 256;                 // 4 waves per workgroup
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr uint64_t kEmpty64 = ~0ull;
constexpr int32_t kInf32 = 0x7fffffff;

// SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014), used as a
// stateless 64-bit mixer for hashing and counter-based random draws.
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p ? 1 : 0); }

// Number of set bits of `mask` in lanes below the calling lane.
__device__ __forceinline__ int rank_below(uint64_t mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int popc64(uint64_t m) { return __popcll(m); }

// Wave-wide inclusive prefix sum over 64 lanes with DPP lane moves (no LDS
// round trips): Hillis-Steele within each row of 16 lanes (row_shr 1, 2, 4,
// 8; lanes shifted in from outside the row read 0), then row 15's total is
// added to rows 1 and 3 (row_bcast:15) and lane 31's to rows 2 and 3
// (row_bcast:31).
__device__ __forceinline__ int wave_incl_scan(int x) {
    constexpr int kRowShr = 0x110, kRowBcast15 = 0x142, kRowBcast31 = 0x143;
    x += __builtin_amdgcn_update_dpp(0, x, kRowShr + 1, 0xf, 0xf, true);
    x += __builtin_amdgcn_update_dpp(0, x, kRowShr + 2, 0xf, 0xf, true);
    x += __builtin_amdgcn_update_dpp(0, x, kRowShr + 4, 0xf, 0xf, true);
    x += __builtin_amdgcn_update_dpp(0, x, kRowShr + 8, 0xf, 0xf, true);
    x += __builtin_amdgcn_update_dpp(0, x, kRowBcast15, 0xa, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, kRowBcast31, 0xc, 0xf, false);
    return x;
}

// Wave-wide sum of 32-bit values (the scan's last lane), in every lane.
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_readlane(wave_incl_scan((int)x), kWave - 1);
}

// Value of lane `src` (the same for every lane of the wave) in every lane.
__device__ __forceinline__ int wave_bcast(int x, int src) { return __builtin_amdgcn_readlane(x, src); }
__device__ __forceinline__ uint32_t wave_bcast_u(uint32_t x, int src) {
    return (uint32_t)__builtin_amdgcn_readlane((int)x, src);
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        unsigned lo = (unsigned)x, hi = (unsigned)(x >> 32);
        lo = (unsigned)__shfl_xor((int)lo, d, kWave);
        hi = (unsigned)__shfl_xor((int)hi, d, kWave);
        x += ((unsigned long long)hi << 32) | lo;
    }
    return x;
}

// Orders this wave's LDS traffic: all lanes' earlier LDS writes are visible to
// all lanes' later LDS reads.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t ld_relaxed(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_relaxed64(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Reachability signature terms (Algorithm 1 relabels unfinished vertices by a
// hash of (old label, R_in, R_out)).  The set hashes are sums of per-source
// terms, so they do not depend on the order in which pairs were found.
__device__ __forceinline__ uint64_t sig_term_out(int32_t s) { return mix64((uint64_t)(uint32_t)s ^ 0xA5A5F00Dull) | 1ull; }
__device__ __forceinline__ uint64_t sig_term_in(int32_t s) { return mix64((uint64_t)(uint32_t)s ^ 0x3C6EF372FE94F82Bull) | 1ull; }

// New subproblem label from (old label, backward set hash, forward set hash);
// non-negative 31-bit.  Empty sets keep the old label.
__device__ __forceinline__ int32_t relabel_hash(int32_t old, uint64_t sig_in, uint64_t sig_out) {
    if ((sig_in | sig_out) == 0) return old;
    uint64_t h = mix64(mix64((uint64_t)(uint32_t)old + 0x632BE59BD9B4E019ull) ^ sig_in);
    h = mix64(h + sig_out);
    return (int32_t)(h & 0x7fffffffull);
}

// Reach table key for the pair (vertex v, source index j).
__device__ __forceinline__ uint64_t pair_key(int32_t v, uint32_t j) { return ((uint64_t)(uint32_t)v << 32) | j; }
__device__ __forceinline__ int32_t key_vertex(uint64_t k) { return (int32_t)(k >> 32); }
__device__ __forceinline__ uint32_t key_source(uint64_t k) { return (uint32_t)k; }

// Pseudorandom bijection on [0, n): a 4-round Feistel network on 2b bits
// (2^{2b} >= n) with cycle walking back into [0, n) (Black and Rogaway,
// "Ciphers with arbitrary finite domains", CT-RSA 2002).  Replaces the random
// permutation of the vertices in Algorithm 1 without storing it.
struct Perm {
    uint32_t n;
    uint32_t half_bits;
    uint64_t key;
};

__host__ __device__ __forceinline__ uint32_t perm_apply(const Perm &P, uint32_t x) {
    const uint32_t hb = P.half_bits, hm = (1u << hb) - 1u;
    do {
        uint32_t L = x >> hb, R = x & hm;
#pragma unroll
        for (int r = 0; r < 4; r++) {
            uint32_t F = (uint32_t)mix64(((uint64_t)R << 8 | (uint64_t)r) ^ P.key) & hm;
            uint32_t t = L ^ F;
            L = R;
            R = t;
        }
        x = (L << hb) | R;
    } while (x >= P.n);
    return x;
}

// Inverse of perm_apply: the Feistel rounds undone in reverse order, walking
// the cycle back until the value is below n.
__host__ __device__ __forceinline__ uint32_t perm_invert(const Perm &P, uint32_t y) {
    const uint32_t hb = P.half_bits, hm = (1u << hb) - 1u;
    do {
        uint32_t L = y >> hb, R = y & hm;
#pragma unroll
        for (int r = 3; r >= 0; r--) {
            // forward round r mapped (L, R) to (R, L ^ F(R, r))
            const uint32_t F = (uint32_t)mix64(((uint64_t)L << 8 | (uint64_t)r) ^ P.key) & hm;
            const uint32_t t = R ^ F;
            R = L;
            L = t;
        }
        y = (L << hb) | R;
    } while (y >= P.n);
    return y;
}

}  // namespace hipscc
