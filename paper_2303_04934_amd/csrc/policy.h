// Learned round policy: a float32 MLP 5 -> 32 -> 32 -> 8 (ReLU) evaluated by
// one wavefront.  Inputs are per-round frontier statistics; the 8 outputs
// score (VGC budget class) x (frontier mode).  The policy only picks the
// schedule of the next round; it never changes which pairs are found.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

namespace hipscc {

constexpr int kPolicyIn = 5;
constexpr int kPolicyHidden = 32;
constexpr int kPolicyOut = 8;
constexpr int kPolicyFloats = kPolicyHidden * kPolicyIn + kPolicyHidden + kPolicyHidden * kPolicyHidden +
                              kPolicyHidden + kPolicyOut * kPolicyHidden + kPolicyOut;
// VGC budgets of the four classes (512, 1024, 2048, 4096 arcs per wavefront
// task); class c with mode m is output 2 c + m.
__host__ __device__ __forceinline__ uint32_t policy_tau(int c) { return 512u << c; }

struct Policy {
    float *w = nullptr;    // device weights
    float *io = nullptr;   // device scratch for the test hook
    uint64_t io_cap = 0;   // floats
    bool loaded = false;
};

// Forward pass of one feature row per block of one wavefront; weights are
// staged through LDS.  Row-major weights, out x in.
__device__ __forceinline__ void policy_forward_wave(const float *__restrict__ W, const float *x, float *out,
                                                    float *lds_h1, float *lds_h2) {
    const int l = threadIdx.x & 63;
    const float *W1 = W;
    const float *b1 = W1 + kPolicyHidden * kPolicyIn;
    const float *W2 = b1 + kPolicyHidden;
    const float *b2 = W2 + kPolicyHidden * kPolicyHidden;
    const float *W3 = b2 + kPolicyHidden;
    const float *b3 = W3 + kPolicyOut * kPolicyHidden;
    if (l < kPolicyHidden) {
        float a = b1[l];
        for (int j = 0; j < kPolicyIn; j++) a = fmaf(W1[l * kPolicyIn + j], x[j], a);
        lds_h1[l] = a > 0.f ? a : 0.f;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (l < kPolicyHidden) {
        float a = b2[l];
        for (int j = 0; j < kPolicyHidden; j++) a = fmaf(W2[l * kPolicyHidden + j], lds_h1[j], a);
        lds_h2[l] = a > 0.f ? a : 0.f;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (l < kPolicyOut) {
        float a = b3[l];
        for (int j = 0; j < kPolicyHidden; j++) a = fmaf(W3[l * kPolicyHidden + j], lds_h2[j], a);
        out[l] = a;
    }
}

__global__ __launch_bounds__(64) void k_policy_rows(const float *W, const float *feats, int32_t rows, float *scores) {
    __shared__ float h1[kPolicyHidden], h2[kPolicyHidden];
    const int r = blockIdx.x;
    if (r >= rows) return;
    policy_forward_wave(W, feats + (int64_t)r * kPolicyIn, scores + (int64_t)r * kPolicyOut, h1, h2);
}

// Round features (all float32, computed on the device from the lane state):
//   0 log2(1 + frontier size)
//   1 log2(1 + summed degree of the frontier)
//   2 visited fraction: entries claimed so far / subproblem size
//   3 log2(1 + round index)
//   4 log2(1 + steps of the deepest local search of the previous round)
__device__ __forceinline__ void policy_features(float nf, float fdeg, float claims, float nsub, float round,
                                                float depth, float *x) {
    x[0] = log2f(1.f + nf);
    x[1] = log2f(1.f + fdeg);
    const float v = nsub > 0.f ? claims / nsub : 0.f;
    x[2] = v < 0.f ? 0.f : (v > 1.f ? 1.f : v);
    x[3] = log2f(1.f + round);
    x[4] = log2f(1.f + depth);
}

// Host copy of the same formulas, for trace rows.
inline void policy_features_host(float nf, float fdeg, float claims, float nsub, float round, float depth, float *x) {
    x[0] = std::log2(1.f + nf);
    x[1] = std::log2(1.f + fdeg);
    const float v = nsub > 0.f ? claims / nsub : 0.f;
    x[2] = v < 0.f ? 0.f : (v > 1.f ? 1.f : v);
    x[3] = std::log2(1.f + round);
    x[4] = std::log2(1.f + depth);
}

// Picks the next round's schedule for one search lane from the scores y: the
// budget class and frontier mode with the highest predicted rate among the
// allowed actions (mode_mask bit m allows mode m).  Non-finite scores fall
// back to the fixed schedule.  One thread; writes the lane's tau_cur /
// mode_pref (fields given by pointer so that this header does not depend on
// the round-control layout).
__device__ __forceinline__ void policy_pick(const float *y, uint32_t mode_mask, uint32_t fallback_tau,
                                            uint32_t *tau_cur, uint32_t *mode_pref, uint32_t *calls,
                                            uint32_t *fallbacks) {
    int best = -1;
    float bv = 0.f;
    bool ok = true;
    for (int a = 0; a < kPolicyOut; a++) {
        if (!isfinite(y[a])) ok = false;
        if (!((mode_mask >> (a & 1)) & 1u)) continue;
        if (best < 0 || y[a] > bv) {
            best = a;
            bv = y[a];
        }
    }
    *calls += 1;
    if (!ok || best < 0) {
        *tau_cur = fallback_tau;
        *mode_pref = 0;
        *fallbacks += 1;
    } else {
        *tau_cur = policy_tau(best >> 1);
        *mode_pref = (uint32_t)(best & 1);
    }
}

// Where one search lane keeps the policy's inputs and outputs.
struct PolicyLane {
    const uint32_t *nF2;               // frontier sizes of both parities
    const unsigned long long *fdeg;    // degree sum of the coming frontier
    const unsigned long long *claims;
    const uint32_t *rounds;
    const uint32_t *lsdepth;           // deepest local search of the previous round
    float nsub;                        // subproblem size
    uint32_t *tau_cur, *mode_pref, *calls, *fallbacks;
    uint32_t mode_mask;                // bit m allows frontier mode m (dense only for single-source lanes)
};

// The policy step before a round, one launch for up to two lanes (block b =
// lane b, one wave each).
__global__ __launch_bounds__(64) void k_policy_round(const float *W, PolicyLane L0, PolicyLane L1,
                                                     uint32_t fallback_tau) {
    __shared__ float x[kPolicyIn], h1[kPolicyHidden], h2[kPolicyHidden], y[kPolicyOut];
    const PolicyLane &L = blockIdx.x == 0 ? L0 : L1;
    const uint32_t nf = L.nF2[0] + L.nF2[1];
    if (nf == 0) return;
    if (threadIdx.x == 0)
        policy_features((float)nf, (float)*L.fdeg, (float)*L.claims, L.nsub, (float)*L.rounds, (float)*L.lsdepth, x);
    __syncthreads();
    policy_forward_wave(W, x, y, h1, h2);
    __syncthreads();
    if (threadIdx.x == 0) policy_pick(y, L.mode_mask, fallback_tau, L.tau_cur, L.mode_pref, L.calls, L.fallbacks);
}

inline void policy_release(Policy &p) {
    if (p.w) (void)hipFree(p.w);
    if (p.io) (void)hipFree(p.io);
    p.w = p.io = nullptr;
    p.io_cap = 0;
    p.loaded = false;
}

// 0 ok, 1 wrong size, 2 non-finite weight, 3 HIP failure.
inline int policy_load(Policy &p, const float *w, int64_t n, hipStream_t s) {
    if (!w || n != kPolicyFloats) return 1;
    for (int64_t i = 0; i < n; i++)
        if (!std::isfinite(w[i])) return 2;
    if (!p.w && hipMalloc((void **)&p.w, sizeof(float) * kPolicyFloats) != hipSuccess) return 3;
    if (hipMemcpyAsync(p.w, w, sizeof(float) * kPolicyFloats, hipMemcpyHostToDevice, s) != hipSuccess) return 3;
    if (hipStreamSynchronize(s) != hipSuccess) return 3;
    p.loaded = true;
    return 0;
}

inline int policy_eval_host(Policy &p, const float *feats, int32_t rows, float *scores, hipStream_t s) {
    const uint64_t need = (uint64_t)rows * (kPolicyIn + kPolicyOut);
    if (p.io_cap < need) {
        if (p.io) (void)hipFree(p.io);
        p.io = nullptr;
        p.io_cap = 0;
        if (hipMalloc((void **)&p.io, sizeof(float) * need) != hipSuccess) return 3;
        p.io_cap = need;
    }
    float *df = p.io, *ds = p.io + (uint64_t)rows * kPolicyIn;
    if (hipMemcpyAsync(df, feats, sizeof(float) * rows * kPolicyIn, hipMemcpyHostToDevice, s) != hipSuccess) return 3;
    hipLaunchKernelGGL(k_policy_rows, dim3(rows), dim3(64), 0, s, p.w, df, rows, ds);
    if (hipGetLastError() != hipSuccess) return 3;
    if (hipMemcpyAsync(scores, ds, sizeof(float) * rows * kPolicyOut, hipMemcpyDeviceToHost, s) != hipSuccess) return 3;
    if (hipStreamSynchronize(s) != hipSuccess) return 3;
    return 0;
}

}  // namespace hipscc
