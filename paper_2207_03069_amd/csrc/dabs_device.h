// dabs_device.h -- device-side building blocks of the bulk-search kernels
// (gfx950, wave64): counter-based generator, wave reductions, and the
// per-wave search instance ("walker") that keeps one instance's state in
// registers.
//
// Data layout of one instance inside a wave.  W rows are read as 16-byte
// vectors: V = 16 / sizeof(weight) elements per lane per slot, SLOTS slots
// cover n.  Lane l holds, for slot s and sub-index e < V, bit
// k = s*64*V + l*V + e at local index j = s*V + e.  Per element the lane keeps
// one word kb[j] = Delta_k 2^KB + j + 2^29 (+ 2^31 while bit k is outside the
// rule's domain), with Delta_k = (1 - 2 x_k)(W_kk + 2 sum_{m != k} W_km x_m)
// (Section III-A Eq. (3) in the full-sum convention), updated on a flip of
// bit i by Delta_k += 2 (1 - 2 x_i)(1 - 2 x_k) W_ik (Eq. (4); the device copy
// of W has a zero diagonal) and Delta_i -> -Delta_i (Eq. (5)); and one
// multiplier word mul[j] = (1 - 2 x_k) 2^(KB+1) for that update.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dabs {

constexpr int WAVE = 64;
constexpr int TAU_MAX = 16;
constexpr int64_t E_INF = INT64_MAX;

enum Rule { GREEDY = 0, STRAIGHT = 1, MAXMIN = 2, CYCLICMIN = 3, RANDOMMIN = 4,
            POSITIVEMIN = 5, TWONEIGHBOR = 6, TABU_GREEDY = 7 };
enum Tag { TAG_MAXMIN = 1, TAG_POSMIN = 2, TAG_RANDMIN = 3, TAG_GA = 4, TAG_POOL = 5 };

constexpr int clog2(int v) { return v <= 1 ? 0 : 1 + clog2((v + 1) / 2); }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten S-box rounds on a
// 128-bit counter, key bumped by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
struct R4 { uint32_t w[4]; };

__device__ __forceinline__ R4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint64_t key) {
    uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32 -> 64-bit product each (v_mad_u64_u32 in vector code
        // instead of a low and a high multiply)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    R4 r; r.w[0] = c0; r.w[1] = c1; r.w[2] = c2; r.w[3] = c3;
    return r;
}

__device__ __forceinline__ uint32_t scale32(uint32_t u, uint32_t m) {
    return (uint32_t)(((uint64_t)u * (uint64_t)m) >> 32);
}

// floor(t 2^32 / T) and its remainder for t = 0, 1, 2, ... (T >= 1): with
// 2^32 = Q T + R the quotient and remainder step by (Q, R) and one carry, so
// a phase divides once instead of once per iteration.
struct FracStep {
    uint64_t q, Q;      // floor(t 2^32 / T), floor(2^32 / T)
    uint32_t r, R, T;   // (t 2^32) mod T, 2^32 mod T
    __device__ __forceinline__ void init(uint32_t T_) {
        T = T_;
        Q = (1ull << 32) / T_;
        R = (uint32_t)((1ull << 32) % T_);
        q = 0;
        r = 0;
    }
    __device__ __forceinline__ void next() {
        q += Q;
        r += R;
        if (r >= T) {
            r -= T;
            q += 1;
        }
    }
    // floor((T - t) 2^32 / T) = 2^32 - ceil(t 2^32 / T)
    __device__ __forceinline__ uint64_t rest() const { return (1ull << 32) - q - (r != 0 ? 1 : 0); }
};

// 32.32 fixed-point cube, floor-chained.
__device__ __forceinline__ uint64_t cube_frac(uint64_t f) { return (((f * f) >> 32) * f) >> 32; }

// ---------------------------------------------------------------------------
// Wave helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() {
    return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ int readlane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t ballot(bool b) { return __builtin_amdgcn_ballot_w64(b); }

// Row-level butterflies (quad xor 1, quad xor 2, half mirror, mirror) leave
// each 16-lane row with its extremum; the four rows are combined in SGPRs.
template <bool MAX>
__device__ __forceinline__ int wave_ext(int v) {
    auto op = [](int a, int b) { return MAX ? max(a, b) : min(a, b); };
    v = op(v, __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true));
    v = op(v, __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true));
    v = op(v, __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true));
    v = op(v, __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, true));
    const int a = readlane(v, 0), b = readlane(v, 16), c = readlane(v, 32), d = readlane(v, 48);
    return op(op(a, b), op(c, d));
}
__device__ __forceinline__ int wave_min(int v) { return wave_ext<false>(v); }

// Two wave minima reduced together so that the two DPP chains interleave.
__device__ __forceinline__ void wave_min2(int a, int b, int &ra, int &rb) {
    a = min(a, __builtin_amdgcn_mov_dpp(a, 0xB1, 0xF, 0xF, true));
    b = min(b, __builtin_amdgcn_mov_dpp(b, 0xB1, 0xF, 0xF, true));
    a = min(a, __builtin_amdgcn_mov_dpp(a, 0x4E, 0xF, 0xF, true));
    b = min(b, __builtin_amdgcn_mov_dpp(b, 0x4E, 0xF, 0xF, true));
    a = min(a, __builtin_amdgcn_mov_dpp(a, 0x141, 0xF, 0xF, true));
    b = min(b, __builtin_amdgcn_mov_dpp(b, 0x141, 0xF, 0xF, true));
    a = min(a, __builtin_amdgcn_mov_dpp(a, 0x140, 0xF, 0xF, true));
    b = min(b, __builtin_amdgcn_mov_dpp(b, 0x140, 0xF, 0xF, true));
    ra = min(min(readlane(a, 0), readlane(a, 16)), min(readlane(a, 32), readlane(a, 48)));
    rb = min(min(readlane(b, 0), readlane(b, 16)), min(readlane(b, 32), readlane(b, 48)));
}
__device__ __forceinline__ int wave_max(int v) { return wave_ext<true>(v); }

// Wave min of a and b and wave max of c, reduced together (interleaved DPP
// chains; c ends in a max).
__device__ __forceinline__ void wave_minmin_max(int a, int b, int c, int &ra, int &rb, int &rc) {
    a = min(a, __builtin_amdgcn_mov_dpp(a, 0xB1, 0xF, 0xF, true));
    b = min(b, __builtin_amdgcn_mov_dpp(b, 0xB1, 0xF, 0xF, true));
    c = max(c, __builtin_amdgcn_mov_dpp(c, 0xB1, 0xF, 0xF, true));
    a = min(a, __builtin_amdgcn_mov_dpp(a, 0x4E, 0xF, 0xF, true));
    b = min(b, __builtin_amdgcn_mov_dpp(b, 0x4E, 0xF, 0xF, true));
    c = max(c, __builtin_amdgcn_mov_dpp(c, 0x4E, 0xF, 0xF, true));
    a = min(a, __builtin_amdgcn_mov_dpp(a, 0x141, 0xF, 0xF, true));
    b = min(b, __builtin_amdgcn_mov_dpp(b, 0x141, 0xF, 0xF, true));
    c = max(c, __builtin_amdgcn_mov_dpp(c, 0x141, 0xF, 0xF, true));
    a = min(a, __builtin_amdgcn_mov_dpp(a, 0x140, 0xF, 0xF, true));
    b = min(b, __builtin_amdgcn_mov_dpp(b, 0x140, 0xF, 0xF, true));
    c = max(c, __builtin_amdgcn_mov_dpp(c, 0x140, 0xF, 0xF, true));
    ra = min(min(readlane(a, 0), readlane(a, 16)), min(readlane(a, 32), readlane(a, 48)));
    rb = min(min(readlane(b, 0), readlane(b, 16)), min(readlane(b, 32), readlane(b, 48)));
    rc = max(max(readlane(c, 0), readlane(c, 16)), max(readlane(c, 32), readlane(c, 48)));
}

// Wave min of a and wave max of c, reduced together.
__device__ __forceinline__ void wave_min_max(int a, int c, int &ra, int &rc) {
    a = min(a, __builtin_amdgcn_mov_dpp(a, 0xB1, 0xF, 0xF, true));
    c = max(c, __builtin_amdgcn_mov_dpp(c, 0xB1, 0xF, 0xF, true));
    a = min(a, __builtin_amdgcn_mov_dpp(a, 0x4E, 0xF, 0xF, true));
    c = max(c, __builtin_amdgcn_mov_dpp(c, 0x4E, 0xF, 0xF, true));
    a = min(a, __builtin_amdgcn_mov_dpp(a, 0x141, 0xF, 0xF, true));
    c = max(c, __builtin_amdgcn_mov_dpp(c, 0x141, 0xF, 0xF, true));
    a = min(a, __builtin_amdgcn_mov_dpp(a, 0x140, 0xF, 0xF, true));
    c = max(c, __builtin_amdgcn_mov_dpp(c, 0x140, 0xF, 0xF, true));
    ra = min(min(readlane(a, 0), readlane(a, 16)), min(readlane(a, 32), readlane(a, 48)));
    rc = max(max(readlane(c, 0), readlane(c, 16)), max(readlane(c, 32), readlane(c, 48)));
}

// value of the neighbouring lane (l xor 1)
__device__ __forceinline__ uint32_t swap_pair(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);
}

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int m) {
    int lo = __shfl_xor((int)(uint32_t)v, m, WAVE), hi = __shfl_xor((int)(uint32_t)(v >> 32), m, WAVE);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

__device__ __forceinline__ long long wave_sum64(long long v) {
    for (int m = 1; m < WAVE; m <<= 1) v += (long long)shfl_xor64((uint64_t)v, m);
    return v;
}

__device__ __forceinline__ int mad24(int a, int b, int c) {
    // sign-extension from 24 bits is a no-op for |a|,|b| < 2^23 and lets the
    // compiler emit one v_mad_i32_i24
    return ((a << 8) >> 8) * ((b << 8) >> 8) + c;
}

typedef short short2v __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// Genetic operations driven by the learned logits of the parent's bits
// (word w of the target):
//   MLP-seed   flips bit k when z_k > 0;
//   MLP-mutate flips bit k when its u32 draw is below 2^29 + q_k 2^22 with
//              q_k = clamp(round-half-even(16 z_k), -128, 127), i.e. with
//              probability (1 + q_k/128)/8 around the Mutation rate 1/8.
// The draws are the genetic operations' per-bit stream: Philox counter
// (round, instance, k/4, TAG_GA<<24 | 2), word k mod 4.
// ---------------------------------------------------------------------------
enum { OP_MLP_SEED = 8, OP_MLP_MUTATE = 9 };

__device__ __forceinline__ uint64_t mlp_op_word(int op, uint64_t parent, const float *logits, int n, int w,
                                                uint64_t seed, uint32_t rd, uint32_t inst) {
    uint64_t flip = 0;
    const int k0 = 64 * w;
    for (int c = 0; c < 16; ++c) {
        if (k0 + 4 * c >= n) break;
        R4 r = {{0u, 0u, 0u, 0u}};
        if (op == OP_MLP_MUTATE) r = philox(rd, inst, (uint32_t)(16 * w + c), ((uint32_t)TAG_GA << 24) | 2u, seed);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = k0 + 4 * c + q;
            if (k >= n) break;
            const float z = logits[k];
            bool f;
            if (op == OP_MLP_SEED) {
                f = z > 0.0f;
            } else {
                const float lv = fminf(fmaxf(rintf(z * 16.0f), -128.0f), 127.0f);
                f = (long long)r.w[q] < (1ll << 29) + (long long)lv * (1ll << 22);
            }
            if (f) flip |= 1ull << (4 * c + q);
        }
    }
    return parent ^ flip;
}

}  // namespace dabs
