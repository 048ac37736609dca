// dabs_mlp.hip -- the learned proposal: per-bit features of pooled vectors,
// a 3-layer MLP (8 -> 64 -> 64 -> 1, ReLU) giving flip-priority logits, its
// training (binary cross-entropy, Adam) and the two genetic operations that
// consume the logits (MLP-seed, MLP-mutate).
//
// Matrix products run on the matrix cores with bfloat16 operands (round to
// nearest even) and float32 accumulation.  Lane l = 0..63, g = l / 16,
// c = l % 16.  The forward pass uses gfx950's v_mfma_f32_16x16x32_bf16:
//   A[i][k] (16 x 32): lane i + 16 floor(k/8), element k mod 8
//   B[k][j] (32 x 16): lane j + 16 floor(k/8), element k mod 8
//   D[i][j] (16 x 16): lane j + 16 floor(i/4), element i mod 4
// Activations are kept transposed (hidden unit x sample).  A layer's output
// tiles D (16 units x 16 samples) hold in lane (g, c) the units 16t + 4g + e
// of sample c; the next layer's 32-deep reduction block u takes the
// elements of tiles 2u and 2u + 1 of a lane, in that order, as its B operand
// (reduction index 8g + e' = unit 16 (2u + e'/4) + 4g + e' mod 4), and
// the weights are loaded in the same order, so the forward pass needs no
// data movement between layers.  The biases start the accumulators.
// The backward products use v_mfma_f32_16x16x16_bf16 (same D layout;
// A and B with element k mod 4 in lane i (j) + 16 floor(k/4)).  The weight
// gradients reduce over samples and need the transposed tiles; each
// wavefront stages them through its own 6.3 KB of LDS.
#include <math.h>
#include <string.h>

#include <mutex>

#include "dabs_device.h"
#include "dabs_internal.h"

#define HIP_OK(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return dabs_fail(DABS_E_HIP, "%s: %s", #call, hipGetErrorString(e_));      \
    } while (0)

namespace dabs {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 hbf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 hbf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

constexpr int NF = 8, HID = 64;
constexpr int OFF_W1 = 0, OFF_B1 = 512, OFF_W2 = 576, OFF_B2 = 4672, OFF_W3 = 4736, OFF_B3 = 4800;
constexpr int NPAR = 4801;
constexpr int GRAD_BLOCKS_MAX = 1024;
constexpr float ADAM_B1 = 0.9f, ADAM_B2 = 0.999f, ADAM_EPS = 1e-8f;

// float32 -> bfloat16, round to nearest even (finite inputs)
__device__ __forceinline__ short to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}
__device__ __forceinline__ float bf16_val(short b) { return __uint_as_float((uint32_t)(uint16_t)b << 16); }
// two float32 -> packed bfloat16 (a low, b high), round to nearest even: one
// v_cvt_pk_bf16_f32, the same values as to_bf16 for finite inputs
__device__ __forceinline__ uint32_t pk_bf16(float a, float b) {
    const f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, hbf16x2));
}

__device__ __forceinline__ f32x4 mma(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mma32(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(hbf16x8, a), __builtin_bit_cast(hbf16x8, b),
                                                   c, 0, 0, 0);
}

// four consecutive bfloat16 values (8-byte aligned)
__device__ __forceinline__ bf16x4 ld4(const short *p) {
    const uint2 u = *(const uint2 *)p;
    bf16x4 v;
    v.x = (short)(u.x & 0xFFFF); v.y = (short)(u.x >> 16);
    v.z = (short)(u.y & 0xFFFF); v.w = (short)(u.y >> 16);
    return v;
}
__device__ __forceinline__ bf16x8 cat8(bf16x4 a, bf16x4 b) {
    return bf16x8{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
}
// hidden unit of reduction index 8g + e' in 32-deep block u (see above)
__device__ __forceinline__ int unit_of(int u, int g, int e) { return 16 * (2 * u + (e >> 2)) + 4 * g + (e & 3); }

// Weights of one wavefront in matrix-core operand form.
struct Net {
    bf16x8 f1[4];          // W1 tile t (units 16 t + c, features 0..7 in lane group 0), 16x16x32 A operand
    bf16x8 f2[4][2];       // W2 tile [out t][block u], 16x16x32 A operand
    bf16x8 f3[2];          // W3 as row 0 of a 16 x 64 matrix, blocks u
    f32x4 c1[4], c2[4];    // biases of units 16 t + 4 g + e: the accumulators' start
    float w3[4][4];        // per lane: unit 16 t + 4 g + e
    float b3;

    __device__ void load(const short *__restrict__ wbf, const float *__restrict__ par, int lane) {
        const int g = lane >> 4, c = lane & 15;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            f1[t] = g == 0 ? cat8(ld4(wbf + OFF_W1 + (16 * t + c) * NF), ld4(wbf + OFF_W1 + (16 * t + c) * NF + 4))
                           : bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int e = 0; e < 8; ++e) f2[t][u][e] = wbf[OFF_W2 + (16 * t + c) * HID + unit_of(u, g, e)];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int u = 16 * t + 4 * g + e;
                c1[t][e] = par[OFF_B1 + u];
                c2[t][e] = par[OFF_B2 + u];
                w3[t][e] = bf16_val(wbf[OFF_W3 + u]);
            }
        }
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int e = 0; e < 8; ++e) f3[u][e] = c == 0 ? wbf[OFF_W3 + unit_of(u, g, e)] : (short)0;
        b3 = par[OFF_B3];
    }
};

// Feature operand of the 16 samples s0 .. s0+15: lane (0, c) holds the 8
// features of sample s0 + c (zero past the end); the other lane groups zero.
__device__ __forceinline__ bf16x8 load_feat(const short *__restrict__ feat, int64_t N, int64_t s0, int lane) {
    const int g = lane >> 4, c = lane & 15;
    if (g != 0 || s0 + c >= N) return bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
    const uint4 v = *(const uint4 *)(feat + (s0 + c) * NF);
    return __builtin_bit_cast(bf16x8, v);
}
// Forward pass of one tile.  h1/h2: bfloat16 activations in the D layout
// (lane (g, c): units 16t + 4g + e of sample c); m1/m2: bit (4t + e) set when
// the pre-activation of unit 16t + 4g + e is > 0.  Returns the logit (valid
// in lanes 0..15, sample s0 + lane).
// ReLU on the bit pattern: a float with the sign bit set (negative, -0)
// is a negative int32 and becomes +0, one integer max per value
__device__ __forceinline__ float relu(float z) { return __int_as_float(max(__float_as_int(z), 0)); }
__device__ __forceinline__ bf16x4 relu_bf16(f32x4 d) {
    const u32x2 v = {pk_bf16(relu(d[0]), relu(d[1])), pk_bf16(relu(d[2]), relu(d[3]))};
    return __builtin_bit_cast(bf16x4, v);
}
__device__ __forceinline__ uint32_t pos_bits(f32x4 d, int t) {
    uint32_t m = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) m |= (d[e] > 0.f ? 1u : 0u) << (4 * t + e);
    return m;
}
__device__ __forceinline__ float fwd_tile(const Net &w, bf16x8 x, bf16x4 (&h1)[4], bf16x4 (&h2)[4], uint32_t &m1,
                                          uint32_t &m2) {
    m1 = 0;
    m2 = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const f32x4 d = mma32(w.f1[t], x, w.c1[t]);
        m1 |= pos_bits(d, t);
        h1[t] = relu_bf16(d);
    }
    const bf16x8 b0 = cat8(h1[0], h1[1]), b1 = cat8(h1[2], h1[3]);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const f32x4 d = mma32(w.f2[t][1], b1, mma32(w.f2[t][0], b0, w.c2[t]));
        m2 |= pos_bits(d, t);
        h2[t] = relu_bf16(d);
    }
    const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
    const f32x4 d = mma32(w.f3[1], cat8(h2[2], h2[3]), mma32(w.f3[0], cat8(h2[0], h2[1]), zero));
    return d[0] + w.b3;
}

// Logits of N samples; one wavefront per workgroup, pairs of 16-sample
// tiles (t, t + gridDim.x) strided over the grid.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void k_mlp_fwd(
    const short *__restrict__ wbf, const float *__restrict__ par, const short *__restrict__ feat, int64_t N,
    float *__restrict__ out) {
    const int lane = (int)threadIdx.x;
    Net w;
    w.load(wbf, par, lane);
    const int64_t tiles = (N + 15) / 16, G = gridDim.x;
    // the next pair's features load while this pair is worked on
    bf16x8 n0 = load_feat(feat, N, (int64_t)blockIdx.x * 16, lane), n1 = load_feat(feat, N, (blockIdx.x + G) * 16, lane);
    for (int64_t t = blockIdx.x; t < tiles; t += 2 * G) {
        const int64_t s0 = t * 16, s1 = (t + G) * 16;   // s1 may lie past N: its samples are zero
        bf16x4 h1[4], h2[4], k1[4], k2[4];
        uint32_t m1, m2, q1, q2;
        const bf16x8 x0 = n0, x1 = n1;
        n0 = load_feat(feat, N, s0 + 32 * G, lane);
        n1 = load_feat(feat, N, s1 + 32 * G, lane);
        const float z0 = fwd_tile(w, x0, h1, h2, m1, m2);
        const float z1 = fwd_tile(w, x1, k1, k2, q1, q2);
        if (lane < 16 && s0 + lane < N) out[s0 + lane] = z0;
        if (lane < 16 && s1 + lane < N) out[s1 + lane] = z1;
    }
}

__device__ __forceinline__ float sum16(float v) {
    // sum over the 16 lanes of a row (lanes with the same l / 16)
#pragma unroll
    for (int m = 1; m < 16; m <<= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Gradient of the mean binary cross-entropy over N samples.  Every
// workgroup (one wavefront) covers the tiles blockIdx.x + k gridDim.x and
// writes its partial sums (4801 gradient values, then the loss sum) to
// part[blockIdx.x]; k_mlp_reduce adds the partials in block order.
__global__ __launch_bounds__(64) void k_mlp_grad(const short *__restrict__ wbf, const float *__restrict__ par,
                                                 const short *__restrict__ feat, const uint8_t *__restrict__ label,
                                                 int64_t N, float invN, float *__restrict__ part) {
    __shared__ __attribute__((aligned(16))) short sA2[HID][16], sH1[HID][16], sA1[HID][16], sF[NF][16];
    // W2 transposed with its output units in the 16x16x32 reduction order:
    // sW2P[in][32 kb + 8 g + e] = W2[unit_of(kb, g, e)][in]
    __shared__ __attribute__((aligned(16))) short sW2P[HID][HID];
    const int lane = (int)threadIdx.x, g = lane >> 4, c = lane & 15;
    for (int i = lane; i < HID * HID; i += WAVE) {
        const int in = i / HID, k = i % HID;
        sW2P[in][k] = wbf[OFF_W2 + unit_of(k >> 5, (k >> 3) & 3, k & 7) * HID + in];
    }
    __syncthreads();
    Net w;
    w.load(wbf, par, lane);
    const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
    f32x4 gW2[4][4], gW1[4];
    float gW3[4][4], gB2[4][4], gB1[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        gW1[t] = zero;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            gW2[t][u] = zero;
            gW3[t][u] = 0.f; gB2[t][u] = 0.f; gB1[t][u] = 0.f;
        }
    }
    float gB3 = 0.f, lsum = 0.f;
    const int64_t tiles = (N + 15) / 16;
    // the next tile's features and labels load while this tile is worked on
    auto load_label = [&](int64_t s) { return lane < 16 && s + lane < N ? label[s + lane] : (uint8_t)0; };
    bf16x8 x_next = load_feat(feat, N, (int64_t)blockIdx.x * 16, lane);
    uint8_t y_next = load_label((int64_t)blockIdx.x * 16);
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const int64_t s0 = t * 16;
        const bf16x8 x = x_next;
        const uint8_t ylab = y_next;
        x_next = load_feat(feat, N, s0 + 16 * (int64_t)gridDim.x, lane);
        y_next = load_label(s0 + 16 * (int64_t)gridDim.x);
        bf16x4 h1[4], h2[4];
        uint32_t m1, m2;
        const float z = fwd_tile(w, x, h1, h2, m1, m2);
        // dL/dz of sample s0 + lane (lanes 0..15), then broadcast by sample
        float dz = 0.f;
        if (lane < 16 && s0 + lane < N) {
            const float y = ylab ? 1.f : 0.f;
            const float s = 1.f / (1.f + expf(-z));
            dz = (s - y) * invN;
            lsum += fmaxf(z, 0.f) - y * z + log1pf(expf(-fabsf(z)));
            gB3 += dz;
        }
        const float dzc = __shfl(dz, c, 64);
        bf16x4 d2[4], d1[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            float d[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                gW3[u][e] += dzc * bf16_val(h2[u][e]);
                d[e] = ((m2 >> (4 * u + e)) & 1) ? w.w3[u][e] * dzc : 0.f;
                gB2[u][e] += d[e];
            }
            const u32x2 v = {pk_bf16(d[0], d[1]), pk_bf16(d[2], d[3])};
            d2[u] = __builtin_bit_cast(bf16x4, v);
        }
        // dH1 = W2^T dA2 on the 16x16x32 products: B = the dA2 tiles 2kb, 2kb + 1
        // of a lane concatenated, A = W2^T rows from LDS in the same order
        const bf16x8 b0 = cat8(d2[0], d2[1]), b1 = cat8(d2[2], d2[3]);
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const bf16x8 a0 = *(const bf16x8 *)&sW2P[16 * it + c][8 * g];
            const bf16x8 a1 = *(const bf16x8 *)&sW2P[16 * it + c][32 + 8 * g];
            const f32x4 acc = mma32(a1, b1, mma32(a0, b0, zero));
            float d[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                d[e] = ((m1 >> (4 * it + e)) & 1) ? acc[e] : 0.f;
                gB1[it][e] += d[e];
            }
            const u32x2 v = {pk_bf16(d[0], d[1]), pk_bf16(d[2], d[3])};
            d1[it] = __builtin_bit_cast(bf16x4, v);
        }
        // stage (unit x sample) tiles for the reductions over samples
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                sA2[16 * u + 4 * g + e][c] = d2[u][e];
                sH1[16 * u + 4 * g + e][c] = h1[u][e];
                sA1[16 * u + 4 * g + e][c] = d1[u][e];
            }
        if (g == 0)
#pragma unroll
            for (int e = 0; e < NF; ++e) sF[e][c] = x[e];
        __syncthreads();
        // dW2[out][in] += sum_s dA2[out][s] a1[in][s];  dW1[out][f] += sum_s dA1[out][s] F[f][s]
        bf16x4 bh[4];
#pragma unroll
        for (int it = 0; it < 4; ++it) bh[it] = ld4(&sH1[16 * it + c][4 * g]);
        const bf16x4 bf = c < NF ? ld4(&sF[c][4 * g]) : bf16x4{0, 0, 0, 0};
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
            const bf16x4 a = ld4(&sA2[16 * ot + c][4 * g]);
#pragma unroll
            for (int it = 0; it < 4; ++it) gW2[ot][it] = mma(a, bh[it], gW2[ot][it]);
            gW1[ot] = mma(ld4(&sA1[16 * ot + c][4 * g]), bf, gW1[ot]);
        }
        __syncthreads();
    }
    float *P = part + (int64_t)blockIdx.x * (NPAR + 1);
    // matrix-core accumulators: D[i][j] at lane j + 16 floor(i/4), element i mod 4
#pragma unroll
    for (int ot = 0; ot < 4; ++ot)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int o = 16 * ot + 4 * g + e;
#pragma unroll
            for (int it = 0; it < 4; ++it) P[OFF_W2 + o * HID + 16 * it + c] = gW2[ot][it][e];
            if (c < NF) P[OFF_W1 + o * NF + c] = gW1[ot][e];
        }
    // per-lane sums over samples: reduce over the 16 lanes of each row
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float a = sum16(gW3[u][e]), b = sum16(gB2[u][e]), d = sum16(gB1[u][e]);
            if (c == 0) {
                P[OFF_W3 + 16 * u + 4 * g + e] = a;
                P[OFF_B2 + 16 * u + 4 * g + e] = b;
                P[OFF_B1 + 16 * u + 4 * g + e] = d;
            }
        }
    const float b3 = sum16(gB3), ls = sum16(lsum);
    if (lane == 0) {
        P[OFF_B3] = b3;
        P[NPAR] = ls;
    }
}

// grad[i] = sum over blocks of part[b][i]; loss = mean.  A workgroup of 1024
// threads covers 64 values: 16 groups sum the blocks b = g, g + 16, ... and
// the 16 group sums are added in group order (a fixed order: reproducible).
constexpr int RED_COLS = 64, RED_GROUPS = 16;
__global__ __launch_bounds__(1024) void k_mlp_reduce(const float *__restrict__ part, int blocks, float invN,
                                                     float *__restrict__ grad, float *__restrict__ loss) {
    __shared__ float acc[RED_GROUPS][RED_COLS];
    const int c = (int)threadIdx.x % RED_COLS, g = (int)threadIdx.x / RED_COLS;
    const int i = blockIdx.x * RED_COLS + c;
    float s = 0.f;
    if (i <= NPAR)
        for (int b = g; b < blocks; b += RED_GROUPS) s += part[(int64_t)b * (NPAR + 1) + i];
    acc[g][c] = s;
    __syncthreads();
    if (g == 0 && i <= NPAR) {
        float t = 0.f;
        for (int q = 0; q < RED_GROUPS; ++q) t += acc[q][c];
        if (i < NPAR) grad[i] = t;
        else if (loss) *loss = t * invN;
    }
}

// Adam (Kingma & Ba) on the float32 master copy; c1 = 1/(1-b1^t),
// c2 = 1/(1-b2^t).  Refreshes the bfloat16 copy.
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ grad, float *__restrict__ m,
                       float *__restrict__ v, short *__restrict__ wbf, float lr, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPAR) return;
    const float gi = grad[i];
    const float mi = ADAM_B1 * m[i] + (1.f - ADAM_B1) * gi;
    const float vi = ADAM_B2 * v[i] + (1.f - ADAM_B2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + ADAM_EPS);
    p[i] = pi;
    wbf[i] = to_bf16(pi);
}

__global__ void k_to_bf16(const float *__restrict__ p, short *__restrict__ wbf) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < NPAR) wbf[i] = to_bf16(p[i]);
}

// Bits set in each pool: cnt[q][k] = #{r : bit k of entry (q, r)}.
__global__ void k_pool_counts(const uint64_t *__restrict__ bits, int P, int m, int n, int nw, int *__restrict__ cnt) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)P * n) return;
    const int q = (int)(t / n), k = (int)(t % n);
    int s = 0;
    for (int r = 0; r < m; ++r) s += (int)((bits[((int64_t)q * m + r) * nw + (k >> 6)] >> (k & 63)) & 1);
    cnt[t] = s;
}

// Features of every pooled vector (one workgroup per entry (q, r)).  The
// local field h_k = W_kk + 2 sum_{j != k} W_kj x_j is accumulated in
// registers (thread t holds k = t + 256 i) over the set bits j of the entry,
// four rows at a time so that their loads are in flight together (the packed
// W has a zero diagonal and zero padding up to its row stride, which covers
// 256 ceil(n/256)).  need (nullable): only the entries flagged there are
// computed (the parents that this round's learned operations read), and
// their flags are cleared.
constexpr int FEAT_NPT = 16;      // n <= 4096 = 256 x 16
template <typename WT>
__global__ __launch_bounds__(256) void k_features(const WT *__restrict__ W, const int *__restrict__ diag,
                                                  const int64_t *__restrict__ rowabs, int64_t ld, int n, int nw,
                                                  int64_t bound, const uint64_t *__restrict__ bits, int m,
                                                  const int *__restrict__ cnt, short *__restrict__ feat,
                                                  int *__restrict__ need) {
    __shared__ int wanted;
    const int cell = blockIdx.x, q = cell / m, r = cell % m;
    const int tid = (int)threadIdx.x;
    if (need) {
        if (tid == 0) wanted = need[cell];
        __syncthreads();
        if (!wanted) return;              // the whole workgroup leaves together
        if (tid == 0) need[cell] = 0;
    }
    const uint64_t *x = bits + (int64_t)cell * nw;
    const uint64_t *best = bits + (int64_t)q * m * nw;
    const int npt = (n + 255) / 256;
    int h[FEAT_NPT];
#pragma unroll
    for (int i = 0; i < FEAT_NPT; ++i) h[i] = 0;
    // rows js[0..3]; the rows past cnt_j repeat js[0] and count zero times
    auto add_rows = [&](const int (&js)[4], int cnt_j) {
        const WT *r0 = W + (int64_t)js[0] * ld + tid, *r1 = W + (int64_t)js[1] * ld + tid;
        const WT *r2 = W + (int64_t)js[2] * ld + tid, *r3 = W + (int64_t)js[3] * ld + tid;
        const int c1 = cnt_j > 1, c2 = cnt_j > 2, c3 = cnt_j > 3;
#pragma unroll
        for (int i = 0; i < FEAT_NPT; ++i) {
            if (i < npt) {
                const int o = 256 * i;
                h[i] += 2 * ((int)r0[o] + c1 * (int)r1[o] + c2 * (int)r2[o] + c3 * (int)r3[o]);
            }
        }
    };
    for (int wd = 0; wd < nw; ++wd) {
        uint64_t word = x[wd];
        if (wd == nw - 1 && (n & 63)) word &= (1ull << (n & 63)) - 1;   // bits >= n are not part of X
        while (word) {
            // up to four set bits of this word
            int js[4];
            int c = 0;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                js[u] = word ? wd * 64 + __builtin_ctzll(word) : js[0];
                c += word ? 1 : 0;
                word &= word - 1;
            }
            add_rows(js, c);
        }
    }
    const float fB = (float)bound, fm = (float)m;
#pragma unroll
    for (int i = 0; i < FEAT_NPT; ++i) {
        const int k = tid + 256 * i;
        if (i >= npt || k >= n) continue;
        const int xk = (int)((x[k >> 6] >> (k & 63)) & 1), bk = (int)((best[k >> 6] >> (k & 63)) & 1);
        const int delta = (1 - 2 * xk) * (diag[k] + h[i]);
        float f[NF];
        f[0] = (float)delta / fB;
        f[1] = (float)(2 * xk - 1);
        f[2] = (float)diag[k] / fB;
        f[3] = (float)rowabs[k] / fB;
        f[4] = 2.0f * ((float)cnt[(int64_t)q * n + k] / fm) - 1.0f;
        f[5] = f[1] * f[4];
        f[6] = (float)(2 * bk - 1);
        f[7] = (float)r / fm;
        uint4 o;
        o.x = (uint32_t)(uint16_t)to_bf16(f[0]) | (uint32_t)(uint16_t)to_bf16(f[1]) << 16;
        o.y = (uint32_t)(uint16_t)to_bf16(f[2]) | (uint32_t)(uint16_t)to_bf16(f[3]) << 16;
        o.z = (uint32_t)(uint16_t)to_bf16(f[4]) | (uint32_t)(uint16_t)to_bf16(f[5]) << 16;
        o.w = (uint32_t)(uint16_t)to_bf16(f[6]) | (uint32_t)(uint16_t)to_bf16(f[7]) << 16;
        *(uint4 *)(feat + ((int64_t)cell * n + k) * NF) = o;
    }
}

// label[e][k] = 1 when bit k of vector e differs from the reference vector;
// with sym, from the reference or its complement, whichever is nearer in
// Hamming distance (ties: the reference).  One workgroup per vector.
__global__ __launch_bounds__(256) void k_labels(const uint64_t *__restrict__ bits, int n, int nw,
                                                const uint64_t *__restrict__ ref, int sym,
                                                uint8_t *__restrict__ label) {
    const int64_t e = blockIdx.x;
    const uint64_t *x = bits + e * nw;
    bool flip = false;
    if (sym) {
        __shared__ int part[256];
        int d = 0;
        for (int w = threadIdx.x; w < nw; w += blockDim.x) {
            uint64_t v = x[w] ^ ref[w];
            if (w == nw - 1 && (n & 63)) v &= (1ull << (n & 63)) - 1;
            d += __builtin_popcountll(v);
        }
        part[threadIdx.x] = d;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
            __syncthreads();
        }
        flip = 2 * part[0] > n;
    }
    for (int k = threadIdx.x; k < n; k += blockDim.x)
        label[e * n + k] = (uint8_t)((((x[k >> 6] ^ ref[k >> 6]) >> (k & 63)) & 1) ^ (flip ? 1 : 0));
}

__global__ void k_apply_op(int op, int n, int nw, int count, const uint64_t *__restrict__ parent,
                           const float *__restrict__ logits, uint64_t seed, uint32_t rd, uint32_t inst0,
                           uint64_t *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)count * nw) return;
    const int i = (int)(t / nw), w = (int)(t % nw);
    out[t] = mlp_op_word(op, parent[t], logits + (int64_t)i * n, n, w, seed, rd, inst0 + (uint32_t)i);
}

}  // namespace dabs

using namespace dabs;

struct dabs_mlp {
    float *par, *m, *v, *grad, *loss, *part;
    short *wbf;
    int step;
};

namespace dabs {

int mlp_pool_logits(const dabs_problem *p, const dabs_mlp *net, const uint64_t *pool_bits, int P, int m,
                    int *cnt, short *feat, float *logits, hipStream_t st, int *need) {
    const int n = p->n, nw = (n + 63) / 64;
    const int64_t pn = (int64_t)P * n;
    hipLaunchKernelGGL(k_pool_counts, dim3((unsigned)((pn + 255) / 256)), dim3(256), 0, st, pool_bits, P, m, n, nw,
                       cnt);
    HIP_OK(hipGetLastError());
    if (p->wtype == DABS_W_I16)
        hipLaunchKernelGGL(k_features<int16_t>, dim3(P * m), dim3(256), 0, st, (const int16_t *)p->W, p->diag,
                           p->rowabs, p->ld, n, nw, p->bound, pool_bits, m, cnt, feat, need);
    else
        hipLaunchKernelGGL(k_features<int32_t>, dim3(P * m), dim3(256), 0, st, (const int32_t *)p->W, p->diag,
                           p->rowabs, p->ld, n, nw, p->bound, pool_bits, m, cnt, feat, need);
    HIP_OK(hipGetLastError());
    if (net && logits) {
        const int64_t N = (int64_t)P * m * n, tiles = (N + 15) / 16;
        const unsigned blocks = (unsigned)(tiles < 8192 ? tiles : 8192);
        hipLaunchKernelGGL(k_mlp_fwd, dim3(blocks), dim3(64), 0, st, net->wbf, net->par, feat, N, logits);
        HIP_OK(hipGetLastError());
    }
    return DABS_OK;
}

}  // namespace dabs

extern "C" {

int dabs_mlp_create(const float *params_host, dabs_mlp **out) {
    if (!out) return dabs_fail(DABS_E_INVALID, "null output");
    dabs_mlp *s = new dabs_mlp();
    const size_t fb = sizeof(float) * NPAR;
    bool ok = hipMalloc(&s->par, fb) == hipSuccess && hipMalloc(&s->m, fb) == hipSuccess &&
              hipMalloc(&s->v, fb) == hipSuccess && hipMalloc(&s->grad, fb) == hipSuccess &&
              hipMalloc(&s->loss, sizeof(float)) == hipSuccess && hipMalloc(&s->wbf, sizeof(short) * NPAR) == hipSuccess &&
              hipMalloc(&s->part, sizeof(float) * (NPAR + 1) * GRAD_BLOCKS_MAX) == hipSuccess;
    if (ok) {
        ok = hipMemset(s->m, 0, fb) == hipSuccess && hipMemset(s->v, 0, fb) == hipSuccess &&
             hipMemset(s->grad, 0, fb) == hipSuccess;
        if (params_host) ok = ok && hipMemcpy(s->par, params_host, fb, hipMemcpyHostToDevice) == hipSuccess;
        else ok = ok && hipMemset(s->par, 0, fb) == hipSuccess;
    }
    if (ok) {
        hipLaunchKernelGGL(k_to_bf16, dim3((NPAR + 255) / 256), dim3(256), 0, 0, s->par, s->wbf);
        ok = hipGetLastError() == hipSuccess && hipDeviceSynchronize() == hipSuccess;
    }
    if (!ok) {
        dabs_mlp_destroy(s);
        return dabs_fail(DABS_E_NOMEM, "MLP allocation / upload failed");
    }
    *out = s;
    return DABS_OK;
}

int dabs_mlp_destroy(dabs_mlp *s) {
    if (!s) return DABS_OK;
    void *ptrs[] = {s->par, s->m, s->v, s->grad, s->loss, s->wbf, s->part};
    for (void *p : ptrs) (void)hipFree(p);
    delete s;
    return DABS_OK;
}

int dabs_mlp_params(const dabs_mlp *s, float *params_dev, void *stream) {
    if (!s || !params_dev) return dabs_fail(DABS_E_INVALID, "null argument");
    HIP_OK(hipMemcpyAsync(params_dev, s->par, sizeof(float) * NPAR, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return DABS_OK;
}

int dabs_mlp_pool_features(const dabs_problem *p, const uint64_t *pool_bits_dev, int32_t npools, int32_t capacity,
                           uint16_t *feat_dev, void *stream) {
    if (!p || !pool_bits_dev || !feat_dev) return dabs_fail(DABS_E_INVALID, "null argument");
    if (npools < 1 || capacity < 1) return dabs_fail(DABS_E_INVALID, "bad pool shape");
    if (p->n > 4096 || p->wtype == DABS_W_SPARSE)
        return dabs_fail(DABS_E_UNSUPPORTED, "features need a dense W with n <= 4096");
    int *cnt = nullptr;
    HIP_OK(hipMalloc((void **)&cnt, sizeof(int) * (size_t)npools * p->n));
    int r = mlp_pool_logits(p, nullptr, pool_bits_dev, npools, capacity, cnt, (short *)feat_dev, nullptr,
                            (hipStream_t)stream, nullptr);
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess && r == DABS_OK)
        r = dabs_fail(DABS_E_HIP, "feature kernels failed");
    (void)hipFree(cnt);
    return r;
}

}  // extern "C"

namespace dabs {
// Per-pool bit counts of dabs_mlp_pool_features_noalloc: one copy per GPU,
// held until the process ends.  Host code never passes this name to a kernel
// (on the host it is a stand-in, not a device address): it uses the address
// that hipGetSymbolAddress returned for the current device.
static __device__ __align__(256) int scratch[DABS_NOALLOC_COUNTS];
constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static int *g_scratch_ptr[NOALLOC_MAX_DEVICES];

// The device address of `scratch` on the current device, looked up once per
// device with that device current.
static int scratch_on_current_device(int **out) {
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return dabs_fail(DABS_E_UNSUPPORTED, "device %d above the %d devices the no-allocation call serves", dev,
                         NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return dabs_fail(DABS_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = (int *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return DABS_OK;
}
}  // namespace dabs

extern "C" {

int dabs_mlp_pool_features_noalloc(const dabs_problem *p, const uint64_t *pool_bits_dev, int32_t npools,
                                   int32_t capacity, uint16_t *feat_dev, void *stream) {
    if (!p || !pool_bits_dev || !feat_dev) return dabs_fail(DABS_E_INVALID, "null argument");
    if (npools < 1 || capacity < 1) return dabs_fail(DABS_E_INVALID, "bad pool shape");
    if (p->n > 4096 || p->wtype == DABS_W_SPARSE)
        return dabs_fail(DABS_E_UNSUPPORTED, "features need a dense W with n <= 4096");
    if ((int64_t)npools * p->n > DABS_NOALLOC_COUNTS)
        return dabs_fail(DABS_E_INVALID, "npools * n = %lld above the %d counts of the static buffer",
                         (long long)npools * p->n, DABS_NOALLOC_COUNTS);
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    if (dev != p->device)
        return dabs_fail(DABS_E_INVALID, "current device %d is not the problem's device %d", dev, p->device);
    int *cnt = nullptr;
    const int r = scratch_on_current_device(&cnt);
    if (r != DABS_OK) return r;
    // every count is written by k_pool_counts before k_features reads it, so
    // nothing has to be cleared between calls
    return mlp_pool_logits(p, nullptr, pool_bits_dev, npools, capacity, cnt, (short *)feat_dev, nullptr,
                           (hipStream_t)stream, nullptr);
}

int dabs_mlp_labels(const dabs_problem *p, const uint64_t *bits_dev, int64_t count, const uint64_t *ref_dev,
                    int32_t symmetric, uint8_t *labels_dev, void *stream) {
    if (!p || !bits_dev || !ref_dev || !labels_dev || count < 0 || count > 0x7fffffff)
        return dabs_fail(DABS_E_INVALID, "bad argument");
    if (count == 0) return DABS_OK;
    hipLaunchKernelGGL(k_labels, dim3((unsigned)count), dim3(256), 0, (hipStream_t)stream, bits_dev, p->n,
                       (p->n + 63) / 64, ref_dev, symmetric ? 1 : 0, labels_dev);
    HIP_OK(hipGetLastError());
    return DABS_OK;
}

int dabs_mlp_forward(const dabs_mlp *s, int64_t count, const uint16_t *feat_dev, float *logits_dev, void *stream) {
    if (!s || !feat_dev || !logits_dev || count < 0) return dabs_fail(DABS_E_INVALID, "bad argument");
    if (count == 0) return DABS_OK;
    const int64_t tiles = (count + 15) / 16;
    const unsigned blocks = (unsigned)(tiles < 8192 ? tiles : 8192);
    hipLaunchKernelGGL(k_mlp_fwd, dim3(blocks), dim3(64), 0, (hipStream_t)stream, s->wbf, s->par,
                       (const short *)feat_dev, count, logits_dev);
    HIP_OK(hipGetLastError());
    return DABS_OK;
}

int dabs_mlp_grad(dabs_mlp *s, int64_t count, const uint16_t *feat_dev, const uint8_t *labels_dev, float *grad_dev,
                  float *loss_dev, void *stream) {
    if (!s || !feat_dev || !labels_dev || count < 1) return dabs_fail(DABS_E_INVALID, "bad argument");
    hipStream_t st = (hipStream_t)stream;
    const int64_t tiles = (count + 15) / 16;
    const int blocks = (int)(tiles < GRAD_BLOCKS_MAX ? tiles : GRAD_BLOCKS_MAX);
    const float invN = (float)(1.0 / (double)count);
    hipLaunchKernelGGL(k_mlp_grad, dim3(blocks), dim3(64), 0, st, s->wbf, s->par, (const short *)feat_dev, labels_dev,
                       count, invN, s->part);
    HIP_OK(hipGetLastError());
    hipLaunchKernelGGL(k_mlp_reduce, dim3((NPAR + 1 + RED_COLS - 1) / RED_COLS), dim3(RED_COLS * RED_GROUPS), 0, st,
                       s->part, blocks, invN, s->grad, s->loss);
    HIP_OK(hipGetLastError());
    if (grad_dev) HIP_OK(hipMemcpyAsync(grad_dev, s->grad, sizeof(float) * NPAR, hipMemcpyDeviceToDevice, st));
    if (loss_dev) HIP_OK(hipMemcpyAsync(loss_dev, s->loss, sizeof(float), hipMemcpyDeviceToDevice, st));
    return DABS_OK;
}

int dabs_mlp_adam(dabs_mlp *s, float lr, void *stream) {
    if (!s || !(lr > 0.f)) return dabs_fail(DABS_E_INVALID, "bad argument");
    s->step++;
    const double c1 = 1.0 / (1.0 - pow((double)ADAM_B1, s->step)), c2 = 1.0 / (1.0 - pow((double)ADAM_B2, s->step));
    hipLaunchKernelGGL(k_adam, dim3((NPAR + 255) / 256), dim3(256), 0, (hipStream_t)stream, s->par, s->grad, s->m,
                       s->v, s->wbf, lr, (float)c1, (float)c2);
    HIP_OK(hipGetLastError());
    return DABS_OK;
}

int dabs_mlp_train_step(dabs_mlp *s, int64_t count, const uint16_t *feat_dev, const uint8_t *labels_dev, float lr,
                        float *loss_dev, void *stream) {
    const int r = dabs_mlp_grad(s, count, feat_dev, labels_dev, nullptr, loss_dev, stream);
    if (r != DABS_OK) return r;
    return dabs_mlp_adam(s, lr, stream);
}

int dabs_mlp_apply_op(int32_t op, int32_t n, int32_t count, const uint64_t *parent_dev, const float *logits_dev,
                      uint64_t seed, uint32_t round, uint32_t inst0, uint64_t *out_dev, void *stream) {
    if (op != DABS_OP_MLP_SEED && op != DABS_OP_MLP_MUTATE) return dabs_fail(DABS_E_INVALID, "not an MLP operation");
    if (n < 1 || count < 0 || !parent_dev || !logits_dev || !out_dev) return dabs_fail(DABS_E_INVALID, "bad argument");
    const int nw = (n + 63) / 64;
    const int64_t tot = (int64_t)count * nw;
    if (tot == 0) return DABS_OK;
    hipLaunchKernelGGL(k_apply_op, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, (hipStream_t)stream, op, n, nw,
                       count, parent_dev, logits_dev, seed, round, inst0, out_dev);
    HIP_OK(hipGetLastError());
    return DABS_OK;
}

}  // extern "C"
