// dabs_sparse.h -- one search instance per wavefront over a sparse W
// (Section III-A, B), for problems whose rows have few nonzeros: max-cut
// graphs of the G-set shape, Ising models of an annealer's hardware graph.
//
// The dense walker keeps its deltas in registers and reads a whole row of W
// per flip.  Here the deltas live in the wave's LDS and a flip of bit i
// touches only the nonzeros of row i (Eq. (4)): lane l takes nonzeros l,
// l + 64, ... of the row, each a 32-bit word (column in the low 16 bits,
// weight in the high 16), and adds 2 W_ik (1 - 2x_i)(1 - 2x_k) to the key of
// column k.  The per-flip W traffic drops from n sizeof(W) bytes to 4 bytes
// per nonzero.  The rules still compare every delta each iteration, as the
// paper's rules do; those passes read the keys from LDS, 16 bytes per lane
// per pass step, conflict-free.
//
// Layout and keys follow the dense walker with four elements per 16-byte
// piece: bit k = 256 s + 4 l + e sits in lane l, piece s, element e, local
// index j = 4 s + e, and its key word is
//     Delta_k 2^K + j + 2^29   (+ 2^31 while excluded: tabu, Straight's
//                               settled bits, padding),
// K = max(2, ceil(log2(4 S))) for S pieces per lane, so that within a lane
// keys order by (Delta, index) and key >> 2 orders by (Delta, piece) across
// lanes; the lowest lane among equal (Delta, piece) holds the lowest index.
// X and BEST are bit arrays in the same LDS region.  A workgroup is exactly
// one wavefront, so "barrier" is a wave-local LDS fence.
#pragma once
#include "dabs_device.h"

namespace dabs {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) uint32_t lds_u32;
typedef __attribute__((address_space(3))) u32x4 lds_u32x4;

// LDS words one sparse walker needs for S pieces per lane: keys, X bits,
// BEST bits.
__host__ __device__ constexpr int sparse_lds_words(int S) { return S * 256 + 2 * S * 8; }
// Most pieces per lane (n <= 256 S): 60 pieces, 15,360 bits, 65,280 bytes.
constexpr int SPARSE_MAX_SLOTS = 60;

__device__ __forceinline__ void lds_fence() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup"); }

struct SparseWalker {
    static constexpr int KBIAS = 1 << 29;
    static constexpr uint32_t XBIT = 0x80000000u;
    static constexpr uint32_t KB_PAD = 0xFFFFFFF0u;
    static constexpr uint32_t UOUT = 0xFFFFFFF0u;
    static constexpr int BIAS_W = KBIAS >> 2;
    static constexpr int NONE_W = (1 << 30) >> 2;

    lds_u32 *K;            // keys [S][64 lanes][4]
    lds_u32 *XW;           // X bits, bit k in word k / 32
    lds_u32 *BW;           // BEST bits
    const int32_t *rp;     // off-diagonal row starts [n + 1]
    const uint32_t *nz;    // off-diagonal nonzeros (column | weight << 16)
    int n, S, KB, SB, lane, nxw;
    int64_t E, Eb;
    int ring;              // tabu ring: lane r holds the bit flipped at iteration r mod 32
    uint32_t kminU, kminM;
    int mU, mM, mX;
    int64_t target;
    unsigned long long *hit;
    unsigned long long t0;
    bool hit_done;
    int *trace;
    int trace_cap;
    int flips;
    uint64_t seed;
    uint32_t inst;

    // ---------------------------------------------------------------- decoding
    static __device__ __forceinline__ int wv(uint32_t u) { return (int)(u >> 2); }
    static __device__ __forceinline__ bool none(int m) { return m >= NONE_W; }
    __device__ __forceinline__ int dlt_w(int m) const { return (m - BIAS_W) >> SB; }
    __device__ __forceinline__ int dlt_k(uint32_t k) const { return ((int)(k & 0x7FFFFFFFu) - KBIAS) >> KB; }
    static __device__ __forceinline__ int local_of(int i) { return ((i >> 8) << 2) | (i & 3); }
    __device__ __forceinline__ u32x4 piece(int s) const { return ((const lds_u32x4 *)K)[s * 64 + lane]; }
    __device__ __forceinline__ void set_piece(int s, u32x4 q) { ((lds_u32x4 *)K)[s * 64 + lane] = q; }
    __device__ __forceinline__ int xbit(int k) const { return (int)((XW[k >> 5] >> (k & 31)) & 1u); }

    // ------------------------------------------------------------- set up
    // X := x (packed words), deltas from scratch: the local field
    // f_k = W_kk + 2 sum_{j != k} W_kj x_j of every bit from its row, Delta_k
    // = (1 - 2x_k) f_k (Eq. (3)) and E = sum_k x_k (W_kk + f_k) / 2.
    __device__ void setup(lds_u32 *smem, const int32_t *diag, const int32_t *rp_, const uint32_t *nz_, int n_,
                          int S_, uint64_t seed_, uint32_t inst_, const uint64_t *x) {
        K = smem;
        XW = smem + S_ * 256;
        BW = XW + S_ * 8;
        rp = rp_; nz = nz_; n = n_; S = S_; seed = seed_; inst = inst_;
        lane = lane_id();
        int kb = 2;
        while ((1 << kb) < 4 * S) ++kb;
        KB = kb;
        SB = kb - 2;
        nxw = S * 8;
        const int nw = (n + 63) / 64;
        for (int w = lane; w < nxw; w += WAVE) {
            const int w64 = w >> 1;
            uint64_t v = (x && w64 < nw) ? x[w64] : 0ull;
            if (w64 == nw - 1 && (n & 63)) v &= (1ull << (n & 63)) - 1;   // bits >= n are ignored
            XW[w] = (uint32_t)(w & 1 ? v >> 32 : v);
            BW[w] = 0;
        }
        lds_fence();
        long long e2 = 0;
        for (int s = 0; s < S; ++s) {
            u32x4 q;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = s * 256 + lane * 4 + e;
                uint32_t key = KB_PAD;
                if (k < n) {
                    int f = diag[k];
                    for (int t = rp[k]; t < rp[k + 1]; ++t) {
                        const uint32_t w = nz[t];
                        if (xbit((int)(w & 0xFFFFu))) f += 2 * ((int)w >> 16);
                    }
                    const int xk = xbit(k);
                    if (xk) e2 += (long long)diag[k] + f;
                    key = (uint32_t)((xk ? -f : f) * (1 << KB) + (4 * s + e) + KBIAS);
                }
                q[e] = key;
            }
            set_piece(s, q);
        }
        E = wave_sum64(e2) / 2;
        lds_fence();
        Eb = E;
        ring = -1;
        hit = nullptr; hit_done = true; target = 0; t0 = 0;
        trace = nullptr; trace_cap = 0; flips = 0;
    }

    __device__ void store_bits(const lds_u32 *bits, uint64_t *out) const {
        const int nw = (n + 63) / 64;
        for (int w = lane; w < nw; w += WAVE) out[w] = ((uint64_t)bits[2 * w + 1] << 32) | bits[2 * w];
    }
    __device__ void store_delta(int *out) const {
        for (int s = 0; s < S; ++s) {
            const u32x4 q = piece(s);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = s * 256 + lane * 4 + e;
                if (k < n) out[k] = dlt_k(q[e]);
            }
        }
    }

    // ------------------------------------------------------------- reductions
    // least word of all bits from a lane's unsigned and signed minima
    static __device__ __forceinline__ uint32_t unmask(uint32_t um, int sm) {
        return min(um, (uint32_t)sm & 0x7FFFFFFFu);
    }
    __device__ __forceinline__ uint32_t lane_umin() const {
        uint32_t m = UOUT;
        for (int s = 0; s < S; ++s) {
            const u32x4 q = piece(s);
            m = min(m, min(min(q[0], q[1]), min(q[2], q[3])));
        }
        return m;
    }
    __device__ __forceinline__ void lane_umin_smin(uint32_t &um, int &sm) const {
        um = UOUT;
        sm = 0x7FFFFFFF;
        for (int s = 0; s < S; ++s) {
            const u32x4 q = piece(s);
            um = min(um, min(min(q[0], q[1]), min(q[2], q[3])));
            sm = min(sm, min(min((int)q[0], (int)q[1]), min((int)q[2], (int)q[3])));
        }
    }

    struct Sel { int d, i, j, L; };

    // Wave argmin of per-lane least words: lowest (delta, global index).
    __device__ __forceinline__ Sel argmin_from(uint32_t kmin, int m) const {
        const uint64_t bal = ballot(wv(kmin) == m);
        const int L = (int)__builtin_ctzll(bal);
        const int kl = readlane((int)kmin, L);
        const int slot = m & ((1 << SB) - 1);
        Sel r;
        r.d = dlt_w(m);
        r.j = (slot << 2) | (kl & 3);
        r.i = slot * 256 + L * 4 + (kl & 3);
        r.L = L;
        return r;
    }
    __device__ __forceinline__ Sel sel_of(int i) const {
        Sel s;
        s.i = i;
        s.j = local_of(i);
        s.L = (i >> 2) & 63;
        s.d = dlt_k(K[i]);
        return s;
    }

    __device__ __forceinline__ void note_best() {
        if (!hit_done && Eb <= target) {
            hit_done = true;
            const unsigned long long now = __builtin_amdgcn_s_memrealtime();
            if (lane == 0) atomicMin(hit, now - t0);
        }
    }

    // Step 1: BEST <- best 1-bit neighbour when strictly better than E(BEST).
    __device__ __forceinline__ void step1() {
        const int d = dlt_w(mU);
        if (E + d < Eb) {
            const Sel s = argmin_from(kminU, mU);
            Eb = E + d;
            const int wi = s.i >> 5;
            const uint32_t bi = 1u << (s.i & 31);
            for (int w = lane; w < nxw; w += WAVE) BW[w] = XW[w] ^ (w == wi ? bi : 0u);
            lds_fence();
            note_best();
        }
    }
    __device__ __forceinline__ void refresh() {
        kminU = lane_umin();
        mU = wave_min(wv(kminU));
        step1();
    }
    __device__ __forceinline__ void refresh_all() {
        uint32_t um;
        int sm;
        lane_umin_smin(um, sm);
        kminU = unmask(um, sm);
        mU = wave_min(wv(kminU));
        step1();
    }
    __device__ __forceinline__ void refresh_dom() {
        uint32_t um;
        int sm;
        lane_umin_smin(um, sm);
        kminM = um;
        kminU = unmask(um, sm);
        wave_min2(wv(kminU), wv(kminM), mU, mM);
        step1();
    }
    __device__ __forceinline__ void dom_minmax() {
        uint32_t um = UOUT;
        int sm = 0x7FFFFFFF, sx = (int)0x80000000;
        for (int s = 0; s < S; ++s) {
            const u32x4 q = piece(s);
            um = min(um, min(min(q[0], q[1]), min(q[2], q[3])));
            sm = min(sm, min(min((int)q[0], (int)q[1]), min((int)q[2], (int)q[3])));
            sx = max(sx, max(max((int)q[0], (int)q[1]), max((int)q[2], (int)q[3])));
        }
        kminM = um;
        kminU = unmask(um, sm);
        wave_minmin_max(wv(kminU), wv(kminM), sx, mU, mM, mX);
    }

    __device__ __forceinline__ void begin() {
        for (int w = lane; w < nxw; w += WAVE) BW[w] = XW[w];
        lds_fence();
        Eb = E;
        note_best();
        refresh();
    }

    // Step 3: flip bit i (uniform) with delta d.  Eq. (4) on the nonzeros of
    // row i, Eq. (5) on the bit's own key (the exclusion bit survives: 2 2^31
    // vanishes mod 2^32), X updated.
    __device__ __forceinline__ void flip_core(const Sel &s0) {
        int i = __builtin_amdgcn_readfirstlane(s0.i);
        const int d = __builtin_amdgcn_readfirstlane(s0.d);
        if ((unsigned)i >= (unsigned)n) i = 0;     // never index outside the rows (a selection bug shows in parity)
        E += d;
        const int yi = xbit(i) ? -1 : 1;
        const int p1 = rp[i + 1];
        for (int t = rp[i] + lane; t < p1; t += WAVE) {
            const uint32_t w = nz[t];
            const int c = (int)(w & 0xFFFFu);
            const int yc = xbit(c) ? -yi : yi;
            K[c] = K[c] + (uint32_t)(2 * ((int)w >> 16) * yc) * (1u << KB);
        }
        lds_fence();
        if (lane == 0) {
            K[i] = (uint32_t)(2 * local_of(i) + 2 * KBIAS) - K[i];
            XW[i >> 5] ^= 1u << (i & 31);
        }
        lds_fence();
        if (trace && flips < trace_cap && lane == 0) trace[flips] = i;
        flips++;
    }
    __device__ __forceinline__ void flip(const Sel &s) {
        flip_core(s);
        refresh();
    }

    // ------------------------------------------------------------- exclusions
    __device__ __forceinline__ void mark(int i) {
        if (lane == 0) K[i] |= XBIT;
        lds_fence();
    }
    __device__ __forceinline__ void unmark(int i) {
        if (lane == 0) K[i] &= ~XBIT;
        lds_fence();
    }
    __device__ __forceinline__ void reset_marks() {
        for (int s = 0; s < S; ++s) {
            u32x4 q = piece(s);
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (s * 256 + lane * 4 + e < n) q[e] &= 0x7FFFFFFFu;
            set_piece(s, q);
        }
        lds_fence();
    }
    // Tabu (R11) of bit i flipped at iteration t (see the dense walker).
    __device__ __forceinline__ void tabu_mark(int i, int t, int tau, bool maybe_marked) {
        if (tau <= 0) return;
        if (maybe_marked && (K[i] & XBIT)) {
            for (int u = t - tau; u < t; ++u)
                if (u >= 1 && readlane(ring, u & 31) == i) ring = lane == (u & 31) ? -1 : ring;
        }
        mark(i);
        ring = lane == (t & 31) ? i : ring;
    }
    __device__ __forceinline__ void tabu_release(int t, int tau) {
        const int t0r = t - tau - 1;
        if (tau > 0 && t0r >= 1) {
            const int e = readlane(ring, t0r & 31);
            if (e >= 0) unmark(e);
        }
    }

    // ------------------------------------------------------------- rules
    __device__ int phase_greedy(int cap) {
        if (cap <= 0) cap = 64 * n;
        int f = 0;
        while (dlt_w(mU) < 0 && f < cap) {
            flip(argmin_from(kminU, mU));
            f++;
        }
        return f;
    }

    __device__ int phase_straight(const uint64_t *target_bits) {
        const int nw = (n + 63) / 64;
        int hd = 0;
        for (int s = 0; s < S; ++s) {
            u32x4 q = piece(s);
            const int k0 = s * 256 + lane * 4;
            const uint64_t word = (k0 >> 6) < nw ? target_bits[k0 >> 6] : 0ull;
            const uint32_t tb = (uint32_t)(word >> (k0 & 63)) & 0xFu;
            const uint32_t xb = (XW[k0 >> 5] >> (k0 & 31)) & 0xFu;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const bool dif = k0 + e < n && (((tb ^ xb) >> e) & 1u);
                q[e] = dif ? (q[e] & 0x7FFFFFFFu) : (q[e] | XBIT);
                hd += dif;
            }
            set_piece(s, q);
        }
        lds_fence();
        hd = (int)wave_sum64(hd);
        kminM = lane_umin();
        mM = wave_min(wv(kminM));
        int f = 0;
        for (; f < hd; ++f) {
            const Sel s = argmin_from(kminM, mM);
            mark(__builtin_amdgcn_readfirstlane(s.i));
            flip_core(s);
            refresh_dom();
        }
        reset_marks();
        return f;
    }

    __device__ int phase_tabu_greedy(int T, int tau) {
        kminM = kminU;
        mM = mU;
        for (int t = 1; t <= T; ++t) {
            const bool emp = none(mM);
            const Sel s = emp ? argmin_from(kminU, mU) : argmin_from(kminM, mM);
            const int i = __builtin_amdgcn_readfirstlane(s.i);
            tabu_mark(i, t, tau, emp);
            flip_core(s);
            tabu_release(t + 1, tau);
            refresh_dom();
        }
        reset_marks();
        return T;
    }

    __device__ int phase_cyclicmin(int T, int tau) {
        int pos = 0;
        FracStep fs;
        fs.init((uint32_t)T);
        for (int t = 1; t <= T; ++t) {
            fs.next();
            int w;
            if (t >= T) {
                w = n;
            } else {
                const int c = n < 32 ? n : 32;
                const int64_t ww = (int64_t)(((uint64_t)n * cube_frac(fs.q)) >> 32);
                w = ww < c ? c : (ww > n ? n : (int)ww);
            }
            tabu_release(t, tau);
            const bool wrap = pos + w > n;
            const int lo = wrap ? pos + w - n : pos;
            const uint32_t span = wrap ? (uint32_t)(n - w) : (uint32_t)w;
            uint32_t km = UOUT, kw = UOUT;
            for (int s = 0; s < S; ++s) {
                const u32x4 q = piece(s);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const uint32_t off = (uint32_t)(s * 256 + lane * 4 + e - lo);
                    const bool in = wrap ? (off >= span) : (off < span);
                    km = min(km, in ? q[e] : UOUT);
                    kw = min(kw, in ? (q[e] & 0x7FFFFFFFu) : UOUT);
                }
            }
            const int m = wave_min(wv(km));
            const bool emp = none(m);
            const Sel s = emp ? argmin_from(kw, wave_min(wv(kw))) : argmin_from(km, m);
            const int i = __builtin_amdgcn_readfirstlane(s.i);
            flip_core(s);
            refresh_all();
            tabu_mark(i, t, tau, emp);
            pos = (pos + w) % n;
        }
        reset_marks();
        return T;
    }

    // Position of set bit number k of a 4-bit mask.
    static __device__ __forceinline__ int kth_bit4(uint32_t b, uint32_t k) {
        const uint32_t c2 = (uint32_t)__builtin_popcount(b & 0x3u);
        const bool up2 = k >= c2;
        k -= up2 ? c2 : 0u;
        b >>= up2 ? 2 : 0;
        return (up2 ? 2 : 0) + (k >= (b & 1u) ? 1 : 0);
    }

    // Candidates: unexcluded keys (IGN: exclusions ignored, padding still out)
    // <= dk.  r = floor(v count / 2^32) and the r-th candidate in increasing
    // bit index (piece, then lane, then element) is returned.
    template <bool IGN>
    __device__ Sel pick_rth(int dk, uint32_t v) {
        const uint32_t lim = (uint32_t)(dk + KBIAS);
        auto cand = [&](uint32_t key, int k) {
            const uint32_t kk = IGN ? (key & 0x7FFFFFFFu) : key;
            return k < n && kk <= lim;
        };
        uint32_t total = 0;
        int cnt = 0;                      // lane s: candidates of piece s
        for (int s = 0; s < S; ++s) {
            const u32x4 q = piece(s);
            uint32_t c = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) c += (uint32_t)__builtin_popcountll(ballot(cand(q[e], s * 256 + lane * 4 + e)));
            cnt = lane == s ? (int)c : cnt;
            total += c;
        }
        if (total == 0) return argmin_from(kminU, mU);   // cannot happen: the domain minimum qualifies
        const uint32_t r = scale32(v, total);
        // inclusive prefix of the per-piece counts over lanes
        int incl = cnt;
        for (int o = 1; o < WAVE; o <<= 1) {
            const int u = __shfl_up(incl, o, WAVE);
            incl += lane >= o ? u : 0;
        }
        const int slot = (int)__builtin_ctzll(ballot((uint32_t)incl > r));
        const uint32_t before = slot > 0 ? (uint32_t)readlane(incl, slot - 1) : 0u;
        const uint32_t rr = r - before;
        const u32x4 q = piece(slot);
        uint32_t excl = 0, cb = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const bool ce = cand(q[e], slot * 256 + lane * 4 + e);
            const uint64_t cm = ballot(ce);
            cb |= ce ? (1u << e) : 0u;
            excl = __builtin_amdgcn_mbcnt_hi((uint32_t)(cm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)cm, excl));
        }
        const uint64_t le = ballot(excl <= rr);
        const int L = 63 - __builtin_clzll(le | 1ull);
        const int left = (int)(rr - (uint32_t)readlane((int)excl, L));
        const int e_sel = __builtin_amdgcn_readfirstlane(kth_bit4((uint32_t)readlane((int)cb, L), (uint32_t)left));
        return sel_of(slot * 256 + L * 4 + e_sel);
    }

    __device__ int phase_maxmin(int T, int tau, uint32_t ph) {
        dom_minmax();
        FracStep fs;
        fs.init((uint32_t)T);
        R4 rv = {{0u, 0u, 0u, 0u}};
        int cbase = -64;
        for (int t = 1; t <= T; ++t) {
            fs.next();
            const uint64_t cf = cube_frac(fs.rest());
            const int c = (t - 1) >> 1;
            if (c >= cbase + 64) {
                cbase += 64;
                rv = philox((uint32_t)(cbase + lane), inst, ph, (uint32_t)TAG_MAXMIN << 24, seed);
            }
            const bool second = (t - 1) & 1;
            const uint32_t u = (uint32_t)readlane((int)(second ? rv.w[2] : rv.w[0]), c - cbase);
            const uint32_t v = (uint32_t)readlane((int)(second ? rv.w[3] : rv.w[1]), c - cbase);
            const bool ign = none(mM);
            if (ign) {
                mM = mU;
                int kx = (int)0x80000000;
                for (int s = 0; s < S; ++s) {
                    const u32x4 q = piece(s);
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        kx = max(kx, s * 256 + lane * 4 + e < n ? (int)(q[e] & 0x7FFFFFFFu) : (int)0x80000000);
                }
                mX = wave_max(kx);
            }
            const int mind = dlt_w(mM);
            const int maxd = (mX - KBIAS) >> KB;
            const uint64_t span = ((uint64_t)(uint32_t)(maxd - mind) * cf) >> 32;
            const int d = mind + (int)(((uint64_t)u * (span + 1)) >> 32);
            const int dk = d * (1 << KB) + ((1 << KB) - 1);
            const Sel s = ign ? pick_rth<true>(dk, v) : pick_rth<false>(dk, v);
            tabu_mark(s.i, t, tau, ign);
            flip_core(s);
            tabu_release(t + 1, tau);
            dom_minmax();
            step1();
        }
        reset_marks();
        return T;
    }

    __device__ int phase_positivemin(int T, int tau, uint32_t ph) {
        const uint32_t C = (uint32_t)KBIAS + (1u << KB);
        const bool may_empty = n <= tau;
        const int d_top = (1 << (29 - KB)) - 2;
        R4 rv = {{0u, 0u, 0u, 0u}};
        int cbase = -64;
        for (int t = 1; t <= T; ++t) {
            tabu_release(t, tau);
            bool ign = false;
            if (may_empty) ign = none(wave_min(wv(lane_umin())));
            uint32_t kp = UOUT;
            for (int s = 0; s < S; ++s) {
                const u32x4 q = piece(s);
#pragma unroll
                for (int e = 0; e < 4; ++e) kp = min(kp, (ign ? (q[e] & 0x7FFFFFFFu) : q[e]) - C);
            }
            const int mw = wave_min(wv(kp));
            const int d = none(mw) ? d_top : (mw >> SB) + 1;
            const int dk = d * (1 << KB) + ((1 << KB) - 1);
            const int c = (t - 1) >> 2;
            if (c >= cbase + 64) {
                cbase += 64;
                rv = philox((uint32_t)(cbase + lane), inst, ph, (uint32_t)TAG_POSMIN << 24, seed);
            }
            const int q4 = (t - 1) & 3;
            const uint32_t wq = q4 == 0 ? rv.w[0] : (q4 == 1 ? rv.w[1] : (q4 == 2 ? rv.w[2] : rv.w[3]));
            const uint32_t u = (uint32_t)readlane((int)wq, c - cbase);
            const Sel s = ign ? pick_rth<true>(dk, u) : pick_rth<false>(dk, u);
            const int i = __builtin_amdgcn_readfirstlane(s.i);
            flip_core(s);
            refresh_all();
            tabu_mark(i, t, tau, ign);
        }
        reset_marks();
        return T;
    }

    // RandomMin (Section III-A.5): the byte of bit k is byte k mod 16 of the
    // draw (t, instance, phase, tag | k / 16); lane l's four bits of piece s
    // are bytes 0..3 of word l mod 4 of the draw for group 16 s + l / 4.
    __device__ int phase_randommin(int T, int tau, uint32_t ph) {
        FracStep fs;
        fs.init((uint32_t)T);
        const uint32_t tag = (uint32_t)TAG_RANDMIN << 24;
        const int wsel = lane & 3;
        for (int t = 1; t <= T; ++t) {
            fs.next();
            int qt;
            if (t >= T) {
                qt = 256;
            } else {
                const int qq = (int)(cube_frac(fs.q) >> 24);
                const int qmin = (8192 + n - 1) / n;
                qt = qq < qmin ? qmin : (qq > 256 ? 256 : qq);
            }
            tabu_release(t, tau);
            uint32_t kr = UOUT;
            for (int s = 0; s < S; ++s) {
                const R4 r = philox((uint32_t)t, inst, ph, tag | (uint32_t)(s * 16 + (lane >> 2)), seed);
                const uint32_t word = wsel == 0 ? r.w[0] : (wsel == 1 ? r.w[1] : (wsel == 2 ? r.w[2] : r.w[3]));
                const u32x4 q = piece(s);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int byte = (int)((word >> (8 * e)) & 0xFFu);
                    kr = min(kr, byte < qt ? q[e] : UOUT);
                }
            }
            const int m = wave_min(wv(kr));
            bool emp = false;
            Sel s;
            if (!none(m)) {
                s = argmin_from(kr, m);
            } else {
                const uint32_t km = lane_umin();
                const int mm = wave_min(wv(km));
                emp = none(mm);
                s = emp ? argmin_from(kminU, mU) : argmin_from(km, mm);
            }
            const int i = __builtin_amdgcn_readfirstlane(s.i);
            flip_core(s);
            refresh_all();
            tabu_mark(i, t, tau, emp);
        }
        reset_marks();
        return T;
    }

    __device__ int phase_twoneighbor() {
        flip(sel_of(0));
        for (int k = 1; k < n; ++k) {
            flip(sel_of(k));
            flip(sel_of(k - 1));
        }
        return 2 * n - 1;
    }

    __device__ int run_phase(int rule, int T, int tau, uint32_t ph, const uint64_t *target_bits, int cap) {
        tau = tau < 0 ? 0 : (tau > TAU_MAX ? TAU_MAX : tau);
        int f = 0;
        if (rule == GREEDY) f = phase_greedy(cap);
        if (rule == STRAIGHT) f = phase_straight(target_bits);
        if (rule == MAXMIN) f = phase_maxmin(T, tau, ph);
        if (rule == CYCLICMIN) f = phase_cyclicmin(T, tau);
        if (rule == RANDOMMIN) f = phase_randommin(T, tau, ph);
        if (rule == POSITIVEMIN) f = phase_positivemin(T, tau, ph);
        if (rule == TWONEIGHBOR) f = phase_twoneighbor();
        if (rule == TABU_GREEDY) f = phase_tabu_greedy(T, tau);
        return f;
    }

    // Batch search (Section III-B), as in the dense walker.
    __device__ int batch(const uint64_t *target_bits, int rule, int T, int Bn, int tau, uint32_t &ph, int cap) {
        begin();
        const bool main_ok = rule >= MAXMIN && rule <= TWONEIGHBOR;
        int f = 0;
        for (int k = 0;; ++k) {
            const int r = k == 0 ? STRAIGHT : ((k & 1) ? GREEDY : rule);
            f += run_phase(r, T, tau, ph, target_bits, cap);
            if (k > 0 && !(k & 1)) ph++;
            if (k & 1) {
                if (f >= Bn || !main_ok || (rule == TWONEIGHBOR && k > 1)) break;
            }
        }
        return f;
    }
};

}  // namespace dabs
