// dabs_walker.h -- one search instance per wavefront (Section III-A, B).
//
// The walker keeps X, the deltas, BEST and the energies of one instance in
// the registers of one wave (layout in dabs_device.h).  Every element holds
// one word, its biased key
//     kb_j = Delta_j 2^KB + j + 2^29  (+ 2^31 while the element is excluded),
// which orders the elements of a lane by (Delta, index) and is updated in
// place on every flip (Eq. (4)): kb_j += 2 (1 - 2 x_i)(1 - 2 x_j) W_ij 2^KB,
// one v_dot2 (int16) or 24-bit multiply-add (int32) per element with a
// per-element multiplier word mul_j = (1 - 2 x_j) 2^(KB+1).
//
// Exclusions (tabu, Straight's settled bits, padding) are the sign bit, so
// that the rule domains cost no per-element test:
//   least key of the domain  = unsigned minimum (excluded words are >= 2^31);
//   greatest key of the domain = signed maximum (excluded words are negative);
//   least key of all bits     = per lane min(unsigned min, signed min & ~2^31),
//     since the signed minimum of a lane is its least excluded word when it
//     has one.
// Valid keys lie in (-2^29, 2^29) (|Delta| <= 2^(29-KB) - 2, checked at the
// problem load), so valid
// unexcluded words lie in (0, 2^30) and anything at or above 2^30 is "none".
// The tabu of R11 (bit flipped at iteration t excluded at t+1 .. t+tau) is
// set on the flip and cleared tau+1 iterations later from a 32-entry ring
// held in one register (lane r: the bit flipped at iteration t = r mod 32).
// Step 1 (BEST) runs at every visited state.
#pragma once
#include "dabs_device.h"

namespace dabs {

constexpr int KBIAS = 1 << 29;
constexpr uint32_t XBIT = 0x80000000u;
// padding element: excluded, and above every key once the sign is cleared
constexpr int KB_PAD = (int)0xFFFFFFF0u;
// masked-out value in unsigned minima (not 0xFFFFFFFF: with the all-ones
// value the compiler turns select + min3 into a min followed by a select)
constexpr uint32_t UOUT = 0xFFFFFFF0u;

// N ints held in registers and indexed by a wave-uniform value without going
// through memory: a uniform dynamic index becomes s_set_gpr_idx on a vector
// of at most 32 registers (a larger vector would be indexed through scratch
// memory, the whole vector stored and reloaded), so 64 elements are two
// halves chosen by a uniform test.  The halves are the kernel's own local
// vectors (which keeps them in registers); this refers to them.  Indices are
// masked into range so that a speculated access of the other half stays
// inside its vector.
template <int N>
struct RegVec {
    static constexpr int H = N > 32 ? 32 : N;
    typedef int vh __attribute__((ext_vector_type(H)));
    vh &lo, &hi;    // hi is used only when N > 32
    __device__ __forceinline__ RegVec(vh &l, vh &h) : lo(l), hi(h) {}
    // (with a run-time index both halves are read and the value chosen, one
    // half's value made opaque by an empty asm, and a store goes through one
    // of two branches kept apart by an empty asm: a load or store through a
    // pointer that selects between the halves would keep both in memory)
    __device__ __forceinline__ int operator[](int j) const {
        if constexpr (N <= 32) {
            return lo[j];
        } else {
            if (__builtin_constant_p(j)) return j < H ? lo[j & (H - 1)] : hi[j & (H - 1)];
            const int a = lo[j & (H - 1)];
            int b = hi[j & (H - 1)];
            asm volatile("" : "+v"(b));
            return j < H ? a : b;
        }
    }
    __device__ __forceinline__ void set(int j, int v) {
        if constexpr (N <= 32) {
            lo[j] = v;
        } else if (__builtin_constant_p(j)) {
            if (j < H) lo[j & (H - 1)] = v;
            else hi[j & (H - 1)] = v;
        } else {
            if (j < H) {
                lo[j & (H - 1)] = v;
            } else {
                hi[j & (H - 1)] = v;
                asm volatile("");
            }
        }
    }
};

template <bool NARROW> struct MaskOf { typedef uint64_t type; };
template <> struct MaskOf<true> { typedef uint32_t type; };
__device__ __forceinline__ uint32_t lane_mask(uint32_t v, int l) { return (uint32_t)readlane((int)v, l); }
__device__ __forceinline__ uint64_t lane_mask(uint64_t v, int l) { return readlane64(v, l); }

struct Sel {
    int d;   // delta of the selected bit
    int i;   // global bit index
    int L;   // lane holding it
    int j;   // local index inside that lane
};

// The selection is wave-uniform by construction; saying so keeps it in SGPRs
// (dynamic register indexing by a VGPR value would become a waterfall loop).
__device__ __forceinline__ Sel uniform(Sel s) {
    s.d = __builtin_amdgcn_readfirstlane(s.d);
    s.i = __builtin_amdgcn_readfirstlane(s.i);
    s.L = __builtin_amdgcn_readfirstlane(s.L);
    s.j = __builtin_amdgcn_readfirstlane(s.j);
    return s;
}

// LDSW: the rows come from a copy of W in the workgroup's LDS (problems of
// one slot whose W fits, see lds_w_bytes) instead of global memory / L2.
template <typename WT, int SLOTS, bool LDSW = false>
struct Walker {
    static_assert(!LDSW || SLOTS == 1, "LDS rows serve problems of one slot");
    static constexpr int V = 16 / (int)sizeof(WT);
    static constexpr int LOGV = V == 8 ? 3 : 2;
    static constexpr int EPL = V * SLOTS;
    static constexpr int KB = clog2(EPL) < LOGV ? LOGV : clog2(EPL);
    // largest |delta| the problem load admits at this key shift; PositiveMin's
    // threshold when no delta of its domain is positive (every key qualifies)
    static constexpr int D_TOP = (1 << (29 - KB)) - 2;
    static constexpr int SB = KB - LOGV;
    static constexpr int SPAN = WAVE * V;   // bits covered by one slot
    // wave reductions run on kb >> LOGV (key order down to the slot; the lane
    // comes from a ballot and the sub-index from that lane's word)
    static constexpr int BIAS_W = KBIAS >> LOGV;
    static constexpr int NONE_W = (1 << 30) >> LOGV;
    // multiplier of an element with x = 0, and the mask that negates one
    // (int16: the element's 16-bit half of the dot2 operand, the other half 0)
    static constexpr int MUL0 = 1 << (KB + 1);
    static constexpr uint32_t MFLIP =
        sizeof(WT) == 2 ? ((0x10000u - (1u << (KB + 2))) & 0xFFFFu) : (uint32_t)(-(1 << (KB + 2)));
    typedef typename RegVec<EPL>::vh vecH;   // the kernel's local vectors (element j = s*V + e)
    RegVec<EPL> kb, mul;

    __device__ __forceinline__ Walker(vecH &kb0, vecH &kb1, vecH &mul0, vecH &mul1)
        : kb(kb0, kb1), mul(mul0, mul1) {}

    const WT *__restrict__ W;
    int64_t ld;
    int n, lane;
    // per-lane bit masks over the lane's EPL elements: one register when they fit
    typedef typename MaskOf<(EPL <= 32)>::type mask_t;
    static constexpr mask_t ONE = 1;
    mask_t xb, bb;            // X and BEST bits of this lane (bit j)
    mask_t vb;                // valid-element bits of this lane (bit j set iff bit index < n)
    int64_t E, Eb;
    int ring;                 // tabu ring (see above); -1: nothing to clear
    // Step 1 state of the current vector: per-lane least word over all bits
    // and its wave minimum (as kb >> LOGV)
    uint32_t kminU;
    int mU;
    // Step 1 can only change BEST when E + min_k Delta_k < E(BEST).  lbU is a
    // lower bound of min_k Delta_k at the current vector: exact after a
    // reduction over all bits, and after a flip of bit i with delta d at
    // least min(lbU - 2 max|W_ik|, -d) (every other delta moves by
    // 2 |W_ik| at most, the flipped one becomes -d).  While E + lbU >= E(BEST)
    // the reduction over all bits is not made; exU says whether kminU / mU
    // describe the current vector.
    int64_t lbU;
    bool exU;
    int wmax2;                // 2 max_{j != k} |W_kj|
    // time to target
    int64_t target;
    unsigned long long *hit;
    unsigned long long t0;
    bool hit_done;
    // trace
    int *trace;
    int trace_cap;
    int flips;
    // generator
    uint64_t seed;
    uint32_t inst;

    // ---------------------------------------------------------------- layout
    static __device__ __forceinline__ int lidx_to_lane(int i) { return (i >> LOGV) & (WAVE - 1); }
    static __device__ __forceinline__ int lidx_of(int i) { return ((i / SPAN) << LOGV) | (i & (V - 1)); }
    __device__ __forceinline__ int gidx(int s, int e) const { return s * SPAN + lane * V + e; }

    template <class F>
    __device__ __forceinline__ void at_slot(int s, F f) {
#pragma unroll
        for (int ss = 0; ss < SLOTS; ++ss)
            if (ss == s) f(ss);
    }

    // ---------------------------------------------------------------- decoding
    static __device__ __forceinline__ int wv(uint32_t u) { return (int)(u >> LOGV); }
    static __device__ __forceinline__ bool none(int m) { return m >= NONE_W; }
    // delta of a wave value / of an element's word
    static __device__ __forceinline__ int dlt_w(int m) { return (m - BIAS_W) >> SB; }
    static __device__ __forceinline__ int dlt_k(int k) { return ((k & 0x7FFFFFFF) - KBIAS) >> KB; }

    // ------------------------------------------------------------- set up
    __device__ __forceinline__ void setup(const WT *Wp, const int *diag, int64_t ld_, int n_, uint64_t seed_,
                                          uint32_t inst_, int wmax2_) {
        W = Wp; ld = ld_; n = n_; seed = seed_; inst = inst_; wmax2 = wmax2_;
        lbU = 0; exU = false;
        lane = lane_id();
        vb = 0;
#pragma unroll
        for (int s = 0; s < SLOTS; ++s)
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int j = s * V + e;
                const int k = gidx(s, e);
                if (k < n) vb |= ONE << j;
                kb.set(j, k < n ? diag[k] * (1 << KB) + j + KBIAS : KB_PAD);   // X = 0: Delta_k = W_kk
                mul.set(j, (sizeof(WT) == 2 && (j & 1)) ? (int)((uint32_t)MUL0 << 16) : MUL0);
            }
        xb = 0; bb = 0; E = 0; Eb = 0;
        ring = -1;
        hit = nullptr; hit_done = true; target = 0; t0 = 0;
        trace = nullptr; trace_cap = 0; flips = 0;
    }

    // Row i of the zero-diagonal copy of W as this lane's 16-byte pieces.  The
    // padded rows hold zeros, so every lane loads every slot.  From LDS, the
    // rows are ldl elements long (n rounded up to a 16-byte piece) and a lane
    // whose piece starts past the row takes zeros.
    __attribute__((address_space(3))) const WT *Wl;
    int ldl;
    __device__ __forceinline__ void load_row(int i, uint4 (&q)[SLOTS]) const {
        if ((unsigned)i >= (unsigned)n) i = 0;     // never read outside W (a selection bug shows in parity)
        if constexpr (LDSW) {
            typedef uint32_t u4 __attribute__((ext_vector_type(4)));
            const int off = lane * V;
            u4 v = {0u, 0u, 0u, 0u};
            if (off < ldl) v = *(__attribute__((address_space(3))) const u4 *)(Wl + i * ldl + off);
            q[0] = make_uint4(v[0], v[1], v[2], v[3]);
        } else {
            const WT *row = W + (int64_t)i * ld + lane * V;
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) q[s] = *(const uint4 *)(row + s * SPAN);
        }
    }
    // kb_k += 2 y_i y_k W_ik 2^KB for all k (y = 1 - 2x) from the loaded row.
    // int16: y_i W is one packed 16-bit multiply per word (the library rejects
    // -32768 in int16 W, so the negation is exact).
    __device__ __forceinline__ void apply_row(const uint4 (&q)[SLOTS], int yi) {
        if constexpr (sizeof(WT) == 2) {
            const short2v y2 = {(short)yi, (short)yi};
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
                const uint32_t d[4] = {q[s].x, q[s].y, q[s].z, q[s].w};
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    const short2v w2 = __builtin_bit_cast(short2v, d[p]) * y2;
                    const int j = s * V + 2 * p;
                    // (element values first: a bit cast of a vector element
                    // expression would read the vector's first element)
                    const int m0 = mul[j], m1 = mul[j + 1];
                    kb.set(j, __builtin_amdgcn_sdot2(w2, __builtin_bit_cast(short2v, m0), kb[j], false));
                    kb.set(j + 1, __builtin_amdgcn_sdot2(w2, __builtin_bit_cast(short2v, m1), kb[j + 1], false));
                }
            }
        } else {
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
                const uint32_t d[4] = {q[s].x, q[s].y, q[s].z, q[s].w};
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    const int j = s * V + p;
                    kb.set(j, mad24(mad24((int)d[p], yi, 0), mul[j], kb[j]));
                }
            }
        }
    }

    // Flip the (uniform) selected bit: every word by Eq. (4), the bit's own
    // word by Eq. (5) (its key k becomes 2j - k; the exclusion bit is kept
    // because 2 * 2^31 vanishes mod 2^32), its multiplier negated.
    // `during` is work independent of the search state, done while the row
    // load is in flight.
    template <class F>
    __device__ __forceinline__ void flip_bit(const Sel &s, F &&during) {
        uint4 q[SLOTS];
        load_row(s.i, q);
        const bool xi = (lane_mask(xb, s.L) >> s.j) & 1;
        during();
        apply_row(q, xi ? -1 : 1);
        const int o = kb[s.j];
        kb.set(s.j, lane == s.L ? (2 * s.j + 2 * KBIAS) - o : o);
        const int mo = mul[s.j];
        const uint32_t mf = (sizeof(WT) == 2 && (s.j & 1)) ? (MFLIP << 16) : MFLIP;
        mul.set(s.j, lane == s.L ? (int)((uint32_t)mo ^ mf) : mo);
        xb ^= lane == s.L ? (ONE << s.j) : (mask_t)0;
    }

    __device__ __forceinline__ Sel sel_of(int i) {
        Sel s;
        s.i = i;
        s.L = lidx_to_lane(i);
        s.j = lidx_of(i);
        s.d = dlt_k(readlane(kb[s.j], s.L));
        return s;
    }

    // X := x (packed words), walking from X = 0 by flips in increasing index.
    __device__ __forceinline__ void load_x(const uint64_t *x) {
        const int nw = (n + 63) / 64;
        for (int w = 0; w < nw; ++w) {
            uint64_t word = x[w];
            if (w == nw - 1 && (n & 63)) word &= (1ull << (n & 63)) - 1;   // bits >= n are ignored
            while (word) {
                const int b = __builtin_ctzll(word);
                word &= word - 1;
                const Sel s = uniform(sel_of(w * 64 + b));
                E += s.d;
                flip_bit(s, [] {});
            }
        }
    }

    // Bits of this lane as packed words (bit field gather across lanes).
    __device__ __forceinline__ void store_bits(uint64_t bits, uint64_t *out) const {
        const int nw = (n + 63) / 64;
        constexpr int LPW = WAVE / V;     // lanes per 64-bit word within a slot
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            uint64_t v = ((bits >> (s * V)) & ((1ull << V) - 1)) << ((lane % LPW) * V);
            for (int m = 1; m < LPW; m <<= 1) v |= shfl_xor64(v, m);
            const int w = s * (SPAN / 64) + lane / LPW;
            if (lane % LPW == 0 && w < nw) out[w] = v;
        }
    }

    __device__ __forceinline__ void store_delta(int *out) const {
#pragma unroll
        for (int s = 0; s < SLOTS; ++s)
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int k = gidx(s, e);
                if (k < n) out[k] = dlt_k(kb[s * V + e]);
            }
    }

    // ------------------------------------------------------------- reductions
    __device__ __forceinline__ uint32_t lane_umin() const {
        uint32_t m = UOUT;
#pragma unroll
        for (int j = 0; j < EPL; j += 2) m = min(m, min((uint32_t)kb[j], (uint32_t)kb[j + 1]));
        return m;
    }
    __device__ __forceinline__ int lane_smin() const {
        int m = 0x7FFFFFFF;
#pragma unroll
        for (int j = 0; j < EPL; j += 2) m = min(m, min(kb[j], kb[j + 1]));
        return m;
    }
    // least word of all bits from the lane's unsigned and signed minima
    static __device__ __forceinline__ uint32_t unmask(uint32_t um, int sm) {
        return min(um, (uint32_t)sm & 0x7FFFFFFFu);
    }

    // Wave argmin of per-lane least words: lowest (delta, global index).
    __device__ __forceinline__ Sel argmin_from(uint32_t kmin, int m) const {
        const uint64_t bal = ballot(wv(kmin) == m);
        const int L = (int)__builtin_ctzll(bal);
        const int kl = readlane((int)kmin, L);
        const int slot = m & ((1 << SB) - 1);
        Sel r;
        r.d = dlt_w(m);
        r.j = (slot << LOGV) | (kl & (V - 1));
        r.i = slot * SPAN + L * V + (kl & (V - 1));
        r.L = L;
        return r;
    }
    __device__ __forceinline__ Sel wave_argmin(uint32_t kmin) const {
        return argmin_from(kmin, wave_min(wv(kmin)));
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
            bb = xb ^ (lane == s.L ? (ONE << s.j) : (mask_t)0);
            note_best();
        }
    }

    __device__ __forceinline__ void exact_now() {
        lbU = dlt_w(mU);
        exU = true;
    }
    // Step 1 when nothing but padding is excluded.
    __device__ __forceinline__ void refresh() {
        kminU = lane_umin();
        mU = wave_min(wv(kminU));
        exact_now();
        step1();
    }
    // Step 1 while exclusions are in force.
    __device__ __forceinline__ void refresh_all() {
        kminU = unmask(lane_umin(), lane_smin());
        mU = wave_min(wv(kminU));
        exact_now();
        step1();
    }
    // Step 1 only when it can change BEST (see lbU)
    __device__ __forceinline__ bool need1() const { return E + lbU < Eb; }
    __device__ __forceinline__ void refresh_lazy() {
        if (need1()) refresh();
    }
    __device__ __forceinline__ void refresh_all_lazy() {
        if (need1()) refresh_all();
    }
    // kminU / mU of the current vector for a selection that needs them
    // (Step 1 at this vector was made or could not change BEST)
    __device__ __forceinline__ void ensure_exact() {
        if (!exU) {
            kminU = unmask(lane_umin(), lane_smin());
            mU = wave_min(wv(kminU));
            exact_now();
        }
    }
    // As refresh_all(), also reducing the least word of the domain (kminM, mM)
    // in the same pass.
    uint32_t kminM;
    int mM;
    __device__ __forceinline__ void refresh_dom() {
        const uint32_t um = lane_umin();
        kminM = um;
        kminU = unmask(um, lane_smin());
        wave_min2(wv(kminU), wv(kminM), mU, mM);
        exact_now();
        step1();
    }
    // the domain's least word, and Step 1 only when it can change BEST
    __device__ __forceinline__ void refresh_dom_lazy() {
        if (need1()) {
            refresh_dom();
        } else {
            kminM = lane_umin();
            mM = wave_min(wv(kminM));
        }
    }
    // MaxMin's reductions: as refresh_dom's, and the domain's greatest word
    // mX (signed maximum), all from one pass over the words.
    int mX;
    __device__ __forceinline__ void dom_minmax() {
        uint32_t um = UOUT;
        int sm = 0x7FFFFFFF, sx = (int)0x80000000;
#pragma unroll
        for (int j = 0; j < EPL; j += 2) {
            um = min(um, min((uint32_t)kb[j], (uint32_t)kb[j + 1]));
            sm = min(sm, min(kb[j], kb[j + 1]));
            sx = max(sx, max(kb[j], kb[j + 1]));
        }
        kminM = um;
        kminU = unmask(um, sm);
        wave_minmin_max(wv(kminU), wv(kminM), sx, mU, mM, mX);
        exact_now();
    }
    // MaxMin's domain reductions alone (least and greatest word)
    __device__ __forceinline__ void dom_min_max() {
        uint32_t um = UOUT;
        int sx = (int)0x80000000;
#pragma unroll
        for (int j = 0; j < EPL; j += 2) {
            um = min(um, min((uint32_t)kb[j], (uint32_t)kb[j + 1]));
            sx = max(sx, max(kb[j], kb[j + 1]));
        }
        kminM = um;
        wave_min_max(wv(kminM), sx, mM, mX);
    }

    // BEST := X, then Step 1.
    __device__ __forceinline__ void begin() {
        bb = xb;
        Eb = E;
        note_best();
        refresh();
    }

    // Step 3: flip the selected bit, update E and every word.
    template <class F>
    __device__ __forceinline__ void flip_core(const Sel &s0, F &&during) {
        const Sel s = uniform(s0);
        E += s.d;
        lbU = min(lbU - (int64_t)wmax2, (int64_t)(-s.d));
        exU = false;
        flip_bit(s, during);
        if (trace && flips < trace_cap && lane == 0) trace[flips] = s.i;
        flips++;
    }
    __device__ __forceinline__ void flip_core(const Sel &s0) { flip_core(s0, [] {}); }
    __device__ __forceinline__ void flip(const Sel &s) {
        flip_core(s);
        refresh();
    }
    __device__ __forceinline__ void flip_lazy(const Sel &s) {
        flip_core(s);
        refresh_lazy();
    }

    // ------------------------------------------------------------- exclusions
    __device__ __forceinline__ void mark(const Sel &s) {
        const int o = kb[s.j];
        kb.set(s.j, lane == s.L ? (int)((uint32_t)o | XBIT) : o);
    }
    __device__ __forceinline__ void unmark(int j, int L) {
        const int o = kb[j];
        kb.set(j, lane == L ? (o & 0x7FFFFFFF) : o);
    }
    // every valid bit back in the domain (padding stays out)
    __device__ __forceinline__ void reset_marks() {
#pragma unroll
        for (int j = 0; j < EPL; ++j) kb.set(j, ((vb >> j) & 1) ? (kb[j] & 0x7FFFFFFF) : kb[j]);
    }

    // Tabu (R11) of the bit flipped at iteration t.  maybe_marked: it was
    // selected from an empty domain, so it may be excluded already; its
    // pending release is then void (the new one replaces it).
    __device__ __forceinline__ void tabu_mark(const Sel &s0, int t, int tau, bool maybe_marked) {
        if (tau <= 0) return;
        const Sel s = uniform(s0);
        const int e = (s.L << 8) | s.j;
        if (maybe_marked && readlane(kb[s.j], s.L) < 0) {
            for (int u = t - tau; u < t; ++u)
                if (u >= 1 && readlane(ring, u & 31) == e) ring = lane == (u & 31) ? -1 : ring;
        }
        mark(s);
        ring = lane == (t & 31) ? e : ring;
    }
    // Before the domain of iteration t: the bit flipped at t - tau - 1 is back.
    __device__ __forceinline__ void tabu_release(int t, int tau) {
        const int t0r = t - tau - 1;
        if (tau > 0 && t0r >= 1) {
            const int e = readlane(ring, t0r & 31);
            if (e >= 0) unmark(e & 255, e >> 8);
        }
    }

    // ------------------------------------------------------------- rules
    // Greedy (Section III-A.1): flip argmin while it is negative.
    __device__ __forceinline__ int phase_greedy(int cap) {
        if (cap <= 0) cap = 64 * n;                   // documented default bound
        ensure_exact();
        int f = 0;
        while (dlt_w(mU) < 0 && f < cap) {
            flip(argmin_from(kminU, mU));
            f++;
        }
        return f;
    }

    // Straight (Section III-A.2): argmin over bits differing from the target.
    // The bits that agree are excluded, and so is each bit once flipped.
    __device__ __forceinline__ int phase_straight(const uint64_t *target_bits) {
        const int nw = (n + 63) / 64;
        uint64_t db = 0;
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            const int k0 = s * SPAN + lane * V;
            const int w = k0 >> 6;
            const uint64_t word = w < nw ? target_bits[w] : 0ull;
            const uint64_t f = ((word >> (k0 & 63)) & ((1ull << V) - 1)) & (vb >> (s * V));   // bits >= n ignored
            db |= f << (s * V);
        }
        const mask_t diff = xb ^ (mask_t)db;
        int hd = 0;
#pragma unroll
        for (int j = 0; j < EPL; ++j) {
            const bool dif = (diff >> j) & 1;
            kb.set(j, dif ? (kb[j] & 0x7FFFFFFF) : (int)((uint32_t)kb[j] | XBIT));
            hd += dif;
        }
        hd = (int)wave_sum64(hd);
        kminM = lane_umin();
        mM = wave_min(wv(kminM));
        int f = 0;
        for (; f < hd; ++f) {
            const Sel s = uniform(argmin_from(kminM, mM));
            mark(s);
            flip_core(s);
            refresh_dom_lazy();
        }
        reset_marks();
        return f;
    }

    // Tabu greedy: T iterations of the non-tabu argmin.
    // The tabu mark of iteration t is set before the flip, so the refresh
    // after it reduces the domain of iteration t + 1 together with Step 1.
    __device__ __forceinline__ int phase_tabu_greedy(int T, int tau) {
        ensure_exact();
        kminM = kminU;            // iteration 1: nothing is tabu
        mM = mU;
        for (int t = 1; t <= T; ++t) {
            const bool emp = none(mM);
            if (emp) ensure_exact();
            const Sel s = emp ? argmin_from(kminU, mU) : argmin_from(kminM, mM);
            tabu_mark(s, t, tau, emp);
            flip_core(s);
            tabu_release(t + 1, tau);
            refresh_dom_lazy();
        }
        reset_marks();
        return T;
    }

    // CyclicMin (Section III-A.4): argmin over a sliding cyclic window.
    __device__ __forceinline__ int phase_cyclicmin(int T, int tau) {
        int pos = 0;
        FracStep fs;
        fs.init((uint32_t)T);
        for (int t = 1; t <= T; ++t) {
            fs.next();                      // fs.q = floor(t 2^32 / T)
            int w;
            if (t >= T) {
                w = n;
            } else {
                const uint64_t hh = fs.q;
                const int c = n < 32 ? n : 32;
                const int64_t ww = (int64_t)(((uint64_t)n * cube_frac(hh)) >> 32);
                w = ww < c ? c : (ww > n ? n : (int)ww);
            }
            tabu_release(t, tau);
            const bool wrap = pos + w > n;
            const int lo = wrap ? pos + w - n : pos;       // start of the excluded / included range
            const uint32_t span = wrap ? (uint32_t)(n - w) : (uint32_t)w;
            auto inwin = [&](int s, int e) {
                const uint32_t off = (uint32_t)(gidx(s, e) - lo);
                return wrap ? (off >= span) : (off < span);
            };
            uint32_t km = UOUT;
#pragma unroll
            for (int s = 0; s < SLOTS; ++s)
#pragma unroll
                for (int e = 0; e < V; ++e) km = min(km, inwin(s, e) ? (uint32_t)kb[s * V + e] : UOUT);
            const int m = wave_min(wv(km));
            const bool emp = none(m);
            Sel s;
            if (emp) {
                // the window holds only tabu bits: the window without tabu
                uint32_t kw = UOUT;
#pragma unroll
                for (int ss = 0; ss < SLOTS; ++ss)
#pragma unroll
                    for (int e = 0; e < V; ++e)
                        kw = min(kw, inwin(ss, e) ? ((uint32_t)kb[ss * V + e] & 0x7FFFFFFFu) : UOUT);
                s = wave_argmin(kw);
            } else {
                s = argmin_from(km, m);
            }
            flip_core(s);
            refresh_all_lazy();
            tabu_mark(s, t, tau, emp);
            pos = (pos + w) % n;
        }
        reset_marks();
        return T;
    }

    // Position of set bit number k (0-based, k < popcount(b)) of a V-bit mask,
    // by halving with popcounts: no data-dependent loop.
    static __device__ __forceinline__ int kth_bit(uint32_t b, uint32_t k) {
        int base = 0;
        if constexpr (V == 8) {
            const uint32_t c = (uint32_t)__builtin_popcount(b & 0xFu);
            const bool up = k >= c;
            k -= up ? c : 0u;
            b >>= up ? 4 : 0;
            base += up ? 4 : 0;
        }
        const uint32_t c2 = (uint32_t)__builtin_popcount(b & 0x3u);
        const bool up2 = k >= c2;
        k -= up2 ? c2 : 0u;
        b >>= up2 ? 2 : 0;
        base += up2 ? 2 : 0;
        return base + (k >= (b & 1u) ? 1 : 0);
    }

    // Candidates: unexcluded elements (IGN: exclusions ignored, padding still
    // out) whose key is <= dk.  Counts them, draws r = floor(v * count / 2^32)
    // and returns the r-th candidate (0-based, in increasing bit index: slot,
    // then lane, then sub-index).
    template <bool IGN>
    __device__ __forceinline__ Sel pick_rth(int dk, uint32_t v) {
        const uint32_t lim = (uint32_t)(dk + KBIAS);
        auto cand = [&](int j) {
            const uint32_t k = IGN ? ((uint32_t)kb[j] & 0x7FFFFFFFu) : (uint32_t)kb[j];
            return k <= lim;
        };
        uint32_t cs[SLOTS];
        uint32_t c = 0;
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            cs[s] = 0;
#pragma unroll
            for (int e = 0; e < V; ++e) cs[s] += (uint32_t)__builtin_popcountll(ballot(cand(s * V + e)));
            c += cs[s];
        }
        if (c == 0) {                                 // cannot happen: the domain minimum qualifies
            ensure_exact();
            return argmin_from(kminU, mU);
        }
        const uint32_t r = scale32(v, c);
        int slot = SLOTS - 1;
        uint32_t before = 0;
        bool found = false;
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            if (!found) {
                if (r < before + cs[s]) { slot = s; found = true; }
                else before += cs[s];
            }
        }
        const uint32_t rr = r - before;
        Sel out;
        out.L = 0; out.j = 0; out.i = 0;
        at_slot(slot, [&](int ss) {
            // excl: candidates of the slot in lower lanes; cb: this lane's own
            uint32_t excl = 0, cb = 0;
#pragma unroll
            for (int e = 0; e < V; ++e) {
                // the same test as cand(), written apart so that it is made
                // here as a lane mask rather than carried over from the counts
                const uint32_t kj = IGN ? ((uint32_t)kb[ss * V + e] & 0x7FFFFFFFu) : (uint32_t)kb[ss * V + e];
                const bool ce = kj < lim + 1u;
                const uint64_t cm = ballot(ce);
                cb |= ce ? (1u << e) : 0u;
                excl = __builtin_amdgcn_mbcnt_hi((uint32_t)(cm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)cm, excl));
            }
            // excl does not decrease with the lane, so the lanes with excl <= rr
            // are a prefix (lane 0 at least) whose last lane holds candidate rr
            const uint64_t le = ballot(excl <= rr);
            const int L = 63 - __builtin_clzll(le | 1ull);
            const int left = (int)(rr - (uint32_t)readlane((int)excl, L));
            // (uniform by construction; said so, the element index stays scalar)
            const int e_sel = __builtin_amdgcn_readfirstlane(kth_bit((uint32_t)readlane((int)cb, L), (uint32_t)left));
            out.L = L;
            out.j = ss * V + e_sel;
            out.i = ss * SPAN + L * V + e_sel;
        });
        out.d = dlt_k(readlane(kb[out.j], out.L));
        return out;
    }

    // MaxMin (Section III-A.3).  The domain reductions of iteration t+1 (its
    // least and greatest key) are made by the refresh after the flip of
    // iteration t; the tabu mark of iteration t precedes that flip.
    __device__ __forceinline__ int phase_maxmin(int T, int tau, uint32_t ph) {
        dom_minmax();                       // iteration 1: nothing is tabu
        FracStep fs;
        fs.init((uint32_t)T);
        // iterations 2c+1 and 2c+2 use words (0, 1) and (2, 3) of draw c (R18);
        // the draws are made 64 at a time, draw cbase + l in lane l
        R4 rv = {{0u, 0u, 0u, 0u}};
        int cbase = -64;
        // the random words u, v and the cube fraction of iteration t depend on
        // t only: they are made for iteration t + 1 while the row of iteration
        // t loads
        uint32_t u, v;
        uint64_t cf;
        auto prepare = [&](int t) {
            fs.next();
            cf = cube_frac(fs.rest());      // fs.rest() = floor(2^32 (T - t) / T)
            const int c = (t - 1) >> 1;
            if (c >= cbase + 64) {
                cbase += 64;
                rv = philox((uint32_t)(cbase + lane), inst, ph, (uint32_t)TAG_MAXMIN << 24, seed);
            }
            const bool second = (t - 1) & 1;
            u = (uint32_t)readlane((int)(second ? rv.w[2] : rv.w[0]), c - cbase);
            v = (uint32_t)readlane((int)(second ? rv.w[3] : rv.w[1]), c - cbase);
        };
        prepare(1);
        for (int t = 1; t <= T; ++t) {
            const bool ign = none(mM);      // every bit tabu: tabu ignored (R11)
            if (ign) {
                ensure_exact();
                mM = mU;
                int kx = (int)0x80000000;
#pragma unroll
                for (int j = 0; j < EPL; ++j) kx = max(kx, ((vb >> j) & 1) ? (kb[j] & 0x7FFFFFFF) : (int)0x80000000);
                mX = wave_max(kx);
            }
            const int mind = dlt_w(mM);
            const int maxd = (mX - KBIAS) >> KB;
            const uint64_t span = ((uint64_t)(uint32_t)(maxd - mind) * cf) >> 32;
            const int d = mind + (int)(((uint64_t)u * (span + 1)) >> 32);
            const int dk = d * (1 << KB) + ((1 << KB) - 1);
            const Sel s = ign ? pick_rth<true>(dk, v) : pick_rth<false>(dk, v);
            tabu_mark(s, t, tau, ign);
            flip_core(s, [&] { if (t < T) prepare(t + 1); });
            tabu_release(t + 1, tau);
            if (need1()) {
                dom_minmax();
                step1();
            } else {
                dom_min_max();
            }
        }
        reset_marks();
        return T;
    }

    // PositiveMin (Section III-A.6).  The least positive key of the domain is
    // the unsigned minimum of kb - (2^29 + 2^KB): keys below 2^KB (delta <= 0)
    // wrap to the top, excluded words stay above 2^30.  The domain can only be
    // empty when n <= tau.
    __device__ __forceinline__ int phase_positivemin(int T, int tau, uint32_t ph) {
        constexpr uint32_t C = (uint32_t)KBIAS + (1u << KB);
        const bool may_empty = n <= tau;
        // iterations 4c+1 .. 4c+4 use words 0 .. 3 of draw c (R18); the draws
        // are made 64 at a time, draw cbase + l in lane l
        R4 rv = {{0u, 0u, 0u, 0u}};
        int cbase = -64;
        for (int t = 1; t <= T; ++t) {
            tabu_release(t, tau);
            bool ign = false;
            if (may_empty) ign = none(wave_min(wv(lane_umin())));
            uint32_t kp = UOUT;
            if (!ign) {
#pragma unroll
                for (int j = 0; j < EPL; j += 2) kp = min(kp, min((uint32_t)kb[j] - C, (uint32_t)kb[j + 1] - C));
            } else {
#pragma unroll
                for (int j = 0; j < EPL; ++j) kp = min(kp, ((uint32_t)kb[j] & 0x7FFFFFFFu) - C);
            }
            const int mw = wave_min(wv(kp));
            const int d = none(mw) ? D_TOP : (mw >> SB) + 1;
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
            flip_core(s);
            refresh_all_lazy();
            tabu_mark(s, t, tau, ign);
        }
        reset_marks();
        return T;
    }

    // RandomMin (Section III-A.5): candidates by random byte < q(t).
    __device__ __forceinline__ int phase_randommin(int T, int tau, uint32_t ph) {
        FracStep fs;
        fs.init((uint32_t)T);
        // Lanes 2m and 2m+1 share the draw of bits 16m .. 16m+15 of a slot
        // (bytes 0..7 and 8..15) when V = 8 and the slots pair up: even lanes
        // draw for even slots, odd lanes for odd slots, and each pair swaps
        // the halves.  Otherwise each lane draws per slot.
        constexpr bool PAIRS = V == 8 && SLOTS % 2 == 0;
        constexpr int ND = PAIRS ? SLOTS / 2 : SLOTS;
        // with few draws per lane, iteration t + 1's draws are made while the
        // row of iteration t loads (they depend on t only)
        constexpr bool AHEAD = ND <= 2;
        const uint32_t tag = (uint32_t)TAG_RANDMIN << 24;
        const bool odd = lane & 1;
        auto draw = [&](int t, int k) -> R4 {
            const int s_own = PAIRS ? 2 * k + (odd ? 1 : 0) : k;
            return philox((uint32_t)t, inst, ph, tag | (uint32_t)((s_own * SPAN + lane * V) >> 4), seed);
        };
        R4 rd[ND];
        if constexpr (AHEAD) {
#pragma unroll
            for (int k = 0; k < ND; ++k) rd[k] = draw(1, k);
        }
        for (int t = 1; t <= T; ++t) {
            fs.next();
            int q;
            if (t >= T) {
                q = 256;
            } else {
                const uint64_t hh = fs.q;
                const int qq = (int)(cube_frac(hh) >> 24);
                const int qmin = (8192 + n - 1) / n;
                q = qq < qmin ? qmin : (qq > 256 ? 256 : qq);
            }
            tabu_release(t, tau);
            uint32_t kr = UOUT;
            // lane's random words for slot s: wa (bytes of elements 0..3), wb (4..7)
            auto cand = [&](int s, uint32_t wa, uint32_t wb) {
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const int j = s * V + e;
                    const uint32_t word = e < 4 ? wa : wb;
                    const int byte = (int)((word >> (8 * (e & 3))) & 0xFFu);
                    kr = min(kr, byte < q ? (uint32_t)kb[j] : UOUT);
                }
            };
#pragma unroll
            for (int k = 0; k < ND; ++k) {
                R4 r;
                if constexpr (AHEAD) r = rd[k];
                else r = draw(t, k);
                if constexpr (PAIRS) {
                    const int u = 2 * k;
                    const uint32_t ra = swap_pair(odd ? r.w[0] : r.w[2]);
                    const uint32_t rb = swap_pair(odd ? r.w[1] : r.w[3]);
                    // slot u: even lane own words 0, 1; odd lane the even neighbour's 2, 3
                    cand(u, odd ? ra : r.w[0], odd ? rb : r.w[1]);
                    // slot u+1: even lane the odd neighbour's 0, 1; odd lane own 2, 3
                    cand(u + 1, odd ? r.w[2] : ra, odd ? r.w[3] : rb);
                } else {
                    // this lane's V bytes start at byte (k0 mod 16) of the draw
                    const int k0 = k * SPAN + lane * V;
                    const int w0 = (k0 & 15) >> 2;
                    const uint32_t wa = w0 == 0 ? r.w[0] : (w0 == 1 ? r.w[1] : (w0 == 2 ? r.w[2] : r.w[3]));
                    const uint32_t wb = w0 == 0 ? r.w[1] : (w0 == 1 ? r.w[2] : r.w[3]);
                    cand(k, wa, wb);
                }
            }
            const int m = wave_min(wv(kr));
            bool emp = false;
            Sel s;
            if (!none(m)) {
                s = argmin_from(kr, m);
            } else {
                // no candidate: the non-tabu argmin, or the plain one when every bit is tabu
                const uint32_t km = lane_umin();
                const int mm = wave_min(wv(km));
                emp = none(mm);
                if (emp) ensure_exact();
                s = emp ? argmin_from(kminU, mU) : argmin_from(km, mm);
            }
            flip_core(s, [&] {
                if constexpr (AHEAD) {
                    if (t < T) {
#pragma unroll
                        for (int k = 0; k < ND; ++k) rd[k] = draw(t + 1, k);
                    }
                }
            });
            refresh_all_lazy();
            tabu_mark(s, t, tau, emp);
        }
        reset_marks();
        return T;
    }

    // TwoNeighbor (Section III-A.7): 0, 1, 0, 2, 1, 3, 2, ...
    __device__ __forceinline__ int phase_twoneighbor() {
        flip_lazy(sel_of(0));
        for (int k = 1; k < n; ++k) {
            flip_lazy(sel_of(k));
            flip_lazy(sel_of(k - 1));
        }
        return 2 * n - 1;
    }

    // (an if-chain rather than a switch: the switch lets the compiler merge
    // the tails of the phases, which costs about a hundred VGPRs)
    __device__ __forceinline__ int run_phase(int rule, int T, int tau, uint32_t ph, const uint64_t *target_bits,
                                             int cap) {
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

    // Batch search (Section III-B): Straight -> Greedy -> {main -> Greedy}*,
    // written as one loop over phases k = 0, 1, 2, ... (Straight, then Greedy
    // at odd k and the main algorithm at even k > 0) so that the phases share
    // one code path and one register allocation.
    __device__ __forceinline__ int batch(const uint64_t *target_bits, int rule, int T, int Bn, int tau, uint32_t &ph,
                                         int cap) {
        bb = xb;
        Eb = E;
        note_best();
        refresh();
        const bool main_ok = rule >= MAXMIN && rule <= TWONEIGHBOR;
        int f = 0;
        for (int k = 0;; ++k) {
            const int r = k == 0 ? STRAIGHT : ((k & 1) ? GREEDY : rule);
            f += run_phase(r, T, tau, ph, target_bits, cap);
            if (k > 0 && !(k & 1)) ph++;
            if (k & 1) {
                // after each Greedy: stop once the batch budget is reached, after
                // the single TwoNeighbor, or when the rule is not a main algorithm
                if (f >= Bn || !main_ok || (rule == TWONEIGHBOR && k > 1)) break;
            }
        }
        return f;
    }
};

}  // namespace dabs
