// dabs_walker.h -- one search instance per wavefront (Section III-A, B).
//
// The walker keeps X, the local fields, BEST and the energies of one instance
// in the registers of one wave (layout in dabs_device.h).  Every flip reads
// one row of W (16-byte loads, one per slot) and updates the local fields with
// one v_dot2 (int16) or v_mad_i32_i24 (int32) per element; the argmin over
// the deltas is a per-lane min3 chain over packed (delta, index) keys followed
// by a DPP wave reduction.  Step 1 (BEST) runs at every visited state.
//
// Rule domains (tabu, Straight's differing bits, padding) are expressed with
// one integer per element, ex[j]: element j is outside the domain of
// iteration t when ex[j] >= t.  Tabu sets ex[j] = t0 + tau when bit j flips
// at iteration t0 (so it is excluded at t0+1 .. t0+tau and expires by
// itself); padding elements hold EX_ALWAYS.  A masked key is one compare and
// one v_cndmask per element.
#pragma once
#include "dabs_device.h"

namespace dabs {

constexpr int EX_NEVER = -(1 << 30);
constexpr int EX_ALWAYS = 0x7fffffff;

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

template <typename WT, int SLOTS>
struct Walker {
    static constexpr int V = 16 / (int)sizeof(WT);
    static constexpr int LOGV = V == 8 ? 3 : 2;
    static constexpr int EPL = V * SLOTS;
    static constexpr int KB = clog2(EPL) < LOGV ? LOGV : clog2(EPL);
    static constexpr int SB = KB - LOGV;
    static constexpr int SPAN = WAVE * V;   // bits covered by one slot
    typedef int vecE __attribute__((ext_vector_type(EPL)));

    // The per-element vectors are the kernel's own local variables, one flat
    // vector each (element j = s*V + e), which keeps them in registers and
    // turns a uniform dynamic index into s_set_gpr_idx; the walker refers to
    // them.
    vecE &h, &s2, &ex, &key;

    __device__ __forceinline__ Walker(vecE &h_, vecE &s2_, vecE &ex_, vecE &key_)
        : h(h_), s2(s2_), ex(ex_), key(key_) {}

    const WT *__restrict__ W;
    int64_t ld;
    int n, lane;
    uint64_t xb, bb;          // X and BEST bits of this lane (bit j)
    uint64_t vb;              // valid-element bits of this lane (bit j set iff bit index < n)
    int64_t E, Eb;
    // Step 1 state of the current vector: per-lane unmasked minimum key and
    // its wave minimum (key >> LOGV)
    int kminU, mU;
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
    __device__ __forceinline__ void set_lane_elem(vecE &a, int j, int L, int v) {
        const int o = a[j];
        a[j] = lane == L ? v : o;
    }
    __device__ __forceinline__ void neg_lane_elem(vecE &a, int j, int L) {
        const int o = a[j];
        a[j] = lane == L ? -o : o;
    }

    // ------------------------------------------------------------- set up
    __device__ __forceinline__ void setup(const WT *Wp, const int *diag, int64_t ld_, int n_, uint64_t seed_,
                                          uint32_t inst_) {
        W = Wp; ld = ld_; n = n_; seed = seed_; inst = inst_;
        lane = lane_id();
        vb = 0;
#pragma unroll
        for (int s = 0; s < SLOTS; ++s)
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int k = gidx(s, e);
                if (k < n) vb |= 1ull << (s * V + e);
                h[s * V + e] = k < n ? diag[k] : H_PAD;      // X = 0: Delta_k = W_kk
                s2[s * V + e] = 1 << KB;
                ex[s * V + e] = k < n ? EX_NEVER : EX_ALWAYS;
            }
        xb = 0; bb = 0; E = 0; Eb = 0;
        hit = nullptr; hit_done = true; target = 0; t0 = 0;
        trace = nullptr; trace_cap = 0; flips = 0;
    }

    __device__ __forceinline__ void ex_reset() {
#pragma unroll
        for (int j = 0; j < EPL; ++j) ex[j] = ((vb >> j) & 1) ? EX_NEVER : EX_ALWAYS;
    }

    // h_k += c W_ik for all k (row i of the zero-diagonal copy of W).  The
    // padded rows hold zeros, so every lane loads every slot.
    __device__ __forceinline__ void update_row(int i, int c) {
        if ((unsigned)i >= (unsigned)n) i = 0;     // never read outside W (a selection bug shows in parity)
        const WT *row = W + (int64_t)i * ld + lane * V;
        uint4 q[SLOTS];
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) q[s] = *(const uint4 *)(row + s * SPAN);
        if constexpr (sizeof(WT) == 2) {
            const short2v clo = {(short)c, 0}, chi = {0, (short)c};
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
                const uint32_t d[4] = {q[s].x, q[s].y, q[s].z, q[s].w};
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    const short2v w2 = __builtin_bit_cast(short2v, d[p]);
                    h[s * V + 2 * p] = __builtin_amdgcn_sdot2(w2, clo, h[s * V + 2 * p], false);
                    h[s * V + 2 * p + 1] = __builtin_amdgcn_sdot2(w2, chi, h[s * V + 2 * p + 1], false);
                }
            }
        } else {
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
                const uint32_t d[4] = {q[s].x, q[s].y, q[s].z, q[s].w};
#pragma unroll
                for (int p = 0; p < 4; ++p) h[s * V + p] = mad24((int)d[p], c, h[s * V + p]);
            }
        }
    }

    // Flip bit i of X without Step 1 (set-up walk from X = 0).
    __device__ __forceinline__ void raw_flip(int i) {
        const int L = lidx_to_lane(i), j = lidx_of(i);
        const int xi = (int)((readlane64(xb, L) >> j) & 1);
        const int hi = readlane(h[j], L);
        E += xi ? -hi : hi;
        update_row(i, xi ? -2 : 2);
        neg_lane_elem(s2, j, L);
        xb ^= lane == L ? (1ull << j) : 0ull;
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
                raw_flip(w * 64 + b);
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
                if (k < n) out[k] = s2[s * V + e] > 0 ? h[s * V + e] : -h[s * V + e];
            }
    }

    // ------------------------------------------------------------- keys
    // key_j = Delta_j 2^KB + j.  Up to 32 elements per lane the keys are kept
    // in registers after each flip; above that they are recomputed where used
    // (one multiply-add), which keeps the walker within the register file.
    static constexpr bool KEEP = EPL <= 32;
    __device__ __forceinline__ int K(int j) const {
        if constexpr (KEEP) return key[j];
        else return mad24(h[j], s2[j], j);
    }
    __device__ __forceinline__ void compute_keys() {
        if constexpr (KEEP) {
#pragma unroll
            for (int j = 0; j < EPL; ++j) key[j] = mad24(h[j], s2[j], j);
        }
    }
    __device__ __forceinline__ int lane_min_key() const {
        int m = KEY_BIG;
#pragma unroll
        for (int j = 0; j < EPL; j += 2) m = min(m, min(K(j), K(j + 1)));
        return m;
    }
    // least key among elements with ex < thr (KEY_OUT when there is none)
    __device__ __forceinline__ int lane_min_dom(int thr) const {
        int m = KEY_OUT;
#pragma unroll
        for (int j = 0; j < EPL; j += 2) {
            const int a = ex[j] < thr ? K(j) : KEY_OUT;
            const int b = ex[j + 1] < thr ? K(j + 1) : KEY_OUT;
            m = min(m, min(a, b));
        }
        return m;
    }

    // Wave argmin of per-lane minimum keys: lowest (delta, global index).
    __device__ __forceinline__ Sel argmin_from(int kmin, int m) const {
        const uint64_t bal = ballot((kmin >> LOGV) == m);
        const int L = (int)__builtin_ctzll(bal);
        const int kl = readlane(kmin, L);
        const int slot = m & ((1 << SB) - 1);
        Sel r;
        r.d = m >> SB;
        r.j = (slot << LOGV) | (kl & (V - 1));
        r.i = slot * SPAN + L * V + (kl & (V - 1));
        r.L = L;
        return r;
    }
    __device__ __forceinline__ Sel wave_argmin(int kmin) const {
        return argmin_from(kmin, wave_min(kmin >> LOGV));
    }
    // wave minimum of k >> LOGV; the domain is empty when it decodes to a
    // delta of H_PAD or more (only padding or excluded elements)
    static __device__ __forceinline__ bool empty_dom(int m) { return (m >> SB) >= H_PAD; }

    __device__ __forceinline__ void note_best() {
        if (!hit_done && Eb <= target) {
            hit_done = true;
            const unsigned long long now = __builtin_amdgcn_s_memrealtime();
            if (lane == 0) atomicMin(hit, now - t0);
        }
    }

    // Step 1: BEST <- best 1-bit neighbour when strictly better than E(BEST).
    __device__ __forceinline__ void step1() {
        const int d = mU >> SB;
        if (E + d < Eb) {
            const Sel s = argmin_from(kminU, mU);
            Eb = E + d;
            bb = xb ^ (lane == s.L ? (1ull << s.j) : 0ull);
            note_best();
        }
    }

    // Keys of the current state, then Step 1.
    __device__ __forceinline__ void refresh() {
        compute_keys();
        kminU = lane_min_key();
        mU = wave_min(kminU >> LOGV);
        step1();
    }

    // As refresh(), also reducing the least key of the domain ex < thr (kminM,
    // mM) in the same pass.
    int kminM, mM;
    __device__ __forceinline__ void refresh_dom(int thr) {
        compute_keys();
        kminU = lane_min_key();
        kminM = lane_min_dom(thr);
        wave_min2(kminU >> LOGV, kminM >> LOGV, mU, mM);
        step1();
    }
    // MaxMin's reductions of the domain ex < thr, made in the pass that
    // recomputes the keys after a flip: least key kminM / mM (as
    // refresh_dom) and greatest key mX (its wave maximum).
    int mX;
    __device__ __forceinline__ void dom_minmax(int thr) {
        int ku = KEY_BIG, km = KEY_OUT, kx = -KEY_OUT;
#pragma unroll
        for (int j = 0; j < EPL; j += 2) {
            const int k0 = K(j), k1 = K(j + 1);
            const bool i0 = ex[j] < thr, i1 = ex[j + 1] < thr;
            ku = min(ku, min(k0, k1));
            km = min(km, min(i0 ? k0 : KEY_OUT, i1 ? k1 : KEY_OUT));
            kx = max(kx, max(i0 ? k0 : -KEY_OUT, i1 ? k1 : -KEY_OUT));
        }
        kminU = ku;
        kminM = km;
        wave_minmin_max(ku >> LOGV, km >> LOGV, kx, mU, mM, mX);
    }
    __device__ __forceinline__ void refresh_minmax(int thr) {
        compute_keys();
        dom_minmax(thr);
        step1();
    }

    // argmin of the domain reduced by refresh_dom, or the plain argmin when
    // the domain is empty
    __device__ __forceinline__ Sel dom_sel() const {
        return empty_dom(mM) ? argmin_from(kminU, mU) : argmin_from(kminM, mM);
    }

    // BEST := X, then Step 1.
    __device__ __forceinline__ void begin() {
        bb = xb;
        Eb = E;
        note_best();
        refresh();
    }

    // Step 3: flip the selected bit, update E and every local field.
    __device__ __forceinline__ void flip_core(const Sel &s0) {
        const Sel s = uniform(s0);
        E += s.d;
        const bool xi = (readlane64(xb, s.L) >> s.j) & 1;
        update_row(s.i, xi ? -2 : 2);
        neg_lane_elem(s2, s.j, s.L);
        xb ^= lane == s.L ? (1ull << s.j) : 0ull;
        if (trace && flips < trace_cap && lane == 0) trace[flips] = s.i;
        flips++;
    }
    __device__ __forceinline__ void flip(const Sel &s) {
        flip_core(s);
        refresh();
    }
    // flip, then refresh with the domain ex < thr of the next selection
    __device__ __forceinline__ void flip_dom(const Sel &s, int thr) {
        flip_core(s);
        refresh_dom(thr);
    }

    __device__ __forceinline__ Sel sel_of(int i) {
        Sel s;
        s.i = i;
        s.L = lidx_to_lane(i);
        s.j = lidx_of(i);
        s.d = readlane(K(s.j), s.L) >> KB;
        return s;
    }

    // tabu (R11): bit flipped at iteration t is excluded at t+1 .. t+tau
    // (one element write in every case: a conditional write would be turned
    // into a select over the whole vector)
    __device__ __forceinline__ void mark_tabu(const Sel &s0, int t, int tau) {
        const Sel s = uniform(s0);
        const int o = ex[s.j];
        ex[s.j] = (lane == s.L && tau > 0) ? t + tau : o;
    }

    // Non-tabu argmin of iteration t, or the plain argmin when every bit is tabu.
    __device__ __forceinline__ Sel dom_argmin(int t) {
        const int km = lane_min_dom(t);
        const int m = wave_min(km >> LOGV);
        return empty_dom(m) ? argmin_from(kminU, mU) : argmin_from(km, m);
    }

    // ------------------------------------------------------------- rules
    // Greedy (Section III-A.1): flip argmin while it is negative.
    __device__ __forceinline__ int phase_greedy(int cap) {
        if (cap <= 0) cap = 64 * n;                   // documented default bound
        int f = 0;
        while ((mU >> SB) < 0 && f < cap) {
            flip(argmin_from(kminU, mU));
            f++;
        }
        return f;
    }

    // Straight (Section III-A.2): argmin over bits differing from the target.
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
        const uint64_t diff = xb ^ db;
        int hd = 0;
#pragma unroll
        for (int j = 0; j < EPL; ++j) {
            const bool dif = (diff >> j) & 1;
            ex[j] = dif ? EX_NEVER : EX_ALWAYS;
            hd += dif;
        }
        hd = (int)wave_sum64(hd);
        kminM = lane_min_dom(0);
        mM = wave_min(kminM >> LOGV);
        int f = 0;
        for (; f < hd; ++f) {
            const Sel s = uniform(argmin_from(kminM, mM));
            set_lane_elem(ex, s.j, s.L, EX_ALWAYS);
            flip_dom(s, 0);
        }
        ex_reset();
        return f;
    }

    // Tabu greedy: T iterations of the non-tabu argmin.
    // The tabu mark of iteration t is set before the flip, so the refresh
    // after it reduces the domain of iteration t + 1 together with Step 1.
    __device__ __forceinline__ int phase_tabu_greedy(int T, int tau) {
        kminM = kminU;            // iteration 1: nothing is tabu
        mM = mU;
        for (int t = 1; t <= T; ++t) {
            const Sel s = dom_sel();
            mark_tabu(s, t, tau);
            flip_dom(s, t + 1);
        }
        ex_reset();
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
            const bool wrap = pos + w > n;
            const int lo = wrap ? pos + w - n : pos;       // start of the excluded / included range
            const uint32_t span = wrap ? (uint32_t)(n - w) : (uint32_t)w;
            int km = KEY_BIG, kw = KEY_BIG;
#pragma unroll
            for (int s = 0; s < SLOTS; ++s)
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const int j = s * V + e;
                    const uint32_t off = (uint32_t)(gidx(s, e) - lo);
                    const bool in = wrap ? (off >= span) : (off < span);
                    km = min(km, in && ex[j] < t ? K(j) : KEY_BIG);
                    kw = min(kw, in ? K(j) : KEY_BIG);
                }
            const int m = wave_min(km >> LOGV);
            const Sel s = empty_dom(m) ? wave_argmin(kw) : argmin_from(km, m);
            flip(s);
            mark_tabu(s, t, tau);
            pos = (pos + w) % n;
        }
        ex_reset();
        return T;
    }

    // Candidates: elements of the domain (ex < thr) whose key is <= dk.
    // Counts them, draws r = floor(v * count / 2^32) and returns the r-th
    // candidate (0-based, in increasing bit index: slot, then lane, then
    // sub-index).
    __device__ __forceinline__ Sel pick_rth(int dk, int thr, uint32_t v) {
        uint32_t cs[SLOTS];
        uint32_t c = 0;
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            cs[s] = 0;
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int j = s * V + e;
                cs[s] += (uint32_t)__builtin_popcountll(ballot(K(j) <= dk && ex[j] < thr));
            }
            c += cs[s];
        }
        if (c == 0) return argmin_from(kminU, mU);   // cannot happen: the domain minimum qualifies
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
            uint64_t cm[V];
            int cnt = 0;
            uint32_t excl = 0;
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int j = ss * V + e;
                cm[e] = ballot(K(j) <= dk && ex[j] < thr);
                cnt += __builtin_amdgcn_inverse_ballot_w64(cm[e]) ? 1 : 0;
                excl = __builtin_amdgcn_mbcnt_hi((uint32_t)(cm[e] >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)cm[e], excl));
            }
            const uint64_t own = ballot(excl <= rr && rr < excl + (uint32_t)cnt);
            const int L = own ? (int)__builtin_ctzll(own) : 0;
            int left = (int)(rr - (uint32_t)readlane((int)excl, L));
            int e_sel = 0;
            bool got = false;
#pragma unroll
            for (int e = 0; e < V; ++e) {
                if (!got && ((cm[e] >> L) & 1)) {
                    if (left == 0) { e_sel = e; got = true; }
                    else left--;
                }
            }
            out.L = L;
            out.j = ss * V + e_sel;
            out.i = ss * SPAN + L * V + e_sel;
        });
        out.d = readlane(K(out.j), out.L) >> KB;
        return out;
    }

    // Domain threshold of iteration t: non-tabu bits, or every valid bit when
    // all are tabu (R11); also returns the domain's least key.
    __device__ __forceinline__ int domain(int t, int &km, int &mm) {
        km = lane_min_dom(t);
        mm = wave_min(km >> LOGV);
        if (!empty_dom(mm)) return t;
        km = kminU;
        mm = mU;
        return EX_ALWAYS;
    }

    // MaxMin (Section III-A.3).  The domain reductions of iteration t+1 (its
    // least and greatest key) are made by the refresh after the flip of
    // iteration t; the tabu mark of iteration t precedes that flip.
    __device__ __forceinline__ int phase_maxmin(int T, int tau, uint32_t ph) {
        dom_minmax(1);                      // iteration 1: nothing is tabu
        FracStep fs;
        fs.init((uint32_t)T);
        R4 r = {{0u, 0u, 0u, 0u}};
        for (int t = 1; t <= T; ++t) {
            fs.next();
            int thr = t;
            if (empty_dom(mM)) {            // every bit tabu: tabu ignored (R11)
                thr = EX_ALWAYS;
                mM = mU;
                int kx = -KEY_OUT;
#pragma unroll
                for (int j = 0; j < EPL; ++j) kx = max(kx, ex[j] < thr ? K(j) : -KEY_OUT);
                mX = wave_max(kx);
            }
            const int mind = mM >> SB;
            const int maxd = mX >> KB;
            // iterations 2c+1 and 2c+2 use words (0, 1) and (2, 3) of draw c (R18)
            if (!((t - 1) & 1)) r = philox((uint32_t)((t - 1) >> 1), inst, ph, (uint32_t)TAG_MAXMIN << 24, seed);
            const uint32_t u = ((t - 1) & 1) ? r.w[2] : r.w[0], v = ((t - 1) & 1) ? r.w[3] : r.w[1];
            const uint64_t g = fs.rest();   // floor(2^32 (T - t) / T)
            const uint64_t span = ((uint64_t)(uint32_t)(maxd - mind) * cube_frac(g)) >> 32;
            const int d = mind + (int)(((uint64_t)u * (span + 1)) >> 32);
            const int dk = d * (1 << KB) + ((1 << KB) - 1);
            const Sel s = pick_rth(dk, thr, v);
            mark_tabu(s, t, tau);
            flip_core(s);
            refresh_minmax(t + 1);
        }
        ex_reset();
        return T;
    }

    // PositiveMin (Section III-A.6).  Its domain's least key only decides
    // whether the domain is empty; with n > tau at most tau bits are tabu, so
    // it never is and that reduction is skipped.
    __device__ __forceinline__ int phase_positivemin(int T, int tau, uint32_t ph) {
        const bool may_empty = n <= tau;
        R4 r = {{0u, 0u, 0u, 0u}};
        for (int t = 1; t <= T; ++t) {
            int thr = t;
            if (may_empty) {
                int km, mm;
                thr = domain(t, km, mm);
            }
            int kp = KEY_OUT;
#pragma unroll
            for (int j = 0; j < EPL; j += 2) {
                const int a = (ex[j] < thr && K(j) >= (1 << KB)) ? K(j) : KEY_OUT;
                const int b = (ex[j + 1] < thr && K(j + 1) >= (1 << KB)) ? K(j + 1) : KEY_OUT;
                kp = min(kp, min(a, b));
            }
            const int pd = wave_min(kp >> LOGV) >> SB;
            const int d = pd >= H_PAD ? H_PAD - 1 : pd;
            const int dk = d * (1 << KB) + ((1 << KB) - 1);
            // iterations 4c+1 .. 4c+4 use words 0 .. 3 of draw c (R18)
            if (!((t - 1) & 3)) r = philox((uint32_t)((t - 1) >> 2), inst, ph, (uint32_t)TAG_POSMIN << 24, seed);
            const int q4 = (t - 1) & 3;
            const uint32_t u = q4 == 0 ? r.w[0] : (q4 == 1 ? r.w[1] : (q4 == 2 ? r.w[2] : r.w[3]));
            const Sel s = pick_rth(dk, thr, u);
            flip(s);
            mark_tabu(s, t, tau);
        }
        ex_reset();
        return T;
    }

    // RandomMin (Section III-A.5): candidates by random byte < q(t).
    __device__ __forceinline__ int phase_randommin(int T, int tau, uint32_t ph) {
        FracStep fs;
        fs.init((uint32_t)T);
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
            int kr = KEY_OUT;
            // lane's random words for slot s: wa (bytes of elements 0..3), wb (4..7)
            auto cand = [&](int s, uint32_t wa, uint32_t wb) {
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const int j = s * V + e;
                    const uint32_t word = e < 4 ? wa : wb;
                    const int byte = (int)((word >> (8 * (e & 3))) & 0xFFu);
                    kr = min(kr, (byte < q && ex[j] < t) ? K(j) : KEY_OUT);
                }
            };
            const uint32_t tag = (uint32_t)TAG_RANDMIN << 24;
            if constexpr (V == 8 && SLOTS % 2 == 0) {
                // Lanes 2m and 2m+1 share the draw of bits 16m .. 16m+15 of a
                // slot (bytes 0..7 and 8..15).  Even lanes draw for even slots,
                // odd lanes for odd slots, and each pair swaps the halves.
                const bool odd = lane & 1;
#pragma unroll
                for (int u = 0; u < SLOTS; u += 2) {
                    const int s_own = u + (odd ? 1 : 0);
                    const R4 r = philox((uint32_t)t, inst, ph, tag | (uint32_t)((s_own * SPAN + lane * V) >> 4), seed);
                    const uint32_t ra = swap_pair(odd ? r.w[0] : r.w[2]);
                    const uint32_t rb = swap_pair(odd ? r.w[1] : r.w[3]);
                    // slot u: even lane own words 0, 1; odd lane the even neighbour's 2, 3
                    cand(u, odd ? ra : r.w[0], odd ? rb : r.w[1]);
                    // slot u+1: even lane the odd neighbour's 0, 1; odd lane own 2, 3
                    cand(u + 1, odd ? r.w[2] : ra, odd ? r.w[3] : rb);
                }
            } else {
#pragma unroll
                for (int s = 0; s < SLOTS; ++s) {
                    const int k0 = s * SPAN + lane * V;
                    const R4 r = philox((uint32_t)t, inst, ph, tag | (uint32_t)(k0 >> 4), seed);
                    // this lane's V bytes start at byte (k0 mod 16) of the draw
                    const int w0 = (k0 & 15) >> 2;
                    const uint32_t wa = w0 == 0 ? r.w[0] : (w0 == 1 ? r.w[1] : (w0 == 2 ? r.w[2] : r.w[3]));
                    const uint32_t wb = w0 == 0 ? r.w[1] : (w0 == 1 ? r.w[2] : r.w[3]);
                    cand(s, wa, wb);
                }
            }
            const int m = wave_min(kr >> LOGV);
            const Sel s = empty_dom(m) ? dom_argmin(t) : argmin_from(kr, m);
            flip(s);
            mark_tabu(s, t, tau);
        }
        ex_reset();
        return T;
    }

    // TwoNeighbor (Section III-A.7): 0, 1, 0, 2, 1, 3, 2, ...
    __device__ __forceinline__ int phase_twoneighbor() {
        flip(sel_of(0));
        for (int k = 1; k < n; ++k) {
            flip(sel_of(k));
            flip(sel_of(k - 1));
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
