// dabs_wide.h -- the search of one instance per wavefront for dense problems
// whose delta bound B does not fit the packed key words of dabs_walker.h:
// any B <= 2^31 - 1 (Section II: every delta Delta_k = E(f_k X) - E(X) is
// then an int32), int16 weights of -32768 and int32 weights beyond 24 bits.
//
// Same rules, readings, random draws and results as the packed walker; only
// the representation differs.  Lane l holds, per slot s, the V = 16 /
// sizeof(W) bits k = s 64 V + l V + e (local index j = s V + e) as plain int32
// deltas, and the rule domains as bit masks over j (exclusions: tabu,
// Straight's settled bits).  A selection is a wave minimum of the deltas in a
// mask, then the lowest bit index holding that minimum (R5) from one ballot
// per slot; padding bits hold INT32_MAX and are outside every mask.
#pragma once
#include "dabs_device.h"
#include "dabs_walker.h"

namespace dabs {

template <typename WT, int SLOTS>
struct WideWalker {
    static constexpr int V = 16 / (int)sizeof(WT);
    static constexpr int LOGV = V == 8 ? 3 : 2;
    static constexpr int EPL = V * SLOTS;
    static constexpr int SPAN = WAVE * V;
    static constexpr int DNONE = 0x7FFFFFFF;          // masked-out value of minima
    typedef typename MaskOf<EPL <= 32>::type mask_t;
    static constexpr mask_t ONE = 1;
    typedef typename RegVec<EPL>::vh vecH;
    RegVec<EPL> dl;                                   // deltas, element j = s V + e

    __device__ __forceinline__ WideWalker(vecH &d0, vecH &d1) : dl(d0, d1) {}

    const WT *W;
    const int *diag;
    int64_t ld;
    int n;
    uint64_t seed;
    uint32_t inst;
    int lane;
    mask_t xb, bb, vb, ex;     // X, BEST, valid bits, excluded bits
    int64_t E, Eb;
    int mAll;                  // least delta over all bits at the current X
    int ring;                  // tabu ring (as in the packed walker)
    unsigned long long *hit;
    bool hit_done;
    int64_t target;
    unsigned long long t0;
    int *trace;
    int trace_cap, flips;

    __device__ __forceinline__ int gidx(int s, int e) const { return s * SPAN + lane * V + e; }

    __device__ __forceinline__ void setup(const WT *Wp, const int *dg, int64_t ld_, int n_, uint64_t seed_,
                                          uint32_t inst_) {
        W = Wp; diag = dg; ld = ld_; n = n_; seed = seed_; inst = inst_;
        lane = lane_id();
        vb = 0;
#pragma unroll
        for (int s = 0; s < SLOTS; ++s)
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int j = s * V + e, k = gidx(s, e);
                if (k < n) vb |= ONE << j;
                dl.set(j, k < n ? diag[k] : DNONE);   // X = 0: Delta_k = W_kk
            }
        xb = 0; bb = 0; ex = 0; E = 0; Eb = 0; mAll = 0;
        ring = -1;
        hit = nullptr; hit_done = true; target = 0; t0 = 0;
        trace = nullptr; trace_cap = 0; flips = 0;
    }

    // --------------------------------------------------------- reductions
    __device__ __forceinline__ int lane_min_all() const {
        int m = DNONE;
#pragma unroll
        for (int j = 0; j < EPL; ++j) m = min(m, dl[j]);
        return m;
    }
    __device__ __forceinline__ int lane_min(mask_t pm) const {
        int m = DNONE;
#pragma unroll
        for (int j = 0; j < EPL; ++j) m = ((pm >> j) & 1) ? min(m, dl[j]) : m;
        return m;
    }
    __device__ __forceinline__ int lane_max(mask_t pm) const {
        int m = (int)0x80000000;
#pragma unroll
        for (int j = 0; j < EPL; ++j) m = ((pm >> j) & 1) ? max(m, dl[j]) : m;
        return m;
    }
    static __device__ __forceinline__ bool any(mask_t pm) { return ballot(pm != 0) != 0; }

    // Lowest bit index of the mask whose delta is m (a value the mask holds).
    __device__ __forceinline__ Sel argmin_eq(mask_t pm, int m) const {
        Sel r;
        r.d = m; r.i = 0; r.L = 0; r.j = 0;
        bool found = false;
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            uint32_t h = 0;
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int j = s * V + e;
                h |= (((pm >> j) & 1) && dl[j] == m) ? (1u << e) : 0u;
            }
            const uint64_t b = ballot(h != 0);
            if (!found && b) {
                found = true;
                const int L = (int)__builtin_ctzll(b);
                const int e = __builtin_ctz((uint32_t)readlane((int)h, L));
                r.L = L;
                r.j = s * V + e;
                r.i = s * SPAN + L * V + e;
            }
        }
        return r;
    }
    // argmin (least delta, then lowest index) over a non-empty mask
    __device__ __forceinline__ Sel argmin(mask_t pm) const { return argmin_eq(pm, wave_min(lane_min(pm))); }

    __device__ __forceinline__ Sel sel_of(int i) {
        Sel s;
        s.i = i;
        s.L = (i >> LOGV) & (WAVE - 1);
        s.j = ((i / SPAN) << LOGV) | (i & (V - 1));
        s.d = readlane(dl[s.j], s.L);
        return s;
    }

    // ------------------------------------------------------------ flips
    __device__ __forceinline__ void load_row(int i, uint4 (&q)[SLOTS]) const {
        if ((unsigned)i >= (unsigned)n) i = 0;     // never read outside W
        const WT *row = W + (int64_t)i * ld + lane * V;
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) q[s] = *(const uint4 *)(row + s * SPAN);
    }
    // Delta_j += 2 W_ij (1 - 2x_i)(1 - 2x_j) (Eq. (4)); |2 W_ij| <= B fits, and
    // so does every updated delta.  Then Delta_i = -Delta_i (Eq. (5)).
    __device__ __forceinline__ void flip_bit(const Sel &s) {
        uint4 q[SLOTS];
        load_row(s.i, q);
        const int si = ((lane_mask(xb, s.L) >> s.j) & 1) ? -1 : 0;
        auto upd = [&](int j, int w) {
            const int c = si ^ -(int)((xb >> j) & 1);             // -1 when x_i != x_j
            const int w2 = (int)((uint32_t)w << 1);
            dl.set(j, (int)((uint32_t)dl[j] + (uint32_t)((w2 ^ c) - c)));
        };
#pragma unroll
        for (int t = 0; t < SLOTS; ++t) {
            const uint32_t d[4] = {q[t].x, q[t].y, q[t].z, q[t].w};
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                if constexpr (sizeof(WT) == 2) {
                    upd(t * V + 2 * p, (int)(int16_t)(d[p] & 0xFFFFu));
                    upd(t * V + 2 * p + 1, (int)d[p] >> 16);
                } else {
                    upd(t * V + p, (int)d[p]);
                }
            }
        }
        const int o = dl[s.j];
        dl.set(s.j, lane == s.L ? -o : o);
        xb ^= lane == s.L ? (ONE << s.j) : (mask_t)0;
    }

    __device__ __forceinline__ void note_best() {
        if (!hit_done && Eb <= target) {
            hit_done = true;
            const unsigned long long now = __builtin_amdgcn_s_memrealtime();
            if (lane == 0) atomicMin(hit, now - t0);
        }
    }
    // Step 1 (R3): BEST <- the best 1-bit neighbour when strictly better.
    __device__ __forceinline__ void step1() {
        mAll = wave_min(lane_min_all());
        if (E + mAll < Eb) {
            const Sel s = argmin_eq(vb, mAll);
            Eb = E + mAll;
            bb = xb ^ (lane == s.L ? (ONE << s.j) : (mask_t)0);
            note_best();
        }
    }
    __device__ __forceinline__ void flip(const Sel &s0) {
        const Sel s = uniform(s0);
        E += s.d;
        flip_bit(s);
        if (trace && flips < trace_cap && lane == 0) trace[flips] = s.i;
        flips++;
        step1();
    }
    __device__ __forceinline__ void begin() {
        bb = xb;
        Eb = E;
        note_best();
        step1();
    }

    // X := x, walking from X = 0 by flips in increasing index.
    __device__ __forceinline__ void load_x(const uint64_t *x) {
        const int nw = (n + 63) / 64;
        for (int w = 0; w < nw; ++w) {
            uint64_t word = x[w];
            // (wave-uniform: a scalar loop over the set bits)
            word = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(word >> 32)) << 32) |
                   (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)word);
            if (w == nw - 1 && (n & 63)) word &= (1ull << (n & 63)) - 1;
            while (word) {
                const int b = __builtin_ctzll(word);
                word &= word - 1;
                const Sel s = uniform(sel_of(w * 64 + b));
                E += s.d;
                flip_bit(s);
            }
        }
    }
    __device__ __forceinline__ void store_bits(mask_t bits, uint64_t *out) const {
        const int nw = (n + 63) / 64;
        constexpr int LPW = WAVE / V;
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            uint64_t v = (((uint64_t)bits >> (s * V)) & ((1ull << V) - 1)) << ((lane % LPW) * V);
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
                if (k < n) out[k] = dl[s * V + e];
            }
    }

    // ------------------------------------------------------- exclusions
    __device__ __forceinline__ void mark(const Sel &s) { ex |= lane == s.L ? (ONE << s.j) : (mask_t)0; }
    __device__ __forceinline__ void unmark(int j, int L) { ex &= lane == L ? ~(ONE << j) : ~(mask_t)0; }
    // Tabu (R11), as in the packed walker: the bit flipped at iteration t is
    // excluded at t+1 .. t+tau; one chosen from an empty domain may be
    // excluded already, and its pending release is then void.
    __device__ __forceinline__ void tabu_mark(const Sel &s0, int t, int tau, bool maybe_marked) {
        if (tau <= 0) return;
        const Sel s = uniform(s0);
        const int e = (s.L << 8) | s.j;
        if (maybe_marked && ((lane_mask(ex, s.L) >> s.j) & 1)) {
            for (int u = t - tau; u < t; ++u)
                if (u >= 1 && readlane(ring, u & 31) == e) ring = lane == (u & 31) ? -1 : ring;
        }
        mark(s);
        ring = lane == (t & 31) ? e : ring;
    }
    __device__ __forceinline__ void tabu_release(int t, int tau) {
        const int t0r = t - tau - 1;
        if (tau > 0 && t0r >= 1) {
            const int e = readlane(ring, t0r & 31);
            if (e >= 0) unmark(e & 255, e >> 8);
        }
    }

    // ------------------------------------------------------------ rules
    // Greedy (Section III-A.1).
    __device__ __forceinline__ int phase_greedy(int cap) {
        if (cap <= 0) cap = 64 * n;
        int f = 0;
        while (mAll < 0 && f < cap) {
            flip(argmin_eq(vb, mAll));
            f++;
        }
        return f;
    }

    // Straight (Section III-A.2): argmin over the bits differing from the
    // target; the agreeing bits and each flipped bit are excluded.
    __device__ __forceinline__ int phase_straight(const uint64_t *target_bits) {
        const int nw = (n + 63) / 64;
        uint64_t db = 0;
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            const int k0 = s * SPAN + lane * V;
            const int w = k0 >> 6;
            const uint64_t word = w < nw ? target_bits[w] : 0ull;
            db |= ((word >> (k0 & 63)) & ((1ull << V) - 1)) << (s * V);
        }
        const mask_t diff = (xb ^ (mask_t)db) & vb;
        ex = ~diff;
        const int hd = (int)wave_sum64((long long)__builtin_popcountll((uint64_t)diff));
        int f = 0;
        for (; f < hd; ++f) {
            const Sel s = uniform(argmin(vb & ~ex));
            mark(s);
            flip(s);
        }
        ex = 0;
        return f;
    }

    // Tabu greedy: T iterations of the non-tabu argmin.
    __device__ __forceinline__ int phase_tabu_greedy(int T, int tau) {
        for (int t = 1; t <= T; ++t) {
            tabu_release(t, tau);
            const mask_t dom = vb & ~ex;
            const bool emp = !any(dom);
            const Sel s = emp ? argmin_eq(vb, mAll) : argmin(dom);
            tabu_mark(s, t, tau, emp);
            flip(s);
        }
        ex = 0;
        return T;
    }

    // CyclicMin (Section III-A.4, R8).
    __device__ __forceinline__ int phase_cyclicmin(int T, int tau) {
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
            mask_t win = 0;
#pragma unroll
            for (int s = 0; s < SLOTS; ++s)
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const uint32_t off = (uint32_t)(gidx(s, e) - lo);
                    win |= (wrap ? (off >= span) : (off < span)) ? (ONE << (s * V + e)) : (mask_t)0;
                }
            win &= vb;
            const mask_t dom = win & ~ex;
            const bool emp = !any(dom);
            const Sel s = emp ? argmin(win) : argmin(dom);
            flip(s);
            tabu_mark(s, t, tau, emp);
            pos = (pos + w) % n;
        }
        ex = 0;
        return T;
    }

    // Position of set bit number k (0-based) of a V-bit mask.
    static __device__ __forceinline__ int kth_bit(uint32_t b, uint32_t k) {
        int pos = 0;
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const bool set = (b >> e) & 1;
            if (set && k == 0) { pos = e; break; }
            k -= set ? 1u : 0u;
        }
        return pos;
    }
    // R6: the candidates are the bits of pm with delta <= d; with c of them,
    // r = floor(v c / 2^32) and the r-th candidate in increasing bit index.
    __device__ __forceinline__ Sel pick_rth(mask_t pm, int d, uint32_t v) {
        mask_t cm = 0;
#pragma unroll
        for (int j = 0; j < EPL; ++j) cm |= (((pm >> j) & 1) && dl[j] <= d) ? (ONE << j) : (mask_t)0;
        uint32_t cs[SLOTS];
        uint32_t c = 0;
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            cs[s] = 0;
#pragma unroll
            for (int e = 0; e < V; ++e) cs[s] += (uint32_t)__builtin_popcountll(ballot((cm >> (s * V + e)) & 1));
            c += cs[s];
        }
        if (c == 0) return argmin(pm);              // cannot happen: the least delta of pm qualifies
        uint32_t r = scale32(v, c);
        Sel out;
        out.L = 0; out.j = 0; out.i = 0;
        bool found = false;
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) {
            if (!found && r < cs[s]) {
                found = true;
                // candidates of the slot in lower lanes, and this lane's own
                uint32_t excl = 0, cb = 0;
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const bool ce = (cm >> (s * V + e)) & 1;
                    const uint64_t bm = ballot(ce);
                    cb |= ce ? (1u << e) : 0u;
                    excl = __builtin_amdgcn_mbcnt_hi((uint32_t)(bm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bm, excl));
                }
                const uint64_t le = ballot(excl <= r);
                const int L = 63 - __builtin_clzll(le | 1ull);
                const uint32_t left = r - (uint32_t)readlane((int)excl, L);
                const int e_sel = __builtin_amdgcn_readfirstlane(kth_bit((uint32_t)readlane((int)cb, L), left));
                out.L = L;
                out.j = s * V + e_sel;
                out.i = s * SPAN + L * V + e_sel;
            } else if (!found) {
                r -= cs[s];
            }
        }
        out.L = __builtin_amdgcn_readfirstlane(out.L);
        out.j = __builtin_amdgcn_readfirstlane(out.j);
        out.i = __builtin_amdgcn_readfirstlane(out.i);
        out.d = readlane(dl[out.j], out.L);
        return out;
    }

    // MaxMin (Section III-A.3, R7).  Iterations 2c+1 and 2c+2 use words (0, 1)
    // and (2, 3) of draw c (R18).
    __device__ __forceinline__ int phase_maxmin(int T, int tau, uint32_t ph) {
        FracStep fs;
        fs.init((uint32_t)T);
        for (int t = 1; t <= T; ++t) {
            fs.next();
            const uint64_t cf = cube_frac(fs.rest());
            const R4 rv = philox((uint32_t)((t - 1) >> 1), inst, ph, (uint32_t)TAG_MAXMIN << 24, seed);
            const bool second = (t - 1) & 1;
            const uint32_t u = second ? rv.w[2] : rv.w[0], v = second ? rv.w[3] : rv.w[1];
            tabu_release(t, tau);
            mask_t dom = vb & ~ex;
            const bool ign = !any(dom);                 // every bit tabu: tabu ignored (R11)
            if (ign) dom = vb;
            const int mind = wave_min(lane_min(dom));
            const int maxd = wave_max(lane_max(dom));
            const uint64_t span = ((uint64_t)((uint32_t)maxd - (uint32_t)mind) * cf) >> 32;
            const int d = (int)((int64_t)mind + (int64_t)(((uint64_t)u * (span + 1)) >> 32));
            const Sel s = pick_rth(dom, d, v);
            tabu_mark(s, t, tau, ign);
            flip(s);
        }
        ex = 0;
        return T;
    }

    // PositiveMin (Section III-A.6): the candidates are the domain's bits with
    // delta <= its least positive delta (all of them when none is positive).
    // Iterations 4c+1 .. 4c+4 use words 0 .. 3 of draw c (R18).
    __device__ __forceinline__ int phase_positivemin(int T, int tau, uint32_t ph) {
        const bool may_empty = n <= tau;
        for (int t = 1; t <= T; ++t) {
            tabu_release(t, tau);
            mask_t dom = vb & ~ex;
            bool ign = false;
            if (may_empty) ign = !any(dom);
            if (ign) dom = vb;
            int lp = DNONE;
#pragma unroll
            for (int j = 0; j < EPL; ++j) lp = (((dom >> j) & 1) && dl[j] > 0) ? min(lp, dl[j]) : lp;
            const int d = wave_min(lp);                 // DNONE: no positive delta, every bit qualifies
            const R4 rv = philox((uint32_t)((t - 1) >> 2), inst, ph, (uint32_t)TAG_POSMIN << 24, seed);
            const int q4 = (t - 1) & 3;
            const uint32_t u = q4 == 0 ? rv.w[0] : (q4 == 1 ? rv.w[1] : (q4 == 2 ? rv.w[2] : rv.w[3]));
            const Sel s = pick_rth(dom, d, u);
            flip(s);
            tabu_mark(s, t, tau, ign);
        }
        ex = 0;
        return T;
    }

    // RandomMin (Section III-A.5, R9): the byte of bit k is byte k mod 16 of
    // the draw (t, instance, phase, tag | k / 16).
    __device__ __forceinline__ int phase_randommin(int T, int tau, uint32_t ph) {
        FracStep fs;
        fs.init((uint32_t)T);
        const uint32_t tag = (uint32_t)TAG_RANDMIN << 24;
        for (int t = 1; t <= T; ++t) {
            fs.next();
            int q;
            if (t >= T) {
                q = 256;
            } else {
                const int qq = (int)(cube_frac(fs.q) >> 24);
                const int qmin = (8192 + n - 1) / n;
                q = qq < qmin ? qmin : (qq > 256 ? 256 : qq);
            }
            tabu_release(t, tau);
            mask_t cm = 0;
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
                const int k0 = s * SPAN + lane * V;
                const R4 r = philox((uint32_t)t, inst, ph, tag | (uint32_t)(k0 >> 4), seed);
                const int w0 = (k0 & 15) >> 2;
                const uint32_t wa = w0 == 0 ? r.w[0] : (w0 == 1 ? r.w[1] : (w0 == 2 ? r.w[2] : r.w[3]));
                const uint32_t wb = w0 == 0 ? r.w[1] : (w0 == 1 ? r.w[2] : r.w[3]);
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const uint32_t word = e < 4 ? wa : wb;
                    const int byte = (int)((word >> (8 * (e & 3))) & 0xFFu);
                    cm |= byte < q ? (ONE << (s * V + e)) : (mask_t)0;
                }
            }
            const mask_t dom = vb & ~ex;
            bool emp = false;
            Sel s;
            if (any(cm & dom)) {
                s = argmin(cm & dom);
            } else if (any(dom)) {
                s = argmin(dom);                        // no candidate: the non-tabu argmin
            } else {
                emp = true;                             // every bit tabu: the plain argmin
                s = argmin_eq(vb, mAll);
            }
            flip(s);
            tabu_mark(s, t, tau, emp);
        }
        ex = 0;
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

    // Batch search (Section III-B): Straight -> Greedy -> {main -> Greedy}*.
    __device__ __forceinline__ int batch(const uint64_t *target_bits, int rule, int T, int Bn, int tau, uint32_t &ph,
                                         int cap) {
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
