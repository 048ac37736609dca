/*
 * dabs_oracle.c -- CPU oracle for the bulk-search hot path of Diverse Adaptive
 * Bulk Search (Nakano, Takafuji, Ito et al., "Diverse Adaptive Bulk Search: a
 * Framework for Solving QUBO Problems on Multiple GPUs", arXiv 2207.03069).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the CPU-baseline leg of the benchmark load this file.  It shares no code,
 * header, table or helper with the HIP implementation, and the product path
 * never calls it.
 *
 * Plain and slow on purpose: one byte per bit, int64 energies and deltas,
 * every selection scans the n bits in increasing index order.  Each function
 * names the passage of the paper it follows; where the paper is silent or
 * ambiguous the reading taken is stated next to the code (the readings are
 * numbered R1.. and listed together with the design notes).
 *
 * Energy convention (R1): E(X) = sum_i sum_j W_ij x_i x_j over ALL ordered
 * pairs (i,j), W symmetric -- Section II, Eq. (2), whose index set E u VxV is
 * the whole of VxV.  Table III's QUBO optima equal C - n p only under this
 * full sum.  Hence the per-pair update of Eq. (4) carries a factor 2.
 *
 * Pins: energies, deltas, Greedy, Straight, TwoNeighbor, tabu-greedy,
 * CyclicMin, Step 1, the batch schedule, rank selection, the genetic
 * operations (IntervalZero's single cyclic segment and its length range
 * included), the learned operations (equivalences with Mutation at
 * hand-derived thresholds), the restart of merged pools and the pools are
 * pinned by the tests against scratch energies, brute force, printed
 * examples and closed forms.  The random choices of MaxMin, PositiveMin and
 * RandomMin are pinned in distribution: RandomMin's candidate rate against
 * the real schedule max((t/T)^3, 32/n), the MaxMin / PositiveMin pick by
 * chi-square uniformity over fixed candidate sets, plus their threshold
 * ranges and candidate sets.  Which candidate one particular draw selects
 * (the readings R6, R7, R9 and R18) is fixed only by agreement with the
 * device.
 */
#include <stdint.h>
#include <stdlib.h>
#include <math.h>
#include <string.h>
#include "dabs_oracle.h"

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11): 10 rounds of the Philox S-box on a 128-bit     */
/* counter under a 64-bit key; the key is bumped by the Weyl constants      */
/* between rounds.  Written from the published round definition.            */
/* ------------------------------------------------------------------------ */
void orc_philox(const uint32_t ctr[4], uint64_t seed, uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw4(uint64_t seed, uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t out[4])
{
    uint32_t ctr[4] = {a, b, c, d};
    orc_philox(ctr, seed, out);
}

/* u32 draw scaled to [0, m): floor(u * m / 2^32). */
static uint32_t scale_u32(uint32_t u, uint32_t m)
{
    return (uint32_t)(((uint64_t)u * (uint64_t)m) >> 32);
}

/* ------------------------------------------------------------------------ */
/* Energy and flip deltas                                                   */
/* ------------------------------------------------------------------------ */

/* Eq. (2), read as the full ordered double sum (R1). */
int64_t orc_energy(const int32_t *W, int32_t n, const uint8_t *x)
{
    int64_t e = 0;
    for (int32_t i = 0; i < n; i++) {
        if (!x[i]) continue;
        for (int32_t j = 0; j < n; j++)
            if (x[j]) e += W[(int64_t)i * n + j];
    }
    return e;
}

/* Definition of Delta_k in Section III: E(f_k(X)) - E(X), both energies
 * computed from scratch.  O(n^3) for all k; for small cases and pins only. */
void orc_delta_scratch(const int32_t *W, int32_t n, const uint8_t *x, int64_t *delta)
{
    uint8_t *y = (uint8_t *)malloc((size_t)n);
    memcpy(y, x, (size_t)n);
    int64_t e = orc_energy(W, n, x);
    for (int32_t k = 0; k < n; k++) {
        y[k] ^= 1;
        delta[k] = orc_energy(W, n, y) - e;
        y[k] ^= 1;
    }
    free(y);
}

/* Closed form of Delta_k (Eq. (3)) under the full-sum convention:
 *   Delta_k = (1 - 2 x_k) * (W_kk + 2 * sum_{j != k} W_kj x_j).
 * Flipping x_k changes the diagonal term by (1-2x_k) W_kk and each of the two
 * ordered off-diagonal terms (k,j), (j,k) by (1-2x_k) W_kj x_j. */
void orc_delta_closed(const int32_t *W, int32_t n, const uint8_t *x, int64_t *delta)
{
    for (int32_t k = 0; k < n; k++) {
        int64_t s = W[(int64_t)k * n + k];
        for (int32_t j = 0; j < n; j++)
            if (j != k && x[j]) s += 2 * (int64_t)W[(int64_t)k * n + j];
        delta[k] = x[k] ? -s : s;
    }
}

/* Largest |Delta_k| any X can produce: max_k |W_kk| + 2 sum_{j!=k} |W_kj|. */
int64_t orc_delta_bound(const int32_t *W, int32_t n)
{
    int64_t b = 0;
    for (int32_t k = 0; k < n; k++) {
        int64_t s = llabs((long long)W[(int64_t)k * n + k]);
        for (int32_t j = 0; j < n; j++)
            if (j != k) s += 2 * llabs((long long)W[(int64_t)k * n + j]);
        if (s > b) b = s;
    }
    return b;
}

int32_t orc_is_symmetric(const int32_t *W, int32_t n)
{
    for (int32_t i = 0; i < n; i++)
        for (int32_t j = i + 1; j < n; j++)
            if (W[(int64_t)i * n + j] != W[(int64_t)j * n + i]) return 0;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Incremental search state (Section III-A)                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n;
    const int32_t *W;
    uint8_t *x;          /* current X */
    int64_t E;           /* E(X) */
    int64_t *delta;      /* Delta_k(X) */
    uint8_t *best;       /* BEST */
    int64_t ebest;       /* E(BEST) */
    int64_t flips;       /* flips executed since the state was set up */
    int32_t *trace;      /* optional: flipped index per flip */
    int64_t trace_cap;
    int32_t verify;      /* if non-zero: recompute Delta and E from scratch after every flip */
    int32_t error;       /* set on a verification mismatch */
    /* search-rule context */
    uint64_t seed;
    uint32_t inst;
} state_t;

static void state_load(state_t *st, const int32_t *W, int32_t n, uint8_t *x, int64_t *delta, uint8_t *best)
{
    memset(st, 0, sizeof(*st));
    st->n = n; st->W = W; st->x = x; st->delta = delta; st->best = best;
    st->E = orc_energy(W, n, x);
    orc_delta_closed(W, n, x, delta);
    /* R4: BEST starts at the starting vector. */
    memcpy(best, x, (size_t)n);
    st->ebest = st->E;
}

/* First index attaining the minimum of delta[] (R5: lowest index on ties). */
static int32_t argmin_all(const state_t *st)
{
    int32_t j = 0;
    for (int32_t k = 1; k < st->n; k++)
        if (st->delta[k] < st->delta[j]) j = k;
    return j;
}

/* Step 1 of the incremental search: the best 1-bit neighbour f_j(X) replaces
 * BEST when strictly better (R3: j = argmin_k E(f_k X), lowest k on ties). */
static void step1(state_t *st)
{
    int32_t j = argmin_all(st);
    int64_t e = st->E + st->delta[j];
    if (e < st->ebest) {
        memcpy(st->best, st->x, (size_t)st->n);
        st->best[j] ^= 1;
        st->ebest = e;
    }
}

static void verify_state(state_t *st)
{
    int64_t *d = (int64_t *)malloc(sizeof(int64_t) * (size_t)st->n);
    orc_delta_closed(st->W, st->n, st->x, d);
    for (int32_t k = 0; k < st->n; k++)
        if (d[k] != st->delta[k]) st->error = 1;
    if (orc_energy(st->W, st->n, st->x) != st->E) st->error = 1;
    free(d);
}

/* Step 3: X <- f_i(X), E <- E + Delta_i, Delta updated by Eq. (4) for k != i
 * (factor 2 from the full sum, sigma taken before the flip) and Eq. (5) for
 * k = i.  Step 1 then runs at the new state (R4: at every visited state). */
static void flip(state_t *st, int32_t i)
{
    const int32_t n = st->n;
    const int64_t si = st->x[i] ? 1 : -1;              /* sigma(x_i) = 2 x_i - 1 */
    const int32_t *row = st->W + (int64_t)i * n;
    for (int32_t k = 0; k < n; k++) {
        if (k == i) continue;
        const int64_t sk = st->x[k] ? 1 : -1;
        st->delta[k] += 2 * (int64_t)row[k] * si * sk;
    }
    st->E += st->delta[i];
    st->delta[i] = -st->delta[i];
    st->x[i] ^= 1;
    if (st->trace && st->flips < st->trace_cap) st->trace[st->flips] = i;
    st->flips++;
    if (st->verify) verify_state(st);
    step1(st);
}

/* ------------------------------------------------------------------------ */
/* Search rules (Section III-A).  Each runs one phase from the current state */
/* and returns the number of flips it made.  t counts the iterations of the  */
/* phase from 1; the tabu list is private to the phase (R11).               */
/* ------------------------------------------------------------------------ */

#define NEVER (INT64_MIN / 4)

typedef struct {
    int64_t *last;   /* iteration at which each bit was last flipped in this phase */
    int32_t tau;
} tabu_t;

static void tabu_init(tabu_t *tb, int32_t n, int32_t tau)
{
    tb->last = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t k = 0; k < n; k++) tb->last[k] = NEVER;
    tb->tau = tau;
}

static void tabu_free(tabu_t *tb) { free(tb->last); }

/* R11: a bit flipped at iteration t0 may not be flipped at t0+1 .. t0+tau. */
static int is_tabu(const tabu_t *tb, int32_t k, int64_t t)
{
    return tb->tau > 0 && tb->last[k] != NEVER && t - tb->last[k] <= tb->tau;
}

/* Integer cube of a 32.32 fixed-point fraction: floor-chained (f^2/2^32) f/2^32. */
static uint64_t cube_frac(uint64_t f)
{
    return (((f * f) >> 32) * f) >> 32;
}

/* R8: CyclicMin window width w(t) = max((t/T)^3 n, c), c = min(32, n), in
 * 32.32 fixed point, and w(T) = n. */
static int64_t cyclic_width(int64_t t, int64_t T, int32_t n)
{
    if (t >= T) return n;
    uint64_t h = ((uint64_t)t << 32) / (uint64_t)T;
    int64_t w = (int64_t)(((uint64_t)n * cube_frac(h)) >> 32);
    int64_t c = n < 32 ? n : 32;
    if (w < c) w = c;
    if (w > n) w = n;
    return w;
}

/* R9: RandomMin candidate threshold q(t) in 1/256 units:
 * p(t) = max((t/T)^3, 32/n) quantised, q(T) = 256. */
static int32_t randmin_q(int64_t t, int64_t T, int32_t n)
{
    if (t >= T) return 256;
    uint64_t h = ((uint64_t)t << 32) / (uint64_t)T;
    int64_t q = (int64_t)(cube_frac(h) >> 24);
    int64_t qmin = (8192 + (int64_t)n - 1) / n;       /* ceil(32 * 256 / n) */
    if (q < qmin) q = qmin;
    if (q > 256) q = 256;
    return (int32_t)q;
}

int32_t orc_randmin_q(int64_t t, int64_t T, int32_t n)
{
    return randmin_q(t, T, n);
}

/* R7: MaxMin threshold d drawn uniformly from [minD, D(t)] with
 * D(t) = (1 - ((T-t)/T)^3) minD + ((T-t)/T)^3 maxD, in fixed point. */
static int64_t maxmin_threshold(int64_t t, int64_t T, int64_t mind, int64_t maxd, uint32_t u)
{
    uint64_t g = ((uint64_t)(T - t) << 32) / (uint64_t)T;
    uint64_t span = ((uint64_t)(maxd - mind) * cube_frac(g)) >> 32;
    return mind + (int64_t)(((uint64_t)u * (span + 1)) >> 32);
}

/* Draw-site tags of the counter-based generator (counter word 3, high byte). */
enum { TAG_MAXMIN = 1, TAG_POSMIN = 2, TAG_RANDMIN = 3, TAG_GA = 4, TAG_POOL = 5 };

/* Byte k%16 of the draw for bit group k/16 (R9). */
static uint32_t randmin_byte(uint64_t seed, uint32_t inst, uint32_t ph, int64_t t, int32_t k)
{
    uint32_t r[4];
    draw4(seed, (uint32_t)t, inst, ph, ((uint32_t)TAG_RANDMIN << 24) | (uint32_t)(k / 16), r);
    int b = k % 16;
    return (r[b / 4] >> (8 * (b % 4))) & 0xFFu;
}

/* r-th member (0-based, increasing index) of the set marked in mask[]. */
static int32_t nth_marked(const uint8_t *mask, int32_t n, int64_t r)
{
    for (int32_t k = 0; k < n; k++)
        if (mask[k]) {
            if (r == 0) return k;
            r--;
        }
    return -1;
}

/* Greedy (Section III-A.1): flip argmin Delta while some Delta < 0.
 * R13: the test comes before the flip, so Greedy never goes uphill.
 * A cap bounds the phase (never reached when cap exceeds the descent). */
static int64_t phase_greedy(state_t *st, int64_t cap)
{
    int64_t f = 0;
    while (f < cap) {
        int32_t j = argmin_all(st);
        if (st->delta[j] >= 0) break;
        flip(st, j);
        f++;
    }
    return f;
}

/* Straight (Section III-A.2): argmin Delta over the bits where X and D differ,
 * until X = D. */
static int64_t phase_straight(state_t *st, const uint8_t *target)
{
    int64_t f = 0;
    for (;;) {
        int32_t j = -1;
        for (int32_t k = 0; k < st->n; k++)
            if (st->x[k] != target[k] && (j < 0 || st->delta[k] < st->delta[j])) j = k;
        if (j < 0) break;
        flip(st, j);
        f++;
    }
    return f;
}

/* Tabu greedy (R12): T iterations, each flips the non-tabu argmin Delta even
 * when it is positive; all-tabu falls back to all bits. */
static int64_t phase_tabu_greedy(state_t *st, int64_t T, int32_t tau)
{
    tabu_t tb; tabu_init(&tb, st->n, tau);
    for (int64_t t = 1; t <= T; t++) {
        int32_t j = -1;
        for (int32_t k = 0; k < st->n; k++)
            if (!is_tabu(&tb, k, t) && (j < 0 || st->delta[k] < st->delta[j])) j = k;
        if (j < 0) j = argmin_all(st);
        flip(st, j);
        tb.last[j] = t;
    }
    tabu_free(&tb);
    return T;
}

/* Non-tabu domain mask; all bits when every bit is tabu (R11). */
static void nontabu_mask(const state_t *st, const tabu_t *tb, int64_t t, uint8_t *mask)
{
    int any = 0;
    for (int32_t k = 0; k < st->n; k++) {
        mask[k] = !is_tabu(tb, k, t);
        any |= mask[k];
    }
    if (!any) memset(mask, 1, (size_t)st->n);
}

/* MaxMin (Section III-A.3) with R6/R7. */
static int64_t phase_maxmin(state_t *st, int64_t T, int32_t tau, uint32_t ph)
{
    const int32_t n = st->n;
    uint8_t *dom = (uint8_t *)malloc((size_t)n), *cand = (uint8_t *)malloc((size_t)n);
    tabu_t tb; tabu_init(&tb, n, tau);
    for (int64_t t = 1; t <= T; t++) {
        nontabu_mask(st, &tb, t, dom);
        int64_t mind = INT64_MAX, maxd = INT64_MIN;
        for (int32_t k = 0; k < n; k++)
            if (dom[k]) {
                if (st->delta[k] < mind) mind = st->delta[k];
                if (st->delta[k] > maxd) maxd = st->delta[k];
            }
        /* R18: iterations 2c+1 and 2c+2 use words (0, 1) and (2, 3) of draw c */
        uint32_t r[4];
        const int64_t half = (t - 1) % 2;
        draw4(st->seed, (uint32_t)((t - 1) / 2), st->inst, ph, (uint32_t)TAG_MAXMIN << 24, r);
        const uint32_t u = r[2 * half], v = r[2 * half + 1];
        int64_t d = maxmin_threshold(t, T, mind, maxd, u);
        int64_t c = 0;
        for (int32_t k = 0; k < n; k++) {
            cand[k] = dom[k] && st->delta[k] <= d;
            c += cand[k];
        }
        int32_t j = nth_marked(cand, n, (int64_t)scale_u32(v, (uint32_t)c));
        flip(st, j);
        tb.last[j] = t;
    }
    tabu_free(&tb); free(dom); free(cand);
    return T;
}

/* CyclicMin (Section III-A.4) with R5/R8: window of width w(t) starting at
 * pos_t, pos_1 = 0, pos_{t+1} = pos_t + w(t) mod n. */
static int64_t phase_cyclicmin(state_t *st, int64_t T, int32_t tau)
{
    const int32_t n = st->n;
    tabu_t tb; tabu_init(&tb, n, tau);
    int64_t pos = 0;
    for (int64_t t = 1; t <= T; t++) {
        int64_t w = cyclic_width(t, T, n);
        int32_t j = -1, jt = -1;   /* j: non-tabu window argmin; jt: window argmin */
        for (int32_t k = 0; k < n; k++) {
            int64_t off = ((int64_t)k - pos + n) % n;
            if (off >= w) continue;
            if (jt < 0 || st->delta[k] < st->delta[jt]) jt = k;
            if (!is_tabu(&tb, k, t) && (j < 0 || st->delta[k] < st->delta[j])) j = k;
        }
        if (j < 0) j = jt;
        flip(st, j);
        tb.last[j] = t;
        pos = (pos + w) % n;
    }
    tabu_free(&tb);
    return T;
}

/* RandomMin (Section III-A.5) with R9: bit k is a candidate when its random
 * byte is below q(t); the non-tabu candidate argmin is flipped; with no
 * non-tabu candidate the non-tabu argmin (or the plain argmin when all bits
 * are tabu) is flipped. */
static int64_t phase_randommin(state_t *st, int64_t T, int32_t tau, uint32_t ph)
{
    const int32_t n = st->n;
    uint8_t *dom = (uint8_t *)malloc((size_t)n);
    tabu_t tb; tabu_init(&tb, n, tau);
    for (int64_t t = 1; t <= T; t++) {
        int32_t q = randmin_q(t, T, n);
        nontabu_mask(st, &tb, t, dom);
        int32_t j = -1, jd = -1;
        for (int32_t k = 0; k < n; k++) {
            if (!dom[k]) continue;
            if (jd < 0 || st->delta[k] < st->delta[jd]) jd = k;
            if ((int32_t)randmin_byte(st->seed, st->inst, ph, t, k) < q &&
                (j < 0 || st->delta[k] < st->delta[j])) j = k;
        }
        if (j < 0) j = jd;
        flip(st, j);
        tb.last[j] = t;
    }
    tabu_free(&tb); free(dom);
    return T;
}

/* PositiveMin (Section III-A.6) with R6/R10. */
static int64_t phase_positivemin(state_t *st, int64_t T, int32_t tau, uint32_t ph)
{
    const int32_t n = st->n;
    uint8_t *dom = (uint8_t *)malloc((size_t)n), *cand = (uint8_t *)malloc((size_t)n);
    tabu_t tb; tabu_init(&tb, n, tau);
    for (int64_t t = 1; t <= T; t++) {
        nontabu_mask(st, &tb, t, dom);
        int64_t posmin = INT64_MAX;
        for (int32_t k = 0; k < n; k++)
            if (dom[k] && st->delta[k] > 0 && st->delta[k] < posmin) posmin = st->delta[k];
        int64_t c = 0;
        for (int32_t k = 0; k < n; k++) {
            cand[k] = dom[k] && (posmin == INT64_MAX || st->delta[k] <= posmin);
            c += cand[k];
        }
        /* R18: iterations 4c+1 .. 4c+4 use words 0 .. 3 of draw c */
        uint32_t r[4];
        draw4(st->seed, (uint32_t)((t - 1) / 4), st->inst, ph, (uint32_t)TAG_POSMIN << 24, r);
        int32_t j = nth_marked(cand, n, (int64_t)scale_u32(r[(t - 1) % 4], (uint32_t)c));
        flip(st, j);
        tb.last[j] = t;
    }
    tabu_free(&tb); free(dom); free(cand);
    return T;
}

/* TwoNeighbor (Section III-A.7): flips 0, 1, 0, 2, 1, 3, 2, ... (2n-1 flips),
 * so every 1-bit neighbour of the start is visited and Step 1 covers every
 * 2-bit neighbour. */
static int64_t phase_twoneighbor(state_t *st)
{
    int64_t f = 0;
    flip(st, 0); f++;
    for (int32_t k = 1; k < st->n; k++) {
        flip(st, k);
        flip(st, k - 1);
        f += 2;
    }
    return f;
}

static int64_t run_phase(state_t *st, int32_t rule, int64_t T, int32_t tau, uint32_t ph,
                         const uint8_t *target, int64_t greedy_cap)
{
    switch (rule) {
    case ORC_GREEDY:      return phase_greedy(st, greedy_cap);
    case ORC_STRAIGHT:    return phase_straight(st, target);
    case ORC_MAXMIN:      return phase_maxmin(st, T, tau, ph);
    case ORC_CYCLICMIN:   return phase_cyclicmin(st, T, tau);
    case ORC_RANDOMMIN:   return phase_randommin(st, T, tau, ph);
    case ORC_POSITIVEMIN: return phase_positivemin(st, T, tau, ph);
    case ORC_TWONEIGHBOR: return phase_twoneighbor(st);
    case ORC_TABU_GREEDY: return phase_tabu_greedy(st, T, tau);
    default:              return -1;
    }
}

/* One search call: start at x, run one phase of `rule`, report BEST, the final
 * state and (optionally) the flip trace.  Returns the flip count, or a
 * negative code (-1 bad rule, -2 verification mismatch). */
int64_t orc_search(const int32_t *W, int32_t n, int32_t rule, int64_t T, int32_t tau,
                   uint64_t seed, uint32_t inst, uint32_t ph, int64_t greedy_cap,
                   uint8_t *x, const uint8_t *target, uint8_t *best, int64_t *ebest,
                   int64_t *e, int64_t *delta, int32_t *trace, int64_t trace_cap, int32_t verify)
{
    state_t st;
    state_load(&st, W, n, x, delta, best);
    st.trace = trace; st.trace_cap = trace_cap; st.verify = verify;
    st.seed = seed; st.inst = inst;
    step1(&st);
    int64_t f = run_phase(&st, rule, T, tau, ph, target, greedy_cap);
    *ebest = st.ebest;
    *e = st.E;
    if (f < 0) return -1;
    if (st.error) return -2;
    return f;
}

/* Batch search (Section III-B) with R14/R15: Straight to the target, Greedy,
 * then {main(T flips), Greedy} while the flips of this batch search are below
 * Bn; TwoNeighbor runs once.  ph is the instance's main-phase counter (it
 * keys the generator) and is advanced by one per main phase. */
typedef struct {
    int64_t flips;
    int32_t mains;
} batch_out_t;

static batch_out_t batch_search(state_t *st, const uint8_t *target, int32_t rule, int64_t T,
                                int64_t Bn, int32_t tau, uint32_t *ph, int64_t greedy_cap,
                                int64_t *phase_flips, int32_t phase_cap, int32_t *nphases)
{
    batch_out_t o = {0, 0};
    int32_t np = 0;
    /* R4: BEST restarts at the current vector for every batch search. */
    memcpy(st->best, st->x, (size_t)st->n);
    st->ebest = st->E;
    step1(st);
    int64_t f;
    f = phase_straight(st, target); o.flips += f;
    if (phase_flips && np < phase_cap) phase_flips[np] = f;
    np++;
    f = phase_greedy(st, greedy_cap); o.flips += f;
    if (phase_flips && np < phase_cap) phase_flips[np] = f;
    np++;
    while (o.flips < Bn) {
        f = run_phase(st, rule, T, tau, *ph, NULL, greedy_cap);
        (*ph)++;
        o.mains++;
        o.flips += f;
        if (phase_flips && np < phase_cap) phase_flips[np] = f;
        np++;
        f = phase_greedy(st, greedy_cap); o.flips += f;
        if (phase_flips && np < phase_cap) phase_flips[np] = f;
        np++;
        if (rule == ORC_TWONEIGHBOR) break;
    }
    if (nphases) *nphases = np;
    return o;
}

int64_t orc_batch_search(const int32_t *W, int32_t n, int32_t rule, int64_t T, int64_t Bn,
                         int32_t tau, uint64_t seed, uint32_t inst, uint32_t *ph, int64_t greedy_cap,
                         uint8_t *x, const uint8_t *target, uint8_t *best, int64_t *ebest,
                         int64_t *e, int64_t *delta, int32_t *trace, int64_t trace_cap,
                         int64_t *phase_flips, int32_t phase_cap, int32_t *nphases, int32_t verify)
{
    if (rule < ORC_MAXMIN || rule > ORC_TABU_GREEDY) return -1;
    if (rule != ORC_TWONEIGHBOR && T < 1) return -1;
    state_t st;
    state_load(&st, W, n, x, delta, best);
    st.trace = trace; st.trace_cap = trace_cap; st.verify = verify;
    st.seed = seed; st.inst = inst;
    batch_out_t o = batch_search(&st, target, rule, T, Bn, tau, ph, greedy_cap,
                                 phase_flips, phase_cap, nphases);
    *ebest = st.ebest;
    *e = st.E;
    if (st.error) return -2;
    return o.flips;
}

/* ------------------------------------------------------------------------ */
/* Genetic algorithm on solution pools (Section IV) in generational mode    */
/* (R16): every instance of round r draws its target from the pools as they  */
/* stood at the start of round r; packets are inserted in instance order.   */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t n, cap, npools;
    uint8_t *bits;     /* [npools][cap][n] */
    int64_t *e;        /* [npools][cap] */
    int32_t *algo;     /* [npools][cap] */
    int32_t *op;       /* [npools][cap] */
} pools_t;

static uint8_t *entry_bits(const pools_t *p, int32_t q, int32_t r)
{
    return p->bits + ((int64_t)q * p->cap + r) * p->n;
}

/* Bit k of a random vector whose 128-bit chunks come from draw (a, b, k/128, tag). */
static int rand_vec_bit(uint64_t seed, uint32_t a, uint32_t b, uint32_t tag, int32_t k)
{
    uint32_t r[4];
    draw4(seed, a, b, (uint32_t)(k / 128), tag, r);
    int m = k % 128;
    return (int)((r[m / 32] >> (m % 32)) & 1u);
}

/* Section IV-A: initial pools hold random vectors with energy +inf and random
 * algorithm / operation columns (R17).  Epoch e > 0 is the refill after the
 * e-th restart (Section IV-B, R24): its own draws, sub-tags 2e and 2e + 1. */
static void pools_init(pools_t *p, const orc_ga_params *g, uint32_t epoch)
{
    for (int32_t q = 0; q < p->npools; q++)
        for (int32_t r = 0; r < p->cap; r++) {
            uint8_t *b = entry_bits(p, q, r);
            for (int32_t k = 0; k < p->n; k++)
                b[k] = (uint8_t)rand_vec_bit(g->seed, (uint32_t)r, (uint32_t)q,
                                             ((uint32_t)TAG_POOL << 24) | (2u * epoch + 1u), k);
            uint32_t w[4];
            draw4(g->seed, (uint32_t)r, (uint32_t)q, 0, ((uint32_t)TAG_POOL << 24) | (2u * epoch), w);
            p->e[(int64_t)q * p->cap + r] = INT64_MAX;
            p->algo[(int64_t)q * p->cap + r] = g->algos[scale_u32(w[0], (uint32_t)g->n_algos)];
            p->op[(int64_t)q * p->cap + r] = g->ops[scale_u32(w[1], (uint32_t)g->n_ops)];
        }
}

/* Section IV-A: the (floor(r^3 m) + 1)-th solution, r uniform in [0,1),
 * in 32.32 fixed point (R17); returns the 0-based rank. */
uint32_t orc_rank_index(uint32_t u, uint32_t m)
{
    return scale_u32((uint32_t)cube_frac(u), m);
}

enum { KIND_CHOICE = 0, KIND_BITS = 2, KIND_MASK = 3, KIND_RANDVEC = 4 };

/* Per-bit uniform u32 for threshold decisions of the genetic operations. */
static uint32_t ga_bit_u32(uint64_t seed, uint32_t round, uint32_t inst, int32_t k)
{
    uint32_t r[4];
    draw4(seed, round, inst, (uint32_t)(k / 4), ((uint32_t)TAG_GA << 24) | KIND_BITS, r);
    return r[k % 4];
}

/* The learned operations (R22; not in the paper) on parent a with logits z
 * (one float32 per bit, the network's scores of that pooled vector):
 *   MLP-seed flips every bit whose logit is positive;
 *   MLP-mutate flips bit k when its per-bit u32 draw is below 2^29 + q_k 2^22,
 *   q_k = clamp(round-half-even(16 z_k), -128, 127): the Mutation rate 1/8
 *   tilted by the logit. */
static void mlp_operation(int32_t op, const uint8_t *a, const float *z, int32_t n, uint64_t seed,
                          uint32_t round, uint32_t inst, uint8_t *target)
{
    for (int32_t k = 0; k < n; k++) {
        int flip;
        if (op == ORC_OP_MLP_SEED) {
            flip = z[k] > 0.0f;
        } else {
            float lv = nearbyintf(16.0f * z[k]);      /* default rounding: half to even */
            if (lv < -128.0f) lv = -128.0f;
            if (lv > 127.0f) lv = 127.0f;
            int64_t thr = ((int64_t)1 << 29) + (int64_t)lv * ((int64_t)1 << 22);
            flip = (int64_t)ga_bit_u32(seed, round, inst, k) < thr;
        }
        target[k] = a[k] ^ (uint8_t)flip;
    }
}

/* Target generation for one instance (Section IV-A, IV-B; R17).  logits
 * (nullable, [npools][cap][n]) are the learned scores of every pooled bit;
 * without them the learned operations copy their parent. */
static void ga_target(const pools_t *p, const orc_ga_params *g, uint32_t round, uint32_t inst,
                      uint8_t *target, int32_t *algo_out, int32_t *op_out, const float *logits)
{
    const int32_t n = p->n, m = p->cap;
    const int32_t q = (int32_t)(inst % (uint32_t)p->npools);
    uint32_t c[4], v[4];
    draw4(g->seed, round, inst, 0, ((uint32_t)TAG_GA << 24) | KIND_CHOICE, c);
    draw4(g->seed, round, inst, 1, ((uint32_t)TAG_GA << 24) | KIND_CHOICE, v);
    /* Adaptive choice: with probability p_explore uniformly, else the column
     * of a uniformly chosen pool row. */
    int32_t op, algo;
    if (c[0] < g->p_explore) op = g->ops[scale_u32(c[1], (uint32_t)g->n_ops)];
    else op = p->op[(int64_t)q * m + scale_u32(c[1], (uint32_t)m)];
    if (c[2] < g->p_explore) algo = g->algos[scale_u32(c[3], (uint32_t)g->n_algos)];
    else algo = p->algo[(int64_t)q * m + scale_u32(c[3], (uint32_t)m)];
    *op_out = op;
    *algo_out = algo;

    const int32_t ra = (int32_t)orc_rank_index(v[0], (uint32_t)m);
    const uint8_t *a = entry_bits(p, q, ra);
    const int32_t qn = (q + 1) % p->npools;
    const uint8_t *b = entry_bits(p, op == ORC_OP_XROSSOVER ? qn : q,
                                  (int32_t)orc_rank_index(v[1], (uint32_t)m));
    switch (op) {
    case ORC_OP_RANDOM:
        for (int32_t k = 0; k < n; k++)
            target[k] = (uint8_t)rand_vec_bit(g->seed, round, inst,
                                              ((uint32_t)TAG_GA << 24) | KIND_RANDVEC, k);
        break;
    case ORC_OP_BEST:
        memcpy(target, entry_bits(p, q, 0), (size_t)n);
        break;
    case ORC_OP_MUTATION:
        for (int32_t k = 0; k < n; k++)
            target[k] = a[k] ^ (uint8_t)(ga_bit_u32(g->seed, round, inst, k) < g->p_mutation);
        break;
    case ORC_OP_CROSSOVER:
    case ORC_OP_XROSSOVER:
        if (g->crossover_kind == 1) {
            /* two-point: bits [lo, hi) from the second parent */
            uint32_t x1 = scale_u32(v[2], (uint32_t)n + 1), x2 = scale_u32(v[3], (uint32_t)n + 1);
            uint32_t lo = x1 < x2 ? x1 : x2, hi = x1 < x2 ? x2 : x1;
            for (int32_t k = 0; k < n; k++)
                target[k] = ((uint32_t)k >= lo && (uint32_t)k < hi) ? b[k] : a[k];
        } else {
            /* uniform: each bit from the second parent when its mask bit is 1 */
            for (int32_t k = 0; k < n; k++)
                target[k] = rand_vec_bit(g->seed, round, inst, ((uint32_t)TAG_GA << 24) | KIND_MASK, k)
                                ? b[k] : a[k];
        }
        break;
    case ORC_OP_ZERO:
        for (int32_t k = 0; k < n; k++)
            target[k] = (ga_bit_u32(g->seed, round, inst, k) < g->p_zero) ? 0 : a[k];
        break;
    case ORC_OP_ONE:
        for (int32_t k = 0; k < n; k++)
            target[k] = (ga_bit_u32(g->seed, round, inst, k) < g->p_one) ? 1 : a[k];
        break;
    case ORC_OP_INTERVALZERO: {
        /* segment length uniform in [min(32,n), max(min(32,n), n/2)], cyclic start */
        uint32_t lo = (uint32_t)(n < 32 ? n : 32);
        uint32_t hi = (uint32_t)(n / 2) > lo ? (uint32_t)(n / 2) : lo;
        uint32_t len = lo + scale_u32(v[2], hi - lo + 1);
        uint32_t s = scale_u32(v[3], (uint32_t)n);
        memcpy(target, a, (size_t)n);
        for (uint32_t o = 0; o < len; o++) target[(s + o) % (uint32_t)n] = 0;
        break;
    }
    case ORC_OP_MLP_SEED:
    case ORC_OP_MLP_MUTATE:
        if (logits)
            mlp_operation(op, a, logits + ((int64_t)q * m + ra) * n, n, g->seed, round, inst, target);
        else
            memcpy(target, a, (size_t)n);
        break;
    default:
        memcpy(target, a, (size_t)n);
        break;
    }
}

/* Section III-C / IV: insert when strictly better than the worst entry and no
 * identical vector is pooled; ascending energy, newcomer after equal energies
 * (R17).  Returns the insert position or -1. */
static int32_t pool_insert(pools_t *p, int32_t q, const uint8_t *bits, int64_t e, int32_t algo, int32_t op)
{
    const int32_t m = p->cap, n = p->n;
    int64_t *pe = p->e + (int64_t)q * m;
    if (!(e < pe[m - 1])) return -1;
    for (int32_t r = 0; r < m; r++)
        if (memcmp(entry_bits(p, q, r), bits, (size_t)n) == 0) return -1;
    int32_t pos = 0;
    while (pos < m && pe[pos] <= e) pos++;
    for (int32_t r = m - 1; r > pos; r--) {
        memcpy(entry_bits(p, q, r), entry_bits(p, q, r - 1), (size_t)n);
        pe[r] = pe[r - 1];
        p->algo[(int64_t)q * m + r] = p->algo[(int64_t)q * m + r - 1];
        p->op[(int64_t)q * m + r] = p->op[(int64_t)q * m + r - 1];
    }
    memcpy(entry_bits(p, q, pos), bits, (size_t)n);
    pe[pos] = e;
    p->algo[(int64_t)q * m + pos] = algo;
    p->op[(int64_t)q * m + pos] = op;
    return pos;
}

/* Restart on merge (Section IV-B, R24): the pools have merged when every
 * entry has been evaluated and lies within Hamming distance h of the best
 * pooled vector (the rank-0 entry of lowest energy, lowest pool on ties). */
static int pools_merged(const pools_t *p, int32_t h)
{
    int32_t qb = 0;
    for (int32_t q = 1; q < p->npools; q++)
        if (p->e[(int64_t)q * p->cap] < p->e[(int64_t)qb * p->cap]) qb = q;
    const uint8_t *best = entry_bits(p, qb, 0);
    for (int32_t q = 0; q < p->npools; q++)
        for (int32_t r = 0; r < p->cap; r++) {
            if (p->e[(int64_t)q * p->cap + r] == INT64_MAX) return 0;
            const uint8_t *b = entry_bits(p, q, r);
            int32_t d = 0;
            for (int32_t k = 0; k < p->n; k++) d += b[k] != best[k];
            if (d > h) return 0;
        }
    return 1;
}

/* Generational DABS loop on one problem.  Instances start at X = 0 (Section
 * III-B) and keep X across rounds.  Outputs the pools and per-instance final
 * X, E and main-phase counters; inserts[] (optional, [rounds][instances])
 * records each packet's insert position (-1 if rejected); targets_out
 * (optional, [instances][n]) the last round's targets; packets_out (optional,
 * [instances]) the last round's packet energies.
 *
 * score (nullable) is called at the start of every round with the pools as
 * they stand and fills logits[npools][cap][n], the learned scores the
 * MLP-seed / MLP-mutate operations use (R22).  With ORC_GA_RESTART set in
 * g->flags the pools restart when merged (R24); best_bits / best_e (nullable)
 * receive the best pooled vector seen over all rounds and epochs and
 * restarts_out the number of restarts; round_best (nullable, [rounds]) the
 * record's energy after each round; stats (nullable, [ORC_STATS]) how often
 * each genetic operation and main algorithm was chosen and how often its
 * packet entered a pool, and the operation / algorithm columns of the
 * record's entry when it was last improved (the bookkeeping behind Section
 * VI-D's tables).  Returns total flips or a negative
 * code. */
int64_t orc_solve_ex(const int32_t *W, int32_t n, const orc_ga_params *g, int32_t instances,
                     int32_t rounds, uint8_t *pool_bits, int64_t *pool_e, int32_t *pool_algo,
                     int32_t *pool_op, uint8_t *x_out, int64_t *e_out, uint32_t *ph_out,
                     int32_t *inserts, uint8_t *targets_out, int64_t *packets_out, int32_t verify,
                     orc_score_fn score, void *score_ctx, uint8_t *best_bits, int64_t *best_e,
                     int32_t *restarts_out, int64_t *round_best, int64_t *stats)
{
    if (stats) {
        memset(stats, 0, sizeof(int64_t) * ORC_STATS);
        stats[ORC_STAT_REC_OP] = stats[ORC_STAT_REC_ALGO] = -1;
    }
    if (n < 1 || instances < 1 || g->npools < 1 || g->capacity < 1) return -1;
    if (g->n_algos < 1 || g->n_ops < 1) return -1;
    pools_t p = {n, g->capacity, g->npools, pool_bits, pool_e, pool_algo, pool_op};
    uint32_t epoch = 0;
    pools_init(&p, g, epoch);
    uint8_t *x = (uint8_t *)calloc((size_t)instances * n, 1);
    uint8_t *tg = (uint8_t *)malloc((size_t)instances * n);
    uint8_t *bb = (uint8_t *)malloc((size_t)instances * n);
    int64_t *eb = (int64_t *)malloc(sizeof(int64_t) * (size_t)instances);
    int32_t *al = (int32_t *)malloc(sizeof(int32_t) * (size_t)instances);
    int32_t *op = (int32_t *)malloc(sizeof(int32_t) * (size_t)instances);
    uint32_t *ph = (uint32_t *)calloc((size_t)instances, sizeof(uint32_t));
    int64_t *delta = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    float *logits = score ? (float *)malloc(sizeof(float) * (size_t)g->npools * g->capacity * n) : NULL;
    uint8_t *record = (uint8_t *)malloc((size_t)n);
    int64_t record_e = INT64_MAX;
    memset(record, 0, (size_t)n);
    int64_t total = 0;
    int err = 0;
    for (int32_t r = 0; r < rounds && !err; r++) {
        if (score) score(score_ctx, r, p.bits, logits);
        for (int32_t i = 0; i < instances; i++)
            ga_target(&p, g, (uint32_t)r, (uint32_t)i, tg + (int64_t)i * n, &al[i], &op[i], logits);
        for (int32_t i = 0; i < instances; i++) {
            state_t st;
            state_load(&st, W, n, x + (int64_t)i * n, delta, bb + (int64_t)i * n);
            st.verify = verify; st.seed = g->seed; st.inst = (uint32_t)i;
            batch_out_t o = batch_search(&st, tg + (int64_t)i * n, al[i], g->T, g->Bn, g->tau,
                                         &ph[i], g->greedy_cap, NULL, 0, NULL);
            total += o.flips;
            eb[i] = st.ebest;
            if (e_out) e_out[i] = st.E;
            if (st.error) err = 1;
        }
        for (int32_t i = 0; i < instances; i++) {
            int32_t pos = pool_insert(&p, (int32_t)(i % g->npools), bb + (int64_t)i * n, eb[i], al[i], op[i]);
            if (inserts) inserts[(int64_t)r * instances + i] = pos;
            if (stats) {
                stats[ORC_STAT_USE_OP + op[i]]++;
                stats[ORC_STAT_USE_ALGO + al[i]]++;
                if (pos >= 0) {
                    stats[ORC_STAT_INS_OP + op[i]]++;
                    stats[ORC_STAT_INS_ALGO + al[i]]++;
                }
            }
        }
        if (packets_out) memcpy(packets_out, eb, sizeof(int64_t) * (size_t)instances);
        /* the run's best pooled vector so far (kept across restarts) */
        for (int32_t q = 0; q < g->npools; q++)
            if (p.e[(int64_t)q * p.cap] < record_e) {
                record_e = p.e[(int64_t)q * p.cap];
                memcpy(record, entry_bits(&p, q, 0), (size_t)n);
                if (stats) {
                    stats[ORC_STAT_REC_OP] = p.op[(int64_t)q * p.cap];
                    stats[ORC_STAT_REC_ALGO] = p.algo[(int64_t)q * p.cap];
                }
            }
        if (round_best) round_best[r] = record_e;
        if ((g->flags & ORC_GA_RESTART) && pools_merged(&p, g->merge_hamming)) {
            epoch++;
            pools_init(&p, g, epoch);
        }
    }
    if (x_out) memcpy(x_out, x, (size_t)instances * n);
    if (targets_out) memcpy(targets_out, tg, (size_t)instances * n);
    if (ph_out) memcpy(ph_out, ph, sizeof(uint32_t) * (size_t)instances);
    if (best_bits) memcpy(best_bits, record, (size_t)n);
    if (best_e) *best_e = record_e;
    if (restarts_out) *restarts_out = (int32_t)epoch;
    free(x); free(tg); free(bb); free(eb); free(al); free(op); free(ph); free(delta); free(logits);
    free(record);
    return err ? -2 : total;
}

int64_t orc_solve(const int32_t *W, int32_t n, const orc_ga_params *g, int32_t instances,
                  int32_t rounds, uint8_t *pool_bits, int64_t *pool_e, int32_t *pool_algo,
                  int32_t *pool_op, uint8_t *x_out, int64_t *e_out, uint32_t *ph_out,
                  int32_t *inserts, uint8_t *targets_out, int64_t *packets_out, int32_t verify)
{
    return orc_solve_ex(W, n, g, instances, rounds, pool_bits, pool_e, pool_algo, pool_op, x_out,
                        e_out, ph_out, inserts, targets_out, packets_out, verify, NULL, NULL, NULL,
                        NULL, NULL, NULL, NULL);
}

/* One target drawn by ga_target from pools the caller supplies (bits
 * [npools][cap][n], energies, columns; logits nullable as in orc_solve_ex),
 * for pinning the genetic operations on chosen parents. */
void orc_target_from_pools(int32_t n, const orc_ga_params *g, uint8_t *pool_bits, int64_t *pool_e,
                           int32_t *pool_algo, int32_t *pool_op, const float *logits, uint32_t round,
                           uint32_t inst, uint8_t *target, int32_t *algo, int32_t *op)
{
    pools_t p = {n, g->capacity, g->npools, pool_bits, pool_e, pool_algo, pool_op};
    ga_target(&p, g, round, inst, target, algo, op, logits);
}

/* One round-0 target as orc_solve would draw it from freshly initialised
 * pools (for sampled checks at sizes where the full loop is too slow). */
int32_t orc_first_target(int32_t n, const orc_ga_params *g, uint32_t inst, uint8_t *target,
                         int32_t *algo, int32_t *op)
{
    int64_t cells = (int64_t)g->npools * g->capacity;
    pools_t p = {n, g->capacity, g->npools,
                 (uint8_t *)malloc((size_t)(cells * n)), (int64_t *)malloc(sizeof(int64_t) * (size_t)cells),
                 (int32_t *)malloc(sizeof(int32_t) * (size_t)cells), (int32_t *)malloc(sizeof(int32_t) * (size_t)cells)};
    pools_init(&p, g, 0);
    ga_target(&p, g, 0, inst, target, algo, op, NULL);
    free(p.bits); free(p.e); free(p.algo); free(p.op);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Exhaustive minimum for small n                                           */
/* ------------------------------------------------------------------------ */

/* Every vector's energy from scratch (definition), for pinning the Gray-code
 * enumeration below on small n.  Writes 2^n energies, vector index v has bit
 * k = (v >> k) & 1. */
void orc_all_energies(const int32_t *W, int32_t n, int64_t *out)
{
    uint8_t x[64];
    for (int64_t v = 0; v < ((int64_t)1 << n); v++) {
        for (int32_t k = 0; k < n; k++) x[k] = (uint8_t)((v >> k) & 1);
        out[v] = orc_energy(W, n, x);
    }
}

/* Minimum over all 2^n vectors by a reflected Gray code walk: step s flips
 * the bit at the position of the lowest set bit of s, the energy follows by
 * E += Delta (Section III-A bookkeeping).  Returns the minimum energy and the
 * lowest-index minimiser in Gray order. */
int64_t orc_bruteforce(const int32_t *W, int32_t n, uint8_t *argmin)
{
    uint8_t x[64] = {0};
    int64_t delta[64];
    for (int32_t k = 0; k < n; k++) delta[k] = W[(int64_t)k * n + k];
    int64_t e = 0, best = 0;
    memset(argmin, 0, (size_t)n);
    for (uint64_t s = 1; s < ((uint64_t)1 << n); s++) {
        int32_t i = __builtin_ctzll(s);
        const int64_t si = x[i] ? 1 : -1;
        for (int32_t k = 0; k < n; k++)
            if (k != i) delta[k] += 2 * (int64_t)W[(int64_t)i * n + k] * si * (x[k] ? 1 : -1);
        e += delta[i];
        delta[i] = -delta[i];
        x[i] ^= 1;
        if (e < best) {
            best = e;
            memcpy(argmin, x, (size_t)n);
        }
    }
    return best;
}
