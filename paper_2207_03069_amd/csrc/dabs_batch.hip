// dabs_batch.hip -- the genetic algorithm of Section IV on device-resident
// solution pools, for one problem (dabs_solver_*) or many problems of uneven
// size in one batch (dabs_batched_*).  A round is: target generation for
// every instance (adaptive operation / algorithm choice, rank selection,
// genetic operation), one batch search per instance (one wavefront each, one
// launch per slot class, on parallel streams), packet insertion into
// the pools in instance order, round counter increment.  A batch can capture
// its round once into a HIP graph and replay it.
#include <algorithm>
#include <string.h>
#include <vector>

#include "dabs_device.h"
#include "dabs_internal.h"

using namespace dabs;

#define HIP_OK(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return dabs_fail(DABS_E_HIP, "%s: %s", #call, hipGetErrorString(e_));      \
    } while (0)

namespace dabs {

enum { KIND_CHOICE = 0, KIND_BITS = 2, KIND_MASK = 3, KIND_RANDVEC = 4 };
constexpr int POOL_MAX = 1024;
constexpr int MAX_CLASSES = 8;

__device__ __forceinline__ uint64_t tail_mask(int n, int w) {
    const int rem = n - 64 * w;
    return rem >= 64 ? ~0ull : (rem <= 0 ? 0ull : ((1ull << rem) - 1));
}

// 64 bits of a random vector: word w is half of the 128-bit chunk w/2 of the
// draw (a, b, chunk, tag).
__device__ __forceinline__ uint64_t rand_word(uint64_t seed, uint32_t a, uint32_t b, uint32_t tag, int w) {
    const R4 r = philox(a, b, (uint32_t)(w >> 1), tag, seed);
    return (w & 1) ? ((uint64_t)r.w[3] << 32 | r.w[2]) : ((uint64_t)r.w[1] << 32 | r.w[0]);
}

// Bits of word w whose per-bit u32 draw is below p (one draw per bit).
__device__ __forceinline__ uint64_t thresh_word(uint64_t seed, uint32_t round, uint32_t inst, int w, uint32_t p) {
    uint64_t m = 0;
    for (int c = 0; c < 16; ++c) {
        const R4 r = philox(round, inst, (uint32_t)(w * 16 + c), ((uint32_t)TAG_GA << 24) | KIND_BITS, seed);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (r.w[q] < p) m |= 1ull << (c * 4 + q);
    }
    return m;
}

// bits [lo, hi) of word w
__device__ __forceinline__ uint64_t range_word(int lo, int hi, int w) {
    const int b0 = 64 * w;
    const int s = lo - b0 < 0 ? 0 : (lo - b0 > 64 ? 64 : lo - b0);
    const int e = hi - b0 < 0 ? 0 : (hi - b0 > 64 ? 64 : hi - b0);
    const uint64_t upto_e = e >= 64 ? ~0ull : ((1ull << e) - 1);
    const uint64_t upto_s = s >= 64 ? ~0ull : ((1ull << s) - 1);
    return upto_e & ~upto_s;
}

__device__ __forceinline__ uint32_t rank_index(uint32_t u, uint32_t m) { return scale32((uint32_t)cube_frac(u), m); }

// Section IV-A: pools start with random vectors, energy +inf and random
// algorithm / operation columns.  Fill number `epoch` (0 at creation, e after
// the e-th restart of merged pools, Section IV-B) draws the bits with Philox
// sub-tag 2 epoch + 1 and the columns with 2 epoch.  Threads t0, t0 + step,
// ... cover the (pool, entry, word) triples of one problem.
__device__ void fill_pools(const BatchDev &b, const ProbDesc &d, uint32_t epoch, int64_t t0, int64_t step) {
    const int P = d.g.npools, m = d.g.capacity, nw = d.nw;
    const int64_t total = (int64_t)P * m * nw;
    const uint32_t tag = (uint32_t)TAG_POOL << 24;
    for (int64_t t = t0; t < total; t += step) {
        const int w = (int)(t % nw);
        const int r = (int)((t / nw) % m);
        const int q = (int)(t / ((int64_t)nw * m));
        b.pool_bits[d.pool_word0 + t] =
            rand_word(d.g.seed, (uint32_t)r, (uint32_t)q, tag | (2u * epoch + 1u), w) & tail_mask(d.n, w);
        if (w == 0) {
            const R4 dr = philox((uint32_t)r, (uint32_t)q, 0, tag | (2u * epoch), d.g.seed);
            const int64_t cell = d.pool_cell0 + (int64_t)q * m + r;
            b.pool_e[cell] = E_INF;
            b.pool_algo[cell] = d.g.algos[scale32(dr.w[0], (uint32_t)d.g.n_algos)];
            b.pool_op[cell] = d.g.ops[scale32(dr.w[1], (uint32_t)d.g.n_ops)];
        }
    }
}

__global__ void k_pool_init(BatchDev b, int p) {
    fill_pools(b, b.desc[p], 0u, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
}

// The choices of instance inst in round rd (Section IV-A, IV-B): operation
// and main algorithm (uniform with probability p_explore, else the column of
// a uniform entry of its pool), parents by rank selection (the second from
// the next pool for Xrossover), and the words v of the operation's draws.
struct GaChoice {
    int op, algo, q, qb, ra, rb;
    R4 v;
};
__device__ __forceinline__ GaChoice ga_choice(const BatchDev &b, const ProbDesc &d, int inst, uint32_t rd) {
    const dabs_ga_params &g = d.g;
    const int m = g.capacity, P = g.npools;
    GaChoice h;
    h.q = inst % P;
    const R4 c = philox(rd, (uint32_t)inst, 0, ((uint32_t)TAG_GA << 24) | KIND_CHOICE, g.seed);
    h.v = philox(rd, (uint32_t)inst, 1, ((uint32_t)TAG_GA << 24) | KIND_CHOICE, g.seed);
    const int64_t cell = d.pool_cell0 + (int64_t)h.q * m;
    h.op = c.w[0] < g.p_explore ? g.ops[scale32(c.w[1], (uint32_t)g.n_ops)]
                                : b.pool_op[cell + scale32(c.w[1], (uint32_t)m)];
    h.algo = c.w[2] < g.p_explore ? g.algos[scale32(c.w[3], (uint32_t)g.n_algos)]
                                  : b.pool_algo[cell + scale32(c.w[3], (uint32_t)m)];
    h.qb = h.op == DABS_OP_XROSSOVER ? (h.q + 1) % P : h.q;
    h.ra = (int)rank_index(h.v.w[0], (uint32_t)m);
    h.rb = (int)rank_index(h.v.w[1], (uint32_t)m);
    return h;
}

// Before the pools are scored: flag the pool entries that this round's
// learned operations take as parents (one thread per global instance), so
// that only their features are computed.
__global__ __launch_bounds__(256) void k_ga_need(BatchDev b, int total) {
    const int gi = blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= total) return;
    const ProbDesc &d = b.desc[b.inst_prob[gi]];
    const GaChoice h = ga_choice(b, d, gi - d.inst0, (uint32_t)b.ctr[2]);
    if (h.op == DABS_OP_MLP_SEED || h.op == DABS_OP_MLP_MUTATE)
        b.need[d.pool_cell0 + (int64_t)h.q * d.g.capacity + h.ra] = 1;
}

// Target generation (Section IV-A, IV-B): one wave per global instance, lane
// w builds word w of the target (n <= 4096: at most 64 words).
__global__ __launch_bounds__(256) void k_ga_target(BatchDev b, int total) {
    const int gi = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (gi >= total) return;
    const int lane = (int)(threadIdx.x & 63);
    const int p = __builtin_amdgcn_readfirstlane(b.inst_prob[gi]);
    const ProbDesc &d = b.desc[p];
    const dabs_ga_params &g = d.g;
    const int inst = gi - d.inst0;
    const int m = g.capacity, n = d.n, nw = d.nw;
    const uint32_t rd = (uint32_t)b.ctr[2];
    const GaChoice h = ga_choice(b, d, inst, rd);
    const int op = h.op, algo = h.algo, q = h.q;
    const R4 v = h.v;
    const uint64_t *pool = b.pool_bits + d.pool_word0;
    const uint64_t *pa = pool + ((int64_t)q * m + h.ra) * nw;
    const uint64_t *pb = pool + ((int64_t)h.qb * m + h.rb) * nw;
    const uint64_t *p0 = pool + (int64_t)q * m * nw;
    uint64_t *out = b.target + d.inst_word0 + (int64_t)inst * nw;
    const uint32_t lo32 = (uint32_t)(n < 32 ? n : 32);
    const uint32_t hi32 = (uint32_t)(n / 2) > lo32 ? (uint32_t)(n / 2) : lo32;
    for (int w = lane; w < nw; w += WAVE) {
        const uint64_t A = pa[w];
        uint64_t t;
        switch (op) {
        case DABS_OP_RANDOM:
            t = rand_word(g.seed, rd, (uint32_t)inst, ((uint32_t)TAG_GA << 24) | KIND_RANDVEC, w);
            break;
        case DABS_OP_BEST:
            t = p0[w];
            break;
        case DABS_OP_MUTATION:
            t = A ^ thresh_word(g.seed, rd, (uint32_t)inst, w, g.p_mutation);
            break;
        case DABS_OP_CROSSOVER:
        case DABS_OP_XROSSOVER: {
            uint64_t sel;
            if (g.crossover_kind == 1) {
                const uint32_t x1 = scale32(v.w[2], (uint32_t)n + 1), x2 = scale32(v.w[3], (uint32_t)n + 1);
                sel = range_word((int)(x1 < x2 ? x1 : x2), (int)(x1 < x2 ? x2 : x1), w);
            } else {
                sel = rand_word(g.seed, rd, (uint32_t)inst, ((uint32_t)TAG_GA << 24) | KIND_MASK, w);
            }
            t = (A & ~sel) | (pb[w] & sel);
            break;
        }
        case DABS_OP_ZERO:
            t = A & ~thresh_word(g.seed, rd, (uint32_t)inst, w, g.p_zero);
            break;
        case DABS_OP_ONE:
            t = A | thresh_word(g.seed, rd, (uint32_t)inst, w, g.p_one);
            break;
        case DABS_OP_MLP_SEED:
        case DABS_OP_MLP_MUTATE:
            // learned operations on parent A, scored by A's logits
            t = b.pool_logits ? mlp_op_word(op, A, b.pool_logits + d.pool_bit0 + ((int64_t)q * m + h.ra) * n, n, w,
                                            g.seed, rd, (uint32_t)inst)
                              : A;
            break;
        case DABS_OP_INTERVALZERO: {
            // zero positions st .. st+len-1 (mod n)
            const uint32_t len = lo32 + scale32(v.w[2], hi32 - lo32 + 1);
            const int st = (int)scale32(v.w[3], (uint32_t)n);
            const int end = st + (int)len;
            uint64_t z = range_word(st, end < n ? end : n, w);
            if (end > n) z |= range_word(0, end - n, w);
            t = A & ~z;
            break;
        }
        default:
            t = A;
            break;
        }
        out[w] = t & tail_mask(n, w);
    }
    if (lane == 0) {
        b.algo[gi] = algo;
        b.op[gi] = op;
    }
}

// Cost rank of a search rule (measured per flip: MaxMin, PositiveMin,
// RandomMin, CyclicMin, tabu greedy, TwoNeighbor, then the rest).
// The launch stamp of a size class in the per-item trace (record_item): word
// 0 of each of its items' records, one clock read for all of them.
__global__ __launch_bounds__(64) void k_trace_start(unsigned long long *trace, int base, int count) {
    const unsigned long long t = __builtin_amdgcn_s_memrealtime();
    const unsigned long long t0 = ((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(t >> 32)) << 32) |
                                  (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)t);
    for (int k = (int)threadIdx.x; k < count; k += (int)blockDim.x) trace[4 * ((int64_t)base + k)] = t0;
}

__device__ __forceinline__ int rule_rank(int a) {
    switch (a) {
    case MAXMIN: return 0;
    case POSITIVEMIN: return 1;
    case RANDOMMIN: return 2;
    case CYCLICMIN: return 3;
    case TABU_GREEDY: return 4;
    case TWONEIGHBOR: return 5;
    default: return 6;
    }
}

// The items of each problem reordered by the cost of the rule its instance
// runs this round, costliest first.  Workgroups are handed to the compute
// units in index order, so each cost class spreads over all SIMDs instead of
// piling up wherever the random choice of rules put it.  Only the launch
// order changes: every item still runs once, and items are independent.
// One workgroup per problem; item0[p] is the problem's first item.
// It also latches the caller's cancel flag for the round: the later kernels
// of the round read the latch, so a round runs entirely or not at all.
__global__ __launch_bounds__(256) void k_sort_items(BatchDev b, int2 *items, const int *item0) {
    const int p = blockIdx.x;
    if (p == 0 && threadIdx.x == 0)
        b.ctr[3] = b.cancel ? (unsigned long long)(__hip_atomic_load(b.cancel, __ATOMIC_RELAXED,
                                                                      __HIP_MEMORY_SCOPE_SYSTEM) != 0)
                            : 0ull;
    const ProbDesc &d = b.desc[p];
    __shared__ int cnt[8];
    if (threadIdx.x < 8) cnt[threadIdx.x] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < d.instances; i += blockDim.x) atomicAdd(&cnt[rule_rank(b.algo[d.inst0 + i])], 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int r = 0; r < 8; ++r) {
            const int c = cnt[r];
            cnt[r] = acc;
            acc += c;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < d.instances; i += blockDim.x) {
        const int pos = atomicAdd(&cnt[rule_rank(b.algo[d.inst0 + i])], 1);
        items[item0[p] + pos] = make_int2(p, i);
    }
}

// Packet insertion (Section III-C, IV): one wave per (problem, pool), the
// pool's instances in increasing order; insert only when strictly better
// than the worst entry and no identical vector is pooled; ascending energies,
// a newcomer after equal energies.  The energy / algorithm / operation
// columns are worked on in LDS; the position search and the moves of the
// rows and columns below the insertion point are spread over the lanes.
// bits_lds: with a nonzero size of dynamic LDS (at least capacity x nwords
// words for every pool of the batch), the pool's bits are worked on in LDS
// as well and written back at the end.
// Hash of a packed bit vector for the duplicate tests of the insertion: the
// XOR over words of a 64-bit finaliser (SplitMix64's) of word + index
// constant, so that lanes can hash words in any order.  Equal vectors have
// equal hashes; equal hashes are confirmed word by word.
__device__ __forceinline__ uint64_t word_mix(uint64_t v, int w) {
    uint64_t z = v + 0x9E3779B97F4A7C15ull * (uint64_t)(w + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(64) void k_pool_insert(BatchDev b, const int2 *pools, int bits_lds) {
    __shared__ long long se[POOL_MAX];
    __shared__ int sal[POOL_MAX], sop[POOL_MAX];
    __shared__ uint64_t pk[WAVE];
    __shared__ unsigned int hist[STAT_WORDS];
    // with the bits in LDS, entry r of the sorted pool lives in row slot[r]:
    // an insertion moves slot numbers, not rows, and the rows are written
    // back in sorted order at the end
    __shared__ int slot[POOL_MAX];
    __shared__ uint64_t shash[POOL_MAX];  // word hash of sorted entry r (moves with the columns)
    extern __shared__ uint64_t sbits[];
    if (b.ctr[3]) return;                 // cancelled round: no packets
    const int2 pq = pools[blockIdx.x];
    const ProbDesc &d = b.desc[pq.x];
    const int q = pq.y, P = d.g.npools, m = d.g.capacity, nw = d.nw;
    const int lane = (int)threadIdx.x;
    const int64_t cell = d.pool_cell0 + (int64_t)q * m;
    int64_t *pe = b.pool_e + cell;
    int32_t *pal = b.pool_algo + cell, *pop = b.pool_op + cell;
    uint64_t *gbits = b.pool_bits + d.pool_word0 + (int64_t)q * m * nw;
    uint64_t *pbits = bits_lds ? sbits : gbits;
    for (int r = lane; r < m; r += WAVE) {
        se[r] = pe[r];
        sal[r] = pal[r];
        sop[r] = pop[r];
        slot[r] = r;
    }
    // the words of sorted entry r
    auto row = [&](int r) -> uint64_t * { return pbits + (int64_t)(bits_lds ? slot[r] : r) * nw; };
    if (bits_lds)
        for (int w = lane; w < m * nw; w += WAVE) sbits[w] = gbits[w];
    if (lane < STAT_WORDS) hist[lane] = 0;
    __syncthreads();
    for (int r = lane; r < m; r += WAVE) {      // one entry per lane
        const uint64_t *rw = row(r);
        uint64_t h = 0;
        for (int w = 0; w < nw; ++w) h ^= word_mix(rw[w], w);
        shash[r] = h;
    }
    __syncthreads();
    // the operations and algorithms the pool's instances used this round
    for (int i = q + lane * P; i < d.instances; i += P * WAVE) {
        atomicAdd(&hist[STAT_USE_OP + (b.op[d.inst0 + i] & 15)], 1u);
        atomicAdd(&hist[STAT_USE_ALGO + (b.algo[d.inst0 + i] & 7)], 1u);
    }
    __syncthreads();
    // the pool's packets in instance order, 64 at a time: the lanes load 64
    // energies at once and only those below the current worst entry are
    // visited (the worst entry never rises, so the others stay rejected)
    for (int i0 = q; i0 < d.instances; i0 += P * WAVE) {
        const int il = i0 + lane * P;
        const int64_t el = il < d.instances ? b.best_e[d.inst0 + il] : E_INF;
        // a packet identical to an entry of the same (finite) energy pooled
        // now is rejected whatever the packets before it do: at its turn that
        // entry is still pooled (a duplicate) or was evicted as the worst
        // entry (then the worst is at most its energy and the strict test
        // fails).  Each lane checks its own packet: binary search for the
        // entries of its energy, then their words.
        bool pass = el < se[m - 1];
        uint64_t ph = 0;                         // the lane's packet hash
        if (pass) {
            const uint64_t *pw = b.best + d.inst_word0 + (int64_t)il * nw;
            for (int w = 0; w < nw; ++w) ph ^= word_mix(pw[w], w);
            int lo = 0, hi = m;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (se[mid] < el) lo = mid + 1;
                else hi = mid;
            }
            for (int r = lo; r < m && se[r] == el && pass; ++r) {
                if (shash[r] != ph) continue;
                uint64_t diff = 0;
                const uint64_t *rw = row(r);
                for (int w = 0; w < nw; ++w) diff |= rw[w] ^ pw[w];
                pass = diff != 0;
            }
        }
        uint64_t cand = __builtin_amdgcn_ballot_w64(pass);
        // the packet's words, one per lane (nw <= 64); the next candidate's
        // are loaded while the current one is processed
        auto words_of = [&](uint64_t c) {
            const int64_t iw = d.inst_word0 + (int64_t)(i0 + (int)__builtin_ctzll(c) * P) * nw;
            return lane < nw ? b.best[iw + lane] : 0ull;
        };
        uint64_t nextw = cand ? words_of(cand) : 0ull;
        while (cand) {
            const int t = (int)__builtin_ctzll(cand);
            cand &= cand - 1;
            const uint64_t curw = nextw;
            if (cand) nextw = words_of(cand);
            const int i = i0 + t * P;
            const int64_t gi = d.inst0 + i;
            const int64_t e = (int64_t)readlane64((uint64_t)el, t);
            if (!(e < se[m - 1])) continue;
            if (lane < nw) pk[lane] = curw;
            __syncthreads();
            const uint64_t *bits = pk;
            const uint64_t hk = (uint64_t)readlane64(ph, t);
            // an identical vector has the same energy, unless the entry is one of
            // the initial random vectors (energy +inf, never evaluated): only
            // those entries are compared bit for bit, one entry per lane
            bool dup = false;
            for (int r0 = 0; r0 < m && !dup; r0 += WAVE) {
                const int r = r0 + lane;
                bool same = false;
                if (r < m && (se[r] == e || se[r] == E_INF) && shash[r] == hk) {
                    uint64_t diff = 0;           // every word read (independent loads), no early exit
                    const uint64_t *rw = row(r);
                    for (int w = 0; w < nw; ++w) diff |= rw[w] ^ bits[w];
                    same = diff == 0;
                }
                dup = __builtin_amdgcn_ballot_w64(same) != 0;
            }
            if (dup) continue;
            // position: the number of entries with energy <= e (they are sorted),
            // one ballot per 64 entries
            int pos = 0;
            for (int r0 = 0; r0 < m; r0 += WAVE)
                pos += (int)__builtin_popcountll(__builtin_amdgcn_ballot_w64(r0 + lane < m && se[r0 + lane] <= e));
            // bits in LDS: the worst entry's row takes the newcomer's words and
            // its slot number moves to position pos with the columns (below)
            const int freed = bits_lds ? slot[m - 1] : 0;
            if (bits_lds)
                for (int w = lane; w < nw; w += WAVE) sbits[(int64_t)freed * nw + w] = bits[w];
            // bits in global memory: rows pos .. m-2 move down one row: the words
            // [pos nw, (m-1) nw) go nw words up, in blocks of 4 x 64 words taken
            // from the top, every block loaded before it is stored
            const int64_t lo = (int64_t)pos * nw;
            for (int64_t top = bits_lds ? lo : (int64_t)(m - 1) * nw; top > lo; top -= 4 * WAVE) {
                uint64_t v[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int64_t idx = top - 1 - (k * WAVE + lane);
                    v[k] = idx >= lo ? pbits[idx] : 0ull;
                }
                __syncthreads();
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int64_t idx = top - 1 - (k * WAVE + lane);
                    if (idx >= lo) pbits[idx + nw] = v[k];
                }
                __syncthreads();
            }
            if (!bits_lds)
                for (int w = lane; w < nw; w += WAVE) pbits[(int64_t)pos * nw + w] = bits[w];
            // the columns (and slot numbers) likewise, 64 entries at a time from the top
            for (int top = m - 1; top > pos; top -= WAVE) {
                const int r = top - lane;
                long long ve = 0;
                int va = 0, vo = 0, vs = 0;
                uint64_t vh = 0;
                if (r > pos) {
                    ve = se[r - 1];
                    va = sal[r - 1];
                    vo = sop[r - 1];
                    vs = slot[r - 1];
                    vh = shash[r - 1];
                }
                __syncthreads();
                if (r > pos) {
                    se[r] = ve;
                    sal[r] = va;
                    sop[r] = vo;
                    slot[r] = vs;
                    shash[r] = vh;
                }
                __syncthreads();
            }
            if (lane == 0) {
                slot[pos] = freed;
                shash[pos] = hk;
                se[pos] = e;
                sal[pos] = b.algo[gi];
                sop[pos] = b.op[gi];
                hist[STAT_INS_OP + (b.op[gi] & 15)]++;
                hist[STAT_INS_ALGO + (b.algo[gi] & 7)]++;
            }
            __syncthreads();
        }
    }
    for (int r = lane; r < m; r += WAVE) {
        pe[r] = se[r];
        pal[r] = sal[r];
        pop[r] = sop[r];
    }
    if (bits_lds)
        for (int w = lane; w < m * nw; w += WAVE) gbits[w] = sbits[(int64_t)slot[w / nw] * nw + w % nw];
    if (lane < STAT_WORDS && hist[lane])
        atomicAdd(&b.stats[(int64_t)pq.x * STAT_WORDS + lane], (unsigned long long)hist[lane]);
}

// After the packets of a round (one workgroup per problem): the record (the
// best rank-0 entry of the pools, lowest pool on ties, when it beats the
// record) and, with DABS_GA_RESTART, the restart of merged pools (Section
// IV-B): every entry evaluated and within Hamming distance merge_hamming of
// the best entry -> a fresh fill of the pools.
__global__ __launch_bounds__(256) void k_pool_record(BatchDev b) {
    if (b.ctr[3]) return;
    ProbDesc &d = b.desc[blockIdx.x];
    const int P = d.g.npools, m = d.g.capacity, nw = d.nw;
    const int tid = (int)threadIdx.x;
    __shared__ int s_qb, s_merged;
    if (tid == 0) {
        int qb = 0;
        for (int q = 1; q < P; ++q)
            if (b.pool_e[d.pool_cell0 + (int64_t)q * m] < b.pool_e[d.pool_cell0 + (int64_t)qb * m]) qb = q;
        s_qb = qb;
        s_merged = 1;
    }
    __syncthreads();
    const int64_t eb = b.pool_e[d.pool_cell0 + (int64_t)s_qb * m];
    const uint64_t *best = b.pool_bits + d.pool_word0 + (int64_t)s_qb * m * nw;
    const bool better = eb < d.record_e;
    if (better)
        for (int w = tid; w < nw; w += blockDim.x) b.record[d.rec_word0 + w] = best[w];
    const uint32_t epoch = (uint32_t)d.epoch;
    __syncthreads();                      // every thread has read record_e and epoch
    if (better && tid == 0) {
        d.record_e = eb;
        d.record_op = b.pool_op[d.pool_cell0 + (int64_t)s_qb * m];
        d.record_algo = b.pool_algo[d.pool_cell0 + (int64_t)s_qb * m];
    }
    if (!(d.g.flags & DABS_GA_RESTART)) return;
    const int h = d.g.merge_hamming;
    for (int c = tid; c < P * m; c += blockDim.x) {
        bool far = b.pool_e[d.pool_cell0 + c] == E_INF;
        const uint64_t *v = b.pool_bits + d.pool_word0 + (int64_t)c * nw;
        int hd = 0;
        for (int w = 0; w < nw && !far; ++w) hd += __popcll(v[w] ^ best[w]);
        if (far || hd > h) atomicAnd(&s_merged, 0);
    }
    __syncthreads();
    if (!s_merged) return;
    __syncthreads();                      // every thread has read the pools' best entry
    if (tid == 0) d.epoch = (int32_t)(epoch + 1);
    fill_pools(b, d, epoch + 1, tid, blockDim.x);
}

// Round counter; a cancelled round does not count.
__global__ void k_round_end(unsigned long long *ctr) {
    if (threadIdx.x == 0 && !ctr[3]) ctr[2] += 1;
}

// Counters of problem p: out [STAT_WORDS + 2] = the counters, then the
// record's operation and algorithm (-1 before the first record).
__global__ void k_stats_out(BatchDev b, int p, int64_t *out) {
    const ProbDesc &d = b.desc[p];
    for (int w = threadIdx.x; w < STAT_WORDS; w += blockDim.x) out[w] = (int64_t)b.stats[(int64_t)p * STAT_WORDS + w];
    if (threadIdx.x == 0) {
        out[STAT_WORDS] = d.record_e == E_INF ? -1 : d.record_op;
        out[STAT_WORDS + 1] = d.record_e == E_INF ? -1 : d.record_algo;
    }
}

// Record of problem p: bits [nw], out [3] = (energy, restarts, rounds).
__global__ void k_record_out(BatchDev b, int p, uint64_t *bits, int64_t *out) {
    const ProbDesc &d = b.desc[p];
    if (bits)
        for (int w = threadIdx.x; w < d.nw; w += blockDim.x) bits[w] = b.record[d.rec_word0 + w];
    if (out && threadIdx.x == 0) {
        out[0] = d.record_e;
        out[1] = d.epoch;
        out[2] = (int64_t)b.ctr[2];
    }
}

// Start of a run: clock, and per-problem targets and first-hit records.
__global__ void k_run_begin(BatchDev b, int nprob, const int64_t *target_e) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0) b.ctr[1] = __builtin_amdgcn_s_memrealtime();
    if (p < nprob) {
        b.desc[p].target_e = target_e ? target_e[p] : INT64_MIN;
        b.desc[p].hit = ~0ull;
    }
}

// per problem: [first-hit ticks or -1, best pooled energy]
__global__ void k_progress(BatchDev b, int nprob, int64_t *out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nprob) return;
    const ProbDesc &d = b.desc[p];
    int64_t best = d.record_e;
    for (int q = 0; q < d.g.npools; ++q) {
        const int64_t e = b.pool_e[d.pool_cell0 + (int64_t)q * d.g.capacity];
        best = e < best ? e : best;
    }
    out[2 * p] = d.hit == ~0ull ? -1 : (int64_t)d.hit;
    out[2 * p + 1] = best;
}

}  // namespace dabs

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct dabs_batched {
    int nprob;
    std::vector<ProbDesc> hdesc;
    std::vector<const dabs_problem *> probs;
    // learned proposal: the network and its per-round scratch
    const dabs_mlp *mlp;
    bool mlp_ops;                      // some problem enables an MLP operation
    int *mlp_cnt;
    short *mlp_feat;
    float *mlp_logits;
    int64_t total_inst, pool_cells, pool_words, inst_words;
    BatchDev d;
    int2 *items;                       // device, grouped by class
    int *item0;                        // device, first item of each problem
    int2 *pool_list;                   // device, (problem, pool)
    int npool_list;
    int insert_lds;                    // dynamic LDS of the pool insertion (0: pool bits in global memory)
    struct Cls { int wtype, slots, begin, count, variant, lds_bytes; };
    std::vector<Cls> classes;
    hipStream_t side[MAX_CLASSES];
    hipEvent_t fork, join[MAX_CLASSES];
    hipStream_t cap;                   // capture stream (the caller's may be the null stream)
    hipGraph_t graph;
    hipGraphExec_t exec;
    bool graph_ready;
    int ttt;                           // time-to-target armed for the captured round
    bool armed;                        // a run armed targets; later runs continue its clock
    const volatile int32_t *cancel_host;  // the caller's pinned cancel flag (nullable)
    // optional timing of the batch-search kernels (DABS_SOLVER_TIME_WALK)
    bool timed;
    unsigned long long *item_trace;    // nullable: the caller's per-item trace of each round
    static constexpr int NEV = 256;
    hipEvent_t ev[2 * NEV];
    int nev;
    double walk_ms;
    long long walk_launches, flips_at_reset;
};

static void batched_free(dabs_batched *s) {
    if (s->graph_ready) {
        (void)hipGraphExecDestroy(s->exec);
        (void)hipGraphDestroy(s->graph);
    }
    for (int i = 0; i < MAX_CLASSES; ++i) {
        if (s->side[i]) (void)hipStreamDestroy(s->side[i]);
        if (s->join[i]) (void)hipEventDestroy(s->join[i]);
    }
    if (s->fork) (void)hipEventDestroy(s->fork);
    if (s->cap) (void)hipStreamDestroy(s->cap);
    for (int i = 0; i < 2 * dabs_batched::NEV; ++i)
        if (s->ev[i]) (void)hipEventDestroy(s->ev[i]);
    void *ptrs[] = {s->d.desc, s->d.pool_bits, s->d.pool_e, s->d.pool_algo, s->d.pool_op, s->d.x, s->d.target,
                    s->d.best, s->d.e, s->d.best_e, s->d.ph, s->d.algo, s->d.op, s->d.inst_prob, s->d.ctr,
                    s->d.record, s->d.stats, s->items, s->item0, s->pool_list};
    for (void *q : ptrs) (void)hipFree(q);
    (void)hipFree(s->mlp_cnt);
    (void)hipFree(s->mlp_feat);
    (void)hipFree(s->mlp_logits);
    (void)hipFree(s->d.need);
    delete s;
}

static int check_params(const dabs_problem *p, const dabs_ga_params *g, int instances) {
    if (!p || !g) return dabs_fail(DABS_E_INVALID, "null problem or params");
    if (instances < 1) return dabs_fail(DABS_E_INVALID, "instances must be >= 1");
    if (g->npools < 1 || g->capacity < 1 || g->capacity > POOL_MAX) return dabs_fail(DABS_E_INVALID, "bad pools");
    if (g->n_algos < 1 || g->n_algos > 8 || g->n_ops < 1 || g->n_ops > 16)
        return dabs_fail(DABS_E_INVALID, "bad algorithm / operation lists");
    for (int i = 0; i < g->n_algos; ++i)
        if (g->algos[i] < DABS_MAXMIN || g->algos[i] > DABS_TWONEIGHBOR)
            return dabs_fail(DABS_E_INVALID, "algorithm %d is not a main search algorithm", g->algos[i]);
    for (int i = 0; i < g->n_ops; ++i)
        if (g->ops[i] < DABS_OP_RANDOM || g->ops[i] > DABS_OP_MLP_MUTATE)
            return dabs_fail(DABS_E_INVALID, "bad genetic operation %d", g->ops[i]);
    if (g->T < 1 || g->Bn < 0 || g->tau < 0 || g->tau > TAU_MAX) return dabs_fail(DABS_E_INVALID, "bad T / Bn / tau");
    if (g->crossover_kind != 0 && g->crossover_kind != 1) return dabs_fail(DABS_E_INVALID, "bad crossover kind");
    return DABS_OK;
}

static int batched_create(const dabs_problem *const *probs, int nprob, const dabs_ga_params *params,
                          const int32_t *instances, uint32_t flags, hipStream_t st, dabs_batched **out) {
    if (!probs || !params || !instances || !out || nprob < 1) return dabs_fail(DABS_E_INVALID, "bad batch arguments");
    for (int p = 0; p < nprob; ++p) {
        const int c = check_params(probs[p], &params[p], instances[p]);
        if (c != DABS_OK) return c;
    }
    dabs_batched *s = new dabs_batched();
    s->nprob = nprob;
    s->hdesc.resize(nprob);
    int64_t inst = 0, cells = 0, pwords = 0, iwords = 0, pbits = 0, rwords = 0;
    for (int p = 0; p < nprob; ++p) {
        ProbDesc &d = s->hdesc[p];
        memset(&d, 0, sizeof(d));
        const dabs_problem *pr = probs[p];
        s->probs.push_back(pr);
        for (int i = 0; i < params[p].n_ops; ++i)
            if (params[p].ops[i] == DABS_OP_MLP_SEED || params[p].ops[i] == DABS_OP_MLP_MUTATE) s->mlp_ops = true;
        d.pool_bit0 = pbits;
        d.W = pr->W; d.rowptr = pr->rowptr; d.nz = pr->nz;
        d.diag = pr->diag; d.ld = pr->ld; d.n = pr->n; d.nw = (pr->n + 63) / 64;
        d.wtype = pr->wtype; d.slots = pr->wide ? (pr->slots | WIDE_SLOTS) : pr->slots;
        d.wmax2 = pr->wide ? 0 : 2 * pr->wmax;
        d.instances = instances[p]; d.inst0 = (int32_t)inst;
        d.g = params[p];
        d.pool_cell0 = cells; d.pool_word0 = pwords; d.inst_word0 = iwords;
        d.target_e = INT64_MIN; d.hit = ~0ull;
        d.rec_word0 = rwords; d.record_e = E_INF; d.epoch = 0; d.record_op = -1; d.record_algo = -1;
        rwords += d.nw;
        const int64_t pc = (int64_t)d.g.npools * d.g.capacity;
        inst += d.instances; cells += pc; pwords += pc * d.nw; iwords += (int64_t)d.instances * d.nw;
        pbits += pc * d.n;
    }
    s->total_inst = inst; s->pool_cells = cells; s->pool_words = pwords; s->inst_words = iwords;
    // items grouped by (wtype, slots), longest first inside a class
    std::vector<int2> items;
    std::vector<int> item0(nprob);
    std::vector<std::pair<int, int>> keys;
    for (int p = 0; p < nprob; ++p) keys.push_back({s->hdesc[p].wtype, s->hdesc[p].slots});
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    if ((int)keys.size() > MAX_CLASSES) {
        delete s;
        return dabs_fail(DABS_E_UNSUPPORTED, "too many size classes");
    }
    for (auto &k : keys) {
        std::vector<int> ps;
        for (int p = 0; p < nprob; ++p)
            if (s->hdesc[p].wtype == k.first && s->hdesc[p].slots == k.second) ps.push_back(p);
        std::stable_sort(ps.begin(), ps.end(), [&](int a, int b) {
            const ProbDesc &A = s->hdesc[a], &B = s->hdesc[b];
            return (int64_t)A.n * (A.g.Bn + A.n) > (int64_t)B.n * (B.g.Bn + B.n);
        });
        // W in LDS (variant 2) when every W of the class fits; the class's
        // items are then laid out in groups of four of one problem (each
        // problem padded with dummies of instance -1)
        int lb = 0;
        for (int p : ps) {
            const int b = (s->hdesc[p].slots & WIDE_SLOTS) ? 0 : lds_w_bytes(s->hdesc[p].wtype, s->hdesc[p].n);
            lb = (b == 0 || lb < 0) ? -1 : std::max(lb, b);
        }
        lb = lb < 0 ? 0 : lb;
        // default variant until tuned: LDS rows where they fit, else measured
        // faster uncapped from 4 slots up
        dabs_batched::Cls c = {k.first, k.second, (int)items.size(), 0, lb > 0 ? 2 : (k.second >= 4 ? 1 : 0), lb};
        for (int p : ps) {
            item0[p] = (int)items.size();
            for (int i = 0; i < s->hdesc[p].instances; ++i) items.push_back(make_int2(p, i));
            if (lb > 0)
                while (items.size() % 4) items.push_back(make_int2(p, -1));
        }
        c.count = (int)items.size() - c.begin;
        s->classes.push_back(c);
    }
    std::vector<int2> pl;
    int64_t pool_words_max = 0;
    for (int p = 0; p < nprob; ++p) {
        for (int q = 0; q < s->hdesc[p].g.npools; ++q) pl.push_back(make_int2(p, q));
        pool_words_max = std::max<int64_t>(pool_words_max, (int64_t)s->hdesc[p].g.capacity * s->hdesc[p].nw);
    }
    // the pool bits go to LDS when every pool's fit in 40 KB (beside the
    // 16 KB of energy / algorithm / operation columns)
    s->insert_lds = pool_words_max * 8 <= 40960 ? (int)(pool_words_max * 8) : 0;
    s->npool_list = (int)pl.size();
    std::vector<int32_t> ip(inst);
    for (int p = 0; p < nprob; ++p)
        for (int i = 0; i < s->hdesc[p].instances; ++i) ip[s->hdesc[p].inst0 + i] = p;
    BatchDev &d = s->d;
    bool ok = hipMalloc(&d.desc, sizeof(ProbDesc) * nprob) == hipSuccess &&
              hipMalloc(&d.pool_bits, 8 * (size_t)pwords) == hipSuccess &&
              hipMalloc(&d.pool_e, 8 * (size_t)cells) == hipSuccess &&
              hipMalloc(&d.pool_algo, 4 * (size_t)cells) == hipSuccess &&
              hipMalloc(&d.pool_op, 4 * (size_t)cells) == hipSuccess &&
              hipMalloc(&d.x, 8 * (size_t)iwords) == hipSuccess && hipMalloc(&d.target, 8 * (size_t)iwords) == hipSuccess &&
              hipMalloc(&d.best, 8 * (size_t)iwords) == hipSuccess && hipMalloc(&d.e, 8 * (size_t)inst) == hipSuccess &&
              hipMalloc(&d.best_e, 8 * (size_t)inst) == hipSuccess && hipMalloc(&d.ph, 4 * (size_t)inst) == hipSuccess &&
              hipMalloc(&d.algo, 4 * (size_t)inst) == hipSuccess && hipMalloc(&d.op, 4 * (size_t)inst) == hipSuccess &&
              hipMalloc(&d.inst_prob, 4 * (size_t)inst) == hipSuccess &&
              hipMalloc(&d.ctr, 8 * 4) == hipSuccess && hipMalloc(&d.record, 8 * (size_t)rwords) == hipSuccess &&
              hipMalloc(&d.stats, 8 * (size_t)STAT_WORDS * nprob) == hipSuccess &&
              hipMalloc(&s->items, sizeof(int2) * items.size()) == hipSuccess &&
              hipMalloc(&s->item0, sizeof(int) * nprob) == hipSuccess &&
              hipMalloc(&s->pool_list, sizeof(int2) * pl.size()) == hipSuccess;
    if (!ok) {
        batched_free(s);
        return dabs_fail(DABS_E_NOMEM, "batch allocation failed");
    }
    s->timed = (flags & DABS_SOLVER_TIME_WALK) != 0;
    ok = hipEventCreateWithFlags(&s->fork, hipEventDisableTiming) == hipSuccess &&
         hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking) == hipSuccess;
    for (size_t c = 0; c < s->classes.size() && ok; ++c)
        ok = hipStreamCreateWithFlags(&s->side[c], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&s->join[c], hipEventDisableTiming) == hipSuccess;
    for (int i = 0; i < 2 * dabs_batched::NEV && ok && s->timed; ++i) ok = hipEventCreate(&s->ev[i]) == hipSuccess;
    if (!ok) {
        batched_free(s);
        return dabs_fail(DABS_E_HIP, "stream / event creation failed");
    }
    // instances start at X = 0 with E = 0 (Section III-B)
    ok = hipMemcpyAsync(d.desc, s->hdesc.data(), sizeof(ProbDesc) * nprob, hipMemcpyHostToDevice, st) == hipSuccess &&
         hipMemcpyAsync(s->items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice, st) == hipSuccess &&
         hipMemcpyAsync(s->item0, item0.data(), sizeof(int) * nprob, hipMemcpyHostToDevice, st) == hipSuccess &&
         hipMemcpyAsync(s->pool_list, pl.data(), sizeof(int2) * pl.size(), hipMemcpyHostToDevice, st) == hipSuccess &&
         hipMemcpyAsync(d.inst_prob, ip.data(), 4 * ip.size(), hipMemcpyHostToDevice, st) == hipSuccess &&
         hipMemsetAsync(d.x, 0, 8 * (size_t)iwords, st) == hipSuccess &&
         hipMemsetAsync(d.e, 0, 8 * (size_t)inst, st) == hipSuccess &&
         hipMemsetAsync(d.ph, 0, 4 * (size_t)inst, st) == hipSuccess &&
         hipMemsetAsync(d.ctr, 0, 8 * 4, st) == hipSuccess &&
         hipMemsetAsync(d.record, 0, 8 * (size_t)rwords, st) == hipSuccess &&
         hipMemsetAsync(d.stats, 0, 8 * (size_t)STAT_WORDS * nprob, st) == hipSuccess;
    for (int p = 0; p < nprob && ok; ++p) {
        const int64_t total = (int64_t)s->hdesc[p].g.npools * s->hdesc[p].g.capacity * s->hdesc[p].nw;
        const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
        hipLaunchKernelGGL(k_pool_init, dim3(blocks), dim3(256), 0, st, d, p);
        ok = hipGetLastError() == hipSuccess;
    }
    // the host vectors must outlive the asynchronous copies
    if (!ok || hipStreamSynchronize(st) != hipSuccess) {
        batched_free(s);
        return dabs_fail(DABS_E_HIP, "batch initialisation failed");
    }
    *out = s;
    return DABS_OK;
}

// One round on stream st: targets, batch searches (one launch per size
// class; classes run on parallel streams), packet insertion, round++.
static int enqueue_round(dabs_batched *s, hipStream_t st, int ttt, bool capturing) {
    if (s->mlp && s->mlp_ops) {       // pools are scored only when an MLP operation can be chosen
        hipLaunchKernelGGL(k_ga_need, dim3((unsigned)((s->total_inst + 255) / 256)), dim3(256), 0, st, s->d,
                           (int)s->total_inst);
        HIP_OK(hipGetLastError());
        for (int p = 0; p < s->nprob; ++p) {
            const ProbDesc &d = s->hdesc[p];
            const int r = mlp_pool_logits(s->probs[p], s->mlp, s->d.pool_bits + d.pool_word0, d.g.npools,
                                          d.g.capacity, s->mlp_cnt, s->mlp_feat, s->mlp_logits + d.pool_bit0, st,
                                          s->d.need + d.pool_cell0);
            if (r != DABS_OK) return r;
        }
    }
    hipLaunchKernelGGL(k_ga_target, dim3((unsigned)((s->total_inst + 3) / 4)), dim3(256), 0, st, s->d,
                       (int)s->total_inst);
    HIP_OK(hipGetLastError());
    hipLaunchKernelGGL(k_sort_items, dim3((unsigned)s->nprob), dim3(256), 0, st, s->d, s->items, s->item0);
    HIP_OK(hipGetLastError());
    const bool timed = s->timed && !capturing;
    if (timed && s->nev == dabs_batched::NEV) {
        double out[3];
        const int r = dabs_batched_timing(s, out, 0);
        if (r != DABS_OK) return r;
    }
    if (timed) HIP_OK(hipEventRecord(s->ev[2 * s->nev], st));
    const int nc = (int)s->classes.size();
    if (nc > 1) HIP_OK(hipEventRecord(s->fork, st));
    for (int c = 0; c < nc; ++c) {
        hipStream_t cs = nc > 1 ? s->side[c] : st;
        if (nc > 1) HIP_OK(hipStreamWaitEvent(cs, s->fork, 0));
        ItemsArgs a;
        a.b = s->d;
        a.items = s->items + s->classes[c].begin;
        a.nitems = s->classes[c].count;
        a.ttt = ttt;
        a.lds_bytes = s->classes[c].lds_bytes;
        a.trace = s->item_trace;
        a.trace_base = s->classes[c].begin;
        if (a.trace) {
            hipLaunchKernelGGL(k_trace_start, dim3(1), dim3(WAVE), 0, cs, a.trace, a.trace_base, a.nitems);
            HIP_OK(hipGetLastError());
        }
        HIP_OK(launch_walk_items(s->classes[c].wtype, s->classes[c].slots, s->classes[c].variant, a, cs));
        if (nc > 1) HIP_OK(hipEventRecord(s->join[c], cs));
    }
    for (int c = 0; c < nc && nc > 1; ++c) HIP_OK(hipStreamWaitEvent(st, s->join[c], 0));
    if (timed) {
        HIP_OK(hipEventRecord(s->ev[2 * s->nev + 1], st));
        s->nev++;
    }
    hipLaunchKernelGGL(k_pool_insert, dim3(s->npool_list), dim3(64), s->insert_lds, st, s->d, s->pool_list,
                       s->insert_lds > 0 ? 1 : 0);
    HIP_OK(hipGetLastError());
    hipLaunchKernelGGL(k_pool_record, dim3(s->nprob), dim3(256), 0, st, s->d);
    HIP_OK(hipGetLastError());
    hipLaunchKernelGGL(k_round_end, dim3(1), dim3(64), 0, st, s->d.ctr);
    HIP_OK(hipGetLastError());
    return DABS_OK;
}

static int batched_run(dabs_batched *s, int rounds, const int64_t *target_e, int use_graph, hipStream_t st) {
    if (rounds < 0) return dabs_fail(DABS_E_INVALID, "rounds < 0");
    if (s->mlp_ops && !s->mlp) return dabs_fail(DABS_E_INVALID, "MLP operations enabled but no network attached");
    if (s->cancel_host && *s->cancel_host) return dabs_fail(DABS_E_CANCELLED, "the cancel flag is set");
    if (target_e) {
        // arm: clock, targets and first-hit records restart here
        hipLaunchKernelGGL(k_run_begin, dim3((s->nprob + 255) / 256), dim3(256), 0, st, s->d, s->nprob, target_e);
        HIP_OK(hipGetLastError());
        s->armed = true;
    }
    const int ttt = s->armed ? 1 : 0;
    if (!use_graph || s->timed) {
        for (int r = 0; r < rounds; ++r) {
            const int c = enqueue_round(s, st, ttt, false);
            if (c != DABS_OK) return c;
        }
        return DABS_OK;
    }
    if (!s->graph_ready || s->ttt != ttt) {
        if (s->graph_ready) {
            (void)hipGraphExecDestroy(s->exec);
            (void)hipGraphDestroy(s->graph);
            s->graph_ready = false;
        }
        // captured on the batch's own stream (the legacy null stream cannot
        // capture); nothing runs during capture, the replays go to st
        HIP_OK(hipStreamBeginCapture(s->cap, hipStreamCaptureModeThreadLocal));
        const int c = enqueue_round(s, s->cap, ttt, true);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(s->cap, &g);
        if (c != DABS_OK) {
            if (g) (void)hipGraphDestroy(g);
            return c;
        }
        if (e != hipSuccess) return dabs_fail(DABS_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
        HIP_OK(hipGraphInstantiate(&s->exec, g, nullptr, nullptr, 0));
        s->graph = g;
        s->graph_ready = true;
        s->ttt = ttt;
    }
    for (int r = 0; r < rounds; ++r) HIP_OK(hipGraphLaunch(s->exec, st));
    return DABS_OK;
}

extern "C" {

int dabs_batched_create(dabs_problem *const *probs, int32_t nprob, const dabs_ga_params *params,
                        const int32_t *instances, void *stream, dabs_batched **out) {
    uint32_t flags = 0;
    for (int p = 0; params && p < nprob; ++p) flags |= params[p].flags;
    return batched_create(probs, nprob, params, instances, flags, (hipStream_t)stream, out);
}

int dabs_batched_destroy(dabs_batched *s) {
    if (s) batched_free(s);
    return DABS_OK;
}

int dabs_batched_run(dabs_batched *s, int32_t rounds, const int64_t *target_e_dev, int32_t use_graph, void *stream) {
    if (!s) return dabs_fail(DABS_E_INVALID, "null batch");
    return batched_run(s, rounds, target_e_dev, use_graph, (hipStream_t)stream);
}

int dabs_batched_progress(const dabs_batched *s, int64_t *out_dev, void *stream) {
    if (!s || !out_dev) return dabs_fail(DABS_E_INVALID, "null argument");
    hipLaunchKernelGGL(k_progress, dim3((s->nprob + 255) / 256), dim3(256), 0, (hipStream_t)stream, s->d, s->nprob,
                       out_dev);
    HIP_OK(hipGetLastError());
    return DABS_OK;
}

int dabs_batched_pools(const dabs_batched *s, int32_t prob, uint64_t *bits_dev, int64_t *e_dev, int32_t *algo_dev,
                       int32_t *op_dev, void *stream) {
    if (!s || prob < 0 || prob >= s->nprob) return dabs_fail(DABS_E_INVALID, "bad batch or problem index");
    hipStream_t st = (hipStream_t)stream;
    const ProbDesc &d = s->hdesc[prob];
    const size_t cells = (size_t)d.g.npools * d.g.capacity;
    if (bits_dev)
        HIP_OK(hipMemcpyAsync(bits_dev, s->d.pool_bits + d.pool_word0, cells * d.nw * 8, hipMemcpyDeviceToDevice, st));
    if (e_dev) HIP_OK(hipMemcpyAsync(e_dev, s->d.pool_e + d.pool_cell0, cells * 8, hipMemcpyDeviceToDevice, st));
    if (algo_dev)
        HIP_OK(hipMemcpyAsync(algo_dev, s->d.pool_algo + d.pool_cell0, cells * 4, hipMemcpyDeviceToDevice, st));
    if (op_dev) HIP_OK(hipMemcpyAsync(op_dev, s->d.pool_op + d.pool_cell0, cells * 4, hipMemcpyDeviceToDevice, st));
    return DABS_OK;
}

int dabs_batched_state(const dabs_batched *s, int32_t prob, uint64_t *x_dev, int64_t *e_dev, uint32_t *phase_dev,
                       void *stream) {
    if (!s || prob < 0 || prob >= s->nprob) return dabs_fail(DABS_E_INVALID, "bad batch or problem index");
    hipStream_t st = (hipStream_t)stream;
    const ProbDesc &d = s->hdesc[prob];
    const size_t I = d.instances;
    if (x_dev) HIP_OK(hipMemcpyAsync(x_dev, s->d.x + d.inst_word0, I * d.nw * 8, hipMemcpyDeviceToDevice, st));
    if (e_dev) HIP_OK(hipMemcpyAsync(e_dev, s->d.e + d.inst0, I * 8, hipMemcpyDeviceToDevice, st));
    if (phase_dev) HIP_OK(hipMemcpyAsync(phase_dev, s->d.ph + d.inst0, I * 4, hipMemcpyDeviceToDevice, st));
    return DABS_OK;
}

int dabs_batched_record(const dabs_batched *s, int32_t prob, uint64_t *bits_dev, int64_t *out_dev, void *stream) {
    if (!s || prob < 0 || prob >= s->nprob) return dabs_fail(DABS_E_INVALID, "bad batch or problem index");
    hipLaunchKernelGGL(k_record_out, dim3(1), dim3(64), 0, (hipStream_t)stream, s->d, prob, bits_dev, out_dev);
    HIP_OK(hipGetLastError());
    return DABS_OK;
}

int dabs_batched_stats(const dabs_batched *s, int32_t prob, int64_t *out_dev, void *stream) {
    if (!s || !out_dev || prob < 0 || prob >= s->nprob) return dabs_fail(DABS_E_INVALID, "bad batch, problem or output");
    hipLaunchKernelGGL(k_stats_out, dim3(1), dim3(64), 0, (hipStream_t)stream, s->d, prob, out_dev);
    HIP_OK(hipGetLastError());
    return DABS_OK;
}

int dabs_batched_set_cancel(dabs_batched *s, const volatile int32_t *flag_host) {
    if (!s) return dabs_fail(DABS_E_INVALID, "null batch");
    const int *dev = nullptr;
    if (flag_host) {
        void *dp = nullptr;
        if (hipHostGetDevicePointer(&dp, (void *)flag_host, 0) != hipSuccess || !dp) {
            (void)hipGetLastError();
            return dabs_fail(DABS_E_INVALID, "the cancel flag must be pinned host memory (hipHostMalloc)");
        }
        dev = (const int *)dp;
    }
    s->cancel_host = flag_host;
    s->d.cancel = dev;
    if (s->graph_ready) {            // the captured round has the old kernel arguments
        (void)hipGraphExecDestroy(s->exec);
        (void)hipGraphDestroy(s->graph);
        s->graph_ready = false;
    }
    return DABS_OK;
}

int dabs_batched_flips(const dabs_batched *s, int64_t *total_flips_dev, void *stream) {
    if (!s || !total_flips_dev) return dabs_fail(DABS_E_INVALID, "null argument");
    HIP_OK(hipMemcpyAsync(total_flips_dev, s->d.ctr, 8, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return DABS_OK;
}

int dabs_batched_timing(dabs_batched *s, double *out, int32_t reset) {
    if (!s || !out) return dabs_fail(DABS_E_INVALID, "null argument");
    if (!s->timed) return dabs_fail(DABS_E_INVALID, "batch created without timing");
    for (int i = 0; i < s->nev; ++i) {
        float ms = 0.f;
        HIP_OK(hipEventSynchronize(s->ev[2 * i + 1]));
        HIP_OK(hipEventElapsedTime(&ms, s->ev[2 * i], s->ev[2 * i + 1]));
        s->walk_ms += ms;
        s->walk_launches++;
    }
    s->nev = 0;
    unsigned long long flips = 0;
    HIP_OK(hipMemcpy(&flips, s->d.ctr, 8, hipMemcpyDeviceToHost));
    out[0] = s->walk_ms;
    out[1] = (double)s->walk_launches;
    out[2] = (double)((long long)flips - s->flips_at_reset);
    if (reset) {
        s->walk_ms = 0;
        s->walk_launches = 0;
        s->flips_at_reset = (long long)flips;
    }
    return DABS_OK;
}

// Per size class, times every compiled variant of the item kernel on the
// batch's own items (targets of the next round, every trial from the same
// saved instance state) and keeps the fastest.  The instance state and the
// flip counter are restored afterwards, so the run continues exactly as it
// would have without tuning (the variants compute identical results).
int dabs_batched_autotune(dabs_batched *s, double *ms_out, int32_t *choice_out, void *stream) {
    if (!s) return dabs_fail(DABS_E_INVALID, "null batch");
    if (s->mlp_ops && !s->mlp) return dabs_fail(DABS_E_INVALID, "MLP operations enabled but no network attached");
    hipStream_t st = (hipStream_t)stream;
    const size_t xw = 8 * (size_t)s->inst_words, i8 = 8 * (size_t)s->total_inst, i4 = 4 * (size_t)s->total_inst;
    void *sx = nullptr, *sb = nullptr, *se = nullptr, *sbe = nullptr, *sph = nullptr, *sc = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int status = DABS_OK;
    if (hipMalloc(&sx, xw) != hipSuccess || hipMalloc(&sb, xw) != hipSuccess || hipMalloc(&se, i8) != hipSuccess ||
        hipMalloc(&sbe, i8) != hipSuccess || hipMalloc(&sph, i4) != hipSuccess || hipMalloc(&sc, 8) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        status = dabs_fail(DABS_E_NOMEM, "autotune scratch allocation failed");
    auto copy = [&](void *dst, const void *src, size_t bytes) {
        if (status == DABS_OK && hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
            status = dabs_fail(DABS_E_HIP, "autotune copy failed");
    };
    copy(sx, s->d.x, xw); copy(sb, s->d.best, xw); copy(se, s->d.e, i8); copy(sbe, s->d.best_e, i8);
    copy(sph, s->d.ph, i4); copy(sc, s->d.ctr, 8);
    if (status == DABS_OK && s->mlp && s->mlp_ops)
        for (int p = 0; p < s->nprob && status == DABS_OK; ++p) {
            const ProbDesc &d = s->hdesc[p];
            status = mlp_pool_logits(s->probs[p], s->mlp, s->d.pool_bits + d.pool_word0, d.g.npools, d.g.capacity,
                                     s->mlp_cnt, s->mlp_feat, s->mlp_logits + d.pool_bit0, st, nullptr);
        }
    if (status == DABS_OK) {
        hipLaunchKernelGGL(k_ga_target, dim3((unsigned)((s->total_inst + 3) / 4)), dim3(256), 0, st, s->d,
                           (int)s->total_inst);
        hipLaunchKernelGGL(k_sort_items, dim3((unsigned)s->nprob), dim3(256), 0, st, s->d, s->items, s->item0);
        if (hipGetLastError() != hipSuccess) status = dabs_fail(DABS_E_HIP, "target generation failed");
    }
    for (size_t c = 0; c < s->classes.size() && status == DABS_OK; ++c) {
        double best = 1e300;
        int pick = 0;
        for (int v = 0; v < WALK_VARIANTS && status == DABS_OK; ++v) {
            if (v == 2 && s->classes[c].lds_bytes <= 0) {          // W does not fit in LDS
                if (ms_out) ms_out[c * WALK_VARIANTS + v] = -1.0;
                continue;
            }
            float ms = 0.f;
            for (int rep = 0; rep < 2 && status == DABS_OK; ++rep) {   // the first launch loads the code object
                copy(s->d.x, sx, xw); copy(s->d.ph, sph, i4);
                ItemsArgs a;
                a.b = s->d;
                a.items = s->items + s->classes[c].begin;
                a.nitems = s->classes[c].count;
                a.ttt = 0;
                a.lds_bytes = s->classes[c].lds_bytes;
                a.trace = nullptr;
                a.trace_base = 0;
                if (status == DABS_OK &&
                    (hipEventRecord(e0, st) != hipSuccess ||
                     launch_walk_items(s->classes[c].wtype, s->classes[c].slots, v, a, st) != hipSuccess ||
                     hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                     hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                    status = dabs_fail(DABS_E_HIP, "autotune trial failed");
            }
            if (ms_out) ms_out[c * WALK_VARIANTS + v] = ms;
            if (ms < best) { best = ms; pick = v; }
        }
        s->classes[c].variant = pick;
        if (choice_out) choice_out[c] = pick;
    }
    copy(s->d.x, sx, xw); copy(s->d.best, sb, xw); copy(s->d.e, se, i8); copy(s->d.best_e, sbe, i8);
    copy(s->d.ph, sph, i4); copy(s->d.ctr, sc, 8);
    if (hipStreamSynchronize(st) != hipSuccess && status == DABS_OK) status = dabs_fail(DABS_E_HIP, "autotune sync");
    void *ptrs[] = {sx, sb, se, sbe, sph, sc};
    for (void *q : ptrs) (void)hipFree(q);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s->graph_ready) {            // the captured round has the old kernels
        (void)hipGraphExecDestroy(s->exec);
        (void)hipGraphDestroy(s->graph);
        s->graph_ready = false;
    }
    return status;
}

// ---------------------------------------------------------------------------
// Checkpoints: the whole search state of a batch between rounds (pools,
// instance state, record, counters, the problems' record / restart / time-to-
// target fields) as one device blob, restorable into a batch built from the
// same problems, parameters and instance counts.
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {
constexpr uint64_t CKPT_MAGIC = 0x544B43534241444Eull;   // "NDABSCKT"
constexpr uint64_t CKPT_VERSION = 1;
struct CkptLayout {
    std::vector<uint64_t> header;    // magic, version, shape words, then 6 words per problem
    size_t off[17];                  // byte offsets of the segments
    size_t bytes[17];
    size_t total;
};
size_t pad8(size_t b) { return (b + 7) & ~(size_t)7; }
CkptLayout ckpt_layout(const dabs_batched *s) {
    CkptLayout L;
    const int64_t rwords = s->hdesc.empty() ? 0 : s->hdesc.back().rec_word0 + s->hdesc.back().nw;
    L.header = {CKPT_MAGIC, CKPT_VERSION, (uint64_t)s->nprob, (uint64_t)s->total_inst, (uint64_t)s->pool_cells,
                (uint64_t)s->pool_words, (uint64_t)s->inst_words, (uint64_t)rwords};
    for (const ProbDesc &d : s->hdesc) {
        L.header.push_back((uint64_t)d.n);
        L.header.push_back((uint64_t)d.instances);
        L.header.push_back((uint64_t)d.g.npools);
        L.header.push_back((uint64_t)d.g.capacity);
        L.header.push_back((uint64_t)d.wtype);
        L.header.push_back(d.g.seed);
    }
    const size_t inst = (size_t)s->total_inst, cells = (size_t)s->pool_cells;
    const size_t sz[17] = {8 * L.header.size(),
                           sizeof(ProbDesc) * (size_t)s->nprob,
                           8 * (size_t)s->pool_words, 8 * cells, 4 * cells, 4 * cells,
                           8 * (size_t)s->inst_words, 8 * (size_t)s->inst_words, 8 * (size_t)s->inst_words,
                           8 * inst, 8 * inst, 4 * inst, 4 * inst, 4 * inst,
                           8 * 4, 8 * (size_t)rwords, 8 * (size_t)STAT_WORDS * s->nprob};
    size_t o = 0;
    for (int k = 0; k < 17; ++k) {
        L.off[k] = o;
        L.bytes[k] = sz[k];
        o += pad8(sz[k]);
    }
    L.total = o;
    return L;
}
// device arrays in segment order (segment 0 is the header, 1 the descriptors)
void ckpt_arrays(dabs_batched *s, void *a[17]) {
    const BatchDev &d = s->d;
    void *v[17] = {nullptr, d.desc, d.pool_bits, d.pool_e, d.pool_algo, d.pool_op, d.x, d.target, d.best,
                   d.e, d.best_e, d.ph, d.algo, d.op, d.ctr, d.record, d.stats};
    for (int k = 0; k < 17; ++k) a[k] = v[k];
}
}  // namespace

extern "C" {

int dabs_batched_checkpoint(dabs_batched *s, void *blob_dev, int64_t *bytes, void *stream) {
    if (!s || !bytes) return dabs_fail(DABS_E_INVALID, "null batch or size");
    const CkptLayout L = ckpt_layout(s);
    if (!blob_dev) {
        *bytes = (int64_t)L.total;
        return DABS_OK;
    }
    if (*bytes < (int64_t)L.total) return dabs_fail(DABS_E_INVALID, "checkpoint needs %zu bytes", L.total);
    hipStream_t st = (hipStream_t)stream;
    void *a[17];
    ckpt_arrays(s, a);
    // the header from host memory: a synchronous copy, so the vector may go
    HIP_OK(hipStreamSynchronize(st));
    HIP_OK(hipMemcpy(blob_dev, L.header.data(), L.bytes[0], hipMemcpyHostToDevice));
    for (int k = 1; k < 17; ++k)
        if (L.bytes[k])
            HIP_OK(hipMemcpyAsync((char *)blob_dev + L.off[k], a[k], L.bytes[k], hipMemcpyDeviceToDevice, st));
    *bytes = (int64_t)L.total;
    return DABS_OK;
}

int dabs_batched_restore(dabs_batched *s, const void *blob_dev, void *stream) {
    if (!s || !blob_dev) return dabs_fail(DABS_E_INVALID, "null batch or checkpoint");
    const CkptLayout L = ckpt_layout(s);
    hipStream_t st = (hipStream_t)stream;
    HIP_OK(hipStreamSynchronize(st));
    std::vector<uint64_t> h(L.header.size());
    HIP_OK(hipMemcpy(h.data(), blob_dev, L.bytes[0], hipMemcpyDeviceToHost));
    if (h[0] != CKPT_MAGIC || h[1] != CKPT_VERSION) return dabs_fail(DABS_E_INVALID, "not a checkpoint of this library");
    if (h != L.header)
        return dabs_fail(DABS_E_INVALID, "checkpoint of another batch shape (problems, instances, pools or seeds)");
    // descriptors: the saved per-problem record, restart and time-to-target
    // fields on this batch's own descriptors (whose pointers are this batch's)
    std::vector<ProbDesc> saved(s->nprob);
    HIP_OK(hipMemcpy(saved.data(), (const char *)blob_dev + L.off[1], L.bytes[1], hipMemcpyDeviceToHost));
    std::vector<ProbDesc> cur(s->hdesc);
    for (int p = 0; p < s->nprob; ++p) {
        cur[p].target_e = saved[p].target_e;
        cur[p].hit = saved[p].hit;
        cur[p].record_e = saved[p].record_e;
        cur[p].epoch = saved[p].epoch;
        cur[p].record_op = saved[p].record_op;
        cur[p].record_algo = saved[p].record_algo;
    }
    HIP_OK(hipMemcpy(s->d.desc, cur.data(), L.bytes[1], hipMemcpyHostToDevice));
    void *a[17];
    ckpt_arrays(s, a);
    for (int k = 2; k < 17; ++k)
        if (L.bytes[k])
            HIP_OK(hipMemcpyAsync(a[k], (const char *)blob_dev + L.off[k], L.bytes[k], hipMemcpyDeviceToDevice, st));
    s->armed = false;
    for (int p = 0; p < s->nprob; ++p) s->armed = s->armed || saved[p].target_e != INT64_MIN;
    return DABS_OK;
}

int dabs_batched_set_variant(dabs_batched *s, int32_t cls, int32_t variant) {
    if (!s) return dabs_fail(DABS_E_INVALID, "null batch");
    if (cls < 0 || cls >= (int)s->classes.size()) return dabs_fail(DABS_E_INVALID, "no size class %d", cls);
    if (variant < 0 || variant >= WALK_VARIANTS) return dabs_fail(DABS_E_INVALID, "no variant %d", variant);
    if (variant == 2 && s->classes[cls].lds_bytes <= 0)
        return dabs_fail(DABS_E_INVALID, "class %d: W does not fit in LDS", cls);
    if (s->classes[cls].variant != variant && s->graph_ready) {   // the captured round has the old kernel
        (void)hipGraphExecDestroy(s->exec);
        (void)hipGraphDestroy(s->graph);
        s->graph_ready = false;
    }
    s->classes[cls].variant = variant;
    return DABS_OK;
}

int dabs_batched_classes(const dabs_batched *s, int32_t *wtype_slots_count_variant, int32_t cap) {
    if (!s) return dabs_fail(DABS_E_INVALID, "null batch");
    const int nc = (int)s->classes.size();
    for (int c = 0; c < nc && c < cap && wtype_slots_count_variant; ++c) {
        wtype_slots_count_variant[4 * c + 0] = s->classes[c].wtype;
        wtype_slots_count_variant[4 * c + 1] = s->classes[c].slots;
        wtype_slots_count_variant[4 * c + 2] = s->classes[c].count;
        wtype_slots_count_variant[4 * c + 3] = s->classes[c].variant;
    }
    return nc;
}

int dabs_batched_trace_items(dabs_batched *s, uint64_t *buf_dev, int64_t words, int64_t *items) {
    if (!s) return dabs_fail(DABS_E_INVALID, "null batch");
    const int64_t n = s->classes.empty() ? 0 : (int64_t)s->classes.back().begin + s->classes.back().count;
    if (items) *items = n;
    if (buf_dev && words < 4 * n)
        return dabs_fail(DABS_E_INVALID, "item trace of %lld words, the round has %lld items (4 words each)",
                         (long long)words, (long long)n);
    s->item_trace = (unsigned long long *)buf_dev;
    if (s->graph_ready) {            // the captured round has the old kernel arguments
        (void)hipGraphExecDestroy(s->exec);
        (void)hipGraphDestroy(s->graph);
        s->graph_ready = false;
    }
    return DABS_OK;
}

int dabs_batched_set_mlp(dabs_batched *s, const dabs_mlp *m) {
    if (!s) return dabs_fail(DABS_E_INVALID, "null batch");
    if (m && !s->mlp_logits) {
        int64_t cnt = 0, feat = 0, bits = 0;
        for (int p = 0; p < s->nprob; ++p) {
            const ProbDesc &d = s->hdesc[p];
            if (d.n > 4096 || d.wtype == DABS_W_SPARSE)
                return dabs_fail(DABS_E_UNSUPPORTED, "the learned proposal needs a dense W with n <= 4096");
            const int64_t pc = (int64_t)d.g.npools * d.g.capacity;
            cnt = std::max<int64_t>(cnt, (int64_t)d.g.npools * d.n);
            feat = std::max<int64_t>(feat, pc * d.n * 8);
            bits += pc * d.n;
        }
        if (hipMalloc(&s->mlp_cnt, sizeof(int) * cnt) != hipSuccess ||
            hipMalloc(&s->mlp_feat, sizeof(short) * feat) != hipSuccess ||
            hipMalloc(&s->mlp_logits, sizeof(float) * bits) != hipSuccess ||
            hipMalloc(&s->d.need, sizeof(int32_t) * s->pool_cells) != hipSuccess ||
            hipMemset(s->d.need, 0, sizeof(int32_t) * s->pool_cells) != hipSuccess)
            return dabs_fail(DABS_E_NOMEM, "learned-proposal scratch allocation failed");
    }
    s->mlp = m;
    s->d.pool_logits = m ? s->mlp_logits : nullptr;
    if (s->graph_ready) {            // the captured round has the old kernel arguments
        (void)hipGraphExecDestroy(s->exec);
        (void)hipGraphDestroy(s->graph);
        s->graph_ready = false;
    }
    return DABS_OK;
}

// ------------------------------------------------- single-problem solver
struct dabs_solver {
    dabs_batched *b;
};

int dabs_solver_create(const dabs_problem *p, const dabs_ga_params *g, int32_t instances, void *stream,
                       dabs_solver **out) {
    if (!out) return dabs_fail(DABS_E_INVALID, "null output");
    dabs_batched *b = nullptr;
    const int c = check_params(p, g, instances);
    if (c != DABS_OK) return c;
    dabs_problem *pp = const_cast<dabs_problem *>(p);
    const int r = batched_create(&pp, 1, g, &instances, g->flags, (hipStream_t)stream, &b);
    if (r != DABS_OK) return r;
    *out = new dabs_solver{b};
    return DABS_OK;
}

int dabs_solver_set_mlp(dabs_solver *s, const dabs_mlp *m) {
    if (!s) return dabs_fail(DABS_E_INVALID, "null solver");
    return dabs_batched_set_mlp(s->b, m);
}

int dabs_solver_trace_items(dabs_solver *s, uint64_t *buf_dev, int64_t words, int64_t *items) {
    if (!s) return dabs_fail(DABS_E_INVALID, "null solver");
    return dabs_batched_trace_items(s->b, buf_dev, words, items);
}

int dabs_solver_autotune(dabs_solver *s, double *ms_out, int32_t *choice_out, void *stream) {
    if (!s) return dabs_fail(DABS_E_INVALID, "null solver");
    return dabs_batched_autotune(s->b, ms_out, choice_out, stream);
}

int dabs_solver_destroy(dabs_solver *s) {
    if (s) {
        batched_free(s->b);
        delete s;
    }
    return DABS_OK;
}

int dabs_solver_run(dabs_solver *s, int32_t rounds, const int64_t *target_e, void *stream) {
    if (!s) return dabs_fail(DABS_E_INVALID, "null solver");
    return batched_run(s->b, rounds, target_e, 0, (hipStream_t)stream);
}

int dabs_solver_pools(const dabs_solver *s, uint64_t *bits_dev, int64_t *e_dev, int32_t *algo_dev, int32_t *op_dev,
                      void *stream) {
    if (!s) return dabs_fail(DABS_E_INVALID, "null solver");
    return dabs_batched_pools(s->b, 0, bits_dev, e_dev, algo_dev, op_dev, stream);
}

int dabs_solver_state(const dabs_solver *s, uint64_t *x_dev, int64_t *e_dev, uint32_t *phase_dev,
                      int64_t *total_flips_dev, void *stream) {
    if (!s) return dabs_fail(DABS_E_INVALID, "null solver");
    const int r = dabs_batched_state(s->b, 0, x_dev, e_dev, phase_dev, stream);
    if (r != DABS_OK || !total_flips_dev) return r;
    return dabs_batched_flips(s->b, total_flips_dev, stream);
}

int dabs_solver_progress(const dabs_solver *s, int64_t *out_dev, void *stream) {
    if (!s) return dabs_fail(DABS_E_INVALID, "null solver");
    return dabs_batched_progress(s->b, out_dev, stream);
}

int dabs_solver_record(const dabs_solver *s, uint64_t *bits_dev, int64_t *out_dev, void *stream) {
    if (!s) return dabs_fail(DABS_E_INVALID, "null solver");
    return dabs_batched_record(s->b, 0, bits_dev, out_dev, stream);
}

int dabs_solver_stats(const dabs_solver *s, int64_t *out_dev, void *stream) {
    if (!s) return dabs_fail(DABS_E_INVALID, "null solver");
    return dabs_batched_stats(s->b, 0, out_dev, stream);
}

int dabs_solver_checkpoint(dabs_solver *s, void *blob_dev, int64_t *bytes, void *stream) {
    if (!s) return dabs_fail(DABS_E_INVALID, "null solver");
    return dabs_batched_checkpoint(s->b, blob_dev, bytes, stream);
}

int dabs_solver_restore(dabs_solver *s, const void *blob_dev, void *stream) {
    if (!s) return dabs_fail(DABS_E_INVALID, "null solver");
    return dabs_batched_restore(s->b, blob_dev, stream);
}

int dabs_solver_set_cancel(dabs_solver *s, const volatile int32_t *flag_host) {
    if (!s) return dabs_fail(DABS_E_INVALID, "null solver");
    return dabs_batched_set_cancel(s->b, flag_host);
}

int dabs_solver_timing(dabs_solver *s, double *out_host, int32_t reset) {
    if (!s) return dabs_fail(DABS_E_INVALID, "null solver");
    return dabs_batched_timing(s->b, out_host, reset);
}

}  // extern "C"
