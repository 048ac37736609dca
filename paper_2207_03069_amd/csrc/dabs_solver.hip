// dabs_solver.hip -- the genetic algorithm of Section IV on device-resident
// solution pools, run in generational rounds: target generation (adaptive
// operation / algorithm choice, rank selection, genetic operation), one batch
// search per instance (dabs_walk.hip), then packet insertion in instance order.
#include <string.h>

#include "dabs_device.h"
#include "dabs_internal.h"

using namespace dabs;

struct dabs_solver {
    const dabs_problem *p;
    dabs_ga_params g;
    int32_t instances, nw;
    int32_t round;            // rounds run so far
    // pools
    uint64_t *pool_bits;      // [P][m][nw]
    int64_t *pool_e;          // [P][m]
    int32_t *pool_algo, *pool_op;
    // instances
    uint64_t *x;              // [I][nw]
    int64_t *e;               // [I]
    uint32_t *ph;             // [I]
    uint64_t *target, *best;  // [I][nw]
    int64_t *best_e;          // [I]
    int32_t *algo, *op;       // [I]
    // counters: [0] total flips, [1] first-hit ticks, [2] run start ticks
    unsigned long long *ctr;
    int64_t *target_e;        // device copy of the time-to-target energy
    // optional batch-search timing (DABS_SOLVER_TIME_WALK)
    static constexpr int NEV = 256;
    hipEvent_t ev[2 * NEV];
    int nev;                  // pending event pairs
    double walk_ms;
    long long walk_launches;
    long long flips_at_reset;
};

namespace dabs {

enum { KIND_CHOICE = 0, KIND_BITS = 2, KIND_MASK = 3, KIND_RANDVEC = 4 };

struct GAArgs {
    int n, nw, P, m, instances;
    uint32_t round;
    dabs_ga_params g;
    uint64_t *pool_bits;
    int64_t *pool_e;
    int32_t *pool_algo, *pool_op;
    uint64_t *target, *best;
    int64_t *best_e;
    int32_t *algo, *op;
};

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

// Section IV-A: pools start with random vectors, energy +inf and random
// algorithm / operation columns.  One thread per (pool, entry, word).
__global__ void k_pool_init(GAArgs a) {
    const int64_t total = (int64_t)a.P * a.m * a.nw;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int w = (int)(t % a.nw);
        const int r = (int)((t / a.nw) % a.m);
        const int q = (int)(t / ((int64_t)a.nw * a.m));
        a.pool_bits[t] = rand_word(a.g.seed, (uint32_t)r, (uint32_t)q, ((uint32_t)TAG_POOL << 24) | 1u, w) &
                         tail_mask(a.n, w);
        if (w == 0) {
            const R4 d = philox((uint32_t)r, (uint32_t)q, 0, (uint32_t)TAG_POOL << 24, a.g.seed);
            const int64_t cell = (int64_t)q * a.m + r;
            a.pool_e[cell] = E_INF;
            a.pool_algo[cell] = a.g.algos[scale32(d.w[0], (uint32_t)a.g.n_algos)];
            a.pool_op[cell] = a.g.ops[scale32(d.w[1], (uint32_t)a.g.n_ops)];
        }
    }
}

__device__ __forceinline__ uint32_t rank_index(uint32_t u, uint32_t m) { return scale32((uint32_t)cube_frac(u), m); }

// Target generation (Section IV-A, IV-B): one wave per instance, lane w
// builds word w of the target.
__global__ __launch_bounds__(256) void k_ga_target(GAArgs a) {
    const int inst = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (inst >= a.instances) return;
    const int lane = (int)(threadIdx.x & 63);
    const dabs_ga_params &g = a.g;
    const int m = a.m, n = a.n;
    const int q = inst % a.P;
    const uint32_t rd = a.round;
    const R4 c = philox(rd, (uint32_t)inst, 0, ((uint32_t)TAG_GA << 24) | KIND_CHOICE, g.seed);
    const R4 v = philox(rd, (uint32_t)inst, 1, ((uint32_t)TAG_GA << 24) | KIND_CHOICE, g.seed);
    const int64_t base = (int64_t)q * m;
    const int op = c.w[0] < g.p_explore ? g.ops[scale32(c.w[1], (uint32_t)g.n_ops)]
                                        : a.pool_op[base + scale32(c.w[1], (uint32_t)m)];
    const int algo = c.w[2] < g.p_explore ? g.algos[scale32(c.w[3], (uint32_t)g.n_algos)]
                                          : a.pool_algo[base + scale32(c.w[3], (uint32_t)m)];
    const int qb = op == DABS_OP_XROSSOVER ? (q + 1) % a.P : q;
    const uint64_t *pa = a.pool_bits + (base + rank_index(v.w[0], (uint32_t)m)) * a.nw;
    const uint64_t *pb = a.pool_bits + ((int64_t)qb * m + rank_index(v.w[1], (uint32_t)m)) * a.nw;
    const uint64_t *p0 = a.pool_bits + base * a.nw;
    uint64_t *out = a.target + (int64_t)inst * a.nw;
    // IntervalZero / two-point parameters
    const uint32_t lo32 = (uint32_t)(n < 32 ? n : 32);
    const uint32_t hi32 = (uint32_t)(n / 2) > lo32 ? (uint32_t)(n / 2) : lo32;
    for (int w = lane; w < a.nw; w += WAVE) {
        const uint64_t tm = tail_mask(n, w);
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
            const uint64_t B = pb[w];
            uint64_t sel;
            if (g.crossover_kind == 1) {
                const uint32_t x1 = scale32(v.w[2], (uint32_t)n + 1), x2 = scale32(v.w[3], (uint32_t)n + 1);
                const int lo = (int)(x1 < x2 ? x1 : x2), hi = (int)(x1 < x2 ? x2 : x1);
                // bits [lo, hi) of this word
                const int b0 = 64 * w;
                const int s = lo - b0 < 0 ? 0 : (lo - b0 > 64 ? 64 : lo - b0);
                const int e = hi - b0 < 0 ? 0 : (hi - b0 > 64 ? 64 : hi - b0);
                const uint64_t upto_e = e >= 64 ? ~0ull : ((1ull << e) - 1);
                const uint64_t upto_s = s >= 64 ? ~0ull : ((1ull << s) - 1);
                sel = upto_e & ~upto_s;
            } else {
                sel = rand_word(g.seed, rd, (uint32_t)inst, ((uint32_t)TAG_GA << 24) | KIND_MASK, w);
            }
            t = (A & ~sel) | (B & sel);
            break;
        }
        case DABS_OP_ZERO:
            t = A & ~thresh_word(g.seed, rd, (uint32_t)inst, w, g.p_zero);
            break;
        case DABS_OP_ONE:
            t = A | thresh_word(g.seed, rd, (uint32_t)inst, w, g.p_one);
            break;
        case DABS_OP_INTERVALZERO: {
            const uint32_t len = lo32 + scale32(v.w[2], hi32 - lo32 + 1);
            const uint32_t st = scale32(v.w[3], (uint32_t)n);
            // zero positions st .. st+len-1 (mod n): the range [st, st+len) and,
            // when it wraps, [0, st+len-n)
            const int b0 = 64 * w;
            auto range = [&](int lo, int hi) -> uint64_t {
                const int s = lo - b0 < 0 ? 0 : (lo - b0 > 64 ? 64 : lo - b0);
                const int e = hi - b0 < 0 ? 0 : (hi - b0 > 64 ? 64 : hi - b0);
                const uint64_t upto_e = e >= 64 ? ~0ull : ((1ull << e) - 1);
                const uint64_t upto_s = s >= 64 ? ~0ull : ((1ull << s) - 1);
                return upto_e & ~upto_s;
            };
            const int end = (int)st + (int)len;
            uint64_t z = range((int)st, end < n ? end : n);
            if (end > n) z |= range(0, end - n);
            t = A & ~z;
            break;
        }
        default:
            t = A;
            break;
        }
        out[w] = t & tm;
    }
    if (lane == 0) {
        a.algo[inst] = algo;
        a.op[inst] = op;
    }
}

// Packet insertion (Section III-C, IV): one wave per pool, packets of the
// pool's instances in increasing instance order; insert only when strictly
// better than the worst entry and no identical vector is pooled; ascending
// energies, a newcomer after equal energies.  The energy / algorithm /
// operation columns are worked on in LDS (read and written by every lane);
// each lane moves only its own words of the bit vectors.
constexpr int POOL_MAX = 1024;

__global__ __launch_bounds__(64) void k_pool_insert(GAArgs a) {
    __shared__ long long se[POOL_MAX];
    __shared__ int sal[POOL_MAX], sop[POOL_MAX];
    const int q = blockIdx.x;
    const int lane = (int)threadIdx.x;
    const int m = a.m, nw = a.nw;
    int64_t *pe = a.pool_e + (int64_t)q * m;
    uint64_t *pbits = a.pool_bits + (int64_t)q * m * nw;
    int32_t *pal = a.pool_algo + (int64_t)q * m, *pop = a.pool_op + (int64_t)q * m;
    for (int r = lane; r < m; r += WAVE) {
        se[r] = pe[r];
        sal[r] = pal[r];
        sop[r] = pop[r];
    }
    __syncthreads();
    for (int i = q; i < a.instances; i += a.P) {
        const int64_t e = a.best_e[i];
        if (!(e < se[m - 1])) continue;
        const uint64_t *bits = a.best + (int64_t)i * nw;
        bool dup = false;
        for (int r = 0; r < m && !dup; ++r) {
            bool diff = false;
            for (int w = lane; w < nw; w += WAVE) diff |= pbits[(int64_t)r * nw + w] != bits[w];
            dup = __builtin_amdgcn_ballot_w64(diff) == 0;
        }
        if (dup) continue;
        int pos = 0;
        while (pos < m && se[pos] <= e) ++pos;
        for (int r = m - 1; r > pos; --r)
            for (int w = lane; w < nw; w += WAVE) pbits[(int64_t)r * nw + w] = pbits[(int64_t)(r - 1) * nw + w];
        for (int w = lane; w < nw; w += WAVE) pbits[(int64_t)pos * nw + w] = bits[w];
        __syncthreads();
        if (lane == 0) {
            for (int r = m - 1; r > pos; --r) {
                se[r] = se[r - 1];
                sal[r] = sal[r - 1];
                sop[r] = sop[r - 1];
            }
            se[pos] = e;
            sal[pos] = a.algo[i];
            sop[pos] = a.op[i];
        }
        __syncthreads();
    }
    for (int r = lane; r < m; r += WAVE) {
        pe[r] = se[r];
        pal[r] = sal[r];
        pop[r] = sop[r];
    }
}

__global__ void k_clock(unsigned long long *ctr, int reset_hit) {
    if (threadIdx.x == 0) {
        ctr[2] = __builtin_amdgcn_s_memrealtime();
        if (reset_hit) ctr[1] = ~0ull;
    }
}

// [first-hit ticks or -1, best pooled energy]
__global__ void k_progress(const int64_t *pool_e, int P, int m, const unsigned long long *ctr, int64_t *out) {
    if (threadIdx.x == 0) {
        int64_t b = E_INF;
        for (int q = 0; q < P; ++q) b = pool_e[(int64_t)q * m] < b ? pool_e[(int64_t)q * m] : b;
        out[0] = ctr[1] == ~0ull ? -1 : (int64_t)ctr[1];
        out[1] = b;
    }
}

}  // namespace dabs

#define HIP_OK(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return dabs_fail(DABS_E_HIP, "%s: %s", #call, hipGetErrorString(e_));      \
    } while (0)

static GAArgs ga_args(const dabs_solver *s) {
    GAArgs a;
    memset(&a, 0, sizeof(a));
    a.n = s->p->n; a.nw = s->nw; a.P = s->g.npools; a.m = s->g.capacity; a.instances = s->instances;
    a.round = (uint32_t)s->round; a.g = s->g;
    a.pool_bits = s->pool_bits; a.pool_e = s->pool_e; a.pool_algo = s->pool_algo; a.pool_op = s->pool_op;
    a.target = s->target; a.best = s->best; a.best_e = s->best_e; a.algo = s->algo; a.op = s->op;
    return a;
}

static void solver_free(dabs_solver *s) {
    if (s->g.flags & DABS_SOLVER_TIME_WALK)
        for (int i = 0; i < 2 * dabs_solver::NEV; ++i)
            if (s->ev[i]) (void)hipEventDestroy(s->ev[i]);
    void *ptrs[] = {s->pool_bits, s->pool_e, s->pool_algo, s->pool_op, s->x, s->e, s->ph, s->target,
                    s->best, s->best_e, s->algo, s->op, s->ctr, s->target_e};
    for (void *q : ptrs) (void)hipFree(q);
    delete s;
}

extern "C" {

int dabs_solver_create(const dabs_problem *p, const dabs_ga_params *g, int32_t instances, void *stream,
                       dabs_solver **out) {
    if (!p || !g || !out) return dabs_fail(DABS_E_INVALID, "null argument");
    if (instances < 1) return dabs_fail(DABS_E_INVALID, "instances must be >= 1");
    if (g->npools < 1 || g->capacity < 1 || g->capacity > 1024) return dabs_fail(DABS_E_INVALID, "bad pools");
    if (g->n_algos < 1 || g->n_algos > 8 || g->n_ops < 1 || g->n_ops > 16)
        return dabs_fail(DABS_E_INVALID, "bad algorithm / operation lists");
    for (int i = 0; i < g->n_algos; ++i)
        if (g->algos[i] < DABS_MAXMIN || g->algos[i] > DABS_TWONEIGHBOR)
            return dabs_fail(DABS_E_INVALID, "algorithm %d is not a main search algorithm", g->algos[i]);
    for (int i = 0; i < g->n_ops; ++i)
        if (g->ops[i] < DABS_OP_RANDOM || g->ops[i] > DABS_OP_INTERVALZERO)
            return dabs_fail(DABS_E_INVALID, "bad genetic operation %d", g->ops[i]);
    if (g->T < 1 || g->Bn < 0 || g->tau < 0 || g->tau > TAU_MAX) return dabs_fail(DABS_E_INVALID, "bad T / Bn / tau");
    if (g->crossover_kind != 0 && g->crossover_kind != 1) return dabs_fail(DABS_E_INVALID, "bad crossover kind");
    dabs_solver *s = new dabs_solver;
    memset(s, 0, sizeof(*s));
    s->p = p; s->g = *g; s->instances = instances; s->nw = (p->n + 63) / 64; s->round = 0;
    const size_t P = g->npools, m = g->capacity, I = instances, nw = s->nw;
    bool ok = hipMalloc(&s->pool_bits, P * m * nw * 8) == hipSuccess &&
              hipMalloc(&s->pool_e, P * m * 8) == hipSuccess && hipMalloc(&s->pool_algo, P * m * 4) == hipSuccess &&
              hipMalloc(&s->pool_op, P * m * 4) == hipSuccess && hipMalloc(&s->x, I * nw * 8) == hipSuccess &&
              hipMalloc(&s->e, I * 8) == hipSuccess && hipMalloc(&s->ph, I * 4) == hipSuccess &&
              hipMalloc(&s->target, I * nw * 8) == hipSuccess && hipMalloc(&s->best, I * nw * 8) == hipSuccess &&
              hipMalloc(&s->best_e, I * 8) == hipSuccess && hipMalloc(&s->algo, I * 4) == hipSuccess &&
              hipMalloc(&s->op, I * 4) == hipSuccess && hipMalloc(&s->ctr, 4 * 8) == hipSuccess &&
              hipMalloc(&s->target_e, 8) == hipSuccess;
    if (!ok) {
        solver_free(s);
        return dabs_fail(DABS_E_NOMEM, "solver allocation failed");
    }
    if (g->flags & DABS_SOLVER_TIME_WALK)
        for (int i = 0; i < 2 * dabs_solver::NEV && ok; ++i) ok = hipEventCreate(&s->ev[i]) == hipSuccess;
    if (!ok) {
        solver_free(s);
        return dabs_fail(DABS_E_HIP, "event creation failed");
    }
    hipStream_t st = (hipStream_t)stream;
    // instances start at X = 0 with E = 0 (Section III-B)
    ok = hipMemsetAsync(s->x, 0, I * nw * 8, st) == hipSuccess && hipMemsetAsync(s->e, 0, I * 8, st) == hipSuccess &&
         hipMemsetAsync(s->ph, 0, I * 4, st) == hipSuccess && hipMemsetAsync(s->ctr, 0, 4 * 8, st) == hipSuccess;
    GAArgs a = ga_args(s);
    const int64_t total = (int64_t)P * m * nw;
    const int blocks = (int)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
    hipLaunchKernelGGL(k_pool_init, dim3(blocks), dim3(256), 0, st, a);
    if (!ok || hipGetLastError() != hipSuccess) {
        solver_free(s);
        return dabs_fail(DABS_E_HIP, "solver initialisation failed");
    }
    *out = s;
    return DABS_OK;
}

int dabs_solver_destroy(dabs_solver *s) {
    if (s) solver_free(s);
    return DABS_OK;
}

int dabs_solver_run(dabs_solver *s, int32_t rounds, const int64_t *target_e, void *stream) {
    if (!s || rounds < 0) return dabs_fail(DABS_E_INVALID, "bad solver run arguments");
    hipStream_t st = (hipStream_t)stream;
    if (target_e) HIP_OK(hipMemcpyAsync(s->target_e, target_e, 8, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_clock, dim3(1), dim3(64), 0, st, s->ctr, target_e ? 1 : 0);
    HIP_OK(hipGetLastError());
    for (int r = 0; r < rounds; ++r) {
        GAArgs a = ga_args(s);
        hipLaunchKernelGGL(k_ga_target, dim3((s->instances + 3) / 4), dim3(256), 0, st, a);
        HIP_OK(hipGetLastError());
        WalkArgs w;
        memset(&w, 0, sizeof(w));
        w.W = s->p->W; w.diag = s->p->diag; w.ld = s->p->ld; w.n = s->p->n; w.nwords = s->nw;
        w.count = s->instances; w.batch = 1; w.T = s->g.T; w.Bn = s->g.Bn; w.tau = s->g.tau;
        w.greedy_cap = s->g.greedy_cap; w.seed = s->g.seed; w.inst0 = 0;
        w.algo = s->algo; w.phase_arr = s->ph; w.x = s->x; w.target = s->target; w.best = s->best;
        w.best_e = s->best_e; w.e = s->e; w.flip_total = (long long *)&s->ctr[0];
        if (target_e) {
            w.target_e = s->target_e;
            w.hit = &s->ctr[1];
            w.t0 = &s->ctr[2];
        }
        const bool timed = (s->g.flags & DABS_SOLVER_TIME_WALK) != 0;
        if (timed && s->nev == dabs_solver::NEV) {
            // fold the pending pairs into the sum to free the slots
            double out[3];
            const int st2 = dabs_solver_timing(s, out, 0);
            if (st2 != DABS_OK) return st2;
        }
        if (timed) HIP_OK(hipEventRecord(s->ev[2 * s->nev], st));
        HIP_OK(launch_walk(s->p, w, st));
        if (timed) {
            HIP_OK(hipEventRecord(s->ev[2 * s->nev + 1], st));
            s->nev++;
        }
        hipLaunchKernelGGL(k_pool_insert, dim3(s->g.npools), dim3(64), 0, st, a);
        HIP_OK(hipGetLastError());
        s->round++;
    }
    return DABS_OK;
}

int dabs_solver_pools(const dabs_solver *s, uint64_t *bits_dev, int64_t *e_dev, int32_t *algo_dev, int32_t *op_dev,
                      void *stream) {
    if (!s) return dabs_fail(DABS_E_INVALID, "null solver");
    hipStream_t st = (hipStream_t)stream;
    const size_t cells = (size_t)s->g.npools * s->g.capacity;
    if (bits_dev) HIP_OK(hipMemcpyAsync(bits_dev, s->pool_bits, cells * s->nw * 8, hipMemcpyDeviceToDevice, st));
    if (e_dev) HIP_OK(hipMemcpyAsync(e_dev, s->pool_e, cells * 8, hipMemcpyDeviceToDevice, st));
    if (algo_dev) HIP_OK(hipMemcpyAsync(algo_dev, s->pool_algo, cells * 4, hipMemcpyDeviceToDevice, st));
    if (op_dev) HIP_OK(hipMemcpyAsync(op_dev, s->pool_op, cells * 4, hipMemcpyDeviceToDevice, st));
    return DABS_OK;
}

int dabs_solver_state(const dabs_solver *s, uint64_t *x_dev, int64_t *e_dev, uint32_t *phase_dev,
                      int64_t *total_flips_dev, void *stream) {
    if (!s) return dabs_fail(DABS_E_INVALID, "null solver");
    hipStream_t st = (hipStream_t)stream;
    const size_t I = s->instances;
    if (x_dev) HIP_OK(hipMemcpyAsync(x_dev, s->x, I * s->nw * 8, hipMemcpyDeviceToDevice, st));
    if (e_dev) HIP_OK(hipMemcpyAsync(e_dev, s->e, I * 8, hipMemcpyDeviceToDevice, st));
    if (phase_dev) HIP_OK(hipMemcpyAsync(phase_dev, s->ph, I * 4, hipMemcpyDeviceToDevice, st));
    if (total_flips_dev) HIP_OK(hipMemcpyAsync(total_flips_dev, s->ctr, 8, hipMemcpyDeviceToDevice, st));
    return DABS_OK;
}

int dabs_solver_timing(dabs_solver *s, double *out, int32_t reset) {
    if (!s || !out) return dabs_fail(DABS_E_INVALID, "null argument");
    if (!(s->g.flags & DABS_SOLVER_TIME_WALK)) return dabs_fail(DABS_E_INVALID, "solver created without timing");
    for (int i = 0; i < s->nev; ++i) {
        float ms = 0.f;
        HIP_OK(hipEventSynchronize(s->ev[2 * i + 1]));
        HIP_OK(hipEventElapsedTime(&ms, s->ev[2 * i], s->ev[2 * i + 1]));
        s->walk_ms += ms;
        s->walk_launches++;
    }
    s->nev = 0;
    unsigned long long flips = 0;
    HIP_OK(hipMemcpy(&flips, s->ctr, 8, hipMemcpyDeviceToHost));
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

int dabs_solver_progress(const dabs_solver *s, int64_t *out_dev, void *stream) {
    if (!s || !out_dev) return dabs_fail(DABS_E_INVALID, "null argument");
    hipLaunchKernelGGL(k_progress, dim3(1), dim3(64), 0, (hipStream_t)stream, s->pool_e, s->g.npools,
                       s->g.capacity, s->ctr, out_dev);
    HIP_OK(hipGetLastError());
    return DABS_OK;
}

}  // extern "C"
