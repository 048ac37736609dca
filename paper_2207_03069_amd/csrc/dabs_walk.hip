// dabs_walk.hip -- the search kernels: one instance per wavefront, four
// instances per 256-thread workgroup, one template instance per weight type
// and slot count (slots = ceil(n / (64 * 16 / sizeof(weight)))).
#include "dabs_internal.h"
#include "dabs_walker.h"

namespace dabs {

template <typename WT, int SLOTS>
__global__ __launch_bounds__(256) void k_walk(WalkArgs a) {
    const int wid = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (wid >= a.count) return;                       // whole wave leaves together
    typedef typename Walker<WT, SLOTS>::vecE vecE;
    vecE h, s2, ex, key;
    Walker<WT, SLOTS> w(h, s2, ex, key);
    w.setup((const WT *)a.W, a.diag, a.ld, a.n, a.seed, a.inst0 + (uint32_t)wid);
    uint64_t *x = a.x + (int64_t)wid * a.nwords;
    w.load_x(x);
    if (a.target_e && a.hit) {
        w.hit = a.hit;
        w.target = *a.target_e;
        w.t0 = *a.t0;
        w.hit_done = false;
    }
    int f;
    if (!a.batch) {
        if (a.trace) {
            w.trace = a.trace + (int64_t)wid * a.trace_cap;
            w.trace_cap = a.trace_cap;
        }
        w.begin();
        f = w.run_phase(a.rule, a.T, a.tau, a.phase,
                        a.target ? a.target + (int64_t)wid * a.nwords : nullptr, a.greedy_cap);
        if (a.trace)
            for (int q = f + w.lane; q < a.trace_cap; q += WAVE) w.trace[q] = -1;
    } else {
        uint32_t ph = a.phase_arr[wid];
        f = w.batch(a.target + (int64_t)wid * a.nwords, a.algo[wid], a.T, a.Bn, a.tau, ph, a.greedy_cap);
        if (w.lane == 0) a.phase_arr[wid] = ph;
    }
    w.store_bits(w.xb, x);
    w.store_bits(w.bb, a.best + (int64_t)wid * a.nwords);
    if (a.delta) w.store_delta(a.delta + (int64_t)wid * a.n);
    if (w.lane == 0) {
        a.best_e[wid] = w.Eb;
        a.e[wid] = w.E;
        if (a.flips) a.flips[wid] = f;
        if (a.flip_total) atomicAdd((unsigned long long *)a.flip_total, (unsigned long long)f);
    }
}

template <typename WT, int SLOTS>
static hipError_t go(const WalkArgs &a, hipStream_t st) {
    const int blocks = (a.count + 3) / 4;
    hipLaunchKernelGGL((k_walk<WT, SLOTS>), dim3(blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

int max_n(int wtype) { return wtype == DABS_W_I16 ? 4 * 512 : 4 * 256; }

hipError_t launch_walk(const dabs_problem *p, const WalkArgs &a, hipStream_t st) {
    if (p->wtype == DABS_W_I16) {
        const int slots = (p->n + 511) / 512;
        switch (slots) {
        case 1: return go<int16_t, 1>(a, st);
        case 2: return go<int16_t, 2>(a, st);
        case 3: return go<int16_t, 4>(a, st);
        case 4: return go<int16_t, 4>(a, st);
        default: return hipErrorInvalidValue;
        }
    } else {
        const int slots = (p->n + 255) / 256;
        switch (slots) {
        case 1: return go<int32_t, 1>(a, st);
        case 2: return go<int32_t, 2>(a, st);
        case 3: return go<int32_t, 4>(a, st);
        case 4: return go<int32_t, 4>(a, st);
        default: return hipErrorInvalidValue;
        }
    }
}

}  // namespace dabs
