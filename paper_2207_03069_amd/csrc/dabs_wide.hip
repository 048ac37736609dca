// dabs_wide.hip -- the search kernels of dense problems whose delta bound
// exceeds the packed key words (WideWalker, dabs_wide.h): dabs_search /
// dabs_batch_search (k_walk_wide, four instances per 256-thread workgroup)
// and the batch searches of the generational rounds (k_walk_items_wide, one
// 64-thread workgroup per item).  One template instance per weight type and
// slot count, as for the packed kernels.
#include "dabs_internal.h"
#include "dabs_wide.h"

namespace dabs {

template <typename WT, int SLOTS>
__device__ __forceinline__ void walk_one_wide(const WalkArgs &a, int wid) {
    typedef typename WideWalker<WT, SLOTS>::vecH vecH;
    vecH d0, d1;
    WideWalker<WT, SLOTS> w(d0, d1);
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
__global__ __launch_bounds__(256) void k_walk_wide(WalkArgs a) {
    const int wid = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (wid >= a.count) return;                       // whole wave leaves together
    walk_one_wide<WT, SLOTS>(a, wid);
}

// One (problem, instance) item of a round, as walk_item of the packed kernels.
template <typename WT, int SLOTS>
__global__ __launch_bounds__(64) void k_walk_items_wide(ItemsArgs a) {
    if (a.b.ctr[3]) return;               // the round is cancelled (latched before the launch)
    const int2 item = a.items[blockIdx.x];
    if (item.y < 0) return;
    typedef typename WideWalker<WT, SLOTS>::vecH vecH;
    vecH d0, d1;
    const BatchDev &b = a.b;
    const int p = __builtin_amdgcn_readfirstlane(item.x), i = __builtin_amdgcn_readfirstlane(item.y);
    ProbDesc *d = b.desc + p;
    WideWalker<WT, SLOTS> w(d0, d1);
    w.setup((const WT *)d->W, d->diag, d->ld, d->n, d->g.seed, (uint32_t)i);
    const int64_t gi = d->inst0 + i;
    const int64_t wo = d->inst_word0 + (int64_t)i * d->nw;
    w.load_x(b.x + wo);
    if (a.ttt && d->target_e != INT64_MIN) {
        w.hit = &d->hit;
        w.target = d->target_e;
        w.t0 = b.ctr[1];
        w.hit_done = false;
    }
    uint32_t ph = b.ph[gi];
    const int f = w.batch(b.target + wo, b.algo[gi], d->g.T, d->g.Bn, d->g.tau, ph, d->g.greedy_cap);
    w.store_bits(w.xb, b.x + wo);
    w.store_bits(w.bb, b.best + wo);
    if (w.lane == 0) {
        b.ph[gi] = ph;
        b.e[gi] = w.E;
        b.best_e[gi] = w.Eb;
        atomicAdd(&b.ctr[0], (unsigned long long)f);
        record_item(a, (int)blockIdx.x, f, b.algo[gi], p);
    }
}

template <typename WT, int SLOTS>
static hipError_t go_wide(const WalkArgs &a, hipStream_t st) {
    hipLaunchKernelGGL((k_walk_wide<WT, SLOTS>), dim3((a.count + 3) / 4), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <typename WT, int SLOTS>
static hipError_t go_items_wide(const ItemsArgs &a, hipStream_t st) {
    if (a.nitems < 1) return hipSuccess;
    hipLaunchKernelGGL((k_walk_items_wide<WT, SLOTS>), dim3(a.nitems), dim3(WAVE), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_walk_wide(int wtype, int slots, const WalkArgs &a, hipStream_t st) {
    if (wtype == DABS_W_I16) {
        switch (slots) {
        case 1: return go_wide<int16_t, 1>(a, st);
        case 2: return go_wide<int16_t, 2>(a, st);
        case 4: return go_wide<int16_t, 4>(a, st);
        case 8: return go_wide<int16_t, 8>(a, st);
        default: return hipErrorInvalidValue;
        }
    }
    switch (slots) {
    case 1: return go_wide<int32_t, 1>(a, st);
    case 2: return go_wide<int32_t, 2>(a, st);
    case 4: return go_wide<int32_t, 4>(a, st);
    case 8: return go_wide<int32_t, 8>(a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_walk_items_wide(int wtype, int slots, const ItemsArgs &a, hipStream_t st) {
    if (wtype == DABS_W_I16) {
        switch (slots) {
        case 1: return go_items_wide<int16_t, 1>(a, st);
        case 2: return go_items_wide<int16_t, 2>(a, st);
        case 4: return go_items_wide<int16_t, 4>(a, st);
        case 8: return go_items_wide<int16_t, 8>(a, st);
        default: return hipErrorInvalidValue;
        }
    }
    switch (slots) {
    case 1: return go_items_wide<int32_t, 1>(a, st);
    case 2: return go_items_wide<int32_t, 2>(a, st);
    case 4: return go_items_wide<int32_t, 4>(a, st);
    case 8: return go_items_wide<int32_t, 8>(a, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace dabs
