// dabs_walk.hip -- the search kernels: one instance per wavefront, four
// instances per 256-thread workgroup, one template instance per weight type
// and slot count (slots = ceil(n / (64 * 16 / sizeof(weight)))).  Problems of
// one slot whose W fits in 40 KB read their rows from an LDS copy shared by
// the workgroup's waves.
#include "dabs_internal.h"
#include "dabs_walker.h"
#include "dabs_sparse.h"

namespace dabs {

template <typename WT>
using lds_ptr = __attribute__((address_space(3))) WT *;

// Copy the n x ldl block of W (ldl a multiple of a 16-byte piece) into the
// workgroup's LDS, every thread of the workgroup taking pieces.
template <typename WT>
__device__ __forceinline__ void stage_w(const WT *__restrict__ W, int64_t ld, int n, lds_ptr<WT> Wl, int ldl) {
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));
    constexpr int V = 16 / (int)sizeof(WT);
    const int per = ldl / V, total = n * per;
    for (int c = threadIdx.x; c < total; c += blockDim.x) {
        const int r = c / per, q = c - r * per;
        const uint4 v = *(const uint4 *)(W + (int64_t)r * ld + q * V);
        const u4 u = {v.x, v.y, v.z, v.w};
        *(__attribute__((address_space(3))) u4 *)(Wl + r * ldl + q * V) = u;
    }
    __syncthreads();
}

template <typename WT>
__host__ __device__ constexpr int lds_row(int n) {
    return (n + 16 / (int)sizeof(WT) - 1) / (16 / (int)sizeof(WT)) * (16 / (int)sizeof(WT));
}

// dabs_search / dabs_batch_search for instance wid.
template <typename WT, int SLOTS, bool LDSW>
__device__ __forceinline__ void walk_one(const WalkArgs &a, int wid, lds_ptr<const WT> Wl) {
    typedef typename Walker<WT, SLOTS, LDSW>::vecH vecH;
    vecH kb0, kb1, mul0, mul1;
    Walker<WT, SLOTS, LDSW> w(kb0, kb1, mul0, mul1);
    w.setup((const WT *)a.W, a.diag, a.ld, a.n, a.seed, a.inst0 + (uint32_t)wid, a.wmax2);
    w.Wl = Wl;
    w.ldl = lds_row<WT>(a.n);
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
__global__ __launch_bounds__(256) void k_walk(WalkArgs a) {
    const int wid = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (wid >= a.count) return;                       // whole wave leaves together
    walk_one<WT, SLOTS, false>(a, wid, nullptr);
}

// As k_walk for a problem of one slot whose W fits in LDS: the workgroup's
// four waves share one copy (staged before any wave leaves).
template <typename WT>
__global__ __launch_bounds__(256) void k_walk_lds(WalkArgs a) {
    extern __shared__ uint4 smem_w[];
    const lds_ptr<WT> Wl = (lds_ptr<WT>)(void *)smem_w;
    stage_w<WT>((const WT *)a.W, a.ld, a.n, Wl, lds_row<WT>(a.n));
    const int wid = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (wid >= a.count) return;
    walk_one<WT, 1, true>(a, wid, Wl);
}

// One wavefront (one 64-thread workgroup) per (problem, instance) item.  The
// problems of a size class are ordered longest first, and inside a problem the
// items are reordered every round by the cost of the rule they run, costliest
// first; the hardware dispatcher hands out workgroups in index order as waves
// retire, which balances the uneven items without a software queue.  Items
// are deliberately not popped from an atomic counter inside a loop: with a
// lane-0 epilogue in the same loop, the compiler may split it into nested
// loops so that lanes 1..63 re-enter the pop without lane 0 (and read item 0
// again, forever).
// WPE: the minimum waves per SIMD the register allocation must allow (4 caps
// a wave at 128 VGPRs, 2 at 256; 1 leaves the whole register file to the
// allocator).  The capped variant asks for 4 waves, except with eight slots,
// whose 128 key and multiplier words alone fill 128 registers: there it asks
// for 2.
template <int SLOTS> constexpr int CAPPED_WPE = SLOTS >= 8 ? 2 : 4;
template <typename WT, int SLOTS, bool LDSW>
__device__ __forceinline__ void walk_item(const ItemsArgs &a, int2 item, int idx, lds_ptr<const WT> Wl) {
    typedef typename Walker<WT, SLOTS, LDSW>::vecH vecH;
    vecH kb0, kb1, mul0, mul1;
    const int lane = lane_id();
    const BatchDev &b = a.b;
    const int p = __builtin_amdgcn_readfirstlane(item.x), i = __builtin_amdgcn_readfirstlane(item.y);
    ProbDesc *d = b.desc + p;
    Walker<WT, SLOTS, LDSW> w(kb0, kb1, mul0, mul1);
    w.setup((const WT *)d->W, d->diag, d->ld, d->n, d->g.seed, (uint32_t)i, d->wmax2);
    w.Wl = Wl;
    w.ldl = lds_row<WT>(d->n);
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
    if (lane == 0) {
        b.ph[gi] = ph;
        b.e[gi] = w.E;
        b.best_e[gi] = w.Eb;
        atomicAdd(&b.ctr[0], (unsigned long long)f);
        record_item(a, idx, f, b.algo[gi], p);
    }
}

template <typename WT, int SLOTS, int WPE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE))) void k_walk_items(ItemsArgs a) {
    if (a.b.ctr[3]) return;               // the round is cancelled (latched before the launch)
    const int2 item = a.items[blockIdx.x];
    if (item.y < 0) return;               // padding of a class laid out for the LDS variant
    walk_item<WT, SLOTS, false>(a, item, (int)blockIdx.x, nullptr);
}

// Variant 2: four items of one problem per workgroup (the class's items are
// laid out so: every problem's items padded to a multiple of four with
// dummies of instance -1), sharing one LDS copy of that problem's W.
template <typename WT>
__global__ __launch_bounds__(256) void k_walk_items_lds(ItemsArgs a) {
    extern __shared__ uint4 smem_w[];
    if (a.b.ctr[3]) return;
    const lds_ptr<WT> Wl = (lds_ptr<WT>)(void *)smem_w;
    const int p = a.items[4 * blockIdx.x].x;          // the first item of a group is never a dummy
    const ProbDesc *d = a.b.desc + p;
    stage_w<WT>((const WT *)d->W, d->ld, d->n, Wl, lds_row<WT>(d->n));
    const int idx = 4 * (int)blockIdx.x + (int)(threadIdx.x >> 6);
    const int2 item = a.items[idx];
    if (item.y < 0) return;
    walk_item<WT, 1, true>(a, item, idx, Wl);
}

template <typename WT, int SLOTS>
static hipError_t go_items(int variant, const ItemsArgs &a, hipStream_t st) {
    if (a.nitems < 1) return hipSuccess;
    if (variant == 2) {
        if constexpr (SLOTS == 1) {
            if (a.nitems % 4 || a.lds_bytes <= 0 || a.lds_bytes > LDS_W_MAX) return hipErrorInvalidValue;
            hipLaunchKernelGGL((k_walk_items_lds<WT>), dim3(a.nitems / 4), dim3(4 * WAVE), a.lds_bytes, st, a);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    if (variant == 0)
        hipLaunchKernelGGL((k_walk_items<WT, SLOTS, CAPPED_WPE<SLOTS>>), dim3(a.nitems), dim3(WAVE), 0, st, a);
    else
        hipLaunchKernelGGL((k_walk_items<WT, SLOTS, 1>), dim3(a.nitems), dim3(WAVE), 0, st, a);
    return hipGetLastError();
}

int walk_slots(int wtype, int n) {
    const int span = wtype == DABS_W_I16 ? 512 : 256;
    const int slots = (n + span - 1) / span;
    int p2 = 1;
    while (p2 < slots) p2 <<= 1;
    return p2;
}

hipError_t launch_walk_items(int wtype, int slots, int variant, const ItemsArgs &a, hipStream_t st) {
    if (variant < 0 || variant >= WALK_VARIANTS) return hipErrorInvalidValue;
    if (wtype == DABS_W_SPARSE) return launch_sparse_items(slots, a, st);
    if (slots & WIDE_SLOTS) {                 // one kernel: variants 0 and 1 run it, no LDS form
        if (variant == 2) return hipErrorInvalidValue;
        return launch_walk_items_wide(wtype, slots & ~WIDE_SLOTS, a, st);
    }
    if (wtype == DABS_W_I16) {
        switch (slots) {
        case 1: return go_items<int16_t, 1>(variant, a, st);
        case 2: return go_items<int16_t, 2>(variant, a, st);
        case 4: return go_items<int16_t, 4>(variant, a, st);
        case 8: return go_items<int16_t, 8>(variant, a, st);
        default: return hipErrorInvalidValue;
        }
    }
    switch (slots) {
    case 1: return go_items<int32_t, 1>(variant, a, st);
    case 2: return go_items<int32_t, 2>(variant, a, st);
    case 4: return go_items<int32_t, 4>(variant, a, st);
    case 8: return go_items<int32_t, 8>(variant, a, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename WT, int SLOTS>
static hipError_t go(const WalkArgs &a, hipStream_t st) {
    const int blocks = (a.count + 3) / 4;
    const int lb = SLOTS == 1 ? lds_w_bytes(sizeof(WT) == 2 ? DABS_W_I16 : DABS_W_I32, a.n) : 0;
    if (lb > 0)
        hipLaunchKernelGGL((k_walk_lds<WT>), dim3(blocks), dim3(256), lb, st, a);
    else
        hipLaunchKernelGGL((k_walk<WT, SLOTS>), dim3(blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

int max_n(int wtype) {
    if (wtype == DABS_W_SPARSE) return SPARSE_MAX_SLOTS * 256;
    return wtype == DABS_W_I16 ? 8 * 512 : 8 * 256;
}

hipError_t launch_walk(const dabs_problem *p, const WalkArgs &a, hipStream_t st) {
    if (p->wtype == DABS_W_SPARSE) return launch_sparse_walk(p, a, st);
    const int slots = walk_slots(p->wtype, p->n);
    if (p->wide) return launch_walk_wide(p->wtype, slots, a, st);
    if (p->wtype == DABS_W_I16) {
        switch (slots) {
        case 1: return go<int16_t, 1>(a, st);
        case 2: return go<int16_t, 2>(a, st);
        case 4: return go<int16_t, 4>(a, st);
        case 8: return go<int16_t, 8>(a, st);
        default: return hipErrorInvalidValue;
        }
    }
    switch (slots) {
    case 1: return go<int32_t, 1>(a, st);
    case 2: return go<int32_t, 2>(a, st);
    case 4: return go<int32_t, 4>(a, st);
    case 8: return go<int32_t, 8>(a, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace dabs
