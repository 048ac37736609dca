// dabs_internal.h -- host-side structures shared by the library's translation
// units (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/dabs.h"

struct dabs_problem {
    int32_t n;
    int32_t wtype;       // dabs_wtype (DABS_W_SPARSE: CSR rows below instead of W)
    int64_t ld;          // padded row stride (elements), multiple of 512
    int64_t bound;       // max_k |W_kk| + 2 sum_{j!=k} |W_kj|
    void *W;             // device, n rows x ld, zero diagonal, zero padding
    int32_t *diag;       // device, n
    int64_t *rowabs;     // device, n: R_k = |W_kk| + 2 sum_{j != k} |W_kj|
    int32_t wmax;        // max_{j != k} |W_kj|: a flip moves any other delta by at most 2 wmax
    int32_t wide;        // dense W searched by the wide-delta kernels (dabs_wide.h)
    int32_t packed_ok;   // dense W that the packed-key kernels can serve (B, weight ranges)
    int device;
    // sparse problems: off-diagonal rows, each nonzero one word (column in the
    // low 16 bits, weight in the high 16), and the walker's pieces per lane
    int32_t *rowptr;     // device, n + 1
    uint32_t *nz;        // device, nnz off the diagonal
    int64_t nnz;
    int32_t slots;
};

namespace dabs {

// Kernel arguments of the per-wave search kernels.
struct WalkArgs {
    const void *W;
    const int32_t *rowptr;       // sparse problems
    const uint32_t *nz;
    int32_t slots;
    const int32_t *diag;
    int64_t ld;
    int32_t n, nwords, count;
    int32_t wmax2;               // 2 max_{j != k} |W_kj|
    int32_t batch;               // 0: one phase of `rule`; 1: batch search
    int32_t rule, T, Bn, tau, greedy_cap;
    uint64_t seed;
    uint32_t phase, inst0;
    const int32_t *algo;         // batch: main rule per instance
    uint32_t *phase_arr;         // batch: per-instance phase counters (in/out)
    uint64_t *x;                 // [count][nwords] in/out
    const uint64_t *target;      // [count][nwords]
    uint64_t *best;              // [count][nwords]
    int64_t *best_e, *e;         // [count]
    int32_t *delta;              // nullable [count][n]
    int32_t *trace;              // nullable [count][trace_cap]
    int32_t trace_cap;
    int32_t *flips;              // nullable [count]
    long long *flip_total;       // nullable: atomic sum of flips
    const int64_t *target_e;     // nullable: time-to-target energy
    unsigned long long *hit;     // first-hit ticks (atomicMin), with target_e
    const unsigned long long *t0;
};

// Launches the walker kernel matching the problem's weight type and size.
hipError_t launch_walk(const dabs_problem *p, const WalkArgs &a, hipStream_t stream);

// Slot count (power of two) of the walker kernel that serves n bits.
int walk_slots(int wtype, int n);
// Shift K of the walker's key words (delta 2^K + local index) for a weight
// type and slot count: valid keys stay in (-2^29, 2^29) while |delta| <=
// 2^(29-K) - 2.  (The sparse walker holds four keys per piece, like int32.)
inline int key_shift(int wtype, int slots) {
    const int v = wtype == DABS_W_I16 ? 8 : 4, logv = wtype == DABS_W_I16 ? 3 : 2;
    int k = 0;
    while ((1 << k) < v * slots) ++k;
    return k < logv ? logv : k;
}

// ---------------------------------------------------------------- batches
// One problem of a batch as the device sees it.  Per-instance arrays of all
// problems are concatenated: instance i of problem p is global instance
// inst0 + i; its bit vectors start at word inst_word0 + i * nw.  Pools are
// concatenated likewise (cells pool_cell0 + q * m + r, words pool_word0 +
// (q * m + r) * nw).
struct ProbDesc {
    const void *W;
    const int32_t *rowptr;         // sparse problems (wtype DABS_W_SPARSE)
    const uint32_t *nz;
    const int32_t *diag;
    int64_t ld;
    int32_t n, nw, wtype, slots;
    int32_t instances, inst0;
    int64_t pool_cell0, pool_word0, inst_word0;
    int64_t pool_bit0;             // first logit of the problem's pooled bits (cells x n)
    dabs_ga_params g;
    int64_t target_e;              // time-to-target energy; INT64_MIN when unset
    unsigned long long hit;        // ticks of the first E(BEST) <= target_e (atomicMin)
    int64_t rec_word0;             // first word of the problem's record vector
    int64_t record_e;              // energy of the record (E_INF before the first round)
    int32_t epoch;                 // restarts of merged pools so far
    int32_t record_op, record_algo;// columns of the record's entry when it was last improved
    int32_t wmax2;                 // 2 max_{j != k} |W_kj| (dense problems)
};
// Per problem, the counters of the adaptive choice (Section IV-A): uses of
// every operation and main algorithm, and the packets each put into a pool.
enum { STAT_USE_OP = 0, STAT_USE_ALGO = 16, STAT_INS_OP = 24, STAT_INS_ALGO = 40, STAT_WORDS = 48 };

struct BatchDev {
    ProbDesc *desc;
    uint64_t *pool_bits;
    int64_t *pool_e;
    int32_t *pool_algo, *pool_op;
    uint64_t *x, *target, *best;   // word arrays
    int64_t *e, *best_e;
    uint32_t *ph;
    int32_t *algo, *op;
    int32_t *inst_prob;            // global instance -> problem
    const float *pool_logits;      // nullable: learned logits of every pooled bit
    int32_t *need;                 // with pool_logits: per pool cell, read by a learned operation this round
    unsigned long long *ctr;       // [0] flips, [1] run start ticks, [2] round, [3] round cancelled
    uint64_t *record;              // per problem: best pooled vector of the run (kept across restarts)
    unsigned long long *stats;     // per problem: STAT_WORDS counters
    const int *cancel;             // nullable: device view of the caller's pinned cancel flag
};

// Batch search of a list of (problem, instance) items, one wavefront each.
struct ItemsArgs {
    BatchDev b;
    const int2 *items;
    int32_t nitems;
    int32_t ttt;                   // record time to target
    int32_t lds_bytes;             // variant 2: LDS for the largest W of the class
    int32_t trace_base;            // position of the class's first item in the round's item list
    unsigned long long *trace;     // nullable: four words per item of the round (record_item)
};

// The per-item trace of a round (dabs_batched_trace_items): at the item's
// position, the ticks of the 100 MHz device clock when its size class was
// launched (written by k_trace_start: a start stamp written by the item itself
// costs the search kernels ten registers) and when it ended, the wave's
// hardware ids (HW_ID register, XCC_ID << 32) and flips | rule << 32 |
// problem << 40.  Written by lane 0 after the batch search.
__device__ __forceinline__ void record_item(const ItemsArgs &a, int idx, int flips, int rule, int prob) {
    if (!a.trace) return;
    const unsigned long long t_end = __builtin_amdgcn_s_memrealtime();
    const unsigned hw = __builtin_amdgcn_s_getreg((31 << 11) | 4);
    const unsigned xcc = __builtin_amdgcn_s_getreg((31 << 11) | 20);
    unsigned long long *r = a.trace + 4 * ((int64_t)a.trace_base + idx);
    r[1] = t_end;
    r[2] = (unsigned long long)hw | ((unsigned long long)xcc << 32);
    r[3] = (unsigned long long)(unsigned)flips | ((unsigned long long)(rule & 0xFF) << 32) |
           ((unsigned long long)(unsigned)prob << 40);
}
// Compiled variants of the item kernel per (weight type, slot count): 0 caps a
// wave at 128 VGPRs (4 waves per SIMD), 1 leaves the register file uncapped,
// 2 (problems of one slot whose W fits, see lds_w_bytes) stages W in LDS,
// one copy per workgroup of four waves running four items of one problem.
constexpr int WALK_VARIANTS = DABS_WALK_VARIANTS;
constexpr int LDS_W_MAX = 40960;
// Bytes of the LDS copy of W (rows n rounded up to a 16-byte piece), or 0
// when the problem cannot use it (more than one slot, larger than LDS_W_MAX,
// sparse).
inline int lds_w_bytes(int wtype, int n) {
    if (wtype != DABS_W_I16 && wtype != DABS_W_I32) return 0;
    const int v = wtype == DABS_W_I16 ? 8 : 4, es = wtype == DABS_W_I16 ? 2 : 4;
    if (n > 64 * v) return 0;
    const long long b = (long long)n * ((n + v - 1) / v * v) * es;
    return b <= LDS_W_MAX ? (int)b : 0;
}
hipError_t launch_walk_items(int wtype, int slots, int variant, const ItemsArgs &a, hipStream_t stream);
// A size class of the rounds served by the wide-delta kernels carries this
// flag in its slot count (one class per weight type and slot count).
constexpr int WIDE_SLOTS = 0x100;
// The wide-delta kernels (dabs_wide.hip) for a weight type and slot count.
hipError_t launch_walk_wide(int wtype, int slots, const WalkArgs &a, hipStream_t stream);
hipError_t launch_walk_items_wide(int wtype, int slots, const ItemsArgs &a, hipStream_t stream);
// The sparse walker's item kernel (dabs_sparse.hip), one launch per piece count.
hipError_t launch_sparse_items(int slots, const ItemsArgs &a, hipStream_t stream);
// The sparse walker for dabs_search / dabs_batch_search.
hipError_t launch_sparse_walk(const dabs_problem *p, const WalkArgs &a, hipStream_t stream);
// E(X) of `count` packed vectors on a sparse problem (dabs_sparse.hip).
hipError_t sparse_energy(const dabs_problem *p, const uint64_t *x, int count, int64_t *e, hipStream_t st);
// Pieces per lane of the sparse walker for n bits.
inline int sparse_slots(int n) { return (n + 255) / 256; }
// Largest n the walker kernels support for a weight type.
int max_n(int wtype);

}  // namespace dabs

namespace dabs {
// Features and (with a network) logits of every entry of P pools of capacity
// m (dabs_mlp.hip); cnt [P][n] int and feat [P m n][8] bfloat16 are scratch;
// need (nullable, [P m]): only the flagged entries' features are computed
// (and their flags cleared); the logits of the others are left meaningless.
int mlp_pool_logits(const dabs_problem *p, const dabs_mlp *net, const uint64_t *pool_bits, int P, int m, int *cnt,
                    short *feat, float *logits, hipStream_t st, int *need);
}  // namespace dabs

// Thread-local error text (dabs_capi.hip).
int dabs_fail(int status, const char *fmt, ...);
