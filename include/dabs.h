/*
 * dabs.h -- C-ABI of the MI355X bulk-search library (libdabs.so).
 *
 * The library implements the data-parallel hot path of Diverse Adaptive Bulk
 * Search (Nakano et al., arXiv 2207.03069): many independent search instances
 * over one QUBO matrix W, each keeping a bit vector X, its energy E(X) and the
 * flip deltas, choosing a bit by a search rule, flipping it and updating every
 * delta from one row of W; plus the batch search, packets and the genetic
 * algorithm on device-resident solution pools.
 *
 * Conventions shared by every call
 *  - Energy: E(X) = sum_i sum_j W_ij x_i x_j over all ordered pairs (Section
 *    II, Eq. (2)); W must be symmetric.  Energies are int64.
 *  - Bit vectors: packed little-endian uint64 words, bit k of a vector is bit
 *    (k mod 64) of word k/64; a vector of n bits occupies nwords(n) =
 *    ceil(n/64) words; padding bits must be zero on input and are zero on
 *    output.  Arrays of vectors are [count][nwords(n)] row-major.
 *  - Memory: every pointer argument named *_dev is device memory owned by the
 *    caller (for instance a torch tensor's data pointer); the library never
 *    frees or retains it after the call's stream work completes.  Handles
 *    (dabs_problem, dabs_solver) are library-owned and freed by their
 *    destroy call.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *    stream).  Calls that take a stream enqueue their work on it and return
 *    without waiting, unless stated otherwise.
 *  - Errors: every call returns a dabs_status; nothing throws or aborts across
 *    the ABI.  dabs_last_error() returns a thread-local message for the last
 *    failing call of the calling thread.
 */
#ifndef DABS_H
#define DABS_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DABS_OK = 0,
    DABS_E_INVALID = -1,        /* bad argument (null pointer, size, rule, ...) */
    DABS_E_NOT_SYMMETRIC = -2,  /* W_ij != W_ji for some i, j */
    DABS_E_RANGE = -3,          /* W too large for the exact device representation */
    DABS_E_NOMEM = -4,          /* device allocation failed */
    DABS_E_HIP = -5,            /* a HIP runtime call failed */
    DABS_E_UNSUPPORTED = -6,    /* n outside the sizes this build supports */
    DABS_E_CANCELLED = -7       /* the caller's cancel flag is set (see dabs_solver_set_cancel) */
} dabs_status;

/* Weight types: dense int16 or int32 W (dabs_problem_create), or sparse
 * (dabs_problem_create_csr). */
typedef enum { DABS_W_I16 = 0, DABS_W_I32 = 1, DABS_W_SPARSE = 2 } dabs_wtype;

/* Search rules: Section III-A (Greedy, Straight, MaxMin, CyclicMin,
 * RandomMin, PositiveMin, TwoNeighbor) and tabu greedy (T iterations, each
 * flipping the non-tabu argmin delta). */
typedef enum {
    DABS_GREEDY = 0, DABS_STRAIGHT = 1, DABS_MAXMIN = 2, DABS_CYCLICMIN = 3,
    DABS_RANDOMMIN = 4, DABS_POSITIVEMIN = 5, DABS_TWONEIGHBOR = 6, DABS_TABU_GREEDY = 7
} dabs_rule;

/* Genetic operations: Section IV-A (Random, Best, Mutation, Crossover, Zero,
 * One, IntervalZero) and IV-B (Xrossover); MLP-seed and MLP-mutate are the
 * learned proposal's operations (they need an MLP attached to the solver, see
 * dabs_mlp_*), added to the adaptive choice of Section IV-A like any other. */
typedef enum {
    DABS_OP_RANDOM = 0, DABS_OP_BEST = 1, DABS_OP_MUTATION = 2, DABS_OP_CROSSOVER = 3,
    DABS_OP_XROSSOVER = 4, DABS_OP_ZERO = 5, DABS_OP_ONE = 6, DABS_OP_INTERVALZERO = 7,
    DABS_OP_MLP_SEED = 8, DABS_OP_MLP_MUTATE = 9
} dabs_op;

typedef struct dabs_problem dabs_problem;
typedef struct dabs_solver dabs_solver;

/* Static text for a status code. */
const char *dabs_strerror(int status);
/* Message of the calling thread's last failing call ("" if none). */
const char *dabs_last_error(void);
/* Largest n this build supports for a weight type. */
int32_t dabs_max_n(int32_t wtype);
/* Largest delta bound B (see dabs_problem_create) the search accepts for n
 * bits of a weight type (Section II: every delta E(f_k X) - E(X) then fits
 * the device's int32): 2^31 - 1 for dense W; for sparse W, its key bound
 * (dabs_fast_bound).  -1 for an unsupported n or type. */
int64_t dabs_max_bound(int32_t wtype, int32_t n);
/* Largest B served by the packed-key search kernels (each delta and its bit
 * index in one 32-bit word): 2^(29 - K) - 2 with K = max(log2 V,
 * ceil(log2(V s))) (V = 8 int16 / 4 int32 elements per 16-byte piece, s the
 * power-of-two count of 64 V-bit slots that covers n).  Dense problems above
 * it, up to dabs_max_bound, run the wide-delta kernels (the same results, at
 * a lower flip rate).  -1 for an unsupported n or type. */
int64_t dabs_fast_bound(int32_t wtype, int32_t n);

/*
 * Load a QUBO matrix (the W of Section II, Eq. (2)).
 *   w_dev  device pointer to an n x n row-major matrix of int16 (wtype
 *          DABS_W_I16) or int32 (DABS_W_I32) with row stride ld >= n elements.
 * The library validates W on the device (symmetry; delta bound
 * B = max_k |W_kk| + 2 sum_{j!=k} |W_kj| <= dabs_max_bound(wtype, n) =
 * 2^31 - 1, which keeps every delta and local field exact in int32), then
 * copies it into its own padded layout and picks the search kernels: the
 * packed-key kernels when B <= dabs_fast_bound(wtype, n) (2^23 - 2 at
 * n = 4096 int16, up to 2^27 - 2 at n <= 256 int32), int16 weights off the
 * diagonal lie in [-32767, 32767] (that update negates them in 16 bits) and
 * int32 weights off the diagonal in [-(2^23 - 1), 2^23 - 1] (the operand
 * range of its 24-bit multiply); the wide-delta kernels otherwise
 * (dabs_problem_wide).  This call synchronises `stream` once (validation
 * result); the caller may free w_dev afterwards.
 * Errors: DABS_E_INVALID (null, n < 1, ld < n, bad wtype), DABS_E_UNSUPPORTED
 * (n > dabs_max_n), DABS_E_NOT_SYMMETRIC, DABS_E_RANGE (B above
 * dabs_max_bound), DABS_E_NOMEM, DABS_E_HIP.  *out is set only on success.
 */
int dabs_problem_create(const void *w_dev, int32_t n, int64_t ld, int32_t wtype,
                        void *stream, dabs_problem **out);
/*
 * Load a sparse QUBO matrix in CSR form for the sparse search kernel, which
 * keeps the deltas of an instance in LDS and on each flip updates only the
 * deltas of the nonzeros of the flipped row (Eq. (4)): n <= 15,360 bits,
 * for graphs of bounded degree such as the G-set max-cut instances and the
 * annealer graph of Section II-C.
 *   row_ptr_dev [n + 1] int32 (row_ptr[0] = 0, non-decreasing, row_ptr[n] =
 *   nnz), col_dev [nnz] int32 (strictly increasing within a row), val_dev
 *   [nnz] int32: the full symmetric matrix, diagonal entries included where
 *   nonzero.  Off-diagonal weights must lie in [-32767, 32767] (they are
 *   stored with their column in one 32-bit word); the delta bound B <=
 *   dabs_max_bound(DABS_W_SPARSE, n).  Validation (ranges, order, symmetry,
 *   B) runs on the device; the call synchronises `stream`.
 * Every call that takes a dabs_problem accepts a sparse one, except the
 * learned proposal's feature calls (DABS_E_UNSUPPORTED).
 * Errors: DABS_E_INVALID (null, n < 1, nnz < 0, bad row_ptr or column
 * order), DABS_E_UNSUPPORTED (n > 15,360), DABS_E_NOT_SYMMETRIC,
 * DABS_E_RANGE, DABS_E_NOMEM, DABS_E_HIP.
 */
int dabs_problem_create_csr(const int32_t *row_ptr_dev, const int32_t *col_dev, const int32_t *val_dev,
                            int32_t n, int64_t nnz, void *stream, dabs_problem **out);
int dabs_problem_destroy(dabs_problem *p);
/* n, weight type and delta bound B of a loaded problem (any pointer may be NULL). */
int dabs_problem_info(const dabs_problem *p, int32_t *n, int32_t *wtype, int64_t *bound);
/* 1 when the problem's searches run the wide-delta kernels (deltas as plain
 * int32 words, domains as bit masks), 0 for the packed-key kernels; a
 * negative status for a NULL problem. */
int32_t dabs_problem_wide(const dabs_problem *p);
/* Choose the kernels of a dense problem: 1 the wide-delta kernels (any dense
 * W), 0 the packed-key kernels (only W that dabs_problem_create would give
 * them).  Both give identical results.  Read when a search call is made and
 * when a solver or batch is created (existing ones keep their choice).
 * Errors: DABS_E_INVALID (NULL, wide not 0 / 1), DABS_E_UNSUPPORTED (a
 * sparse problem), DABS_E_RANGE (0 for W outside the packed kernels'
 * ranges). */
int dabs_problem_set_wide(dabs_problem *p, int32_t wide);

/*
 * Energies of `count` vectors (Eq. (2)) computed from scratch.
 *   x_dev [count][nwords] packed vectors; e_dev [count] int64 output.
 */
int dabs_energy(const dabs_problem *p, const uint64_t *x_dev, int32_t count, int64_t *e_dev,
                void *stream);

/* Parameters of one search call (one phase of one rule per instance). */
typedef struct {
    int32_t rule;        /* dabs_rule */
    int32_t T;           /* iterations for MaxMin, CyclicMin, RandomMin, PositiveMin,
                            tabu greedy; ignored by Straight and TwoNeighbor */
    int32_t tau;         /* tabu tenure (0 = no tabu) */
    int32_t greedy_cap;  /* upper bound on the flips of one Greedy phase (<= 0: 64 n) */
    uint64_t seed;       /* key of the counter-based generator */
    uint32_t phase;      /* phase counter word of the generator's counter */
    uint32_t inst0;      /* instance id of the first vector (generator counter word) */
} dabs_search_params;

/*
 * One search call (Section III-A, Steps 1-4) for `count` independent
 * instances.  Instance c starts at x_dev[c] (BEST := X), runs one phase of
 * params->rule, and writes:
 *   x_dev[c]        final X (in/out)
 *   best_dev[c]     BEST, the best vector seen by Step 1 at every visited state
 *   best_e_dev[c]   E(BEST)
 *   e_dev[c]        E(final X)
 *   delta_dev       nullable; [count][n] int32 final deltas
 *   trace_dev       nullable; [count][trace_cap] int32 flipped bit per flip,
 *                   -1 after the last flip
 *   flips_dev       nullable; [count] int32 flips made
 *   target_dev      [count][nwords] target vectors, required by DABS_STRAIGHT,
 *                   ignored otherwise.
 * Instance c uses generator counter words (iteration, inst0 + c, phase, tag).
 */
int dabs_search(const dabs_problem *p, const dabs_search_params *params, int32_t count,
                uint64_t *x_dev, const uint64_t *target_dev, uint64_t *best_dev,
                int64_t *best_e_dev, int64_t *e_dev, int32_t *delta_dev, int32_t *trace_dev,
                int32_t trace_cap, int32_t *flips_dev, void *stream);

/* Parameters of a batch search (Section III-B). */
typedef struct {
    int32_t T;           /* main-search flips, round(s n) */
    int32_t Bn;          /* batch flips, round(b n) */
    int32_t tau;         /* tabu tenure of the main searches */
    int32_t greedy_cap;  /* as in dabs_search_params */
    uint64_t seed;
    uint32_t inst0;
    uint32_t reserved;
} dabs_batch_params;

/*
 * Batch search for `count` instances (Section III-B): BEST := X, Straight to
 * target_dev[c], Greedy, then {main search algo_dev[c] (T flips; TwoNeighbor
 * 2n-1 flips, once), Greedy} while the flips of this batch search are below
 * Bn.  Packets (Section III-C): the target goes in, BEST and E(BEST) come
 * out; the algorithm field is read only.
 *   x_dev      [count][nwords] in/out current X (kept between batch searches)
 *   target_dev [count][nwords] targets D
 *   algo_dev   [count] int32 main rule (MaxMin .. TwoNeighbor)
 *   phase_dev  [count] uint32 in/out main-phase counters (one per main phase)
 *   best_dev, best_e_dev, e_dev  as in dabs_search
 *   flips_dev  nullable [count] int32 flips of this batch search
 */
int dabs_batch_search(const dabs_problem *p, const dabs_batch_params *params, int32_t count,
                      uint64_t *x_dev, const uint64_t *target_dev, const int32_t *algo_dev,
                      uint32_t *phase_dev, uint64_t *best_dev, int64_t *best_e_dev,
                      int64_t *e_dev, int32_t *flips_dev, void *stream);

/* Parameters of the genetic algorithm on device pools (Section IV). */
typedef struct {
    int32_t n_algos;
    int32_t algos[8];        /* enabled main algorithms (dabs_rule values) */
    int32_t n_ops;
    int32_t ops[16];         /* enabled genetic operations (dabs_op values) */
    uint32_t p_explore;      /* u32 threshold of the uniform op/algo choice (5% = 214748365) */
    uint32_t p_mutation;     /* per-bit u32 thresholds (1/8 = 536870912) */
    uint32_t p_zero;
    uint32_t p_one;
    int32_t crossover_kind;  /* 0 uniform, 1 two-point */
    int32_t capacity;        /* pool capacity m (1..1024) */
    int32_t npools;          /* pools in the ring (instance i belongs to pool i mod npools) */
    int32_t tau;
    int32_t T;
    int32_t Bn;
    int32_t greedy_cap;
    uint32_t flags;          /* DABS_SOLVER_TIME_WALK, DABS_GA_RESTART */
    int32_t merge_hamming;   /* DABS_GA_RESTART: merged when every entry is within this distance of the best */
    uint64_t seed;
} dabs_ga_params;

/* time every batch-search launch with HIP events (dabs_solver_timing) */
#define DABS_SOLVER_TIME_WALK 1u
/* Restart of merged pools (Section IV-B): after the packets of a round are
 * inserted, the pools count as merged when every entry has been evaluated
 * (finite energy) and lies within Hamming distance merge_hamming of the best
 * pooled vector (the rank-0 entry of least energy, lowest pool on ties); they
 * are then refilled with fresh random vectors of energy +inf and random
 * algorithm / operation columns (the draws of refill e use Philox sub-tags
 * 2e + 1 for the bits and 2e for the columns of TAG_POOL; the first fill is
 * e = 0).  Instances keep their X.  The best vector of the run survives in
 * the record (dabs_solver_record). */
#define DABS_GA_RESTART 2u

/*
 * Solver: `instances` search instances and `npools` solution pools on one
 * problem, all device resident.  Instances start at X = 0; pools start full
 * of random vectors with energy +inf (INT64_MAX) and random algorithm /
 * operation columns.  Allocates its state on the device; the problem must
 * outlive the solver.
 */
int dabs_solver_create(const dabs_problem *p, const dabs_ga_params *params, int32_t instances,
                       void *stream, dabs_solver **out);
int dabs_solver_destroy(dabs_solver *s);

/*
 * Run `rounds` generational rounds (Section IV with the batch search of
 * Section III-B): every instance draws a target from its pool (adaptive
 * op/algorithm choice, rank selection, genetic operation), runs one batch
 * search, and the packets are inserted into the pools in instance order.
 * target_e (device, int64): if not NULL, arms time-to-target: the clock
 * restarts at the start of this call and the device records the first time
 * (ticks of the 100 MHz device clock) at which some instance's
 * E(BEST) <= *target_e.  NULL continues the last armed run: same target,
 * same clock, same first-hit record (no target if none was ever armed).
 */
int dabs_solver_run(dabs_solver *s, int32_t rounds, const int64_t *target_e, void *stream);

/*
 * Copy the pools out (device to device, on `stream`): bits [npools][capacity]
 * [nwords], energies [npools][capacity] int64, algorithm and op columns
 * [npools][capacity] int32.  Any pointer may be NULL.
 */
int dabs_solver_pools(const dabs_solver *s, uint64_t *bits_dev, int64_t *e_dev, int32_t *algo_dev,
                      int32_t *op_dev, void *stream);

/*
 * Copy per-instance state out: current X [instances][nwords], E(X)
 * [instances], main-phase counters [instances], and the total flips of all
 * rounds so far (int64, one value).  Any pointer may be NULL.
 */
int dabs_solver_state(const dabs_solver *s, uint64_t *x_dev, int64_t *e_dev, uint32_t *phase_dev,
                      int64_t *total_flips_dev, void *stream);

/*
 * Time-to-target record (ticks of the 100 MHz device clock since the start of
 * the run that set it; -1 if not reached) and the best energy found so far, as
 * two int64 values written to out_dev.
 */
int dabs_solver_progress(const dabs_solver *s, int64_t *out_dev, void *stream);

/*
 * The run's record: the best pooled vector seen at the end of any round so
 * far (kept across restarts), bits_dev [nwords] (nullable), and out_dev int64
 * [3] = (its energy (INT64_MAX before the first round), restarts so far,
 * rounds completed; cancelled rounds are not counted).
 */
int dabs_solver_record(const dabs_solver *s, uint64_t *bits_dev, int64_t *out_dev, void *stream);

/*
 * Counters of the adaptive choice (Section IV-A), the bookkeeping behind the
 * per-operation and per-algorithm tables of Section VI-D.  out_dev int64
 * [DABS_STATS]: how many times each genetic operation (16 slots, dabs_op)
 * and each main algorithm (8 slots, dabs_rule) was chosen, how many of their
 * packets entered a pool (same slots), then the operation and algorithm
 * columns of the record's entry when the record was last improved (-1 before
 * the first round).  Cancelled rounds count nothing.
 */
#define DABS_STATS 50
int dabs_solver_stats(const dabs_solver *s, int64_t *out_dev, void *stream);

/* As dabs_batched_checkpoint / dabs_batched_restore for a single problem. */
int dabs_solver_checkpoint(dabs_solver *s, void *blob_dev, int64_t *bytes, void *stream);
int dabs_solver_restore(dabs_solver *s, const void *blob_dev, void *stream);

/*
 * Cancellation (Section III-B: the device repeats batch searches until the
 * host requests termination).  flag_host is a 32-bit word of pinned host
 * memory that the device can read (hipHostMalloc, or a tensor created with
 * pin_memory=True); NULL detaches.  While *flag_host != 0:
 *   - dabs_solver_run returns DABS_E_CANCELLED at once and enqueues nothing;
 *   - a round already enqueued that starts its searches while the flag is
 *     set does nothing: no batch search runs, the pools, instances, record
 *     and round counter stay as they were (so a run resumed after the flag is
 *     cleared continues exactly as if the cancelled rounds had not been
 *     enqueued).  The flag is read once per round, before its searches
 *     start, so a round in progress finishes.
 * Every kernel still runs to its normal end.  The memory must stay valid
 * until it is detached or the solver is destroyed.
 * Errors: DABS_E_INVALID (null solver, or flag_host not pinned host memory
 * visible to the device).
 */
int dabs_solver_set_cancel(dabs_solver *s, const volatile int32_t *flag_host);

/*
 * Batch-search kernel timing of a solver created with DABS_SOLVER_TIME_WALK:
 * out_host[0] = summed elapsed milliseconds of the batch-search launches,
 * out_host[1] = number of launches, out_host[2] = flips they made (all since
 * the last reset).  Synchronises on the recorded events.  reset != 0 clears
 * the sums after reading.  DABS_E_INVALID when the solver was created
 * without the flag.
 */
int dabs_solver_timing(dabs_solver *s, double *out_host, int32_t reset);

/*
 * Per-item trace of the batch searches of later rounds (Section III-B's batch
 * search per instance; tracing, to see what sets a round's length).  Every
 * round overwrites buf_dev (caller-owned device memory of at least 4 x items
 * uint64 words) with one record per item of the round, at the item's
 * position in the round's launch order (size classes in turn, each problem's
 * items in the order its rules were sorted that round):
 *   [0] the launch of the item's size class, [1] the item's end, in ticks
 *       of the device's 100 MHz clock (items beyond the resident waves of
 *       a launch start later than [0]);
 *   [2] the wave's hardware ids: HW_ID register (bits 4-5 SIMD, 8-11 CU,
 *       13-15 shader engine) | XCC_ID << 32;
 *   [3] flips | main rule << 32 | problem << 40.
 * Padding items of the LDS variant get word [0] only.  buf_dev
 * NULL stops tracing.  *items (nullable) receives the round's item count.
 * Records cost one store per item; a captured round is captured again.
 * Errors: DABS_E_INVALID (null handle, buffer shorter than 4 x items).
 */
int dabs_solver_trace_items(dabs_solver *s, uint64_t *buf_dev, int64_t words, int64_t *items);

/*
 * Batched solver: many problems of uneven n served by one device loop.  Every
 * round draws the targets of all instances of all problems, runs their batch
 * searches (one wavefront per instance, one launch per weight type and slot
 * count, on parallel streams, longest problems first), inserts the packets
 * into each problem's pools and advances the round.  Each problem has its
 * own parameters, pools, instances and generator key (params[p].seed), and
 * evolves exactly as dabs_solver_* on that problem alone would.
 *   probs[p], params[p], instances[p]  for p < nprob (the problems must
 *   outlive the batch).
 */
typedef struct dabs_batched dabs_batched;
int dabs_batched_create(dabs_problem *const *probs, int32_t nprob, const dabs_ga_params *params,
                        const int32_t *instances, void *stream, dabs_batched **out);
int dabs_batched_destroy(dabs_batched *b);
/*
 * Run `rounds` rounds.  use_graph != 0 captures one round into a HIP graph
 * on first use and replays it (ignored when the batch times its kernels).
 * target_e_dev: nullable [nprob] int64 time-to-target energies; non-NULL
 * arms them (clock restarts, first hits cleared), NULL continues the last
 * armed run; first hits are in 100 MHz device ticks from the arming call.
 */
int dabs_batched_run(dabs_batched *b, int32_t rounds, const int64_t *target_e_dev, int32_t use_graph,
                     void *stream);
/* [nprob][2] int64: first-hit ticks (-1 if not reached) and best pooled energy. */
int dabs_batched_progress(const dabs_batched *b, int64_t *out_dev, void *stream);
/* Pools / instance state of problem `prob`, as dabs_solver_pools / _state. */
int dabs_batched_pools(const dabs_batched *b, int32_t prob, uint64_t *bits_dev, int64_t *e_dev,
                       int32_t *algo_dev, int32_t *op_dev, void *stream);
int dabs_batched_state(const dabs_batched *b, int32_t prob, uint64_t *x_dev, int64_t *e_dev,
                       uint32_t *phase_dev, void *stream);
/* Total flips of all instances of all problems so far (one int64). */
int dabs_batched_flips(const dabs_batched *b, int64_t *total_flips_dev, void *stream);
/* As dabs_solver_timing (DABS_SOLVER_TIME_WALK in any problem's flags). */
int dabs_batched_timing(dabs_batched *b, double *out_host, int32_t reset);
/* As dabs_solver_record for problem `prob` (the round counter is the batch's). */
int dabs_batched_record(const dabs_batched *b, int32_t prob, uint64_t *bits_dev, int64_t *out_dev, void *stream);
/* As dabs_solver_stats for problem `prob`. */
int dabs_batched_stats(const dabs_batched *b, int32_t prob, int64_t *out_dev, void *stream);
/* As dabs_solver_set_cancel, for every problem of the batch (graph replays
 * included: the flag is read by the device). */
int dabs_batched_set_cancel(dabs_batched *b, const volatile int32_t *flag_host);
/*
 * Checkpoint and resume.  dabs_batched_checkpoint writes the batch's whole
 * search state between rounds into blob_dev, caller-owned device memory of
 * *bytes bytes: the pools, every instance's X / E / phase counter and last
 * packet, the round and flip counters, the records, the counters of the
 * adaptive choice and each problem's record, restart and time-to-target
 * fields, behind a header that names the batch's shape.  blob_dev == NULL
 * only sets *bytes to the size needed; a smaller *bytes is DABS_E_INVALID.
 * Ordered on `stream` (the header copy synchronises it).
 * dabs_batched_restore loads such a blob into a batch created from problems
 * of the same sizes and weight types with the same parameters and instance
 * counts (DABS_E_INVALID otherwise, checked on the header: n, instances,
 * pools, capacity, weight type and seed of every problem); later rounds then
 * evolve exactly as they would have in the saved batch.  A time-to-target
 * clock continues from its saved start tick, which is meaningful on the same
 * device in the same process only.  Synchronises `stream` for the header.
 */
int dabs_batched_checkpoint(dabs_batched *b, void *blob_dev, int64_t *bytes, void *stream);
int dabs_batched_restore(dabs_batched *b, const void *blob_dev, void *stream);

/*
 * Autotuner: for every size class of the batch (weight type x slot count),
 * times each compiled variant of the batch-search kernel on the batch's own
 * next-round items and keeps the fastest for the following rounds:
 *   0  W rows from global memory / L2, registers capped for 4 waves per SIMD
 *      (2 for classes of eight slots),
 *   1  the same with the register file uncapped,
 *   2  W staged in LDS, one copy per workgroup of four waves (classes of one
 *      slot whose every W fits in 40 KB; -1 ms for other classes).
 * The instance state is saved and restored, so results are unchanged (only
 * speed).  Sparse classes have one kernel (every variant runs it).
 * Synchronises the stream.
 *   ms_out     nullable [nclasses][DABS_WALK_VARIANTS] milliseconds per variant
 *   choice_out nullable [nclasses] chosen variant
 * dabs_batched_classes fills [min(nclasses, cap)][4] = (wtype, slots, items,
 * variant) and returns nclasses.
 */
#define DABS_WALK_VARIANTS 3
int dabs_batched_autotune(dabs_batched *b, double *ms_out, int32_t *choice_out, void *stream);
/* Pins size class `cls` (an index into dabs_batched_classes) to `variant`
 * instead of timing them; results do not depend on the variant, only speed.
 * Variant 0 caps registers for 4 waves per SIMD (2 for classes of eight
 * slots).  DABS_E_INVALID: bad class or variant, or variant 2 for a class
 * whose W does not all fit in LDS.  Host only (no stream). */
int dabs_batched_set_variant(dabs_batched *b, int32_t cls, int32_t variant);
int dabs_solver_autotune(dabs_solver *s, double *ms_out, int32_t *choice_out, void *stream);
int dabs_batched_classes(const dabs_batched *b, int32_t *wtype_slots_count_variant, int32_t cap);
/* As dabs_solver_trace_items, for a batch. */
int dabs_batched_trace_items(dabs_batched *b, uint64_t *buf_dev, int64_t words, int64_t *items);

/*
 * Ising front-end (Section I, Eq. (1)): H(S) = sum_{(i,j) in E} J_ij s_i s_j
 * + sum_i h_i s_i over spins s_i in {-1, +1}.  With s_i = 2 x_i - 1 the
 * equivalent QUBO (Eq. (2), full ordered sum) has W_ij = W_ji = 2 J_ij
 * (i != j) and W_ii = 2 h_i - 2 sum_{j ~ i} J_ij, and E(X) = H(S) + c with
 * c = sum_i h_i - sum_E J_ij.
 *   edges_dev [nedges][2] int32 node pairs (i != j, both < n), J_dev [nedges]
 *   int32 interactions (an edge listed twice adds), h_dev [n] int32 biases;
 *   W_dev: n x n int32 output, row stride ld >= n (its first n columns are
 *   overwritten: the call clears them first); offset_dev: int64 [2] = (c,
 *   number of edges skipped because i == j or an index is out of range).
 * Asynchronous on `stream`; the result is exact as long as every W entry fits
 * int32 (|2 h_i| + 2 sum_j |J_ij| < 2^31); load W with dabs_problem_create.
 * Errors: DABS_E_INVALID (null, n < 1, ld < n, nedges < 0).
 */
int dabs_ising_to_qubo(int32_t n, int64_t nedges, const int32_t *edges_dev, const int32_t *J_dev,
                       const int32_t *h_dev, int32_t *W_dev, int64_t ld, int64_t *offset_dev, void *stream);

/*
 * Read-bandwidth probe of one memory level of the current device, for
 * setting the search kernels' achieved bandwidth against a measured peak:
 * a streaming kernel reads with 16-byte loads per lane (the walker's access
 * width), on every compute unit, from
 *   DABS_PROBE_HBM   a 4 GiB buffer, one pass (larger than the Infinity Cache),
 *   DABS_PROBE_MALL  a 128 MiB buffer (fits the 256 MB Infinity Cache),
 *   DABS_PROBE_L2    a 2 MiB buffer (fits each XCD's 4 MB L2, not the 32 KB
 *                    vector caches: the re-reads are shifted every pass so that
 *                    no compute unit re-reads its own chunks),
 *   DABS_PROBE_LDS   64 KB of LDS per workgroup, 256 passes.
 * out_host[3] = (GB/s of the fastest of three timed launches, bytes read per
 * launch, its milliseconds).  Allocates and frees its own buffers and
 * synchronises the device.  Errors: DABS_E_INVALID, DABS_E_NOMEM, DABS_E_HIP.
 */
enum { DABS_PROBE_HBM = 0, DABS_PROBE_MALL = 1, DABS_PROBE_L2 = 2, DABS_PROBE_LDS = 3 };
int dabs_bandwidth_probe(int32_t level, double *out_host);

/*
 * The same Ising front-end into a sparse problem (dabs_problem_create_csr)
 * for models on sparse graphs such as an annealer's hardware graph (Section
 * II-C: 5,627 nodes, 40,279 edges): the QUBO rows hold the edges and the
 * diagonal only.  edges_dev [nedges][2], J_dev [nedges], h_dev [n] int32 as
 * above (repeated edges add; a loop or an index out of range is an error);
 * *offset_host = c.  The rows are assembled on the host (the call
 * synchronises `stream`).
 * Errors: as dabs_problem_create_csr, and DABS_E_INVALID for a bad edge.
 */
int dabs_problem_create_ising(int32_t n, int64_t nedges, const int32_t *edges_dev, const int32_t *J_dev,
                              const int32_t *h_dev, void *stream, dabs_problem **out, int64_t *offset_host);

/*
 * Learned proposal.  Not in the paper: a small network that scores every bit
 * of a pooled vector and two genetic operations that use the scores; the
 * exact search of Section III still evaluates every vector (energies are
 * never approximated) and the adaptive operation choice of Section IV-A
 * decides how often the learned operations are used.
 *
 * Features of bit k of pooled vector X (pool q, rank r, capacity m), float32
 * expressions rounded to bfloat16 (round to nearest even):
 *   f0 = Delta_k(X)/B (Eq. (3), B the problem's Delta bound), f1 = 2x_k - 1,
 *   f2 = W_kk/B, f3 = R_k/B with R_k = |W_kk| + 2 sum_{j != k} |W_kj|,
 *   f4 = 2 c_k/m - 1 (c_k entries of pool q with bit k set), f5 = f1 f4,
 *   f6 = 2 b_k - 1 (b the pool's rank-0 entry), f7 = r/m.
 * Network: z = W3 relu(W2 relu(W1 f + b1) + b2) + b3, 8 -> 64 -> 64 -> 1.
 * Weights and activations are bfloat16 on the matrix cores, accumulation and
 * biases float32; the float32 master parameters (4801) are laid out
 * W1[64][8] | b1[64] | W2[64][64] | b2[64] | W3[64] | b3.
 * Training minimises the mean binary cross-entropy with logits (label 1 = the
 * bit differs from a reference vector, e.g. the best vector a plain search
 * found later) with Adam (beta1 0.9, beta2 0.999, eps 1e-8).
 *   MLP-seed:   target = parent with every bit of positive logit flipped.
 *   MLP-mutate: flip bit k when its per-bit u32 draw (the genetic operations'
 *               stream: Philox counter (round, instance, k/4, 4<<24 | 2),
 *               word k mod 4) is below 2^29 + q_k 2^22,
 *               q_k = clamp(round-half-even(16 z_k), -128, 127).
 */
typedef struct dabs_mlp dabs_mlp;
#define DABS_MLP_PARAMS 4801
/* params_host: nullable float32[4801] initial parameters (zeros if NULL). */
int dabs_mlp_create(const float *params_host, dabs_mlp **out);
int dabs_mlp_destroy(dabs_mlp *m);
/* Copies the float32 master parameters to params_dev[4801]. */
int dabs_mlp_params(const dabs_mlp *m, float *params_dev, void *stream);
/* Features of every entry of npools pools of `capacity` entries:
 * pool_bits_dev [npools][capacity][ceil(n/64)] u64, feat_dev
 * [npools][capacity][n][8] bfloat16 bit patterns.  n <= 4096.  Synchronises
 * the stream. */
int dabs_mlp_pool_features(const dabs_problem *p, const uint64_t *pool_bits_dev, int32_t npools, int32_t capacity,
                           uint16_t *feat_dev, void *stream);
/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * features as dabs_mlp_pool_features, bit for bit, with no allocation and no
 * synchronisation (asynchronous on `stream`).  The per-pool bit counts
 * ([npools][n] int) that the other call allocates per call live here in a
 * static device buffer of DABS_NOALLOC_COUNTS ints (1 MiB) that the library
 * keeps on each GPU it runs on until the process ends; its address is looked
 * up on the first call on a device.  Every count is rewritten before it is
 * read, so nothing carries over between calls, but calls that overlap on one
 * GPU (two streams, or two threads) share the buffer and race: serialise them.
 * The current device must be the problem's.
 * Errors: DABS_E_INVALID (null, bad shape, npools * n > DABS_NOALLOC_COUNTS,
 * another device current), DABS_E_UNSUPPORTED (n > 4096), DABS_E_HIP.
 */
#define DABS_NOALLOC_COUNTS 262144
int dabs_mlp_pool_features_noalloc(const dabs_problem *p, const uint64_t *pool_bits_dev, int32_t npools,
                                   int32_t capacity, uint16_t *feat_dev, void *stream);
/* labels_dev[e][k] = bit k of bits_dev[e] != bit k of ref_dev (u8, count x n).
 * symmetric != 0: against ref or its complement, whichever is nearer in
 * Hamming distance (ties: ref) -- for problems whose energy is invariant under
 * complementing every bit, such as max-cut (Section II-A). */
int dabs_mlp_labels(const dabs_problem *p, const uint64_t *bits_dev, int64_t count, const uint64_t *ref_dev,
                    int32_t symmetric, uint8_t *labels_dev, void *stream);
/* logits_dev[count] float32 of the samples feat_dev[count][8]. */
int dabs_mlp_forward(const dabs_mlp *m, int64_t count, const uint16_t *feat_dev, float *logits_dev, void *stream);
/* Gradient of the mean loss over `count` samples into the network's gradient
 * buffer; optional copies to grad_dev[4801] and loss_dev[1] (float32). */
int dabs_mlp_grad(dabs_mlp *m, int64_t count, const uint16_t *feat_dev, const uint8_t *labels_dev, float *grad_dev,
                  float *loss_dev, void *stream);
/* One Adam step with the gradient buffer (step count kept by the network). */
int dabs_mlp_adam(dabs_mlp *m, float lr, void *stream);
/* dabs_mlp_grad then dabs_mlp_adam. */
int dabs_mlp_train_step(dabs_mlp *m, int64_t count, const uint16_t *feat_dev, const uint8_t *labels_dev, float lr,
                        float *loss_dev, void *stream);
/* One MLP operation (DABS_OP_MLP_SEED / _MUTATE) on `count` parents
 * [count][ceil(n/64)] with their logits [count][n]; parent i uses instance
 * number inst0 + i and the given round in the draw counters. */
int dabs_mlp_apply_op(int32_t op, int32_t n, int32_t count, const uint64_t *parent_dev, const float *logits_dev,
                      uint64_t seed, uint32_t round, uint32_t inst0, uint64_t *out_dev, void *stream);
/* Attach (or detach with NULL) the network whose logits the MLP operations
 * use: every round then scores all pooled vectors before target generation.
 * The network must outlive the solver / batch or be detached first. */
int dabs_solver_set_mlp(dabs_solver *s, const dabs_mlp *m);
int dabs_batched_set_mlp(dabs_batched *b, const dabs_mlp *m);

#ifdef __cplusplus
}
#endif
#endif
