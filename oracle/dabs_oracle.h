/*
 * dabs_oracle.h -- CPU oracle of the Diverse Adaptive Bulk Search hot path.
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product library.
 *
 * Conventions: W is an n x n row-major int32 matrix, symmetric; vectors are
 * one byte (0 or 1) per bit; energies and deltas are int64.
 */
#ifndef DABS_ORACLE_H
#define DABS_ORACLE_H
#include <stdint.h>

/* Search rules (Section III-A) and the tabu-greedy reading of R12. */
enum {
    ORC_GREEDY = 0, ORC_STRAIGHT = 1, ORC_MAXMIN = 2, ORC_CYCLICMIN = 3,
    ORC_RANDOMMIN = 4, ORC_POSITIVEMIN = 5, ORC_TWONEIGHBOR = 6, ORC_TABU_GREEDY = 7
};

/* Genetic operations (Section IV-A, IV-B). */
enum {
    ORC_OP_RANDOM = 0, ORC_OP_BEST = 1, ORC_OP_MUTATION = 2, ORC_OP_CROSSOVER = 3,
    ORC_OP_XROSSOVER = 4, ORC_OP_ZERO = 5, ORC_OP_ONE = 6, ORC_OP_INTERVALZERO = 7,
    ORC_OP_MLP_SEED = 8, ORC_OP_MLP_MUTATE = 9   /* learned operations (R22) */
};

/* flags of orc_ga_params */
enum { ORC_GA_RESTART = 2 };   /* restart the pools when they have merged (R24) */

typedef struct {
    int32_t n_algos;
    int32_t algos[8];        /* enabled main search algorithms (rule ids) */
    int32_t n_ops;
    int32_t ops[16];         /* enabled genetic operations */
    uint32_t p_explore;      /* u32 threshold of the uniform choice (5% = 214748365) */
    uint32_t p_mutation;     /* per-bit u32 thresholds */
    uint32_t p_zero;
    uint32_t p_one;
    int32_t crossover_kind;  /* 0 uniform, 1 two-point */
    int32_t capacity;        /* pool capacity m */
    int32_t npools;          /* pools in the ring */
    int32_t tau;             /* tabu tenure */
    int64_t T;               /* main-phase flips (s n) */
    int64_t Bn;              /* batch flips (b n) */
    int64_t greedy_cap;      /* bound on one Greedy phase */
    uint64_t seed;           /* key of the counter-based generator */
    uint32_t flags;          /* ORC_GA_RESTART */
    int32_t merge_hamming;   /* restart: merged when every entry is within this distance of the best */
} orc_ga_params;

/* Scores of every pooled bit at the start of round `round`:
 * pool_bits [npools][cap][n] -> logits [npools][cap][n]. */
typedef void (*orc_score_fn)(void *ctx, int32_t round, const uint8_t *pool_bits, float *logits);

void orc_philox(const uint32_t ctr[4], uint64_t seed, uint32_t out[4]);
int64_t orc_energy(const int32_t *W, int32_t n, const uint8_t *x);
void orc_delta_scratch(const int32_t *W, int32_t n, const uint8_t *x, int64_t *delta);
void orc_delta_closed(const int32_t *W, int32_t n, const uint8_t *x, int64_t *delta);
int64_t orc_delta_bound(const int32_t *W, int32_t n);
int32_t orc_is_symmetric(const int32_t *W, int32_t n);
uint32_t orc_rank_index(uint32_t u, uint32_t m);

int64_t orc_search(const int32_t *W, int32_t n, int32_t rule, int64_t T, int32_t tau,
                   uint64_t seed, uint32_t inst, uint32_t ph, int64_t greedy_cap,
                   uint8_t *x, const uint8_t *target, uint8_t *best, int64_t *ebest,
                   int64_t *e, int64_t *delta, int32_t *trace, int64_t trace_cap, int32_t verify);

int64_t orc_batch_search(const int32_t *W, int32_t n, int32_t rule, int64_t T, int64_t Bn,
                         int32_t tau, uint64_t seed, uint32_t inst, uint32_t *ph, int64_t greedy_cap,
                         uint8_t *x, const uint8_t *target, uint8_t *best, int64_t *ebest,
                         int64_t *e, int64_t *delta, int32_t *trace, int64_t trace_cap,
                         int64_t *phase_flips, int32_t phase_cap, int32_t *nphases, int32_t verify);

int64_t orc_solve(const int32_t *W, int32_t n, const orc_ga_params *g, int32_t instances,
                  int32_t rounds, uint8_t *pool_bits, int64_t *pool_e, int32_t *pool_algo,
                  int32_t *pool_op, uint8_t *x_out, int64_t *e_out, uint32_t *ph_out,
                  int32_t *inserts, uint8_t *targets_out, int64_t *packets_out, int32_t verify);

int64_t orc_solve_ex(const int32_t *W, int32_t n, const orc_ga_params *g, int32_t instances,
                     int32_t rounds, uint8_t *pool_bits, int64_t *pool_e, int32_t *pool_algo,
                     int32_t *pool_op, uint8_t *x_out, int64_t *e_out, uint32_t *ph_out,
                     int32_t *inserts, uint8_t *targets_out, int64_t *packets_out, int32_t verify,
                     orc_score_fn score, void *score_ctx, uint8_t *best_bits, int64_t *best_e,
                     int32_t *restarts_out, int64_t *round_best, int64_t *stats);

/* layout of orc_solve_ex's stats: uses of operations 0..15, of algorithms
 * 0..7, pool entries made by each, then the record's operation and algorithm */
enum { ORC_STAT_USE_OP = 0, ORC_STAT_USE_ALGO = 16, ORC_STAT_INS_OP = 24, ORC_STAT_INS_ALGO = 40,
       ORC_STAT_REC_OP = 48, ORC_STAT_REC_ALGO = 49, ORC_STATS = 50 };

void orc_target_from_pools(int32_t n, const orc_ga_params *g, uint8_t *pool_bits, int64_t *pool_e,
                           int32_t *pool_algo, int32_t *pool_op, const float *logits, uint32_t round,
                           uint32_t inst, uint8_t *target, int32_t *algo, int32_t *op);

int32_t orc_randmin_q(int64_t t, int64_t T, int32_t n);

int32_t orc_first_target(int32_t n, const orc_ga_params *g, uint32_t inst, uint8_t *target,
                         int32_t *algo, int32_t *op);

void orc_all_energies(const int32_t *W, int32_t n, int64_t *out);
int64_t orc_bruteforce(const int32_t *W, int32_t n, uint8_t *argmin);

#endif
