// dabs_capi.hip -- C-ABI of the bulk-search library: problem load and
// validation, energies from scratch, search and batch-search launches.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>

#include "dabs_internal.h"
#include "dabs_device.h"

static thread_local char g_err[512];

int dabs_fail(int status, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return status;
}

#define HIP_OK(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return dabs_fail(DABS_E_HIP, "%s: %s", #call, hipGetErrorString(e_));      \
    } while (0)

namespace dabs {

// largest |W_ij| (i != j) of int32 W: operand range of the 24-bit multiply
constexpr long long I24_MAX = (1 << 23) - 1;

// Symmetry and delta bound of the caller's W: one block per row i; every
// thread compares its W_ij with W_ji and sums |W_ij| (counted twice off the
// diagonal).  bad: bit 0 asymmetric, bit 1 an int16 -32768 off the diagonal
// (the search negates off-diagonal int16 weights in 16 bits), bit 2 an int32
// weight off the diagonal outside the 24-bit multiply's operand range.
// bad[1] receives the largest |W_ij| off the diagonal (clamped to 2^31 - 1).
template <typename WT>
__global__ __launch_bounds__(256) void k_validate(const WT *__restrict__ W, int64_t ld, int n,
                                                  int *__restrict__ bad, long long *__restrict__ rowb) {
    const int i = blockIdx.x;
    long long acc = 0, amax = 0;
    int asym = 0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const long long a = W[(int64_t)i * ld + j], b = W[(int64_t)j * ld + i];
        asym |= a != b;
        if (sizeof(WT) == 2 && j != i && a == -32768) asym |= 2;
        if (sizeof(WT) == 4 && j != i && (a > I24_MAX || a < -I24_MAX)) asym |= 4;
        const long long aa = a < 0 ? -a : a;
        acc += (j == i ? 1 : 2) * aa;
        if (j != i && aa > amax) amax = aa;
    }
    if (amax > 0) atomicMax(&bad[1], (int)(amax > 0x7FFFFFFFll ? 0x7FFFFFFFll : amax));
    __shared__ long long part[256];
    __shared__ int pbad[256];
    part[threadIdx.x] = acc;
    pbad[threadIdx.x] = asym;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            part[threadIdx.x] += part[threadIdx.x + s];
            pbad[threadIdx.x] |= pbad[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        rowb[i] = part[0];
        if (pbad[0]) atomicOr(bad, pbad[0]);
    }
}

// Library layout: rows of length ld (multiple of 512) with a zero diagonal and
// zero padding; the diagonal goes to its own array.
template <typename WT>
__global__ __launch_bounds__(256) void k_pack(const WT *__restrict__ W, int64_t ldin, int n, WT *__restrict__ out,
                                              int64_t ld, int *__restrict__ diag) {
    const int i = blockIdx.y;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < ld; j += (int64_t)gridDim.x * blockDim.x) {
        WT v = 0;
        if (j < n) v = W[(int64_t)i * ldin + j];
        if (j == i) {
            diag[i] = (int)v;
            v = 0;
        }
        out[(int64_t)i * ld + j] = v;
    }
}

// E(X) = sum_i x_i (W_ii + sum_{j != i} W_ij x_j) from scratch, one wave per
// vector; lane l handles columns l, l+64, ...
template <typename WT>
__global__ __launch_bounds__(256) void k_energy(const WT *__restrict__ W, const int *__restrict__ diag, int64_t ld,
                                                int n, int nwords, const uint64_t *__restrict__ x, int count,
                                                int64_t *__restrict__ e) {
    const int wid = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (wid >= count) return;
    const int lane = (int)(threadIdx.x & 63);
    const uint64_t *xv = x + (int64_t)wid * nwords;
    long long acc = 0;
    for (int i = 0; i < n; ++i) {
        if (!((xv[i >> 6] >> (i & 63)) & 1)) continue;
        if (lane == 0) acc += diag[i];
        for (int w = 0; w < nwords; ++w) {
            const int j = w * 64 + lane;
            if (j < n && ((xv[w] >> lane) & 1)) acc += W[(int64_t)i * ld + j];
        }
    }
    for (int m = 32; m > 0; m >>= 1) acc += __shfl_xor(acc, m, 64);
    if (lane == 0) e[wid] = acc;
}

// Ising front-end (Eq. (1) -> Eq. (2)): clear the n x n block, then every
// edge and bias adds its terms with integer atomics (order-free, so exact).
__global__ __launch_bounds__(256) void k_clear_block(int32_t *__restrict__ W, int64_t ld, int n,
                                                     long long *__restrict__ off) {
    const int64_t total = (int64_t)n * n;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x)
        W[(t / n) * ld + t % n] = 0;
    if (blockIdx.x == 0 && threadIdx.x < 2) off[threadIdx.x] = 0;
}

__global__ __launch_bounds__(256) void k_ising_edges(int n, int64_t ne, const int32_t *__restrict__ edges,
                                                     const int32_t *__restrict__ J, int32_t *__restrict__ W,
                                                     int64_t ld, long long *__restrict__ off) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = edges[2 * e], j = edges[2 * e + 1];
        if (i == j || i < 0 || j < 0 || i >= n || j >= n) {
            atomicAdd((unsigned long long *)&off[1], 1ull);
            continue;
        }
        const int v = J[e];
        // s_i s_j = 4 x_i x_j - 2 x_i - 2 x_j + 1: W_ij = W_ji = 2J, W_ii and W_jj lose 2J, c loses J
        atomicAdd(&W[(int64_t)i * ld + j], 2 * v);
        atomicAdd(&W[(int64_t)j * ld + i], 2 * v);
        atomicAdd(&W[(int64_t)i * ld + i], -2 * v);
        atomicAdd(&W[(int64_t)j * ld + j], -2 * v);
        atomicAdd((unsigned long long *)&off[0], (unsigned long long)(-(long long)v));
    }
}

__global__ __launch_bounds__(256) void k_ising_bias(int n, const int32_t *__restrict__ h, int32_t *__restrict__ W,
                                                    int64_t ld, long long *__restrict__ off) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // h_i s_i = 2 h_i x_i - h_i
    atomicAdd(&W[(int64_t)i * ld + i], 2 * h[i]);
    atomicAdd((unsigned long long *)&off[0], (unsigned long long)(long long)h[i]);
}

}  // namespace dabs

using namespace dabs;

extern "C" {

const char *dabs_strerror(int status) {
    switch (status) {
    case DABS_OK: return "ok";
    case DABS_E_INVALID: return "invalid argument";
    case DABS_E_NOT_SYMMETRIC: return "W is not symmetric";
    case DABS_E_RANGE: return "W exceeds the exact device range (delta bound above dabs_max_bound, or a weight out of range)";
    case DABS_E_CANCELLED: return "cancelled by the caller's flag";
    case DABS_E_NOMEM: return "device allocation failed";
    case DABS_E_HIP: return "HIP runtime error";
    case DABS_E_UNSUPPORTED: return "size not supported by this build";
    default: return "unknown status";
    }
}

const char *dabs_last_error(void) { return g_err; }

int32_t dabs_max_n(int32_t wtype) { return dabs::max_n(wtype); }

int64_t dabs_fast_bound(int32_t wtype, int32_t n) {
    if ((wtype != DABS_W_I16 && wtype != DABS_W_I32 && wtype != DABS_W_SPARSE) || n < 1 || n > dabs::max_n(wtype))
        return -1;
    const int slots = wtype == DABS_W_SPARSE ? sparse_slots(n) : walk_slots(wtype, n);
    return ((int64_t)1 << (29 - key_shift(wtype, slots))) - 2;
}

int64_t dabs_max_bound(int32_t wtype, int32_t n) {
    const int64_t fast = dabs_fast_bound(wtype, n);
    if (fast < 0 || wtype == DABS_W_SPARSE) return fast;
    return 0x7FFFFFFFll;                  // dense: every delta an int32 (the wide-delta kernels)
}

int dabs_problem_create(const void *w_dev, int32_t n, int64_t ld, int32_t wtype, void *stream,
                        dabs_problem **out) {
    g_err[0] = 0;
    if (!w_dev || !out) return dabs_fail(DABS_E_INVALID, "null pointer");
    if (n < 1 || ld < n) return dabs_fail(DABS_E_INVALID, "need n >= 1 and ld >= n (n=%d ld=%lld)", n, (long long)ld);
    if (wtype != DABS_W_I16 && wtype != DABS_W_I32) return dabs_fail(DABS_E_INVALID, "bad wtype %d", wtype);
    if (n > dabs::max_n(wtype)) return dabs_fail(DABS_E_UNSUPPORTED, "n=%d above %d", n, dabs::max_n(wtype));
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    const size_t es = wtype == DABS_W_I16 ? 2 : 4;
    const int64_t lds = ((int64_t)n + 511) / 512 * 512;
    // the search kernels run with a power-of-two slot count; pad rows to it
    const int64_t span = wtype == DABS_W_I16 ? 512 : 256;
    int64_t slots = ((int64_t)n + span - 1) / span, p2 = 1;
    while (p2 < slots) p2 <<= 1;
    const int64_t ldp = p2 * span > lds ? p2 * span : lds;
    int *bad = nullptr;
    long long *rowb = nullptr;
    void *Wp = nullptr;
    int *diag = nullptr;
    if (hipMalloc(&bad, 2 * sizeof(int)) != hipSuccess || hipMalloc(&rowb, sizeof(long long) * n) != hipSuccess ||
        hipMalloc(&Wp, es * (size_t)n * (size_t)ldp) != hipSuccess || hipMalloc(&diag, sizeof(int) * n) != hipSuccess) {
        (void)hipFree(bad); (void)hipFree(rowb); (void)hipFree(Wp); (void)hipFree(diag);
        return dabs_fail(DABS_E_NOMEM, "allocating %zu bytes for W", es * (size_t)n * (size_t)ldp);
    }
    int status = DABS_OK;
    long long *hb = (long long *)malloc(sizeof(long long) * n);
    int hbad2[2] = {0, 0};
    int &hbad = hbad2[0];
    do {
        if (hipMemsetAsync(bad, 0, 2 * sizeof(int), st) != hipSuccess) { status = DABS_E_HIP; break; }
        if (wtype == DABS_W_I16)
            hipLaunchKernelGGL(k_validate<int16_t>, dim3(n), dim3(256), 0, st, (const int16_t *)w_dev, ld, n, bad, rowb);
        else
            hipLaunchKernelGGL(k_validate<int32_t>, dim3(n), dim3(256), 0, st, (const int32_t *)w_dev, ld, n, bad, rowb);
        if (hipGetLastError() != hipSuccess) { status = DABS_E_HIP; break; }
        if (hipMemcpyAsync(hbad2, bad, 2 * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(hb, rowb, sizeof(long long) * n, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) { status = DABS_E_HIP; break; }
    } while (0);
    long long bound = 0;
    for (int i = 0; i < n && status == DABS_OK; ++i) bound = hb[i] > bound ? hb[i] : bound;
    free(hb);
    if (status == DABS_OK && (hbad & 1)) status = dabs_fail(DABS_E_NOT_SYMMETRIC, "W is not symmetric");
    const long long maxb = dabs_max_bound(wtype, n);
    if (status == DABS_OK && bound > maxb)
        status = dabs_fail(DABS_E_RANGE, "delta bound %lld above %lld for n = %d", bound, maxb, n);
    // the packed-key kernels need B within their key words and weights their
    // update can negate (int16) or multiply (int32, 24 bits); the wide-delta
    // kernels take every other W
    const bool packed_ok = bound <= dabs_fast_bound(wtype, n) && !(hbad & 6);
    if (status == DABS_OK) {
        const int gx = (int)((ldp + 255) / 256);
        if (wtype == DABS_W_I16)
            hipLaunchKernelGGL(k_pack<int16_t>, dim3(gx, n), dim3(256), 0, st, (const int16_t *)w_dev, ld, n,
                               (int16_t *)Wp, ldp, diag);
        else
            hipLaunchKernelGGL(k_pack<int32_t>, dim3(gx, n), dim3(256), 0, st, (const int32_t *)w_dev, ld, n,
                               (int32_t *)Wp, ldp, diag);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
            status = dabs_fail(DABS_E_HIP, "packing W failed");
    } else if (status == DABS_E_HIP) {
        dabs_fail(DABS_E_HIP, "validating W failed");
    }
    (void)hipFree(bad);
    if (status != DABS_OK) {
        (void)hipFree(rowb);
        (void)hipFree(Wp);
        (void)hipFree(diag);
        return status;
    }
    dabs_problem *p = new dabs_problem;
    p->n = n;
    p->wtype = wtype;
    p->ld = ldp;
    p->bound = bound;
    p->wmax = hbad2[1];
    p->W = Wp;
    p->diag = diag;
    p->rowabs = (int64_t *)rowb;
    p->device = dev;
    p->rowptr = nullptr;
    p->nz = nullptr;
    p->nnz = 0;
    p->slots = walk_slots(wtype, n);
    p->packed_ok = packed_ok ? 1 : 0;
    p->wide = packed_ok ? 0 : 1;
    *out = p;
    return DABS_OK;
}

int32_t dabs_problem_wide(const dabs_problem *p) {
    if (!p) return dabs_fail(DABS_E_INVALID, "null problem");
    return p->wide;
}

int dabs_problem_set_wide(dabs_problem *p, int32_t wide) {
    if (!p) return dabs_fail(DABS_E_INVALID, "null problem");
    if (wide != 0 && wide != 1) return dabs_fail(DABS_E_INVALID, "wide must be 0 or 1");
    if (p->wtype == DABS_W_SPARSE) return dabs_fail(DABS_E_UNSUPPORTED, "a sparse problem has no wide-delta form");
    if (!wide && !p->packed_ok)
        return dabs_fail(DABS_E_RANGE, "W does not fit the packed key words (delta bound %lld above %lld, or weights "
                         "out of the packed update's range)", (long long)p->bound,
                         (long long)dabs_fast_bound(p->wtype, p->n));
    p->wide = wide;
    return DABS_OK;
}

int dabs_problem_destroy(dabs_problem *p) {
    if (!p) return DABS_OK;
    (void)hipFree(p->W);
    (void)hipFree(p->diag);
    (void)hipFree(p->rowabs);
    (void)hipFree(p->rowptr);
    (void)hipFree(p->nz);
    delete p;
    return DABS_OK;
}

int dabs_problem_info(const dabs_problem *p, int32_t *n, int32_t *wtype, int64_t *bound) {
    if (!p) return dabs_fail(DABS_E_INVALID, "null problem");
    if (n) *n = p->n;
    if (wtype) *wtype = p->wtype;
    if (bound) *bound = p->bound;
    return DABS_OK;
}

int dabs_energy(const dabs_problem *p, const uint64_t *x_dev, int32_t count, int64_t *e_dev, void *stream) {
    if (!p || (!x_dev && count > 0) || (!e_dev && count > 0) || count < 0)
        return dabs_fail(DABS_E_INVALID, "bad energy arguments");
    if (count == 0) return DABS_OK;
    hipStream_t st = (hipStream_t)stream;
    if (p->wtype == DABS_W_SPARSE) {
        HIP_OK(sparse_energy(p, x_dev, count, e_dev, st));
        return DABS_OK;
    }
    const int nw = (p->n + 63) / 64;
    const int blocks = (count + 3) / 4;
    if (p->wtype == DABS_W_I16)
        hipLaunchKernelGGL(k_energy<int16_t>, dim3(blocks), dim3(256), 0, st, (const int16_t *)p->W, p->diag, p->ld,
                           p->n, nw, x_dev, count, e_dev);
    else
        hipLaunchKernelGGL(k_energy<int32_t>, dim3(blocks), dim3(256), 0, st, (const int32_t *)p->W, p->diag, p->ld,
                           p->n, nw, x_dev, count, e_dev);
    HIP_OK(hipGetLastError());
    return DABS_OK;
}

int dabs_ising_to_qubo(int32_t n, int64_t nedges, const int32_t *edges_dev, const int32_t *J_dev,
                       const int32_t *h_dev, int32_t *W_dev, int64_t ld, int64_t *offset_dev, void *stream) {
    if (n < 1 || ld < n || nedges < 0) return dabs_fail(DABS_E_INVALID, "need n >= 1, ld >= n, nedges >= 0");
    if (!h_dev || !W_dev || !offset_dev || (nedges > 0 && (!edges_dev || !J_dev)))
        return dabs_fail(DABS_E_INVALID, "null pointer");
    hipStream_t st = (hipStream_t)stream;
    long long *off = (long long *)offset_dev;
    const int64_t cells = (int64_t)n * n;
    const unsigned cb = (unsigned)std::min<int64_t>((cells + 255) / 256, 8192);
    hipLaunchKernelGGL(k_clear_block, dim3(cb), dim3(256), 0, st, W_dev, ld, n, off);
    HIP_OK(hipGetLastError());
    if (nedges > 0) {
        const unsigned eb = (unsigned)std::min<int64_t>((nedges + 255) / 256, 8192);
        hipLaunchKernelGGL(k_ising_edges, dim3(eb), dim3(256), 0, st, n, nedges, edges_dev, J_dev, W_dev, ld, off);
        HIP_OK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_ising_bias, dim3((n + 255) / 256), dim3(256), 0, st, n, h_dev, W_dev, ld, off);
    HIP_OK(hipGetLastError());
    return DABS_OK;
}

static bool rule_ok(int r) { return r >= DABS_GREEDY && r <= DABS_TABU_GREEDY; }

int dabs_search(const dabs_problem *p, const dabs_search_params *sp, int32_t count, uint64_t *x_dev,
                const uint64_t *target_dev, uint64_t *best_dev, int64_t *best_e_dev, int64_t *e_dev,
                int32_t *delta_dev, int32_t *trace_dev, int32_t trace_cap, int32_t *flips_dev, void *stream) {
    if (!p || !sp) return dabs_fail(DABS_E_INVALID, "null problem or params");
    if (count < 0) return dabs_fail(DABS_E_INVALID, "count < 0");
    if (count == 0) return DABS_OK;
    if (!x_dev || !best_dev || !best_e_dev || !e_dev) return dabs_fail(DABS_E_INVALID, "null output");
    if (!rule_ok(sp->rule)) return dabs_fail(DABS_E_INVALID, "bad rule %d", sp->rule);
    if (sp->rule == DABS_STRAIGHT && !target_dev) return dabs_fail(DABS_E_INVALID, "Straight needs targets");
    const bool fixed = sp->rule != DABS_GREEDY && sp->rule != DABS_STRAIGHT && sp->rule != DABS_TWONEIGHBOR;
    if (fixed && sp->T < 1) return dabs_fail(DABS_E_INVALID, "T must be >= 1");
    if (sp->tau < 0 || sp->tau > TAU_MAX) return dabs_fail(DABS_E_INVALID, "tau must be in [0, %d]", TAU_MAX);
    if (trace_dev && trace_cap < 1) return dabs_fail(DABS_E_INVALID, "trace_cap must be >= 1");
    WalkArgs a;
    memset(&a, 0, sizeof(a));
    a.W = p->W; a.rowptr = p->rowptr; a.nz = p->nz; a.slots = p->slots; a.diag = p->diag; a.ld = p->ld; a.n = p->n; a.nwords = (p->n + 63) / 64; a.count = count; a.wmax2 = p->wide ? 0 : 2 * p->wmax;
    a.batch = 0; a.rule = sp->rule; a.T = sp->T; a.tau = sp->tau; a.greedy_cap = sp->greedy_cap;
    a.seed = sp->seed; a.phase = sp->phase; a.inst0 = sp->inst0;
    a.x = x_dev; a.target = target_dev; a.best = best_dev; a.best_e = best_e_dev; a.e = e_dev;
    a.delta = delta_dev; a.trace = trace_dev; a.trace_cap = trace_cap; a.flips = flips_dev;
    HIP_OK(launch_walk(p, a, (hipStream_t)stream));
    return DABS_OK;
}

int dabs_batch_search(const dabs_problem *p, const dabs_batch_params *bp, int32_t count, uint64_t *x_dev,
                      const uint64_t *target_dev, const int32_t *algo_dev, uint32_t *phase_dev, uint64_t *best_dev,
                      int64_t *best_e_dev, int64_t *e_dev, int32_t *flips_dev, void *stream) {
    if (!p || !bp) return dabs_fail(DABS_E_INVALID, "null problem or params");
    if (count < 0) return dabs_fail(DABS_E_INVALID, "count < 0");
    if (count == 0) return DABS_OK;
    if (!x_dev || !target_dev || !algo_dev || !phase_dev || !best_dev || !best_e_dev || !e_dev)
        return dabs_fail(DABS_E_INVALID, "null pointer");
    if (bp->T < 1) return dabs_fail(DABS_E_INVALID, "T must be >= 1");
    if (bp->tau < 0 || bp->tau > TAU_MAX) return dabs_fail(DABS_E_INVALID, "tau must be in [0, %d]", TAU_MAX);
    WalkArgs a;
    memset(&a, 0, sizeof(a));
    a.W = p->W; a.rowptr = p->rowptr; a.nz = p->nz; a.slots = p->slots; a.diag = p->diag; a.ld = p->ld; a.n = p->n; a.nwords = (p->n + 63) / 64; a.count = count; a.wmax2 = p->wide ? 0 : 2 * p->wmax;
    a.batch = 1; a.T = bp->T; a.Bn = bp->Bn; a.tau = bp->tau; a.greedy_cap = bp->greedy_cap;
    a.seed = bp->seed; a.inst0 = bp->inst0;
    a.algo = algo_dev; a.phase_arr = phase_dev;
    a.x = x_dev; a.target = target_dev; a.best = best_dev; a.best_e = best_e_dev; a.e = e_dev; a.flips = flips_dev;
    HIP_OK(launch_walk(p, a, (hipStream_t)stream));
    return DABS_OK;
}

}  // extern "C"
