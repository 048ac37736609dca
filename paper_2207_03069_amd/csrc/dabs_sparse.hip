// dabs_sparse.hip -- sparse QUBO problems: CSR load and validation, energies,
// and the search kernels of the sparse walker (dabs_sparse.h) for
// dabs_search / dabs_batch_search and for the batched rounds.
#include <string.h>

#include <algorithm>
#include <vector>

#include "dabs_internal.h"
#include "dabs_sparse.h"

#define HIP_OK(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return dabs_fail(DABS_E_HIP, "%s: %s", #call, hipGetErrorString(e_));      \
    } while (0)

namespace dabs {

// One thread per row: column range and order, off-diagonal weight range,
// symmetry (the mirrored entry found by binary search in its row, with the
// same value), |W_ii| + 2 sum |W_ij| and the count of off-diagonal entries.
// bad: bit 0 asymmetric, bit 1 weight out of range, bit 3 malformed rows.
__global__ __launch_bounds__(256) void k_csr_check(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                   const int32_t *__restrict__ val, int n, int64_t nnz,
                                                   int *__restrict__ bad, long long *__restrict__ rowb,
                                                   int *__restrict__ offcnt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int a = rp[i], b = rp[i + 1];
    if (a < 0 || b < a || (int64_t)b > nnz) {
        atomicOr(bad, 8);
        rowb[i] = 0;
        offcnt[i] = 0;
        return;
    }
    long long acc = 0;
    int prev = -1, off = 0, flag = 0;
    for (int t = a; t < b; ++t) {
        const int j = col[t];
        const long long v = val[t];
        if (j < 0 || j >= n || j <= prev) {
            flag |= 8;
            break;
        }
        prev = j;
        acc += (j == i ? 1 : 2) * (v < 0 ? -v : v);
        if (j == i) continue;
        off++;
        if (v > 32767 || v < -32767) flag |= 2;
        // the entry (j, i)
        int lo = rp[j], hi = rp[j + 1] - 1;
        bool found = false;
        if (lo >= 0 && hi < (int)nnz)
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                const int cm = col[mid];
                if (cm == i) {
                    found = val[mid] == (int)v;
                    break;
                }
                if (cm < i) lo = mid + 1;
                else hi = mid - 1;
            }
        if (!found) flag |= 1;
    }
    if (flag) atomicOr(bad, flag);
    rowb[i] = acc;
    offcnt[i] = off;
}

// The library's rows: off-diagonal entries packed as column | weight << 16,
// the diagonal apart.
__global__ __launch_bounds__(256) void k_csr_pack(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                  const int32_t *__restrict__ val, int n,
                                                  const int32_t *__restrict__ rp2, uint32_t *__restrict__ nz,
                                                  int32_t *__restrict__ diag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int o = rp2[i], d = 0;
    for (int t = rp[i]; t < rp[i + 1]; ++t) {
        const int j = col[t];
        if (j == i) d = val[t];
        else nz[o++] = (uint32_t)j | ((uint32_t)val[t] << 16);
    }
    diag[i] = d;
}

// E(X) = sum_i x_i (W_ii + sum_{j != i} W_ij x_j), one wave per vector, lane
// l taking rows l, l + 64, ...
__global__ __launch_bounds__(256) void k_energy_sparse(const int32_t *__restrict__ rp, const uint32_t *__restrict__ nz,
                                                       const int32_t *__restrict__ diag, int n, int nwords,
                                                       const uint64_t *__restrict__ x, int count,
                                                       int64_t *__restrict__ e) {
    const int wid = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (wid >= count) return;
    const int lane = (int)(threadIdx.x & 63);
    const uint64_t *xv = x + (int64_t)wid * nwords;
    long long acc = 0;
    for (int i = lane; i < n; i += WAVE) {
        if (!((xv[i >> 6] >> (i & 63)) & 1)) continue;
        long long r = diag[i];
        for (int t = rp[i]; t < rp[i + 1]; ++t) {
            const uint32_t w = nz[t];
            const int c = (int)(w & 0xFFFFu);
            if ((xv[c >> 6] >> (c & 63)) & 1) r += (int)w >> 16;
        }
        acc += r;
    }
    acc = wave_sum64(acc);
    if (lane == 0) e[wid] = acc;
}

hipError_t sparse_energy(const dabs_problem *p, const uint64_t *x, int count, int64_t *e, hipStream_t st) {
    hipLaunchKernelGGL(k_energy_sparse, dim3((count + 3) / 4), dim3(256), 0, st, p->rowptr, p->nz, p->diag, p->n,
                       (p->n + 63) / 64, x, count, e);
    return hipGetLastError();
}

// dabs_search / dabs_batch_search on a sparse problem: one wavefront (and
// workgroup) per instance, its keys and bits in dynamic LDS.
__global__ __launch_bounds__(64) void k_sparse_walk(WalkArgs a) {
    extern __shared__ uint32_t smem[];
    const int wid = blockIdx.x;
    SparseWalker w;
    uint64_t *x = a.x + (int64_t)wid * a.nwords;
    w.setup((lds_u32 *)smem, a.diag, a.rowptr, a.nz, a.n, a.slots, a.seed, a.inst0 + (uint32_t)wid, x);
    int f;
    if (!a.batch) {
        if (a.trace) {
            w.trace = a.trace + (int64_t)wid * a.trace_cap;
            w.trace_cap = a.trace_cap;
        }
        w.begin();
        f = w.run_phase(a.rule, a.T, a.tau, a.phase, a.target ? a.target + (int64_t)wid * a.nwords : nullptr,
                        a.greedy_cap);
        if (a.trace)
            for (int q = f + w.lane; q < a.trace_cap; q += WAVE) w.trace[q] = -1;
    } else {
        uint32_t ph = a.phase_arr[wid];
        f = w.batch(a.target + (int64_t)wid * a.nwords, a.algo[wid], a.T, a.Bn, a.tau, ph, a.greedy_cap);
        if (w.lane == 0) a.phase_arr[wid] = ph;
    }
    w.store_bits(w.XW, x);
    w.store_bits(w.BW, a.best + (int64_t)wid * a.nwords);
    if (a.delta) w.store_delta(a.delta + (int64_t)wid * a.n);
    if (w.lane == 0) {
        a.best_e[wid] = w.Eb;
        a.e[wid] = w.E;
        if (a.flips) a.flips[wid] = f;
        if (a.flip_total) atomicAdd((unsigned long long *)a.flip_total, (unsigned long long)f);
    }
}

// The batch searches of a round for the sparse problems of one piece count:
// one wavefront (and workgroup) per (problem, instance) item, as the dense
// item kernel.
__global__ __launch_bounds__(64) void k_sparse_items(ItemsArgs a) {
    extern __shared__ uint32_t smem[];
    const BatchDev &b = a.b;
    if (b.ctr[3]) return;                 // the round is cancelled (latched before the launch)
    const int2 item = a.items[blockIdx.x];
    const int p = __builtin_amdgcn_readfirstlane(item.x), i = __builtin_amdgcn_readfirstlane(item.y);
    ProbDesc *d = b.desc + p;
    const int64_t gi = d->inst0 + i;
    const int64_t wo = d->inst_word0 + (int64_t)i * d->nw;
    SparseWalker w;
    w.setup((lds_u32 *)smem, d->diag, d->rowptr, d->nz, d->n, d->slots, d->g.seed, (uint32_t)i, b.x + wo);
    if (a.ttt && d->target_e != INT64_MIN) {
        w.hit = &d->hit;
        w.target = d->target_e;
        w.t0 = b.ctr[1];
        w.hit_done = false;
    }
    uint32_t ph = b.ph[gi];
    const int f = w.batch(b.target + wo, b.algo[gi], d->g.T, d->g.Bn, d->g.tau, ph, d->g.greedy_cap);
    w.store_bits(w.XW, b.x + wo);
    w.store_bits(w.BW, b.best + wo);
    if (w.lane == 0) {
        b.ph[gi] = ph;
        b.e[gi] = w.E;
        b.best_e[gi] = w.Eb;
        atomicAdd(&b.ctr[0], (unsigned long long)f);
        record_item(a, (int)blockIdx.x, f, b.algo[gi], p);
    }
}

hipError_t launch_sparse_walk(const dabs_problem *p, const WalkArgs &a, hipStream_t st) {
    if (a.count < 1) return hipSuccess;
    const size_t lds = sizeof(uint32_t) * (size_t)sparse_lds_words(p->slots);
    hipLaunchKernelGGL(k_sparse_walk, dim3(a.count), dim3(WAVE), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_sparse_items(int slots, const ItemsArgs &a, hipStream_t st) {
    if (a.nitems < 1) return hipSuccess;
    if (slots < 1 || slots > SPARSE_MAX_SLOTS) return hipErrorInvalidValue;
    const size_t lds = sizeof(uint32_t) * (size_t)sparse_lds_words(slots);
    hipLaunchKernelGGL(k_sparse_items, dim3(a.nitems), dim3(WAVE), lds, st, a);
    return hipGetLastError();
}

}  // namespace dabs

using namespace dabs;

extern "C" {

int dabs_problem_create_csr(const int32_t *row_ptr_dev, const int32_t *col_dev, const int32_t *val_dev, int32_t n,
                            int64_t nnz, void *stream, dabs_problem **out) {
    if (!row_ptr_dev || !out || (nnz > 0 && (!col_dev || !val_dev))) return dabs_fail(DABS_E_INVALID, "null pointer");
    if (n < 1 || nnz < 0 || nnz > 0x7FFFFFFF) return dabs_fail(DABS_E_INVALID, "need n >= 1 and 0 <= nnz < 2^31");
    if (n > max_n(DABS_W_SPARSE))
        return dabs_fail(DABS_E_UNSUPPORTED, "n=%d above %d for sparse problems", n, max_n(DABS_W_SPARSE));
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    std::vector<int32_t> hrp(n + 1);
    HIP_OK(hipMemcpyAsync(hrp.data(), row_ptr_dev, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    if (hrp[0] != 0 || (int64_t)hrp[n] != nnz) return dabs_fail(DABS_E_INVALID, "row_ptr must run from 0 to nnz");
    int *bad = nullptr, *offcnt = nullptr;
    long long *rowb = nullptr;
    int32_t *rp2 = nullptr, *diag = nullptr;
    uint32_t *nzp = nullptr;
    auto release = [&]() {
        (void)hipFree(bad); (void)hipFree(offcnt); (void)hipFree(rowb);
        (void)hipFree(rp2); (void)hipFree(diag); (void)hipFree(nzp);
    };
    if (hipMalloc(&bad, sizeof(int)) != hipSuccess || hipMalloc(&offcnt, sizeof(int) * n) != hipSuccess ||
        hipMalloc(&rowb, sizeof(long long) * n) != hipSuccess) {
        release();
        return dabs_fail(DABS_E_NOMEM, "allocating validation buffers");
    }
    std::vector<int> hoff(n);
    std::vector<long long> hb(n);
    int hbad = 0;
    int status = DABS_OK;
    if (hipMemsetAsync(bad, 0, sizeof(int), st) != hipSuccess) status = DABS_E_HIP;
    if (status == DABS_OK) {
        hipLaunchKernelGGL(k_csr_check, dim3((n + 255) / 256), dim3(256), 0, st, row_ptr_dev, col_dev, val_dev, n, nnz,
                           bad, rowb, offcnt);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(hoff.data(), offcnt, sizeof(int) * n, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(hb.data(), rowb, sizeof(long long) * n, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            status = DABS_E_HIP;
    }
    if (status == DABS_E_HIP) {
        release();
        return dabs_fail(DABS_E_HIP, "validating the CSR rows failed");
    }
    if (hbad & 8) status = dabs_fail(DABS_E_INVALID, "malformed rows (column out of range or not increasing)");
    else if (hbad & 1) status = dabs_fail(DABS_E_NOT_SYMMETRIC, "W is not symmetric");
    else if (hbad & 2) status = dabs_fail(DABS_E_RANGE, "an off-diagonal weight lies outside [-32767, 32767]");
    long long bound = 0;
    for (int i = 0; i < n; ++i) bound = hb[i] > bound ? hb[i] : bound;
    const long long maxb = dabs_max_bound(DABS_W_SPARSE, n);
    if (status == DABS_OK && bound > maxb)
        status = dabs_fail(DABS_E_RANGE, "delta bound %lld above %lld for n = %d", bound, maxb, n);
    if (status != DABS_OK) {
        release();
        return status;
    }
    std::vector<int32_t> h2(n + 1);
    h2[0] = 0;
    for (int i = 0; i < n; ++i) h2[i + 1] = h2[i] + hoff[i];
    const int64_t nnz2 = h2[n];
    if (hipMalloc(&rp2, sizeof(int32_t) * (n + 1)) != hipSuccess || hipMalloc(&diag, sizeof(int32_t) * n) != hipSuccess ||
        hipMalloc(&nzp, sizeof(uint32_t) * (size_t)(nnz2 > 0 ? nnz2 : 1)) != hipSuccess) {
        release();
        return dabs_fail(DABS_E_NOMEM, "allocating the sparse rows");
    }
    if (hipMemcpyAsync(rp2, h2.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, st) != hipSuccess)
        status = DABS_E_HIP;
    if (status == DABS_OK) {
        hipLaunchKernelGGL(k_csr_pack, dim3((n + 255) / 256), dim3(256), 0, st, row_ptr_dev, col_dev, val_dev, n, rp2,
                           nzp, diag);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) status = DABS_E_HIP;
    }
    if (status != DABS_OK) {
        release();
        return dabs_fail(DABS_E_HIP, "packing the sparse rows failed");
    }
    (void)hipFree(bad);
    (void)hipFree(offcnt);
    dabs_problem *p = new dabs_problem;
    memset(p, 0, sizeof(*p));
    p->n = n;
    p->wtype = DABS_W_SPARSE;
    p->ld = 0;
    p->bound = bound;
    p->wmax = (int32_t)(bound > 0x3FFFFFFF ? 0x3FFFFFFF : bound);   // unused by the sparse walker
    p->W = nullptr;
    p->diag = diag;
    p->rowabs = (int64_t *)rowb;
    p->device = dev;
    p->rowptr = rp2;
    p->nz = nzp;
    p->nnz = nnz2;
    p->slots = sparse_slots(n);
    *out = p;
    return DABS_OK;
}

int dabs_problem_create_ising(int32_t n, int64_t nedges, const int32_t *edges_dev, const int32_t *J_dev,
                              const int32_t *h_dev, void *stream, dabs_problem **out, int64_t *offset_host) {
    if (n < 1 || nedges < 0 || !h_dev || !out || (nedges > 0 && (!edges_dev || !J_dev)))
        return dabs_fail(DABS_E_INVALID, "bad Ising arguments");
    if (n > max_n(DABS_W_SPARSE))
        return dabs_fail(DABS_E_UNSUPPORTED, "n=%d above %d for sparse problems", n, max_n(DABS_W_SPARSE));
    hipStream_t st = (hipStream_t)stream;
    std::vector<int32_t> he(2 * (size_t)nedges), hJ((size_t)nedges), hh(n);
    if (nedges > 0) {
        HIP_OK(hipMemcpyAsync(he.data(), edges_dev, sizeof(int32_t) * 2 * nedges, hipMemcpyDeviceToHost, st));
        HIP_OK(hipMemcpyAsync(hJ.data(), J_dev, sizeof(int32_t) * nedges, hipMemcpyDeviceToHost, st));
    }
    HIP_OK(hipMemcpyAsync(hh.data(), h_dev, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    // s_i s_j = 4 x_i x_j - 2 x_i - 2 x_j + 1 and h s_i = 2 h x_i - h (Eq. (1)
    // into Eq. (2), ordered pairs): W_ij = W_ji = 2 J_ij, W_ii = 2 h_i - 2 sum
    // J_ij, c = sum h - sum J; repeated edges add
    std::vector<long long> diag(n, 0);
    std::vector<std::vector<std::pair<int, long long>>> rows(n);
    long long c = 0;
    for (int64_t e = 0; e < nedges; ++e) {
        const int i = he[2 * e], j = he[2 * e + 1];
        if (i == j || i < 0 || j < 0 || i >= n || j >= n)
            return dabs_fail(DABS_E_INVALID, "edge %lld: (%d, %d) is a loop or out of range", (long long)e, i, j);
        const long long v = hJ[e];
        rows[i].push_back({j, 2 * v});
        rows[j].push_back({i, 2 * v});
        diag[i] -= 2 * v;
        diag[j] -= 2 * v;
        c -= v;
    }
    for (int i = 0; i < n; ++i) {
        diag[i] += 2 * (long long)hh[i];
        c += hh[i];
    }
    std::vector<int32_t> rp(n + 1, 0), col, val;
    for (int i = 0; i < n; ++i) {
        auto &r = rows[i];
        r.push_back({i, diag[i]});
        std::sort(r.begin(), r.end());
        for (size_t t = 0; t < r.size();) {
            const int cj = r[t].first;
            long long sum = 0;
            while (t < r.size() && r[t].first == cj) sum += r[t++].second;   // a repeated edge adds
            if (sum > 0x7FFFFFFFll || sum < -0x7FFFFFFFll)
                return dabs_fail(DABS_E_RANGE, "a QUBO weight of row %d does not fit int32", i);
            col.push_back(cj);
            val.push_back((int32_t)sum);
        }
        rp[i + 1] = (int32_t)col.size();
    }
    const int64_t nnz = (int64_t)col.size();
    int32_t *drp = nullptr, *dcol = nullptr, *dval = nullptr;
    if (hipMalloc(&drp, sizeof(int32_t) * (n + 1)) != hipSuccess || hipMalloc(&dcol, sizeof(int32_t) * nnz) != hipSuccess ||
        hipMalloc(&dval, sizeof(int32_t) * nnz) != hipSuccess) {
        (void)hipFree(drp); (void)hipFree(dcol); (void)hipFree(dval);
        return dabs_fail(DABS_E_NOMEM, "allocating the Ising rows");
    }
    int r = DABS_OK;
    if (hipMemcpyAsync(drp, rp.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(dcol, col.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(dval, val.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, st) != hipSuccess)
        r = dabs_fail(DABS_E_HIP, "uploading the Ising rows failed");
    if (r == DABS_OK) r = dabs_problem_create_csr(drp, dcol, dval, n, nnz, stream, out);
    (void)hipStreamSynchronize(st);
    (void)hipFree(drp); (void)hipFree(dcol); (void)hipFree(dval);
    if (r == DABS_OK && offset_host) *offset_host = c;
    return r;
}

}  // extern "C"
