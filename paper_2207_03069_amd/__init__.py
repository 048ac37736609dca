"""Python binding of libdabs.so, the MI355X bulk-search library.

Argument marshalling only: every function here has the name of a C-ABI call
in ``include/dabs.h``, takes torch tensors (device memory) and forwards their
data pointers and the current HIP stream.  All work runs in the library's HIP
kernels; there is no fallback path.  If ``libdabs.so`` has not been built the
first call raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdabs.so")

DABS_OK, DABS_E_INVALID, DABS_E_NOT_SYMMETRIC, DABS_E_RANGE, DABS_E_NOMEM, DABS_E_HIP, DABS_E_UNSUPPORTED, \
    DABS_E_CANCELLED = 0, -1, -2, -3, -4, -5, -6, -7
DABS_W_I16, DABS_W_I32, DABS_W_SPARSE = 0, 1, 2
(DABS_GREEDY, DABS_STRAIGHT, DABS_MAXMIN, DABS_CYCLICMIN, DABS_RANDOMMIN, DABS_POSITIVEMIN,
 DABS_TWONEIGHBOR, DABS_TABU_GREEDY) = range(8)
(DABS_OP_RANDOM, DABS_OP_BEST, DABS_OP_MUTATION, DABS_OP_CROSSOVER, DABS_OP_XROSSOVER, DABS_OP_ZERO,
 DABS_OP_ONE, DABS_OP_INTERVALZERO, DABS_OP_MLP_SEED, DABS_OP_MLP_MUTATE) = range(10)
DABS_MLP_PARAMS = 4801
DABS_NOALLOC_COUNTS = 262144
MAIN_ALGOS = (DABS_MAXMIN, DABS_CYCLICMIN, DABS_RANDOMMIN, DABS_POSITIVEMIN, DABS_TWONEIGHBOR)


class DabsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s (status %d)" % (msg, status))
        self.status = status


class dabs_search_params(C.Structure):
    _fields_ = [("rule", C.c_int32), ("T", C.c_int32), ("tau", C.c_int32), ("greedy_cap", C.c_int32),
                ("seed", C.c_uint64), ("phase", C.c_uint32), ("inst0", C.c_uint32)]


class dabs_batch_params(C.Structure):
    _fields_ = [("T", C.c_int32), ("Bn", C.c_int32), ("tau", C.c_int32), ("greedy_cap", C.c_int32),
                ("seed", C.c_uint64), ("inst0", C.c_uint32), ("reserved", C.c_uint32)]


class dabs_ga_params(C.Structure):
    _fields_ = [("n_algos", C.c_int32), ("algos", C.c_int32 * 8), ("n_ops", C.c_int32), ("ops", C.c_int32 * 16),
                ("p_explore", C.c_uint32), ("p_mutation", C.c_uint32), ("p_zero", C.c_uint32),
                ("p_one", C.c_uint32), ("crossover_kind", C.c_int32), ("capacity", C.c_int32),
                ("npools", C.c_int32), ("tau", C.c_int32), ("T", C.c_int32), ("Bn", C.c_int32),
                ("greedy_cap", C.c_int32), ("flags", C.c_uint32), ("merge_hamming", C.c_int32),
                ("seed", C.c_uint64)]


DABS_SOLVER_TIME_WALK = 1
DABS_GA_RESTART = 2
DABS_WALK_VARIANTS = 3


# every function the header declares: name -> (argtypes, restype)
_P = C.c_void_p
_SIGS = {
    "dabs_strerror": ([C.c_int], C.c_char_p),
    "dabs_last_error": ([], C.c_char_p),
    "dabs_max_n": ([C.c_int32], C.c_int32),
    "dabs_max_bound": ([C.c_int32, C.c_int32], C.c_int64),
    "dabs_fast_bound": ([C.c_int32, C.c_int32], C.c_int64),
    "dabs_problem_wide": ([_P], C.c_int32),
    "dabs_problem_set_wide": ([_P, C.c_int32], C.c_int),
    "dabs_bandwidth_probe": ([C.c_int32, C.POINTER(C.c_double)], C.c_int),
    "dabs_ising_to_qubo": ([C.c_int32, C.c_int64, _P, _P, _P, _P, C.c_int64, _P, _P], C.c_int),
    "dabs_solver_record": ([_P, _P, _P, _P], C.c_int),
    "dabs_solver_stats": ([_P, _P, _P], C.c_int),
    "dabs_batched_stats": ([_P, C.c_int32, _P, _P], C.c_int),
    "dabs_solver_set_cancel": ([_P, _P], C.c_int),
    "dabs_batched_record": ([_P, C.c_int32, _P, _P, _P], C.c_int),
    "dabs_batched_set_cancel": ([_P, _P], C.c_int),
    "dabs_problem_create": ([_P, C.c_int32, C.c_int64, C.c_int32, _P, C.POINTER(_P)], C.c_int),
    "dabs_problem_destroy": ([_P], C.c_int),
    "dabs_problem_create_csr": ([_P, _P, _P, C.c_int32, C.c_int64, _P, C.POINTER(_P)], C.c_int),
    "dabs_problem_create_ising": ([C.c_int32, C.c_int64, _P, _P, _P, _P, C.POINTER(_P), C.POINTER(C.c_int64)],
                                  C.c_int),
    "dabs_problem_info": ([_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int64)], C.c_int),
    "dabs_energy": ([_P, _P, C.c_int32, _P, _P], C.c_int),
    "dabs_search": ([_P, C.POINTER(dabs_search_params), C.c_int32, _P, _P, _P, _P, _P, _P, _P, C.c_int32, _P, _P],
                    C.c_int),
    "dabs_batch_search": ([_P, C.POINTER(dabs_batch_params), C.c_int32, _P, _P, _P, _P, _P, _P, _P, _P, _P],
                          C.c_int),
    "dabs_solver_create": ([_P, C.POINTER(dabs_ga_params), C.c_int32, _P, C.POINTER(_P)], C.c_int),
    "dabs_solver_destroy": ([_P], C.c_int),
    "dabs_solver_run": ([_P, C.c_int32, _P, _P], C.c_int),
    "dabs_solver_pools": ([_P, _P, _P, _P, _P, _P], C.c_int),
    "dabs_solver_state": ([_P, _P, _P, _P, _P, _P], C.c_int),
    "dabs_solver_progress": ([_P, _P, _P], C.c_int),
    "dabs_solver_timing": ([_P, C.POINTER(C.c_double), C.c_int32], C.c_int),
    "dabs_solver_trace_items": ([_P, _P, C.c_int64, C.POINTER(C.c_int64)], C.c_int),
    "dabs_batched_trace_items": ([_P, _P, C.c_int64, C.POINTER(C.c_int64)], C.c_int),
    "dabs_batched_create": ([_P, C.c_int32, _P, _P, _P, C.POINTER(_P)], C.c_int),
    "dabs_batched_destroy": ([_P], C.c_int),
    "dabs_batched_run": ([_P, C.c_int32, _P, C.c_int32, _P], C.c_int),
    "dabs_batched_progress": ([_P, _P, _P], C.c_int),
    "dabs_batched_pools": ([_P, C.c_int32, _P, _P, _P, _P, _P], C.c_int),
    "dabs_batched_state": ([_P, C.c_int32, _P, _P, _P, _P], C.c_int),
    "dabs_batched_flips": ([_P, _P, _P], C.c_int),
    "dabs_batched_timing": ([_P, C.POINTER(C.c_double), C.c_int32], C.c_int),
    "dabs_mlp_create": ([_P, C.POINTER(_P)], C.c_int),
    "dabs_mlp_destroy": ([_P], C.c_int),
    "dabs_mlp_params": ([_P, _P, _P], C.c_int),
    "dabs_mlp_pool_features": ([_P, _P, C.c_int32, C.c_int32, _P, _P], C.c_int),
    "dabs_mlp_pool_features_noalloc": ([_P, _P, C.c_int32, C.c_int32, _P, _P], C.c_int),
    "dabs_mlp_labels": ([_P, _P, C.c_int64, _P, C.c_int32, _P, _P], C.c_int),
    "dabs_mlp_forward": ([_P, C.c_int64, _P, _P, _P], C.c_int),
    "dabs_mlp_grad": ([_P, C.c_int64, _P, _P, _P, _P, _P], C.c_int),
    "dabs_mlp_adam": ([_P, C.c_float, _P], C.c_int),
    "dabs_mlp_train_step": ([_P, C.c_int64, _P, _P, C.c_float, _P, _P], C.c_int),
    "dabs_mlp_apply_op": ([C.c_int32, C.c_int32, C.c_int32, _P, _P, C.c_uint64, C.c_uint32, C.c_uint32, _P, _P],
                          C.c_int),
    "dabs_solver_set_mlp": ([_P, _P], C.c_int),
    "dabs_batched_autotune": ([_P, _P, _P, _P], C.c_int),
    "dabs_solver_autotune": ([_P, _P, _P, _P], C.c_int),
    "dabs_batched_classes": ([_P, _P, C.c_int32], C.c_int),
    "dabs_batched_set_variant": ([_P, C.c_int32, C.c_int32], C.c_int),
    "dabs_batched_checkpoint": ([_P, _P, _P, _P], C.c_int),
    "dabs_batched_restore": ([_P, _P, _P], C.c_int),
    "dabs_solver_checkpoint": ([_P, _P, _P, _P], C.c_int),
    "dabs_solver_restore": ([_P, _P, _P], C.c_int),
    "dabs_batched_set_mlp": ([_P, _P], C.c_int),
}

_lib = None


def lib():
    """The loaded library; raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libdabs.so is not built (run __graft_entry__.build() or "
                               "python paper_2207_03069_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            if hasattr(L, name):
                f = getattr(L, name)
                f.argtypes = args
                f.restype = res
        _lib = L
    return _lib


def _check(status: int):
    if status != DABS_OK:
        msg = lib().dabs_last_error().decode(errors="replace") or lib().dabs_strerror(status).decode()
        raise DabsError(status, msg)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def dabs_strerror(status: int) -> str:
    return lib().dabs_strerror(status).decode()


def dabs_last_error() -> str:
    return lib().dabs_last_error().decode()


def dabs_max_n(wtype: int) -> int:
    return int(lib().dabs_max_n(wtype))


DABS_PROBE_HBM, DABS_PROBE_MALL, DABS_PROBE_L2, DABS_PROBE_LDS = range(4)


def dabs_bandwidth_probe(level: int):
    """(GB/s, bytes per launch, ms per launch) of the read probe of a level."""
    out = (C.c_double * 3)()
    _check(lib().dabs_bandwidth_probe(level, out))
    return out[0], out[1], out[2]


def dabs_max_bound(wtype: int, n: int) -> int:
    return int(lib().dabs_max_bound(wtype, n))


def dabs_fast_bound(wtype: int, n: int) -> int:
    return int(lib().dabs_fast_bound(wtype, n))


def _host_ptr(t):
    if t is None:
        return None
    if t.is_cuda or not t.is_pinned() or not t.is_contiguous():
        raise ValueError("the flag must be a contiguous pinned host tensor")
    return C.c_void_p(t.data_ptr())


def dabs_ising_to_qubo(n: int, edges, J, h, W, offset, stream=None):
    """edges [E][2] int32, J [E] int32, h [n] int32 (device); W [n][>=n] int32
    output (row stride W.stride(0)); offset [2] int64 output."""
    ne = 0 if edges is None else edges.shape[0]
    _check(lib().dabs_ising_to_qubo(n, ne, _ptr(edges) if ne else None, _ptr(J) if ne else None, _ptr(h),
                                    C.c_void_p(W.data_ptr()), W.stride(0), _ptr(offset), _stream(stream)))


class Problem:
    """Handle of a loaded QUBO matrix (library-owned)."""

    def __init__(self, handle, n, wtype, bound):
        self.handle, self.n, self.wtype, self.bound = handle, n, wtype, bound
        self.nwords = (n + 63) // 64

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _lib is not None:
            _lib.dabs_problem_destroy(h)


def dabs_problem_create(W, stream=None) -> Problem:
    """W: square int16 or int32 CUDA tensor (row stride W.stride(0))."""
    import torch
    if W.dim() != 2 or W.shape[0] != W.shape[1] or W.stride(1) != 1:
        raise ValueError("W must be a square row-major matrix")
    wtype = {torch.int16: DABS_W_I16, torch.int32: DABS_W_I32}.get(W.dtype)
    if wtype is None:
        raise ValueError("W must be int16 or int32")
    h = C.c_void_p()
    _check(lib().dabs_problem_create(_ptr(W), W.shape[0], W.stride(0), wtype, _stream(stream), C.byref(h)))
    return _problem(h)


def _problem(h) -> Problem:
    n, wt, b = C.c_int32(), C.c_int32(), C.c_int64()
    _check(lib().dabs_problem_info(h, C.byref(n), C.byref(wt), C.byref(b)))
    return Problem(h, n.value, wt.value, b.value)


def dabs_problem_create_csr(row_ptr, col, val, n: int, stream=None) -> Problem:
    """A sparse problem from CSR rows (int32 CUDA tensors, the full symmetric
    matrix with its diagonal entries)."""
    h = C.c_void_p()
    nnz = int(col.shape[0])
    _check(lib().dabs_problem_create_csr(_ptr(row_ptr), _ptr(col) if nnz else None, _ptr(val) if nnz else None,
                                         n, nnz, _stream(stream), C.byref(h)))
    return _problem(h)


def dabs_problem_create_ising(n: int, edges, J, h, stream=None):
    """(sparse problem, c) for the Ising model (edges [E][2], J [E], h [n]
    int32 CUDA tensors): E(X) = H(S) + c."""
    hd = C.c_void_p()
    off = C.c_int64()
    ne = 0 if edges is None else int(edges.shape[0])
    _check(lib().dabs_problem_create_ising(n, ne, _ptr(edges) if ne else None, _ptr(J) if ne else None, _ptr(h),
                                           _stream(stream), C.byref(hd), C.byref(off)))
    return _problem(hd), int(off.value)


def dabs_problem_destroy(p: Problem):
    h, p.handle = p.handle, None
    if h:
        _check(lib().dabs_problem_destroy(h))


def dabs_problem_info(p: Problem):
    n, wt, b = C.c_int32(), C.c_int32(), C.c_int64()
    _check(lib().dabs_problem_info(p.handle, C.byref(n), C.byref(wt), C.byref(b)))
    return n.value, wt.value, b.value


def dabs_problem_wide(p: Problem) -> int:
    r = int(lib().dabs_problem_wide(p.handle))
    if r < 0:
        _check(r)
    return r


def dabs_problem_set_wide(p: Problem, wide: int):
    _check(lib().dabs_problem_set_wide(p.handle, int(wide)))


def dabs_energy(p: Problem, x, e, stream=None):
    _check(lib().dabs_energy(p.handle, _ptr(x), x.shape[0], _ptr(e), _stream(stream)))


def dabs_search(p: Problem, params: dabs_search_params, x, target, best, best_e, e, delta=None, trace=None,
                flips=None, stream=None):
    cap = trace.shape[1] if trace is not None else 0
    _check(lib().dabs_search(p.handle, C.byref(params), x.shape[0], _ptr(x), _ptr(target), _ptr(best),
                             _ptr(best_e), _ptr(e), _ptr(delta), _ptr(trace), cap, _ptr(flips), _stream(stream)))


def dabs_batch_search(p: Problem, params: dabs_batch_params, x, target, algo, phase, best, best_e, e, flips=None,
                      stream=None):
    _check(lib().dabs_batch_search(p.handle, C.byref(params), x.shape[0], _ptr(x), _ptr(target), _ptr(algo),
                                   _ptr(phase), _ptr(best), _ptr(best_e), _ptr(e), _ptr(flips), _stream(stream)))


class Solver:
    def __init__(self, handle, problem, params, instances):
        self.handle, self.problem, self.params, self.instances = handle, problem, params, instances

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _lib is not None:
            _lib.dabs_solver_destroy(h)


def ga_params(*, T, Bn, tau=8, seed=0, capacity=100, npools=1, algos=MAIN_ALGOS, ops=tuple(range(8)),
              p_explore=214748365, p_mutation=1 << 29, p_zero=1 << 29, p_one=1 << 29, crossover_kind=0,
              greedy_cap=0, flags=0, merge_hamming=0) -> dabs_ga_params:
    g = dabs_ga_params()
    g.n_algos = len(algos)
    for i, a in enumerate(algos):
        g.algos[i] = a
    g.n_ops = len(ops)
    for i, o in enumerate(ops):
        g.ops[i] = o
    g.p_explore, g.p_mutation, g.p_zero, g.p_one = p_explore, p_mutation, p_zero, p_one
    g.crossover_kind, g.capacity, g.npools, g.tau = crossover_kind, capacity, npools, tau
    g.T, g.Bn, g.greedy_cap, g.seed, g.flags = T, Bn, greedy_cap, seed, flags
    g.merge_hamming = merge_hamming
    return g


def dabs_solver_create(p: Problem, params: dabs_ga_params, instances: int, stream=None) -> Solver:
    h = C.c_void_p()
    _check(lib().dabs_solver_create(p.handle, C.byref(params), instances, _stream(stream), C.byref(h)))
    return Solver(h, p, params, instances)


def dabs_solver_destroy(s: Solver):
    h, s.handle = s.handle, None
    if h:
        _check(lib().dabs_solver_destroy(h))


def dabs_solver_run(s: Solver, rounds: int, target_e=None, stream=None):
    _check(lib().dabs_solver_run(s.handle, rounds, _ptr(target_e), _stream(stream)))


def dabs_solver_pools(s: Solver, bits=None, e=None, algo=None, op=None, stream=None):
    _check(lib().dabs_solver_pools(s.handle, _ptr(bits), _ptr(e), _ptr(algo), _ptr(op), _stream(stream)))


def dabs_solver_state(s: Solver, x=None, e=None, phase=None, total_flips=None, stream=None):
    _check(lib().dabs_solver_state(s.handle, _ptr(x), _ptr(e), _ptr(phase), _ptr(total_flips), _stream(stream)))


def dabs_solver_progress(s: Solver, out, stream=None):
    _check(lib().dabs_solver_progress(s.handle, _ptr(out), _stream(stream)))


def dabs_solver_timing(s: Solver, reset: bool = False):
    """(walk milliseconds, walk launches, flips) since the last reset."""
    out = (C.c_double * 3)()
    _check(lib().dabs_solver_timing(s.handle, out, int(reset)))
    return out[0], int(out[1]), int(out[2])


def _trace_items(fn, handle, buf):
    n = C.c_int64(0)
    _check(fn(handle, _ptr(buf), 0 if buf is None else buf.numel(), C.byref(n)))
    return n.value


def dabs_solver_trace_items(s: Solver, buf=None) -> int:
    """Per-item trace of later rounds into `buf` (int64 device tensor of at
    least 4 x items words; None stops tracing).  Returns the item count."""
    return _trace_items(lib().dabs_solver_trace_items, s.handle, buf)


class Batched:
    def __init__(self, handle, problems, params, instances):
        self.handle, self.problems, self.params, self.instances = handle, problems, params, instances

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _lib is not None:
            _lib.dabs_batched_destroy(h)


def dabs_batched_create(problems, params, instances, stream=None) -> Batched:
    """problems: list of Problem; params: list of dabs_ga_params; instances: list of int."""
    n = len(problems)
    hp = (C.c_void_p * n)(*[p.handle.value if isinstance(p.handle, C.c_void_p) else p.handle for p in problems])
    gp = (dabs_ga_params * n)(*params)
    ip = (C.c_int32 * n)(*instances)
    h = C.c_void_p()
    _check(lib().dabs_batched_create(hp, n, gp, ip, _stream(stream), C.byref(h)))
    return Batched(h, list(problems), list(params), list(instances))


def dabs_batched_destroy(b: Batched):
    h, b.handle = b.handle, None
    if h:
        _check(lib().dabs_batched_destroy(h))


def dabs_batched_run(b: Batched, rounds: int, target_e=None, use_graph: bool = True, stream=None):
    _check(lib().dabs_batched_run(b.handle, rounds, _ptr(target_e), int(use_graph), _stream(stream)))


def dabs_batched_progress(b: Batched, out, stream=None):
    _check(lib().dabs_batched_progress(b.handle, _ptr(out), _stream(stream)))


def dabs_batched_pools(b: Batched, prob: int, bits=None, e=None, algo=None, op=None, stream=None):
    _check(lib().dabs_batched_pools(b.handle, prob, _ptr(bits), _ptr(e), _ptr(algo), _ptr(op), _stream(stream)))


def dabs_batched_state(b: Batched, prob: int, x=None, e=None, phase=None, stream=None):
    _check(lib().dabs_batched_state(b.handle, prob, _ptr(x), _ptr(e), _ptr(phase), _stream(stream)))


def dabs_batched_flips(b: Batched, out, stream=None):
    _check(lib().dabs_batched_flips(b.handle, _ptr(out), _stream(stream)))


def dabs_solver_record(s: Solver, bits=None, out=None, stream=None):
    """bits [nwords] int64, out [3] int64 = (energy, restarts, rounds)."""
    _check(lib().dabs_solver_record(s.handle, _ptr(bits), _ptr(out), _stream(stream)))


DABS_STATS = 50


def dabs_solver_stats(s: Solver, out, stream=None):
    """out [50] int64: uses of operations (16) and algorithms (8), their
    packets that entered a pool (16 + 8), the record's operation and
    algorithm."""
    _check(lib().dabs_solver_stats(s.handle, _ptr(out), _stream(stream)))


def dabs_batched_stats(b: Batched, prob: int, out, stream=None):
    _check(lib().dabs_batched_stats(b.handle, prob, _ptr(out), _stream(stream)))


def dabs_solver_set_cancel(s: Solver, flag):
    """flag: pinned host int32 tensor (torch.zeros(1, dtype=torch.int32, pin_memory=True)) or None."""
    s.cancel_flag = flag            # keep it alive while attached
    _check(lib().dabs_solver_set_cancel(s.handle, _host_ptr(flag)))


def dabs_batched_record(b: Batched, prob: int, bits=None, out=None, stream=None):
    _check(lib().dabs_batched_record(b.handle, prob, _ptr(bits), _ptr(out), _stream(stream)))


def dabs_batched_set_cancel(b: Batched, flag):
    b.cancel_flag = flag
    _check(lib().dabs_batched_set_cancel(b.handle, _host_ptr(flag)))


def dabs_batched_timing(b: Batched, reset: bool = False):
    out = (C.c_double * 3)()
    _check(lib().dabs_batched_timing(b.handle, out, int(reset)))
    return out[0], int(out[1]), int(out[2])


# ------------------------------------------------------------------ learned proposal
class Mlp:
    def __init__(self, handle):
        self.handle = handle

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _lib is not None:
            _lib.dabs_mlp_destroy(h)


def dabs_mlp_create(params=None) -> Mlp:
    """params: optional float32 array of DABS_MLP_PARAMS initial values (host)."""
    import numpy as np
    h = C.c_void_p()
    buf = None
    if params is not None:
        buf = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        if buf.shape != (DABS_MLP_PARAMS,):
            raise ValueError("need %d parameters" % DABS_MLP_PARAMS)
    _check(lib().dabs_mlp_create(None if buf is None else buf.ctypes.data_as(C.c_void_p), C.byref(h)))
    return Mlp(h)


def dabs_mlp_destroy(m: Mlp):
    h, m.handle = m.handle, None
    if h:
        _check(lib().dabs_mlp_destroy(h))


def dabs_mlp_params(m: Mlp, out, stream=None):
    _check(lib().dabs_mlp_params(m.handle, _ptr(out), _stream(stream)))


def dabs_mlp_pool_features(p: Problem, pool_bits, npools: int, capacity: int, feat, stream=None):
    _check(lib().dabs_mlp_pool_features(p.handle, _ptr(pool_bits), npools, capacity, _ptr(feat), _stream(stream)))


def dabs_mlp_pool_features_noalloc(p: Problem, pool_bits, npools: int, capacity: int, feat, stream=None):
    _check(lib().dabs_mlp_pool_features_noalloc(p.handle, _ptr(pool_bits), npools, capacity, _ptr(feat),
                                                _stream(stream)))


def dabs_mlp_labels(p: Problem, bits, count: int, ref, labels, symmetric: bool = False, stream=None):
    _check(lib().dabs_mlp_labels(p.handle, _ptr(bits), count, _ptr(ref), int(symmetric), _ptr(labels),
                                 _stream(stream)))


def dabs_mlp_forward(m: Mlp, count: int, feat, logits, stream=None):
    _check(lib().dabs_mlp_forward(m.handle, count, _ptr(feat), _ptr(logits), _stream(stream)))


def dabs_mlp_grad(m: Mlp, count: int, feat, labels, grad=None, loss=None, stream=None):
    _check(lib().dabs_mlp_grad(m.handle, count, _ptr(feat), _ptr(labels), _ptr(grad), _ptr(loss), _stream(stream)))


def dabs_mlp_adam(m: Mlp, lr: float, stream=None):
    _check(lib().dabs_mlp_adam(m.handle, lr, _stream(stream)))


def dabs_mlp_train_step(m: Mlp, count: int, feat, labels, lr: float, loss=None, stream=None):
    _check(lib().dabs_mlp_train_step(m.handle, count, _ptr(feat), _ptr(labels), lr, _ptr(loss), _stream(stream)))


def dabs_mlp_apply_op(op: int, n: int, count: int, parents, logits, seed: int, round: int, inst0: int, out,
                      stream=None):
    _check(lib().dabs_mlp_apply_op(op, n, count, _ptr(parents), _ptr(logits), seed, round, inst0, _ptr(out),
                                   _stream(stream)))


def dabs_solver_set_mlp(s: Solver, m):
    _check(lib().dabs_solver_set_mlp(s.handle, None if m is None else m.handle))
    s.mlp = m                                   # keep the network alive while attached


def dabs_batched_set_mlp(b: Batched, m):
    _check(lib().dabs_batched_set_mlp(b.handle, None if m is None else m.handle))
    b.mlp = m


# ------------------------------------------------------------------ autotuner
def dabs_batched_trace_items(b: Batched, buf=None) -> int:
    return _trace_items(lib().dabs_batched_trace_items, b.handle, buf)


def dabs_batched_classes(b: Batched):
    """[(wtype, slots, items, variant)] of the batch's size classes."""
    nc = lib().dabs_batched_classes(b.handle, None, 0)
    if nc < 0:
        _check(nc)
    out = (C.c_int32 * (4 * max(nc, 1)))()
    lib().dabs_batched_classes(b.handle, C.cast(out, C.c_void_p), nc)
    return [tuple(out[4 * c:4 * c + 4]) for c in range(nc)]


def _checkpoint(fn, handle, blob, stream):
    n = C.c_int64(0)
    if blob is None:
        _check(fn(handle, None, C.byref(n), _stream(stream)))
        return n.value
    n.value = blob.numel() * blob.element_size()
    _check(fn(handle, _ptr(blob), C.byref(n), _stream(stream)))
    return n.value


def dabs_batched_checkpoint(b: Batched, blob=None, stream=None) -> int:
    """Bytes of the batch's checkpoint (blob None), or writes it into the
    device tensor `blob` and returns its size."""
    return _checkpoint(lib().dabs_batched_checkpoint, b.handle, blob, stream)


def dabs_batched_restore(b: Batched, blob, stream=None):
    _check(lib().dabs_batched_restore(b.handle, _ptr(blob), _stream(stream)))


def dabs_solver_checkpoint(s: Solver, blob=None, stream=None) -> int:
    return _checkpoint(lib().dabs_solver_checkpoint, s.handle, blob, stream)


def dabs_solver_restore(s: Solver, blob, stream=None):
    _check(lib().dabs_solver_restore(s.handle, _ptr(blob), _stream(stream)))


def dabs_batched_set_variant(b: Batched, cls: int, variant: int):
    _check(lib().dabs_batched_set_variant(b.handle, cls, variant))


def walk_slots(wtype: int, n: int) -> int:
    """Slots (16-byte pieces per lane, a power of two) of the dense walker."""
    span = 512 if wtype == DABS_W_I16 else 256
    s = 1
    while s * span < n:
        s *= 2
    return s


def lds_w_bytes(wtype: int, n: int) -> int:
    """Bytes of the LDS copy of a dense W of one slot (rows rounded up to a
    16-byte piece), 0 when the problem cannot use it (more than 40 KB)."""
    v, es = (8, 2) if wtype == DABS_W_I16 else (4, 4)
    if wtype not in (DABS_W_I16, DABS_W_I32) or n > 64 * v:
        return 0
    b = n * ((n + v - 1) // v * v) * es
    return b if b <= 40960 else 0


def dabs_batched_autotune(b: Batched, stream=None):
    """Returns (milliseconds [class][variant], chosen variant per class)."""
    nc = len(dabs_batched_classes(b))
    V = DABS_WALK_VARIANTS
    ms = (C.c_double * (V * nc))()
    ch = (C.c_int32 * nc)()
    _check(lib().dabs_batched_autotune(b.handle, C.cast(ms, C.c_void_p), C.cast(ch, C.c_void_p), _stream(stream)))
    return [[ms[V * c + v] for v in range(V)] for c in range(nc)], list(ch)


def dabs_solver_autotune(s: Solver, stream=None):
    V = DABS_WALK_VARIANTS
    ms = (C.c_double * V)()
    ch = (C.c_int32 * 1)()
    _check(lib().dabs_solver_autotune(s.handle, C.cast(ms, C.c_void_p), C.cast(ch, C.c_void_p), _stream(stream)))
    return [[ms[v] for v in range(V)]], list(ch)
