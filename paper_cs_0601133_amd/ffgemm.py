"""Python binding of libffgemm.so: the C ABI of include/ffgemm.h, same names.

Argument marshalling only.  Every step of the computation runs in the HIP
library; if the library is missing this module raises at import-time use
(there is no fallback).  Matrices may be given as torch tensors (int32 or
uint32 storage of residues, row-major with unit column stride, on a ROCm
device) or as raw device addresses (ints).
"""
import ctypes
import os

from . import build as _build

FF_OK = 0
FF_EINVAL = -1
FF_EUNSUPPORTED = -2
FF_ENOMEM = -3
FF_EHIP = -4
FF_EBUSY = -5
FF_ENOTFOUND = -6

FF_NOTRANS = 0
FF_TRANS = 1
FF_UPPER = 0
FF_LOWER = 1
FF_NONUNIT = 0
FF_UNIT = 1

FF_PATH_AUTO = 0
FF_PATH_FP64 = 1
FF_PATH_INT8 = 2

FF_PROFILE_GEMM = 1
FF_PROFILE_PREP = 2

FF_NOALLOC_SCRATCH_BYTES = 128 << 20   # size of ff_fgemm_noalloc's static scratch

_I64 = ctypes.c_int64
_U32 = ctypes.c_uint32
_INT = ctypes.c_int
_VP = ctypes.c_void_p


class ff_opts(ctypes.Structure):
    _fields_ = [("path", _INT), ("winograd_levels", _INT), ("digit_bits", _INT),
                ("validate", _INT), ("preadd_mode", _INT), ("stream", _VP),
                ("digit_pairing", _INT)]


class ff_plan_info(ctypes.Structure):
    _fields_ = [("path", _INT), ("winograd_levels", _INT), ("preadds_reduced", _INT),
                ("digit_bits", _INT), ("slices", _INT), ("operand_lo", _I64),
                ("operand_hi", _I64), ("max_abs_product", _I64), ("kblock", _I64),
                ("workspace_bytes", _I64), ("tile_config", _INT), ("digit_products", _INT)]


class ff_job(ctypes.Structure):
    _fields_ = [("p", _U32), ("transA", _INT), ("transB", _INT), ("m", _I64), ("n", _I64),
                ("k", _I64), ("alpha", _U32), ("beta", _U32), ("A", _VP), ("lda", _I64),
                ("B", _VP), ("ldb", _I64), ("C", _VP), ("ldc", _I64)]


class ff_server_info(ctypes.Structure):
    _fields_ = [("submitted", _I64), ("completed", _I64), ("failed", _I64), ("queued", _I64),
                ("running", _I64), ("batches", _I64), ("max_batch_requests", _I64),
                ("max_inflight", _I64), ("hbm_budget", _I64), ("hbm_in_use", _I64),
                ("last_i8_tile", _INT), ("stream_slots", _INT)]


# name -> (argtypes, restype)
_SIGS = {
    "ff_init": ([], _INT),
    "ff_finalize": ([], _INT),
    "ff_set_stream": ([_VP], _INT),
    "ff_fgemm": ([_U32, _INT, _INT, _I64, _I64, _I64, _U32, _VP, _I64, _VP, _I64, _U32,
                  _VP, _I64], _INT),
    "ff_fgemm_ex": ([_U32, _INT, _INT, _I64, _I64, _I64, _U32, _VP, _I64, _VP, _I64, _U32,
                     _VP, _I64, ctypes.POINTER(ff_opts)], _INT),
    "ff_fgemm_noalloc": ([_U32, _INT, _INT, _I64, _I64, _I64, _U32, _VP, _I64, _VP, _I64,
                          _U32, _VP, _I64, ctypes.POINTER(ff_opts)], _INT),
    "ff_ftrsm": ([_U32, _INT, _INT, _INT, _I64, _I64, _U32, _VP, _I64, _VP, _I64], _INT),
    "ff_ftrsm_ex": ([_U32, _INT, _INT, _INT, _I64, _I64, _U32, _VP, _I64, _VP, _I64,
                     ctypes.POINTER(ff_opts)], _INT),
    "ff_faat": ([_U32, _I64, _I64, _U32, _VP, _I64, _VP, _U32, _VP, _I64,
                 ctypes.POINTER(ff_opts)], _INT),
    "ff_flqup": ([_U32, _I64, _I64, _VP, _I64, _VP, _VP, _VP, ctypes.POINTER(ff_opts)], _INT),
    "ff_frank": ([_U32, _I64, _I64, _VP, _I64, _VP, ctypes.POINTER(ff_opts)], _INT),
    "ff_fdet": ([_U32, _I64, _VP, _I64, _VP, ctypes.POINTER(ff_opts)], _INT),
    "ff_finv": ([_U32, _I64, _VP, _I64, _VP, _I64, _VP, ctypes.POINTER(ff_opts)], _INT),
    "ff_plan_query": ([_U32, _INT, _INT, _I64, _I64, _I64, ctypes.POINTER(ff_opts),
                       ctypes.POINTER(ff_plan_info)], _INT),
    "ff_fgemm_batched": ([ctypes.POINTER(ff_job), _INT, ctypes.POINTER(ff_opts)], _INT),
    "ff_batch_graph_create": ([ctypes.POINTER(ff_job), _INT, ctypes.POINTER(ff_opts),
                               ctypes.POINTER(_VP)], _INT),
    "ff_batch_graph_launch": ([_VP, _VP], _INT),
    "ff_batch_graph_destroy": ([_VP], _INT),
    "ff_server_create": ([_I64, ctypes.POINTER(ff_opts), ctypes.POINTER(_VP)], _INT),
    "ff_server_submit": ([_VP, ctypes.POINTER(ff_job), ctypes.POINTER(ctypes.c_uint64)],
                         _INT),
    "ff_server_poll": ([_VP, ctypes.c_uint64, ctypes.POINTER(_INT)], _INT),
    "ff_server_wait": ([_VP, ctypes.c_uint64], _INT),
    "ff_server_stats": ([_VP, ctypes.POINTER(ctypes.c_double),
                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                         ctypes.POINTER(_I64), ctypes.POINTER(_I64)], _INT),
    "ff_server_query": ([_VP, ctypes.POINTER(ff_server_info)], _INT),
    "ff_server_destroy": ([_VP], _INT),
    "ff_autotune": ([_INT, _I64, _I64, _I64, ctypes.POINTER(_INT),
                     ctypes.POINTER(ctypes.c_double)], _INT),
    "ff_profile_enable": ([_INT], _INT),
    "ff_profile_read": ([ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I64),
                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I64)], _INT),
    "ff_last_error": ([], ctypes.c_char_p),
}

EXPORTED = sorted(_SIGS)

_lib = None


def library_path():
    # FF_LIBRARY points at another build of the same library (kernel
    # experiments); the default is the in-tree build.
    return os.environ.get("FF_LIBRARY") or _build.LIB


def _init_torch_runtime():
    # Loaded after torch, the library resolves to torch's HIP runtime, and
    # torch must initialise that runtime itself: its own initialisation
    # reports no devices when another caller (a library call) initialised it
    # first.  So torch is imported and initialised before the library loads.
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


def load():
    """Load libffgemm.so (it must have been built: see build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: the HIP library has not been built "
                           "(python -m paper_cs_0601133_amd.build)")
    _init_torch_runtime()
    lib = ctypes.CDLL(path)
    for name, (args, res) in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


class FFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"status {status}: {msg}")
        self.status = status


def _check(rc):
    if rc != FF_OK:
        raise FFError(rc, load().ff_last_error().decode())
    return rc


def _addr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _ld(x, default):
    if x is None or isinstance(x, int):
        return default
    sh, st = x.shape, x.stride()
    if len(sh) != 2:
        raise ValueError("matrices must be 2-D")
    if sh[1] > 1 and st[1] != 1:
        raise ValueError("matrices must have unit column stride (row-major)")
    return max(st[0], sh[1], 1)


def make_opts(path=FF_PATH_AUTO, winograd_levels=-1, digit_bits=0, validate=0,
              preadd_mode=0, stream=None, digit_pairing=0):
    return ff_opts(path, winograd_levels, digit_bits, validate, preadd_mode, stream,
                   digit_pairing)


def _torch_stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


# --- the C ABI, same names --------------------------------------------------

def ff_init():
    return _check(load().ff_init())


def ff_finalize():
    return _check(load().ff_finalize())


def ff_set_stream(stream):
    return _check(load().ff_set_stream(stream))


def ff_last_error():
    return load().ff_last_error().decode()


def ff_fgemm(p, transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc):
    return load().ff_fgemm(p, transA, transB, m, n, k, alpha, _addr(A), lda, _addr(B), ldb,
                           beta, _addr(C), ldc)


def ff_fgemm_ex(p, transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, opts=None):
    o = ctypes.byref(opts) if opts is not None else None
    return load().ff_fgemm_ex(p, transA, transB, m, n, k, alpha, _addr(A), lda, _addr(B),
                              ldb, beta, _addr(C), ldc, o)


def ff_fgemm_noalloc(p, transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                     opts=None):
    o = ctypes.byref(opts) if opts is not None else None
    return load().ff_fgemm_noalloc(p, transA, transB, m, n, k, alpha, _addr(A), lda,
                                   _addr(B), ldb, beta, _addr(C), ldc, o)


def ff_ftrsm(p, uplo, transT, diag, m, n, alpha, T, ldt, B, ldb):
    return load().ff_ftrsm(p, uplo, transT, diag, m, n, alpha, _addr(T), ldt, _addr(B), ldb)


def ff_ftrsm_ex(p, uplo, transT, diag, m, n, alpha, T, ldt, B, ldb, opts=None):
    o = ctypes.byref(opts) if opts is not None else None
    return load().ff_ftrsm_ex(p, uplo, transT, diag, m, n, alpha, _addr(T), ldt, _addr(B), ldb,
                              o)


def ff_faat(p, m, k, alpha, A, lda, D, beta, C, ldc, opts=None):
    o = ctypes.byref(opts) if opts is not None else None
    return load().ff_faat(p, m, k, alpha, _addr(A), lda, _addr(D) if D is not None else None,
                          beta, _addr(C), ldc, o)


def ff_flqup(p, m, n, A, lda, rank, pivrows, colperm, opts=None):
    """rank, pivrows, colperm: numpy int64 arrays (host) of sizes 1, m, n."""
    o = ctypes.byref(opts) if opts is not None else None
    return load().ff_flqup(p, m, n, _addr(A), lda, rank.ctypes.data, pivrows.ctypes.data,
                           colperm.ctypes.data, o)


def ff_frank(p, m, n, A, lda, rank, opts=None):
    o = ctypes.byref(opts) if opts is not None else None
    return load().ff_frank(p, m, n, _addr(A), lda, rank.ctypes.data, o)


def ff_fdet(p, n, A, lda, det, opts=None):
    """det: numpy uint32 array (host) of size 1."""
    o = ctypes.byref(opts) if opts is not None else None
    return load().ff_fdet(p, n, _addr(A), lda, det.ctypes.data, o)


def ff_finv(p, n, A, lda, X, ldx, invertible, opts=None):
    """invertible: numpy int32 array (host) of size 1."""
    o = ctypes.byref(opts) if opts is not None else None
    return load().ff_finv(p, n, _addr(A), lda, _addr(X), ldx, invertible.ctypes.data, o)


def ff_plan_query(p, transA, transB, m, n, k, opts=None):
    info = ff_plan_info()
    o = ctypes.byref(opts) if opts is not None else None
    _check(load().ff_plan_query(p, transA, transB, m, n, k, o, ctypes.byref(info)))
    return info


def _jobs(jobs):
    arr = (ff_job * len(jobs))()
    for i, j in enumerate(jobs):
        arr[i] = j
    return arr


def ff_fgemm_batched(jobs, opts=None):
    arr = _jobs(jobs)
    o = ctypes.byref(opts) if opts is not None else None
    return load().ff_fgemm_batched(arr, len(jobs), o)


def ff_batch_graph_create(jobs, opts=None):
    arr = _jobs(jobs)
    o = ctypes.byref(opts) if opts is not None else None
    g = _VP()
    _check(load().ff_batch_graph_create(arr, len(jobs), o, ctypes.byref(g)))
    return g.value


def ff_batch_graph_launch(graph, stream=None):
    return _check(load().ff_batch_graph_launch(graph, stream))


def ff_batch_graph_destroy(graph):
    return _check(load().ff_batch_graph_destroy(graph))


def ff_server_create(hbm_budget_bytes, opts=None):
    o = ctypes.byref(opts) if opts is not None else None
    s = _VP()
    _check(load().ff_server_create(hbm_budget_bytes, o, ctypes.byref(s)))
    return s.value


def ff_server_submit(server, job):
    rid = ctypes.c_uint64()
    _check(load().ff_server_submit(server, ctypes.byref(job), ctypes.byref(rid)))
    return rid.value


def ff_server_poll(server, rid):
    done = _INT()
    _check(load().ff_server_poll(server, rid, ctypes.byref(done)))
    return bool(done.value)


def ff_server_wait(server, rid):
    return _check(load().ff_server_wait(server, rid))


def ff_server_stats(server):
    p50, p99, gops = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    done, mx = _I64(), _I64()
    _check(load().ff_server_stats(server, ctypes.byref(p50), ctypes.byref(p99),
                                  ctypes.byref(gops), ctypes.byref(done), ctypes.byref(mx)))
    return {"p50_ms": p50.value, "p99_ms": p99.value, "gops": gops.value,
            "completed": done.value, "max_inflight": mx.value}


def ff_autotune(slices, m, n, k):
    best, ms = _INT(), ctypes.c_double()
    _check(load().ff_autotune(slices, m, n, k, ctypes.byref(best), ctypes.byref(ms)))
    return best.value, ms.value


def ff_profile_enable(mask):
    """mask: FF_PROFILE_GEMM | FF_PROFILE_PREP (True: both), 0 disables."""
    if mask is True:
        mask = FF_PROFILE_GEMM | FF_PROFILE_PREP
    return _check(load().ff_profile_enable(int(mask)))


def ff_profile_read():
    g, s = ctypes.c_double(), ctypes.c_double()
    ng, ns = _I64(), _I64()
    _check(load().ff_profile_read(ctypes.byref(g), ctypes.byref(ng), ctypes.byref(s),
                                  ctypes.byref(ns)))
    return {"gemm_ms": g.value, "gemm_launches": ng.value, "slice_ms": s.value,
            "slice_launches": ns.value}


def ff_server_query(server):
    info = ff_server_info()
    _check(load().ff_server_query(server, ctypes.byref(info)))
    return info


def ff_server_destroy(server):
    return _check(load().ff_server_destroy(server))


# --- marshalling helpers for torch tensors ----------------------------------

def job(p, A, B, C, alpha=1, beta=0, transA=False, transB=False):
    """An ff_job for torch tensors A, B, C (op(A) is m x k, op(B) k x n)."""
    m = A.shape[1] if transA else A.shape[0]
    k = A.shape[0] if transA else A.shape[1]
    n = B.shape[0] if transB else B.shape[1]
    return ff_job(p, int(transA), int(transB), m, n, k, alpha % p, beta % p, _addr(A),
                  _ld(A, 1), _addr(B), _ld(B, 1), _addr(C), _ld(C, 1))


def ftrsm(p, T, B, alpha=1, lower=False, trans=False, unit=False, opts=None):
    """B <- X with op(T) X = alpha B (mod p) for torch tensors T (m x m) and B
    (m x n), on torch's current stream."""
    m, n = B.shape[0], B.shape[1]
    if opts is None:
        opts = make_opts()
    if not opts.stream:
        opts.stream = _torch_stream()
    return _check(ff_ftrsm_ex(p, int(lower), int(trans), int(unit), m, n, alpha % p, T,
                              _ld(T, 1), B, _ld(B, 1), opts))


def aat(p, A, C, D=None, alpha=1, beta=0, opts=None):
    """C <- alpha A diag(D) A^T + beta C mod p for torch tensors (C m x m,
    symmetric on return), on torch's current stream."""
    m, k = A.shape[0], A.shape[1]
    if opts is None:
        opts = make_opts()
    if not opts.stream:
        opts.stream = _torch_stream()
    return _check(ff_faat(p, m, k, alpha % p, A, _ld(A, 1), D, beta % p, C, _ld(C, 1), opts))


def lqup(p, A, opts=None):
    """LQUP of the torch tensor A (m x n, overwritten by the compressed form)
    on torch's current stream; returns (rank, pivrows, colperm) as Python
    int and numpy int64 arrays."""
    import numpy as np
    m, n = A.shape[0], A.shape[1]
    if opts is None:
        opts = make_opts()
    if not opts.stream:
        opts.stream = _torch_stream()
    rank = np.zeros(1, dtype=np.int64)
    piv = np.zeros(max(m, 1), dtype=np.int64)
    perm = np.zeros(max(n, 1), dtype=np.int64)
    _check(ff_flqup(p, m, n, A, _ld(A, 1), rank, piv, perm, opts))
    return int(rank[0]), piv[:m], perm[:n]


def det(p, A, opts=None):
    """det of the square torch tensor A over Z/p (A is overwritten)."""
    import numpy as np
    if opts is None:
        opts = make_opts()
    if not opts.stream:
        opts.stream = _torch_stream()
    d = np.zeros(1, dtype=np.uint32)
    _check(ff_fdet(p, A.shape[0], A, _ld(A, 1), d, opts))
    return int(d[0])


def inv(p, A, X, opts=None):
    """X <- A^-1 over Z/p for the square torch tensor A (A is overwritten by
    its LQUP factorisation; X may be A).  Returns False, X untouched, when A
    is singular."""
    import numpy as np
    if opts is None:
        opts = make_opts()
    if not opts.stream:
        opts.stream = _torch_stream()
    ok = np.zeros(1, dtype=np.int32)
    _check(ff_finv(p, A.shape[0], A, _ld(A, 1), X, _ld(X, 1), ok, opts))
    return bool(ok[0])


def fgemm(p, A, B, C, alpha=1, beta=0, transA=False, transB=False, opts=None):
    """C <- (alpha*op(A)*op(B) + beta*C) mod p on torch's current stream."""
    m = A.shape[1] if transA else A.shape[0]
    k = A.shape[0] if transA else A.shape[1]
    n = B.shape[0] if transB else B.shape[1]
    if opts is None:
        opts = make_opts()
    if not opts.stream:
        opts.stream = _torch_stream()
    # straight to the C entry point (small products are latency-bound)
    rc = load().ff_fgemm_ex(p, int(transA), int(transB), m, n, k, alpha % p, _addr(A),
                            _ld(A, 1), _addr(B), _ld(B, 1), beta % p, _addr(C), _ld(C, 1),
                            ctypes.byref(opts))
    return rc if rc == FF_OK else _check(rc)
