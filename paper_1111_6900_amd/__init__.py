"""Python binding of libgf2e (dense matrix multiplication over F_{2^e} on MI355X).

Argument marshalling only: every step of a product runs in the library's HIP
kernels (see include/gf2e.h for the C ABI).  PyTorch supplies device memory
and streams.  If the built library is missing, importing this package still
works but every call raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch  # loads the HIP runtime the library then shares

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgf2e.so")

OK, EINVAL, EFIELD, ESHAPE, EALIAS, ERANGE, ENOMEM, EDEVICE, EBUSY, ESINGULAR = \
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9
KERNEL_AUTO, KERNEL_MFMA_256, KERNEL_MFMA_128, KERNEL_MFMA_256x128, KERNEL_MFMA_64, KERNEL_VALU_128, \
    KERNEL_MFMA_256_W8, KERNEL_FP4_256_W8, KERNEL_FP4_128, KERNEL_FP4_128_PLANES = -1, 0, 1, 2, 3, 4, 5, 6, 7, 8
FORM_AUTO, FORM_SCHEDULE, FORM_ALPHA = -1, 0, 1
STAGE_SLICE_A, STAGE_SLICE_B, STAGE_PRODUCTS, STAGE_COMBINE, STAGE_BATCH = 0, 1, 2, 3, 4


class GF2EError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = strerror(code) if _lib is not None else f"error {code}"
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")


class Mat(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("rows", ctypes.c_int64), ("cols", ctypes.c_int64),
                ("ld", ctypes.c_int64)]


class Config(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int), ("autotune", ctypes.c_int),
                ("workspace_limit", ctypes.c_int64)]


class Geometry(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int), ("Mp", ctypes.c_int64), ("Np", ctypes.c_int64),
                ("K64p", ctypes.c_int64), ("a_bytes", ctypes.c_int64), ("b_bytes", ctypes.c_int64),
                ("p_bytes", ctypes.c_int64)]


class BatchStats(ctypes.Structure):
    _fields_ = [("items_large", ctypes.c_int64), ("items_small", ctypes.c_int64),
                ("arena_bytes", ctypes.c_int64), ("graphs_cached", ctypes.c_int),
                ("graph_builds", ctypes.c_int64), ("threshold", ctypes.c_int64),
                ("items_fused", ctypes.c_int64), ("fusion", ctypes.c_int)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("memory_budget", ctypes.c_int64), ("max_inflight", ctypes.c_int),
                ("quantum_macs", ctypes.c_int64), ("max_items_per_iteration", ctypes.c_int64),
                ("bypass_limit", ctypes.c_int)]


class ReqTimes(ctypes.Structure):
    _fields_ = [("t_submit_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64), ("status", ctypes.c_int)]


class ServerCounters(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int64), ("iterations", ctypes.c_int64),
                ("element_macs", ctypes.c_int64), ("peak_arena_bytes", ctypes.c_int64),
                ("peak_inflight", ctypes.c_int), ("memory_waits", ctypes.c_int64),
                ("bypass_admissions", ctypes.c_int64), ("shared_iterations", ctypes.c_int64),
                ("max_iteration_requests", ctypes.c_int)]


_lib = None
_lock = threading.Lock()

_i32, _i64, _u32, _vp = ctypes.c_int, ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p
_P = ctypes.POINTER

# name: (restype, argtypes)
_SIGS = {
    "gf2e_create": (_i32, [_P(_vp), _i32, _P(Config)]),
    "gf2e_destroy": (None, [_vp]),
    "gf2e_mul": (_i32, [_vp, _P(Mat), _P(Mat), _P(Mat), _i32, _u32]),
    "gf2e_mul_async": (_i32, [_vp, _P(Mat), _P(Mat), _P(Mat), _i32, _u32, _vp]),
    "gf2e_mul_noalloc_async": (_i32, [_vp, _P(Mat), _P(Mat), _P(Mat), _i32, _u32, _vp]),
    "gf2e_sync": (_i32, [_vp, _vp]),
    "gf2e_mul_add_async": (_i32, [_vp, _P(Mat), _P(Mat), _P(Mat), _i32, _u32, _vp]),
    "gf2e_mul_add": (_i32, [_vp, _P(Mat), _P(Mat), _P(Mat), _i32, _u32]),
    "gf2e_trsm_async": (_i32, [_vp, _i32, _i32, _P(Mat), _P(Mat), _i32, _u32, _vp]),
    "gf2e_trsm": (_i32, [_vp, _i32, _i32, _P(Mat), _P(Mat), _i32, _u32]),
    "gf2e_echelonize": (_i32, [_vp, _P(Mat), _i32, _u32, _i32, _P(_i64), _vp]),
    "gf2e_ple": (_i32, [_vp, _P(Mat), _P(Mat), _i32, _u32, _P(_i64), _vp, _vp]),
    "gf2e_mul_batched": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp]),
    "gf2e_set_batch_threshold": (_i32, [_vp, _i64]),
    "gf2e_set_batch_fusion": (_i32, [_vp, _i32]),
    "gf2e_tune_batched": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp]),
    "gf2e_batch_info": (_i32, [_vp, _P(BatchStats)]),
    "gf2e_server_create": (_i32, [_vp, _P(ServerConfig), _P(_vp)]),
    "gf2e_server_destroy": (None, [_vp]),
    "gf2e_server_submit": (_i32, [_vp, _P(Mat), _P(Mat), _P(Mat), _i32, _u32, _vp, _P(ctypes.c_uint64)]),
    "gf2e_server_poll": (_i32, [_vp, ctypes.c_uint64, _P(_i32), _P(ReqTimes)]),
    "gf2e_server_wait": (_i32, [_vp, ctypes.c_uint64, _P(ReqTimes)]),
    "gf2e_server_stats": (_i32, [_vp, _P(ServerCounters)]),
    "gf2e_server_run_trace": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "gf2e_strerror": (ctypes.c_char_p, [_i32]),
    "gf2e_field_check": (_i32, [_i32, _u32]),
    "gf2e_num_products": (_i32, [_i32, _u32]),
    "gf2e_schedule": (_i32, [_i32, _u32, _P(_i32), _vp, _vp, _vp, _vp]),
    "gf2e_plane_geometry": (_i32, [_i32, _u32, _i64, _i64, _i64, _P(Geometry)]),
    "gf2e_slice_a": (_i32, [_vp, _P(Mat), _i32, _u32, _vp, _i64, _i64, _vp]),
    "gf2e_slice_b": (_i32, [_vp, _P(Mat), _i32, _u32, _vp, _i64, _i64, _vp]),
    "gf2e_plane_products": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp, _i64, _i64, _i64, _i64, _i64, _vp]),
    "gf2e_combine": (_i32, [_vp, _i32, _u32, _vp, _i64, _i64, _P(Mat), _vp]),
    "gf2e_kernel_count": (_i32, []),
    "gf2e_kernel_name": (ctypes.c_char_p, [_i32]),
    "gf2e_set_kernel": (_i32, [_vp, _i32]),
    "gf2e_chosen_kernel": (_i32, [_vp, _i32, _u32, _i64, _i64, _i64]),
    "gf2e_tune": (_i32, [_vp, _i32, _u32, _i64, _i64, _i64, _vp]),
    "gf2e_set_form": (_i32, [_vp, _i32]),
    "gf2e_chosen_form": (_i32, [_vp, _i32, _u32, _i64, _i64, _i64]),
    "gf2e_profile": (_i32, [_vp, _i32]),
    "gf2e_profile_read": (_i32, [_vp, _i32, _P(ctypes.c_double), _P(_i64)]),
    "gf2e_profile_reset": (_i32, [_vp]),
    "gf2e_workspace_bytes": (_i64, [_vp]),
}


def lib():
    """The loaded libgf2e.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    f"{LIB_PATH} is not built; run __graft_entry__.build() "
                    "(there is no CPU fallback for the GPU path)")
            handle = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in _SIGS.items():
                fn = getattr(handle, name)
                fn.restype = res
                fn.argtypes = args
            _lib = handle
    return _lib


def strerror(code: int) -> str:
    return lib().gf2e_strerror(code).decode()


def _check(rc: int, what: str = ""):
    if rc != OK:
        raise GF2EError(rc, what)
    return rc


# ---------------------------------------------------------------------------
# Host-only queries
# ---------------------------------------------------------------------------

def field_check(e: int, f: int) -> bool:
    return lib().gf2e_field_check(e, f) == OK


def num_products(e: int, f: int) -> int:
    """GF(2) products in the schedule used for F_2[x]/<f>."""
    rc = lib().gf2e_num_products(e, f)
    if rc < 0:
        raise GF2EError(rc, "num_products")
    return rc


MAX_PRODUCTS = 96
# Size of the per-GPU scratch array of gf2e_mul_noalloc_async (include/gf2e.h).
NOALLOC_MAX_BYTES = 64 << 20


def schedule(e: int, f: int) -> dict:
    """The product schedule used for (e, f): u, v (operand subsets), w
    (polynomial recombination; all zero when the schedule has the reduction
    folded in) and m (result planes after reduction mod f).  w[d] and m[c]
    are returned as sets of product indices packed into Python ints (bit s
    for product s)."""
    t = ctypes.c_int(0)
    u = (ctypes.c_uint32 * MAX_PRODUCTS)()
    v = (ctypes.c_uint32 * MAX_PRODUCTS)()
    w = (ctypes.c_uint8 * (31 * MAX_PRODUCTS))()
    m = (ctypes.c_uint8 * (16 * MAX_PRODUCTS))()
    _check(lib().gf2e_schedule(e, f, ctypes.byref(t), u, v, w, m), "schedule")
    T = t.value

    def rows(buf, count):
        return [sum(int(buf[r * T + s]) << s for s in range(T)) for r in range(count)]

    return {"t": T, "u": list(u[:T]), "v": list(v[:T]), "w": rows(w, 2 * e - 1), "m": rows(m, e)}


def plane_geometry(e: int, f: int, m: int, k: int, n: int) -> Geometry:
    g = Geometry()
    _check(lib().gf2e_plane_geometry(e, f, m, k, n, ctypes.byref(g)), "plane_geometry")
    return g


def kernel_names() -> list:
    L = lib()
    return [L.gf2e_kernel_name(i).decode() for i in range(L.gf2e_kernel_count())]


# ---------------------------------------------------------------------------
# Tensors <-> descriptors
# ---------------------------------------------------------------------------

def elem_dtype(e: int):
    """torch storage type of one element: uint8 for e <= 8, uint16 for 9..16."""
    return torch.uint8 if e <= 8 else torch.uint16


def mat(t: torch.Tensor) -> Mat:
    if t.dim() != 2:
        raise ValueError("expected a 2-D tensor")
    if t.numel() > 0 and t.stride(1) != 1:
        raise ValueError("rows must be contiguous (stride(1) == 1)")
    ld = t.stride(0) if t.size(0) > 1 else max(t.size(1), 1)
    return Mat(t.data_ptr() if t.numel() > 0 else None, t.size(0), t.size(1), ld)


def _check_elem(t: torch.Tensor, e: int, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not 2 <= e <= 16:
        return  # the library reports GF2E_EFIELD
    ok = (t.dtype == torch.uint8) if e <= 8 else (t.dtype in (torch.int16, torch.uint16))
    if not ok:
        raise TypeError(f"{name}: elements of F_2^{e} are stored as "
                        f"{'uint8' if e <= 8 else 'int16/uint16'}, got {t.dtype}")


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class PreparedBatch:
    """A batch whose descriptors are marshalled once (see Context.prepare_batched).
    It keeps its tensors alive; launch() enqueues the batch on a stream."""

    def __init__(self, ctx, As, Bs, outs, args):
        self.ctx, self.As, self.Bs, self.outs, self._args = ctx, list(As), list(Bs), list(outs), args

    def launch(self, stream=None):
        n, MA, MB, MC, E, F = self._args
        _check(lib().gf2e_mul_batched(self.ctx.handle, n, MA, MB, MC, E, F, _stream_handle(stream)),
               "gf2e_mul_batched")
        return self.outs


class Context:
    """Owns a gf2e context (workspace, tuning cache) on one device."""

    def __init__(self, device: int = 0, kernel: int = KERNEL_AUTO, autotune: bool = False,
                 workspace_limit: int = 0):
        self.device = device
        cfg = Config(kernel, 1 if autotune else 0, workspace_limit)
        h = ctypes.c_void_p()
        _check(lib().gf2e_create(ctypes.byref(h), device, ctypes.byref(cfg)), "gf2e_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().gf2e_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- products ----------------------------------------------------------
    def mul_async(self, A, B, e: int, f: int, out=None, stream=None):
        _check_elem(A, e, "A")
        _check_elem(B, e, "B")
        if out is None:
            out = torch.empty((A.size(0), B.size(1)), dtype=A.dtype, device=A.device)
        _check_elem(out, e, "out")
        a, b, c = mat(A), mat(B), mat(out)
        _check(lib().gf2e_mul_async(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                    e, f, _stream_handle(stream)), "gf2e_mul_async")
        return out

    def sync(self, stream=None):
        _check(lib().gf2e_sync(self.handle, _stream_handle(stream)), "gf2e_sync")

    def mul_noalloc_async(self, A, B, e: int, f: int, out, stream=None):
        """gf2e_mul_noalloc_async: C = A * B into `out` with the planes in the
        library's fixed per-GPU scratch array (nothing allocated)."""
        _check_elem(A, e, "A")
        _check_elem(B, e, "B")
        _check_elem(out, e, "out")
        a, b, c = mat(A), mat(B), mat(out)
        _check(lib().gf2e_mul_noalloc_async(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                            e, f, _stream_handle(stream)), "gf2e_mul_noalloc_async")
        return out

    def mul(self, A, B, e: int, f: int, out=None, stream=None):
        out = self.mul_async(A, B, e, f, out=out, stream=stream)
        self.sync(stream)
        return out

    def mul_add_async(self, A, B, C, e: int, f: int, stream=None):
        """C += A * B (in place)."""
        _check_elem(A, e, "A")
        _check_elem(B, e, "B")
        _check_elem(C, e, "C")
        a, b, c = mat(A), mat(B), mat(C)
        _check(lib().gf2e_mul_add_async(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                        e, f, _stream_handle(stream)), "gf2e_mul_add_async")
        return C

    def mul_add(self, A, B, C, e: int, f: int, stream=None):
        self.mul_add_async(A, B, C, e, f, stream=stream)
        self.sync(stream)
        return C

    # -- triangular solving ---------------------------------------------------
    def trsm_async(self, T, B, e: int, f: int, lower: bool = False, unit: bool = False, stream=None):
        """B <- T^{-1} B in place, T triangular (see gf2e_trsm_async)."""
        _check_elem(T, e, "T")
        _check_elem(B, e, "B")
        t, b = mat(T), mat(B)
        _check(lib().gf2e_trsm_async(self.handle, 1 if lower else 0, 1 if unit else 0, ctypes.byref(t),
                                     ctypes.byref(b), e, f, _stream_handle(stream)), "gf2e_trsm_async")
        return B

    def trsm(self, T, B, e: int, f: int, lower: bool = False, unit: bool = False, stream=None):
        self.trsm_async(T, B, e, f, lower=lower, unit=unit, stream=stream)
        self.sync(stream)
        return B

    # -- echelon forms ----------------------------------------------------------
    def echelonize(self, A, e: int, f: int, full: bool = True):
        """Row echelon form of A in place (reduced when full); returns
        (rank, pivot columns as a list)."""
        _check_elem(A, e, "A")
        a = mat(A)
        rank = ctypes.c_int64(0)
        piv = (ctypes.c_int64 * max(1, min(A.size(0), A.size(1))))()
        _check(lib().gf2e_echelonize(self.handle, ctypes.byref(a), e, f, 1 if full else 0, ctypes.byref(rank),
                                     ctypes.cast(piv, ctypes.c_void_p)), "gf2e_echelonize")
        r = int(rank.value)
        return r, [int(piv[t]) for t in range(r)]

    def ple(self, A, e: int, f: int, L=None):
        """PLE decomposition in place (gf2e_ple): A becomes E; returns
        (L, P as a list, Q as a list, rank) with input row P[i] = (L E)[i]."""
        _check_elem(A, e, "A")
        m, n = A.size(0), A.size(1)
        if L is None:
            L = torch.empty((m, min(m, n)), dtype=A.dtype, device=A.device)
        _check_elem(L, e, "L")
        a, l = mat(A), mat(L)
        rank = ctypes.c_int64(0)
        P = (ctypes.c_int64 * max(1, m))()
        Q = (ctypes.c_int64 * max(1, min(m, n)))()
        _check(lib().gf2e_ple(self.handle, ctypes.byref(a), ctypes.byref(l), e, f, ctypes.byref(rank),
                              ctypes.cast(P, ctypes.c_void_p), ctypes.cast(Q, ctypes.c_void_p)), "gf2e_ple")
        r = int(rank.value)
        return L, [int(P[i]) for i in range(m)], [int(Q[t]) for t in range(r)], r

    # -- batched -------------------------------------------------------------
    def _batch_args(self, As, Bs, Cs, es, fs):
        n = len(As)
        if not (len(Bs) == len(Cs) == len(es) == len(fs) == n):
            raise ValueError("batch lists differ in length")
        for i in range(n):
            _check_elem(As[i], es[i], f"A[{i}]")
            _check_elem(Bs[i], es[i], f"B[{i}]")
            _check_elem(Cs[i], es[i], f"C[{i}]")
        MA = (Mat * max(n, 1))(*[mat(t) for t in As])
        MB = (Mat * max(n, 1))(*[mat(t) for t in Bs])
        MC = (Mat * max(n, 1))(*[mat(t) for t in Cs])
        E = (ctypes.c_int * max(n, 1))(*es)
        F = (ctypes.c_uint32 * max(n, 1))(*fs)
        return n, MA, MB, MC, E, F

    def mul_batched_async(self, As, Bs, es, fs, outs=None, stream=None):
        """C[p] = A[p] * B[p] over F_2^e[p] for every p: one graph launch."""
        if outs is None:
            outs = [torch.empty((a.size(0), b.size(1)), dtype=a.dtype, device=a.device)
                    for a, b in zip(As, Bs)]
        n, MA, MB, MC, E, F = self._batch_args(As, Bs, outs, es, fs)
        _check(lib().gf2e_mul_batched(self.handle, n, MA, MB, MC, E, F, _stream_handle(stream)),
               "gf2e_mul_batched")
        return outs

    def prepare_batched(self, As, Bs, es, fs, outs=None) -> "PreparedBatch":
        """The marshalled arguments of one batch, to launch it again and again
        (the library replays its cached graph for the same descriptors)."""
        if outs is None:
            outs = [torch.empty((a.size(0), b.size(1)), dtype=a.dtype, device=a.device)
                    for a, b in zip(As, Bs)]
        return PreparedBatch(self, As, Bs, outs, self._batch_args(As, Bs, outs, es, fs))

    def mul_batched(self, As, Bs, es, fs, outs=None, stream=None):
        outs = self.mul_batched_async(As, Bs, es, fs, outs=outs, stream=stream)
        self.sync(stream)
        return outs

    def tune_batched(self, As, Bs, es, fs, outs, stream=None):
        n, MA, MB, MC, E, F = self._batch_args(As, Bs, outs, es, fs)
        _check(lib().gf2e_tune_batched(self.handle, n, MA, MB, MC, E, F, _stream_handle(stream)),
               "gf2e_tune_batched")

    def set_batch_threshold(self, min_dim: int):
        _check(lib().gf2e_set_batch_threshold(self.handle, min_dim), "gf2e_set_batch_threshold")

    def set_batch_fusion(self, on: bool):
        """gf2e_set_batch_fusion: fused recombination in the batched 128x128 class."""
        _check(lib().gf2e_set_batch_fusion(self.handle, 1 if on else 0), "gf2e_set_batch_fusion")

    def batch_info(self) -> dict:
        st = BatchStats()
        _check(lib().gf2e_batch_info(self.handle, ctypes.byref(st)), "gf2e_batch_info")
        return {k: getattr(st, k) for k, _ in BatchStats._fields_}

    # -- stages --------------------------------------------------------------
    def slice_a(self, A, e, f, planes, Mp, K64p, stream=None):
        a = mat(A)
        _check(lib().gf2e_slice_a(self.handle, ctypes.byref(a), e, f, ctypes.c_void_p(planes.data_ptr()),
                                  Mp, K64p, _stream_handle(stream)), "gf2e_slice_a")

    def slice_b(self, B, e, f, planes, Np, K64p, stream=None):
        b = mat(B)
        _check(lib().gf2e_slice_b(self.handle, ctypes.byref(b), e, f, ctypes.c_void_p(planes.data_ptr()),
                                  Np, K64p, _stream_handle(stream)), "gf2e_slice_b")

    def plane_products(self, kernel, t, a_planes, b_planes, p_planes, m, n, Mp, Np, K64p,
                       stream=None):
        _check(lib().gf2e_plane_products(self.handle, kernel, t, ctypes.c_void_p(a_planes.data_ptr()),
                                         ctypes.c_void_p(b_planes.data_ptr()),
                                         ctypes.c_void_p(p_planes.data_ptr()), m, n, Mp, Np, K64p,
                                         _stream_handle(stream)), "gf2e_plane_products")

    def combine(self, e, f, p_planes, Mp, Np, C, stream=None):
        c = mat(C)
        _check(lib().gf2e_combine(self.handle, e, f, ctypes.c_void_p(p_planes.data_ptr()), Mp, Np,
                                  ctypes.byref(c), _stream_handle(stream)), "gf2e_combine")

    # -- kernels, tuning, timers --------------------------------------------
    def set_kernel(self, kernel: int):
        _check(lib().gf2e_set_kernel(self.handle, kernel), "gf2e_set_kernel")

    def chosen_kernel(self, e, f, m, k, n) -> int:
        rc = lib().gf2e_chosen_kernel(self.handle, e, f, m, k, n)
        if rc < 0:
            raise GF2EError(rc, "gf2e_chosen_kernel")
        return rc

    def tune(self, e, f, m, k, n, stream=None):
        _check(lib().gf2e_tune(self.handle, e, f, m, k, n, _stream_handle(stream)), "gf2e_tune")

    def set_form(self, form: int):
        """FORM_AUTO, FORM_SCHEDULE or FORM_ALPHA (see gf2e_set_form)."""
        _check(lib().gf2e_set_form(self.handle, form), "gf2e_set_form")

    def chosen_form(self, e, f, m, k, n) -> int:
        rc = lib().gf2e_chosen_form(self.handle, e, f, m, k, n)
        if rc < 0:
            raise GF2EError(rc, "gf2e_chosen_form")
        return rc

    def profile(self, enable: bool = True):
        _check(lib().gf2e_profile(self.handle, 1 if enable else 0), "gf2e_profile")

    def profile_read(self, stage: int):
        ms = ctypes.c_double(0)
        n = ctypes.c_int64(0)
        _check(lib().gf2e_profile_read(self.handle, stage, ctypes.byref(ms), ctypes.byref(n)),
               "gf2e_profile_read")
        return ms.value, n.value

    def profile_reset(self):
        _check(lib().gf2e_profile_reset(self.handle), "gf2e_profile_reset")

    def workspace_bytes(self) -> int:
        return int(lib().gf2e_workspace_bytes(self.handle))


_default_ctx = {}


def default_context(device: int = None) -> Context:
    if device is None:
        device = torch.cuda.current_device()
    ctx = _default_ctx.get(device)
    if ctx is None:
        ctx = _default_ctx[device] = Context(device)
    return ctx


def mul(A, B, e: int, f: int, out=None, stream=None):
    """C = A * B over F_2[x]/<f> (blocking; raises on entries >= 2^e)."""
    return default_context(A.device.index).mul(A, B, e, f, out=out, stream=stream)


def mul_async(A, B, e: int, f: int, out=None, stream=None):
    return default_context(A.device.index).mul_async(A, B, e, f, out=out, stream=stream)


class Server:
    """Continuous-batching request loop (see gf2e_server_* in include/gf2e.h)."""

    def __init__(self, ctx: Context, memory_budget: int = 4 << 30, max_inflight: int = 64,
                 quantum_macs: int = 1 << 40, max_items_per_iteration: int = 0,
                 bypass_limit: int = 0):
        self.ctx = ctx
        cfg = ServerConfig(memory_budget, max_inflight, quantum_macs, max_items_per_iteration,
                           bypass_limit)
        h = ctypes.c_void_p()
        _check(lib().gf2e_server_create(ctx.handle, ctypes.byref(cfg), ctypes.byref(h)),
               "gf2e_server_create")
        self.handle = h
        self._keep = {}

    def close(self):
        if getattr(self, "handle", None):
            lib().gf2e_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, A, B, e: int, f: int, out=None, stream=None) -> int:
        """Queue A*B; the server reads A and B after the work already enqueued
        on `stream` (default: torch's current stream)."""
        _check_elem(A, e, "A")
        _check_elem(B, e, "B")
        if out is None:
            out = torch.empty((A.size(0), B.size(1)), dtype=A.dtype, device=A.device)
        t = ctypes.c_uint64(0)
        a, b, c = mat(A), mat(B), mat(out)
        _check(lib().gf2e_server_submit(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                        e, f, _stream_handle(stream), ctypes.byref(t)), "gf2e_server_submit")
        self._keep[t.value] = (A, B, out)  # tensors stay alive until waited for
        return t.value

    def wait(self, ticket: int):
        """(output tensor, times dict); raises on a failed request."""
        tm = ReqTimes()
        rc = lib().gf2e_server_wait(self.handle, ticket, ctypes.byref(tm))
        A, B, out = self._keep.pop(ticket, (None, None, None))
        _check(rc, "gf2e_server_wait")
        return out, {k: getattr(tm, k) for k, _ in ReqTimes._fields_}

    def stats(self) -> dict:
        st = ServerCounters()
        _check(lib().gf2e_server_stats(self.handle, ctypes.byref(st)), "gf2e_server_stats")
        return {k: getattr(st, k) for k, _ in ServerCounters._fields_}

    def run_trace(self, As, Bs, Cs, es, fs, arrival_s, stream=None):
        """Open-loop run: request i submitted at arrival_s[i] s; per-request times."""
        n = len(As)
        MA = (Mat * max(n, 1))(*[mat(t) for t in As])
        MB = (Mat * max(n, 1))(*[mat(t) for t in Bs])
        MC = (Mat * max(n, 1))(*[mat(t) for t in Cs])
        E = (ctypes.c_int * max(n, 1))(*es)
        F = (ctypes.c_uint32 * max(n, 1))(*fs)
        T = (ctypes.c_double * max(n, 1))(*[float(x) for x in arrival_s])
        out = (ReqTimes * max(n, 1))()
        rc = lib().gf2e_server_run_trace(self.handle, n, MA, MB, MC, E, F, T, _stream_handle(stream), out)
        _check(rc, "gf2e_server_run_trace")
        return [{k: getattr(out[i], k) for k, _ in ReqTimes._fields_} for i in range(n)]
