"""CPU oracle for dense matrix multiplication over F_{2^e} -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU product path shares no code
with it and never calls it.

The arithmetic lives in ``gf2e_oracle.c`` (plain C + OpenMP, built into
``liboracle.so`` next to this file); this module only marshals numpy arrays.
What each entry point follows in the M4RIE paper:

* field product: Section 2 (elements are polynomials of degree < e over F_2,
  identified with the integer sum a_i 2^i; arithmetic modulo an irreducible f);
* ``matmul``: Section 4, Algorithm 1 (cubic multiplication), read as
  C_i += A[i][l] * B_l;
* ``freivalds``: a randomized check A (B R) == C R with caller-drawn R.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SOURCE = os.path.join(_HERE, "gf2e_oracle.c")

_lib = None


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with gcc (plain C, OpenMP)."""
    import subprocess

    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-Wall", "-Wextra",
           "-o", LIB_PATH + ".tmp", SOURCE]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    lib = ctypes.CDLL(LIB_PATH)
    i64, u32, i32, vp = ctypes.c_int64, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p
    lib.gf2e_oracle_is_irreducible.argtypes = [i32, u32]
    lib.gf2e_oracle_is_primitive.argtypes = [i32, u32]
    lib.gf2e_oracle_mul_def.argtypes = [i32, u32, u32, u32]
    lib.gf2e_oracle_mul_def.restype = u32
    lib.gf2e_oracle_order.argtypes = [i32, u32, u32]
    lib.gf2e_oracle_order.restype = u32
    lib.gf2e_oracle_tables.argtypes = [i32, u32, ctypes.POINTER(u32), vp]
    lib.gf2e_oracle_mul_table_all.argtypes = [i32, u32, vp]
    lib.gf2e_oracle_matmul.argtypes = [i32, u32, i64, i64, i64, vp, i64, vp, i64, vp, i64,
                                       i64, i64, i32]
    lib.gf2e_oracle_entries.argtypes = [i32, u32, i64, i64, i64, vp, i64, vp, i64, vp, vp,
                                        i64, vp, i32]
    lib.gf2e_oracle_freivalds.argtypes = [i32, u32, i64, i64, i64, vp, i64, vp, i64, vp, i64,
                                          vp, i64, i32]
    lib.gf2e_oracle_freivalds.restype = i64
    lib.gf2e_oracle_max_threads.restype = i32
    lib.gf2e_oracle_trsm.argtypes = [i32, u32, i32, i32, i64, i64, vp, i64, vp, i64, i32]
    lib.gf2e_oracle_echelon.argtypes = [i32, u32, i32, i64, i64, vp, i64, vp, vp]
    lib.gf2e_oracle_ple.argtypes = [i32, u32, i64, i64, vp, i64, vp, i64, vp, vp, vp]
    _lib = lib
    return lib


class OracleError(RuntimeError):
    pass


def _check(rc):
    if rc != 0:
        raise OracleError(f"oracle returned error code {rc}")


def elem_dtype(e: int):
    """Storage type of one element: uint8 for e <= 8, uint16 for e = 9, 10."""
    return np.uint8 if e <= 8 else np.uint16


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _as_field_matrix(M, e):
    M = np.ascontiguousarray(M)
    if M.dtype != elem_dtype(e):
        M = M.astype(elem_dtype(e))
    return M


def is_irreducible(e: int, f: int) -> bool:
    return bool(_load().gf2e_oracle_is_irreducible(e, f))


def is_primitive(e: int, f: int) -> bool:
    return bool(_load().gf2e_oracle_is_primitive(e, f))


def mul_def(e: int, f: int, a: int, b: int) -> int:
    """a*b in F_2[x]/<f> by shift-and-add then long division (Section 2)."""
    return int(_load().gf2e_oracle_mul_def(e, f, a, b))


def order(e: int, f: int, a: int) -> int:
    return int(_load().gf2e_oracle_order(e, f, a))


def generator(e: int, f: int) -> int:
    g = ctypes.c_uint32(0)
    _check(_load().gf2e_oracle_tables(e, f, ctypes.byref(g), None))
    return int(g.value)


def antilog(e: int, f: int) -> np.ndarray:
    q = (1 << e) - 1
    out = np.zeros(q, dtype=np.uint16)
    _check(_load().gf2e_oracle_tables(e, f, None, _ptr(out)))
    return out


def mul_table(e: int, f: int) -> np.ndarray:
    """Full 2^e x 2^e product table computed through the log/antilog tables."""
    s = 1 << e
    out = np.zeros((s, s), dtype=np.uint16)
    _check(_load().gf2e_oracle_mul_table_all(e, f, _ptr(out)))
    return out


def matmul(A, B, e: int, f: int, rows=None, nthreads: int = 0) -> np.ndarray:
    """C = A * B over F_{2^e} by the cubic algorithm.  ``rows=(r0, r1)``
    computes only that row range (the result then has r1 - r0 rows)."""
    A = _as_field_matrix(A, e)
    B = _as_field_matrix(B, e)
    m, k = A.shape
    k2, n = B.shape
    if k != k2:
        raise ValueError("inner dimensions differ")
    r0, r1 = (0, m) if rows is None else rows
    C = np.zeros((m, n), dtype=elem_dtype(e))
    _check(_load().gf2e_oracle_matmul(e, f, m, k, n, _ptr(A), k, _ptr(B), n, _ptr(C), n,
                                      r0, r1, nthreads))
    return C[r0:r1] if rows is not None else C


def entries(A, B, e: int, f: int, I, J, nthreads: int = 0) -> np.ndarray:
    """C[I[s], J[s]] for sampled positions, each by its own dot product."""
    A = _as_field_matrix(A, e)
    B = _as_field_matrix(B, e)
    m, k = A.shape
    _, n = B.shape
    I = np.ascontiguousarray(I, dtype=np.int64)
    J = np.ascontiguousarray(J, dtype=np.int64)
    out = np.zeros(len(I), dtype=np.uint32)
    _check(_load().gf2e_oracle_entries(e, f, m, k, n, _ptr(A), k, _ptr(B), n, _ptr(I),
                                       _ptr(J), len(I), _ptr(out), nthreads))
    return out


def freivalds(A, B, C, e: int, f: int, R, nthreads: int = 0) -> int:
    """Number of rows where A (B R) differs from C R (0 means consistent).
    R is an n x t matrix of field elements drawn by the caller."""
    A = _as_field_matrix(A, e)
    B = _as_field_matrix(B, e)
    C = _as_field_matrix(C, e)
    R = _as_field_matrix(R, e)
    m, k = A.shape
    _, n = B.shape
    if C.shape != (m, n) or R.shape[0] != n:
        raise ValueError("shape mismatch")
    rc = _load().gf2e_oracle_freivalds(e, f, m, k, n, _ptr(A), k, _ptr(B), n, _ptr(C), n,
                                       _ptr(R), R.shape[1], nthreads)
    if rc < 0:
        raise OracleError(f"oracle returned error code {rc}")
    return int(rc)


def trsm(T, B, e: int, f: int, lower: bool = False, unit: bool = False, nthreads: int = 0) -> np.ndarray:
    """X with T X = B for triangular T (Section 4.3's row algorithm); B is
    not modified.  Raises OracleError(-9) for a zero on the diagonal."""
    T = _as_field_matrix(T, e)
    X = _as_field_matrix(B, e).copy()
    m = T.shape[0]
    if T.shape != (m, m) or X.shape[0] != m:
        raise ValueError("shape mismatch")
    n = X.shape[1]
    _check(_load().gf2e_oracle_trsm(e, f, 1 if lower else 0, 1 if unit else 0, m, n, _ptr(T), m,
                                    _ptr(X), n, nthreads))
    return X


def echelon(A, e: int, f: int, full: bool = True):
    """(E, rank, pivots): the row echelon form of A by the elimination loop of
    Section 4.1 (reduced when full), its rank and the pivot column of each of
    its first rank rows.  A is not modified."""
    E = _as_field_matrix(A, e).copy()
    m, n = E.shape
    rank = ctypes.c_int64(0)
    piv = np.zeros(max(min(m, n), 1), dtype=np.int64)
    _check(_load().gf2e_oracle_echelon(e, f, 1 if full else 0, m, n, _ptr(E), n, ctypes.byref(rank),
                                       _ptr(piv)))
    r = int(rank.value)
    return E, r, piv[:r].copy()


def ple(A, e: int, f: int):
    """(P, L, E, Q, rank) with A[P[i]] = sum_t L[i][t] E[t] (A = P L E), by the
    elimination loop of Section 4.1 modified as Section 4.2 describes: L is
    m x min(m, n) lower trapezoidal with the pivots on its diagonal, E is in
    row echelon form with leading 1 in column Q[t] of row t < rank (rows from
    rank on are zero).  A is not modified."""
    E = _as_field_matrix(A, e).copy()
    m, n = E.shape
    mn = min(m, n)
    L = np.zeros((m, max(mn, 1)), dtype=elem_dtype(e))
    P = np.zeros(max(m, 1), dtype=np.int64)
    Q = np.zeros(max(mn, 1), dtype=np.int64)
    rank = ctypes.c_int64(0)
    _check(_load().gf2e_oracle_ple(e, f, m, n, _ptr(E), n, _ptr(L), L.shape[1], _ptr(P), _ptr(Q),
                                   ctypes.byref(rank)))
    r = int(rank.value)
    return P[:m].copy(), L[:, :mn].copy(), E, Q[:r].copy(), r


def max_threads() -> int:
    return int(_load().gf2e_oracle_max_threads())
