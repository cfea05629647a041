"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module draws random numbers and shapes only; it holds none of the
arithmetic of F_{2^e} multiplication.  Entries are i.i.d. uniform in
{0, ..., 2^e - 1}: the paper measures on random dense matrices (Section 1 and
the captions of Tables 1-4).  One uint8 per element when e <= 8, one uint16
when e is 9 or 10.
"""
from __future__ import annotations

import math

import numpy as np

# Field polynomials, bit e set (x^2+x+1 = 0x7).  e=2 is the polynomial of the
# paper's Karatsuba example (Section 5); the rest are primitive trinomials or
# pentanomials.  Primitivity is verified by the test suite, not assumed.
DEFAULT_POLY = {2: 0x7, 3: 0xB, 4: 0x13, 5: 0x25, 6: 0x43, 7: 0x83, 8: 0x11D,
                9: 0x211, 10: 0x409}
# Fields past the paper's range (its Section 1 footnote: the method extends
# to e <= 16): primitive polynomials x^11+x^2+1, x^12+x^6+x^4+x+1,
# x^13+x^4+x^3+x+1, x^14+x^10+x^6+x+1, x^15+x+1, x^16+x^12+x^3+x+1.
WIDE_POLY = {11: 0x805, 12: 0x1053, 13: 0x201B, 14: 0x4443, 15: 0x8003, 16: 0x1100B}

BASE_SEED = 20260


def elem_dtype(e: int):
    return np.uint8 if e <= 8 else np.uint16


def rng(tag: int, stream: int = 0) -> np.random.Generator:
    """Independent stream `stream` of the seed family `tag`."""
    ss = np.random.SeedSequence(BASE_SEED + int(tag))
    return np.random.default_rng(ss.spawn(stream + 1)[stream])


def field_matrix(gen: np.random.Generator, rows: int, cols: int, e: int) -> np.ndarray:
    """rows x cols matrix with entries uniform in {0..2^e-1}."""
    return gen.integers(0, 1 << e, size=(rows, cols), dtype=elem_dtype(e))


# The three plain-product workloads: (e, f, m, k, n).
PLAIN_CONFIGS = {
    "f4_256": (2, 0x7, 256, 256, 256),
    "f16_4096": (4, 0x13, 4096, 4096, 4096),
    "f256_8192": (8, 0x11D, 8192, 8192, 8192),
}
PLAIN_TAG = {"f4_256": 0, "f16_4096": 1, "f256_8192": 2}


def plain_inputs(name: str):
    """(e, f, A, B) for one of PLAIN_CONFIGS, from its own seed family."""
    e, f, m, k, n = PLAIN_CONFIGS[name]
    tag = PLAIN_TAG[name]
    A = field_matrix(rng(tag, 0), m, k, e)
    B = field_matrix(rng(tag, 1), k, n, e)
    return e, f, A, B


def log_uniform_int(gen: np.random.Generator, lo: int, hi: int, size=None):
    """round(exp(U(ln lo, ln hi))), clipped to [lo, hi]."""
    v = np.exp(gen.uniform(math.log(lo), math.log(hi), size=size))
    return np.clip(np.rint(v), lo, hi).astype(np.int64)


def batch_specs(count: int = 512, lo: int = 32, hi: int = 2048, tag: int = 3):
    """Shapes and fields of the batched workload: e ~ U{2..10}, m, n, k each
    log-uniform in [lo, hi].  Returns a list of (e, f, m, k, n)."""
    g = rng(tag, 0)
    es = g.integers(2, 11, size=count)
    m = log_uniform_int(g, lo, hi, count)
    k = log_uniform_int(g, lo, hi, count)
    n = log_uniform_int(g, lo, hi, count)
    return [(int(e), DEFAULT_POLY[int(e)], int(mm), int(kk), int(nn))
            for e, mm, kk, nn in zip(es, m, k, n)]


def batch_inputs(specs, tag: int = 3):
    """Matrices for batch_specs(...), product p drawn from stream p+1."""
    out = []
    for p, (e, f, m, k, n) in enumerate(specs):
        g = rng(tag, p + 1)
        out.append((field_matrix(g, m, k, e), field_matrix(g, k, n, e)))
    return out


def serve_specs(count: int = 10000, lo: int = 64, hi: int = 4096, tag: int = 4):
    """Serving workload: e ~ U{2..10}, square size log-uniform in [lo, hi].
    Returns a list of (e, f, n)."""
    g = rng(tag, 0)
    es = g.integers(2, 11, size=count)
    ns = log_uniform_int(g, lo, hi, count)
    return [(int(e), DEFAULT_POLY[int(e)], int(n)) for e, n in zip(es, ns)]


def poisson_arrivals(count: int, rate_per_s: float, tag: int = 4) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process with the given rate."""
    g = rng(tag, 1)
    return np.cumsum(g.exponential(1.0 / rate_per_s, size=count))


def freivalds_vectors(gen: np.random.Generator, n: int, e: int, trials=None) -> np.ndarray:
    """n x t matrix of uniform field elements; t = ceil(64/e) by default, so a
    wrong product passes every trial with probability at most 2^-64."""
    t = trials if trials is not None else -(-64 // e)
    return field_matrix(gen, n, t, e)


def serve_pools(specs, tag: int = 4):
    """Input pools of a served workload: for every field in `specs` one pair
    (A, B) of nmax x nmax matrices, nmax the largest request size.  A request
    of size n reads the leading n x n windows of its field's pair (entries
    are uniform in the field either way; the values do not change the work)."""
    gen = rng(tag, 2)
    nmax = max(n for _, _, n in specs)
    return {e: (field_matrix(gen, nmax, nmax, e), field_matrix(gen, nmax, nmax, e))
            for e in sorted({e for e, _, _ in specs})}
