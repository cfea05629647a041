"""Independent textbook definitions used to pin the oracle (tests only).

Vectorized numpy versions of the field product of Section 2 (carry-less
multiplication, then reduction modulo f) and of the cubic matrix product.
Nothing here is shared with the oracle's C code or with the GPU library.
"""
import numpy as np


def mul(a, b, e, f):
    """Elementwise a*b in F_2[x]/<f>: shift-and-add, then long division."""
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    r = np.zeros(np.broadcast(a, b).shape, dtype=np.int64)
    for i in range(e):
        r ^= np.where((b >> i) & 1, a << i, 0)
    for d in range(2 * e - 2, e - 1, -1):
        r = np.where((r >> d) & 1, r ^ (f << (d - e)), r)
    return r


def table(e, f):
    s = np.arange(1 << e, dtype=np.int64)
    return mul(s[:, None], s[None, :], e, f)


def matmul(A, B, e, f):
    """Cubic product: C[i, j] = XOR over l of A[i, l] * B[l, j]."""
    T = table(e, f)
    A = np.asarray(A, dtype=np.int64)
    B = np.asarray(B, dtype=np.int64)
    C = np.zeros((A.shape[0], B.shape[1]), dtype=np.int64)
    for l in range(A.shape[1]):
        C ^= T[A[:, l][:, None], B[l][None, :]]
    return C


def poly_rem(a, b):
    db = b.bit_length() - 1
    while a.bit_length() - 1 >= db:
        a ^= b << (a.bit_length() - 1 - db)
    return a


def is_irreducible(e, f):
    """Trial division by every polynomial of degree 1..e/2."""
    if f.bit_length() - 1 != e:
        return False
    return all(poly_rem(f, g) != 0 for g in range(2, 1 << (e // 2 + 1)))


def read_golden(path):
    """Key/value header lines and numeric rows of a tests/golden fixture."""
    meta, rows = {}, []
    with open(path) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            parts = line.split()
            if parts[0].isalpha() or parts[0].startswith("slice") or parts[0] == "packed":
                meta[parts[0]] = [int(x, 0) for x in parts[1:]]
            else:
                rows.append([int(x, 0) for x in parts])
    return meta, rows
