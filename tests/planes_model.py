"""numpy models of the documented bit-plane layouts (tests only).

They restate the layouts of include/gf2e.h so that each HIP stage can be
checked on its own: operand planes (Karatsuba sums of slices, Section 3.2 and
Section 5), GF(2) plane products, and the recombination/reduction/clinging
step.  The expected values come from these definitions, never from the GPU.
"""
import numpy as np


def bits_of(M, e):
    """(rows, cols, e) array of the coefficient bits of every element."""
    M = np.asarray(M).astype(np.int64)
    return (M[..., None] >> np.arange(e)) & 1


def pack_rows(bits, words):
    """bits: (rows, L) 0/1 -> (rows, words) uint64, bit b of word w = column 64w+b."""
    rows, L = bits.shape
    padded = np.zeros((rows, words * 64), dtype=np.uint64)
    padded[:, :L] = bits
    weights = np.left_shift(np.uint64(1), np.arange(64, dtype=np.uint64))
    return (padded.reshape(rows, words, 64) * weights).sum(axis=2, dtype=np.uint64)


def unpack_rows(words_arr, L):
    rows, words = words_arr.shape
    b = (words_arr[:, :, None] >> np.arange(64, dtype=np.uint64)) & np.uint64(1)
    return b.reshape(rows, words * 64)[:, :L].astype(np.int64)


def operand_planes_a(A, e, u, Mp, K64p):
    """Expected A-side planes: shape (t, K64p, Mp) uint64."""
    m, k = A.shape
    bits = bits_of(A, e)  # m, k, e
    out = np.zeros((len(u), K64p, Mp), dtype=np.uint64)
    for s, mask in enumerate(u):
        sel = [i for i in range(e) if (mask >> i) & 1]
        op = np.bitwise_xor.reduce(bits[:, :, sel], axis=2) if sel else np.zeros((m, k), np.int64)
        out[s, :, :m] = pack_rows(op, K64p).T
    return out


def b_side_order(words):
    """Swap bits 4g and 4g+2 of every word (the B-side bit order of the
    layout: bits 4g..4g+3 hold k = 4g+2, 4g+1, 4g, 4g+3).  The swap is its
    own inverse, so it also turns B-side words back into k order."""
    w = np.asarray(words, dtype=np.uint64)
    out = w.copy()
    for g in range(16):
        lo, hi = np.uint64(4 * g), np.uint64(4 * g + 2)
        b0 = (w >> lo) & np.uint64(1)
        b2 = (w >> hi) & np.uint64(1)
        out &= ~((np.uint64(1) << lo) | (np.uint64(1) << hi))
        out |= (b0 << hi) | (b2 << lo)
    return out


def operand_planes_b(B, e, v, Np, K64p):
    """Expected B-side planes (columns of B along k, B-side bit order):
    (t, K64p, Np)."""
    return b_side_order(operand_planes_a(np.asarray(B).T, e, v, Np, K64p))


def gf2_products(Ap, Bp, m, n):
    """P_s = Ahat_s Bhat_s^T mod 2 from plane arrays (t, K64p, rows); B-side
    words are read in B-side bit order."""
    t, K64p, _ = Ap.shape
    out = []
    for s in range(t):
        a = unpack_rows(np.ascontiguousarray(Ap[s, :, :m].T), K64p * 64)
        b = unpack_rows(np.ascontiguousarray(b_side_order(Bp[s, :, :n]).T), K64p * 64)
        out.append((a @ b.T) & 1)
    return out


def combine(P_bits, mmap, e):
    """Elements of C from product bit-matrices via the reduced map m."""
    m, n = P_bits[0].shape
    C = np.zeros((m, n), dtype=np.int64)
    for c in range(e):
        acc = np.zeros((m, n), dtype=np.int64)
        for s in range(len(P_bits)):
            if (mmap[c] >> s) & 1:
                acc ^= P_bits[s]
        C |= acc << c
    return C
