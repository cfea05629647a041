"""End-to-end parity of gf2e_mul (GPU) against the CPU oracle.

The bar is bit-exact equality: the product over F_{2^e} is unique and every
step of the path is integer arithmetic.  Every shape is compared in full,
the full-size workloads (4096^3 over F_16, 8192^3 over F_256) too, each in
every kernel the benchmark may time, together with Freivalds' check.
"""
import numpy as np
import pytest
import torch

import oracle
import workload
from tests import fielddef

pytestmark = pytest.mark.gpu

ALL_E = sorted(workload.DEFAULT_POLY.items())


@pytest.fixture(scope="module")
def g():
    import paper_1111_6900_amd as g
    return g


@pytest.fixture(scope="module")
def ctx(g):
    return g.Context(0)


def dev(M, e):
    import paper_1111_6900_amd as g
    return torch.from_numpy(np.ascontiguousarray(M).astype(np.int64)).to(g.elem_dtype(e)).cuda()


def host(t):
    return t.cpu().numpy().astype(np.int64)


def gpu_mul(ctx, A, B, e, f):
    return host(ctx.mul(dev(A, e), dev(B, e), e, f))


def test_config_f4_256_full(ctx):
    e, f, A, B = workload.plain_inputs("f4_256")
    print("f4_256 full", flush=True)
    assert (gpu_mul(ctx, A, B, e, f) == oracle.matmul(A, B, e, f)).all()


@pytest.mark.parametrize("e,f", ALL_E + [(4, 0x1F), (8, 0x11B)])
@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 3, 4), (63, 65, 64), (129, 127, 130),
                                   (257, 300, 255), (64, 1000, 64)])
def test_small_shapes_every_field(ctx, e, f, shape):
    m, k, n = shape
    print(f"mul e={e} f={f:#x} shape={shape}", flush=True)
    gen = np.random.default_rng(e * 131 + m * 7 + k)
    A = workload.field_matrix(gen, m, k, e)
    B = workload.field_matrix(gen, k, n, e)
    assert (gpu_mul(ctx, A, B, e, f) == oracle.matmul(A, B, e, f)).all()


@pytest.mark.parametrize("kind", list(range(9)))
@pytest.mark.parametrize("e", [2, 5, 8, 10])
def test_every_product_kernel(g, e, kind):
    f = workload.DEFAULT_POLY[e]
    print(f"kernel {kind} e={e}", flush=True)
    c = g.Context(0, kernel=kind)
    gen = np.random.default_rng(kind * 10 + e)
    A = workload.field_matrix(gen, 300, 517, e)
    B = workload.field_matrix(gen, 517, 270, e)
    assert (gpu_mul(c, A, B, e, f) == oracle.matmul(A, B, e, f)).all()
    c.close()


@pytest.fixture(scope="module")
def actx(g):
    """A context that always takes the alpha-power form."""
    c = g.Context(0)
    c.set_form(g.FORM_ALPHA)
    yield c
    c.close()


@pytest.mark.parametrize("e,f", ALL_E + [(4, 0x1F), (8, 0x11B)])
@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 3, 4), (63, 65, 64), (129, 127, 130), (257, 300, 255)])
def test_alpha_form_small_shapes(actx, e, f, shape):
    m, k, n = shape
    print(f"alpha form e={e} f={f:#x} shape={shape}", flush=True)
    gen = np.random.default_rng(e * 17 + m * 3 + k)
    A = workload.field_matrix(gen, m, k, e)
    B = workload.field_matrix(gen, k, n, e)
    assert (gpu_mul(actx, A, B, e, f) == oracle.matmul(A, B, e, f)).all()


@pytest.mark.parametrize("kind", list(range(9)))
@pytest.mark.parametrize("e", [2, 4, 7])
def test_alpha_form_every_kernel(g, e, kind):
    f = workload.DEFAULT_POLY[e]
    print(f"alpha form kernel {kind} e={e}", flush=True)
    c = g.Context(0, kernel=kind)
    c.set_form(g.FORM_ALPHA)
    gen = np.random.default_rng(kind * 10 + e + 1000)
    A = workload.field_matrix(gen, 300, 517, e)
    B = workload.field_matrix(gen, 517, 270, e)
    assert c.chosen_form(e, f, 300, 517, 270) == g.FORM_ALPHA
    assert (gpu_mul(c, A, B, e, f) == oracle.matmul(A, B, e, f)).all()
    c.close()


@pytest.mark.parametrize("e,f", ALL_E + [(5, 0x29), (8, 0x11B), (11, 0x805)])
def test_alpha_form_clinging_in_the_product(g, e, f):
    """The alpha form on an fp4 kernel clings its result in the product's
    epilogue (e <= 10; e = 11 takes the separate combining pass): C = A*B and
    C += A*B against the oracle, for k of one word per block (even and odd e),
    two words, and several 256-bit stages, with ragged m and n."""
    c = g.Context(0, kernel=g.KERNEL_FP4_128)
    c.set_form(g.FORM_ALPHA)
    gen = np.random.default_rng(e * 7 + f)
    for m, k, n in [(1, 1, 1), (70, 33, 150), (129, 64, 257), (200, 65, 64), (256, 128, 131), (131, 300, 190)]:
        assert c.chosen_form(e, f, m, k, n) == g.FORM_ALPHA
        A = workload.field_matrix(gen, m, k, e)
        B = workload.field_matrix(gen, k, n, e)
        want = oracle.matmul(A, B, e, f)
        assert (gpu_mul(c, A, B, e, f) == want).all(), (m, k, n)
        C0 = workload.field_matrix(gen, m, n, e)
        Cd = dev(C0, e)
        c.mul_add(dev(A, e), dev(B, e), Cd, e, f)
        assert (host(Cd) == (C0 ^ want)).all(), (m, k, n)
    c.close()


def test_alpha_form_falls_back_from_fp4_past_its_count_limit(g):
    """The alpha form's product has e*k bits of inner dimension, so the fp4
    kernels (exact below 2^24) are replaced by the int8 kernel earlier."""
    c = g.Context(0, kernel=g.KERNEL_FP4_128)
    k = 2**22 + 1
    assert c.chosen_kernel(4, 0x13, 64, k, 64) == g.KERNEL_FP4_128
    c.set_form(g.FORM_ALPHA)
    assert c.chosen_kernel(4, 0x13, 64, k, 64) == g.KERNEL_MFMA_256_W8
    assert c.chosen_kernel(4, 0x13, 64, 2**21, 64) == g.KERNEL_FP4_128
    c.close()


def test_autotuned_form_is_exact_and_leaves_inputs_alone(g):
    c = g.Context(0, autotune=True)
    for name in ["f4_256"]:
        e, f, A, B = workload.plain_inputs(name)
        m, k, n = A.shape[0], A.shape[1], B.shape[1]
        Ad, Bd = dev(A, e), dev(B, e)
        c.tune(e, f, m, k, n)
        form = c.chosen_form(e, f, m, k, n)
        print(f"{name}: tuned form {form}, kernel {c.chosen_kernel(e, f, m, k, n)}", flush=True)
        assert form in (g.FORM_SCHEDULE, g.FORM_ALPHA)
        assert (host(Ad) == A).all() and (host(Bd) == B).all()
        assert (host(c.mul(Ad, Bd, e, f)) == oracle.matmul(A, B, e, f)).all()
        # forcing either form after tuning keeps the result
        for fm in (g.FORM_SCHEDULE, g.FORM_ALPHA):
            c.set_form(fm)
            assert (host(c.mul(Ad, Bd, e, f)) == oracle.matmul(A, B, e, f)).all()
        c.set_form(g.FORM_AUTO)
    c.close()


def test_brute_force_all_2x2_over_f4(ctx):
    mats = np.array(np.meshgrid(*[np.arange(4)] * 4, indexing="ij")).reshape(4, -1).T.reshape(-1, 2, 2)
    A = mats.reshape(-1, 2)
    B = mats.transpose(1, 0, 2).reshape(2, -1)
    assert (gpu_mul(ctx, A, B, 2, 0x7) == oracle.matmul(A, B, 2, 0x7)).all()


@pytest.mark.parametrize("e,f", ALL_E + [(4, 0x1F), (8, 0x11B)])
def test_multiplication_table_probe(ctx, e, f):
    """A = column of all field elements, B = row of all elements: C is the
    full multiplication table."""
    s = np.arange(1 << e)
    C = gpu_mul(ctx, s[:, None], s[None, :], e, f)
    assert (C == oracle.mul_table(e, f)).all()
    assert (C == fielddef.table(e, f)).all()


@pytest.mark.parametrize("k", [1, 2, 63, 64, 65, 128, 129, 2**20 + 1])
def test_large_k_parity(ctx, k):
    """1 x k ones times k x 1 ones over F_4 is k mod 2 (characteristic 2)."""
    A = np.ones((1, k), dtype=np.uint8)
    B = np.ones((k, 1), dtype=np.uint8)
    assert gpu_mul(ctx, A, B, 2, 0x7)[0, 0] == k % 2


@pytest.mark.parametrize("kind", [6, 7, 8])
@pytest.mark.parametrize("k", [2**23 - 64, 2**23, 2**23 + 1, 2**24 + 1])
def test_fp4_count_limit(g, kind, k):
    """The fp4 kernels keep exact f32 counts (biased by 2^23) for k up to
    2^23; beyond that the plain path falls back to the int8 kernel and stays
    exact."""
    c = g.Context(0, kernel=kind)
    A = np.ones((1, k), dtype=np.uint8)
    B = np.ones((k, 1), dtype=np.uint8)
    assert gpu_mul(c, A, B, 2, 0x7)[0, 0] == k % 2
    c.close()


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("e", [3, 8, 13])
def test_short_k_products(g, e, form):
    """Products with k <= 128 pad k to 128 bits and run on the kernel with
    128-bit stages, whatever kernel is forced; the result stays exact for
    ragged m, n and every k up to 129."""
    f = {**workload.DEFAULT_POLY, **workload.WIDE_POLY}[e]
    c = g.Context(0, kernel=g.KERNEL_MFMA_256)
    c.set_form(form)
    gen = np.random.default_rng(e * 7 + form)
    for k in (1, 64, 65, 127, 128, 129):
        print(f"short k e={e} form={form} k={k}", flush=True)
        # the alpha form's product has e * K64p words of k: a multiple of 4
        # words, which every kernel steps, when e is even
        short = k <= 128 and (form == g.FORM_SCHEDULE or e % 2 == 1)
        expect = g.KERNEL_FP4_128_PLANES if short else g.KERNEL_MFMA_256
        assert c.chosen_kernel(e, f, 300, k, 400) == expect
        A = workload.field_matrix(gen, 300, k, e)
        B = workload.field_matrix(gen, k, 400, e)
        assert (gpu_mul(c, A, B, e, f) == oracle.matmul(A, B, e, f)).all()
    c.close()


def test_char2_cancellation(ctx):
    gen = np.random.default_rng(3)
    a = workload.field_matrix(gen, 40, 1, 8)
    b = workload.field_matrix(gen, 1, 50, 8)
    A = np.concatenate([a, a], axis=1)
    B = np.concatenate([b, b], axis=0)
    assert (gpu_mul(ctx, A, B, 8, 0x11D) == 0).all()


@pytest.mark.parametrize("e", [3, 8, 10])
def test_invariants(ctx, e):
    f = workload.DEFAULT_POLY[e]
    gen = np.random.default_rng(e + 50)
    A = workload.field_matrix(gen, 70, 90, e)
    B = workload.field_matrix(gen, 90, 80, e)
    B2 = workload.field_matrix(gen, 90, 80, e)
    D = workload.field_matrix(gen, 80, 60, e)
    mm = lambda X, Y: gpu_mul(ctx, X, Y, e, f)
    assert (mm(A, np.eye(90, dtype=np.int64)) == A).all()
    assert (mm(mm(A, B), D) == mm(A, mm(B, D))).all()
    assert (mm(A, B ^ B2) == (mm(A, B) ^ mm(A, B2))).all()
    assert (mm(B.T, A.T) == mm(A, B).T).all()
    sq = fielddef.table(e, f)[np.arange(1 << e), np.arange(1 << e)]
    assert (sq[mm(A, B)] == mm(sq[A], sq[B])).all()
    xI = 2 * np.eye(90, dtype=np.int64)
    assert (mm(xI, B) == fielddef.mul(B, 2, e, f)).all()


def test_subfield_f4_in_f16(ctx):
    T16 = fielddef.table(4, 0x13)
    w = 1
    for _ in range(5):
        w = int(T16[w, 2])
    emb = np.array([0, 1, w, w ^ 1])
    gen = np.random.default_rng(9)
    A = workload.field_matrix(gen, 100, 77, 2)
    B = workload.field_matrix(gen, 77, 90, 2)
    C4 = gpu_mul(ctx, A, B, 2, 0x7)
    assert (gpu_mul(ctx, emb[A], emb[B], 4, 0x13) == emb[C4]).all()


def test_leading_dimension_and_offsets(ctx):
    e, f = 8, 0x11D
    gen = np.random.default_rng(12)
    big_a = workload.field_matrix(gen, 120, 200, e)
    big_b = workload.field_matrix(gen, 150, 180, e)
    Ad, Bd = dev(big_a, e), dev(big_b, e)
    A = Ad[3:103, 5:150]          # ld 200, unaligned start
    B = Bd[2:147, 1:171]          # ld 180
    Cbig = torch.zeros((110, 190), dtype=torch.uint8, device="cuda")
    C = Cbig[4:104, 7:177]
    ctx.mul(A, B, e, f, out=C)
    want = oracle.matmul(big_a[3:103, 5:150], big_b[2:147, 1:171], e, f)
    got = host(Cbig)
    assert (got[4:104, 7:177] == want).all()
    mask = np.ones_like(got, dtype=bool)
    mask[4:104, 7:177] = False
    assert (got[mask] == 0).all()  # nothing written outside C


def test_empty_and_k_zero(g, ctx):
    e, f = 4, 0x13
    A = torch.zeros((0, 5), dtype=torch.uint8, device="cuda")
    B = torch.zeros((5, 7), dtype=torch.uint8, device="cuda")
    assert ctx.mul(A, B, e, f).shape == (0, 7)
    A = torch.zeros((6, 0), dtype=torch.uint8, device="cuda")
    B = torch.zeros((0, 7), dtype=torch.uint8, device="cuda")
    C = torch.full((6, 7), 9, dtype=torch.uint8, device="cuda")
    ctx.mul(A, B, e, f, out=C)
    assert (host(C) == 0).all()


def test_zero_f_rejected_at_every_entry_point(g, ctx):
    """Section 2: f is irreducible of degree e, so f = 0 is rejected before
    anything is enqueued, by the plain, batched and served entry points."""
    A = dev(np.full((8, 8), 3), 8)
    for e in (8, 2, 4):
        with pytest.raises(g.GF2EError) as ei:
            ctx.mul(A, A, e, 0)
        assert ei.value.code == g.EFIELD
    with pytest.raises(g.GF2EError) as ei:
        ctx.mul_batched([A, A], [A, A], [8, 8], [0x11D, 0])
    assert ei.value.code == g.EFIELD
    srv = g.Server(ctx, memory_budget=64 << 20, max_inflight=2)
    with pytest.raises(g.GF2EError) as ei:
        srv.submit(A, A, 8, 0)
    assert ei.value.code == g.EFIELD
    srv.close()
    # a valid field still works afterwards
    assert (host(ctx.mul(A, A, 8, 0x11D)) == oracle.matmul(host(A), host(A), 8, 0x11D)).all()


def test_errors(g, ctx):
    e, f = 4, 0x13
    A = dev(np.full((10, 10), 3), e)
    B = dev(np.full((10, 12), 3), e)
    with pytest.raises(g.GF2EError) as ei:
        ctx.mul(A, B, e, 0x11)                      # reducible f
    assert ei.value.code == g.EFIELD
    with pytest.raises(g.GF2EError) as ei:
        ctx.mul(A, B, 17, 0x20009)                  # e out of range
    assert ei.value.code == g.EFIELD
    with pytest.raises(g.GF2EError) as ei:
        ctx.mul(A, dev(np.ones((9, 12)), e), e, f)  # inner dimensions
    assert ei.value.code == g.ESHAPE
    with pytest.raises(g.GF2EError) as ei:
        ctx.mul(A, A, e, f, out=A)                  # C aliases A
    assert ei.value.code == g.EALIAS
    bad = A.clone()
    bad[3, 4] = 16                                  # not in F_16
    with pytest.raises(g.GF2EError) as ei:
        ctx.mul(bad, B, e, f)
    assert ei.value.code == g.ERANGE
    badw = dev(np.full((4, 4), 5), 10)
    badw[1, 1] = 1024
    with pytest.raises(g.GF2EError) as ei:
        ctx.mul(badw, dev(np.ones((4, 4)), 10), 10, 0x409)
    assert ei.value.code == g.ERANGE
    # the flag is cleared once reported
    assert (host(ctx.mul(A, B, e, f)) == oracle.matmul(host(A), host(B), e, f)).all()


def test_side_stream_and_async(g, ctx):
    e, f = 8, 0x11D
    gen = np.random.default_rng(21)
    A = workload.field_matrix(gen, 300, 400, e)
    B = workload.field_matrix(gen, 400, 200, e)
    Ad, Bd = dev(A, e), dev(B, e)
    s = torch.cuda.Stream()
    outs = []
    with torch.cuda.stream(s):
        for _ in range(3):
            outs.append(ctx.mul_async(Ad, Bd, e, f, stream=s))
    ctx.sync(s)
    want = oracle.matmul(A, B, e, f)
    for o in outs:
        assert (host(o) == want).all()
    # back on the default stream with the same context
    assert (host(ctx.mul(Ad, Bd, e, f)) == want).all()


_FULL = {}


def _full_oracle(name):
    """(e, f, A, B, C) of a plain workload with C the whole oracle product
    (all host threads), computed once per session."""
    if name not in _FULL:
        e, f, A, B = workload.plain_inputs(name)
        print(f"{name}: full oracle product", flush=True)
        _FULL[name] = (e, f, A, B, oracle.matmul(A, B, e, f))
    return _FULL[name]


def _full_size_check(ctx, name, kinds):
    """Every kernel's C compared with the full oracle product, entry by
    entry, and Freivalds' check with ceil(64/e) trials (a wrong C passes
    with probability at most 2^-64)."""
    e, f, A, B, want = _full_oracle(name)
    n = B.shape[1]
    Ad, Bd = dev(A, e), dev(B, e)
    R = workload.freivalds_vectors(np.random.default_rng(99), n, e)
    assert R.shape[1] == -(-64 // e)
    for kind in kinds:
        print(f"{name} kernel={kind}", flush=True)
        ctx.set_kernel(kind)
        C = ctx.mul(Ad, Bd, e, f).cpu().numpy()
        bad = np.count_nonzero(C != want)
        assert bad == 0, (kind, bad)
        assert oracle.freivalds(A, B, C, e, f, R) == 0, kind
    ctx.set_kernel(-1)


def test_config_f16_4096_full(ctx):
    _full_size_check(ctx, "f16_4096", [-1, 0, 4, 5, 6])


def test_config_f16_4096_full_alpha_form(actx):
    _full_size_check(actx, "f16_4096", [-1, 5, 7])


def test_config_f256_8192_full(ctx):
    """The benchmark's workload, in the launch configurations it may time."""
    _full_size_check(ctx, "f256_8192", [-1, 0, 1, 2, 3, 4, 5, 6, 7])
