"""Context configuration on the GPU: the workspace limit and the tuning cache.

A context created with a workspace limit reports GF2E_ENOMEM for a product
whose planes need more, and still runs (exactly) the products that fit.  A
tuning cache written by one context through GF2E_TUNE_CACHE is read by the
next: the cached choice is used as stored, no product is tuned again, and
lines for another architecture are ignored.
"""
import json

import numpy as np
import pytest
import torch

import oracle
import workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import paper_1111_6900_amd as g
    return g


def dev(g, M, e):
    return torch.from_numpy(np.ascontiguousarray(M).astype(np.int64)).to(g.elem_dtype(e)).cuda()


def test_workspace_limit_returns_enomem(g):
    e, f, n = 8, 0x11D, 1024
    geo = g.plane_geometry(e, f, n, n, n)
    need = geo.a_bytes + geo.b_bytes + geo.p_bytes
    gen = np.random.default_rng(5)
    a = workload.field_matrix(gen, n, n, e)
    b = workload.field_matrix(gen, n, n, e)
    ctx = g.Context(0, workspace_limit=need // 2)
    try:
        with pytest.raises(g.GF2EError) as ei:
            ctx.mul(dev(g, a, e), dev(g, b, e), e, f)
        assert ei.value.code == g.ENOMEM
        # a product whose planes fit runs, and is exact
        small = 96
        got = ctx.mul(dev(g, a[:small, :small], e), dev(g, b[:small, :small], e), e, f)
        assert (got.cpu().numpy() == oracle.matmul(a[:small, :small], b[:small, :small], e, f)).all()
        assert 0 < ctx.workspace_bytes() <= need // 2
    finally:
        ctx.close()


def test_tune_cache_round_trip(g, tmp_path, monkeypatch):
    path = tmp_path / "tune.jsonl"
    monkeypatch.setenv("GF2E_TUNE_CACHE", str(path))
    e, f, m, k, n = 8, 0x11D, 512, 384, 640
    gen = np.random.default_rng(6)
    a = workload.field_matrix(gen, m, k, e)
    b = workload.field_matrix(gen, k, n, e)
    want = oracle.matmul(a, b, e, f)

    c1 = g.Context(0, autotune=True)
    try:
        assert (c1.mul(dev(g, a, e), dev(g, b, e), e, f).cpu().numpy() == want).all()
        kind, form = c1.chosen_kernel(e, f, m, k, n), c1.chosen_form(e, f, m, k, n)
    finally:
        c1.close()
    lines = path.read_text().splitlines()
    assert len(lines) == 1
    entry = json.loads(lines[0])
    assert entry["arch"] == "gfx950" and entry["kernel"] in g.kernel_names()
    # the choice packs the schedule form's kernel, the alpha form's kernel and the form
    assert (entry["choice"] >> 16) == form
    assert ((entry["choice"] >> (8 * form)) & 0xFF) == kind

    # A second context takes the stored choice without tuning again.
    c2 = g.Context(0, autotune=True)
    try:
        assert c2.chosen_kernel(e, f, m, k, n) == kind and c2.chosen_form(e, f, m, k, n) == form
        assert (c2.mul(dev(g, a, e), dev(g, b, e), e, f).cpu().numpy() == want).all()
    finally:
        c2.close()
    assert path.read_text().splitlines() == lines

    # An edited entry is used as stored (the packed-word kernel in both forms,
    # schedule form); a line for another architecture is ignored.
    valu = g.kernel_names().index("valu_xor_128x128")
    edited = dict(entry, choice=valu | (valu << 8))
    other = dict(entry, arch="gfx942", choice=1 | (1 << 8) | (1 << 16))
    path.write_text(json.dumps(edited) + "\n" + json.dumps(other) + "\n")
    c3 = g.Context(0, autotune=True)
    try:
        assert c3.chosen_form(e, f, m, k, n) == 0
        assert c3.chosen_kernel(e, f, m, k, n) == valu
        assert (c3.mul(dev(g, a, e), dev(g, b, e), e, f).cpu().numpy() == want).all()
    finally:
        c3.close()
    assert len(path.read_text().splitlines()) == 2
