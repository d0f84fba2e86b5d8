"""md_bubbles_noalloc: the allocation-free variant of md_bubbles, called through
the C ABI and compared with md_bubbles (and the oracle) on the same state.

Two calls in a row, the second on a smaller subcell grid, so the fixed scratch
the variant shares across calls holds the first call's contents when the second
starts.  Bar: byte counts, labels, roots, sizes and the summary bit-exact.  The
device's free memory is read before and after the variant's calls: it must not
change (the outputs are allocated before).
"""
import ctypes as C
import math

import numpy as np
import pytest

import oracle
from paper_1210_3450_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def B():
    from paper_1210_3450_amd import binding
    return binding


def raw_call(fn, ctx, side, rho, counts, labels, cap):
    b = B()
    info = b.md_bubble_info()
    roots = np.zeros(max(cap, 1), dtype=np.int64)
    sizes = np.zeros(max(cap, 1), dtype=np.int64)
    torch.cuda.synchronize()
    s = fn(ctx.ctx, 0, float(side), float(rho), C.c_void_p(counts.data_ptr()), C.c_void_p(labels.data_ptr()),
           roots.ctypes.data_as(b._PI64), sizes.ctypes.data_as(b._PI64), cap, C.byref(info))
    assert s == b.MD_OK, b.md_last_error(ctx.ctx)
    m = min(cap, int(info.nbubbles))
    return info, counts.cpu().numpy().copy(), labels.cpu().numpy().copy(), roots[:m].copy(), sizes[:m].copy()


def field_state(shape, L, p, seed):
    gas, counts = inputs.bubble_field(shape, p, seed, border=False)
    return inputs.subcell_field_positions(counts, L, seed)


CASES = [  # (nz, ny, nx) = floor(L / 3) per axis; the second grid is smaller
    ((40, 50, 60), (180.0, 150.0, 120.0), 0.3116, 3),
    ((8, 9, 10), (30.0, 27.0, 24.0), 0.3, 1),
]


def test_noalloc_matches_md_bubbles_twice_second_smaller():
    b = B()
    ctxs, runs = [], []
    for shape, L, p, seed in CASES:
        assert shape == tuple(math.floor(L[a] / 3.0) for a in (2, 1, 0))
        q = field_state(shape, L, p, seed)
        c = b.Context(b.make_params(q.shape[0], L))
        c.set_state(q, np.zeros_like(q))
        nsub = int(np.prod(shape))
        outs = [torch.empty(nsub, dtype=torch.uint8, device="cuda") for _ in range(2)]
        labs = [torch.empty(nsub, dtype=torch.int32, device="cuda") for _ in range(2)]
        ctxs.append((c, q, L, nsub, outs, labs))
    # reference: the allocating entry point (its work buffers are allocated here)
    for c, q, L, nsub, outs, labs in ctxs:
        runs.append(raw_call(b.md_bubbles, c, 3.0, 0.2, outs[0], labs[0], nsub))
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    got = [raw_call(b.md_bubbles_noalloc, c, 3.0, 0.2, outs[1], labs[1], nsub)
           for c, q, L, nsub, outs, labs in ctxs]
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, (free0, free1)
    for (c, q, L, nsub, outs, labs), ref, res in zip(ctxs, runs, got):
        ri, rc, rl, rr, rs = ref
        gi, gc, gl, gr, gs = res
        assert tuple(gi.nsub) == tuple(ri.nsub)
        assert gi.threshold == ri.threshold
        assert (gi.ngas, gi.nbubbles, gi.largest) == (ri.ngas, ri.nbubbles, ri.largest)
        np.testing.assert_array_equal(gc, rc)
        np.testing.assert_array_equal(gl, rl)
        np.testing.assert_array_equal(gr, rr)
        np.testing.assert_array_equal(gs, rs)
        o = oracle.bubbles(q, L)
        np.testing.assert_array_equal(gl, o.labels)
        np.testing.assert_array_equal(gr, o.roots)
        np.testing.assert_array_equal(gs, o.sizes)
        print("noalloc: %d subcells, %d bubbles, largest %d" % (nsub, gi.nbubbles, gi.largest))
    for c, *_ in ctxs:
        c.close()


def test_noalloc_cap_and_limits():
    b = B()
    shape, L, p, seed = CASES[1]
    q = field_state(shape, L, p, seed)
    with b.Context(b.make_params(q.shape[0], L)) as c:
        c.set_state(q, np.zeros_like(q))
        full = c.bubbles(noalloc=True)
        ref = c.bubbles()
        np.testing.assert_array_equal(full["roots"], ref["roots"])
        part = c.bubbles(cap=2, noalloc=True, fields=False)
        np.testing.assert_array_equal(part["roots"], ref["roots"][:2])
        assert part["nbubbles"] == ref["nbubbles"]
    # beyond the fixed scratch: 102^3 subcells of edge 1
    Lb = 102.0
    rng = np.random.default_rng(7)
    q = rng.uniform(0.0, Lb, size=(1000, 3))
    with b.Context(b.make_params(q.shape[0], Lb)) as c:
        c.set_state(q, np.zeros_like(q))
        info = b.md_bubble_info()
        s = b.md_bubbles_noalloc(c.ctx, 0, 1.0, 0.2, None, None, None, None, 0, C.byref(info))
        assert s == b.MD_EINVAL
        assert b"fixed scratch" in b.md_last_error(c.ctx)
        # the allocating entry point still serves it
        s = b.md_bubbles(c.ctx, 0, 1.0, 0.2, None, None, None, None, 0, C.byref(info))
        assert s == b.MD_OK
