"""C-ABI checks that need no GPU: the library loads, exports every entry point
that include/md.h declares, and validates arguments before any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1210_3450_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "md.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(md_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) >= 20
    lib = C.CDLL(B.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(B.EXPORTED)


def test_struct_sizes_match_header_layout():
    # md_params: int64 + 3 doubles + 4 doubles + 6 int32 + 1 double + 5 uint64
    assert C.sizeof(B.md_params) == 8 + 24 + 32 + 24 + 8 + 40
    assert C.sizeof(B.md_stats) == 5 * 8 + 4 * 4 + 8 + 8 + 8 + 8 + 8 + 4 + 12 + 8
    # md_bubble_info: 4 int32 + 3 doubles + 1 double + 3 int64
    assert C.sizeof(B.md_bubble_info) == 16 + 24 + 8 + 24


def test_status_strings():
    assert B.md_status_str(B.MD_OK) == b"MD_OK"
    assert B.md_status_str(B.MD_EINVAL) == b"MD_EINVAL"
    assert B.md_status_str(B.MD_ELIST) == b"MD_ELIST"
    assert B.md_status_str(-99) == b"MD_UNKNOWN"


def test_null_safety():
    assert B.md_destroy(None) == B.MD_OK
    assert B.md_step(None, 1, 0) == B.MD_EINVAL
    assert B.md_set_state(None, None, None) == B.MD_EINVAL
    assert B.md_energy(None, None, None) == B.MD_EINVAL
    info = B.md_bubble_info()
    assert B.md_bubbles(None, 0, 3.0, 0.2, None, None, None, None, 0, C.byref(info)) == B.MD_EINVAL
    assert B.md_last_error(None) is not None


BAD = [
    dict(n=1),
    dict(cell_scale=0.5),
    dict(cell_scale=2.5),
    dict(cell_scale=float("nan")),
    dict(rc=0.0),
    dict(rc=float("nan")),
    dict(skin=-0.1),
    dict(dt=0.0),
    dict(mass=-1.0),
    dict(box=(8.3, 20.0, 20.0)),          # 8.3 < 3 * 2.8
    dict(box=(float("inf"), 20.0, 20.0)),
    dict(precision=7),
    dict(cutoff=9),
    dict(rebuild=5),
    dict(flags=1 << 7),
    dict(flags=4 | 8),                    # tile on and off together
    dict(flags=16, precision=1),          # fast reciprocal on the mixed path
    dict(flags=32 | 1),                   # half list with the verifier
    dict(flags=32 | 4, precision=1),      # half list with staged tiles
    dict(flags=32, threads_per_key=2),    # half list takes one lane per key
    dict(flags=1 << 6),
    dict(threads_per_key=3),
    dict(list_cap=-1),
    dict(box=(3000.0, 20.0, 20.0)),       # > 1023 cells on one axis
    dict(n=(1 << 27) + 1, box=(400.0, 400.0, 400.0)),
]


@pytest.mark.parametrize("kw", BAD)
def test_create_rejects_bad_params(kw):
    base = dict(n=4000, box=(20.0, 20.0, 20.0))
    base.update(kw)
    p = B.make_params(**base)
    out = C.c_void_p()
    assert B.md_create(C.byref(p), None, C.byref(out)) == B.MD_EINVAL
    assert not out.value
    assert len(B.md_last_error(None)) > 0


def test_create_rejects_nonzero_reserved():
    p = B.make_params(4000, 20.0)
    p.reserved[3] = 1
    out = C.c_void_p()
    assert B.md_create(C.byref(p), None, C.byref(out)) == B.MD_EINVAL
    assert b"reserved" in B.md_last_error(None)


def test_batch_rejects_mismatched_shared_fields():
    a = B.make_params(4000, 20.0)
    b = B.make_params(5000, 22.0, rc=3.0)
    arr = (B.md_params * 2)(a, b)
    out = C.c_void_p()
    assert B.md_batch_create(arr, 2, None, C.byref(out)) == B.MD_EINVAL
    assert B.md_batch_create(arr, 0, None, C.byref(out)) == B.MD_EINVAL


def test_cell_division_multipliers_are_exact():
    """The box geometry divides cell indices by n[0], n[1] and n[0] * n[1] with a
    multiplier floor(2^(30 + l) / d) + 1 and a shift of 32 + l - 2 (l = ceil(log2 d)),
    which is exact for every 0 <= x < 2^30 (the multiplier's excess m d - 2^(30 + l)
    lies in (0, d]); checked here for every divisor the cell grid can have on one axis
    and for products of two, at the edges of every quotient class and at random."""
    rng = np.random.Generator(np.random.PCG64(5))
    X = (1 << 30) - 1
    divisors = list(range(3, 1024)) + [a * b for a in (3, 7, 45, 142, 1000, 1023) for b in (3, 64, 142, 999, 1023)]
    for d in divisors:
        l = (d - 1).bit_length()  # ceil(log2 d)
        m = (1 << (30 + l)) // d + 1
        assert m < (1 << 32)
        ks = np.unique(np.concatenate([[0, 1, 2], rng.integers(0, X // d + 1, 64), [X // d - 1, X // d]]))
        xs = np.concatenate([ks * d, ks * d + d - 1, rng.integers(0, X + 1, 256)])
        xs = xs[(xs >= 0) & (xs <= X)].astype(object)
        q = [((int(x) * m) >> 32) >> (l - 2) for x in xs]
        assert q == [int(x) // d for x in xs], d
