"""The small parity cases reach the list build's less common paths (checked on the
CPU with the oracle's cell assignment, so a change to a case cannot drop them
silently): a home cell with more than 128 members (key blocks at 64 and 128, whose
own candidates lie outside the first chunk of the pass, and the unstaged write of
the entries), home cells whose candidates need more than one pass (over 384, or
over 192 where the stencil holds a periodic image), a box of three cells per axis,
and a cell with a single member."""
import numpy as np

import oracle
from test_gpu_parity import case


def _cells(name):
    q, _, L = case(name)
    _, cell, nc = oracle.cells(q, L, 2.8)
    n0, n1, n2 = (int(x) for x in nc)
    cnt = np.bincount(cell, minlength=n0 * n1 * n2).reshape(n2, n1, n0)
    # candidates of each home cell: its 27 stencil cells (distinct for >= 3 cells per axis)
    tot = np.zeros_like(cnt)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                tot += np.roll(cnt, (-dz, -dy, -dx), axis=(0, 1, 2))
    return (n0, n1, n2), cnt, tot


def test_clustered_case_has_cells_beyond_two_key_blocks():
    nc, cnt, tot = _cells("clustered")
    assert min(nc) >= 3
    assert cnt.max() > 128
    assert tot.max() > 2 * 384


def test_dense_case_needs_two_candidate_passes():
    (n0, n1, n2), cnt, tot = _cells("dense07")
    inner = tot[1:n2 - 1, 1:n1 - 1, 1:n0 - 1]  # no stencil cell is a periodic image
    assert inner.size > 0 and inner.min() > 384
    assert cnt.max() <= 64


def test_small_boxes_and_single_members():
    nc, _, _ = _cells("jitter_ragged")
    assert min(nc) == 3
    nc, cnt, _ = _cells("minimal")
    assert nc == (3, 3, 3) and cnt.max() == 1
