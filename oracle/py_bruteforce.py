"""Second, independent oracle in numpy for tiny boxes: O(n^2) over all pairs.

TEST INFRASTRUCTURE ONLY.  Written separately from md_oracle.c (no shared
helpers) so that each pins the other: minimum image along each axis, the pair
potential of Eq. (1) and the force scalar of Algorithm 1, f = V'(r)/r, applied
as F_i += f (q_j - q_i).
"""
from __future__ import annotations

import numpy as np


def lj_coeffs(rc: float):
    """c2, c0 from solving V(rc) = 0 and V'(rc) = 0 as a 2x2 linear system in
    (c2, c0) -- a different route from the oracle's closed form."""
    # V/4 = rc^-12 - rc^-6 + c2 rc^2 + c0 = 0
    # V'/4 = -12 rc^-13 + 6 rc^-7 + 2 c2 rc = 0
    A = np.array([[rc * rc, 1.0], [2.0 * rc, 0.0]])
    b = np.array([-(rc ** -12 - rc ** -6), 12.0 * rc ** -13 - 6.0 * rc ** -7])
    c2, c0 = np.linalg.solve(A, b)
    return float(c2), float(c0)


def pair_table(q: np.ndarray, L, cutoff: float):
    """All ordered pairs (i, j), i != j, with minimum-image distance < cutoff.
    Returns (i, j, d, r2) with d = minimum image of q_j - q_i."""
    L = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,))
    t = q[None, :, :] - q[:, None, :]
    d = t - L * np.rint(t / L)
    r2 = (d * d).sum(axis=2)
    n = q.shape[0]
    mask = r2 < cutoff * cutoff
    mask[np.arange(n), np.arange(n)] = False
    i, j = np.nonzero(mask)
    return i, j, d[i, j], r2[i, j]


def neighbor_sets(q, L, r_list):
    i, j, _, _ = pair_table(q, L, r_list)
    n = q.shape[0]
    out = [[] for _ in range(n)]
    for a, b in zip(i.tolist(), j.tolist()):
        out[a].append(b)
    return [np.array(sorted(x), dtype=np.int32) for x in out]


def forces(q, L, rc, c2, c0):
    """F_i, total PE over unordered pairs, per-particle sum |f d|."""
    i, j, d, r2 = pair_table(q, L, rc)
    r = np.sqrt(r2)
    V = 4.0 * (r ** -12 - r ** -6 + c2 * r2 + c0)
    f = (24.0 * r ** 6 - 48.0) / r ** 14 + 8.0 * c2
    F = np.zeros_like(q)
    np.add.at(F, i, f[:, None] * d)
    A = np.zeros(q.shape[0])
    np.add.at(A, i, np.abs(f) * r)
    pe = 0.5 * V.sum()
    return F, pe, A
