"""Pins of the FP64 CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: closed forms,
textbook special cases, an independent numpy brute force, lattice sums by
enumeration, finite differences and dynamical invariants.  A dropped term, a
flipped sign, a wrong image or a transposed operand in the oracle fails at least
one of them.
"""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import py_bruteforce as pb
from paper_1210_3450_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ Eq. (1)

@pytest.mark.parametrize("rc", [2.5, 3.0])
def test_cutoff_conditions_vanish(rc):
    """Eq. (1): c2, c0 make V(rc) = V'(rc) = 0 (Sec. II.A)."""
    c2, c0 = oracle.coeffs(rc)
    assert abs(oracle.pair_v(rc * rc, c2, c0)) < 1e-15
    assert abs(oracle.pair_f(rc * rc, c2)) < 1e-15
    # derivative of V at rc by central difference of the oracle's own V
    h = 1e-5
    dV = (oracle.pair_v((rc + h) ** 2, c2, c0) - oracle.pair_v((rc - h) ** 2, c2, c0)) / (2 * h)
    assert abs(dV) < 1e-10


@pytest.mark.parametrize("rc", [2.5, 3.0])
def test_coeffs_match_linear_solve(rc):
    """The oracle's closed form equals the solution of the 2x2 system V(rc)=V'(rc)=0."""
    c2, c0 = oracle.coeffs(rc)
    c2b, c0b = pb.lj_coeffs(rc)
    assert c2 == pytest.approx(c2b, rel=1e-12)
    assert c0 == pytest.approx(c0b, rel=1e-12)


def test_textbook_lj_special_case():
    """Untruncated 12-6 shape (c2 = c0 = 0): V(1) = 0, V(2^(1/6)) = -1, f(2^(1/6)) = 0."""
    r_min = 2.0 ** (1.0 / 6.0)
    assert oracle.pair_v(1.0, 0.0, 0.0) == 0.0
    assert oracle.pair_v(r_min ** 2, 0.0, 0.0) == pytest.approx(-1.0, abs=1e-15)
    assert abs(oracle.pair_f(r_min ** 2, 0.0)) < 1e-14
    # the force scalar at r = 1: (24 - 48)/1 = -24 (attraction sign convention d = q_j - q_i)
    assert oracle.pair_f(1.0, 0.0) == -24.0


def test_eq1_force_at_raw_minimum():
    """At r = 2^(1/6) the 12-6 part of f vanishes, leaving f = 8 c2 (Algorithm 1's scalar)."""
    for rc in (2.5, 3.0):
        c2, c0 = oracle.coeffs(rc)
        assert oracle.pair_f(2.0 ** (1.0 / 3.0), c2) == pytest.approx(8.0 * c2, rel=1e-12)
        assert oracle.pair_v(2.0 ** (1.0 / 3.0), c2, c0) == pytest.approx(
            -1.0 + 4.0 * (c2 * 2.0 ** (1.0 / 3.0) + c0), rel=1e-14)


@pytest.mark.parametrize("mode", [oracle.CUT_EQ1, oracle.CUT_SHIFT, oracle.CUT_RAW])
def test_force_scalar_is_derivative_over_r(mode):
    """f(r) = V'(r)/r over r in [0.8, rc), by central differences of V."""
    rc = 2.5
    c2, c0 = oracle.coeffs(rc, mode)
    for r in np.linspace(0.8, rc - 1e-3, 97):
        h = 1e-6 * r
        dV = (oracle.pair_v((r + h) ** 2, c2, c0) - oracle.pair_v((r - h) ** 2, c2, c0)) / (2 * h)
        f = oracle.pair_f(r * r, c2)
        assert f * r == pytest.approx(dV, rel=1e-6, abs=1e-9)


def test_pair_values_match_numpy_bruteforce():
    """Two particles at known separations: oracle and numpy brute force agree on F and PE."""
    L = 10.0
    for r in (0.95, 1.12, 1.5, 2.2, 2.49):
        q = np.array([[1.0, 2.0, 3.0], [1.0 + r, 2.0, 3.0]])
        F, pe, _ = oracle.forces_brute(q, L, 2.5)
        c2, c0 = pb.lj_coeffs(2.5)
        Fb, peb, _ = pb.forces(q, L, 2.5, c2, c0)
        np.testing.assert_allclose(F, Fb, rtol=1e-12, atol=1e-15)
        assert pe == pytest.approx(peb, rel=1e-12)
        # Newton's third law for the pair, and attraction/repulsion sign:
        assert F[0, 0] == -F[1, 0]
        assert (F[0, 0] > 0) == (r > 2.0 ** (1 / 6))  # attracted towards +x beyond the minimum


# ------------------------------------------------------------------ geometry

def test_minimum_image_across_boundary():
    """A pair split by the periodic boundary interacts at its short distance."""
    L = np.array([9.0, 10.0, 11.0])
    q = np.array([[0.3, 4.0, 5.0], [8.6, 4.0, 5.0]])  # 0.7 apart through x = 0
    kp, pl = oracle.neighbors(q, L, 2.8)
    assert list(pl) == [1, 0]
    F, pe, _ = oracle.forces(q, L, 2.5, 0.3)
    c2, c0 = oracle.coeffs(2.5)
    assert pe == pytest.approx(oracle.pair_v(0.7 ** 2, c2, c0), rel=1e-12)
    # repulsion: particle 0 pushed towards +x (away from its image at -0.4)
    assert F[0, 0] > 0 and F[1, 0] < 0


def test_wrap_and_cell_ids_edge_values():
    """Wrap into [0, L), cell count floor(L/r_list), index min((int)(x n/L), n-1)."""
    L = 400.0
    # x = 200 lies on a cell face: 200 * (142/400) rounds to 71.0 -> cell 71
    q = np.array([[200.0, 0.0, 399.99999999999994],
                  [-1e-300, 400.0, -400.0],
                  [799.9999999999999, 1e-300, 2.8169014084507045]])
    qw, cell, nc = oracle.cells(q, L, 2.8)
    assert list(nc) == [142, 142, 142]
    cx = cell % 142
    cy = (cell // 142) % 142
    cz = cell // (142 * 142)
    assert cx[0] == 71 and cy[0] == 0 and cz[0] == 141
    # -1e-300 + 400 rounds to 400, and the second wrap line maps it to 0
    assert qw[1, 0] == 0.0 and cx[1] == 0
    assert qw[1, 1] == 0.0 and cy[1] == 0
    assert qw[1, 2] == 0.0 and cz[1] == 0
    assert 0.0 <= qw[2, 0] < L
    assert (qw >= 0).all() and (qw < L).all()


def test_cells_reject_bad_positions():
    with pytest.raises(ValueError):
        oracle.cells(np.array([[np.nan, 1.0, 1.0]]), 10.0, 2.8)
    with pytest.raises(ValueError):
        oracle.cells(np.array([[20.0, 1.0, 1.0]]), 10.0, 2.8)  # 2L is outside [-L, 2L)
    with pytest.raises(ValueError):
        oracle.cells(np.array([[1.0, 1.0, 1.0]]), 8.0, 2.8)    # only 2 cells per axis


# ------------------------------------------------------------------ lattice sums

def _fcc_shells():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "fcc_shells.txt")) if not l.startswith("#")]
    return [(int(a), int(b)) for a, b in rows if a]


def test_fcc_shells_by_enumeration():
    """The golden shell table equals a direct enumeration of FCC lattice vectors."""
    r = np.arange(-4, 5)
    v = np.array(np.meshgrid(r, r, r, indexing="ij")).reshape(3, -1).T
    v = v[(v.sum(axis=1) % 2 == 0) & (np.abs(v).sum(axis=1) > 0)]
    d2 = (v * v).sum(axis=1)
    for s2, cnt in _fcc_shells():
        assert int((d2 == s2).sum()) == cnt


@pytest.mark.parametrize("ncell,rho,rc,nlist,nin", [(5, 0.5, 2.5, 42, 42), (6, 0.7, 3.0, 86, 78)])
def test_fcc_lattice_energy_and_zero_force(ncell, rho, rc, nlist, nin):
    """FCC at rho: U/N = 1/2 sum_shells n_k V(r_k) over shells inside rc; F_i = 0 by
    inversion symmetry; every site has the same list length."""
    a = 2.0 if rho == 0.5 else (4.0 / rho) ** (1.0 / 3.0)
    q = inputs.fcc_positions(ncell, a)
    L = ncell * a
    c2, c0 = oracle.coeffs(rc)
    F, pe, _ = oracle.forces(q, L, rc, 0.3)
    u = 0.0
    n_in = 0
    for s2, cnt in _fcc_shells():
        r2 = s2 * (a / 2.0) ** 2
        if r2 < rc * rc:
            u += 0.5 * cnt * oracle.pair_v(r2, c2, c0)
            n_in += cnt
    assert n_in == nin
    assert pe / q.shape[0] == pytest.approx(u, rel=1e-13)
    assert np.abs(F).max() < 1e-13
    kp, _ = oracle.neighbors(q, L, rc + 0.3)
    assert set(np.diff(kp).tolist()) == {nlist}


def test_fcc_rho05_lattice_energy_value():
    """Density 0.5, rc = 2.5: 12, 6 and 24 sites at r^2 = 2, 4, 6 lie inside rc
    (r^2 = 8 is beyond rc^2 = 6.25), so U/N = 1/2 (12 V(sqrt2) + 6 V(2) + 24 V(sqrt6)),
    evaluated here with coefficients from the independent linear solve."""
    c2, c0 = pb.lj_coeffs(2.5)

    def V(r2):
        return 4.0 * (r2 ** -6 - r2 ** -3 + c2 * r2 + c0)

    u = 0.5 * (12 * V(2.0) + 6 * V(4.0) + 24 * V(6.0))
    assert u == pytest.approx(-2.413162698239619, rel=1e-14)
    _, pe, _ = oracle.forces(inputs.fcc_positions(5, 2.0), 10.0, 2.5, 0.3)
    assert pe / 500 == pytest.approx(u, rel=1e-13)


# ------------------------------------------------------------------ brute force

CASES = [
    ("random", 300, (9.0, 10.0, 11.0), 11),
    ("jitter", 512, (12.0, 12.0, 12.0), 12),
    ("clustered", 400, (8.5, 8.5, 14.0), 13),
]


def _case_positions(kind, n, L, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    if kind == "random":
        return inputs.random_box(n, L, seed)
    if kind == "jitter":
        return inputs.random_box(n, L, seed, min_sep=0.9)
    centers = rng.uniform(0, 1, size=(6, 3)) * np.array(L)
    q = centers[rng.integers(0, 6, size=n)] + rng.normal(0, 1.2, size=(n, 3))
    return np.mod(q, np.array(L))


@pytest.mark.parametrize("kind,n,L,seed", CASES)
def test_cell_list_equals_brute_force(kind, n, L, seed):
    """Full and half lists from the cell grid equal the all-pairs sets (C and numpy)."""
    q = _case_positions(kind, n, L, seed)
    rl = 2.8
    kp, pl = oracle.neighbors(q, L, rl)
    kpb, plb = oracle.neighbors(q, L, rl, brute=True)
    np.testing.assert_array_equal(kp, kpb)
    np.testing.assert_array_equal(pl, plb)
    sets = pb.neighbor_sets(q, L, rl)
    for i in range(n):
        np.testing.assert_array_equal(pl[kp[i]:kp[i + 1]], sets[i])
    hk, hp = oracle.neighbors(q, L, rl, half=True)
    assert hk[-1] * 2 == kp[-1]
    for i in range(n):
        h = hp[hk[i]:hk[i + 1]]
        assert (h > i).all()
        np.testing.assert_array_equal(h, sets[i][sets[i] > i])


@pytest.mark.parametrize("kind,n,L,seed", CASES[1:])
def test_forces_equal_brute_force(kind, n, L, seed):
    q = _case_positions(kind, n, L, seed)
    F, pe, A = oracle.forces(q, L, 2.5, 0.3)
    Fb, peb, Ab = oracle.forces_brute(q, L, 2.5)
    c2, c0 = pb.lj_coeffs(2.5)
    Fn, pen, An = pb.forces(q, L, 2.5, c2, c0)
    scale = np.maximum(A, 1e-300)
    assert (np.linalg.norm(F - Fb, axis=1) / scale).max() < 1e-13
    assert (np.linalg.norm(F - Fn, axis=1) / scale).max() < 1e-12
    assert pe == pytest.approx(peb, rel=1e-12)
    assert pe == pytest.approx(pen, rel=1e-11)
    np.testing.assert_allclose(A, An, rtol=1e-11)


def test_force_is_minus_gradient_of_energy():
    """F_i = -dPE/dq_i by central differences of the oracle's total energy:
    pins the sign convention d = q_j - q_i and the factor of Algorithm 1."""
    q = inputs.random_box(64, 9.0, 21, min_sep=1.0)
    F, _, _ = oracle.forces_brute(q, 9.0, 2.5)
    rng = np.random.Generator(np.random.PCG64(3))
    for i in rng.choice(64, 6, replace=False):
        for ax in range(3):
            h = 1e-6
            qp, qm = q.copy(), q.copy()
            qp[i, ax] += h
            qm[i, ax] -= h
            _, ep, _ = oracle.forces_brute(qp, 9.0, 2.5)
            _, em, _ = oracle.forces_brute(qm, 9.0, 2.5)
            assert F[i, ax] == pytest.approx(-(ep - em) / (2 * h), rel=1e-5, abs=1e-6)


def test_newton_third_law_and_translation_invariance():
    q = _case_positions("jitter", 512, (12.0, 12.0, 12.0), 12)
    L = 12.0
    F, pe, A = oracle.forces(q, L, 2.5, 0.3)
    assert np.linalg.norm(F.sum(axis=0)) <= 1e-12 * np.abs(F).sum()
    shift = np.array([3.3, -7.1, 11.9])
    F2, pe2, _ = oracle.forces(np.mod(q + shift, L), L, 2.5, 0.3)
    assert (np.linalg.norm(F2 - F, axis=1) / A).max() < 1e-12
    assert pe2 == pytest.approx(pe, rel=1e-12)


# ------------------------------------------------------------------ dynamics

def _hot_small(seed=7, ncell=5, T=1.0):
    a = 2.0
    q = inputs.fcc_positions(ncell, a)
    rng = np.random.Generator(np.random.PCG64(seed))
    v = inputs.maxwell_boltzmann(q.shape[0], T, 1.0, rng)
    return q, v, ncell * a


def test_time_reversibility():
    """Velocity Verlet is time reversible: run, negate v, run again -> start state."""
    q0, v0, L = _hot_small()
    r1 = oracle.run(q0, v0, L, 100)
    r2 = oracle.run(r1.q, -r1.v, L, 100)
    d = r2.q - q0
    d -= L * np.rint(d / L)
    assert np.abs(d).max() < 1e-8
    np.testing.assert_allclose(-r2.v, v0, atol=1e-8)


def test_dutc_list_stays_valid_and_never_fails():
    """With the DUTC rule no pair within rc is ever missing from the list; without
    rebuilds pairs go missing (the failure the paper's per-step check prevents)."""
    q0, v0, L = _hot_small(T=2.0)
    ok = oracle.run(q0, v0, L, 150, verify=True)
    assert ok.rebuilds > 3 and ok.missed_pairs == 0
    disp = oracle.run(q0, v0, L, 150, verify=True, rebuild=oracle.REBUILD_DISPLACEMENT)
    assert disp.missed_pairs == 0 and disp.rebuilds <= ok.rebuilds
    bad = oracle.run(q0, v0, L, 150, verify=True, rebuild=oracle.REBUILD_NEVER)
    assert bad.missed_pairs > 0


# (dt, vmax, skin): dt * vmax is a power of two times a small integer, so the DUTC
# sum D = k * dt * vmax is exact; in the last case skin / (2 vmax dt) = 64 exactly and
# 2 D = skin at step 64 must not rebuild (the rule is a strict inequality)
DUTC_CADENCE = [(2.0 ** -7, 0.5, 0.3), (2.0 ** -8, 0.75, 0.3), (2.0 ** -6, 0.25, 0.5)]


@pytest.mark.parametrize("dt,vmax,skin", DUTC_CADENCE)
def test_dutc_cadence_of_free_particles(dt, vmax, skin):
    """Sec. II.A's DUTC bound grows by dt * max|v| per step and the list is rebuilt
    once 2 D exceeds the skin: free particles whose fastest one moves at vmax are
    rebuilt every K = floor(skin / (2 vmax dt)) + 1 steps exactly."""
    K = int(math.floor(skin / (2.0 * vmax * dt))) + 1
    q, v, L = inputs.free_gas(vmax)
    for n in (K - 1, K, 2 * K - 1, 2 * K, 5 * K + 3):
        r = oracle.run(q, v, L, n, dt=dt, skin=skin)
        assert r.rebuilds == 1 + n // K, (n, K, r.rebuilds)  # the initial build counts
        np.testing.assert_array_equal(r.v, v)  # no forces: velocities unchanged
        assert r.D == pytest.approx((n % K) * dt * vmax, abs=1e-15)


def test_momentum_and_energy_conservation():
    """Total momentum stays ~0; total energy stays bounded with Eq. (1) at dt = 0.005."""
    w = inputs.small_nve()
    r = oracle.run(w.pos, w.vel, w.box, 200, energy_every=10)
    assert np.abs(r.v.sum(axis=0)).max() < 1e-10
    E = (r.ke + r.pe) / w.n
    assert np.abs(E - E[0]).max() < 2e-3
    # the exact list is exact: every-step rebuild gives the same trajectory to roundoff
    r2 = oracle.run(w.pos, w.vel, w.box, 200, energy_every=10, rebuild=oracle.REBUILD_EVERY_STEP)
    d = r2.q - r.q
    d -= w.box[0] * np.rint(d / w.box[0])
    assert np.abs(d).max() < 1e-9


def test_sampled_evaluations_match_full():
    q = _case_positions("jitter", 512, (12.0, 12.0, 12.0), 12)
    L = 12.0
    F, pe, A, pei = oracle.forces_list(*_list_args(q, L), per_particle_pe=True)
    ids = np.array([0, 5, 77, 300, 511])
    Fs, As, pes = oracle.forces_sample(q, L, 2.5, ids)
    np.testing.assert_allclose(Fs, F[ids], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(pes, pei[ids], rtol=1e-13)
    kp, pl = oracle.neighbors(q, L, 2.8)
    ns = oracle.neighbors_sample(q, L, 2.8, ids)
    for s, i in enumerate(ids):
        np.testing.assert_array_equal(ns[s], pl[kp[i]:kp[i + 1]])


def _list_args(q, L):
    qw, _, _ = oracle.cells(q, L, 2.8)
    kp, pl = oracle.neighbors(qw, L, 2.8)
    c2, c0 = oracle.coeffs(2.5)
    return qw, L, 2.5, kp, pl, c2, c0


# ---------------------------------------------------------------- approximate reciprocal (Sec. III.C)

def test_rcp_approx_model_error_below_1_over_256():
    """The model instruction: relative error below 1/256, and not exact in general."""
    r2 = np.linspace(0.6, 9.0, 2001)
    xt = np.array([oracle.rcp_approx(x) for x in r2])
    rel = np.abs(xt * r2 - 1.0)
    assert rel.max() < 1.0 / 256.0
    assert rel.max() > 1.0 / 2048.0


@pytest.mark.parametrize("n,second", [(4, 10.0), (7, 28.0)])
def test_rcp_correction_is_second_order(n, second):
    """With xt r^2 = 1 + e: xt^n ((n+1) - n xt r^2) = r^-2n (1 - n(n+1)/2 e^2 + O(e^3)),
    against (1 + n e) without the correction: the factors 10 and 28 for r^-8 and
    r^-14, and 4 and 7 uncorrected."""
    for r in (0.9, 1.12, 1.7, 2.5):
        r2 = r * r
        for e in (1.0 / 256, -1.0 / 256, 1.0 / 4096):
            xt = (1.0 + e) / r2
            exact = r2 ** (-n)
            corr = oracle.rpow_approx(r2, xt, n, True) / exact - 1.0
            plain = oracle.rpow_approx(r2, xt, n, False) / exact - 1.0
            assert corr == pytest.approx(-second * e * e, rel=0.05)
            assert plain == pytest.approx(n * e, rel=0.03)


def test_exact_reciprocal_through_corrected_formulas_is_exact():
    """Feeding the exact reciprocal to the corrected formulas reproduces the plain
    forces and energy (the correction factor is then 1)."""
    w = inputs.small_nve()
    qw, _, _ = oracle.cells(w.pos, w.box, 2.8)
    kp, pl = oracle.neighbors(qw, w.box, 2.8)
    c2, c0 = oracle.coeffs(2.5)
    F0, pe0, A = oracle.forces_list(qw, w.box, 2.5, kp, pl, c2, c0)
    F3, pe3, _ = oracle.forces_list(qw, w.box, 2.5, kp, pl, c2, c0, rcp=oracle.RCP_EXACT_CORR)
    assert (np.linalg.norm(F3 - F0, axis=1) / A).max() < 1e-13
    assert pe3 == pytest.approx(pe0, rel=1e-13)


@pytest.mark.slow
def test_reciprocal_correction_restores_energy_conservation():
    """The energy-conservation comparison of Sec. III.C at 4000 particles: with
    the 1/256 reciprocal the total energy drifts away; with the correction it
    stays at the level of exact division."""
    w = inputs.small_nve()
    dev = {}
    for mode in (oracle.RCP_DIV, oracle.RCP_APPROX, oracle.RCP_APPROX_CORR):
        r = oracle.run(w.pos, w.vel, w.box, 1000, energy_every=10, rcp=mode)
        E = r.ke + r.pe
        dev[mode] = float(np.abs(E - E[0]).max() / abs(E[0]))
    assert dev[oracle.RCP_APPROX] > 3.0 * dev[oracle.RCP_APPROX_CORR]
    assert dev[oracle.RCP_APPROX_CORR] < 1.5 * dev[oracle.RCP_DIV] + 1e-5


# ---------------------------------------------------------------- virial and thermostat

def test_virial_is_the_scaling_derivative_of_the_energy():
    """sum_{i<j} f r^2 = sum_{i<j} V'(r) r = d PE(lambda q, lambda L) / d lambda at 1,
    by central differences of the oracle's energy (V and V' vanish at rc, so the
    derivative is smooth)."""
    q = inputs.random_box(500, (10.5, 11.0, 12.0), 21, min_sep=0.85)
    L = np.array([10.5, 11.0, 12.0])
    w = oracle.virial(q, L, 2.5)
    h = 1e-6
    _, pp, _ = oracle.forces(q * (1 + h), L * (1 + h), 2.5, 0.3)
    _, pm, _ = oracle.forces(q * (1 - h), L * (1 - h), 2.5, 0.3)
    assert w == pytest.approx((pp - pm) / (2 * h), rel=1e-7)


def test_fcc_lattice_virial_from_shells():
    """At rest on the rho = 0.5 FCC lattice (rc = 2.5): sum_{i<j} f r^2 per site is
    1/2 sum over the shells inside rc of n_k f(r_k) r_k^2, with f from the
    coefficients of the independent linear solve."""
    c2, _ = pb.lj_coeffs(2.5)

    def f(r2):
        return 24.0 * r2 ** -4 - 48.0 * r2 ** -7 + 8.0 * c2

    per_site = 0.5 * sum(cnt * f(s2 * 1.0) * s2 for s2, cnt in _fcc_shells() if s2 < 6.25)
    q = inputs.fcc_positions(5, 2.0)
    assert oracle.virial(q, 10.0, 2.5) / 500 == pytest.approx(per_site, rel=1e-13)
    assert oracle.pressure(0.0, oracle.virial(q, 10.0, 2.5), 1000.0) == pytest.approx(-per_site * 500 / 3000.0,
                                                                                       rel=1e-13)


def test_thermostat_with_infinite_mass_is_nve():
    """A Nose-Hoover thermostat whose mass is effectively infinite leaves the
    velocity-Verlet trajectory unchanged bit for bit."""
    w = inputs.small_nve()
    a = oracle.run(w.pos, w.vel, w.box, 60, energy_every=10)
    b = oracle.run_obs(w.pos, w.vel, w.box, 60, energy_every=10, T=2.0, tau=1e150)
    np.testing.assert_array_equal(a.q, b.q)
    np.testing.assert_array_equal(a.v, b.v)
    np.testing.assert_array_equal(a.ke, b.ke)


@pytest.mark.slow
def test_thermostat_conserves_extended_energy_and_reaches_temperature():
    """Heating from T = 1.0 to T = 1.5 with tau = 0.1: KE + PE changes by far more
    than its NVE fluctuation while KE + PE + Q xi^2 / 2 + g T eta stays conserved
    to the NVE level, and the temperature of the second half averages to 1.5."""
    w = inputs.small_nve()
    r = oracle.run_obs(w.pos, w.vel, w.box, 2000, energy_every=10, T=1.5, tau=0.1)
    E = r.ke + r.pe
    H = E + r.thermo
    g = 3 * w.n - 3
    T = 2 * r.ke / g
    assert abs(E[-1] - E[0]) / abs(E[0]) > 0.2
    assert np.abs(H - H[0]).max() / abs(H[0]) < 2e-3
    assert T[T.size // 2:].mean() == pytest.approx(1.5, rel=0.05)


# ------------------------------------------------------------------ bubble identification

def _union_find_components(gas, periodic):
    """Reference clustering: scipy's face-connected labelling, then, on a torus,
    labels on opposite faces merged when both subcells are gas."""
    from scipy import ndimage
    lab, nl = ndimage.label(gas)
    parent = list(range(nl + 1))

    def find(a):
        while parent[a] != a:
            a = parent[a]
        return a

    if periodic:
        for ax in range(3):
            a = np.take(lab, 0, axis=ax)
            b = np.take(lab, -1, axis=ax)
            for u, v in zip(a[(a > 0) & (b > 0)], b[(a > 0) & (b > 0)]):
                ru, rv = find(int(u)), int(find(int(v)))
                if ru != rv:
                    parent[max(ru, rv)] = min(ru, rv)
    comp = np.array([find(k) for k in range(nl + 1)])[lab]
    flat = comp.reshape(-1)
    out = np.full(flat.shape, -1, dtype=np.int64)
    idx = np.arange(flat.size)
    for c in np.unique(flat[flat > 0]):
        members = idx[flat == c]
        out[members] = members.min()
    return out


def test_bubble_counts_match_histogram():
    """Byte counts per subcell equal numpy's histogram over the same edges
    (positions off the faces, some one box length outside [0, L))."""
    L = (13.1, 9.7, 16.4)
    rng = np.random.Generator(np.random.PCG64(3))
    q = rng.uniform(0.0, 1.0, size=(2000, 3)) * np.array(L)
    q[:200, 0] -= L[0]
    q[200:400, 2] += L[2]
    r = oracle.bubbles(q, L, 3.0, 0.2)
    assert r.nsub == (4, 3, 5)
    edges = [np.linspace(0.0, L[a], r.nsub[a] + 1) for a in range(3)]
    H, _ = np.histogramdd(np.mod(q, np.array(L)), bins=edges)
    np.testing.assert_array_equal(r.counts.reshape(5, 3, 4).transpose(2, 1, 0), H.astype(np.uint8))
    assert r.threshold == pytest.approx(0.2 * (13.1 / 4) * (9.7 / 3) * (16.4 / 5), rel=1e-15)


def test_bubble_threshold_and_saturation():
    """Edge 3, volume 27: 5 particles (density 0.185) is gas and 6 (0.222) is
    liquid at rho_gas = 0.2; 300 particles in one subcell saturate the byte."""
    counts = np.full((4, 4, 4), 8)
    counts[0, 0, 0] = 5
    counts[1, 1, 1] = 6
    counts[2, 2, 2] = 300
    q = inputs.subcell_field_positions(counts, 12.0, 1)
    r = oracle.bubbles(q, 12.0)
    assert r.threshold == pytest.approx(5.4)
    assert r.counts[0] == 5 and r.labels[0] == 0
    assert r.counts[(1 * 4 + 1) * 4 + 1] == 6 and r.labels[(1 * 4 + 1) * 4 + 1] == -1
    assert r.counts[(2 * 4 + 2) * 4 + 2] == 255
    assert list(r.roots) == [0] and list(r.sizes) == [1]


@pytest.mark.parametrize("seed,p", [(1, 0.2), (2, 0.3), (3, 0.45)])
def test_bubble_labels_match_scipy_interior(seed, p):
    """Gas patterns kept off the box faces: clusters equal scipy's face-connected
    labelling, each labelled by its smallest linear subcell index."""
    shape = (8, 9, 10)
    L = (30.0, 27.0, 24.0)
    gas, counts = inputs.bubble_field(shape, p, seed, border=True)
    q = inputs.subcell_field_positions(counts, L, seed)
    r = oracle.bubbles(q, L)
    assert r.nsub == (10, 9, 8)
    np.testing.assert_array_equal(r.labels, _union_find_components(gas, periodic=False))


@pytest.mark.parametrize("seed,p", [(4, 0.25), (5, 0.32), (6, 0.5)])
def test_bubble_labels_match_scipy_periodic(seed, p):
    """Gas patterns touching the faces: clusters equal scipy's labelling merged
    across the periodic boundaries."""
    shape = (7, 6, 9)
    L = (27.0, 18.0, 21.0)
    gas, counts = inputs.bubble_field(shape, p, seed)
    q = inputs.subcell_field_positions(counts, L, seed + 10)
    r = oracle.bubbles(q, L)
    ref = _union_find_components(gas, periodic=True)
    np.testing.assert_array_equal(r.labels, ref)
    assert r.sizes.sum() == gas.sum()


def test_bubble_special_shapes():
    """A tube through the periodic x faces is one bubble; subcells touching only
    along an edge are two; all gas is one bubble; all liquid is none."""
    n = 6
    L = 18.0

    def run(gas):
        counts = np.where(gas, 0, 9)
        return oracle.bubbles(inputs.subcell_field_positions(counts, L, 7), L)

    g = np.zeros((n, n, n), bool)
    g[2, 3, :] = True
    r = run(g)
    assert list(r.sizes) == [n] and list(r.roots) == [(2 * n + 3) * n]
    g = np.zeros((n, n, n), bool)
    g[1, 1, 0] = g[1, 1, n - 1] = True         # neighbours across the x face
    g[4, 4, 4] = g[4, 3, 3] = True             # edge contact only
    r = run(g)
    assert sorted(r.sizes.tolist()) == [1, 1, 2]
    assert r.labels[(1 * n + 1) * n + n - 1] == (1 * n + 1) * n
    r = run(np.ones((n, n, n), bool))
    assert list(r.sizes) == [n ** 3] and list(r.roots) == [0]
    r = run(np.zeros((n, n, n), bool))
    assert r.roots.size == 0 and (r.labels == -1).all()


def test_bubble_single_subcell_axis():
    """An axis with one subcell is its own periodic neighbour."""
    counts = np.zeros((1, 2, 3), dtype=np.int64)
    counts[0, 1, :] = 30
    q = inputs.subcell_field_positions(counts, (15.0, 10.0, 5.0), 2)
    r = oracle.bubbles(q, (15.0, 10.0, 5.0), side=5.0, rho_gas=0.2)
    assert r.nsub == (3, 2, 1)
    assert list(r.roots) == [0] and list(r.sizes) == [3]


def test_thermostat_splitting_is_time_reversible():
    """thermostat(dt/2) . velocity Verlet . thermostat(dt/2) is a symmetric
    splitting: 50 steps forward, then 50 with v and xi negated, return to the
    start (positions and velocities to rounding, xi to zero).  An asymmetric
    order of the half steps, or a wrong sign in the friction, breaks this."""
    w = inputs.small_nve()
    r1 = oracle.run_obs(w.pos, w.vel, w.box, 50, energy_every=10, T=1.5, tau=0.1)
    assert abs(r1.xi) > 1e-3  # the thermostat acted
    r2 = oracle.run_obs(r1.q, -r1.v, w.box, 50, energy_every=10, T=1.5, tau=0.1, xi=-r1.xi)
    d = r2.q - w.pos
    d -= 20.0 * np.rint(d / 20.0)
    assert np.abs(d).max() < 1e-11
    assert np.abs(r2.v + w.vel).max() < 1e-11
    assert abs(r2.xi) < 1e-12
