"""The half list with Newton's third law (MD_F_HALF_LIST) against the oracle.

Each unordered pair within the list radius appears exactly once (bit-exact
decisions, so the pair set equals the oracle's half list of Fig. 1); forces,
energies and pressure meet the same bars as the full list (FP64 1e-12,
FP32-mixed 1e-5 normalised); trajectories as for the full list.  The order of
the atomic additions varies, so results are compared within tolerance, never
bitwise.
"""
import numpy as np
import pytest

import oracle
from paper_1210_3450_amd import inputs
from test_gpu_parity import CASES, _wrapdiff, case, norm_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def B():
    from paper_1210_3450_amd import binding
    return binding


def half_ctx(pos, vel, L, precision=0, flags=0, **kw):
    b = B()
    p = b.make_params(pos.shape[0], L, precision=precision, flags=b.MD_F_HALF_LIST | flags, **kw)
    c = b.Context(p)
    c.set_state(pos, vel)
    return c


def pairs_of(kp, pl):
    kp = np.asarray(kp)
    keys = np.repeat(np.arange(kp.shape[0] - 1), np.diff(kp))
    return keys, np.asarray(pl)


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("precision", [0, 1])
def test_half_list_holds_each_pair_once(name, precision):
    q, v, L = case(name)
    with half_ctx(q, v, L, precision=precision) as c:
        c.build_neighbors()
        kp, pl = c.get_neighbors()
        st = c.stats()
    i, j = pairs_of(kp.cpu().numpy(), pl.cpu().numpy())
    lo, hi = np.minimum(i, j), np.maximum(i, j)
    assert (lo != hi).all()
    n = q.shape[0]
    code = lo.astype(np.int64) * n + hi
    assert np.unique(code).size == code.size  # no pair twice
    kpr, plr = oracle.neighbors(q, L, 2.8, half=True)
    ir, jr = pairs_of(kpr, plr)
    np.testing.assert_array_equal(np.sort(code), np.sort(ir.astype(np.int64) * n + jr))
    assert st["list_entries"] == kpr[-1]
    assert st["threads_per_key"] == 1


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("precision,tol,etol", [(0, 1e-12, 1e-12), (1, 1e-5, 1e-6)])
def test_half_list_forces_energy_pressure(name, precision, tol, etol):
    q, v, L = case(name)
    with half_ctx(q, v, L, precision=precision) as c:
        F = c.compute_forces().cpu().numpy()
        ke, pe = c.energy()
        P = c.pressure()[0]
    Fr, per, A = oracle.forces(q, L, 2.5, 0.3)
    assert norm_err(F, Fr, A) <= tol
    assert pe == pytest.approx(per, rel=etol, abs=etol * 1e-3)
    Lv = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,))
    Pr = oracle.pressure(oracle.kinetic(v), oracle.virial(q, L, 2.5), float(np.prod(Lv)))
    assert P == pytest.approx(Pr, rel=etol, abs=etol * 1e-3)


@pytest.mark.parametrize("graph", [False, True])
def test_half_list_trajectory_fp64_matches_oracle(graph):
    """4000-particle FCC, 100 steps: positions within 1e-9 of the oracle, the
    energy series within 1e-10, the same rebuilds."""
    b = B()
    w = inputs.small_nve()
    r = oracle.run(w.pos, w.vel, w.box, 100, energy_every=10)
    with half_ctx(w.pos, w.vel, w.box[0], flags=b.MD_F_GRAPH if graph else 0) as c:
        c.step(60, energy_every=10)
        c.step(40, energy_every=10)
        pos, vel = c.get_state()
        ke, pe = c.energy_series()
        st = c.stats()
    assert np.abs(_wrapdiff(pos.cpu().numpy(), r.q, w.box)).max() < 1e-9
    assert np.abs(vel.cpu().numpy() - r.v).max() < 1e-9
    np.testing.assert_allclose(ke[:, 0], r.ke, rtol=1e-10)
    np.testing.assert_allclose(pe[:, 0], r.pe, rtol=1e-10)
    assert st["rebuilds"] == r.rebuilds


def test_half_list_mixed_tracks_fp64_and_conserves_energy():
    w = inputs.small_nve()
    r = oracle.run(w.pos, w.vel, w.box, 100, energy_every=10)
    with half_ctx(w.pos, w.vel, w.box[0], precision=1) as c:
        c.step(100, energy_every=10)
        pos, _ = c.get_state()
        ke, pe = c.energy_series()
    assert np.abs(_wrapdiff(pos.cpu().numpy(), r.q, w.box)).max() < 1e-5
    E = ke[:, 0] + pe[:, 0]
    Er = r.ke + r.pe
    assert np.abs(E - Er).max() / abs(Er[0]) < 1e-5


def test_half_list_thermostat_matches_oracle():
    w = inputs.small_nve()
    r = oracle.run_obs(w.pos, w.vel, w.box, 100, energy_every=10, T=1.5, tau=0.1)
    with half_ctx(w.pos, w.vel, w.box[0]) as c:
        c.set_thermostat(1.5, 0.1)
        c.step(100, 10)
        q, _ = c.get_state()
        ke, pe = c.energy_series()
        vir, th = c.observable_series()
    assert np.abs(_wrapdiff(q.cpu().numpy(), r.q, w.box)).max() < 1e-9
    np.testing.assert_allclose(ke[:, 0], r.ke, rtol=1e-9)
    np.testing.assert_allclose(vir[:, 0], r.vir, rtol=1e-9)
    np.testing.assert_allclose(th[:, 0], r.thermo, rtol=1e-8, atol=1e-8)


@pytest.mark.parametrize("precision", [0, 1])
def test_half_list_ensemble_matches_per_box_oracle(precision):
    b = B()
    spec = inputs.batch_spec(4, seed=7, nmin=2000, nmax=9000)
    boxes = [inputs.batch_box(spec, k) for k in range(4)]
    params = [b.make_params(p.shape[0], L, precision=precision, flags=b.MD_F_HALF_LIST | b.MD_F_GRAPH)
              for p, _, L in boxes]
    tol = 1e-12 if precision == 0 else 1e-5
    with b.Context(params) as c:
        c.set_state(np.concatenate([p for p, _, _ in boxes]), np.concatenate([v for _, v, _ in boxes]))
        F = c.compute_forces().cpu().numpy()
        _, pe = c.batch_energy()
        c.autotune()  # nothing to choose: still one lane per key
        c.step(50, energy_every=25)
        pos, _ = c.get_state()
        st = c.stats()
    pos = pos.cpu().numpy()
    assert st["threads_per_key"] == 1
    off = 0
    for k, (p, v, L) in enumerate(boxes):
        n = p.shape[0]
        Fr, per, A = oracle.forces(p, L, 2.5, 0.3)
        assert norm_err(F[off:off + n], Fr, A) <= tol
        assert pe[k] == pytest.approx(per, rel=1e-12 if precision == 0 else 1e-6)
        if precision == 0:
            rr = oracle.run(p, v, L, 50, energy_every=25)
            assert np.abs(_wrapdiff(pos[off:off + n], rr.q, L)).max() < 1e-9
        off += n


def test_half_list_full_size_1m_forces():
    """1,048,576 particles: every force of both precisions within its bar.  The
    potential energy sums 1.7e7 pair terms of one sign in an order that differs
    from the oracle's; its rounding grows like sqrt(terms) * eps (about 5e-13
    relative here), so the FP64 energy bar at this size is 1e-11."""
    w = inputs.medium_1m()
    Fr, per, A = oracle.forces(w.pos, w.box, 2.5, 0.3)
    for precision, tol in ((0, 1e-12), (1, 1e-5)):
        with half_ctx(w.pos, w.vel, w.box[0], precision=precision) as c:
            F = c.compute_forces().cpu().numpy()
            _, pe = c.energy()
        assert norm_err(F, Fr, A) <= tol
        assert pe == pytest.approx(per, rel=1e-11 if precision == 0 else 1e-6)


@pytest.mark.parametrize("policy", [1, 2])
def test_half_list_other_rebuild_policies_match_oracle(policy):
    """Displacement and every-step rebuilds with the half list (the integration
    pass carries the displacement maximum)."""
    w = inputs.small_nve()
    r = oracle.run(w.pos, w.vel, w.box, 60, rebuild=policy)
    with half_ctx(w.pos, w.vel, w.box[0], rebuild=policy) as c:
        c.step(60)
        pos, _ = c.get_state()
        st = c.stats()
    assert np.abs(_wrapdiff(pos.cpu().numpy(), r.q, w.box)).max() < 1e-9
    assert st["rebuilds"] == r.rebuilds


def test_half_list_overflow_regrows_at_build_and_during_steps():
    q, v, L = case("clustered")
    with half_ctx(q, v, L, list_cap=8) as c:
        c.build_neighbors()
        kp, pl = c.get_neighbors()
        assert c.stats()["list_regrows"] >= 1
    i, j = pairs_of(kp.cpu().numpy(), pl.cpu().numpy())
    n = q.shape[0]
    kpr, plr = oracle.neighbors(q, L, 2.8, half=True)
    ir, jr = pairs_of(kpr, plr)
    np.testing.assert_array_equal(np.sort(np.minimum(i, j).astype(np.int64) * n + np.maximum(i, j)),
                                  np.sort(ir.astype(np.int64) * n + jr))
    # a lattice heated to T = 3: the longest half list grows past the capacity of the first build
    rng = np.random.Generator(np.random.PCG64(11))
    q0, v0 = inputs.fcc_positions(5, 2.0), inputs.maxwell_boltzmann(500, 3.0, 1.0, rng)
    with half_ctx(q0, v0, 10.0) as c:
        c.build_neighbors()
        cap0 = (c.stats()["max_list_len"] + 7) // 8 * 8
    r = oracle.run(q0, v0, 10.0, 120)
    with half_ctx(q0, v0, 10.0, list_cap=cap0) as c:
        c.step(120)
        pos, _ = c.get_state()
        st = c.stats()
    assert st["list_regrows"] >= 1
    assert np.abs(_wrapdiff(pos.cpu().numpy(), r.q, 10.0)).max() < 1e-9
