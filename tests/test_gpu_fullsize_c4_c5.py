"""GPU parity at the full sizes of the cavitation box and the 256-box ensemble.

Cavitation (Sec. IV.A protocol): 128^3 simple-cubic sites at density 0.7
(2,097,152 particles, rc = 3.0, skin 0.3) held at T = 0.9 by the Nose-Hoover
thermostat for 200 steps, every length scaled by 1.1, then 200 NVE steps on the
FP32-mixed path (default format, and row tiles).  Lists are uneven after the
expansion; all cell ids must be bit-exact, 2000 sampled neighbour sets bit-exact (a random sample plus the
longest and shortest lists) and the sampled forces within 1e-5 of the FP64
oracle.

Ensemble: the 256 boxes of inputs.batch_spec(256) (N from 2,000 to 65,536,
density 0.3 to 0.8, T 0.7 to 1.2), FP32-mixed, autotuned, advanced in
captured graphs.  For 16 boxes, among them the smallest and largest N and the
lowest and highest density: E(0) against the oracle, then after 50 steps every
cell id, every neighbour set and every force against the oracle, and the
per-particle energy deviation over the 50 steps.  The 50 graph steps equal 50
eager steps bit for bit.
"""
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


@pytest.mark.parametrize("tiles", [False, True], ids=["default", "row-tiles"])
def test_cavitation_2m_after_expansion_sampled_parity(tiles):
    b = B()
    w = inputs.cavitation_liquid()
    assert w.n == 2097152
    alpha = 1.1
    L1 = w.box[0] * alpha
    rl = w.rc + w.skin
    flags = b.MD_F_TILE_ON if tiles else 0
    with b.Context(b.make_params(w.n, w.box, rc=w.rc, skin=w.skin, dt=w.dt, precision=b.MD_PREC_FP32_MIXED,
                                 flags=flags)) as c:
        c.set_state(w.pos, w.vel)
        c.set_thermostat(w.T, 0.5)
        c.step(200)
        c.set_thermostat(None, 0.0)
        c.rescale_box(alpha)
        c.step(200)
        q, _ = c.get_state()
        c.build_neighbors()
        F = c.compute_forces()
        cells, nc = c.get_cells()
        kp, pl = c.get_neighbors()
        cnt = (kp[1:] - kp[:-1]).cpu().numpy()
        rng = np.random.Generator(np.random.PCG64(91))
        order = np.argsort(cnt, kind="stable")
        ids = np.unique(np.concatenate([rng.choice(w.n, 1900, replace=False), order[:50], order[-50:]]))
        idt = torch.as_tensor(ids, device=kp.device)
        starts, ends = kp[idt].cpu().numpy(), kp[idt + 1].cpu().numpy()
        sets = [pl[s:e].cpu().numpy() for s, e in zip(starts, ends)]
        F = F[idt].cpu().numpy()
        cells = cells.cpu().numpy()
        del kp, pl
    assert cnt.max() > 1.3 * cnt.mean() and cnt.min() < 0.7 * cnt.mean()  # uneven lists
    q = q.cpu().numpy()
    qw, cref, ncref = oracle.cells(q, (L1, L1, L1), rl)
    assert tuple(ncref) == tuple(nc)
    np.testing.assert_array_equal(cells, cref)
    ref = oracle.neighbors_sample(qw, (L1, L1, L1), rl, ids)
    for s_, r in zip(sets, ref):
        np.testing.assert_array_equal(s_, r)
    Fr, A, _ = oracle.forces_sample(qw, (L1, L1, L1), w.rc, ids)
    assert (np.linalg.norm(F - Fr, axis=1) / A).max() <= 1e-5


def _picked(spec, k=16):
    n, rho = spec.n, spec.rho
    pick = {int(np.argmin(n)), int(np.argmax(n)), int(np.argmin(rho)), int(np.argmax(rho))}
    for b in range(0, n.size, 17):
        if len(pick) >= k:
            break
        pick.add(b)
    return sorted(pick)


def test_ensemble256_per_box_parity_and_graph_equals_eager(tmp_path):
    b = B()
    spec = inputs.batch_spec(256)
    boxes = [inputs.batch_box(spec, k) for k in range(256)]
    offs = np.concatenate([[0], np.cumsum([p.shape[0] for p, _, _ in boxes])])
    pos = np.concatenate([p for p, _, _ in boxes])
    vel = np.concatenate([v for _, v, _ in boxes])
    cache = str(tmp_path / "tune.txt")
    picked = _picked(spec)
    assert len(picked) >= 16
    res = {}
    for name, flags in (("graph", b.MD_F_GRAPH), ("eager", 0)):
        params = [b.make_params(p.shape[0], L, precision=b.MD_PREC_FP32_MIXED, flags=flags) for p, _, L in boxes]
        with b.Context(params) as c:
            c.set_state(pos, vel)
            ke0, pe0 = c.batch_energy()
            c.autotune(cache)  # the second context reads the first one's choice
            c.step(50, energy_every=10)
            q, v = c.get_state()
            kes, pes = c.energy_series()
            r = {"q": q.cpu().numpy(), "v": v.cpu().numpy(), "ke0": ke0, "pe0": pe0, "E": kes + pes,
                 "st": c.stats()}
            if name == "graph":
                c.build_neighbors()
                kp, pl = c.get_neighbors()
                r["kp"], r["pl"] = kp.cpu().numpy(), pl.cpu().numpy()
                r["cells"] = c.get_cells()[0].cpu().numpy()
                r["F"] = c.compute_forces().cpu().numpy()
            res[name] = r
    g, e = res["graph"], res["eager"]
    np.testing.assert_array_equal(g["q"], e["q"])
    np.testing.assert_array_equal(g["v"], e["v"])
    np.testing.assert_array_equal(g["E"], e["E"])
    assert g["st"]["rebuilds"] == e["st"]["rebuilds"]
    for k in picked:
        p0, v0, L = boxes[k]
        a, z = offs[k], offs[k + 1]
        n = z - a
        # E(0) of the box against the oracle
        _, pe_r, _ = oracle.forces(p0, L, 2.5, 0.3)
        assert g["pe0"][k] == pytest.approx(pe_r, rel=1e-6, abs=1e-6 * n)
        assert g["ke0"][k] == pytest.approx(oracle.kinetic(v0), rel=1e-13)
        # energy deviation per particle over the 50 steps (E recorded every 10 steps)
        E = g["E"][:, k]
        assert np.abs(E - (g["ke0"][k] + g["pe0"][k])).max() / n <= 2e-3
        # after 50 steps: cells, every neighbour set and every force of the box
        q = g["q"][a:z]
        qw, cref, _ = oracle.cells(q, L, 2.8)
        np.testing.assert_array_equal(g["cells"][a:z], cref)
        kpr, plr = oracle.neighbors(qw, L, 2.8)
        kpb = g["kp"][a:z + 1]
        np.testing.assert_array_equal(kpb - kpb[0], kpr)
        np.testing.assert_array_equal(g["pl"][kpb[0]:kpb[-1]] - a, plr)
        c2, c0 = oracle.coeffs(2.5)
        Fr, _, A = oracle.forces_list(qw, L, 2.5, kpr, plr, c2, c0)
        assert (np.linalg.norm(g["F"][a:z] - Fr, axis=1) / A).max() <= 1e-5, k
