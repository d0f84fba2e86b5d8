"""Plain FP64 CPU oracle for the truncated-LJ hot path (ctypes over md_oracle.c).

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg import this package.  It shares no code with the
HIP library and never calls it.

Arrays are numpy float64 (n, 3) in caller order unless stated.  Functions that
bin particles wrap a *copy* of the positions unless ``inplace=True``.

Constants of the cutoff schemes and rebuild policies mirror the C file.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import sys
from dataclasses import dataclass

import numpy as np

CUT_EQ1, CUT_SHIFT, CUT_RAW = 0, 1, 2
REBUILD_DUTC, REBUILD_DISPLACEMENT, REBUILD_EVERY_STEP, REBUILD_NEVER = 0, 1, 2, 3

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "md_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC", "-std=c11"]


def build_sanitized(out: str) -> str:
    """Compile md_oracle.c with AddressSanitizer and UndefinedBehaviorSanitizer into
    out (load it by setting MD_ORACLE_LIB, with gcc's libasan preloaded)."""
    flags = [f for f in _CFLAGS if not f.startswith("-O")]
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", *flags, "-o", out, _SRC, "-lm"])
    return out


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *_CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None

P_D = C.POINTER(C.c_double)
P_I32 = C.POINTER(C.c_int32)
P_I64 = C.POINTER(C.c_int64)


class OrcParams(C.Structure):
    _fields_ = [("rc", C.c_double), ("skin", C.c_double), ("dt", C.c_double), ("mass", C.c_double),
                ("cutoff", C.c_int32), ("rebuild", C.c_int32), ("verify", C.c_int32), ("rcp", C.c_int32)]


class OrcThermo(C.Structure):
    _fields_ = [("T", C.c_double), ("tau", C.c_double), ("xi", C.c_double), ("eta", C.c_double)]


class OrcStats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("rebuilds", C.c_int64), ("missed_pairs", C.c_int64),
                ("D", C.c_double)]


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("MD_ORACLE_LIB")  # another build of md_oracle.c (sanitizer runs)
        if not path:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            path = _LIB
        L = C.CDLL(path)
        L.orc_num_threads.restype = C.c_int
        L.orc_coeffs.argtypes = [C.c_double, C.c_int, P_D, P_D]
        L.orc_pair_v.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_pair_v.restype = C.c_double
        L.orc_pair_f.argtypes = [C.c_double, C.c_double]
        L.orc_pair_f.restype = C.c_double
        L.orc_cell_grid.argtypes = [P_D, C.c_double, P_I32, P_D]
        L.orc_cells.argtypes = [C.c_int64, P_D, P_D, C.c_double, P_I32, P_I32]
        L.orc_cells.restype = C.c_int
        for name in ("orc_neighbors", "orc_neighbors_brute"):
            f = getattr(L, name)
            f.argtypes = [C.c_int64, P_D, P_D, C.c_double, C.c_int, P_I64, P_I32, C.c_int64]
            f.restype = C.c_int64
        L.orc_forces_list.argtypes = [C.c_int64, P_D, P_D, C.c_double, C.c_double, C.c_double,
                                      P_I64, P_I32, P_D, P_D, P_D]
        L.orc_forces_list.restype = C.c_double
        L.orc_forces_list_rcp.argtypes = [C.c_int64, P_D, P_D, C.c_double, C.c_double, C.c_double,
                                          P_I64, P_I32, P_D, P_D, P_D, C.c_int]
        L.orc_forces_list_rcp.restype = C.c_double
        L.orc_rcp_approx.argtypes = [C.c_double]
        L.orc_rcp_approx.restype = C.c_double
        L.orc_rpow_approx.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int]
        L.orc_rpow_approx.restype = C.c_double
        L.orc_virial_list.argtypes = [C.c_int64, P_D, P_D, C.c_double, C.c_double, P_I64, P_I32]
        L.orc_virial_list.restype = C.c_double
        L.orc_run_obs.argtypes = [C.c_int64, P_D, P_D, P_D, P_D, C.POINTER(OrcParams), C.POINTER(OrcThermo),
                                  C.c_int64, C.c_int64, P_D, P_D, P_D, P_D, C.POINTER(OrcStats), C.c_int32]
        L.orc_run_obs.restype = C.c_int
        L.orc_forces_brute.argtypes = [C.c_int64, P_D, P_D, C.c_double, C.c_double, C.c_double, P_D, P_D]
        L.orc_forces_brute.restype = C.c_double
        L.orc_forces_sample.argtypes = [C.c_int64, P_D, P_D, C.c_double, C.c_double, C.c_double,
                                        C.c_int64, P_I64, P_D, P_D, P_D]
        L.orc_forces_sample.restype = C.c_int
        L.orc_neighbors_sample.argtypes = [C.c_int64, P_D, P_D, C.c_double, C.c_int64, P_I64,
                                           P_I32, C.c_int64, P_I64]
        L.orc_neighbors_sample.restype = C.c_int
        L.orc_kinetic.argtypes = [C.c_int64, P_D, C.c_double]
        L.orc_kinetic.restype = C.c_double
        L.orc_run.argtypes = [C.c_int64, P_D, P_D, P_D, P_D, C.POINTER(OrcParams), C.c_int64,
                              C.c_int64, P_D, P_D, C.POINTER(OrcStats), C.c_int32]
        L.orc_run.restype = C.c_int
        L.orc_bubbles.argtypes = [C.c_int64, P_D, P_D, C.c_double, C.c_double, C.POINTER(C.c_uint8), P_I32]
        L.orc_bubbles.restype = C.c_int64
        L.orc_subcell_grid.argtypes = [P_D, C.c_double, P_I32, P_D, P_D, C.c_double]
        _lib = L
    return _lib


def _pd(a):
    return a.ctypes.data_as(P_D)


def _box(L):
    return np.ascontiguousarray(np.broadcast_to(np.asarray(L, dtype=np.float64), (3,)).copy())


def _q(q, inplace=False):
    q = np.asarray(q, dtype=np.float64)
    if inplace:
        assert q.flags.c_contiguous and q.shape[1] == 3
        return q
    return np.ascontiguousarray(q).copy()


def num_threads() -> int:
    return int(lib().orc_num_threads())


def coeffs(rc: float, mode: int = CUT_EQ1):
    c2, c0 = C.c_double(), C.c_double()
    lib().orc_coeffs(rc, mode, C.byref(c2), C.byref(c0))
    return c2.value, c0.value


def pair_v(r2: float, c2: float, c0: float) -> float:
    return lib().orc_pair_v(r2, c2, c0)


def pair_f(r2: float, c2: float) -> float:
    return lib().orc_pair_f(r2, c2)


def cell_grid(L, r_list):
    Lb = _box(L)
    n = np.zeros(3, np.int32)
    inv = np.zeros(3, np.float64)
    lib().orc_cell_grid(_pd(Lb), r_list, n.ctypes.data_as(P_I32), _pd(inv))
    return n, inv


def cells(q, L, r_list, inplace=False):
    """Returns (wrapped positions, cell id per particle, ncell[3]); raises on bad input."""
    q = _q(q, inplace)
    Lb = _box(L)
    cell = np.zeros(q.shape[0], np.int32)
    nc = np.zeros(3, np.int32)
    rc = lib().orc_cells(q.shape[0], _pd(q), _pd(Lb), r_list, cell.ctypes.data_as(P_I32),
                         nc.ctypes.data_as(P_I32))
    if rc != 0:
        raise ValueError("orc_cells failed with code %d" % rc)
    return q, cell, nc


def neighbors(q, L, r_list, half=False, brute=False):
    """Pair list within r_list as CSR (key_ptr[n+1] int64, partners int32 ascending).
    half=True gives the sorted half list (key = smaller id), else the full list."""
    q = _q(q)
    Lb = _box(L)
    n = q.shape[0]
    kp = np.zeros(n + 1, np.int64)
    f = lib().orc_neighbors_brute if brute else lib().orc_neighbors
    tot = f(n, _pd(q), _pd(Lb), r_list, int(half), kp.ctypes.data_as(P_I64), None, 0)
    if tot < 0:
        raise ValueError("oracle neighbour search failed with code %d" % tot)
    pl = np.zeros(max(tot, 1), np.int32)
    q2 = _q(q)
    f(n, _pd(q2), _pd(Lb), r_list, int(half), kp.ctypes.data_as(P_I64), pl.ctypes.data_as(P_I32), tot)
    return kp, pl[:tot]


# reciprocal modes of the force evaluation (Sec. III.C): IEEE division, the
# paper's approximate reciprocal (relative error < 1/256) without and with its
# correction, and an exact reciprocal through the corrected formulas
RCP_DIV, RCP_APPROX, RCP_APPROX_CORR, RCP_EXACT_CORR = 0, 1, 2, 3


def rcp_approx(x):
    return lib().orc_rcp_approx(float(x))


def rpow_approx(r2, xt, n, corr):
    """xt^n, times the correction (n + 1) - n xt r^2 when corr."""
    return lib().orc_rpow_approx(float(r2), float(xt), int(n), int(bool(corr)))


def forces_list(q, L, rc, kp, pl, c2, c0, per_particle_pe=False, rcp=RCP_DIV):
    q = _q(q)
    Lb = _box(L)
    n = q.shape[0]
    F = np.zeros((n, 3))
    A = np.zeros(n)
    pe_i = np.zeros(n) if per_particle_pe else None
    kp = np.ascontiguousarray(kp, dtype=np.int64)
    pl = np.ascontiguousarray(pl, dtype=np.int32)
    pe = lib().orc_forces_list_rcp(n, _pd(q), _pd(Lb), rc, c2, c0, kp.ctypes.data_as(P_I64),
                                   pl.ctypes.data_as(P_I32), _pd(F), _pd(A),
                                   _pd(pe_i) if pe_i is not None else None, int(rcp))
    return (F, pe, A, pe_i) if per_particle_pe else (F, pe, A)


def forces(q, L, rc, skin=0.0, mode=CUT_EQ1, rcp=RCP_DIV):
    """F, PE and the absolute pair-force sum A at positions q (list at rc + skin)."""
    c2, c0 = coeffs(rc, mode)
    qw, _, _ = cells(q, L, rc + skin)
    kp, pl = neighbors(qw, L, rc + skin)
    return forces_list(qw, L, rc, kp, pl, c2, c0, rcp=rcp)


def forces_brute(q, L, rc, mode=CUT_EQ1):
    q = _q(q)
    Lb = _box(L)
    c2, c0 = coeffs(rc, mode)
    F = np.zeros((q.shape[0], 3))
    A = np.zeros(q.shape[0])
    pe = lib().orc_forces_brute(q.shape[0], _pd(q), _pd(Lb), rc, c2, c0, _pd(F), _pd(A))
    return F, pe, A


def forces_sample(q, L, rc, ids, mode=CUT_EQ1):
    """F, A and per-particle PE (1/2 sum V) for the sampled ids only."""
    q = _q(q)
    Lb = _box(L)
    c2, c0 = coeffs(rc, mode)
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    m = ids.shape[0]
    F = np.zeros((m, 3))
    A = np.zeros(m)
    pe = np.zeros(m)
    rcode = lib().orc_forces_sample(q.shape[0], _pd(q), _pd(Lb), rc, c2, c0, m,
                                    ids.ctypes.data_as(P_I64), _pd(F), _pd(A), _pd(pe))
    if rcode != 0:
        raise ValueError("orc_forces_sample failed with code %d" % rcode)
    return F, A, pe


def neighbors_sample(q, L, r_list, ids, cap=512):
    """Full-list partner sets of the sampled ids: list of int32 arrays, ascending."""
    q = _q(q)
    Lb = _box(L)
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    m = ids.shape[0]
    out = np.zeros((m, cap), np.int32)
    cnt = np.zeros(m, np.int64)
    rcode = lib().orc_neighbors_sample(q.shape[0], _pd(q), _pd(Lb), r_list, m, ids.ctypes.data_as(P_I64),
                                       out.ctypes.data_as(P_I32), cap, cnt.ctypes.data_as(P_I64))
    if rcode != 0:
        raise ValueError("orc_neighbors_sample failed with code %d" % rcode)
    if (cnt > cap).any():
        raise ValueError("sample capacity too small")
    return [out[s, :cnt[s]].copy() for s in range(m)]


def kinetic(v, mass=1.0) -> float:
    v = np.ascontiguousarray(v, dtype=np.float64)
    return lib().orc_kinetic(v.shape[0], _pd(v), mass)


@dataclass
class RunResult:
    q: np.ndarray
    v: np.ndarray
    F: np.ndarray
    ke: np.ndarray
    pe: np.ndarray
    steps: int
    rebuilds: int
    missed_pairs: int
    D: float


def run(q, v, L, nsteps, rc=2.5, skin=0.3, dt=0.005, mass=1.0, mode=CUT_EQ1,
        rebuild=REBUILD_DUTC, energy_every=0, verify=False, rcp=RCP_DIV) -> RunResult:
    """Velocity-Verlet NVE run from (q, v) with a fresh initial list and forces."""
    q = _q(q)
    v = np.ascontiguousarray(v, dtype=np.float64).copy()
    Lb = _box(L)
    n = q.shape[0]
    F = np.zeros((n, 3))
    p = OrcParams(rc, skin, dt, mass, mode, rebuild, int(verify), int(rcp))
    st = OrcStats(0, 0, 0, 0.0)
    ns = nsteps // energy_every if energy_every > 0 else 0
    ke = np.zeros(max(ns, 1))
    pe = np.zeros(max(ns, 1))
    rcode = lib().orc_run(n, _pd(q), _pd(v), _pd(F), _pd(Lb), C.byref(p), nsteps, energy_every,
                          _pd(ke), _pd(pe), C.byref(st), 0)
    if rcode != 0:
        raise ValueError("orc_run failed with code %d" % rcode)
    return RunResult(q, v, F, ke[:ns], pe[:ns], st.steps, st.rebuilds, st.missed_pairs, st.D)


def virial(q, L, rc, skin=0.3, mode=CUT_EQ1):
    """Pair virial sum_{i<j, r<rc} f(r) r^2 at positions q (f = V'(r)/r)."""
    c2, _ = coeffs(rc, mode)
    qw, _, _ = cells(q, L, rc + skin)
    kp, pl = neighbors(qw, L, rc + skin)
    return lib().orc_virial_list(qw.shape[0], _pd(qw), _pd(_box(L)), rc, c2, kp.ctypes.data_as(P_I64),
                                 pl.ctypes.data_as(P_I32))


def pressure(ke, vir, volume):
    """Virial pressure P = (2 KE - sum_{i<j} f r^2) / (3 V)."""
    return (2.0 * ke - vir) / (3.0 * volume)


@dataclass
class ObsResult:
    q: np.ndarray
    v: np.ndarray
    F: np.ndarray
    ke: np.ndarray
    pe: np.ndarray
    vir: np.ndarray
    thermo: np.ndarray   # thermostat share Q xi^2 / 2 + g T eta of the conserved quantity
    xi: float
    eta: float
    steps: int
    rebuilds: int


def run_obs(q, v, L, nsteps, rc=2.5, skin=0.3, dt=0.005, mass=1.0, mode=CUT_EQ1, energy_every=10,
            T=None, tau=0.0, xi=0.0, eta=0.0, rcp=RCP_DIV) -> ObsResult:
    """Velocity-Verlet run with energies, pair virial and, when tau > 0, a
    Nose-Hoover thermostat at temperature T (relaxation time tau)."""
    q = _q(q)
    v = np.ascontiguousarray(v, dtype=np.float64).copy()
    Lb = _box(L)
    n = q.shape[0]
    F = np.zeros((n, 3))
    p = OrcParams(rc, skin, dt, mass, mode, REBUILD_DUTC, 0, int(rcp))
    th = OrcThermo(float(T) if T is not None else 0.0, float(tau), float(xi), float(eta))
    st = OrcStats(0, 0, 0, 0.0)
    ns = nsteps // energy_every if energy_every > 0 else 0
    ke, pe, vir, tho = (np.zeros(max(ns, 1)) for _ in range(4))
    rcode = lib().orc_run_obs(n, _pd(q), _pd(v), _pd(F), _pd(Lb), C.byref(p), C.byref(th), nsteps,
                              energy_every, _pd(ke), _pd(pe), _pd(vir), _pd(tho), C.byref(st), 0)
    if rcode != 0:
        raise ValueError("orc_run_obs failed with code %d" % rcode)
    return ObsResult(q, v, F, ke[:ns], pe[:ns], vir[:ns], tho[:ns], th.xi, th.eta, st.steps, st.rebuilds)


def csr_sets(kp, pl):
    """Per-key partner arrays of a CSR list."""
    return [pl[kp[i]:kp[i + 1]] for i in range(len(kp) - 1)]


@dataclass
class BubbleResult:
    nsub: tuple          # subcells per axis (nx, ny, nz)
    threshold: float     # gas iff count < threshold
    counts: np.ndarray   # uint8 [nz * ny * nx], linear index (cz*ny + cy)*nx + cx
    labels: np.ndarray   # int32, smallest linear index of the subcell's bubble; -1 liquid
    roots: np.ndarray    # int64 bubble labels, ascending
    sizes: np.ndarray    # int64 subcells per bubble, in the order of roots


def bubbles(q, L, side=3.0, rho_gas=0.2) -> BubbleResult:
    """Bubble identification of Sec. IV.B: byte counts per subcell of edge
    >= side, gas iff count < rho_gas * subcell volume, face-adjacent gas
    subcells (periodic) form one bubble."""
    q = _q(q)
    Lb = _box(L)
    ns = np.zeros(3, dtype=np.int32)
    inv = np.zeros(3)
    thr = C.c_double()
    lib().orc_subcell_grid(_pd(Lb), side, ns.ctypes.data_as(P_I32), _pd(inv), C.byref(thr), rho_gas)
    nsub = int(np.prod(ns.astype(np.int64)))
    counts = np.zeros(nsub, dtype=np.uint8)
    labels = np.zeros(nsub, dtype=np.int32)
    nb = lib().orc_bubbles(q.shape[0], _pd(q), _pd(Lb), side, rho_gas,
                           counts.ctypes.data_as(C.POINTER(C.c_uint8)), labels.ctypes.data_as(P_I32))
    if nb < 0:
        raise ValueError("orc_bubbles failed (%d)" % nb)
    gas = labels[labels >= 0]
    roots, sizes = np.unique(gas, return_counts=True)
    assert roots.shape[0] == nb
    return BubbleResult(tuple(int(x) for x in ns), thr.value, counts, labels, roots.astype(np.int64),
                        sizes.astype(np.int64))
