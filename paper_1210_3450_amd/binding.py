"""ctypes binding of libmdgpu (include/md.h): argument marshalling only.

Every computation happens in the HIP library.  Device arrays are torch CUDA
(HIP) tensors; torch only supplies device memory and streams.  Importing this
module raises if the built library is missing: there is no CPU fallback.

The low-level functions carry the C names (``md_create``, ``md_step``, ...)
and return md_status codes; ``Context`` wraps them, raising ``MDError`` on any
status other than MD_OK.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmdgpu.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libmdgpu.so is not built (expected at %s); run `python -m paper_1210_3450_amd.build`" % LIB_PATH)

# torch ships its own HIP runtime under the same soname (libamdhip64.so.7).  Load
# it first so libmdgpu.so binds to that one runtime: torch's device pointers and
# streams are then valid inside the library, and no second HSA runtime starts.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

# status codes
MD_OK, MD_EINVAL, MD_ENOMEM, MD_EHIP, MD_ENUMERIC, MD_ESTATE, MD_ELIST = 0, -1, -2, -3, -4, -5, -6
MD_PREC_FP64, MD_PREC_FP32_MIXED = 0, 1
MD_CUT_EQ1, MD_CUT_SHIFT, MD_CUT_RAW = 0, 1, 2
MD_REBUILD_DUTC, MD_REBUILD_DISPLACEMENT, MD_REBUILD_EVERY_STEP, MD_REBUILD_NEVER = 0, 1, 2, 3
MD_F_VERIFY_LIST, MD_F_GRAPH, MD_F_TILE_ON, MD_F_TILE_OFF, MD_F_FAST_RCP, MD_F_HALF_LIST = 1, 2, 4, 8, 16, 32


class md_params(C.Structure):
    _fields_ = [("n", C.c_int64), ("box", C.c_double * 3), ("rc", C.c_double), ("skin", C.c_double),
                ("dt", C.c_double), ("mass", C.c_double), ("precision", C.c_int32), ("cutoff", C.c_int32),
                ("rebuild", C.c_int32), ("flags", C.c_uint32), ("threads_per_key", C.c_int32),
                ("list_cap", C.c_int32), ("cell_scale", C.c_double), ("reserved", C.c_uint64 * 5)]


class md_stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("rebuilds", C.c_int64), ("list_regrows", C.c_int64),
                ("missed_pairs", C.c_int64), ("list_entries", C.c_int64), ("max_list_len", C.c_int32),
                ("list_cap", C.c_int32), ("threads_per_key", C.c_int32), ("nbox", C.c_int32),
                ("D", C.c_double), ("force_ms", C.c_double), ("force_launches", C.c_int64),
                ("rebuild_ms", C.c_double), ("rebuild_launches", C.c_int64), ("row_tiles", C.c_int32),
                ("ncell", C.c_int32 * 3), ("cell_scale", C.c_double)]


class md_bubble_info(C.Structure):
    _fields_ = [("nsub", C.c_int32 * 3), ("pad", C.c_int32), ("side", C.c_double * 3), ("threshold", C.c_double),
                ("ngas", C.c_int64), ("nbubbles", C.c_int64), ("largest", C.c_int64)]


_P = C.c_void_p
_PD = C.POINTER(C.c_double)
_PI32 = C.POINTER(C.c_int32)
_PI64 = C.POINTER(C.c_int64)
_S = C.c_int

_SIGS = {
    "md_create": (_S, [C.POINTER(md_params), _P, C.POINTER(_P)]),
    "md_batch_create": (_S, [C.POINTER(md_params), C.c_int32, _P, C.POINTER(_P)]),
    "md_destroy": (_S, [_P]),
    "md_set_state": (_S, [_P, _P, _P]),
    "md_get_state": (_S, [_P, _P, _P]),
    "md_rescale_box": (_S, [_P, C.c_double]),
    "md_scale_velocities": (_S, [_P, _PD]),
    "md_build_cells": (_S, [_P]),
    "md_build_neighbors": (_S, [_P]),
    "md_compute_forces": (_S, [_P, _P]),
    "md_step": (_S, [_P, C.c_int32, C.c_int32]),
    "md_energy": (_S, [_P, _PD, _PD]),
    "md_batch_energy": (_S, [_P, _PD, _PD]),
    "md_energy_series": (_S, [_P, _PD, _PD, C.c_int32, _PI32]),
    "md_observable_series": (_S, [_P, _PD, _PD, C.c_int32, _PI32]),
    "md_pressure": (_S, [_P, _PD]),
    "md_set_thermostat": (_S, [_P, _PD, C.c_double]),
    "md_get_thermostat": (_S, [_P, _PD, _PD]),
    "md_bubbles": (_S, [_P, C.c_int32, C.c_double, C.c_double, _P, _P, _PI64, _PI64, C.c_int64,
                        C.POINTER(md_bubble_info)]),
    "md_bubbles_noalloc": (_S, [_P, C.c_int32, C.c_double, C.c_double, _P, _P, _PI64, _PI64, C.c_int64,
                                C.POINTER(md_bubble_info)]),
    "md_get_cells": (_S, [_P, _P, _PI32]),
    "md_get_neighbors": (_S, [_P, _P, _P, C.c_int64, _PI64]),
    "md_get_stats": (_S, [_P, C.POINTER(md_stats)]),
    "md_set_timing": (_S, [_P, C.c_int32]),
    "md_autotune": (_S, [_P, C.c_char_p]),
    "md_status_str": (C.c_char_p, [_S]),
    "md_last_error": (C.c_char_p, [_P]),
}

for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args
    globals()[_name] = _f

EXPORTED = tuple(_SIGS)


class MDError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__("%s: %s (%s)" % (where, md_status_str(status).decode(), msg))
        self.status = status


def make_params(n, box, rc=2.5, skin=0.3, dt=0.005, mass=1.0, precision=MD_PREC_FP64, cutoff=MD_CUT_EQ1,
                rebuild=MD_REBUILD_DUTC, flags=0, threads_per_key=0, list_cap=0, cell_scale=0.0) -> md_params:
    b = np.broadcast_to(np.asarray(box, dtype=np.float64), (3,))
    p = md_params()
    p.n = int(n)
    for a in range(3):
        p.box[a] = float(b[a])
    p.rc, p.skin, p.dt, p.mass = float(rc), float(skin), float(dt), float(mass)
    p.precision, p.cutoff, p.rebuild = int(precision), int(cutoff), int(rebuild)
    p.flags, p.threads_per_key, p.list_cap = int(flags), int(threads_per_key), int(list_cap)
    p.cell_scale = float(cell_scale)
    return p


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _dev_f64(a, shape, device):
    import torch
    t = torch.as_tensor(a, dtype=torch.float64)
    t = t.to(device).contiguous()
    if tuple(t.shape) != tuple(shape):
        raise ValueError("expected shape %s, got %s" % (shape, tuple(t.shape)))
    return t


class Context:
    """One box (``params`` an md_params) or an ensemble (a list of md_params)."""

    def __init__(self, params, stream=None, device="cuda"):
        import torch
        self.device = torch.device(device)
        if self.device.index is not None:
            torch.cuda.set_device(self.device)
        out = C.c_void_p()
        st = C.c_void_p(stream.cuda_stream) if stream is not None else None
        if isinstance(params, (list, tuple)):
            arr = (md_params * len(params))(*params)
            s = md_batch_create(arr, len(params), st, C.byref(out))
            self.nbox = len(params)
            self.sizes = [int(p.n) for p in params]
        else:
            s = md_create(C.byref(params), st, C.byref(out))
            self.nbox = 1
            self.sizes = [int(params.n)]
        if s != MD_OK:
            raise MDError(s, "md_create", md_last_error(None).decode())
        self.ctx = out
        self.n = sum(self.sizes)

    def _chk(self, s, where):
        if s != MD_OK:
            raise MDError(s, where, md_last_error(self.ctx).decode())

    def close(self):
        if getattr(self, "ctx", None):
            md_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ---- state
    def set_state(self, pos, vel):
        import torch
        p = _dev_f64(pos, (self.n, 3), self.device)
        v = _dev_f64(vel, (self.n, 3), self.device)
        torch.cuda.synchronize(self.device)  # inputs written on torch's stream
        self._chk(md_set_state(self.ctx, _ptr(p), _ptr(v)), "md_set_state")
        torch.cuda.synchronize(self.device)

    def get_state(self):
        import torch
        p = torch.empty((self.n, 3), dtype=torch.float64, device=self.device)
        v = torch.empty((self.n, 3), dtype=torch.float64, device=self.device)
        torch.cuda.synchronize(self.device)
        self._chk(md_get_state(self.ctx, _ptr(p), _ptr(v)), "md_get_state")
        return p, v

    def rescale_box(self, alpha):
        self._chk(md_rescale_box(self.ctx, float(alpha)), "md_rescale_box")

    def scale_velocities(self, scale):
        s = np.ascontiguousarray(np.broadcast_to(np.asarray(scale, dtype=np.float64), (self.nbox,)))
        self._chk(md_scale_velocities(self.ctx, s.ctypes.data_as(_PD)), "md_scale_velocities")

    # ---- hot path
    def build_cells(self):
        self._chk(md_build_cells(self.ctx), "md_build_cells")

    def build_neighbors(self):
        self._chk(md_build_neighbors(self.ctx), "md_build_neighbors")

    def compute_forces(self, out=True):
        import torch
        f = torch.empty((self.n, 3), dtype=torch.float64, device=self.device) if out else None
        torch.cuda.synchronize(self.device)
        self._chk(md_compute_forces(self.ctx, _ptr(f)), "md_compute_forces")
        torch.cuda.synchronize(self.device)  # the library's stream wrote f
        return f

    def step(self, nsteps, energy_every=0):
        self._chk(md_step(self.ctx, int(nsteps), int(energy_every)), "md_step")

    def energy(self):
        ke, pe = C.c_double(), C.c_double()
        self._chk(md_energy(self.ctx, C.byref(ke), C.byref(pe)), "md_energy")
        return ke.value, pe.value

    def batch_energy(self):
        ke = np.zeros(self.nbox)
        pe = np.zeros(self.nbox)
        self._chk(md_batch_energy(self.ctx, ke.ctypes.data_as(_PD), pe.ctypes.data_as(_PD)), "md_batch_energy")
        return ke, pe

    def energy_series(self, max_samples=4096):
        ke = np.zeros((max_samples, self.nbox))
        pe = np.zeros((max_samples, self.nbox))
        cnt = C.c_int32()
        self._chk(md_energy_series(self.ctx, ke.ctypes.data_as(_PD), pe.ctypes.data_as(_PD), max_samples,
                                   C.byref(cnt)), "md_energy_series")
        k = min(cnt.value, max_samples)
        return ke[:k], pe[:k]

    def observable_series(self, max_samples=4096):
        """(vir, thermostat) per sample: pair virial sum_{i<j} f r^2 and Q xi^2/2 + g T eta."""
        vir = np.zeros((max_samples, self.nbox))
        th = np.zeros((max_samples, self.nbox))
        cnt = C.c_int32()
        self._chk(md_observable_series(self.ctx, vir.ctypes.data_as(_PD), th.ctypes.data_as(_PD), max_samples,
                                       C.byref(cnt)), "md_observable_series")
        k = min(cnt.value, max_samples)
        return vir[:k], th[:k]

    def pressure(self):
        P = np.zeros(self.nbox)
        self._chk(md_pressure(self.ctx, P.ctypes.data_as(_PD)), "md_pressure")
        return P

    def set_thermostat(self, T, tau):
        """Nose-Hoover at temperature T (scalar or per box) with relaxation time tau (<= 0: off)."""
        Tb = np.ascontiguousarray(np.broadcast_to(np.asarray(T if T is not None else 0.0, dtype=np.float64),
                                                  (self.nbox,)))
        self._chk(md_set_thermostat(self.ctx, Tb.ctypes.data_as(_PD), float(tau)), "md_set_thermostat")

    def get_thermostat(self):
        xi = np.zeros(self.nbox)
        eta = np.zeros(self.nbox)
        self._chk(md_get_thermostat(self.ctx, xi.ctypes.data_as(_PD), eta.ctypes.data_as(_PD)),
                  "md_get_thermostat")
        return xi, eta

    # ---- bubble analysis
    def bubbles(self, box=0, side=3.0, rho_gas=0.2, fields=True, cap=None, noalloc=False):
        """Bubbles of one box (md_bubbles, or md_bubbles_noalloc with noalloc=True).
        Returns a dict: nsub (nx, ny, nz), side, threshold, ngas, nbubbles, largest,
        roots and sizes (numpy int64, ascending roots; all bubbles unless cap is
        given) and, with fields=True, the byte counts and labels per subcell as
        device tensors (uint8, int32)."""
        import torch
        md_bubbles = md_bubbles_noalloc if noalloc else globals()["md_bubbles"]
        info = md_bubble_info()
        counts = labels = None
        torch.cuda.synchronize(self.device)
        if fields:
            self._chk(md_bubbles(self.ctx, int(box), float(side), float(rho_gas), None, None, None, None, 0,
                                 C.byref(info)), "md_bubbles")
            nsub = int(info.nsub[0]) * int(info.nsub[1]) * int(info.nsub[2])
            counts = torch.empty(nsub, dtype=torch.uint8, device=self.device)
            labels = torch.empty(nsub, dtype=torch.int32, device=self.device)
        k = int(cap) if cap is not None else None
        if k is None:
            if not fields:
                self._chk(md_bubbles(self.ctx, int(box), float(side), float(rho_gas), None, None, None, None, 0,
                                     C.byref(info)), "md_bubbles")
            k = int(info.nbubbles)
        roots = np.zeros(max(k, 1), dtype=np.int64)
        sizes = np.zeros(max(k, 1), dtype=np.int64)
        self._chk(md_bubbles(self.ctx, int(box), float(side), float(rho_gas),
                             _ptr(counts) if fields else None, _ptr(labels) if fields else None,
                             roots.ctypes.data_as(_PI64), sizes.ctypes.data_as(_PI64), k, C.byref(info)),
                  "md_bubbles")
        m = min(k, int(info.nbubbles))
        return {"nsub": tuple(info.nsub), "side": tuple(info.side), "threshold": info.threshold,
                "ngas": info.ngas, "nbubbles": info.nbubbles, "largest": info.largest,
                "roots": roots[:m], "sizes": sizes[:m], "counts": counts, "labels": labels}

    # ---- diagnostics
    def get_cells(self):
        import torch
        c = torch.empty(self.n, dtype=torch.int32, device=self.device)
        nc = (C.c_int32 * 3)()
        torch.cuda.synchronize(self.device)
        self._chk(md_get_cells(self.ctx, _ptr(c), nc), "md_get_cells")
        return c, tuple(nc)

    def get_neighbors(self):
        import torch
        kp = torch.empty(self.n + 1, dtype=torch.int64, device=self.device)
        total = C.c_int64()
        torch.cuda.synchronize(self.device)
        s = md_get_neighbors(self.ctx, _ptr(kp), None, 0, C.byref(total))
        if s not in (MD_OK, MD_EINVAL):
            self._chk(s, "md_get_neighbors")
        pl = torch.empty(max(total.value, 1), dtype=torch.int32, device=self.device)
        torch.cuda.synchronize(self.device)
        self._chk(md_get_neighbors(self.ctx, _ptr(kp), _ptr(pl), total.value, C.byref(total)),
                  "md_get_neighbors")
        return kp, pl[:total.value]

    def stats(self) -> dict:
        st = md_stats()
        self._chk(md_get_stats(self.ctx, C.byref(st)), "md_get_stats")
        out = {name: getattr(st, name) for name, _ in md_stats._fields_}
        out["ncell"] = list(out["ncell"])
        return out

    def set_timing(self, on=True):
        self._chk(md_set_timing(self.ctx, int(bool(on))), "md_set_timing")

    def autotune(self, cache_path=None):
        self._chk(md_autotune(self.ctx, cache_path.encode() if cache_path else None), "md_autotune")
