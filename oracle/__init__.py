"""ctypes binding of the plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

Only tests/, the smoke check and the benchmark's CPU-baseline leg import this
package.  The product library never loads it and shares no code with it.
Arrays are float64 numpy arrays in the [j][k][i] layout (longitude fastest):
U (ny+1, nz, nx), V (ny, nz, nx), Phi (ny+1, nz, nx), ps (ny+1, nx).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dycore_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile the oracle with g++ -O3 (no fast-math), OpenMP over latitude rows."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        L.orc_substeps.restype = ctypes.c_int
        L.orc_substeps.argtypes = [ctypes.c_void_p, ctypes.c_double]
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


class Oracle:
    """One grid: nx longitudes, ny latitude intervals (ny+1 scalar rows incl. poles), nz levels."""

    def __init__(self, nx, ny, nz, phis=None, sigma_half=None, consts=None, filters=False, kstar=0.0):
        self.nx, self.ny, self.nz = nx, ny, nz
        L = _load()
        self._phis = None if phis is None else np.ascontiguousarray(phis, dtype=np.float64)
        sh = None if sigma_half is None else np.ascontiguousarray(sigma_half, dtype=np.float64)
        cs = None if consts is None else np.ascontiguousarray(consts, dtype=np.float64)
        self.h = L.orc_create(nx, ny, nz, _p(sh), _p(self._phis), _p(cs))
        if not self.h:
            raise ValueError("bad grid")
        self.L = L
        L.orc_set_filters(ctypes.c_void_p(self.h), 1 if filters else 0)
        L.orc_set_kstar(ctypes.c_void_p(self.h), ctypes.c_double(kstar))

    def __del__(self):
        if getattr(self, "h", None):
            self.L.orc_destroy(ctypes.c_void_p(self.h))
            self.h = None

    # shapes
    def shapes(self):
        nx, ny, nz = self.nx, self.ny, self.nz
        return {"U": (ny + 1, nz, nx), "V": (ny, nz, nx), "Phi": (ny + 1, nz, nx), "ps": (ny + 1, nx)}

    def zeros(self):
        return {k: np.zeros(s) for k, s in self.shapes().items()}

    def _vh(self):
        return ctypes.c_void_p(self.h)

    @staticmethod
    def _c(st):
        return {k: np.ascontiguousarray(st[k], dtype=np.float64) for k in ("U", "V", "Phi", "ps")}

    def constants(self):
        out = np.zeros(10)
        self.L.orc_constants(self._vh(), _p(out))
        keys = ["a", "omega", "g", "rd", "cp", "p0", "t0", "kappa", "b", "acap"]
        return dict(zip(keys, out.tolist()))

    def leap_table(self):
        m = np.zeros(self.ny + 1, dtype=np.int32)
        mv = np.zeros(self.ny, dtype=np.int32)
        r = np.zeros(self.ny + 1)
        rv = np.zeros(self.ny)
        self.L.orc_leap_table(self._vh(), m.ctypes.data_as(_ip), mv.ctypes.data_as(_ip), _p(r), _p(rv))
        return m, mv, r, rv

    def zonal_spacing(self):
        d = np.zeros(self.ny + 1)
        dv = np.zeros(self.ny)
        self.L.orc_zonal_spacing(self._vh(), _p(d), _p(dv))
        return d, dv

    def tendency(self, st, which):
        """which: 'A' adaptation or 'L' advection (returns -L)."""
        s = self._c(st)
        t = self.zeros()
        self.L.orc_tendency(self._vh(), 0 if which == "A" else 1, _p(s["U"]), _p(s["V"]), _p(s["Phi"]),
                            _p(s["ps"]), _p(t["U"]), _p(t["V"]), _p(t["Phi"]), _p(t["ps"]))
        return t

    def column_diag(self, st):
        s = self._c(st)
        nx, ny, nz = self.nx, self.ny, self.nz
        D = np.zeros((ny + 1, nz, nx)); phi = np.zeros_like(D); wp = np.zeros_like(D)
        sd = np.zeros((ny + 1, nz + 1, nx)); Pi = np.zeros((ny + 1, nx)); vgl = np.zeros_like(D)
        self.L.orc_column_diag(self._vh(), _p(s["U"]), _p(s["V"]), _p(s["Phi"]), _p(s["ps"]),
                               _p(D), _p(phi), _p(wp), _p(sd), _p(Pi), _p(vgl))
        return {"D": D, "phi": phi, "wp": wp, "sd": sd, "Pi": Pi, "vgl": vgl}

    def stage(self, base, yin, ch, which):
        b = self._c(base)
        s = self._c(yin)
        o = self.zeros()
        self.L.orc_stage(self._vh(), 0 if which == "A" else 1, ctypes.c_double(ch),
                         _p(b["U"]), _p(b["V"]), _p(b["Phi"]), _p(b["ps"]),
                         _p(s["U"]), _p(s["V"]), _p(s["Phi"]), _p(s["ps"]),
                         _p(o["U"]), _p(o["V"]), _p(o["Phi"]), _p(o["ps"]))
        return o

    def filter(self, st):
        """The low-latitude filters (Sec. III-B, Table IV rows 1-2) applied once to a copy of st."""
        s = {k: np.array(v, dtype=np.float64, copy=True, order="C") for k, v in self._c(st).items()}
        self.L.orc_filter(self._vh(), _p(s["U"]), _p(s["V"]), _p(s["Phi"]), _p(s["ps"]))
        return s

    def substeps(self, dt):
        return int(self.L.orc_substeps(self._vh(), ctypes.c_double(dt)))

    def step(self, st, nsteps, dt, msub=None):
        if msub is None:
            msub = self.substeps(dt)
        s = {k: np.array(v, dtype=np.float64, copy=True, order="C") for k, v in self._c(st).items()}
        self.L.orc_step(self._vh(), _p(s["U"]), _p(s["V"]), _p(s["Phi"]), _p(s["ps"]),
                        ctypes.c_int(nsteps), ctypes.c_double(dt), ctypes.c_int(msub))
        return s

    def tl_step(self, st, d, dt, msub=None, nsteps=1):
        if msub is None:
            msub = self.substeps(dt)
        s = self._c(st); dd = self._c(d); o = self.zeros()
        self.L.orc_tl_step_cs(self._vh(), _p(s["U"]), _p(s["V"]), _p(s["Phi"]), _p(s["ps"]),
                              _p(dd["U"]), _p(dd["V"]), _p(dd["Phi"]), _p(dd["ps"]),
                              _p(o["U"]), _p(o["V"]), _p(o["Phi"]), _p(o["ps"]),
                              ctypes.c_int(nsteps), ctypes.c_double(dt), ctypes.c_int(msub))
        return o

    def tl_tendency(self, st, d, which):
        s = self._c(st); dd = self._c(d); o = self.zeros()
        self.L.orc_tl_tendency_cs(self._vh(), 0 if which == "A" else 1,
                                  _p(s["U"]), _p(s["V"]), _p(s["Phi"]), _p(s["ps"]),
                                  _p(dd["U"]), _p(dd["V"]), _p(dd["Phi"]), _p(dd["ps"]),
                                  _p(o["U"]), _p(o["V"]), _p(o["Phi"]), _p(o["ps"]))
        return o

    def adj_tendency(self, st, a, which):
        s = self._c(st); aa = self._c(a); o = self.zeros()
        self.L.orc_adj_tendency(self._vh(), 0 if which == "A" else 1,
                                _p(s["U"]), _p(s["V"]), _p(s["Phi"]), _p(s["ps"]),
                                _p(aa["U"]), _p(aa["V"]), _p(aa["Phi"]), _p(aa["ps"]),
                                _p(o["U"]), _p(o["V"]), _p(o["Phi"]), _p(o["ps"]))
        return o

    def adj_stage(self, yin, a_out, ch, which):
        """Adjoint of out = base + ch T(yin): returns (adjoint of base, adjoint of yin)."""
        s = self._c(yin); a = self._c(a_out); b = self.zeros(); i = self.zeros()
        self.L.orc_adj_stage(self._vh(), 0 if which == "A" else 1, ctypes.c_double(ch),
                             _p(s["U"]), _p(s["V"]), _p(s["Phi"]), _p(s["ps"]),
                             _p(a["U"]), _p(a["V"]), _p(a["Phi"]), _p(a["ps"]),
                             _p(b["U"]), _p(b["V"]), _p(b["Phi"]), _p(b["ps"]),
                             _p(i["U"]), _p(i["V"]), _p(i["Phi"]), _p(i["ps"]))
        return b, i

    def adj_step(self, st0, a_out, dt, msub=None):
        if msub is None:
            msub = self.substeps(dt)
        s = self._c(st0)
        a = {k: np.array(v, dtype=np.float64, copy=True, order="C") for k, v in self._c(a_out).items()}
        self.L.orc_adj_step(self._vh(), _p(s["U"]), _p(s["V"]), _p(s["Phi"]), _p(s["ps"]),
                            _p(a["U"]), _p(a["V"]), _p(a["Phi"]), _p(a["ps"]),
                            ctypes.c_double(dt), ctypes.c_int(msub))
        return a

    def diagnostics(self, st):
        s = self._c(st)
        m = ctypes.c_double(); e = ctypes.c_double()
        self.L.orc_diagnostics(self._vh(), _p(s["U"]), _p(s["V"]), _p(s["Phi"]), _p(s["ps"]),
                               ctypes.byref(m), ctypes.byref(e))
        return m.value, e.value


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Thread count of the forward map's OpenMP loops (timing only; results do not depend on it)."""
    _load().orc_set_num_threads(int(n))


def dot(a: dict, b: dict) -> float:
    """Plain Euclidean inner product over every stored entry of the four fields."""
    return float(sum(np.vdot(a[k], b[k]) for k in ("U", "V", "Phi", "ps")))
