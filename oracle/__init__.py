"""ctypes wrapper of the FP64 CPU oracle (dgsem_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg; never by the library or its binding.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dgsem_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """compile the oracle (gcc, -O2, no FMA contraction, no fast-math, OpenMP)"""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off",
                               "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp,
                               "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_long, _dp,
                                 np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS"),
                                 np.ctypeslib.ndpointer(dtype=np.int8, flags="C_CONTIGUOUS"),
                                 _dp, C.c_char_p, C.c_int]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_params.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double,
                                     C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                     C.c_double, C.c_double, C.c_double]
        L.orc_rhs.argtypes = [C.c_void_p, _dp, C.c_double, _dp]
        L.orc_advance.argtypes = [C.c_void_p, _dp, C.c_double, C.c_double, C.c_int]
        L.orc_get_alpha.argtypes = [C.c_void_p, _dp]
        L.orc_set_alpha.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_integrals.argtypes = [C.c_void_p, _dp, _dp]
        L.orc_stable_dt.restype = C.c_double
        L.orc_stable_dt.argtypes = [C.c_void_p, _dp, C.c_double, C.c_double]
        L.orc_rk_coefficients.argtypes = [_dp, _dp, _dp]
        L.orc_basis.argtypes = [C.c_void_p] + [_dp] * 8
        L.orc_geometry.argtypes = [C.c_void_p] + [C.c_void_p] * 5
        L.orc_metric_identity.argtypes = [C.c_void_p, _dp]
        L.orc_riemann.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp, _dp]
        L.orc_fv_volume.argtypes = [C.c_void_p, _dp, C.c_long, _dp]
        L.orc_indicator.restype = C.c_double
        L.orc_indicator.argtypes = [C.c_void_p, _dp, C.c_long]
        L.orc_set_params2.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int]
        L.orc_rk_scheme.restype = C.c_int
        L.orc_rk_scheme.argtypes = [C.c_int, _dp, _dp, _dp]
        L.orc_dissipation.restype = C.c_int
        L.orc_dissipation.argtypes = [C.c_void_p, _dp, _dp]
        L.orc_two_point.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp, _dp]
        L.orc_viscosity.restype = C.c_double
        L.orc_viscosity.argtypes = [C.c_void_p, C.c_double]
        _lib = L
    return _lib


def rk_coefficients(scheme: int = 0):
    """(A, B, c) of the low-storage scheme: 0 five stages, 1 fourteen"""
    A, B, Cc = np.zeros(14), np.zeros(14), np.zeros(14)
    ns = lib().orc_rk_scheme(int(scheme), A, B, Cc)
    return A[:ns].copy(), B[:ns].copy(), Cc[:ns].copy()


class Oracle:
    """One mesh + parameter set.  State arrays are (5, E, (N+1)^3) float64."""

    def __init__(self, params: dict, mesh):
        L = lib()
        self.N = int(params["N"])
        self.n = self.N + 1
        self.E = mesh.n_elems
        err = C.create_string_buffer(256)
        self.h = L.orc_create(self.N, int(params.get("nodes", 0)), int(mesh.ngeo), self.E,
                              np.ascontiguousarray(mesh.x_geo, dtype=np.float64),
                              np.ascontiguousarray(mesh.nbr_elem, dtype=np.int64),
                              np.ascontiguousarray(mesh.nbr_face, dtype=np.int8),
                              np.ascontiguousarray(mesh.period, dtype=np.float64), err, 256)
        if not self.h:
            raise ValueError("oracle: " + err.value.decode())
        self.params = dict(params)
        self.set_params(params)

    def set_params(self, p):
        lib().orc_set_params(self.h, p["gamma"], p["R"], p["Pr"], p["mu"], int(p["riemann"]),
                             int(p["viscous"]), int(p["source"]), int(p.get("shock_capturing", 0)),
                             p.get("alpha_max", 1.0), p.get("alpha_min", 0.001), p.get("ind_a", 0.5),
                             p.get("ind_c", 1.8), p.get("ind_s", np.log(9999.0)))
        lib().orc_set_params2(self.h, int(p.get("alpha_smooth", 0)), int(p.get("volume_flux", 0)),
                              int(p.get("viscosity", 0)), float(p.get("T_ref", 1.0)),
                              int(p.get("time_scheme", 0)))

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    def _state(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        assert U.shape == (5, self.E, self.n ** 3), U.shape
        return U

    def rhs(self, U, t=0.0):
        U = self._state(U)
        out = np.empty_like(U)
        lib().orc_rhs(self.h, U, float(t), out)
        return out

    def advance(self, U, dt, nsteps, t0=0.0):
        U = self._state(U).copy()
        lib().orc_advance(self.h, U, float(t0), float(dt), int(nsteps))
        return U

    def alpha(self):
        a = np.empty(self.E)
        lib().orc_get_alpha(self.h, a)
        return a

    def set_alpha(self, alpha):
        if alpha is None:
            lib().orc_set_alpha(self.h, None)
        else:
            a = np.ascontiguousarray(alpha, dtype=np.float64)
            lib().orc_set_alpha(self.h, a.ctypes.data)
            self._frozen = a  # keep alive

    def integrals(self, U):
        out = np.empty(7)
        lib().orc_integrals(self.h, self._state(U), out)
        return out

    def stable_dt(self, U, cfl=0.9, dfl=0.9):
        return lib().orc_stable_dt(self.h, self._state(U), cfl, dfl)

    def basis(self):
        n = self.n
        arrs = [np.zeros(n), np.zeros(n), np.zeros((n, n)), np.zeros((n, n)), np.zeros(n),
                np.zeros(n), np.zeros(n), np.zeros(n)]
        lib().orc_basis(self.h, *arrs)
        return dict(zip(["x", "w", "D", "Dhat", "lhm", "lhp", "lm", "lp"], arrs))

    def geometry(self):
        n, E = self.n, self.E
        Ja = np.zeros((E, n ** 3, 3, 3))
        J = np.zeros((E, n ** 3))
        nS = np.zeros((E, 6, n * n, 3))
        Xs = np.zeros((E, n ** 3, 3))
        fmap = np.zeros((E, 6, n * n), dtype=np.int32)
        lib().orc_geometry(self.h, Ja.ctypes.data, J.ctypes.data, nS.ctypes.data, Xs.ctypes.data,
                           fmap.ctypes.data)
        return dict(Ja=Ja, J=J, nS=nS, Xs=Xs, fmap=fmap)

    def metric_identity(self):
        out = np.zeros((self.E, self.n ** 3, 3))
        lib().orc_metric_identity(self.h, out)
        return out

    def riemann(self, which, UL, UR, nv):
        F = np.zeros(5)
        lib().orc_riemann(self.h, int(which), np.ascontiguousarray(UL, dtype=np.float64),
                          np.ascontiguousarray(UR, dtype=np.float64),
                          np.ascontiguousarray(nv, dtype=np.float64), F)
        return F

    def fv_volume(self, U, e):
        out = np.zeros((self.n ** 3, 5))
        lib().orc_fv_volume(self.h, self._state(U), int(e), out)
        return out

    def indicator(self, U, e):
        return lib().orc_indicator(self.h, self._state(U), int(e))

    def dissipation(self, U):
        """(eps_S, eps_D) of Sec. 5.2 from the lifted gradients of U"""
        out = np.zeros(2)
        if lib().orc_dissipation(self.h, self._state(U), out) != 0:
            raise ValueError("dissipation rates need the viscous operator")
        return out

    def two_point(self, which, UL, UR, m):
        F = np.zeros(5)
        lib().orc_two_point(self.h, int(which), np.ascontiguousarray(UL, dtype=np.float64),
                            np.ascontiguousarray(UR, dtype=np.float64),
                            np.ascontiguousarray(m, dtype=np.float64), F)
        return F

    def viscosity(self, T):
        return lib().orc_viscosity(self.h, float(T))
