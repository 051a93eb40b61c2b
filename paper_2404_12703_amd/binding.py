"""ctypes binding of libdgsem.so (include/dgsem.h): argument marshalling only.

PyTorch supplies device memory (the workspace is a uint8 CUDA tensor) and the
stream; every step of the time derivative runs in the library's HIP kernels.
The binding refuses to run without the built library or without a GPU: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdgsem.so")

DG_OK, DG_EINVAL, DG_EMESH, DG_ENOMEM, DG_EDEVICE, DG_ENONFINITE, DG_EBUSY, DG_ESTATE = 0, -1, -2, -3, -4, -5, -6, -7
_NAMES = {-1: "DG_EINVAL", -2: "DG_EMESH", -3: "DG_ENOMEM", -4: "DG_EDEVICE", -5: "DG_ENONFINITE",
          -6: "DG_EBUSY", -7: "DG_ESTATE"}
REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = 0, 1, 2, 3
ABI_VERSION = 2


class DGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class dg_params(C.Structure):
    _fields_ = [("abi_version", C.c_int32), ("N", C.c_int32), ("nodes", C.c_int32), ("riemann", C.c_int32),
                ("precision", C.c_int32), ("viscous", C.c_int32), ("source", C.c_int32),
                ("shock_capturing", C.c_int32), ("check_finite", C.c_int32), ("reserved", C.c_int32),
                ("gamma", C.c_double), ("R", C.c_double), ("Pr", C.c_double), ("mu", C.c_double),
                ("alpha_max", C.c_double), ("alpha_min", C.c_double), ("ind_a", C.c_double),
                ("ind_c", C.c_double), ("ind_s", C.c_double),
                ("volume_flux", C.c_int32), ("viscosity_law", C.c_int32), ("time_scheme", C.c_int32),
                ("alpha_smooth", C.c_int32), ("T_ref", C.c_double), ("p_ref", C.c_double)]


class dg_mesh(C.Structure):
    _fields_ = [("n_elems", C.c_int64), ("n_geo", C.c_int32), ("reserved", C.c_int32),
                ("x_geo", C.c_void_p), ("nbr_elem", C.c_void_p), ("nbr_face", C.c_void_p),
                ("nbr_orient", C.c_void_p)]


class dg_timing(C.Structure):
    _fields_ = [("t_arrival", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
                ("state", C.c_int32), ("reserved", C.c_int32)]


_lib = None


def lib():
    """load libdgsem.so; raises if it has not been built"""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "or python paper_2404_12703_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        P, M = C.POINTER(dg_params), C.POINTER(dg_mesh)
        sig = {
            "dg_abi_version": (i32, []),
            "dg_last_error": (C.c_char_p, []),
            "dg_workspace_bytes": (i32, [P, i64, C.POINTER(C.c_size_t)]),
            "dg_create": (i32, [P, M, vp, C.c_size_t, vp, C.POINTER(vp)]),
            "dg_set_state": (i32, [vp, vp, i32, f64]),
            "dg_get_state": (i32, [vp, vp, i32, C.POINTER(f64)]),
            "dg_stable_dt": (i32, [vp, f64, f64, C.POINTER(f64)]),
            "dg_advance": (i32, [vp, i32, f64]),
            "dg_rhs": (i32, [vp, f64, vp, i32]),
            "dg_alpha": (i32, [vp, vp]),
            "dg_set_alpha": (i32, [vp, vp]),
            "dg_integrals": (i32, [vp, vp]),
            "dg_synchronize": (i32, [vp]),
            "dg_dissipation": (i32, [vp, vp]),
            "dg_dissipation_noalloc": (i32, [vp, vp]),
            "dg_destroy": (None, [vp]),
            "dg_profile_enable": (i32, [vp, i32]),
            "dg_profile_read": (i32, [vp, i32, vp, vp]),
            "dg_server_create": (i32, [vp, C.c_size_t, C.c_size_t, i32, vp, vp, C.POINTER(vp)]),
            "dg_server_submit": (i32, [vp, P, M, vp, i32, f64, f64, C.POINTER(i64)]),
            "dg_server_run": (i32, [vp, i32]),
            "dg_server_poll": (i32, [vp, i64, C.POINTER(i32)]),
            "dg_server_fetch": (i32, [vp, i64, vp, C.POINTER(dg_timing)]),
            "dg_server_stats": (i32, [vp, vp]),
            "dg_server_destroy": (None, [vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != DG_OK:
        raise DGError(rc, lib().dg_last_error().decode())


def make_params(p: dict) -> dg_params:
    return dg_params(abi_version=ABI_VERSION, N=int(p["N"]), nodes=int(p.get("nodes", 0)),
                     riemann=int(p.get("riemann", 0)), precision=int(p.get("precision", 0)),
                     viscous=int(p.get("viscous", 1)), source=int(p.get("source", 0)),
                     shock_capturing=int(p.get("shock_capturing", 0)),
                     check_finite=int(p.get("check_finite", 0)), reserved=0,
                     gamma=float(p.get("gamma", 1.4)), R=float(p.get("R", 1.0)), Pr=float(p.get("Pr", 0.72)),
                     mu=float(p.get("mu", 0.0)), alpha_max=float(p.get("alpha_max", 1.0)),
                     alpha_min=float(p.get("alpha_min", 0.001)), ind_a=float(p.get("ind_a", 0.5)),
                     ind_c=float(p.get("ind_c", 1.8)), ind_s=float(p.get("ind_s", np.log(9999.0))),
                     volume_flux=int(p.get("volume_flux", 0)), viscosity_law=int(p.get("viscosity", 0)),
                     time_scheme=int(p.get("time_scheme", 0)), alpha_smooth=int(p.get("alpha_smooth", 0)),
                     T_ref=float(p.get("T_ref", 1.0)), p_ref=float(p.get("p_ref", 0.0)))


class _MeshArrays:
    """host copies kept alive while the C call reads them"""

    def __init__(self, mesh):
        self.x = np.ascontiguousarray(mesh.x_geo, dtype=np.float64)
        self.ne = np.ascontiguousarray(mesh.nbr_elem, dtype=np.int64)
        self.nf = np.ascontiguousarray(mesh.nbr_face, dtype=np.int8)
        self.no = np.ascontiguousarray(mesh.nbr_orient, dtype=np.int8)
        self.c = dg_mesh(n_elems=self.x.shape[0], n_geo=int(mesh.ngeo), reserved=0,
                         x_geo=self.x.ctypes.data, nbr_elem=self.ne.ctypes.data,
                         nbr_face=self.nf.ctypes.data, nbr_orient=self.no.ctypes.data)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the DGSEM library needs a GPU; none is visible")
    return torch


def workspace_bytes(params: dict, n_elems: int) -> int:
    p = make_params(params)
    out = C.c_size_t(0)
    _check(lib().dg_workspace_bytes(C.byref(p), int(n_elems), C.byref(out)))
    return out.value


class Solver:
    """One solve on the current GPU.  State arrays are (5, E, (N+1)^3) float64."""

    def __init__(self, params: dict, mesh, stream=None):
        torch = _torch()
        self.params = dict(params)
        self.N = int(params["N"])
        self.E = int(mesh.n_elems)
        self.shape = (5, self.E, (self.N + 1) ** 3)
        self._p = make_params(params)
        nbytes = workspace_bytes(params, self.E)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        m = _MeshArrays(mesh)
        h = C.c_void_p()
        _check(lib().dg_create(C.byref(self._p), C.byref(m.c), C.c_void_p(self._ws_ptr), nbytes,
                               C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().dg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, U, t: float = 0.0):
        torch = _torch()
        if isinstance(U, torch.Tensor) and U.is_cuda:
            assert U.dtype == torch.float64 and U.is_contiguous() and tuple(U.shape) == self.shape
            _check(lib().dg_set_state(self._h, C.c_void_p(U.data_ptr()), 1, float(t)))
        else:
            a = np.ascontiguousarray(U, dtype=np.float64)
            assert a.shape == self.shape, a.shape
            _check(lib().dg_set_state(self._h, C.c_void_p(a.ctypes.data), 0, float(t)))

    def state(self):
        out = np.empty(self.shape)
        t = C.c_double(0)
        _check(lib().dg_get_state(self._h, C.c_void_p(out.ctypes.data), 0, C.byref(t)))
        return out

    def state_into(self, U_dev):
        t = C.c_double(0)
        _check(lib().dg_get_state(self._h, C.c_void_p(U_dev.data_ptr()), 1, C.byref(t)))
        return t.value

    def time(self) -> float:
        t = C.c_double(0)
        tmp = np.empty(self.shape)
        _check(lib().dg_get_state(self._h, C.c_void_p(tmp.ctypes.data), 0, C.byref(t)))
        return t.value

    def advance(self, n_steps: int, dt: float):
        _check(lib().dg_advance(self._h, int(n_steps), float(dt)))

    def rhs(self, t: float = 0.0):
        out = np.empty(self.shape)
        _check(lib().dg_rhs(self._h, float(t), C.c_void_p(out.ctypes.data), 0))
        return out

    def rhs_into(self, out_dev, t: float = 0.0):
        _check(lib().dg_rhs(self._h, float(t), C.c_void_p(out_dev.data_ptr()), 1))

    def stable_dt(self, cfl: float = 0.9, dfl: float = 0.9) -> float:
        out = C.c_double(0)
        _check(lib().dg_stable_dt(self._h, float(cfl), float(dfl), C.byref(out)))
        return out.value

    def alpha(self):
        out = np.empty(self.E)
        _check(lib().dg_alpha(self._h, C.c_void_p(out.ctypes.data)))
        return out

    def set_alpha(self, alpha):
        if alpha is None:
            _check(lib().dg_set_alpha(self._h, None))
        else:
            a = np.ascontiguousarray(alpha, dtype=np.float64)
            _check(lib().dg_set_alpha(self._h, C.c_void_p(a.ctypes.data)))

    def integrals(self):
        out = np.empty(7)
        _check(lib().dg_integrals(self._h, C.c_void_p(out.ctypes.data)))
        return out

    def synchronize(self):
        _check(lib().dg_synchronize(self._h))

    def dissipation(self):
        """(eps_S, eps_D) of the current state"""
        out = np.zeros(2)
        _check(lib().dg_dissipation(self._h, C.c_void_p(out.ctypes.data)))
        return out

    def dissipation_noalloc(self):
        """(eps_S, eps_D) through the entry point that allocates nothing"""
        out = np.zeros(2)
        _check(lib().dg_dissipation_noalloc(self._h, C.c_void_p(out.ctypes.data)))
        return out

    def profile(self, on: bool):
        _check(lib().dg_profile_enable(self._h, 1 if on else 0))

    def profile_read(self):
        ms = np.zeros(3)
        cnt = np.zeros(3, dtype=np.int64)
        _check(lib().dg_profile_read(self._h, 3, C.c_void_p(ms.ctypes.data), C.c_void_p(cnt.ctypes.data)))
        return dict(zip(("trace", "lift", "rhs"), zip(ms.tolist(), cnt.tolist())))


class Server:
    """Continuous-batching server over a caller-owned arena (include/dgsem.h)."""

    def __init__(self, arena_bytes: int, hbm_budget: int, max_active: int = 64, stream=None, copy_stream=None):
        torch = _torch()
        self.arena = torch.empty(arena_bytes + 256, dtype=torch.uint8, device="cuda")
        self._ptr = (self.arena.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.copy_stream = copy_stream if copy_stream is not None else self.stream
        h = C.c_void_p()
        _check(lib().dg_server_create(C.c_void_p(self._ptr), int(arena_bytes), int(hbm_budget), int(max_active),
                                      C.c_void_p(self.stream.cuda_stream),
                                      C.c_void_p(self.copy_stream.cuda_stream), C.byref(h)))
        self._h = h
        self._shapes = {}

    def close(self):
        if getattr(self, "_h", None):
            lib().dg_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, params: dict, mesh, U0, n_steps: int, dt: float, t_arrival: float = 0.0) -> int:
        p = make_params(params)
        m = _MeshArrays(mesh)
        a = np.ascontiguousarray(U0, dtype=np.float64)
        rid = C.c_int64(0)
        _check(lib().dg_server_submit(self._h, C.byref(p), C.byref(m.c), C.c_void_p(a.ctypes.data), int(n_steps),
                                      float(dt), float(t_arrival), C.byref(rid)))
        self._shapes[rid.value] = a.shape
        return rid.value

    def run(self, max_ticks: int = 0):
        _check(lib().dg_server_run(self._h, int(max_ticks)))

    def poll(self, rid: int) -> int:
        st = C.c_int32(0)
        _check(lib().dg_server_poll(self._h, int(rid), C.byref(st)))
        return st.value

    def stats(self):
        out = np.zeros(10)
        _check(lib().dg_server_stats(self._h, C.c_void_p(out.ctypes.data)))
        keys = ("ticks", "mean_active", "host_admit_s", "host_tick_s", "host_retire_s", "gpu_wait_s", "idle_s",
                "upload_bytes", "geometry_uploads", "geometry_hits")
        return dict(zip(keys, out.tolist()))

    def fetch(self, rid: int):
        out = np.empty(self._shapes[rid])
        tm = dg_timing()
        _check(lib().dg_server_fetch(self._h, int(rid), C.c_void_p(out.ctypes.data), C.byref(tm)))
        return out, dict(t_arrival=tm.t_arrival, t_admit=tm.t_admit, t_done=tm.t_done, state=tm.state)
