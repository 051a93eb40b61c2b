"""The C ABI on the CPU: the library loads, exports every entry point the
header declares, sizes workspaces and rejects bad parameters and meshes
before any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dgsem.h")


def _lib():
    from paper_2404_12703_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libdgsem.so not built")
    return binding


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    b = _lib()
    raw = C.CDLL(b.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 20
    for nm in names:
        assert hasattr(raw, nm), nm
    assert b.lib().dg_abi_version() == 2


def test_workspace_bytes_and_parameter_checks():
    b = _lib()
    p = W.params(7)
    nb = b.workspace_bytes(p, 13824)
    n3, n2, E = 512, 64, 13824
    # state + RK register + metrics + normals + two U traces, then (viscous,
    # no shock capturing) one side's viscous face flux (4 values per face
    # node) and the volume integral (5 per node), all FP64
    core = 8 * E * (5 * n3 + 5 * n3 + 9 * n3 + n3 + 3 * 6 * n2 + 2 * 5 * 6 * n2 + 4 * 6 * n2 + 5 * n3)
    assert core <= nb <= core * 1.01
    pm = dict(p)
    pm["precision"] = 1
    assert b.workspace_bytes(pm, E) < nb
    # shock capturing exchanges the same quantities between the two sweeps
    ps = W.params(7, node_type=1, shock=1)
    assert abs(b.workspace_bytes(ps, E) - nb) <= 0.01 * nb
    # Euler: no viscous face flux; with shock capturing the volume integral is kept
    pe = W.params(7, viscous=0)
    ce = 8 * E * (5 * n3 + 5 * n3 + 9 * n3 + n3 + 3 * 6 * n2 + 2 * 5 * 6 * n2)
    assert ce <= b.workspace_bytes(pe, E) <= ce * 1.01
    pes = W.params(7, node_type=1, viscous=0, shock=1)
    assert ce + 8 * E * 5 * n3 <= b.workspace_bytes(pes, E) <= (ce + 8 * E * 5 * n3) * 1.01
    # every row of a volume array must stay below 2^31 entries (32-bit lane offsets)
    assert b.workspace_bytes(p, (2**31 - 1) // n3) > 0
    with pytest.raises(b.DGError) as ei:
        b.workspace_bytes(p, (2**31 - 1) // n3 + 1)
    assert ei.value.code == b.DG_EINVAL
    inf, nan = float("inf"), float("nan")
    lob = dict(nodes=1, shock_capturing=1)
    for bad in (dict(N=0), dict(N=12), dict(gamma=1.0), dict(Pr=0.0), dict(mu=-1.0), dict(riemann=3),
                dict(nodes=0, shock_capturing=1), dict(gamma=inf), dict(R=nan), dict(Pr=inf), dict(mu=inf),
                dict(lob, ind_s=0.0), dict(lob, ind_s=nan), dict(lob, ind_c=inf), dict(lob, ind_a=inf),
                dict(lob, alpha_min=0.5), dict(lob, alpha_max=1.5), dict(viscosity=1, T_ref=inf),
                dict(p_ref=nan)):
        q = dict(p)
        q.update(bad)
        with pytest.raises(b.DGError) as ei:
            b.workspace_bytes(q, 10)
        assert ei.value.code == b.DG_EINVAL


def _create_raw(b, params, mesh, ws_bytes):
    """dg_create with a placeholder device address: only valid for inputs the
    library rejects before touching the device"""
    p = b.make_params(params)
    m = b._MeshArrays(mesh)
    h = C.c_void_p()
    return b.lib().dg_create(C.byref(p), C.byref(m.c), C.c_void_p(1 << 20), ws_bytes, None, C.byref(h))


def test_mesh_rejections_before_device_work():
    b = _lib()
    p = W.params(3)
    big = 1 << 40
    # asymmetric neighbour table
    m = W.box_mesh(2, -1.0, 1.0, 3)
    m.nbr_elem = m.nbr_elem.copy()
    m.nbr_elem[0, 1] = 3
    assert _create_raw(b, p, m, big) == b.DG_EMESH
    assert "symmetric" in b.lib().dg_last_error().decode()
    # orientation codes that are not inverse of each other
    m = W.box_mesh(2, -1.0, 1.0, 3, rotate=True)
    m.nbr_orient = m.nbr_orient.copy()
    m.nbr_orient[1, 2] ^= 1
    assert _create_raw(b, p, m, big) == b.DG_EMESH
    # an inverted element (negative Jacobian)
    m = W.box_mesh(2, -1.0, 1.0, 3)
    m.x_geo = m.x_geo.copy()
    m.x_geo[0, 0] = -m.x_geo[0, 0]
    assert _create_raw(b, p, m, big) == b.DG_EMESH
    # workspace too small
    m = W.box_mesh(2, -1.0, 1.0, 3)
    assert _create_raw(b, p, m, 1024) == b.DG_ENOMEM


def test_geometric_faces_must_be_watertight():
    """a mesh whose faces do not coincide (one element displaced) is rejected"""
    b = _lib()
    m = W.box_mesh(2, -1.0, 1.0, 2)
    m.x_geo = m.x_geo.copy()
    m.x_geo[3, 1] += 0.1 * np.linspace(0.0, 1.0, m.x_geo.shape[2])
    assert _create_raw(b, W.params(2), m, 1 << 40) == b.DG_EMESH
