"""The host half of the library's set-up (parameter checks, workspace layout,
bases, curl-form metrics, face and connectivity checks, the time-step
estimate) built with AddressSanitizer and UndefinedBehaviorSanitizer for the
host and run on valid and broken inputs.  It makes no HIP call, so it runs on
any CPU; the time step of every valid case is compared with the oracle's."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_2404_12703_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2404_12703_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
DG_EINVAL, DG_EMESH = -1, -2


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("sanitize") / "host_setup")
    # host-only compilation: the sanitizers apply to the host code alone
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    cmd = ([HIPCC, "-x", "hip", "--offload-host-only", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer"] + san +
           ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
            os.path.join(ROOT, "tests", "sanitize", "host_setup_driver.cpp"),
            os.path.join(CSRC, "setup.cpp"), os.path.join(CSRC, "solver.cpp")] + san +
           # the device launches in solver.cpp are never reached
           ["-Wl,--unresolved-symbols=ignore-in-object-files", "-o", out])
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return out


def _write_case(f, p, m, U):
    f.write(struct.pack("<i", 1))
    f.write(bytes(B.make_params(p)))
    f.write(struct.pack("<qi", m.x_geo.shape[0], int(m.ngeo)))
    for a, dt in ((m.x_geo, np.float64), (m.nbr_elem, np.int64), (m.nbr_face, np.int8), (m.nbr_orient, np.int8)):
        f.write(np.ascontiguousarray(a, dtype=dt).tobytes())
    f.write(struct.pack("<q", U.size))
    f.write(np.ascontiguousarray(U, dtype=np.float64).tobytes())


def _run(driver, tmp_path, cases):
    path = tmp_path / "cases.bin"
    with open(path, "wb") as f:
        for p, m, U in cases:
            _write_case(f, p, m, U)
        f.write(struct.pack("<i", 0))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([driver, str(path)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    rows = []
    for line in r.stdout.splitlines():
        t = line.split()
        rows.append(dict(rc=int(t[3]), dt=float(t[5]), bytes=int(t[7]), err=" ".join(t[9:])))
    assert len(rows) == len(cases)
    return rows


def _state(m, N, nodes, seed):
    X = m.points(W.lgl_points(N) if nodes else W.gl_points(N))
    return W.random_smooth_state(X, seed, 1.4, m.period)


def _valid_cases():
    cases = []
    for N in range(1, 10):  # Gauss, Navier-Stokes, curved and relabelled (trilinear at N = 1)
        m = W.box_mesh((3, 2, 2), 0.0, 2 * np.pi, N, amp=0.05 if N > 1 else 0.0, rotate=True)
        cases.append((W.params(N, riemann=1, mu=1e-2), m, _state(m, N, 0, N)))
    for N in (2, 5, 7):  # Gauss-Lobatto with shock capturing, the split form, mixed precision
        m = W.box_mesh(2, 0.0, 2 * np.pi, N, amp=0.05, rotate=True)
        cases.append((W.params(N, node_type=1, shock=1, mu=1e-2), m, _state(m, N, 1, 10 + N)))
        cases.append((W.params(N, node_type=1, volume_flux=1, viscosity=1, mu=1e-2, T_ref=0.8), m,
                      _state(m, N, 1, 20 + N)))
        m = W.box_mesh(2, 0.0, 2 * np.pi, N, amp=0.05, rotate=True)
        cases.append((W.params(N, precision=1, mu=1e-2), m, _state(m, N, 0, 30 + N)))
    m = W.box_mesh(2, -1.0, 1.0, 2, amp=0.03, rotate=True)  # geometry of lower degree than the solution
    cases.append((W.params(6, riemann=1, mu=1e-2), m, _state(m, 6, 0, 41)))
    wl = W.mms_workload(K=3, N=3)  # manufactured solution: node positions for the source
    cases.append((wl.params, wl.mesh, wl.U0))
    m = W.box_mesh(1, 0.0, 2 * np.pi, 4, amp=0.05)  # one element, its own neighbour on every face
    cases.append((W.params(4, riemann=1, mu=1e-2), m, _state(m, 4, 0, 42)))
    return cases


def test_host_setup_of_valid_cases_is_clean_and_matches_the_oracle(driver, tmp_path):
    cases = _valid_cases()
    rows = _run(driver, tmp_path, cases)
    for (p, m, U), r in zip(cases, rows):
        assert r["rc"] == 0, r["err"]
        assert r["bytes"] > 0
        dto = O.Oracle(p, m).stable_dt(U, 0.9, 0.9)
        # the mixed form estimates from its FP32 metrics
        tol = 1e-6 if p["precision"] else 1e-12
        assert abs(r["dt"] - dto) <= tol * dto, (p["N"], r["dt"], dto)


def _broken(kind):
    m = W.box_mesh(2, -1.0, 1.0, 3, amp=0.03, rotate=kind == "orient")
    p = W.params(3, mu=1e-2)
    U = _state(m, 3, 0, 50)
    for name in ("x_geo", "nbr_elem", "nbr_face", "nbr_orient"):
        setattr(m, name, getattr(m, name).copy())
    if kind == "asymmetric":
        m.nbr_elem[0, 1] = 3
    elif kind == "orient":
        m.nbr_orient[1, 2] ^= 1
    elif kind == "inverted":
        m.x_geo[0, 0] = -m.x_geo[0, 0]
    elif kind == "leaky":
        m.x_geo[3, 1] += 0.1 * np.linspace(0.0, 1.0, m.x_geo.shape[2])
    elif kind == "elem_range":
        m.nbr_elem[5, 4] = m.x_geo.shape[0]
    elif kind == "elem_negative":
        m.nbr_elem[2, 0] = -1
    elif kind == "face_range":
        m.nbr_face[1, 3] = 6
    elif kind == "orient_range":
        m.nbr_orient[4, 5] = 8
    elif kind == "nan_geometry":
        m.x_geo[6, 2, 3] = np.nan
    elif kind == "bad_params":
        p = dict(p, N=12)
    elif kind == "geo_degree":  # geometry of degree 4 under a solution of degree 3
        m = W.box_mesh(2, -1.0, 1.0, 4, amp=0.03)
    return p, m, U


BROKEN = {"asymmetric": DG_EMESH, "orient": DG_EMESH, "inverted": DG_EMESH, "leaky": DG_EMESH,
          "elem_range": DG_EMESH, "elem_negative": DG_EMESH, "face_range": DG_EMESH, "orient_range": DG_EMESH,
          "nan_geometry": DG_EMESH, "bad_params": DG_EINVAL, "geo_degree": DG_EINVAL}


def test_host_setup_rejects_broken_inputs_without_memory_errors(driver, tmp_path):
    kinds = list(BROKEN)
    rows = _run(driver, tmp_path, [_broken(k) for k in kinds])
    for k, r in zip(kinds, rows):
        assert r["rc"] == BROKEN[k], (k, r)
        assert r["err"], k
