"""Pins of the oracle's Riemann solvers (FillFlux, App. A) and of the two
low-storage Runge-Kutta schemes (Sec. 2.2 Time integration): Carpenter and
Kennedy's five stages and Niegemann, Diehl and Busch's fourteen."""
import json
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))
GAMMA = 1.4


def _o():
    return O.Oracle(W.params(1, viscous=0), W.box_mesh(2, -1.0, 1.0, 1))


def _cons(rho, u, p):
    u = np.asarray(u, dtype=float)
    return np.array([rho, *(rho * u), p / (GAMMA - 1) + 0.5 * rho * u @ u])


def _flux_n(U, n):
    """Euler flux along unit normal n, written independently of the oracle"""
    rho = U[0]
    u = U[1:4] / rho
    p = (GAMMA - 1) * (U[4] - 0.5 * rho * u @ u)
    un = u @ n
    return np.array([rho * un, *(rho * u * un + p * n), (U[4] + p) * un])


STATES = [
    (_cons(1.0, [0.3, -0.1, 0.2], 1.0), _cons(0.8, [0.1, 0.2, -0.1], 0.7)),
    (_cons(2.0, [-0.5, 0.4, 0.0], 3.0), _cons(1.1, [0.2, -0.3, 0.6], 1.4)),
]
NORMALS = [np.array([1.0, 0.0, 0.0]), np.array([0.48, -0.6, 0.64])]


@pytest.mark.parametrize("which", [0, 1])
def test_consistency_and_antisymmetry(which):
    o = _o()
    for UL, UR in STATES:
        for n in NORMALS:
            F = o.riemann(which, UL, UL, n)
            assert np.allclose(F, _flux_n(UL, n), atol=1e-14, rtol=1e-14)
            a = o.riemann(which, UL, UR, n)
            b = o.riemann(which, UR, UL, -n)
            assert np.allclose(a, -b, atol=1e-14, rtol=1e-13)


def test_llf_hand_values():
    """brute force: 1/2 (F_L + F_R) - 1/2 max(|u.n| + c) (U_R - U_L)"""
    o = _o()
    for UL, UR in STATES:
        for n in NORMALS:
            lam = 0.0
            for U in (UL, UR):
                u = U[1:4] / U[0]
                p = (GAMMA - 1) * (U[4] - 0.5 * U[0] * u @ u)
                lam = max(lam, abs(u @ n) + np.sqrt(GAMMA * p / U[0]))
            ref = 0.5 * (_flux_n(UL, n) + _flux_n(UR, n)) - 0.5 * lam * (UR - UL)
            assert np.allclose(o.riemann(0, UL, UR, n), ref, atol=1e-14, rtol=1e-13)


def _roe_bruteforce(UL, UR, n):
    """Roe flux from the numerical eigen-decomposition of the flux Jacobian at
    the Roe-average state (Jacobian by complex-step differentiation)."""
    def prim(U):
        rho = U[0]
        u = U[1:4] / rho
        p = (GAMMA - 1) * (U[4] - 0.5 * rho * u @ u)
        return rho, u, p, (U[4] + p) / rho
    rL, uL, pL, HL = prim(UL)
    rR, uR, pR, HR = prim(UR)
    sL, sR = np.sqrt(rL), np.sqrt(rR)
    u = (sL * uL + sR * uR) / (sL + sR)
    H = (sL * HL + sR * HR) / (sL + sR)
    rho = sL * sR
    p = (GAMMA - 1) / GAMMA * rho * (H - 0.5 * u @ u)
    Ut = _cons(rho, u, p)
    A = np.zeros((5, 5))
    for j in range(5):
        dU = np.zeros(5, dtype=complex)
        dU[j] = 1e-30j
        A[:, j] = np.imag(_flux_n(Ut + dU, n)) / 1e-30
    lam, Rm = np.linalg.eig(A)
    absA = (Rm @ np.diag(np.abs(lam)) @ np.linalg.inv(Rm)).real
    return 0.5 * (_flux_n(UL, n) + _flux_n(UR, n)) - 0.5 * absA @ (UR - UL)


def test_roe_matches_eigendecomposition_bruteforce():
    o = _o()
    for UL, UR in STATES:
        for n in NORMALS:
            assert np.allclose(o.riemann(1, UL, UR, n), _roe_bruteforce(UL, UR, n), atol=1e-12,
                               rtol=1e-11)


def test_roe_is_upwind_for_supersonic_flow():
    o = _o()
    n = NORMALS[1]
    UL = _cons(1.0, 3.0 * n, 1.0)
    UR = _cons(0.9, 2.8 * n + np.array([0.1, 0.1, 0.0]), 0.8)
    assert np.allclose(o.riemann(1, UL, UR, n), _flux_n(UL, n), atol=1e-12, rtol=1e-12)
    # flow towards the left state: all waves run left, the flux is the right state's
    VL = _cons(1.0, -3.0 * n, 1.0)
    VR = _cons(0.9, -2.8 * n + np.array([0.1, 0.1, 0.0]), 0.8)
    assert np.allclose(o.riemann(1, VL, VR, n), _flux_n(VR, n), atol=1e-12, rtol=1e-12)


def _butcher(scheme=0):
    A, B, C = O.rk_coefficients(scheme)
    s = len(A)
    a = np.zeros((s, s))
    b = np.zeros(s)
    # du_r = sum_{j<=r} (prod_{m=j+1}^{r} A_m) k_j ;  U_r = U_0 + sum_{r'<=r} B_r' du_r'
    def coef(j, r):
        return np.prod(A[j + 1:r + 1])
    for st in range(s):  # stage st evaluates at U_{st}
        for j in range(st):
            a[st, j] = sum(B[r] * coef(j, r) for r in range(j, st))
    for j in range(s):
        b[j] = sum(B[r] * coef(j, r) for r in range(j, s))
    return a, b, C


def test_lserk_order_conditions():
    a, b, C = _butcher()
    c = a.sum(axis=1)
    assert np.abs(c - C).max() < 1e-15
    conds = [b.sum(), b @ c, b @ c ** 2, b @ (a @ c), b @ c ** 3, b @ (c * (a @ c)),
             b @ (a @ c ** 2), b @ (a @ (a @ c))]
    assert np.allclose(conds, GOLD["lserk45_order_conditions"]["value"], atol=1e-15, rtol=0)


def test_lserk_temporal_convergence_order_four():
    """the time step of the oracle on a fixed mesh: errors against a tiny-dt
    solution decay as dt^4"""
    wl = W.mms_workload(K=2, N=3)
    o = O.Oracle(wl.params, wl.mesh)
    T = 0.4
    ref = o.advance(wl.U0, T / 256, 256)
    errs = []
    for ns in (8, 16, 32):
        errs.append(np.abs(o.advance(wl.U0, T / ns, ns) - ref).max())
    eoc = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert eoc.min() > 3.7, eoc


def test_fourteen_stage_scheme_order_conditions():
    """the 2N-storage coefficients of the fourteen-stage scheme, turned into a
    Butcher tableau, meet the eight fourth-order conditions (to the 16 digits
    the coefficients are published with) and their stage times are the row sums"""
    a, b, C = _butcher(1)
    assert len(b) == 14
    c = a.sum(axis=1)
    assert np.abs(c - C).max() < 1e-14
    conds = [b.sum(), b @ c, b @ c ** 2, b @ (a @ c), b @ c ** 3, b @ (c * (a @ c)),
             b @ (a @ c ** 2), b @ (a @ (a @ c))]
    assert np.allclose(conds, GOLD["lserk45_order_conditions"]["value"], atol=1e-13, rtol=0)


def test_fourteen_stage_temporal_convergence_order_four():
    wl = W.mms_workload(K=2, N=3)
    p = dict(wl.params, time_scheme=1)
    o = O.Oracle(p, wl.mesh)
    T = 0.8
    ref = o.advance(wl.U0, T / 256, 256)
    errs = [np.abs(o.advance(wl.U0, T / ns, ns) - ref).max() for ns in (8, 16, 32)]
    eoc = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert eoc.min() > 3.6, eoc


def test_fourteen_stage_scheme_is_stable_at_its_larger_step():
    """the scheme's stability region is about 3.8 times longer on the imaginary
    axis; at 3 times the five-stage step of the manufactured solution it still
    converges to the same solution"""
    wl = W.mms_workload(K=2, N=3)
    o5 = O.Oracle(wl.params, wl.mesh)
    o14 = O.Oracle(dict(wl.params, time_scheme=1), wl.mesh)
    dt = o5.stable_dt(wl.U0, 0.9, 0.9)
    U5 = o5.advance(wl.U0, dt, 30)
    U14 = o14.advance(wl.U0, 3 * dt, 10)
    assert np.abs(U14 - U5).max() < 1e-6 * np.abs(U5).max()
