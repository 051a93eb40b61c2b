"""Pins of the oracle's DG operator (Sec. 2.2 Eq. dgsem with BR1 lifting and
the Navier-Stokes fluxes of Sec. 2.1) and of the full time step, against what
the method and the mathematics fix: freestream preservation, conservation,
the design order N+1 on the manufactured solution (Sec. 5.1), the
Taylor-Green kinetic energy and its initial decay rate (Sec. 5.2), the viscous
decay of a shear wave, and invariance under element relabelling."""
import json
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def _wJ(o):
    b, g = o.basis(), o.geometry()
    wq = np.einsum("k,j,i->kji", b["w"], b["w"], b["w"]).ravel()
    return g["J"] * wq[None, :]


@pytest.mark.parametrize("nodes,riemann", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_freestream_on_curved_relabelled_mesh(nodes, riemann):
    """a uniform state is a steady solution; only round-off remains.  Bound:
    1e-10 * flux scale / h (a wrong metric sign or index gives O(flux/h))."""
    N = 5
    m = W.box_mesh(3, 0.0, 2 * np.pi, N, amp=0.05, seed=0, rotate=True)
    p = W.params(N, node_type=nodes, riemann=riemann, viscous=1, mu=1e-2)
    o = O.Oracle(p, m)
    X = m.points(W.ref_points(N, nodes))
    U = W.uniform_state(X, 1.2, (0.3, -0.2, 0.5), 2.0, 1.4)
    R = o.rhs(U)
    h = 2 * np.pi / 3
    assert np.abs(R).max() < 1e-10 * np.abs(U).max() / h


def test_conservation_over_steps():
    """periodic, no source: sum_e sum_ijk w J U is constant (single-valued face fluxes)"""
    N = 4
    m = W.box_mesh(3, 0.0, 2 * np.pi, N, amp=0.05, seed=1, rotate=True)
    p = W.params(N, node_type=0, riemann=1, viscous=1, mu=5e-2)
    o = O.Oracle(p, m)
    X = m.points(W.gl_points(N))
    U0 = W.random_smooth_state(X, 2, 1.4, m.period)
    dt = o.stable_dt(U0)
    U1 = o.advance(U0, dt, 10)
    I0, I1 = o.integrals(U0), o.integrals(U1)
    scale = o.integrals(np.abs(U0))
    assert np.all(np.abs(I1[:5] - I0[:5]) <= 1e-13 * scale[:5])
    # and the state did change
    assert np.abs(U1 - U0).max() > 1e-3


def _mms_errors(N, Ks, T, cfl):
    errs = []
    for K in Ks:
        wl = W.mms_workload(K=K, N=N)
        o = O.Oracle(wl.params, wl.mesh)
        dt0 = o.stable_dt(wl.U0, cfl, cfl)
        ns = int(np.ceil(T / dt0))
        U = o.advance(wl.U0, T / ns, ns)
        Ue = W.mms_state(wl.mesh.points(W.gl_points(N)), T, 1.4)
        errs.append(np.sqrt((((U - Ue) ** 2).sum(0) * _wJ(o)).sum()))
    return np.log2(np.array(errs[:-1]) / np.array(errs[1:]))


def test_manufactured_solution_converges_at_design_order():
    """Sec. 5.1: error of the manufactured solution at t = 0.5 decays as
    h^(N+1): N = 3 on 2^3 .. 16^3 elements at CFL 0.9 (measured 4.12, 4.03, 3.99)"""
    eoc = _mms_errors(3, (2, 4, 8, 16), 0.5, 0.9)
    assert eoc[-1] > 3.7, eoc


def test_manufactured_solution_converges_at_design_order_n5():
    """N = 5 on 2^3 .. 8^3 elements to t = 0.25 at CFL 0.3 (the time error stays
    below the spatial one): order 6 (measured 6.2, 5.9)"""
    eoc = _mms_errors(5, (2, 4, 8), 0.25, 0.3)
    assert eoc[-1] > 5.5, eoc


def test_manufactured_source_is_the_closed_form():
    """with the source switched on, the exact solution's residual R(U_e) - dU_e/dt
    must be the pure discretisation error, and the difference of the two RHS
    evaluations (source on - off) must equal 0.1 pi cos(.) (2,3,3,3,11)"""
    wl = W.mms_workload(K=2, N=3)
    o = O.Oracle(wl.params, wl.mesh)
    t = 0.3
    X = wl.mesh.points(W.gl_points(3))
    U = W.mms_state(X, t, 1.4)
    R1 = o.rhs(U, t)
    p0 = dict(wl.params)
    p0["source"] = 0
    o.set_params(p0)
    R0 = o.rhs(U, t)
    c = 0.1 * np.pi * np.cos(np.pi * (X[0] + X[1] + X[2] - t))
    fac = GOLD["mms_source_factors_gamma_1p4"]["value"]
    for v in range(5):
        assert np.abs((R1[v] - R0[v]) - fac[v] * c).max() < 1e-12


def test_taylor_green_kinetic_energy_and_decay_rate():
    """Sec. 5.2: E_k(0) = 1/8 and dE_k/dt(0) = -3/(4 Re) (div u = 0 at t = 0)"""
    Re = 1600.0
    wl = W.tgv_workload(K=4, N=7, curved=True, Re=Re)
    o = O.Oracle(wl.params, wl.mesh)
    U = wl.U0
    I = o.integrals(U)
    assert abs(I[5] - GOLD["tgv_Ek0"]["value"]) < 1e-10
    R = o.rhs(U)
    wJ = _wJ(o)
    u = U[1:4] / U[0]
    dEk = (wJ * ((u * R[1:4]).sum(0) - 0.5 * (u * u).sum(0) * R[0])).sum() / wJ.sum()
    ref = GOLD["tgv_dEk_dt0_times_Re"]["value"] / Re
    assert abs(dEk / ref - 1.0) < 1e-3


def test_shear_wave_decays_at_viscous_rate():
    """u = (0, A sin(kx), 0), uniform rho, p: velocity decays as exp(-nu k^2 t)"""
    nu, A, k = 0.05, 1e-4, 1.0
    m = W.box_mesh((4, 2, 2), 0.0, 2 * np.pi, 5)
    o = O.Oracle(W.params(5, riemann=1, viscous=1, mu=nu), m)
    X = m.points(W.gl_points(5))
    U = W.shear_wave_state(X, A, k, 1.0, 1.0 / (1.4 * 0.1 ** 2), 1.4)
    dt = o.stable_dt(U)
    ns = 200
    U1 = o.advance(U, dt, ns)
    v0, v1 = U[2] / U[0], U1[2] / U1[0]
    rate = -np.log((v1 * v0).sum() / (v0 * v0).sum()) / (ns * dt)
    assert abs(rate / (nu * k * k) - 1.0) < 1e-4


def test_viscous_terms_vanish_for_constant_fields():
    """BR1 lifting of a constant field is zero: viscous and inviscid RHS agree"""
    N = 4
    m = W.box_mesh(2, 0.0, 2 * np.pi, N, amp=0.05, rotate=True)
    X = m.points(W.gl_points(N))
    U = W.uniform_state(X, 0.8, (0.1, 0.2, -0.3), 1.5, 1.4)
    pv = W.params(N, riemann=1, viscous=1, mu=0.1)
    pi = dict(pv)
    pi["viscous"] = 0
    o = O.Oracle(pv, m)
    Rv = o.rhs(U)
    o.set_params(pi)
    Ri = o.rhs(U)
    assert np.abs(Rv - Ri).max() < 1e-11


def _match_nodes(Xa, Xb):
    """permutation perm[e][a] such that Xb[:, e, perm[e][a]] == Xa[:, e, a]"""
    E, n3 = Xa.shape[1], Xa.shape[2]
    perm = np.zeros((E, n3), dtype=np.int64)
    for e in range(E):
        d = ((Xa[:, e, :, None] - Xb[:, e, None, :]) ** 2).sum(0)
        perm[e] = d.argmin(axis=1)
        assert d.min(axis=1).max() < 1e-20
    return perm


@pytest.mark.parametrize("nodes", [0, 1])
def test_relabelling_elements_leaves_the_operator_invariant(nodes):
    N = 3
    p = W.params(N, node_type=nodes, riemann=1, viscous=1, mu=2e-2, shock=nodes)
    ma = W.box_mesh(2, 0.0, 2 * np.pi, N, amp=0.05, seed=3)
    mb = W.box_mesh(2, 0.0, 2 * np.pi, N, amp=0.05, seed=3, rotate=True, rot_seed=11)
    r = W.ref_points(N, nodes)
    Xa, Xb = ma.points(r), mb.points(r)
    perm = _match_nodes(Xa, Xb)
    Ua = W.random_smooth_state(Xa, 5, 1.4, ma.period)
    Ub = W.random_smooth_state(Xb, 5, 1.4, mb.period)
    oa, ob = O.Oracle(p, ma), O.Oracle(p, mb)
    if nodes == 1:
        alpha = np.linspace(0.0, 1.0, ma.n_elems)
        oa.set_alpha(alpha)
        ob.set_alpha(alpha)
    Ra, Rb = oa.rhs(Ua), ob.rhs(Ub)
    Rb_on_a = np.take_along_axis(Rb, perm[None], axis=2)
    assert np.abs(Ra - Rb_on_a).max() < 1e-11 * np.abs(Ra).max()
