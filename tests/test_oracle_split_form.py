"""Pins of the oracle's split-form DG operator (Sec. 2.2 "Nonlinear Stability":
strong form with two-point volume fluxes on Gauss-Lobatto nodes, Pirozzoli's
kinetic-energy-preserving flux) against what the method fixes:

* the two-point flux is consistent (F#(U, U; m) = F(U).m, the Riemann
  solvers' consistent value) and symmetric, and Pirozzoli's flux meets the
  kinetic-energy-preservation condition on its momentum component;
* with the mean of the two fluxes as two-point flux, the split form on a mesh
  with constant metric terms is the standard DG operator (summation by parts);
* freestream preservation on curved meshes (metric terms averaged between the
  two nodes), with and without the FV blend;
* conservation of mass, momentum and energy;
* the design order on the manufactured solution with Gauss-Lobatto nodes
  (Sec. 5.1: the paper's convergence test of the split form).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

GAMMA = 1.4


def _cons(rho, u, p):
    u = np.asarray(u, dtype=float)
    return np.array([rho, *(rho * u), p / (GAMMA - 1) + 0.5 * rho * u @ u])


STATES = [(_cons(1.0, [0.3, -0.1, 0.2], 1.0), _cons(0.8, [0.1, 0.2, -0.1], 0.7)),
          (_cons(2.0, [-0.5, 0.4, 0.0], 3.0), _cons(1.1, [0.2, -0.3, 0.6], 1.4))]
DIRS = [np.array([1.0, 0.0, 0.0]), np.array([0.3, -1.2, 0.45])]


def _o():
    return O.Oracle(W.params(1, node_type=1, viscous=0), W.box_mesh(2, -1.0, 1.0, 1))


@pytest.mark.parametrize("which", [1, 2])
def test_two_point_flux_consistent_and_symmetric(which):
    o = _o()
    for UL, UR in STATES:
        for m in DIRS:
            s = np.linalg.norm(m)
            # the Riemann solvers reduce to the physical flux for equal states
            Fphys = o.riemann(0, UL, UL, m / s) * s
            assert np.allclose(o.two_point(which, UL, UL, m), Fphys, rtol=1e-14, atol=1e-14)
            assert np.allclose(o.two_point(which, UL, UR, m), o.two_point(which, UR, UL, m),
                               rtol=1e-15, atol=1e-15)


def test_pirozzoli_flux_is_kinetic_energy_preserving():
    """Jameson's condition: the momentum flux is the mean velocity times the
    mass flux plus a pressure term (here the mean pressure); and the energy flux
    carries the mean total enthalpy with the mass flux"""
    o = _o()
    for UL, UR in STATES:
        for m in DIRS:
            F = o.two_point(1, UL, UR, m)
            uL, uR = UL[1:4] / UL[0], UR[1:4] / UR[0]
            pL = (GAMMA - 1) * (UL[4] - 0.5 * UL[0] * uL @ uL)
            pR = (GAMMA - 1) * (UR[4] - 0.5 * UR[0] * uR @ uR)
            ub, pb = 0.5 * (uL + uR), 0.5 * (pL + pR)
            assert np.allclose(F[1:4], ub * F[0] + pb * m, rtol=1e-14, atol=1e-14)
            Hb = 0.5 * ((UL[4] + pL) / UL[0] + (UR[4] + pR) / UR[0])
            assert abs(F[4] - Hb * F[0]) < 1e-14 * abs(F[4])
            # and it is not the mean of the fluxes
            assert not np.allclose(F, o.two_point(2, UL, UR, m), rtol=1e-6)


@pytest.mark.parametrize("N", [2, 4])
def test_mean_flux_split_form_is_the_standard_operator_on_affine_meshes(N):
    """W D + D^T W = B on Gauss-Lobatto nodes: with F# = (F(U_a) + F(U_b))/2 and
    constant metric terms the split form equals the weak form; a wrong
    boundary correction or a missing factor 2 breaks this"""
    m = W.box_mesh((3, 2, 2), 0.0, 2 * np.pi, N, rotate=True)
    X = m.points(W.lgl_points(N))
    U = W.random_smooth_state(X, 4, GAMMA, m.period)
    pw = W.params(N, node_type=1, riemann=1, viscous=1, mu=2e-2)
    ps = dict(pw, volume_flux=2)
    Rw = O.Oracle(pw, m).rhs(U)
    Rs = O.Oracle(ps, m).rhs(U)
    assert np.abs(Rs - Rw).max() < 1e-12 * np.abs(Rw).max()
    # Pirozzoli's flux differs from it at truncation level
    Rk = O.Oracle(dict(pw, volume_flux=1), m).rhs(U)
    assert np.abs(Rk - Rw).max() > 1e-6 * np.abs(Rw).max()


@pytest.mark.parametrize("alpha", [None, 1.0, 0.4])
def test_kep_freestream_on_curved_relabelled_mesh(alpha):
    N = 5
    m = W.box_mesh(3, 0.0, 2 * np.pi, N, amp=0.05, seed=0, rotate=True)
    p = W.params(N, node_type=1, riemann=0, viscous=1, mu=1e-2, volume_flux=1, shock=alpha is not None)
    o = O.Oracle(p, m)
    if alpha is not None:
        o.set_alpha(np.full(m.n_elems, alpha))
    X = m.points(W.lgl_points(N))
    U = W.uniform_state(X, 1.2, (0.3, -0.2, 0.5), 2.0, GAMMA)
    R = o.rhs(U)
    assert np.abs(R).max() < 1e-10 * np.abs(U).max() / (2 * np.pi / 3)


def test_kep_conservation_over_steps():
    N = 4
    m = W.box_mesh(3, 0.0, 2 * np.pi, N, amp=0.05, seed=1, rotate=True)
    p = W.params(N, node_type=1, riemann=1, viscous=1, mu=5e-2, volume_flux=1)
    o = O.Oracle(p, m)
    X = m.points(W.lgl_points(N))
    U0 = W.random_smooth_state(X, 2, GAMMA, m.period)
    U1 = o.advance(U0, o.stable_dt(U0), 10)
    I0, I1 = o.integrals(U0), o.integrals(U1)
    scale = o.integrals(np.abs(U0))
    assert np.all(np.abs(I1[:5] - I0[:5]) <= 1e-13 * scale[:5])
    assert np.abs(U1 - U0).max() > 1e-3


def _wJ(o):
    b, g = o.basis(), o.geometry()
    return g["J"] * np.einsum("k,j,i->kji", b["w"], b["w"], b["w"]).ravel()[None, :]


def test_kep_manufactured_solution_converges_at_design_order():
    """Sec. 5.1 (Fig. convtest, left): the split form on Gauss-Lobatto nodes
    converges at order N + 1; N = 3 here"""
    T, N = 0.2, 3
    errs = []
    for K in (2, 4, 8):
        mesh = W.box_mesh(K, -1.0, 1.0, N)
        p = W.params(N, node_type=1, riemann=0, viscous=1, source=1, mu=1e-3, volume_flux=1)
        X = mesh.points(W.lgl_points(N))
        U0 = W.mms_state(X, 0.0, GAMMA)
        o = O.Oracle(p, mesh)
        ns = int(np.ceil(T / o.stable_dt(U0, 0.9, 0.9)))
        U = o.advance(U0, T / ns, ns)
        errs.append(np.sqrt((((U - W.mms_state(X, T, GAMMA)) ** 2).sum(0) * _wJ(o)).sum()))
    eoc = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert eoc[-1] > 3.7, eoc
