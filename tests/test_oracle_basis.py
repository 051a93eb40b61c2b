"""Pins of the oracle's 1-D building blocks (Sec. 2.2, Eq. dgsem and the
definitions of D-hat and l-hat beside it) against quadrature exactness,
textbook node sets and the summation-by-parts identity."""
import json
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def _basis(N, nodes):
    m = W.box_mesh(2, -1.0, 1.0, 1)
    return O.Oracle(W.params(N, node_type=nodes, viscous=0), m).basis()


@pytest.mark.parametrize("N", [1, 2, 3, 5, 7, 9])
def test_gauss_nodes_match_numpy_and_integrate_2N_plus_1(N):
    b = _basis(N, 0)
    x_ref, w_ref = np.polynomial.legendre.leggauss(N + 1)
    assert np.allclose(b["x"], x_ref, atol=1e-14, rtol=0)
    assert np.allclose(b["w"], w_ref, atol=1e-14, rtol=0)
    for k in range(2 * N + 2):
        exact = (1.0 - (-1.0) ** (k + 1)) / (k + 1)
        assert abs((b["w"] * b["x"] ** k).sum() - exact) < 1e-13


@pytest.mark.parametrize("N", [2, 3, 5, 7])
def test_lobatto_nodes_integrate_2N_minus_1(N):
    b = _basis(N, 1)
    assert b["x"][0] == -1.0 and b["x"][-1] == 1.0
    for k in range(2 * N):
        exact = (1.0 - (-1.0) ** (k + 1)) / (k + 1)
        assert abs((b["w"] * b["x"] ** k).sum() - exact) < 1e-13
    # degree 2N is not integrated exactly by N+1 Lobatto points
    k = 2 * N
    assert abs((b["w"] * b["x"] ** k).sum() - 2.0 / (k + 1)) > 1e-6


def test_golden_small_node_sets():
    b = _basis(1, 0)
    assert np.allclose(b["x"], GOLD["gl_N1_nodes"]["value"], atol=1e-15)
    assert np.allclose(b["w"], GOLD["gl_N1_weights"]["value"], atol=1e-15)
    b = _basis(2, 1)
    assert np.allclose(b["x"], GOLD["lgl_N2_nodes"]["value"], atol=1e-15)
    assert np.allclose(b["w"], GOLD["lgl_N2_weights"]["value"], atol=1e-15)


@pytest.mark.parametrize("N,nodes", [(3, 0), (5, 0), (7, 0), (4, 1), (5, 1)])
def test_derivative_matrix_exact_on_polynomials(N, nodes):
    b = _basis(N, nodes)
    x, D = b["x"], b["D"]
    for k in range(N + 1):
        d = D @ x ** k
        ref = k * x ** (k - 1) if k > 0 else np.zeros_like(x)
        assert np.abs(d - ref).max() < 1e-11 * max(1, k ** 2)


@pytest.mark.parametrize("N,nodes", [(3, 0), (7, 0), (5, 1)])
def test_dhat_row_sums_and_sbp(N, nodes):
    """sum_j Dhat_ij = lhat^-_i - lhat^+_i (Dhat applied to a constant flux
    equals minus the surface terms), and W D + D^T W = l(1)l(1)^T - l(-1)l(-1)^T."""
    b = _basis(N, nodes)
    rs = b["Dhat"].sum(axis=1)
    assert np.abs(rs - (b["lhm"] - b["lhp"])).max() < 1e-12
    Wm = np.diag(b["w"])
    Q = Wm @ b["D"]
    B = np.outer(b["lp"], b["lp"]) - np.outer(b["lm"], b["lm"])
    assert np.abs(Q + Q.T - B).max() < 1e-12


@pytest.mark.parametrize("N,nodes", [(3, 0), (4, 1)])
def test_boundary_values_of_lagrange_basis(N, nodes):
    """l_j(+-1) against scipy's Lagrange interpolant of the unit vectors"""
    from scipy.interpolate import BarycentricInterpolator
    b = _basis(N, nodes)
    for j in range(N + 1):
        e = np.zeros(N + 1)
        e[j] = 1.0
        P = BarycentricInterpolator(b["x"], e)
        assert abs(P(1.0) - b["lp"][j]) < 1e-13
        assert abs(P(-1.0) - b["lm"][j]) < 1e-13
    if nodes == 1:
        assert np.allclose(b["lhp"], np.eye(N + 1)[-1] / b["w"][-1])
