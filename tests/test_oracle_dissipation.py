"""Pins of the oracle's dissipation rates (Sec. 5.2: solenoidal eps_S from the
vorticity, dilatational eps_D from the divergence, both weighted with mu(T)),
computed from the BR1 lifted gradients, against closed forms:

* TGV at t = 0 (Eq. tgv_ic): <|omega|^2> = 3/4 and div u = 0, so eps_S = 3/(4 Re),
  eps_D = 0, and eps_S equals -dE_k/dt of the operator (incompressible start);
* a shear wave has vorticity and no divergence, a compression wave the
  opposite, with mean squares A^2 k^2 / 2;
* Sutherland's law weights both with the viscosity at the local temperature.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))
GAMMA = 1.4


def _state(rho, u, v, w, p):
    return np.stack([rho, rho * u, rho * v, rho * w, p / (GAMMA - 1) + 0.5 * rho * (u * u + v * v + w * w)])


def test_tgv_initial_dissipation_rates():
    Re = 1600.0
    wl = W.tgv_workload(K=4, N=7, Re=Re)
    o = O.Oracle(wl.params, wl.mesh)
    epsS, epsD = o.dissipation(wl.U0)
    ref = -GOLD["tgv_dEk_dt0_times_Re"]["value"] / Re
    assert abs(epsS / ref - 1) < 1e-3
    assert abs(epsD) < 1e-6 * epsS
    # the same number from the kinetic-energy budget of the time derivative
    U, R = wl.U0, o.rhs(wl.U0)
    b, g = o.basis(), o.geometry()
    wJ = g["J"] * np.einsum("k,j,i->kji", b["w"], b["w"], b["w"]).ravel()[None, :]
    u = U[1:4] / U[0]
    dEk = (wJ * ((u * R[1:4]).sum(0) - 0.5 * (u * u).sum(0) * R[0])).sum() / wJ.sum()
    assert abs(epsS + dEk) < 2e-3 * epsS


@pytest.mark.parametrize("law", [0, 1])
def test_shear_and_compression_waves(law):
    """u_y = A sin x: omega_z = A cos x, eps_S = mu A^2/2, eps_D = 0;
    u_x = A sin x: div u = A cos x, eps_S = 0, eps_D = (4/3) mu A^2/2.
    With Sutherland's law at uniform T0 = 2 T_ref both scale with mu(T0)/mu."""
    N, mu, A = 7, 0.01, 0.3
    m = W.box_mesh(6, 0.0, 2 * np.pi, N, amp=0.05, rotate=True)
    X = m.points(W.gl_points(N))
    x = X[0]
    z, one = np.zeros_like(x), np.ones_like(x)
    T0 = 2.0 if law else 1.0
    p = W.params(N, riemann=1, viscous=1, mu=mu, viscosity=law, T_ref=1.0)
    o = O.Oracle(p, m)
    mT = o.viscosity(T0)
    if law:
        assert abs(mT / mu - 1.4042 * 2 ** 1.5 / 2.4042) < 1e-14
    eS, eD = o.dissipation(_state(one, z, A * np.sin(x), z, T0 * one))
    assert abs(eS / (mT * A * A / 2) - 1) < 1e-6 and abs(eD) < 1e-8 * eS
    eS, eD = o.dissipation(_state(one, A * np.sin(x), z, z, T0 * one))
    assert abs(eD / (4.0 / 3.0 * mT * A * A / 2) - 1) < 1e-6 and abs(eS) < 1e-8 * eD
    # a wave along z with a y velocity: omega_x = -A cos z
    eS, eD = o.dissipation(_state(one, z, A * np.sin(X[2]), z, T0 * one))
    assert abs(eS / (mT * A * A / 2) - 1) < 1e-6 and abs(eD) < 1e-8 * eS
