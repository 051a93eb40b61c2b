"""GPU parity of the split form (Sec. 2.2 "Nonlinear Stability": Pirozzoli's
kinetic-energy-preserving two-point flux on Gauss-Lobatto nodes), Sutherland's
law (Sec. 2.1 Eq. sutherland), the fourteen-stage RK scheme (Sec. 2.2 "Time
integration"), the supersonic Taylor-Green vortex that combines them with
shock capturing (Sec. 5.2), the dissipation rates of Sec. 5.2 and the
optional neighbour smoothing of the blending factor.  The HIP library through
its C ABI against the FP64 oracle on the same seeded inputs; tolerances as in
the other parity tests (relative L2 over all variables and nodes, stacked)."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _solver(params, mesh):
    import paper_2404_12703_amd as P
    return P.Solver(params, mesh)


def _split_case(N, K=3, viscous=1, viscosity=0, riemann=0, seed=21, rotate=True, curved=True):
    m = W.box_mesh(K, 0.0, 2 * np.pi, N, amp=0.05 if curved else 0.0, rotate=rotate)
    p = W.params(N, node_type=1, riemann=riemann, viscous=viscous, mu=1e-2, volume_flux=1,
                 viscosity=viscosity, T_ref=0.8)
    X = m.points(W.lgl_points(N))
    return p, m, W.random_smooth_state(X, seed, 1.4, m.period)


@pytest.mark.parametrize("N,viscous,viscosity,riemann", [(3, 1, 0, 0), (4, 0, 0, 1), (5, 1, 1, 1), (7, 1, 1, 0),
                                                         (2, 1, 0, 1), (1, 1, 0, 0), (9, 1, 0, 1)])
def test_split_form_rhs_and_step_parity(N, viscous, viscosity, riemann):
    """curved, relabelled meshes (every face orientation): one evaluation and one step"""
    p, m, U = _split_case(N, K=3 if N < 9 else 2, viscous=viscous, viscosity=viscosity, riemann=riemann)
    _say(f"[split] N={N} viscous={viscous} sutherland={viscosity} riemann={riemann} E={m.n_elems}")
    o = O.Oracle(p, m)
    s = _solver(p, m)
    s.set_state(U)
    e = rel(s.rhs(0.1), o.rhs(U, 0.1))
    _say(f"  rhs rel L2 {e:.3e}")
    assert e <= 1e-12
    dt = o.stable_dt(U, 0.5, 0.5)
    assert abs(s.stable_dt(0.5, 0.5) / dt - 1.0) < 1e-12
    s.set_state(U)
    s.advance(2, dt)
    Uo = o.advance(U, dt, 2)
    assert rel(s.state(), Uo) <= 1e-12
    assert rel(s.state() - U, Uo - U) <= 1e-9


def test_split_form_freestream_and_conservation_on_gpu():
    p, m, U = _split_case(4, K=3)
    X = m.points(W.lgl_points(4))
    s = _solver(p, m)
    Uf = W.uniform_state(X, 1.2, (0.3, -0.2, 0.5), 2.0, 1.4)
    s.set_state(Uf)
    assert np.abs(s.rhs()).max() < 1e-10 * np.abs(Uf).max() / (2 * np.pi / 3)
    s.set_state(U)
    I0 = s.integrals()
    s.advance(10, s.stable_dt(0.5, 0.5))
    I1 = s.integrals()
    scale = O.Oracle(p, m).integrals(np.abs(U))
    assert np.all(np.abs(I1[:5] - I0[:5]) <= 1e-13 * scale[:5])


@pytest.mark.parametrize("scheme", [0, 1])
def test_time_schemes_parity(scheme):
    """five and fourteen stages: 3 steps of a curved TGV, N = 5"""
    wl = W.tgv_workload(K=3, N=5, rotate=True)
    p = dict(wl.params)
    p["time_scheme"] = scheme
    o = O.Oracle(p, wl.mesh)
    s = _solver(p, wl.mesh)
    dt = o.stable_dt(wl.U0)
    s.set_state(wl.U0)
    s.advance(3, dt)
    Uo = o.advance(wl.U0, dt, 3)
    assert rel(s.state(), Uo) <= 1e-12
    assert rel(s.state() - wl.U0, Uo - wl.U0) <= 1e-9


def test_sutherland_standard_form_parity():
    """Sutherland's law with the standard weak form on Gauss nodes, on a state
    with O(1) variation of the temperature (no large background)"""
    m = W.box_mesh(3, 0.0, 2 * np.pi, 4, amp=0.05, rotate=True)
    p = W.params(4, riemann=1, viscous=1, mu=5e-2, viscosity=1, T_ref=0.8)
    U = W.random_smooth_state(m.points(W.gl_points(4)), 31, 1.4, m.period)
    o = O.Oracle(p, m)
    s = _solver(p, m)
    s.set_state(U)
    assert rel(s.rhs(0.0), o.rhs(U, 0.0)) <= 1e-12
    dt = o.stable_dt(U)
    assert abs(s.stable_dt(0.9, 0.9) / dt - 1.0) < 1e-12
    s.advance(2, dt)
    Uo = o.advance(U, dt, 2)
    assert rel(s.state(), Uo) <= 1e-12
    assert rel(s.state() - U, Uo - U) <= 1e-9


def _ctgv(K=4, N=5):
    return W.compressible_tgv_workload(K=K, N=N, curved=True, rotate=True)


def test_compressible_tgv_alpha_and_rhs_parity():
    """Ma = 1.25: split form + Sutherland + blending, with the factors of both
    sides compared, then frozen to the oracle's for the state parity"""
    wl = _ctgv()
    _say(f"[ctgv] E={wl.mesh.n_elems} N={wl.params['N']}")
    o = O.Oracle(wl.params, wl.mesh)
    s = _solver(wl.params, wl.mesh)
    s.set_state(wl.U0)
    Rg = s.rhs(0.0)
    Ro = o.rhs(wl.U0, 0.0)
    ag, ao = s.alpha(), o.alpha()
    flips = int(np.sum((ag > 0) != (ao > 0)))
    _say(f"  alpha>0 {np.mean(ao > 0):.3f}, flips {flips}, max |dalpha| {np.abs(ag - ao).max():.2e}")
    assert flips == 0
    assert np.abs(ag - ao).max() <= 1e-10
    assert rel(Rg, Ro) <= 1e-12
    # every element blended with its own factor: the split-form blend pass
    alpha = np.random.default_rng(5).uniform(0.0, 1.0, wl.mesh.n_elems)
    o.set_alpha(alpha)
    s.set_alpha(alpha)
    assert rel(s.rhs(0.0), o.rhs(wl.U0, 0.0)) <= 1e-12


def test_compressible_tgv_steps_parity():
    """five steps of the fourteen-stage scheme at the workload's CFL (70
    evaluations of the operator: the state bound lies between one step's
    1e-12 and a hundred steps' 1e-10)"""
    wl = _ctgv(K=3, N=5)
    o = O.Oracle(wl.params, wl.mesh)
    s = _solver(wl.params, wl.mesh)
    dt = o.stable_dt(wl.U0, wl.cfl, wl.cfl)
    s.set_state(wl.U0)
    s.advance(5, dt)
    Uo = o.advance(wl.U0, dt, 5)
    ag, ao = s.alpha(), o.alpha()
    assert int(np.sum((ag > 0) != (ao > 0))) == 0
    assert rel(s.state(), Uo) <= 1e-11
    assert rel(s.state() - wl.U0, Uo - wl.U0) <= 1e-9


@pytest.mark.parametrize("smooth", [0, 1])
def test_alpha_smoothing_option(smooth):
    """the element-local factor (default) and the optional neighbour smoothing"""
    wl = W.blast_workload(K=5, N=4, rotate=True)
    p = dict(wl.params)
    p["alpha_smooth"] = smooth
    o = O.Oracle(p, wl.mesh)
    s = _solver(p, wl.mesh)
    s.set_state(wl.U0)
    Rg = s.rhs(0.0)
    Ro = o.rhs(wl.U0, 0.0)
    ag, ao = s.alpha(), o.alpha()
    assert int(np.sum((ag > 0) != (ao > 0))) == 0
    assert np.abs(ag - ao).max() <= 1e-10
    assert rel(Rg, Ro) <= 1e-12


@pytest.mark.parametrize("case", ["tgv_gauss", "ctgv_split"])
def test_dissipation_rates_match_oracle(case):
    if case == "tgv_gauss":
        wl = W.tgv_workload(K=3, N=5, rotate=True)
    else:
        wl = _ctgv(K=3, N=4)
    o = O.Oracle(wl.params, wl.mesh)
    s = _solver(wl.params, wl.mesh)
    s.set_state(wl.U0)
    eg, eo = s.dissipation(), o.dissipation(wl.U0)
    _say(f"  eps_S {eg[0]:.6e} vs {eo[0]:.6e}, eps_D {eg[1]:.3e} vs {eo[1]:.3e}")
    assert abs(eg[0] - eo[0]) <= 1e-11 * abs(eo[0])
    assert abs(eg[1] - eo[1]) <= 1e-11 * abs(eo[0])
    # the state and the time stepping are untouched by the diagnostic
    assert np.array_equal(s.state(), wl.U0)
    dt = o.stable_dt(wl.U0, wl.cfl, wl.cfl)
    s.advance(1, dt)
    assert rel(s.state(), o.advance(wl.U0, dt, 1)) <= 1e-12


def test_dissipation_rate_of_the_tgv_at_t0():
    """eps_S(0) = 3/(4 Re) for the Taylor-Green vortex (its velocity field is
    solenoidal at t = 0, Sec. 5.2); to the discretisation error"""
    wl = W.tgv_workload(K=4, N=7, curved=False)
    s = _solver(wl.params, wl.mesh)
    s.set_state(wl.U0)
    eS, eD = s.dissipation()
    assert abs(eS / (3.0 / (4.0 * 1600.0)) - 1.0) < 1e-3
    assert abs(eD) < 1e-6 * eS
