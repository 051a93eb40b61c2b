"""The mixed-precision form (FP32 fluxes and contractions with FP32
accumulation; FP64 state, RK register and set-up) against the FP64 path.
Parity unpinned: there is no exact reference for the FP32 arithmetic; the
bounds are the measured errors with a margin, and the kinetic-energy bound is
the target of 1e-6 relative to FP64."""
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


def _run(wl, steps, dt):
    import paper_2404_12703_amd as P
    s = P.Solver(wl.params, wl.mesh)
    s.set_state(wl.U0)
    s.advance(steps, dt)
    return s.state(), s.integrals()


def _mixed_rhs_error(K, N, Ma, p_ref):
    import paper_2404_12703_amd as P
    wl = W.tgv_workload(K=K, N=N, rotate=True, precision=1, Ma=Ma)
    prm = dict(wl.params, p_ref=p_ref)
    s = P.Solver(prm, wl.mesh)
    s.set_state(wl.U0)
    Rm = s.rhs(0.0)
    Ro = O.Oracle(wl.params, wl.mesh).rhs(wl.U0, 0.0)
    comp = [rel(Rm[c], Ro[c]) for c in range(5)]
    return rel(Rm, Ro), comp


@pytest.mark.parametrize("K,N", [(3, 7), (4, 5)])
def test_mixed_rhs_close_to_oracle(K, N):
    """without the background shift: FP32 rounding of the p0 = 71 pressure
    flux, differentiated, sets the error (measured 6.8e-3)"""
    e, comp = _mixed_rhs_error(K, N, 0.1, 0.0)
    _say(f"[mixed rhs] N = {N}: rel L2 vs oracle {e:.3e}, per variable {np.array(comp)}")
    assert e < 2e-2


@pytest.mark.parametrize("K,N,Ma", [(3, 7, 0.1), (4, 5, 0.1), (3, 7, 0.05)])
def test_mixed_rhs_with_background_shift(K, N, Ma):
    """with p_ref = p0 (the FP32 state carries rho e - p_ref/(gamma-1)
    and the momentum fluxes drop the constant p_ref, exact by freestream) the
    momentum error falls to the FP32 rounding of the flow itself; the energy
    flux still carries the background enthalpy gamma p0/(gamma-1) u, whose FP32
    rounding bounds that variable"""
    p0 = 1.0 / (1.4 * Ma * Ma)
    e0, c0 = _mixed_rhs_error(K, N, Ma, 0.0)
    e1, c1 = _mixed_rhs_error(K, N, Ma, p0)
    _say(f"[mixed rhs, Ma {Ma}] N = {N}: rel L2 {e0:.3e} -> {e1:.3e} with p_ref; per variable "
         f"{np.array(c0)} -> {np.array(c1)}")
    assert max(c1[1:4]) < 0.1 * max(c0[1:4])  # momentum: an order of magnitude at least
    # measured 7.2e-4 and 6.6e-4 at Ma 0.1 (was 6.8e-3 and 6.4e-3), 2.8e-3 at Ma 0.05 (was 5.3e-2)
    assert e1 < (2e-3 if Ma >= 0.1 else 6e-3)


@pytest.mark.parametrize("K,N", [(4, 7), (5, 5)])
def test_mixed_kinetic_energy_error_after_steps(K, N):
    """TGV, curved mesh, 100 steps: E_k of the mixed form within 1e-6 of FP64
    (N = 7 and 5 take the two-nodes-per-thread volume sweep)"""
    wd = W.tgv_workload(K=K, N=N, precision=0)
    wm = W.tgv_workload(K=K, N=N, precision=1)
    dt = O.Oracle(wd.params, wd.mesh).stable_dt(wd.U0)
    Ud, Id = _run(wd, 100, dt)
    Um, Im = _run(wm, 100, dt)
    ek = abs(Im[5] - Id[5]) / abs(Id[5])
    el2 = rel(Um, Ud)
    _say(f"[mixed 100 steps] N = {N}: Ek rel err {ek:.3e}, state rel L2 {el2:.3e}")
    assert ek <= 1e-6
    assert el2 <= 1e-5


def _lobatto_case(N, seed, **kw):
    m = W.box_mesh(3, 0.0, 2 * np.pi, N, amp=0.05, rotate=True)
    p = W.params(N, node_type=1, mu=1e-2, **kw)
    return p, m, W.random_smooth_state(m.points(W.lgl_points(N)), seed, 1.4, m.period)


@pytest.mark.parametrize("N,kw", [
    (5, dict(riemann=0, volume_flux=1)),
    (7, dict(riemann=1, volume_flux=1, viscosity=1, T_ref=0.8)),
    (4, dict(riemann=1, viscosity=1, T_ref=0.8)),
    (5, dict(riemann=0, shock=1)),
    (3, dict(riemann=1, shock=1, volume_flux=1, viscosity=1, T_ref=0.8)),
])
def test_mixed_form_with_split_form_sutherland_and_blending(N, kw):
    """the mixed form beside the split form, Sutherland's law and the blend (the
    blending factor frozen at random values on both sides: the FP32 indicator
    is checked below on its own) against the FP64 oracle on an O(1) state"""
    p, m, U = _lobatto_case(N, 200 + N, **kw)
    o = O.Oracle(p, m)
    import paper_2404_12703_amd as P
    s = P.Solver(dict(p, precision=1), m)
    if kw.get("shock"):
        alpha = np.random.default_rng(N).uniform(0.0, 1.0, m.n_elems)
        o.set_alpha(alpha)
        s.set_alpha(alpha)
    s.set_state(U, 0.0)
    e = rel(s.rhs(0.05), o.rhs(U, 0.05))
    _say(f"[mixed] N = {N} {kw}: rhs vs oracle {e:.2e}")
    assert e <= 1e-4


def test_mixed_supersonic_tgv_and_dissipation():
    """the supersonic Taylor-Green workload (split form, Sutherland, blend,
    fourteen-stage RK) in mixed precision against FP64 on the GPU over 20
    steps at CFL 1.5 (the blend engages after a few steps on this coarse
    mesh, and the FP32 indicator decides it), and its dissipation rates
    against the oracle's.  At the workload's CFL of 2.5 the fourteen-stage
    scheme only just damps the highest modes of the 4^3 mesh, and the FP32
    rounding fed into them every stage grows to about 1e-5 in 20 steps"""
    import paper_2404_12703_amd as P
    wl = W.compressible_tgv_workload(K=4, N=5, curved=True, rotate=True)
    o = O.Oracle(wl.params, wl.mesh)
    dt = o.stable_dt(wl.U0, 1.5, 1.5)
    res = {}
    for prec in (0, 1):
        s = P.Solver(dict(wl.params, precision=prec), wl.mesh)
        s.set_state(wl.U0, 0.0)
        res[prec] = dict(diss=s.dissipation())
        s.advance(20, dt)
        res[prec].update(U=s.state(), I=s.integrals(), alpha=s.alpha())
    do = o.dissipation(wl.U0)
    dd = np.abs(res[1]["diss"] - do) / do[0]  # against eps_S (eps_D is small at t = 0)
    eu = rel(res[1]["U"], res[0]["U"])
    ek = abs(res[1]["I"][5] - res[0]["I"][5]) / abs(res[0]["I"][5])
    a64 = res[0]["alpha"]
    _say(f"[mixed supersonic TGV] eps {do} errors {dd}; 20 steps: alpha > 0 on {(a64 > 0).sum()} of "
         f"{a64.size} (max {a64.max():.2f}), |d alpha| {np.abs(res[1]['alpha'] - a64).max():.1e}, "
         f"state {eu:.2e}, E_k {ek:.2e}")
    assert dd.max() <= 1e-4
    assert eu <= 1e-4
    assert ek <= 1e-5


@pytest.mark.parametrize("N", range(2, 8))
def test_mixed_indicator_matches_oracle(N):
    """the FP32 indicator on states with energy in their top modes (smooth
    field plus per-node noise), the threshold at the median of the elements'
    top-mode energy: the logistic's steep part is where the FP32 value could
    move.  The shell energies are summed directly, so their rounding is
    relative (measured up to 8e-6 in alpha; formed as differences of nearly
    equal totals it was up to 1.2e-2)"""
    import paper_2404_12703_amd as P
    m = W.box_mesh((3, 2, 2), 0.0, 2 * np.pi, N, amp=0.05, rotate=True)
    U = W.random_smooth_state(m.points(W.lgl_points(N)), 90 + N, 1.4, m.period)
    rng = np.random.default_rng(90 + N)
    amp = 10.0 ** rng.uniform(-2.3, -1.7, m.n_elems)
    U = U * (1.0 + amp[None, :, None] * rng.uniform(-1.0, 1.0, U.shape))
    kw = dict(node_type=1, riemann=0, viscous=1, shock=1, mu=1e-2)
    T0 = 10.0 ** (-1.8 * (N + 1) ** 0.25)
    o = O.Oracle(W.params(N, ind_a=1.0, ind_s=2.0, **kw), m)
    a0 = np.array([o.indicator(U, el) for el in range(m.n_elems)])
    T = float(np.median(T0 - 0.5 * T0 * np.log(1.0 / a0 - 1.0)))
    p = W.params(N, ind_a=T / T0, **kw)
    o = O.Oracle(p, m)
    o.rhs(U, 0.0)
    ao = o.alpha()
    s = P.Solver(dict(p, precision=1), m)
    s.set_state(U)
    s.rhs(0.0)
    da = float(np.abs(s.alpha() - ao).max())
    _say(f"[mixed indicator] N = {N}: {int(((ao > 0) & (ao < 1)).sum())} of {ao.size} inside (0, 1), "
         f"max |d alpha| {da:.1e}")
    assert ((ao > 0) & (ao < 1)).sum() >= m.n_elems // 2
    assert da <= 5e-5
