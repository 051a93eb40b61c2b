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
