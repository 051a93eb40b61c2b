"""GPU parity at every polynomial degree the library builds (one translation
unit per degree, each with its own thread layout and LDS tiling): the
standard form on Gauss and Gauss-Lobatto nodes, the mixed-precision form,
shock capturing over its whole degree range and the split form, each on a
small curved, relabelled mesh (every face orientation) whose element count
leaves a ragged last workgroup at most degrees."""
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


def _mesh(N, shape=(3, 2, 2)):
    # at N = 1 the geometry is trilinear: no curvature to resolve
    return W.box_mesh(shape, 0.0, 2 * np.pi, N, amp=0.05 if N > 1 else 0.0, rotate=True)


def _check(p, m, U, what, tol=1e-12):
    o = O.Oracle(p, m)
    s = _solver(p, m)
    s.set_state(U, 0.0)
    er = rel(s.rhs(0.07), o.rhs(U, 0.07))
    dt = o.stable_dt(U)
    s.set_state(U, 0.0)
    s.advance(1, dt)
    Ug, Uo = s.state(), o.advance(U, dt, 1)
    es, ed = rel(Ug, Uo), rel(Ug - U, Uo - U)
    _say(f"  {what}: rhs {er:.2e}, step {es:.2e}, increment {ed:.2e}")
    assert er <= tol
    assert es <= tol
    assert ed <= 1e3 * tol


@pytest.mark.parametrize("N", range(1, 10))
def test_gauss_navier_stokes_every_degree(N):
    m = _mesh(N)
    p = W.params(N, riemann=1, mu=1e-2)
    U = W.random_smooth_state(m.points(W.gl_points(N)), 20 + N, 1.4, m.period)
    _say(f"[degree {N}] Gauss, Navier-Stokes, Roe, E = {m.n_elems}")
    _check(p, m, U, f"N = {N} Gauss")


@pytest.mark.parametrize("N", range(1, 10))
def test_lobatto_euler_every_degree(N):
    m = _mesh(N)
    p = W.params(N, node_type=1, riemann=0, viscous=0)
    U = W.random_smooth_state(m.points(W.lgl_points(N)), 40 + N, 1.4, m.period)
    _say(f"[degree {N}] Gauss-Lobatto, Euler, LLF, E = {m.n_elems}")
    _check(p, m, U, f"N = {N} Lobatto")


@pytest.mark.parametrize("N", range(1, 10))
def test_mixed_precision_every_degree(N):
    """parity unpinned (FP32 arithmetic): the mixed form against the oracle on
    an O(1) state, where FP32 rounding amplified by the differentiation stays
    near 1e-6; a wrong index or term would show at O(1)"""
    m = _mesh(N)
    p = W.params(N, riemann=1, mu=1e-2)
    U = W.random_smooth_state(m.points(W.gl_points(N)), 60 + N, 1.4, m.period)
    s = _solver(dict(p, precision=1), m)
    s.set_state(U, 0.0)
    e = rel(s.rhs(0.07), O.Oracle(p, m).rhs(U, 0.07))
    _say(f"[degree {N}] mixed precision: rhs {e:.2e}")
    assert e <= 1e-4


def _noisy_lobatto_state(m, N, seed):
    """a smooth state with per-node noise of relative size 0.5% to 2% per
    element, so that every element has energy in its top modes"""
    U = W.random_smooth_state(m.points(W.lgl_points(N)), seed, 1.4, m.period)
    rng = np.random.default_rng(seed)
    amp = 10.0 ** rng.uniform(-2.3, -1.7, m.n_elems)
    return U * (1.0 + amp[None, :, None] * rng.uniform(-1.0, 1.0, U.shape))


@pytest.mark.parametrize("N", range(2, 8))
def test_shock_capturing_every_degree(N):
    """every element blended with its own alpha in [0, 1] (frozen on both
    sides); then the indicator itself, with its threshold at the median of the
    elements' top-mode energy and a gentle logistic (s = 2), so that (almost)
    every element takes a value strictly inside (0, 1)"""
    m = _mesh(N)
    kw = dict(node_type=1, riemann=0, viscous=1, shock=1, mu=1e-2)
    p = W.params(N, **kw)
    U = W.random_smooth_state(m.points(W.lgl_points(N)), 80 + N, 1.4, m.period)
    alpha = np.random.default_rng(N).uniform(0.0, 1.0, m.n_elems)
    alpha[:2] = [0.0, 1.0]
    o = O.Oracle(p, m)
    o.set_alpha(alpha)
    s = _solver(p, m)
    s.set_alpha(alpha)
    s.set_state(U)
    e = rel(s.rhs(0.0), o.rhs(U, 0.0))
    _say(f"[degree {N}] frozen random alpha: rhs {e:.2e}")
    assert e <= 1e-12
    # threshold from the oracle: invert its logistic (no clip is reached at s = 2)
    U = _noisy_lobatto_state(m, N, 90 + N)
    T0 = 10.0 ** (-1.8 * (N + 1) ** 0.25)
    o = O.Oracle(W.params(N, ind_a=1.0, ind_s=2.0, **kw), m)
    a0 = np.array([o.indicator(U, el) for el in range(m.n_elems)])
    T = float(np.median(T0 - 0.5 * T0 * np.log(1.0 / a0 - 1.0)))
    p = W.params(N, ind_a=T / T0, ind_s=2.0, **kw)
    o = O.Oracle(p, m)
    s = _solver(p, m)
    s.set_state(U)
    Rg, Ro = s.rhs(0.0), o.rhs(U, 0.0)
    ag, ao = s.alpha(), o.alpha()
    inside = int(((ao > 0.01) & (ao < 0.99)).sum())
    assert inside >= m.n_elems - 2
    # no element may cross a clipping edge between the two sides
    assert ((ag > 0) == (ao > 0)).all() and ((ag < 1) == (ao < 1)).all()
    # the top-mode energy is a difference of sums of squares near 1 (rounding
    # about 1e-14 at most); the logistic's slope s / 4T carries it into alpha
    tol = max(1e-12, 2.0 / (4.0 * T) * 1e-14)
    da = float(np.abs(ag - ao).max())
    er = rel(Rg, Ro)
    _say(f"  indicator: threshold {T:.2e}, {inside} of {m.n_elems} inside (0.01, 0.99), "
         f"max |d alpha| {da:.2e} (bound {tol:.1e}), rhs {er:.2e}")
    assert da <= tol
    assert er <= 1e-12 + 10.0 * da


@pytest.mark.parametrize("N", [6, 8])
def test_split_form_remaining_degrees(N):
    m = _mesh(N)
    p = W.params(N, node_type=1, riemann=1, mu=1e-2, volume_flux=1)
    U = W.random_smooth_state(m.points(W.lgl_points(N)), 100 + N, 1.4, m.period)
    _say(f"[degree {N}] split form, E = {m.n_elems}")
    _check(p, m, U, f"N = {N} split")
