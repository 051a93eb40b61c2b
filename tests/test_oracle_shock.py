"""Pins of the oracle's shock capturing (Sec. 2.3): the convex DG/FV blend,
the FV subcell operator on the Gauss-Lobatto subcells, and the a-priori
modal indicator."""
import numpy as np
import pytest

import oracle as O
import workloads as W

GAMMA = 1.4


def test_alpha_zero_is_bitwise_the_dg_operator():
    """Sec. 2.3: alpha = 0 recovers the DG scheme"""
    N = 4
    m = W.box_mesh(2, 0.0, 2 * np.pi, N, amp=0.05, rotate=True)
    X = m.points(W.lgl_points(N))
    U = W.random_smooth_state(X, 1, GAMMA, m.period)
    p = W.params(N, node_type=1, viscous=1, mu=1e-2, shock=1)
    o = O.Oracle(p, m)
    o.set_alpha(np.zeros(m.n_elems))
    p0 = dict(p)
    p0["shock_capturing"] = 0
    assert np.array_equal(o.rhs(U), O.Oracle(p0, m).rhs(U))


@pytest.mark.parametrize("alpha", [1.0, 0.37])
def test_fv_blend_freestream_and_conservation(alpha):
    N = 4
    m = W.box_mesh(3, 0.0, 2 * np.pi, N, amp=0.05, rotate=True)
    X = m.points(W.lgl_points(N))
    p = W.params(N, node_type=1, viscous=1, mu=1e-2, shock=1)
    o = O.Oracle(p, m)
    o.set_alpha(np.full(m.n_elems, alpha))
    Uf = W.uniform_state(X, 1.2, (0.3, -0.2, 0.5), 2.0, GAMMA)
    assert np.abs(o.rhs(Uf)).max() < 1e-10 * np.abs(Uf).max() / (2 * np.pi / 3)
    U = W.random_smooth_state(X, 3, GAMMA, m.period)
    R = o.rhs(U)
    b, g = o.basis(), o.geometry()
    wJ = g["J"] * np.einsum("k,j,i->kji", b["w"], b["w"], b["w"]).ravel()[None]
    tot = (R * wJ[None]).sum(axis=(1, 2))
    scale = np.abs(R * wJ[None]).sum(axis=(1, 2))
    assert np.all(np.abs(tot) < 1e-13 * scale)


def _minmod(a, b):
    return 0.0 if a * b <= 0 else np.sign(a) * min(abs(a), abs(b))


def _fv1d_rhs(q_nodes, xs, ws, h, K):
    """Brute-force 1-D reference: K elements of width h, LGL subcells of width
    w_l h/2, MUSCL-minmod on primitives inside each element (zero slope in the
    two boundary subcells), first-order LLF at element interfaces."""
    n = len(xs)
    N = n - 1
    xh = -1.0 + np.concatenate([[0.0], np.cumsum(ws)])

    def cons(q):
        rho, u, p = q
        return np.array([rho, rho * u, p / (GAMMA - 1) + 0.5 * rho * u * u])

    def flux(q):
        rho, u, p = q
        E = p / (GAMMA - 1) + 0.5 * rho * u * u
        return np.array([rho * u, rho * u * u + p, (E + p) * u])

    def llf(qL, qR):
        lam = max(abs(qL[1]) + np.sqrt(GAMMA * qL[2] / qL[0]), abs(qR[1]) + np.sqrt(GAMMA * qR[2] / qR[0]))
        return 0.5 * (flux(qL) + flux(qR)) - 0.5 * lam * (cons(qR) - cons(qL))

    out = np.zeros((K, n, 3))
    for e in range(K):
        q = q_nodes[e]
        sl = np.zeros((n, 3))
        for l in range(1, N):
            for v in range(3):
                sl[l, v] = _minmod((q[l, v] - q[l - 1, v]) / (xs[l] - xs[l - 1]),
                                   (q[l + 1, v] - q[l, v]) / (xs[l + 1] - xs[l]))
        F = np.zeros((n + 1, 3))
        for m_ in range(N):
            qL = q[m_] + sl[m_] * (xh[m_ + 1] - xs[m_])
            qR = q[m_ + 1] - sl[m_ + 1] * (xs[m_ + 1] - xh[m_ + 1])
            F[m_ + 1] = llf(qL, qR)
        F[0] = llf(q_nodes[(e - 1) % K][N], q[0])
        F[N + 1] = llf(q[N], q_nodes[(e + 1) % K][0])
        for l in range(n):
            out[e, l] = -(F[l + 1] - F[l]) / (ws[l] * h / 2)
    return out


def test_fv_subcells_match_bruteforce_1d_muscl():
    """alpha = 1, Euler, data varying along x only on a Cartesian mesh: the 3-D
    operator is the 1-D subcell finite-volume scheme"""
    N, K = 4, 4
    m = W.box_mesh((K, 1, 1), 0.0, 2 * np.pi, N)
    X = m.points(W.lgl_points(N))
    g = np.random.default_rng(0)
    xs = W.lgl_points(N)
    n = N + 1
    # random nodal values along x (strong jumps), constant along y and z
    qn = np.stack([1.0 + 0.5 * g.random((K, n)), 0.3 * g.standard_normal((K, n)),
                   1.0 + g.random((K, n))], axis=-1)
    ii = np.arange(n ** 3) % n
    rho = qn[:, ii, 0]
    u = qn[:, ii, 1]
    pp = qn[:, ii, 2]
    z = np.zeros_like(rho)
    U = np.stack([rho, rho * u, z, z, pp / (GAMMA - 1) + 0.5 * rho * u * u])
    p = W.params(N, node_type=1, riemann=0, viscous=0, shock=1)
    o = O.Oracle(p, m)
    o.set_alpha(np.ones(m.n_elems))
    R = o.rhs(U)
    ref = _fv1d_rhs(qn, o.basis()["x"], o.basis()["w"], 2 * np.pi / K, K)
    for e in range(K):
        for a in range(n ** 3):
            l = a % n
            assert np.allclose(R[[0, 1, 4], e, a], ref[e, l], rtol=1e-11, atol=1e-11)
            assert abs(R[2, e, a]) < 1e-12 and abs(R[3, e, a]) < 1e-12
    assert np.allclose(xs, o.basis()["x"], atol=1e-14)


def _alpha_bruteforce(eps, N, a=0.5, c=1.8, s=np.log(9999.0), amin=0.001, amax=1.0):
    """modal energies by solving V m = eps with numpy on the tensor Vandermonde"""
    x = W.lgl_points(N)
    n = N + 1
    V = np.zeros((n, n))
    for k in range(n):
        V[:, k] = np.sqrt((2 * k + 1) / 2) * np.polynomial.legendre.Legendre.basis(k)(x)
    V3 = np.kron(np.kron(V, V), V)  # index (k,j,i) with i fastest
    mcoef = np.linalg.solve(V3, eps).reshape(n, n, n)  # [c][b][a]
    m2 = mcoef ** 2
    tot = m2.sum()
    c1 = m2[:N, :N, :N].sum()
    c2 = m2[:N - 1, :N - 1, :N - 1].sum()
    E = max((tot - c1) / tot, (c1 - c2) / c1)
    T = a * 10 ** (-c * (N + 1) ** 0.25)
    al = 1.0 / (1.0 + np.exp(-(s / T) * (E - T)))
    if al < amin:
        al = 0.0
    elif al > 1 - amin:
        al = 1.0
    return min(al, amax)


def test_indicator_limits_and_bruteforce():
    N = 5
    m = W.box_mesh(2, -1.0, 1.0, N)
    X = m.points(W.lgl_points(N))
    p = W.params(N, node_type=1, viscous=0, shock=1, alpha_max=0.8)
    o = O.Oracle(p, m)
    # constant epsilon = rho p -> no high modes -> alpha = 0
    Uc = W.uniform_state(X, 1.0, (0.1, 0.0, 0.0), 1.0, GAMMA)
    assert o.indicator(Uc, 0) == 0.0
    # a nodal step -> strongly non-smooth -> alpha_max
    Us = W.blast_state(X, np.array([-0.5, -0.5, -0.5]), m.period, GAMMA, radius=0.45)
    assert o.indicator(Us, 0) == pytest.approx(0.8, abs=0)
    # intermediate values against the brute force
    hits = 0
    noise = np.random.default_rng(4).standard_normal(X.shape[1:])
    for amp in np.geomspace(1e-3, 0.3, 25):
        rho = 1.0 + amp * noise
        z = np.zeros_like(rho)
        U = np.stack([rho, z, z, z, 1.0 / (GAMMA - 1) + z])
        for e in range(m.n_elems):
            a_or = o.indicator(U, e)
            eps = rho[e] * 1.0
            a_bf = _alpha_bruteforce(eps, N, amax=0.8)
            assert a_or == pytest.approx(a_bf, rel=1e-9, abs=1e-12)
            hits += 0.0 < a_bf < 0.8
    assert hits > 0
