"""Pins of the oracle's metric terms (Sec. 2.2 "Mapping the Equations", curl
form) and of its geometric face matching (Sec. 2.2, unstructured orientation)."""
import numpy as np
import pytest

import oracle as O
import workloads as W


def test_cartesian_metrics_closed_form():
    K, N = 3, 4
    m = W.box_mesh(K, 0.0, 2 * np.pi, N)
    g = O.Oracle(W.params(N, viscous=0), m).geometry()
    h = 2 * np.pi / K
    Ja = g["Ja"]
    ref = (h / 2) ** 2 * np.eye(3)
    assert np.abs(Ja - ref[None, None]).max() < 1e-13
    assert np.abs(g["J"] - (h / 2) ** 3).max() < 1e-13
    # outward normals of a Cartesian cube: -+ e_d, surface element (h/2)^2
    nS = g["nS"]
    for f in range(6):
        d, s = f // 2, (1.0 if f % 2 else -1.0)
        assert np.abs(nS[:, f, :, d] - s * (h / 2) ** 2).max() < 1e-13


@pytest.mark.parametrize("nodes", [0, 1])
def test_curved_metric_identities_and_watertight_faces(nodes):
    N = 5
    m = W.box_mesh(3, 0.0, 2 * np.pi, N, amp=0.05, seed=0, rotate=True)
    o = O.Oracle(W.params(N, node_type=nodes, viscous=0), m)
    g = o.geometry()
    scale = np.abs(g["Ja"]).max()
    # discrete metric identity sum_i D_i (Ja^i) = 0
    assert np.abs(o.metric_identity()).max() < 1e-12 * scale
    # watertight: primary n*shat = - replica n*shat at coincident nodes, periodic faces included
    nS, fmap = g["nS"], g["fmap"]
    worst = 0.0
    for e in range(m.n_elems):
        for f in range(6):
            e2, f2 = m.nbr_elem[e, f], m.nbr_face[e, f]
            worst = max(worst, np.abs(nS[e, f] + nS[e2, f2][fmap[e, f]]).max())
    # round-off of two nested differentiations: about N^4 eps relative
    assert worst < 1e-12 * scale
    # volume of the periodic box is preserved by the periodic perturbation
    b = o.basis()
    wq = np.einsum("k,j,i->kji", b["w"], b["w"], b["w"]).ravel()
    vol = (g["J"] * wq[None]).sum()
    assert abs(vol - (2 * np.pi) ** 3) < 1e-8 * (2 * np.pi) ** 3
    assert g["J"].min() > 0


def test_geometric_matching_agrees_with_orientation_codes():
    """the oracle finds coincident face nodes by position; the generator's
    orientation codes must describe the same correspondence"""
    N = 3
    m = W.box_mesh(2, -1.0, 1.0, N, rotate=True, rot_seed=7)
    g = O.Oracle(W.params(N, viscous=0), m).geometry()
    n = N + 1
    for e in range(m.n_elems):
        for f in range(6):
            code = int(m.nbr_orient[e, f])
            for q in range(n):
                for p in range(n):
                    pp, qq = W.apply_orient(code, p, q, N)
                    assert g["fmap"][e, f, p + n * q] == pp + n * qq


def test_mismatched_connectivity_is_rejected():
    m = W.box_mesh(2, -1.0, 1.0, 2)
    m.nbr_elem = m.nbr_elem.copy()
    m.nbr_elem[0, 1] = 0  # face xi+ of element 0 does not touch its own xi+ face
    m.nbr_face = m.nbr_face.copy()
    m.nbr_face[0, 1] = 3
    with pytest.raises(ValueError):
        O.Oracle(W.params(2, viscous=0), m)


@pytest.mark.parametrize("K", [(3, 2, 1), (1, 1, 1)])
def test_faces_touching_their_own_periodic_image(K):
    """one element across the box: edge nodes of a face coincide with several
    neighbour nodes modulo the period; the matching must still find the one
    consistent correspondence (freestream and conservation hold)"""
    N = 4
    m = W.box_mesh(K, 0.0, 2 * np.pi, N, amp=0.05, rotate=True)
    o = O.Oracle(W.params(N, riemann=1, mu=1e-2), m)
    X = m.points(W.gl_points(N))
    U = W.uniform_state(X, 1.2, (0.3, -0.2, 0.5), 2.0, 1.4)
    assert np.abs(o.rhs(U)).max() < 1e-10 * 2.0 / np.pi
    U = W.random_smooth_state(X, 1, 1.4, m.period)
    R = o.rhs(U)
    b, g = o.basis(), o.geometry()
    wJ = g["J"] * np.einsum("k,j,i->kji", b["w"], b["w"], b["w"]).ravel()[None]
    assert np.all(np.abs((R * wJ[None]).sum(axis=(1, 2))) < 1e-13 * np.abs(R * wJ[None]).sum(axis=(1, 2)))
    # and the correspondence agrees with the generator's orientation codes
    n = N + 1
    for e in range(m.n_elems):
        for f in range(6):
            for q in range(n):
                for p in range(n):
                    pp, qq = W.apply_orient(int(m.nbr_orient[e, f]), p, q, N)
                    assert g["fmap"][e, f, p + n * q] == pp + n * qq


def test_ambiguous_face_matching_is_refused():
    """N = 1 on one element across the box: the two faces' four corners are all
    periodic images of each other, so no unique correspondence exists"""
    m = W.box_mesh(1, 0.0, 1.0, 1)
    with pytest.raises(ValueError):
        O.Oracle(W.params(1, viscous=0), m)
