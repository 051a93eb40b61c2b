"""The serving loop: continuous batching of independent solves.  Each result
must equal the same request run alone through a plain solver (bitwise: a
request's arithmetic does not depend on the rest of the batch), for FP64 and
the mixed form; a poisoned request fails alone; admission waits for memory."""
import copy
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _requests(n, seed, precision_mix=True):
    g = np.random.default_rng(seed)
    out = []
    for i in range(n):
        req = dict(id=i, K=int(g.integers(2, 5)), N=int(g.choice([3, 5, 7])), Ma=float(g.uniform(0.05, 0.3)),
                   Re=float(g.uniform(400, 1600)), steps=int(g.integers(2, 9)))
        prec = int(g.integers(0, 2)) if precision_mix else 0
        out.append((req, W.request_workload(req, precision=prec)))
    return out


def _alone(wl, dt):
    import paper_2404_12703_amd as P
    s = P.Solver(wl.params, wl.mesh)
    s.set_state(wl.U0)
    s.advance(wl.steps, dt)
    return s.state()


def _dt(wl):
    import paper_2404_12703_amd as P
    s = P.Solver(wl.params, wl.mesh)
    s.set_state(wl.U0)
    return s.stable_dt(0.9, 0.9)


def test_batched_equals_alone_bitwise():
    import paper_2404_12703_amd as P
    reqs = _requests(16, 0)
    _say("[server] 16 mixed requests")
    sv = P.Server(arena_bytes=2 << 30, hbm_budget=2 << 30, max_active=8)
    ids = []
    dts = []
    for req, wl in reqs:
        dt = _dt(wl)
        dts.append(dt)
        ids.append(sv.submit(wl.params, wl.mesh, wl.U0, wl.steps, dt, 0.0))
    sv.run(0)
    for (req, wl), rid, dt in zip(reqs, ids, dts):
        assert sv.poll(rid) == P.REQ_DONE
        U, tm = sv.fetch(rid)
        assert tm["t_done"] >= tm["t_admit"] >= 0.0
        assert np.array_equal(U, _alone(wl, dt)), (req, wl.params["precision"])


def test_batched_blast_equals_alone_bitwise():
    """Shock-capturing requests: workgroups with a blended element go to the
    blend pass, which walks every request's list in one launch."""
    import paper_2404_12703_amd as P
    _say("[server] blast requests, N = 5 and 3, FP64 and mixed")
    wls = []
    for K, N, seed, prec in ((4, 5, 1, 0), (5, 5, 2, 0), (4, 3, 3, 0), (6, 3, 4, 0), (4, 5, 5, 1)):
        wl = W.blast_workload(K=K, N=N, steps=3, seed=seed)
        wl.params = dict(wl.params, precision=prec)
        wls.append(wl)
    sv = P.Server(arena_bytes=1 << 30, hbm_budget=1 << 30, max_active=8)
    ids, dts, blended = [], [], []
    for wl in wls:
        s = P.Solver(wl.params, wl.mesh)
        s.set_state(wl.U0)
        dts.append(s.stable_dt(wl.cfl, wl.cfl))
        ids.append(sv.submit(wl.params, wl.mesh, wl.U0, wl.steps, dts[-1], 0.0))
    sv.run(0)
    for wl, rid, dt in zip(wls, ids, dts):
        assert sv.poll(rid) == P.REQ_DONE
        U, _ = sv.fetch(rid)
        s = P.Solver(wl.params, wl.mesh)
        s.set_state(wl.U0)
        s.advance(wl.steps, dt)
        assert np.array_equal(U, s.state()), (wl.mesh.n_elems, wl.params["N"], wl.params["precision"])
        blended.append(int(np.sum(s.alpha() > 0)))
    _say(f"[server] blended elements after 3 steps: {blended}")
    assert max(blended) > 0


def test_gauss_and_lobatto_requests_group_apart():
    """Requests of one degree with Gauss and with Gauss-Lobatto nodes run in
    separate groups (their kernels differ) in the same ticks; each result is
    still the request's own solve, bitwise."""
    import math
    import paper_2404_12703_amd as P
    _say("[server] N = 5 requests, Gauss and Lobatto nodes mixed")
    wls = []
    for i, (K, nodes) in enumerate(((3, 0), (3, 1), (4, 1), (4, 0))):
        mesh = W.box_mesh(K, 0.0, 2 * math.pi, 5)
        p = W.params(5, node_type=nodes, riemann=1, viscous=1, mu=1.0 / 800.0)
        X = mesh.points(W.lgl_points(5) if nodes else W.gl_points(5))
        wls.append(W.Workload("tgv_req", p, mesh, W.tgv_state(X, 0.1 + 0.05 * i, p["gamma"]), 4))
    sv = P.Server(arena_bytes=1 << 30, hbm_budget=1 << 30, max_active=8)
    ids, dts = [], []
    for wl in wls:
        dts.append(_dt(wl))
        ids.append(sv.submit(wl.params, wl.mesh, wl.U0, wl.steps, dts[-1], 0.0))
    sv.run(0)
    for wl, rid, dt in zip(wls, ids, dts):
        assert sv.poll(rid) == P.REQ_DONE
        U, _ = sv.fetch(rid)
        assert np.array_equal(U, _alone(wl, dt)), (wl.mesh.n_elems, wl.params["nodes"])


def test_poisoned_request_fails_alone_and_budget_binds():
    import paper_2404_12703_amd as P
    reqs = _requests(6, 1, precision_mix=False)
    _say("[server] poison + tight budget")
    need = max(P.workspace_bytes(wl.params, wl.mesh.n_elems) for _, wl in reqs)
    # room for about two requests at a time: admission must wait for retirements
    sv = P.Server(arena_bytes=64 << 20, hbm_budget=int(2.2 * need), max_active=8)
    ids, dts = [], []
    for i, (req, wl) in enumerate(reqs):
        U0 = wl.U0.copy()
        if i == 2:
            U0[0, 0, 0] = np.nan
        dt = _dt(wl)
        dts.append(dt)
        ids.append(sv.submit(wl.params, wl.mesh, U0, wl.steps, dt, 0.0))
    sv.run(0)
    for i, ((req, wl), rid, dt) in enumerate(zip(reqs, ids, dts)):
        if i == 2:
            assert sv.poll(rid) == P.REQ_FAILED
            continue
        assert sv.poll(rid) == P.REQ_DONE
        U, _ = sv.fetch(rid)
        assert np.array_equal(U, _alone(wl, dt))
    # a request that can never fit is refused at submission
    big = W.request_workload(dict(K=12, N=7, Ma=0.1, Re=1000.0, steps=1))
    with pytest.raises(P.DGError) as ei:
        sv.submit(big.params, big.mesh, big.U0, 1, 1e-3, 0.0)
    assert ei.value.code == -6


def test_arrivals_are_admitted_while_others_run():
    """requests arriving later join a running batch (continuous batching)"""
    import paper_2404_12703_amd as P
    reqs = _requests(6, 2, precision_mix=False)
    sv = P.Server(arena_bytes=1 << 30, hbm_budget=1 << 30, max_active=8)
    ids = []
    for i, (req, wl) in enumerate(reqs):
        # the early requests run long enough (about 0.1 s) for the late ones,
        # arriving 5 ms after the loop starts, to join them
        n = 300 if i < 3 else 40
        ids.append(sv.submit(wl.params, wl.mesh, wl.U0, n, _dt(wl), 0.0 if i < 3 else 0.005))
    sv.run(0)
    tms = [sv.fetch(r)[1] for r in ids]
    first_done = min(t["t_done"] for t in tms[:3])
    late_admit = min(t["t_admit"] for t in tms[3:])
    assert all(t["state"] == P.REQ_DONE for t in tms)
    assert late_admit < first_done  # a late arrival ran alongside the early ones


def test_cfl_step_and_broken_mesh():
    """dt < 0 asks for the stable step on the initial state (computed on the
    host while the request is prepared): the result matches a plain solver
    advanced with its own stable step.  A mesh whose neighbour table is not
    symmetric passes the size checks at submit, fails its set-up, and ends
    FAILED without disturbing the others."""
    import paper_2404_12703_amd as P
    reqs = _requests(4, 7, precision_mix=False)
    _say("[server] CFL step and a broken mesh")
    sv = P.Server(arena_bytes=1 << 30, hbm_budget=1 << 30, max_active=4)
    ids = [sv.submit(wl.params, wl.mesh, wl.U0, wl.steps, -0.9, 0.0) for _, wl in reqs]
    bad_req, bad = reqs[0]
    m = copy.copy(bad.mesh)
    m.nbr_elem = m.nbr_elem.copy()
    m.nbr_elem[0, 0] = 0  # element 0 names itself across its xi- face; its xi+ face disagrees
    bad_id = sv.submit(bad.params, m, bad.U0, bad.steps, -0.9, 0.0)
    sv.run(0)
    assert sv.poll(bad_id) == P.REQ_FAILED
    for (req, wl), rid in zip(reqs, ids):
        assert sv.poll(rid) == P.REQ_DONE
        U, _ = sv.fetch(rid)
        ref = _alone(wl, _dt(wl))
        assert np.linalg.norm(U - ref) <= 1e-12 * np.linalg.norm(ref), req


def test_cfl_step_with_sutherland_viscosity():
    """the host step of a CFL request takes Sutherland's viscosity at each
    node's temperature, as dg_stable_dt does on the device: served supersonic
    Taylor-Green requests (split form, Sutherland, blend, fourteen stages)
    with dt < 0 match plain solvers advanced with their own stable step"""
    import paper_2404_12703_amd as P
    wls = [W.compressible_tgv_workload(K=3, N=N, steps=3, curved=True, rotate=True) for N in (5, 7)]
    _say("[server] CFL step with Sutherland's law")
    sv = P.Server(arena_bytes=1 << 30, hbm_budget=1 << 30, max_active=4)
    ids = [sv.submit(wl.params, wl.mesh, wl.U0, wl.steps, -0.9, 0.0) for wl in wls]
    sv.run(0)
    for wl, rid in zip(wls, ids):
        assert sv.poll(rid) == P.REQ_DONE
        U, _ = sv.fetch(rid)
        ref = _alone(wl, _dt(wl))
        e = np.linalg.norm(U - ref) / np.linalg.norm(ref)
        _say(f"  N = {wl.params['N']}: served vs alone {e:.2e}")
        assert e <= 1e-12


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def test_served_request_matches_oracle():
    """a served FP64 request, batched with two others, against the oracle"""
    import oracle as O
    import paper_2404_12703_amd as P
    req = dict(id=0, K=3, N=5, Ma=0.2, Re=800.0, steps=4)
    wl = W.request_workload(req)
    o = O.Oracle(wl.params, wl.mesh)
    dt = o.stable_dt(wl.U0)
    sv = P.Server(arena_bytes=1 << 30, hbm_budget=1 << 30, max_active=4)
    rid = sv.submit(wl.params, wl.mesh, wl.U0, wl.steps, dt, 0.0)
    for i, n in ((1, 5), (2, 3)):
        w = W.request_workload(dict(id=i, K=2 + i, N=n, Ma=0.1, Re=1000.0, steps=3))
        sv.submit(w.params, w.mesh, w.U0, w.steps, -0.9, 0.0)
    sv.run(0)
    U, tm = sv.fetch(rid)
    Uo = o.advance(wl.U0, dt, wl.steps)
    assert _rel(U, Uo) <= 1e-12
    assert _rel(U - wl.U0, Uo - wl.U0) <= 1e-9


def test_large_state_leaves_through_several_staging_chunks():
    """a 20 MiB state (more than one 16 MiB staging slot) comes back whole"""
    import paper_2404_12703_amd as P
    req = dict(id=0, K=10, N=7, Ma=0.1, Re=1600.0, steps=1)
    wl = W.request_workload(req)
    dt = _dt(wl)
    sv = P.Server(arena_bytes=2 << 30, hbm_budget=2 << 30, max_active=2)
    rid = sv.submit(wl.params, wl.mesh, wl.U0, 1, dt, 0.0)
    small = W.request_workload(dict(id=1, K=2, N=3, Ma=0.1, Re=1000.0, steps=2))
    rid2 = sv.submit(small.params, small.mesh, small.U0, 2, _dt(small), 0.0)
    sv.run(0)
    U, _ = sv.fetch(rid)
    assert U.nbytes > 16 << 20
    assert np.array_equal(U, _alone(wl, dt))
    U2, _ = sv.fetch(rid2)
    assert np.array_equal(U2, _alone(small, _dt(small)))


def test_resident_geometry_is_shared_and_evicted():
    """requests of one mesh share its geometry block; under a tight budget the
    blocks of meshes no running request uses are evicted and uploaded again
    later; every result still equals its solve alone, bit for bit"""
    import paper_2404_12703_amd as P
    specs = [(3, 5), (4, 3), (3, 5), (4, 3), (2, 7), (3, 5), (2, 7), (4, 3)]
    wls = [W.request_workload(dict(id=i, K=K, N=N, Ma=0.1 + 0.02 * i, Re=900.0, steps=3))
           for i, (K, N) in enumerate(specs)]
    need = max(P.workspace_bytes(w.params, w.mesh.n_elems) for w in wls)
    # room for about two requests with their geometry: blocks must be evicted
    sv = P.Server(arena_bytes=3 * need + (64 << 20), hbm_budget=int(2.2 * need), max_active=8)
    ids, dts = [], []
    for w in wls:
        dt = _dt(w)
        dts.append(dt)
        ids.append(sv.submit(w.params, w.mesh, w.U0, w.steps, dt, 0.0))
    sv.run(0)
    st = sv.stats()
    _say(f"[server] geometry uploads {st['geometry_uploads']:.0f}, hits {st['geometry_hits']:.0f}")
    assert st["geometry_uploads"] + st["geometry_hits"] == len(wls)
    assert st["geometry_uploads"] >= 3  # one per distinct mesh at least
    for w, rid, dt in zip(wls, ids, dts):
        U, _ = sv.fetch(rid)
        assert np.array_equal(U, _alone(w, dt))
    # a roomy budget: each distinct mesh is uploaded once
    sv2 = P.Server(arena_bytes=1 << 30, hbm_budget=1 << 30, max_active=8)
    for w, dt in zip(wls, dts):
        sv2.submit(w.params, w.mesh, w.U0, w.steps, dt, 0.0)
    sv2.run(0)
    st2 = sv2.stats()
    assert st2["geometry_uploads"] == 3 and st2["geometry_hits"] == len(wls) - 3
