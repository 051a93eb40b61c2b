"""The allocation-free dissipation entry point (dg_dissipation_noalloc)
against dg_dissipation through the C ABI: the same rates (Sec. 5.2) on two
calls in a row, the second on a smaller mesh, so the static device array
still holds the first call's larger contents; and the size limit."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _solver(wl):
    import paper_2404_12703_amd as P
    s = P.Solver(wl.params, wl.mesh)
    s.set_state(wl.U0, 0.0)
    return s


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_dissipation_two_calls(precision):
    big = W.tgv_workload(K=4, N=5, rotate=True, precision=precision)
    small = W.tgv_workload(K=3, N=5, rotate=True, precision=precision)
    sb, ss = _solver(big), _solver(small)
    for s in (sb, ss):
        ref = s.dissipation()
        got = s.dissipation_noalloc()
        assert np.all(np.isfinite(got))
        assert np.abs(got - ref).max() <= 1e-13 * abs(ref[0])
        assert np.array_equal(got, ref)  # the same kernels in the same order
    # and again on the larger mesh after the smaller one
    assert np.array_equal(sb.dissipation_noalloc(), sb.dissipation())


def test_noalloc_rejects_meshes_beyond_its_array():
    import paper_2404_12703_amd as P
    m = W.box_mesh(65, 0.0, 2 * np.pi, 1)
    p = W.params(1, riemann=1, mu=1e-3)
    U = W.tgv_state(m.points(W.gl_points(1)), 0.1, 1.4)
    s = P.Solver(p, m)
    s.set_state(U, 0.0)
    with pytest.raises(P.DGError) as ei:
        s.dissipation_noalloc()
    assert ei.value.code == -1 and "262144" in str(ei.value)
    assert np.all(np.isfinite(s.dissipation()))
