"""The synthetic observation generator (input recipe, not the method)."""
import numpy as np

from workloads import generate as g


def _data(refine, v=(1.0, 0.5, 0.25), faces=0b000011):
    n, M = (6, 6, 6), 8
    coef = g._Coefficient(np.random.default_rng(3), n, (1.0, 1.0, 1.0))
    src = g._Sources([[0.3, 0.4, 0.5]], [[0.7, 0.6, 0.4]], 0.15)
    return g._forward_fv(n, (1.0, 1.0, 1.0), M, 1.0, coef, v, src, faces, g.lattice_nodes(6, 2), refine=refine)


def test_sensor_data_converge_under_refinement():
    """The forward model behind the data (Section 4: data from a forward solve
    on a finer mesh) is second order in space and time: refining its mesh and
    step by 2 shrinks the change of the sensor values by about 4."""
    d = {r: _data(r) for r in (1, 2, 4, 8)}
    gaps = [np.linalg.norm(d[r] - d[2 * r]) / np.linalg.norm(d[2 * r]) for r in (1, 2, 4)]
    ratios = [gaps[k] / gaps[k + 1] for k in range(2)]
    assert all(3.0 <= q <= 5.0 for q in ratios), (gaps, ratios)
    assert gaps[-1] < 5e-3


def test_sensor_data_shape_and_initial_state():
    d = _data(2)
    assert d.shape == (9, 8) and np.all(d[0] == 0.0) and np.all(np.isfinite(d)) and np.abs(d[1:]).max() > 0


def test_configs_use_refined_data_mesh():
    """Every named configuration draws its data on a mesh refined twice."""
    prob, _ = g.make_problem("cube8x16")
    coarse = g._forward_fv(prob.n, prob.length, prob.M, prob.T, None, prob.v,
                           g._Sources([[0.25] * 3], [[0.75] * 3], 0.1, sin_intensity=False),
                           prob.dirichlet_faces, prob.sensor_node, refine=2)
    assert np.array_equal(coarse, prob.data_clean)
