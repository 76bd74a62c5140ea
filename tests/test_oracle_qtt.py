"""The oracle's QTT operator and load equal the sparse element-by-element assembly."""
import numpy as np
import pytest

from oracle import fem, qtt, tt
from paper_2501_12151_amd import workloads

CASES = [
    dict(dim=2, level=2, E=1.0, nu=0.3, clamp=[(0, 0)], tractions=[(0, 1, [1.0, 0.0])]),
    dict(dim=2, level=3, E=2.0, nu=0.25, clamp=[(0, 0), (1, 1)], body_force=[0.3, -1.0], extent=[2.0, 1.0]),
    dict(dim=2, level=4, E=1.0, nu=0.33, plane_stress=True, clamp=[(0, 0)], body_force=[0.0, -1.0], extent=[20.0, 1.0]),
    dict(dim=2, level=3, E=1.0, nu=0.3, clamp=[(0, 0), (0, 1), (1, 0), (1, 1)], manufactured_c=[0.7, -0.4]),
    dict(dim=3, level=2, E=1.0, nu=0.3, clamp=[(0, 0)], body_force=[0.0, 0.0, -1.0]),
    dict(dim=3, level=3, E=0.5, nu=0.4, clamp=[(2, 0)], tractions=[(2, 1, [0.0, 0.0, -1.0]), (0, 1, [0.3, 0.2, 0.1])]),
    dict(dim=3, level=3, E=1.0, nu=0.3, clamp=[(2, 0)], tractions=[(2, 1, [0.0, 0.0, -1.0])],
         layered_E=(2, [1.0, 1.0, 10.0, 10.0, 1.0, 1.0, 10.0])),
    dict(dim=3, level=2, E=1.0, nu=0.3, clamp=[(a, s) for a in range(3) for s in (0, 1)], manufactured_c=[0.5, 1.0, -0.3]),
    # anisotropic materials (constant Voigt stiffness), one also layered
    dict(dim=2, level=3, E=1.0, nu=0.3, clamp=[(0, 0)], tractions=[(0, 1, [1.0, 0.3])],
         stiffness_voigt=workloads.random_anisotropic_voigt(2, 1), extent=[2.0, 1.0]),
    dict(dim=3, level=2, E=1.0, nu=0.3, clamp=[(2, 0)], body_force=[0.1, 0.0, -1.0],
         stiffness_voigt=workloads.random_anisotropic_voigt(3, 2)),
    dict(dim=3, level=3, E=2.0, nu=0.3, clamp=[(2, 0)], tractions=[(2, 1, [0.0, 0.0, -1.0])],
         layered_E=(2, [2.0, 2.0, 20.0, 20.0, 2.0, 2.0, 20.0]), stiffness_voigt=workloads.orthotropic_voigt(3, 1.0, 3.0, 0.5)),
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("component_first", [False, True])
def test_qtt_operator_and_load_equal_sparse(case, component_first):
    prob = CASES[case]
    A, b, grid, info = fem.build_system(prob)
    D, d = prob["dim"], prob["level"]
    Aq = qtt.assemble_operator(prob, component_first=component_first)
    bq = qtt.assemble_load(prob, component_first=component_first)
    Ad = tt.mpo_full(Aq)
    Ap = qtt.matrix_to_qtt_order(A, D, d, component_first).toarray()
    assert np.abs(Ad - Ap).max() <= 1e-12 * np.abs(Ap).max()
    bp = qtt.to_qtt_order(b, D, d, component_first)
    assert np.abs(tt.tt_full(bq) - bp).max() <= 1e-12 * np.abs(bp).max()
    # mode layout: component core (dim D) first or last, level cores of dim 2^D
    modes = [C.shape[1] for C in Aq]
    want = [2 ** D] * d
    want = [D] + want if component_first else want + [D]
    assert modes == want


def test_dof_index_matches_flattening():
    D, d = 3, 2
    q = qtt.natural_to_qtt(D, d)
    assert sorted(q) == list(range(D * 4 ** 3))
    grid = fem.Grid(D, d)
    rng = np.random.default_rng(0)
    v = rng.standard_normal(grid.n_dofs)
    vq = qtt.to_qtt_order(v, D, d)
    cores = tt.tt_svd(vq, [8, 8, 3])
    coords = np.array([[0, 1, 2], [3, 3, 0], [1, 0, 3]])
    for c in range(D):
        idx = qtt.qtt_dof_index(D, d, c, coords)
        nat = c * grid.n_nodes + grid.node_index(coords)
        assert np.allclose(tt.tt_eval(cores, idx), v[nat])


def test_operator_ranks_component_last_smaller():
    prob = dict(dim=2, level=5, E=1.0, nu=0.3, clamp=[(0, 0)], tractions=[(0, 1, [1.0, 0.0])])
    last = qtt.assemble_operator(prob)
    first = qtt.assemble_operator(prob, component_first=True)
    assert max(C.shape[3] for C in last) <= 25
    assert max(C.shape[3] for C in first) > max(C.shape[3] for C in last)
