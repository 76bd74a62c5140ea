"""Pins of the oracle AMEn sweep (O2) against the sparse direct solve and invariants."""
import numpy as np
import pytest

from oracle import amen, fem, qtt, tt


def _solve_both(prob, **opt):
    A, b, grid, info = fem.build_system(prob)
    u = fem.direct_solve(A, b)
    Aq = qtt.assemble_operator(prob)
    bq = qtt.assemble_load(prob)
    X, st = amen.amen_solve(Aq, bq, amen.Options(**opt))
    return X, st, qtt.to_qtt_order(u, prob["dim"], prob["level"]), grid


@pytest.mark.parametrize("prob", [
    dict(dim=2, level=3, E=1.0, nu=0.3, clamp=[(0, 0)], tractions=[(0, 1, [1.0, 0.0])]),
    dict(dim=2, level=4, E=3.0, nu=0.2, clamp=[(0, 0)], body_force=[0.0, -1.0]),
    dict(dim=3, level=2, E=1.0, nu=0.3, clamp=[(0, 0)], body_force=[0.0, 0.0, -1.0]),
    dict(dim=3, level=3, E=1.0, nu=0.45, clamp=[(2, 0)], tractions=[(2, 1, [0.0, 0.0, -1.0])]),
])
def test_unconstrained_amen_equals_direct_solve(prob):
    X, st, u, _ = _solve_both(prob, tol=1e-10, rank_cap=256)
    assert st.max_res[-1] <= 1e-10
    assert np.linalg.norm(tt.tt_full(X) - u) <= 1e-8 * np.linalg.norm(u)


def test_truncation_rank_rule():
    s = np.array([10.0, 1.0, 1e-3, 1e-6])
    assert amen.truncation_rank(s, 1e-9, 10) == 4
    assert amen.truncation_rank(s, 1e-5, 10) == 3
    assert amen.truncation_rank(s, 1e-3, 10) == 2
    assert amen.truncation_rank(s, 1e-3, 1) == 1
    assert amen.truncation_rank(np.zeros(3), 1e-3, 5) == 1


def test_pcg_solves_spd_system():
    r = np.random.default_rng(0)
    Q = r.standard_normal((30, 30))
    Bm = Q @ Q.T + 30 * np.eye(30)
    g = r.standard_normal(30)
    x, it = amen.pcg(lambda v: Bm @ v, g, np.zeros(30), 1 / np.diag(Bm), 1e-12 * np.linalg.norm(g), 200)
    assert np.allclose(x, np.linalg.solve(Bm, g), rtol=1e-9)
    assert it <= 30 + 5


def test_scaling_and_superposition():
    base = dict(dim=2, level=3, nu=0.3, clamp=[(0, 0)])
    p1 = dict(base, E=1.0, tractions=[(0, 1, [1.0, 0.0])])
    p2 = dict(base, E=4.0, tractions=[(0, 1, [1.0, 0.0])])
    X1, *_ = _solve_both(p1, tol=1e-11, rank_cap=64)
    X2, *_ = _solve_both(p2, tol=1e-11, rank_cap=64)
    assert np.linalg.norm(tt.tt_full(X1) - 4.0 * tt.tt_full(X2)) <= 1e-8 * np.linalg.norm(tt.tt_full(X1))
    p3 = dict(base, E=1.0, body_force=[0.0, -1.0])
    p4 = dict(base, E=1.0, tractions=[(0, 1, [1.0, 0.0])], body_force=[0.0, -1.0])
    X3, *_ = _solve_both(p3, tol=1e-11, rank_cap=64)
    X4, *_ = _solve_both(p4, tol=1e-11, rank_cap=64)
    lhs = tt.tt_full(X4)
    assert np.linalg.norm(lhs - tt.tt_full(X1) - tt.tt_full(X3)) <= 1e-8 * np.linalg.norm(lhs)


def test_mirror_symmetry_body_force_cube():
    """Clamp x = 0, load along -z: u_x, u_z even and u_y odd under y -> 1 - y."""
    prob = dict(dim=3, level=3, E=1.0, nu=0.3, clamp=[(0, 0)], body_force=[0.0, 0.0, -1.0])
    X, st, u, grid = _solve_both(prob, tol=1e-10, rank_cap=128)
    n = grid.n
    coords = np.array([[i, j, k] for i in range(n) for j in range(n) for k in range(n)])
    mirror = coords.copy(); mirror[:, 1] = n - 1 - coords[:, 1]
    for c, sign in ((0, 1), (1, -1), (2, 1)):
        v = tt.tt_eval(X, qtt.qtt_dof_index(3, 3, c, coords))
        w = tt.tt_eval(X, qtt.qtt_dof_index(3, 3, c, mirror))
        assert np.abs(v - sign * w).max() <= 1e-8 * np.abs(u).max()
