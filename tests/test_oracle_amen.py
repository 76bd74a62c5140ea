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
    dinv = 1 / np.diag(Bm)
    x, it = amen.pcg(lambda v: Bm @ v, g, np.zeros(30), lambda v: dinv * v, 1e-12 * np.linalg.norm(g), 200)
    assert np.allclose(x, np.linalg.solve(Bm, g), rtol=1e-9)
    assert it <= 30 + 5


def _spd(rng, k):
    Q = rng.standard_normal((k, k))
    return Q @ Q.T + k * np.eye(k)


def _local_problem(seed, p=3, n=4, t=2, spd=False):
    """Interfaces L[p, 2, p], Rt[t, 2, t] and core A[2, n, n, 2] with symmetric slices; with
    spd=True the first term is a Kronecker product of SPD matrices and the second is small,
    so the local operator sum_{b,e} L_b (x) A_be (x) R_e is SPD."""
    rng = np.random.default_rng(seed)
    def sym(k):
        S = rng.standard_normal((k, k))
        return S + S.T
    L = np.zeros((p, 2, p))
    A = np.zeros((2, n, n, 2))
    Rt = np.zeros((t, 2, t))
    w = 0.01 if spd else 1.0
    L[:, 0, :] = _spd(rng, p) if spd else sym(p)
    L[:, 1, :] = w * sym(p)
    A[0, :, :, 0] = _spd(rng, n) if spd else sym(n)
    A[1, :, :, 1] = w * sym(n)
    A[0, :, :, 1] = A[1, :, :, 0] = w * sym(n)
    Rt[:, 0, :] = _spd(rng, t) if spd else sym(t)
    Rt[:, 1, :] = w * sym(t)
    return L, A, Rt


def _dense_local(L, A, Rt):
    p, n, t = L.shape[0], A.shape[1], Rt.shape[0]
    N = p * n * t
    B = np.zeros((N, N))
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1.0
        B[:, k] = amen.local_apply(L, A, e.reshape(p, n, t), Rt).reshape(-1)
    return B


def test_local_block_is_the_diagonal_mode_block_of_the_local_operator():
    L, A, Rt = _local_problem(1)
    p, n, t = L.shape[0], A.shape[1], Rt.shape[0]
    B = _dense_local(L, A, Rt).reshape(p, n, t, p, n, t)
    blk = amen.local_block(L, A, Rt)
    for a in range(p):
        for c in range(t):
            assert np.allclose(blk[a, c], B[a, :, c, a, :, c], rtol=1e-13, atol=1e-12)


def test_block_preconditioned_pcg_solves_spd_local_system():
    L, A, Rt = _local_problem(2, spd=True)
    p, n, t = L.shape[0], A.shape[1], Rt.shape[0]
    B = _dense_local(L, A, Rt)
    assert np.allclose(B, B.T) and np.linalg.eigvalsh(B).min() > 0
    g = np.random.default_rng(3).standard_normal(p * n * t)
    pre = amen.block_preconditioner(amen.local_block(L, A, Rt))
    x, it = amen.pcg(lambda v: amen.local_apply(L, A, v, Rt), g.reshape(p, n, t), np.zeros((p, n, t)), pre,
                     1e-12 * np.linalg.norm(g), 500)
    assert np.allclose(x.reshape(-1), np.linalg.solve(B, g), rtol=1e-8, atol=1e-10)
    # with one interface index on each side the whole operator is one block: the
    # preconditioner is its inverse and CG stops after one iteration
    L1, A1, R1 = _local_problem(4, p=1, t=1, spd=True)
    g1 = np.random.default_rng(5).standard_normal((1, A1.shape[1], 1))
    x1, it1 = amen.pcg(lambda v: amen.local_apply(L1, A1, v, R1), g1, np.zeros_like(g1),
                       amen.block_preconditioner(amen.local_block(L1, A1, R1)), 1e-10 * np.linalg.norm(g1), 50)
    assert it1 == 1
    assert np.allclose(x1.reshape(-1), np.linalg.solve(_dense_local(L1, A1, R1), g1.reshape(-1)), rtol=1e-10)
