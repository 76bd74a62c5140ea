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


def test_scaling_and_superposition():
    """u(sE) = u(E)/s (A scales with E, the loads do not), and solutions of summed loads add."""
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
    mirror = coords.copy()
    mirror[:, 1] = n - 1 - coords[:, 1]
    for c, sign in ((0, 1), (1, -1), (2, 1)):
        v = tt.tt_eval(X, qtt.qtt_dof_index(3, 3, c, coords))
        w = tt.tt_eval(X, qtt.qtt_dof_index(3, 3, c, mirror))
        assert np.abs(v - sign * w).max() <= 1e-8 * np.abs(u).max()


def _ranks(cores):
    return [C.shape[0] for C in cores] + [cores[-1].shape[2]]


@pytest.mark.parametrize("prob,cap", [
    (dict(dim=2, level=3, E=1.0, nu=0.3, clamp=[(0, 0)], tractions=[(0, 1, [1.0, 0.0])]), 4),
    (dict(dim=2, level=4, E=2.0, nu=0.35, clamp=[(0, 0)], body_force=[0.2, -1.0]), 6),
    (dict(dim=3, level=2, E=1.0, nu=0.3, clamp=[(0, 0)], body_force=[0.0, 0.0, -1.0]), 5),
    (dict(dim=3, level=3, E=1.0, nu=0.3, clamp=[(2, 0)], tractions=[(2, 1, [0.0, 0.0, -1.0])]), 7),
])
def test_rank_capped_sweep_keeps_cap_and_lowers_energy(prob, cap):
    """A binding rank cap: every bond stays <= cap after every step (truncation at the cap
    and the clipped enrichment), the cap is reached, and no local solve raises the energy
    J(x) = x^T A x / 2 - b^T x of the whole iterate (A, b: the sparse element assembly,
    permuted to the QTT order; each local solve is a Galerkin step on a subspace that holds
    the current iterate, and CG does not raise the energy)."""
    A, b, grid, _ = fem.build_system(prob)
    D, d = prob["dim"], prob["level"]
    Ap = qtt.matrix_to_qtt_order(A, D, d).tocsr()
    bp = qtt.to_qtt_order(b, D, d)

    def energy(cores):
        x = tt.tt_full(cores)
        return 0.5 * x @ (Ap @ x) - bp @ x

    seen = dict(max_rank=0, solves=0, sweeps=0)
    last = {}

    def observe(event, k, cores):
        r = _ranks(cores)
        assert max(r) <= cap, (event, k, r)
        seen["max_rank"] = max(seen["max_rank"], max(r))
        if event == "before_solve":
            last["J"] = energy(cores)
        elif event == "after_solve":
            J = energy(cores)
            assert J <= last["J"] + 1e-12 * abs(last["J"]), (k, J, last["J"])
            seen["solves"] += 1
        else:
            seen["sweeps"] += 1

    Aq = qtt.assemble_operator(prob)
    bq = qtt.assemble_load(prob)
    X, st = amen.amen_solve(Aq, bq, amen.Options(tol=1e-12, rank_cap=cap, max_sweeps=6), observe=observe)
    assert seen["max_rank"] == cap  # the cap binds
    assert seen["sweeps"] == st.sweeps == 6 and seen["solves"] == 6 * (d + 1)
    assert max(_ranks(X)) <= cap
    # the capped iterate is still a good approximation: its energy lies above the
    # exact discrete minimum and within a few per cent of it
    u = fem.direct_solve(A, b)
    Jmin = 0.5 * u @ (A @ u) - b @ u
    Jx = energy(X)
    assert Jmin - 1e-12 * abs(Jmin) <= Jx <= Jmin + 0.05 * abs(Jmin)
