"""Pins of the sparse FEM oracle (O1) against facts fixed outside it."""
import itertools
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_lame_closed_form():
    lam, mu = fem.lame(1.0, 0.3)
    assert lam == pytest.approx(0.3 / (1.3 * 0.4), rel=1e-15)
    assert mu == pytest.approx(1.0 / 2.6, rel=1e-15)
    lps, mps = fem.lame(68e9, 0.33, plane_stress=True)
    assert lps == pytest.approx(68e9 * 0.33 / (1 - 0.33 ** 2), rel=1e-14)
    assert mps == pytest.approx(68e9 / 2.66, rel=1e-14)


def _load_q4(nu, E):
    coef, P = {}, []
    for line in open(os.path.join(GOLD, "q4_plane_stress_element.txt")):
        if line.startswith("coef"):
            _, i, c0, c1 = line.split()
            coef[int(i)] = float(Fraction(c0)) + float(Fraction(c1)) * nu
        elif line.startswith("P"):
            P.append([int(v) for v in line.split()[1:]])
    return E / (1 - nu ** 2) * np.array([[coef[v] for v in row] for row in P])


@pytest.mark.parametrize("nu", [0.3, 0.33, 0.45])
def test_element_matches_textbook_q4(nu):
    """The quadrature element equals Sigmund's closed-form Q4 plane-stress matrix.

    The textbook orders dofs node by node around the element; we search the
    node orders (cyclic, either orientation, either start) and the two axis
    reflections, and require an exact match for one of them.
    """
    E = 2.5
    lam, mu = fem.lame(E, nu, plane_stress=True)
    Ke, _ = fem.element_matrices(2, 0.7, lam, mu)  # square element; side does not matter in 2D
    KE = _load_q4(nu, E)
    bits = fem.corner_bits(2)  # our corners: (x bit, y bit), x most significant
    best = np.inf
    for perm in itertools.permutations(range(4)):
        for sx, sy in itertools.product((1, -1), repeat=2):
            idx, sgn = [], []
            for node in perm:
                idx += [0 * 4 + node, 1 * 4 + node]
                sgn += [sx, sy]
            T = np.array(sgn)[:, None] * Ke[np.ix_(idx, idx)] * np.array(sgn)[None, :]
            best = min(best, np.abs(T - KE).max())
    assert best < 1e-12 * np.abs(KE).max()
    # the textbook matrix also fixes the eigenvalues (order free)
    assert np.allclose(np.sort(np.linalg.eigvalsh(Ke)), np.sort(np.linalg.eigvalsh(KE)), atol=1e-12)
    del bits


def test_1d_element_closed_forms():
    h = 0.37
    lam, mu = 0.8, 0.6
    Ke, Me = fem.element_matrices(1, h, lam, mu)
    assert np.allclose(Ke, (lam + 2 * mu) / h * np.array([[1, -1], [-1, 1]]), rtol=1e-14)
    assert np.allclose(Me, h / 6 * np.array([[2, 1], [1, 2]]), rtol=1e-14)


@pytest.mark.parametrize("D", [2, 3])
def test_element_equals_kronecker_form(D):
    """Element stiffness = lambda D_ab + mu D_ba + mu delta_ab sum_c D_cc with 1D closed forms."""
    h = np.array([0.3, 0.5, 0.7])[:D]
    lam, mu = 1.3, 0.45
    Ke, Me = fem.element_matrices(D, h, lam, mu)
    S = [1 / h[a] * np.array([[1, -1], [-1, 1]]) for a in range(D)]
    M = [h[a] / 6 * np.array([[2, 1], [1, 2]]) for a in range(D)]
    G = [0.5 * np.array([[-1, -1], [1, 1]]) for a in range(D)]  # int phi_p' phi_q

    def atom(a, b):
        out = np.ones((1, 1))
        for c in range(D):
            if a == b:
                F = S[c] if c == a else M[c]
            else:
                F = G[c] if c == a else (G[c].T if c == b else M[c])
            out = np.kron(out, F)
        return out

    nc = 2 ** D
    for a in range(D):
        for b in range(D):
            ref = lam * atom(a, b) + mu * atom(b, a)
            if a == b:
                ref = ref + mu * sum(atom(c, c) for c in range(D))
            assert np.allclose(Ke[a * nc:(a + 1) * nc, b * nc:(b + 1) * nc], ref, rtol=1e-13, atol=1e-14)
    Mref = np.ones((1, 1))
    for c in range(D):
        Mref = np.kron(Mref, M[c])
    assert np.allclose(Me, Mref, rtol=1e-13)


def _rigid_modes(grid):
    x = grid.node_coords()
    D, nn = grid.D, grid.n_nodes
    modes = []
    for a in range(D):
        v = np.zeros((D, nn)); v[a] = 1.0
        modes.append(v.reshape(-1))
    for a, b in itertools.combinations(range(D), 2):
        v = np.zeros((D, nn)); v[a] = -x[:, b]; v[b] = x[:, a]
        modes.append(v.reshape(-1))
    return modes


@pytest.mark.parametrize("D,d", [(2, 3), (2, 4), (3, 2), (3, 3)])
def test_stiffness_symmetric_and_rigid_null_space(D, d):
    grid = fem.Grid(D, d, extent=[2.0, 1.0, 0.5][:D])
    K, M = fem.assemble(grid, 0.7, 0.4)
    nK = abs(K).max()
    assert abs(K - K.T).max() <= 1e-15 * nK  # symmetric up to quadrature summation order
    modes = _rigid_modes(grid)
    assert len(modes) == (3 if D == 2 else 6)
    for v in modes:
        assert np.abs(K @ v).max() <= 1e-13 * nK * np.abs(v).max() * 10


@pytest.mark.parametrize("D,d", [(2, 4), (3, 3)])
def test_patch_test_linear_field(D, d):
    """A linear displacement field has constant stress: interior nodal forces vanish."""
    grid = fem.Grid(D, d)
    K, _ = fem.assemble(grid, 1.1, 0.6)
    x = grid.node_coords()
    rng = np.random.default_rng(3)
    Gm = rng.standard_normal((D, D))
    c = rng.standard_normal(D)
    u = (x @ Gm.T + c).T.reshape(-1)
    f = (K @ u).reshape(D, -1)
    coords = np.array(list(itertools.product(range(grid.n), repeat=D)))
    interior = np.all((coords > 0) & (coords < grid.n - 1), axis=1)
    assert np.abs(f[:, interior]).max() <= 1e-12 * np.abs(K).max() * np.abs(u).max()
    assert np.abs(f[:, ~interior]).max() > 1e-3  # boundary tractions do not vanish


@pytest.mark.parametrize("D,d", [(2, 3), (3, 2)])
def test_load_totals(D, d):
    ext = np.array([2.0, 1.5, 0.5])[:D]
    grid = fem.Grid(D, d, extent=ext)
    K, M = fem.assemble(grid, 1.0, 1.0)
    f = np.array([0.3, -1.2, 2.0])[:D]
    b = fem.body_load(grid, M, np.repeat(f[:, None], grid.n_nodes, axis=1))
    tot = b.reshape(D, -1).sum(axis=1)
    assert np.allclose(tot, f * np.prod(ext), rtol=1e-13)
    t = np.array([1.0, -0.5, 0.25])[:D]
    bt = fem.traction_load(grid, 0, 1, t)
    area = np.prod(ext[1:])
    assert np.allclose(bt.reshape(D, -1).sum(axis=1), t * area, rtol=1e-13)
    # traction sits on the face x = L only
    on = np.zeros(grid.n_nodes, bool); on[fem.face_nodes(grid, 0, 1)] = True
    assert np.all(bt.reshape(D, -1)[:, ~on] == 0)


@pytest.mark.parametrize("D", [2, 3])
def test_manufactured_force_finite_difference(D):
    """f = -div sigma(u*) checked by central differences of u* (independent of the closed form)."""
    lam, mu = 0.9, 0.35
    c = np.array([0.4, -1.1, 0.7])[:D]
    rng = np.random.default_rng(7)
    pts = rng.uniform(0.1, 0.9, size=(5, D))
    hh = 1e-3

    def sigma(x):
        # gradient of u* by central differences
        Gd = np.zeros((D, D))
        for j in range(D):
            e = np.zeros(D); e[j] = hh
            Gd[:, j] = (fem.manufactured_u((x + e)[None], c)[:, 0] - fem.manufactured_u((x - e)[None], c)[:, 0]) / (2 * hh)
        eps = 0.5 * (Gd + Gd.T)
        return lam * np.trace(eps) * np.eye(D) + 2 * mu * eps

    for x in pts:
        div = np.zeros(D)
        for j in range(D):
            e = np.zeros(D); e[j] = hh
            div += (sigma(x + e)[:, j] - sigma(x - e)[:, j]) / (2 * hh)
        f = fem.manufactured_f(x[None], c, lam, mu)[:, 0]
        assert np.allclose(f, -div, rtol=1e-4, atol=1e-4)


def _manufactured_problem(D, d):
    faces = [(a, s) for a in range(D) for s in (0, 1)]
    return dict(dim=D, level=d, E=1.0, nu=0.3, clamp=faces, manufactured_c=[0.5, -1.0, 0.8][:D])


@pytest.mark.parametrize("D,levels", [(2, [3, 4, 5, 6]), (3, [3, 4])])
def test_manufactured_convergence_second_order(D, levels):
    errs = []
    for d in levels:
        A, b, grid, info = fem.build_system(_manufactured_problem(D, d))
        u = fem.direct_solve(A, b)
        assert np.linalg.norm(A @ u - b) <= 1e-10 * np.linalg.norm(b)
        ustar = fem.manufactured_u(grid.node_coords(), [0.5, -1.0, 0.8][:D]).reshape(-1)
        errs.append(np.linalg.norm(u - ustar) / np.linalg.norm(ustar))
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(ratios > 3.0) and np.all(ratios < 5.0), (errs, ratios)


def test_bc_system_is_spd_and_alpha_free():
    prob = dict(dim=2, level=3, E=1.0, nu=0.3, clamp=[(0, 0)], tractions=[(0, 1, [1.0, 0.0])])
    A, b, grid, info = fem.build_system(prob)
    Ad = A.toarray()
    np.linalg.cholesky(Ad)  # SPD
    u1 = fem.direct_solve(A, b)
    A2, b2 = fem.apply_dirichlet(info["K"], info["b_raw"], info["mask"], 17.0 * info["alpha"])
    u2 = fem.direct_solve(A2, b2)
    assert np.allclose(u1, u2, rtol=1e-11, atol=1e-14)
    assert np.all(u1[~info["mask"]] == 0.0)
    # energy identity 1/2 u^T A u = 1/2 b^T u at the solution
    assert u1 @ (A @ u1) == pytest.approx(b @ u1, rel=1e-12)
    assert spla.norm(A - A.T) <= 1e-15 * spla.norm(A)


def test_cantilever_tip_deflection_approaches_euler_bernoulli():
    """Sec. 6: 20 m x 1 m aluminium plate in plane stress, clamped at x = 0, under its own
    weight.  The discrete tip deflection converges to the Euler-Bernoulli value
    3 rho g L_x^4 / (2 E L_y^2) (the paper's closed form; shear deformation adds a few
    tenths of a percent at this slenderness), rising monotonically as the grid refines, and
    the strain energy u^T K u / 2 equals b^T u / 2 at every level."""
    rho, g, E, nu, Lx, Ly = 2700.0, 9.81, 68e9, 0.33, 20.0, 1.0
    ymax = 3 * rho * g * Lx ** 4 / (2 * E * Ly ** 2)
    ratios, energies = [], []
    for d in (5, 6, 7, 8):
        prob = dict(dim=2, level=d, E=E, nu=nu, plane_stress=True, extent=[Lx, Ly], clamp=[(0, 0)],
                    body_force=[0.0, -rho * g])
        A, b, grid, info = fem.build_system(prob)
        u = fem.direct_solve(A, b)
        uy = u[grid.n_nodes:].reshape(grid.n, grid.n)
        ratios.append(np.abs(uy).max() / ymax)
        # the tip (x = L_x) carries the largest deflection
        assert np.abs(uy[-1]).max() == np.abs(uy).max()
        e_k = 0.5 * u @ (info["K"] @ u)
        energies.append(e_k)
        assert e_k == pytest.approx(0.5 * b @ u, rel=1e-6)  # up to the direct solve's residual (kappa ~ 1e9)
    assert np.all(np.diff(ratios) > 0) and np.all(np.diff(energies) > 0)
    assert abs(ratios[-1] - 1.0) <= 5e-3, ratios


# ----------------------------------------------------------------------------- anisotropic material

def _random_spd_voigt(D, seed):
    rng = np.random.default_rng(seed)
    nv = 3 if D == 2 else 6
    B = rng.standard_normal((nv, nv))
    return B @ B.T / nv + np.eye(nv)


@pytest.mark.parametrize("D", [2, 3])
def test_isotropic_voigt_matrix_reproduces_isotropic_element(D):
    """The tensor from the isotropic Voigt matrix (lambda + 2 mu, lambda, mu) gives the element
    of sigma = lambda tr(eps) I + 2 mu eps exactly."""
    lam, mu = fem.lame(1.7, 0.27)
    nv = 3 if D == 2 else 6
    Cv = np.zeros((nv, nv))
    Cv[:D, :D] = lam
    for i in range(D):
        Cv[i, i] = lam + 2 * mu
    for k in range(D, nv):
        Cv[k, k] = mu
    C = fem.voigt_to_tensor(Cv, D)
    assert np.abs(C - fem.isotropic_tensor(lam, mu, D)).max() == 0.0
    h = [0.3, 0.7, 0.2][:D]
    K1, _ = fem.element_matrices(D, h, lam, mu)
    K2, _ = fem.element_matrices(D, h, 0.0, 0.0, C)
    assert np.abs(K1 - K2).max() <= 1e-14 * np.abs(K1).max()


@pytest.mark.parametrize("D,d", [(2, 3), (3, 2)])
def test_anisotropic_stiffness_symmetric_with_rigid_null_space(D, d):
    C = fem.voigt_to_tensor(_random_spd_voigt(D, 3), D)
    g = fem.Grid(D, d, [1.0, 2.0, 0.5][:D])
    K, _ = fem.assemble(g, 0.0, 0.0, None, C)
    assert abs(K - K.T).max() <= 1e-14 * abs(K).max()
    x = g.node_coords()
    modes = [np.concatenate([np.full(g.n_nodes, float(a == c)) for c in range(D)]) for a in range(D)]
    rots = [(0, 1)] if D == 2 else [(0, 1), (0, 2), (1, 2)]
    for i, j in rots:  # u_i = -x_j, u_j = x_i
        u = np.zeros((D, g.n_nodes))
        u[i], u[j] = -x[:, j], x[:, i]
        modes.append(u.reshape(-1))
    for m in modes:
        assert np.abs(K @ m).max() <= 1e-13 * abs(K).max() * np.abs(m).max()
    # positive definite once clamped
    A, _ = fem.apply_dirichlet(K, np.zeros(g.n_dofs), fem.clamp_mask(g, [(0, 0)]), 1.0)
    np.linalg.cholesky(A.toarray())


def linear_field_problem(D, d, Cv, grad):
    """Clamped at x = 0, with the face tractions sigma . n of the constant stress of
    u_i = grad[i] x: the exact solution is that linear field (Q1 reproduces it exactly)."""
    C = fem.voigt_to_tensor(Cv, D)
    Gm = np.zeros((D, D))
    Gm[:, 0] = grad
    sig = np.einsum("ijkl,kl->ij", C, 0.5 * (Gm + Gm.T))
    tr = [(0, 1, list(sig[:, 0]))]
    for a in range(1, D):
        tr.append((a, 0, list(-sig[:, a])))
        tr.append((a, 1, list(sig[:, a])))
    return dict(dim=D, level=d, E=1.0, nu=0.3, clamp=[(0, 0)], tractions=tr,
                stiffness_voigt=np.asarray(Cv).tolist())


@pytest.mark.parametrize("D,d", [(2, 4), (3, 3)])
def test_anisotropic_patch_problem_reproduces_linear_field(D, d):
    """Patch test for an anisotropic material: the direct solve returns u = grad x exactly."""
    grad = np.array([0.7, -0.4, 0.25])[:D]
    prob = linear_field_problem(D, d, _random_spd_voigt(D, 5), grad)
    A, b, grid, _ = fem.build_system(prob)
    u = fem.direct_solve(A, b).reshape(D, -1)
    x = grid.node_coords()
    exact = grad[:, None] * x[None, :, 0]
    assert np.abs(u - exact).max() <= 1e-11 * np.abs(exact).max()


# ----------------------------------------------------------------------------- quadrilateral domains

TRAPEZOID = [[0.0, 0.0], [2.0, 0.0], [0.0, 1.0], [1.4, 0.7]]


def test_quad_on_a_rectangle_equals_box_assembly():
    C = fem.isotropic_tensor(*fem.lame(1.3, 0.28), 2)
    g = fem.QuadGrid(3, [[0, 0], [2.0, 0], [0, 0.5], [2.0, 0.5]])
    for frozen in (True, False):
        K, M = fem.assemble_quad(g, C, frozen)
        Kb, Mb = fem.assemble(fem.Grid(2, 3, [2.0, 0.5]), *fem.lame(1.3, 0.28))
        assert abs(K - Kb).max() <= 1e-14 * abs(Kb).max()
        assert abs(M - Mb).max() <= 1e-14 * abs(Mb).max()


def test_quad_frozen_jacobian_is_exact_on_parallelograms():
    """An affine map has one constant Jacobian per element: the centre-frozen rule equals the
    isoparametric element exactly, which passes the rigid-body and patch tests."""
    C = fem.voigt_to_tensor(_random_spd_voigt(2, 9), 2)
    g = fem.QuadGrid(3, [[0, 0], [2.0, 0.3], [0.5, 1.0], [2.5, 1.3]])
    Kf, Mf = fem.assemble_quad(g, C, True)
    Ki, Mi = fem.assemble_quad(g, C, False)
    assert abs(Kf - Ki).max() <= 1e-13 * abs(Ki).max() and abs(Mf - Mi).max() <= 1e-15
    x = g.node_coords()
    for u in (np.concatenate([np.ones(g.n_nodes), np.zeros(g.n_nodes)]),
              np.concatenate([-x[:, 1], x[:, 0]])):
        assert np.abs(Kf @ u).max() <= 1e-12 * abs(Kf).max()
    assert abs(Mf.sum() - 2.0 * 1.0 + 0.3 * 0.5) <= 1e-13  # area = |det [[2, 0.3], [0.5, 1]]|


def test_quad_trapezoid_properties_and_convergence_of_frozen_rule():
    """On a trapezoid: the isoparametric element integrates the area exactly and reproduces
    rigid motions; the centre-frozen rule keeps symmetry, translations, the area, and its
    solutions approach the isoparametric ones as the elements approach parallelograms."""
    C = fem.isotropic_tensor(*fem.lame(1.0, 0.3), 2)
    P = np.array(TRAPEZOID)
    u, v = P[3] - P[0], P[2] - P[1]
    area = 0.5 * abs(u[0] * v[1] - u[1] * v[0])  # half the cross product of the diagonals
    diffs = []
    for d in (3, 4, 5, 6):
        g = fem.QuadGrid(d, TRAPEZOID)
        Kf, Mf = fem.assemble_quad(g, C, True)
        Ki, Mi = fem.assemble_quad(g, C, False)
        assert abs(Kf - Kf.T).max() <= 1e-14 * abs(Kf).max()
        assert abs(Mi.sum() - area) <= 1e-12 and abs(Mf.sum() - area) <= 1e-12
        x = g.node_coords()
        tx = np.concatenate([np.ones(g.n_nodes), np.zeros(g.n_nodes)])
        rot = np.concatenate([-x[:, 1], x[:, 0]])
        assert np.abs(Kf @ tx).max() <= 1e-12 * abs(Kf).max()
        assert np.abs(Ki @ rot).max() <= 1e-12 * abs(Ki).max()
        probs = [dict(dim=2, level=d, E=1.0, nu=0.3, quad=TRAPEZOID, clamp=[(0, 0)], tractions=[(0, 1, [0.3, -1.0])],
                      quad_rule=r) for r in ("frozen", "isoparametric")]
        us = []
        for pr in probs:
            A, b, _, _ = fem.build_system(pr)
            us.append(fem.direct_solve(A, b))
        diffs.append(np.linalg.norm(us[0] - us[1]) / np.linalg.norm(us[1]))
    # second order: the frozen Jacobian deviates by O(h) inside an element of size O(h)
    ratios = np.array(diffs[:-1]) / np.array(diffs[1:])
    assert np.all(ratios > 3.0), diffs
