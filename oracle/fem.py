"""O1 -- plain sparse Q1 finite elements for linear elasticity (test oracle).

Follows the paper's Sec. 2 (isotropic Hooke law with Lame parameters, eq.
linelastic / diffeq, plane-stress reduction) and Sec. 3 (weak form, Galerkin
system eq. femsys, element-by-element assembly on a reference element eq.
elassembly with gradients mapped by the inverse-transpose Jacobian eq. grads),
on the tensor-product grid of Sec. 5 (2^d equidistant points per axis,
(2^d - 1)^D elements, boundary points included).

Readings of the paper taken here (each also listed in the design doc):
* The weak form a(u, v) = L(v) of Sec. 3 is authoritative for the sign, i.e. the
  strong form is -div(sigma) = f.
* Dirichlet faces are imposed by symmetric elimination,
  A_bc = P A P + alpha (I - P), b_bc = P b, with P the 0/1 mask of free dofs and
  alpha = (lambda + 2 mu) h^(D-2); the solution does not depend on alpha.
* A Neumann face with a given traction t contributes the face integral of t . v.
* Quadrature is 2-point Gauss per axis, which is exact for Q1 on rectangles.

Dof ordering (the "natural" order used by this module only):
    dof = c * n^D + node,  node = (ix * n + iy) [* n + iz],  n = 2^d.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def lame(E: float, nu: float, plane_stress: bool = False):
    """Lame parameters from Young's modulus and Poisson's ratio (Sec. 2).

    Plane strain and 3D use lambda = E nu / ((1+nu)(1-2nu)), mu = E / (2(1+nu)).
    The plane-stress reduction of Sec. 2 replaces lambda by
    2 lambda mu / (lambda + 2 mu) = E nu / (1 - nu^2).
    Pinned by tests/test_oracle_fem.py (closed-form values).
    """
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    if plane_stress:
        lam = 2.0 * lam * mu / (lam + 2.0 * mu)
    return lam, mu


def voigt_to_tensor(Cv, D: int) -> np.ndarray:
    """Stiffness tensor C[i, j, k, l] (sigma_ij = sum_kl C_ijkl eps_kl) from a Voigt matrix
    with engineering shear strains: order (xx, yy, xy) in 2D, (xx, yy, zz, yz, xz, xy) in 3D.
    With the engineering shear, C_ijkl is the Voigt entry of the pairs (ij) and (kl)."""
    Cv = np.asarray(Cv, dtype=np.float64)
    pairs = {2: {(0, 0): 0, (1, 1): 1, (0, 1): 2},
             3: {(0, 0): 0, (1, 1): 1, (2, 2): 2, (1, 2): 3, (0, 2): 4, (0, 1): 5}}[D]
    idx = lambda i, j: pairs[(min(i, j), max(i, j))]  # noqa: E731
    C = np.zeros((D, D, D, D))
    for i, j, k, l in itertools.product(range(D), repeat=4):
        C[i, j, k, l] = Cv[idx(i, j), idx(k, l)]
    return C


def isotropic_tensor(lam: float, mu: float, D: int) -> np.ndarray:
    """C_ijkl = lambda d_ij d_kl + mu (d_ik d_jl + d_il d_jk) (Sec. 2)."""
    e = np.eye(D)
    return (lam * np.einsum("ij,kl->ijkl", e, e) + mu * (np.einsum("ik,jl->ijkl", e, e)
                                                          + np.einsum("il,jk->ijkl", e, e)))


def material_tensor(problem: dict) -> np.ndarray:
    """The problem's stiffness tensor: its Voigt matrix if given, else the isotropic law."""
    D = problem["dim"]
    if problem.get("stiffness_voigt") is not None:
        return voigt_to_tensor(problem["stiffness_voigt"], D)
    lam, mu = lame(problem["E"], problem["nu"], problem.get("plane_stress", False))
    return isotropic_tensor(lam, mu, D)


def corner_bits(D: int) -> np.ndarray:
    """Corners of the reference element [-1, 1]^D as 0/1 bits, x most significant."""
    return np.array(list(itertools.product((0, 1), repeat=D)), dtype=np.int64)


def gauss_points(D: int):
    """Tensor 2-point Gauss rule on [-1, 1]^D (points, weights)."""
    g = 1.0 / np.sqrt(3.0)
    pts = np.array(list(itertools.product((-g, g), repeat=D)))
    w = np.ones(len(pts))
    return pts, w


def ref_shape(D: int, xi: np.ndarray):
    """Q1 shape functions on the reference element and their reference gradients.

    phi_c(xi) = prod_a (1 + s_{c,a} xi_a) / 2 with s = +-1 the corner sign.
    Returns (phi[c], dphi[c, a]).
    """
    s = 2.0 * corner_bits(D) - 1.0
    fac = 0.5 * (1.0 + s * xi[None, :])  # [corner, axis]
    phi = np.prod(fac, axis=1)
    dphi = np.empty_like(fac)
    for a in range(D):
        other = np.prod(np.delete(fac, a, axis=1), axis=1) if D > 1 else 1.0
        dphi[:, a] = 0.5 * s[:, a] * other
    return phi, dphi


def element_matrices(D: int, h, lam: float, mu: float, C=None):
    """Element stiffness and (scalar) mass matrices of one rectangular Q1 element.

    The element map Phi(xi) = x0 + (xi + 1) h / 2 has constant Jacobian
    J = diag(h / 2); gradients are J^{-T} times reference gradients (eq. grads)
    and the integrand is weighted by |det J| (eq. elassembly).  The stiffness
    entry for test function e_a phi_p and trial function e_b phi_q is the
    integral of sigma(e_b phi_q) : eps(e_a phi_p) with
    sigma = lambda tr(eps) I + 2 mu eps (Sec. 2), or sigma_ij = sum_kl C_ijkl eps_kl
    when a stiffness tensor C is given (anisotropic material).

    Returns Ke[(a, p), (b, q)] of size (D 2^D)^2 with index a * 2^D + p, and the
    scalar mass Me[p, q] (the vector mass is block diagonal in components).
    Pinned by tests/test_oracle_fem.py (textbook element, rigid modes, closed
    1D integrals).
    """
    h = np.broadcast_to(np.asarray(h, dtype=np.float64), (D,))
    nc = 2 ** D
    Jinv_T = np.diag(2.0 / h)
    detJ = abs(np.prod(h / 2.0))
    pts, wts = gauss_points(D)
    Ke = np.zeros((D * nc, D * nc))
    Me = np.zeros((nc, nc))
    eye = np.eye(D)
    for xi, w in zip(pts, wts):
        phi, dphi_ref = ref_shape(D, xi)
        grad = dphi_ref @ Jinv_T.T  # grad[c] = J^{-T} dphi_ref[c]
        Me += w * detJ * np.outer(phi, phi)
        # strain of each vector basis function e_a phi_p
        eps = np.zeros((D, nc, D, D))
        for a in range(D):
            for p in range(nc):
                G = np.outer(eye[a], grad[p])  # (grad u)_ij = d u_i / d x_j
                eps[a, p] = 0.5 * (G + G.T)
        for b in range(D):
            for q in range(nc):
                e = eps[b, q]
                sig = lam * np.trace(e) * eye + 2.0 * mu * e if C is None else np.einsum("ijkl,kl->ij", C, e)
                for a in range(D):
                    for p in range(nc):
                        Ke[a * nc + p, b * nc + q] += w * detJ * np.sum(sig * eps[a, p])
    return Ke, Me


class Grid:
    """Tensor-product grid of 2^d nodes per axis on the box [0, extent]."""

    def __init__(self, D: int, d: int, extent=None):
        self.D, self.d = D, d
        self.n = 2 ** d
        self.extent = np.ones(D) if extent is None else np.asarray(extent, dtype=np.float64)[:D]
        self.h = self.extent / (self.n - 1)
        self.n_nodes = self.n ** D
        self.n_dofs = D * self.n_nodes

    def node_index(self, idx):
        """Natural node index of integer coordinates idx[..., D]."""
        out = np.zeros(np.shape(idx)[:-1], dtype=np.int64)
        for a in range(self.D):
            out = out * self.n + idx[..., a]
        return out

    def node_coords(self):
        """Coordinates x[node, a] of all nodes in natural order."""
        ax = [np.arange(self.n) * self.h[a] for a in range(self.D)]
        mesh = np.meshgrid(*ax, indexing="ij")
        return np.stack([m.reshape(-1) for m in mesh], axis=1)

    def element_nodes(self):
        """Natural node indices of the 2^D corners of every element, [elem, corner]."""
        ne = self.n - 1
        elems = np.array(list(itertools.product(range(ne), repeat=self.D)), dtype=np.int64)
        bits = corner_bits(self.D)
        return self.node_index(elems[:, None, :] + bits[None, :, :]), elems


# ----------------------------------------------------------------------------- quadrilateral domains

def quad_corners(corners):
    """Corners of a quadrilateral domain as a [4, 2] array in the order P00, P10, P01, P11
    (images of the unit-square corners (s, t) = (0,0), (1,0), (0,1), (1,1))."""
    P = np.asarray(corners, dtype=np.float64).reshape(4, 2)
    return P


def quad_map(corners, s, t):
    """Bilinear map of the unit square onto the quadrilateral: x(s, t) (arrays broadcast)."""
    P = quad_corners(corners)
    s = np.asarray(s, dtype=np.float64)[..., None]
    t = np.asarray(t, dtype=np.float64)[..., None]
    return P[0] * (1 - s) * (1 - t) + P[1] * s * (1 - t) + P[2] * (1 - s) * t + P[3] * s * t


class QuadGrid(Grid):
    """2^d x 2^d nodes on a quadrilateral (Sec. 5): node (i, j) at x(i / (2^d - 1), j / (2^d - 1))."""

    def __init__(self, d: int, corners):
        super().__init__(2, d)
        self.corners = quad_corners(corners)

    def node_coords(self):
        ij = np.array(list(itertools.product(range(self.n), repeat=2)), dtype=np.float64) / (self.n - 1)
        return quad_map(self.corners, ij[:, 0], ij[:, 1])


def quad_element_matrices(xc, C, frozen: bool = True):
    """Stiffness and scalar mass of one Q1 element with corner coordinates xc[c, 2] (corner c
    in the order of corner_bits(2)).  The element map Phi(xi) = sum_c x_c phi_c(xi) has the
    Jacobian J(xi) = sum_c x_c (x) grad phi_c(xi); gradients are J^{-T} times reference
    gradients (eq. grads), the integrand is weighted by det J (eq. elassembly), and the
    element stiffness is the integral of C grad(v) : grad(u) over the 2-point Gauss rule.
    frozen=True takes J and det J at the element centre xi = (0, 0) for every quadrature
    point (Alg. 1 evaluates them there), which is exact for parallelograms; frozen=False
    is the isoparametric element (J at each Gauss point, exact for the bilinear element)."""
    xc = np.asarray(xc, dtype=np.float64)
    pts, wts = gauss_points(2)
    nc = 4
    Ke = np.zeros((2 * nc, 2 * nc))
    Me = np.zeros((nc, nc))
    _, d0 = ref_shape(2, np.zeros(2))
    J0 = xc.T @ d0  # J[k, gamma] = sum_c x_c[k] dphi_c/dxi_gamma
    for xi, w in zip(pts, wts):
        phi, dphi = ref_shape(2, xi)
        J = J0 if frozen else xc.T @ dphi
        det = np.linalg.det(J)
        grad = dphi @ np.linalg.inv(J)  # grad[c, alpha] = sum_gamma dphi[c, gamma] (J^-1)[gamma, alpha]
        Me += w * det * np.outer(phi, phi)
        for a in range(2):
            for b in range(2):
                # sum_{alpha beta} C[a, alpha, b, beta] grad_p[alpha] grad_q[beta]
                Ke[a * nc:(a + 1) * nc, b * nc:(b + 1) * nc] += w * det * grad @ C[a, :, b, :] @ grad.T
    return Ke, Me


def assemble_quad(grid: QuadGrid, C, frozen: bool = True, elem_weight=None):
    """Global stiffness (2 n^2 dofs, natural order) and scalar mass (n^2 nodes) on a
    quadrilateral grid, element by element; elem_weight[i, j] scales element (i, j)'s
    stiffness (a non-homogeneous material)."""
    x = grid.node_coords()
    enodes, elems = grid.element_nodes()
    w = np.ones(len(elems)) if elem_weight is None else np.asarray(elem_weight, dtype=np.float64)[tuple(elems.T)]
    nc = 4
    rows, cols, vals, mr, mc, mv = [], [], [], [], [], []
    for e in range(len(elems)):
        nodes = enodes[e]
        Ke, Me = quad_element_matrices(x[nodes], C, frozen)
        dofs = np.concatenate([a * grid.n_nodes + nodes for a in range(2)])
        rows.append(np.repeat(dofs, 2 * nc)); cols.append(np.tile(dofs, 2 * nc)); vals.append(w[e] * Ke.reshape(-1))
        mr.append(np.repeat(nodes, nc)); mc.append(np.tile(nodes, nc)); mv.append(Me.reshape(-1))
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(grid.n_dofs, grid.n_dofs)).tocsr()
    M = sp.coo_matrix((np.concatenate(mv), (np.concatenate(mr), np.concatenate(mc))),
                      shape=(grid.n_nodes, grid.n_nodes)).tocsr()
    return K, M


def quad_traction_load(grid: QuadGrid, axis: int, side: int, t):
    """Load of a uniform traction t on one straight side of the quadrilateral: the 1D mass
    row sums along the side (length L, node spacing L / (n - 1)) times t."""
    P = grid.corners
    ends = {(0, 0): (0, 2), (0, 1): (1, 3), (1, 0): (0, 1), (1, 1): (2, 3)}[(axis, side)]
    L = np.linalg.norm(P[ends[1]] - P[ends[0]])
    h = L / (grid.n - 1)
    m = np.full(grid.n, h)
    m[0] = m[-1] = 0.5 * h
    b = np.zeros(grid.n_dofs)
    nodes = face_nodes(grid, axis, side)
    for c in range(2):
        b[c * grid.n_nodes + nodes] += t[c] * m
    return b


def assemble(grid: Grid, lam: float, mu: float, elem_weight=None, C=None):
    """Global stiffness K and scalar mass M by element-by-element assembly (Sec. 3).

    elem_weight, if given, is an array over element index tuples (shape
    (n-1,)*D) scaling lambda and mu of each element (a non-homogeneous modulus
    E_e = w_e E at fixed Poisson ratio).  K is returned over all D * n^D dofs in
    natural order, M over the n^D nodes.
    """
    D = grid.D
    Ke, Me = element_matrices(D, grid.h, lam, mu, C)
    enodes, elems = grid.element_nodes()
    ne_tot = len(elems)
    if elem_weight is None:
        w = np.ones(ne_tot)
    else:
        w = np.asarray(elem_weight, dtype=np.float64)[tuple(elems.T)]
    nc = 2 ** D
    edofs = np.concatenate([a * grid.n_nodes + enodes for a in range(D)], axis=1)  # [elem, a*nc+p]
    nl = D * nc
    rows = np.repeat(edofs, nl, axis=1).reshape(-1)
    cols = np.tile(edofs, (1, nl)).reshape(-1)
    vals = (w[:, None] * Ke.reshape(1, -1)).reshape(-1)
    K = sp.coo_matrix((vals, (rows, cols)), shape=(grid.n_dofs, grid.n_dofs)).tocsr()
    mrows = np.repeat(enodes, nc, axis=1).reshape(-1)
    mcols = np.tile(enodes, (1, nc)).reshape(-1)
    mvals = np.tile(Me.reshape(1, -1), (ne_tot, 1)).reshape(-1)
    M = sp.coo_matrix((mvals, (mrows, mcols)), shape=(grid.n_nodes, grid.n_nodes)).tocsr()
    return K, M


def vector_mass(grid: Grid, M):
    """Vector mass matrix: the scalar mass on each displacement component."""
    return sp.kron(sp.identity(grid.D, format="csr"), M, format="csr")


def body_load(grid: Grid, M, f_nodal):
    """RHS f = M f0 from nodal values f0[c, node] of the body force (Sec. 5.3)."""
    f_nodal = np.asarray(f_nodal, dtype=np.float64).reshape(grid.D, grid.n_nodes)
    return np.concatenate([M @ f_nodal[c] for c in range(grid.D)])


def nodal_values_from_tt(cores, D: int, d: int):
    """f0[c, node] from a TT of nodal values in the solution layout: d level cores
    (most significant bit first, mode (bx 2 + by) 2 + bz) then the component core."""
    from . import qtt, tt

    flat = tt.tt_full([np.asarray(c, dtype=np.float64) for c in cores]).reshape(-1)
    return flat[qtt.natural_to_qtt(D, d)].reshape(D, -1)


def face_nodes(grid: Grid, axis: int, side: int):
    """Natural indices of the nodes on face {x_axis = side * extent}."""
    coords = np.array(list(itertools.product(range(grid.n), repeat=grid.D)), dtype=np.int64)
    sel = coords[:, axis] == (0 if side == 0 else grid.n - 1)
    return grid.node_index(coords[sel])


def traction_load(grid: Grid, axis: int, side: int, t):
    """Load of a uniform traction t on one face: integral of t . v over the face.

    Integrated face element by face element with the (D-1)-dimensional Q1 basis
    and 2-point Gauss quadrature (exact).
    """
    D = grid.D
    t = np.asarray(t, dtype=np.float64)[:D]
    b = np.zeros(grid.n_dofs)
    other = [a for a in range(D) if a != axis]
    fixed = 0 if side == 0 else grid.n - 1
    if D == 1:
        node = fixed
        for c in range(D):
            b[c * grid.n_nodes + node] += t[c]
        return b
    Df = D - 1
    hf = grid.h[other]
    pts, wts = gauss_points(Df)
    detJ = np.prod(hf / 2.0)
    phis = np.array([ref_shape(Df, xi)[0] for xi in pts])  # [gauss, corner]
    fe = (wts[:, None] * phis).sum(axis=0) * detJ  # integral of each face basis fn
    bits = corner_bits(Df)
    for fel in itertools.product(range(grid.n - 1), repeat=Df):
        for ci, cb in enumerate(bits):
            idx = np.zeros(D, dtype=np.int64)
            idx[axis] = fixed
            for j, a in enumerate(other):
                idx[a] = fel[j] + cb[j]
            node = grid.node_index(idx[None, :])[0]
            for c in range(D):
                b[c * grid.n_nodes + node] += t[c] * fe[ci]
    return b


def clamp_mask(grid: Grid, faces):
    """0/1 mask over all dofs: 0 on every component of nodes of clamped faces."""
    free = np.ones(grid.n_nodes, dtype=bool)
    for axis, side in faces:
        free[face_nodes(grid, axis, side)] = False
    return np.tile(free, grid.D)


def apply_dirichlet(K, b, mask, alpha: float):
    """Symmetric elimination of clamped dofs: (P K P + alpha (I - P), P b)."""
    P = sp.diags(mask.astype(np.float64))
    Q = sp.diags((~mask).astype(np.float64))
    return (P @ K @ P + alpha * Q).tocsr(), b * mask


def bc_alpha(grid: Grid, lam: float, mu: float, C=None) -> float:
    """Diagonal value given to clamped dofs: max_i C_iiii h^(D-2), h along x (lambda + 2 mu
    for an isotropic material)."""
    cmax = lam + 2.0 * mu if C is None else max(C[i, i, i, i] for i in range(grid.D))
    return cmax * grid.h[0] ** (grid.D - 2)


def manufactured_u(x, c):
    """u*_i(x) = c_i prod_a sin(pi x_a) on the unit box (vanishes on every face)."""
    S = np.prod(np.sin(np.pi * x), axis=1)
    return np.stack([ci * S for ci in c], axis=0)


def manufactured_f(x, c, lam: float, mu: float):
    """Body force f = -div sigma(u*) for u* of manufactured_u, in closed form.

    With S = prod sin(pi x_a): -div sigma(u*)_i =
      pi^2 [ (lambda + (D+1) mu) c_i S - (lambda + mu) sum_{k != i} c_k
             cos(pi x_i) cos(pi x_k) prod_{a != i,k} sin(pi x_a) ].
    Pinned by a finite-difference check in tests/test_oracle_fem.py.
    """
    D = x.shape[1]
    s = np.sin(np.pi * x)
    k = np.cos(np.pi * x)
    S = np.prod(s, axis=1)
    f = np.zeros((D, x.shape[0]))
    for i in range(D):
        f[i] = (lam + (D + 1) * mu) * c[i] * S
        for kk in range(D):
            if kk == i:
                continue
            rest = np.ones(x.shape[0])
            for a in range(D):
                if a not in (i, kk):
                    rest = rest * s[:, a]
            f[i] -= (lam + mu) * c[kk] * k[:, i] * k[:, kk] * rest
    return np.pi ** 2 * f


def build_system(problem: dict):
    """Assemble (A_bc, b_bc, grid, info) for a problem description.

    problem keys: dim, level, E, nu, plane_stress (opt), extent (opt),
    clamp: list of (axis, side), tractions: list of (axis, side, t),
    body_force: constant vector (opt), manufactured_c: vector (opt; load
    f = M f0 with f0 the closed-form manufactured force at the nodes),
    f_nodal_tt: TT cores of nodal force values f0 (opt; load M f0, Alg. 2 / Sec. 5.3),
    layered_E: (axis, values per element along that axis) (opt),
    stiffness_voigt: constant anisotropic stiffness, Voigt matrix (opt; replaces E, nu in
    the element integrals, layered_E / E still scales it), elem_weight: per-element stiffness
    factors (opt; a non-homogeneous material).
    """
    D, d = problem["dim"], problem["level"]
    if problem.get("quad") is not None:
        return _build_quad_system(problem)
    grid = Grid(D, d, problem.get("extent"))
    lam, mu = lame(problem["E"], problem["nu"], problem.get("plane_stress", False))
    weight = None
    if problem.get("elem_weight") is not None:  # per-element field (2D)
        weight = np.asarray(problem["elem_weight"], dtype=np.float64).reshape((grid.n - 1,) * D)
    if problem.get("layered_E") is not None:
        axis, vals = problem["layered_E"]
        vals = np.asarray(vals, dtype=np.float64) / problem["E"]
        shape = [1] * D
        shape[axis] = grid.n - 1
        weight = np.broadcast_to(vals.reshape(shape), (grid.n - 1,) * D)
    C = voigt_to_tensor(problem["stiffness_voigt"], D) if problem.get("stiffness_voigt") is not None else None
    K, M = assemble(grid, lam, mu, weight, C)
    b = np.zeros(grid.n_dofs)
    if problem.get("body_force") is not None:
        f0 = np.repeat(np.asarray(problem["body_force"], dtype=np.float64)[:D, None], grid.n_nodes, axis=1)
        b += body_load(grid, M, f0)
    if problem.get("manufactured_c") is not None:
        x = grid.node_coords()
        f0 = manufactured_f(x, np.asarray(problem["manufactured_c"], dtype=np.float64), lam, mu)
        b += body_load(grid, M, f0)
    if problem.get("f_nodal_tt") is not None:
        b += body_load(grid, M, nodal_values_from_tt(problem["f_nodal_tt"], D, d))
    for axis, side, t in problem.get("tractions", []):
        b += traction_load(grid, axis, side, t)
    mask = clamp_mask(grid, problem.get("clamp", []))
    alpha = bc_alpha(grid, lam, mu, C)
    A, bb = apply_dirichlet(K, b, mask, alpha)
    return A, bb, grid, dict(K=K, M=M, b_raw=b, mask=mask, lam=lam, mu=mu, alpha=alpha)


def _build_quad_system(problem: dict):
    """build_system on a quadrilateral domain (2D; key quad = corners P00, P10, P01, P11):
    stiffness with the Jacobian frozen at element centres (problem key quad_rule =
    "isoparametric" for the exact bilinear element), consistent mass, loads and clamps as on
    the box (the sides are the parametric faces)."""
    D, d = problem["dim"], problem["level"]
    assert D == 2, "quadrilateral domains are 2D"
    grid = QuadGrid(d, problem["quad"])
    lam, mu = lame(problem["E"], problem["nu"], problem.get("plane_stress", False))
    C = material_tensor(problem)
    frozen = problem.get("quad_rule", "frozen") == "frozen"
    ew = problem.get("elem_weight")
    ew = None if ew is None else np.asarray(ew, dtype=np.float64).reshape(grid.n - 1, grid.n - 1)
    K, M = assemble_quad(grid, C, frozen, ew)
    b = np.zeros(grid.n_dofs)
    if problem.get("body_force") is not None:
        f0 = np.repeat(np.asarray(problem["body_force"], dtype=np.float64)[:D, None], grid.n_nodes, axis=1)
        b += body_load(grid, M, f0)
    if problem.get("f_nodal_tt") is not None:
        b += body_load(grid, M, nodal_values_from_tt(problem["f_nodal_tt"], D, d))
    for axis, side, t in problem.get("tractions", []):
        b += quad_traction_load(grid, axis, side, t)
    mask = clamp_mask(grid, problem.get("clamp", []))
    alpha = max(C[i, i, i, i] for i in range(D))
    A, bb = apply_dirichlet(K, b, mask, alpha)
    return A, bb, grid, dict(K=K, M=M, b_raw=b, mask=mask, lam=lam, mu=mu, alpha=alpha)


def direct_solve(A, b):
    """Sparse direct solve (SciPy SuperLU)."""
    return spla.spsolve(A.tocsc(), b)
