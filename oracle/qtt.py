"""Independent QTT construction of the stiffness operator and load (oracle).

Sec. 5 of the paper assembles A and M directly in TT format (Alg. 1): element
quantities become TTs over the element index and are converted to the global
basis-function index; boundary conditions are then applied.  On the Cartesian
grids used here the element Jacobians are constant, and the element-by-element
sum factorises over axes, so the plain definition of the same operator is

    A = sum_{a,b} E_ab (x) K_ab,
    K_ab = lambda D_ab + mu D_ba + mu delta_ab sum_c D_cc,

where E_ab is the D x D component matrix unit and D_ab is the Kronecker product over axes of 1D Q1 integrals:
    a == b:  S (int phi' phi') on axis a, M (int phi phi) elsewhere;
    a != b:  G (int phi' phi) on axis a, G^T on axis b, M elsewhere.
This module forms every 1D factor as a dense matrix by 1D element-by-element
Gauss quadrature, turns it into a QTT by TT-SVD (a plain decomposition, no
hand-made cores), interleaves the axes level by level (the paper's (i_k, j_k)
level indices, most significant bit first, Sec. 4), sums all terms and rounds.
Clamped faces enter as P A P + alpha (I - P) with P a Kronecker product of 1D
masks.  The load is b = P M f0 (Sec. 5.3) plus face tractions.

Index order.  The paper lists the component index first ("d+1 row and column
indices ... dimensions 2, 4, 4, ...", Sec. 5.2).  The order of TT indices does
not change the operator, only its ranks; every function here takes
component_first (default False: level cores first, component core last, the
layout of the GPU library, where the exact operator has smaller ranks).

Parity: the dense reconstruction of these TTs equals the element-by-element
sparse assembly of oracle.fem on small grids (tests/test_oracle_qtt.py).
"""
from __future__ import annotations

import itertools

import numpy as np

from . import fem, tt


# ----------------------------------------------------------------------------- index maps

def natural_to_qtt(D: int, d: int, component_first: bool = False) -> np.ndarray:
    """q[natural dof] = flat QTT index; m_l = bits (ix_l, iy_l[, iz_l]), MSB first.

    component_first: index (c, m_1..m_d); otherwise (m_1..m_d, c).
    """
    n = 2 ** d
    coords = np.array(list(itertools.product(range(n), repeat=D)), dtype=np.int64)  # natural node order
    qnode = np.zeros(len(coords), dtype=np.int64)
    for l in range(d):
        m = np.zeros(len(coords), dtype=np.int64)
        for a in range(D):
            bit = (coords[:, a] >> (d - 1 - l)) & 1
            m = m * 2 + bit
        qnode = qnode * (2 ** D) + m
    nn = n ** D
    if component_first:
        return np.concatenate([c * nn + qnode for c in range(D)])
    return np.concatenate([qnode * D + c for c in range(D)])


def to_qtt_order(v_nat, D, d, component_first=False):
    q = natural_to_qtt(D, d, component_first)
    out = np.empty_like(v_nat)
    out[q] = v_nat
    return out


def matrix_to_qtt_order(A_nat, D, d, component_first=False):
    q = natural_to_qtt(D, d, component_first)
    inv = np.empty_like(q)
    inv[q] = np.arange(len(q))
    A = A_nat.tocsr() if hasattr(A_nat, "tocsr") else A_nat
    return A[inv][:, inv]


def qtt_dof_index(D: int, d: int, comp, coords, component_first=False):
    """TT multi-indices of dofs (component comp, integer node coords[num, D])."""
    coords = np.asarray(coords, dtype=np.int64)
    out = np.zeros((coords.shape[0], d + 1), dtype=np.int64)
    off = 1 if component_first else 0
    out[:, 0 if component_first else d] = comp
    for l in range(d):
        m = np.zeros(coords.shape[0], dtype=np.int64)
        for a in range(D):
            m = m * 2 + ((coords[:, a] >> (d - 1 - l)) & 1)
        out[:, l + off] = m
    return out


# ----------------------------------------------------------------------------- 1D factors

def one_d_factors(d: int, length: float, weight=None):
    """Dense 1D Q1 matrices S, M, G on 2^d nodes by element-wise 2-point Gauss.

    S[p,q] = sum_e w_e int_e phi_p' phi_q',  M[p,q] = sum_e w_e int_e phi_p phi_q,
    G[p,q] = sum_e w_e int_e phi_p' phi_q.
    """
    n = 2 ** d
    h = length / (n - 1)
    w = np.ones(n - 1) if weight is None else np.asarray(weight, dtype=np.float64)
    g = 1.0 / np.sqrt(3.0)
    S = np.zeros((n, n)); M = np.zeros((n, n)); G = np.zeros((n, n))
    for xi in (-g, g):
        phi = np.array([(1 - xi) / 2, (1 + xi) / 2])
        dphi = np.array([-0.5, 0.5]) * (2.0 / h)
        jac = h / 2.0
        for e in range(n - 1):
            idx = np.array([e, e + 1])
            S[np.ix_(idx, idx)] += w[e] * jac * np.outer(dphi, dphi)
            M[np.ix_(idx, idx)] += w[e] * jac * np.outer(phi, phi)
            G[np.ix_(idx, idx)] += w[e] * jac * np.outer(dphi, phi)
    return S, M, G


def matrix_qtt(F, d, eps=1e-15):
    """QTT of an n x n matrix by TT-SVD with level indices (i_l, j_l), MSB first."""
    T = np.asarray(F).reshape([2] * d + [2] * d)
    perm = [x for l in range(d) for x in (l, d + l)]
    T = T.transpose(perm).reshape([4] * d)
    cores = tt.tt_svd(T, [4] * d, eps=eps)
    return [C.reshape(C.shape[0], 2, 2, C.shape[2]) for C in cores]


def vector_qtt(v, d, eps=1e-15):
    return tt.tt_svd(np.asarray(v).reshape([2] * d), [2] * d, eps=eps)


def kron_levels_matrix(factors):
    """Interleave per-axis QTT matrices: level core l = Kronecker of the axes' cores."""
    D = len(factors)
    d = len(factors[0])
    out = []
    for l in range(d):
        C = factors[0][l]
        for a in range(1, D):
            F = factors[a][l]
            R1, m1, n1, S1 = C.shape
            R2, m2, n2, S2 = F.shape
            C = np.einsum("aijb,cklf->acikjlbf", C, F).reshape(R1 * R2, m1 * m2, n1 * n2, S1 * S2)
        out.append(C)
    return out


def kron_levels_vector(factors):
    D = len(factors)
    d = len(factors[0])
    out = []
    for l in range(d):
        C = factors[0][l]
        for a in range(1, D):
            F = factors[a][l]
            R1, m1, S1 = C.shape
            R2, m2, S2 = F.shape
            C = np.einsum("aib,ckf->acikbf", C, F).reshape(R1 * R2, m1 * m2, S1 * S2)
        out.append(C)
    return out


# ----------------------------------------------------------------------------- assembly

def _masks(problem, D, n):
    masks = [np.ones(n) for _ in range(D)]
    for axis, side in problem.get("clamp", []):
        masks[axis][0 if side == 0 else n - 1] = 0.0
    return masks


def _axis_weights(problem, D, n):
    w = [None] * D
    if problem.get("layered_E") is not None:
        axis, vals = problem["layered_E"]
        w[axis] = np.asarray(vals, dtype=np.float64) / problem["E"]
    return w


def _attach_component(comp_core, levels, component_first):
    """Place the component core first (paper's listing) or last."""
    return [comp_core] + levels if component_first else levels + [comp_core]


def _dense_operator_qtt(A_nat, D, d, eps, component_first):
    """MPO of a dense (natural-order) operator by TT-SVD over the paired (out, in) indices of
    each core (tiny grids only)."""
    Aq = matrix_to_qtt_order(A_nat, D, d, component_first).toarray()
    modes = [D] + [2 ** D] * d if component_first else [2 ** D] * d + [D]
    K = len(modes)
    T = Aq.reshape(modes + modes)
    T = T.transpose([x for k in range(K) for x in (k, K + k)]).reshape([m * m for m in modes])
    cores = tt.tt_svd(T, [m * m for m in modes], eps=eps)
    return [C.reshape(C.shape[0], m, m, C.shape[2]) for C, m in zip(cores, modes)]


def assemble_operator(problem: dict, eps=1e-14, component_first=False):
    """QTT operator A_bc: component core + d level cores, rounded at eps.

    A_bc = sum over atoms of C_atom (x) D_atom where, for each ordered axis pair
    (a, b), D_ab is the Kronecker atom described in the module docstring and
    C_ab[i, j] = C_iajb (stiffness tensor; lambda E_ab + mu E_ba + delta_ab mu I for an
    isotropic material) collects every place D_ab occurs in K; the clamped dofs add
    alpha I (x) (I - P).  component_first=True gives
    the paper's index order (component, level 0, ..., level d-1); the default
    puts the component index last.
    """
    D, d = problem["dim"], problem["level"]
    if problem.get("quad") is not None or problem.get("elem_weight") is not None:
        # quadrilateral domain or a general element field: the sparse element-by-element
        # operator, compressed by TT-SVD
        A, _, _, _ = fem.build_system(problem)
        return _dense_operator_qtt(A, D, d, eps, component_first)
    n = 2 ** d
    extent = np.ones(D) if problem.get("extent") is None else np.asarray(problem["extent"], float)[:D]
    lam, mu = fem.lame(problem["E"], problem["nu"], problem.get("plane_stress", False))
    masks = _masks(problem, D, n)
    wts = _axis_weights(problem, D, n)
    S, M, G = [], [], []
    for a in range(D):
        s_, m_, g_ = one_d_factors(d, extent[a], wts[a])
        P = np.diag(masks[a])
        S.append(P @ s_ @ P); M.append(P @ m_ @ P); G.append(P @ g_ @ P)

    def atom(a, b):
        facs = []
        for c in range(D):
            if a == b:
                F = S[c] if c == a else M[c]
            else:
                F = G[c] if c == a else (G[c].T if c == b else M[c])
            facs.append(matrix_qtt(F, d))
        return kron_levels_matrix(facs)

    def comp(Cm):
        return np.asarray(Cm, dtype=np.float64).reshape(1, D, D, 1)

    E = np.eye(D)
    Ct = fem.material_tensor(problem)
    total = None
    for a in range(D):
        for b in range(D):
            Cm = Ct[:, a, :, b]  # test component i, trial component j of d_a phi_p d_b phi_q
            term = _attach_component(comp(Cm), atom(a, b), component_first)
            total = term if total is None else tt.mpo_round(tt.mpo_add(total, term), eps)
    h = extent[0] / (n - 1)
    alpha = max(Ct[i, i, i, i] for i in range(D)) * h ** (D - 2)
    Ilev = kron_levels_matrix([matrix_qtt(np.eye(n), d) for _ in range(D)])
    Plev = kron_levels_matrix([matrix_qtt(np.diag(masks[a]), d) for a in range(D)])
    total = tt.mpo_round(tt.mpo_add(total, _attach_component(comp(alpha * E), Ilev, component_first)), eps)
    total = tt.mpo_round(tt.mpo_add(total, _attach_component(comp(-alpha * E), Plev, component_first)), eps)
    return total


def manufactured_terms(D, lam, mu, c):
    """Separable terms of the manufactured force: list of (component, coef, per-axis kind).

    kind 's' = sin(pi x), 'k' = cos(pi x); see oracle.fem.manufactured_f.
    """
    terms = []
    for i in range(D):
        terms.append((i, np.pi ** 2 * (lam + (D + 1) * mu) * c[i], ["s"] * D))
        for k in range(D):
            if k == i:
                continue
            kinds = ["s"] * D
            kinds[i] = "k"; kinds[k] = "k"
            terms.append((i, -np.pi ** 2 * (lam + mu) * c[k], kinds))
    return terms


def assemble_load(problem: dict, eps=1e-14, component_first=False):
    """QTT of b = P (M f0 + tractions): component core + d level cores (order as in assemble_operator)."""
    D, d = problem["dim"], problem["level"]
    if problem.get("quad") is not None:
        _, bq, _, _ = fem.build_system(problem)
        modes = [D] + [2 ** D] * d if component_first else [2 ** D] * d + [D]
        return tt.tt_svd(to_qtt_order(bq, D, d, component_first).reshape(modes), modes, eps)
    n = 2 ** d
    extent = np.ones(D) if problem.get("extent") is None else np.asarray(problem["extent"], float)[:D]
    lam, mu = fem.lame(problem["E"], problem["nu"], problem.get("plane_stress", False))
    masks = _masks(problem, D, n)
    Ms = [one_d_factors(d, extent[a])[1] for a in range(D)]
    pieces = []  # (component vector, list of per-axis nodal vectors)
    if problem.get("body_force") is not None:
        f = np.asarray(problem["body_force"], dtype=np.float64)[:D]
        pieces.append((f, [masks[a] * (Ms[a] @ np.ones(n)) for a in range(D)]))
    if problem.get("manufactured_c") is not None:
        c = np.asarray(problem["manufactured_c"], dtype=np.float64)
        xs = [np.arange(n) * extent[a] / (n - 1) for a in range(D)]
        for comp, coef, kinds in manufactured_terms(D, lam, mu, c):
            vecs = []
            for a in range(D):
                v = np.sin(np.pi * xs[a]) if kinds[a] == "s" else np.cos(np.pi * xs[a])
                vecs.append(masks[a] * (Ms[a] @ v))
            e = np.zeros(D); e[comp] = coef
            pieces.append((e, vecs))
    for axis, side, t in problem.get("tractions", []):
        t = np.asarray(t, dtype=np.float64)[:D]
        vecs = []
        for a in range(D):
            if a == axis:
                v = np.zeros(n); v[0 if side == 0 else n - 1] = 1.0
            else:
                v = Ms[a] @ np.ones(n)
            vecs.append(masks[a] * v)
        pieces.append((t, vecs))
    total = None
    if problem.get("f_nodal_tt") is not None:
        # nodal load f0 given as a TT (Alg. 2): b = P M f0 formed with the sparse mass
        # matrix on the dense grid, then compressed by TT-SVD
        grid = fem.Grid(D, d, problem.get("extent"))
        _, M = fem.assemble(grid, lam, mu)
        mask = fem.clamp_mask(grid, problem.get("clamp", []))
        bn = mask * fem.body_load(grid, M, fem.nodal_values_from_tt(problem["f_nodal_tt"], D, d))
        modes = [D] + [2 ** D] * d if component_first else [2 ** D] * d + [D]
        total = tt.tt_svd(to_qtt_order(bn, D, d, component_first).reshape(modes), modes, eps)
    for comp, vecs in pieces:
        lev = kron_levels_vector([vector_qtt(v, d) for v in vecs])
        c0 = np.asarray(comp, dtype=np.float64).reshape(1, D, 1)
        term = [c0] + lev if component_first else lev + [c0]
        total = term if total is None else tt.tt_round(tt.tt_add(total, term), eps)
    if total is None:
        zl = [np.zeros((1, 2 ** D, 1)) for _ in range(d)]
        total = [np.zeros((1, D, 1))] + zl if component_first else zl + [np.zeros((1, D, 1))]
    return total
