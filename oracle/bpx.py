"""O5 -- a plain multilevel (BPX-type) preconditioner on the nodal grid (oracle).

Test infrastructure: dense matrices for small grids, used only by the tests.

The paper names preconditioning in tensor format as the step that keeps the solver
stable for very fine grids (Sec. 1.1 and Sec. 7, citing Bachmayr and Kazeev 2020).
This module writes out the additive multilevel preconditioner of Bramble, Pasciak
and Xu (1990) for the vertex grids of this solver, as dense matrices, so that its
properties can be checked before any tensor-format or GPU version is built (none
is built yet).

Grid and levels (per axis): the fine grid has 2^L nodes i = 0 .. 2^L - 1.  Level l
has hat functions phi_{l,j}(i) = max(0, 1 - |i - j s| / s), s = 2^(L - l), centred
at the fine nodes j s, j = 0 .. 2^l; the hat j = 2^l is centred one node past the
last fine node (the fine grid is not dyadically nested with both of its ends, so the
coarse grids are aligned with node 0 and carry one virtual node at the other end).
On an axis clamped at its low end the hat j = 0 is left out, at its high end the
hats j = 2^l - 1 and j = 2^l (their supports reach the clamped node); the remaining
hats vanish on the clamped nodes, so every coarse function is a finite-element
function of the fine grid that satisfies the clamping.  Level L is the identity on
the free nodes.

  M_l  = P_l P_l^T (P_l: fine x coarse, columns phi_{l,j}), tensor product over axes,
  B    = sum_l h_l^(2 - D) M_l / a + (I - P_free) / a     (approximates A^-1),
  C    = sum_l 2^((l - L)(D - 1)) M_l / sqrt(a) + (I - P_free) / sqrt(a)
                                                          (approximates A^-1/2),

h_l = 2^-l the level's mesh size relative to the coarsest, a the diagonal value the
clamped dofs carry in A (oracle.fem.bc_alpha), every displacement component alike.
The weights follow from the multilevel norm equivalences of H^1 and H^(1/2):
cond(B A) and cond(C A C) grow at most polylogarithmically in 2^L where cond(A)
grows like 4^L.
"""
from __future__ import annotations

import numpy as np

from . import fem


def hats(L: int, l: int, clamp_lo: bool = False, clamp_hi: bool = False) -> np.ndarray:
    """P_l for one axis: 2^L x (number of kept hats), column j the hat phi_{l,j}."""
    n, s = 2 ** L, 2 ** (L - l)
    js = [j for j in range(2 ** l + 1)
          if not (clamp_lo and j == 0) and not (clamp_hi and j >= 2 ** l - 1)]
    i = np.arange(n, dtype=np.float64)[:, None]
    j = np.asarray(js, dtype=np.float64)[None, :]
    return np.maximum(0.0, 1.0 - np.abs(i - j * s) / s)


def level_matrix(D: int, L: int, l: int, clamps) -> np.ndarray:
    """Tensor product over the axes of P_l P_l^T, natural node order (axis 0 slowest)."""
    K = None
    for a in range(D):
        P = hats(L, l, (a, 0) in clamps, (a, 1) in clamps)
        M = P @ P.T
        K = M if K is None else np.kron(K, M)
    return K


def preconditioners(problem: dict):
    """(B, C) for the box problem `problem` (dense, natural dof order of oracle.fem)."""
    D, L = problem["dim"], problem["level"]
    A, b, grid, info = fem.build_system(problem)
    clamps = [tuple(c) for c in problem.get("clamp", [])]
    a = info["alpha"]
    clamped = np.diag((~info["mask"]).astype(np.float64))
    nodes_B = sum((2.0 ** -l) ** (2 - D) * level_matrix(D, L, l, clamps) for l in range(L + 1))
    nodes_C = sum(2.0 ** ((l - L) * (D - 1)) * level_matrix(D, L, l, clamps) for l in range(L + 1))
    B = np.kron(np.eye(D), nodes_B) / a + clamped / a
    C = np.kron(np.eye(D), nodes_C) / np.sqrt(a) + clamped / np.sqrt(a)
    return B, C
