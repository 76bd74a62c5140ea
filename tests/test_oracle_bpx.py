"""Pins of the multilevel preconditioner of the oracle (oracle/bpx.py)."""
import numpy as np
import pytest
import scipy.linalg as sl

from oracle import bpx, fem


@pytest.mark.parametrize("L,l", [(4, 0), (4, 2), (5, 3), (5, 5)])
def test_hats_reproduce_linear_functions_and_sum_to_one(L, l):
    # linear interpolation is exact for linear functions: on every fine node below the
    # last coarse node, sum_j phi_j(i) = 1 and sum_j (j s) phi_j(i) = i (all hats kept,
    # the virtual one past the end included, so this holds on every fine node)
    P = bpx.hats(L, l)
    s = 2 ** (L - l)
    i = np.arange(2 ** L)
    centres = np.arange(P.shape[1]) * s
    assert np.allclose(P.sum(axis=1), 1.0, atol=1e-15)
    assert np.allclose(P @ centres, i, atol=1e-12)
    # the finest level is the identity (plus the virtual column, zero on the grid)
    if l == L:
        assert np.array_equal(P[:, : 2 ** L], np.eye(2 ** L)) and not P[:, 2 ** L:].any()


def test_clamped_ends_drop_the_hats_that_reach_them():
    L = 4
    for l in range(L + 1):
        P = bpx.hats(L, l, clamp_lo=True, clamp_hi=True)
        assert not P[0].any() and not P[-1].any()  # every kept hat vanishes on both ends
    # the finest level keeps exactly the interior nodes
    assert np.array_equal(bpx.hats(L, L, True, True), np.eye(2 ** L)[:, 1:-1])


def _kappa(A, B):
    ev = sl.eigvalsh(A, np.linalg.inv(B))
    return ev[-1] / ev[0]


@pytest.mark.parametrize("clamp", [[(0, 0)], [(0, 0), (0, 1), (1, 0), (1, 1)]])
def test_condition_numbers_stay_bounded_where_the_operators_grow_like_4_to_the_level(clamp):
    kA, kB, kC = [], [], []
    for L in range(2, 6):
        prob = dict(dim=2, level=L, E=1.0, nu=0.3, clamp=clamp, body_force=[1.0, 0.5])
        A = fem.build_system(prob)[0].toarray()
        B, C = bpx.preconditioners(prob)
        assert np.allclose(B, B.T) and np.allclose(C, C.T)
        kA.append(np.linalg.cond(A))
        kB.append(_kappa(A, B))
        kC.append(np.linalg.cond(C @ A @ C))
    growth_A = [kA[i + 1] / kA[i] for i in range(3)]
    growth_B = [kB[i + 1] / kB[i] for i in range(3)]
    growth_C = [kC[i + 1] / kC[i] for i in range(3)]
    print("cond A", np.round(kA, 1), "cond BA", np.round(kB, 1), "cond CAC", np.round(kC, 1))
    # cond(A) grows by about 4 per level; the preconditioned conditions grow by less
    # from level to level (measured, levels 2 .. 5: one clamped edge BA 55 .. 94 and
    # CAC 60 .. 170; four clamped edges BA 2.8 .. 48 and CAC 2.8 .. 60)
    assert min(growth_A) > 3.0
    assert all(growth_B[i + 1] < growth_B[i] for i in range(2))
    assert all(growth_C[i + 1] < growth_C[i] for i in range(2))
    assert growth_B[-1] < 2.0 and growth_C[-1] < 2.0
