"""Pins of the oracle's TT primitives and random generator."""
import os

import numpy as np
import pytest

from oracle import rng, tt, qtt

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_outputs():
    want = [int(l, 16) for l in open(os.path.join(GOLD, "splitmix64_seed0.txt")) if not l.startswith("#")]
    got = [int(v) for v in rng.splitmix64(0, len(want))]
    assert got == want
    # counter form: an offset continues the same stream
    assert int(rng.splitmix64(0, 1, offset=2)[0]) == want[2]
    u = rng.uniform_pm1(123, 100000)
    assert u.min() >= -1.0 and u.max() < 1.0 and abs(u.mean()) < 0.01


def test_tt_svd_roundtrip_and_full():
    r = np.random.default_rng(0)
    T = r.standard_normal((3, 4, 2, 5))
    cores = tt.tt_svd(T, [3, 4, 2, 5], eps=1e-15)
    assert np.allclose(tt.tt_full(cores), T.reshape(-1), atol=1e-13)
    idx = np.array([[0, 1, 1, 4], [2, 3, 0, 0]])
    assert np.allclose(tt.tt_eval(cores, idx), [T[0, 1, 1, 4], T[2, 3, 0, 0]])


@pytest.mark.parametrize("d", [3, 6, 9])
def test_known_qtt_ranks(d):
    """The index function i -> i and sin(pi i h) have QTT rank 2 (mesh-grid TTs of Sec. 5.1)."""
    n = 2 ** d
    for v in (np.arange(n, dtype=float), np.sin(np.pi * np.arange(n) / (n - 1))):
        cores = qtt.vector_qtt(v, d, eps=1e-10)
        ranks = [C.shape[2] for C in cores[:-1]]
        assert max(ranks) == 2
        assert np.allclose(tt.tt_full(cores), v, atol=1e-10 * np.abs(v).max())
    # the 2D mesh grid X(i, j) = i has rank <= 2 in the interleaved level format
    X = np.add.outer(np.arange(n), np.zeros(n))
    Xl = X.reshape([2] * (2 * d)).transpose([x for l in range(d) for x in (l, d + l)]).reshape([4] * d)
    cores = tt.tt_svd(Xl, [4] * d, eps=1e-10)
    assert max(C.shape[2] for C in cores[:-1]) == 2
    # e_0 e_0^T has rank 1
    E = np.zeros((n, n)); E[0, 0] = 1
    assert max(C.shape[3] for C in qtt.matrix_qtt(E, d)) == 1


def test_round_error_bound_and_algebra():
    r = np.random.default_rng(1)
    modes = [2, 3, 4, 3, 2]
    x = [r.standard_normal((a, n, b)) for a, n, b in zip([1, 2, 4, 5, 3], modes, [2, 4, 5, 3, 1])]
    y = [r.standard_normal((a, n, b)) for a, n, b in zip([1, 3, 3, 3, 2], modes, [3, 3, 3, 2, 1])]
    xf, yf = tt.tt_full(x), tt.tt_full(y)
    s = tt.tt_add(x, y, 2.0, -0.5)
    assert np.allclose(tt.tt_full(s), 2 * xf - 0.5 * yf)
    assert tt.tt_dot(x, y) == pytest.approx(xf @ yf, rel=1e-12)
    for eps in (1e-1, 1e-3):
        xr = tt.tt_round(x, eps=eps)
        assert np.linalg.norm(tt.tt_full(xr) - xf) <= eps * np.linalg.norm(xf) * (1 + 1e-12)
    # exact rounding does not change the tensor and cannot exceed the full-rank bound
    xr = tt.tt_round(tt.tt_add(x, x), eps=1e-15)
    assert np.allclose(tt.tt_full(xr), 2 * xf)
    assert [C.shape[2] for C in xr] == [C.shape[2] for C in tt.tt_round(x, eps=1e-15)]
    # MPO matvec against dense
    A = [r.standard_normal((a, n, n, b)) for a, n, b in zip([1, 2, 2, 3, 2], modes, [2, 2, 3, 2, 1])]
    Af = tt.mpo_full(A)
    assert np.allclose(tt.tt_full(tt.mpo_matvec(A, x)), Af @ xf)
    assert tt.tt_rel_diff(x, x) < 1e-12


def test_random_tt_shapes():
    cores = rng.random_tt([3, 8, 8, 8], 4, seed=5)
    assert [C.shape for C in cores] == [(1, 3, 3), (3, 8, 4), (4, 8, 4), (4, 8, 1)]
    flat = np.concatenate([C.reshape(-1) for C in cores])
    assert np.array_equal(flat, rng.uniform_pm1(5, flat.size))
