"""Tensor-train primitives (Sec. 4) for the oracle, written for clarity not speed.

A TT vector (matrix product state, fig. ttvec) is a list of cores C_k of shape
[r_k, n_k, r_{k+1}] with r_0 = r_K = 1; entry (i_0, ..., i_{K-1}) is the matrix
product C_0[:, i_0, :] ... C_{K-1}[:, i_{K-1}, :].  A TT operator (matrix
product operator, fig. ttop) has cores [R_k, m_k, n_k, R_{k+1}], output
(row) index before input (column) index.

Flattening of multi-indices is row-major with the first core most significant,
which for QTT folding is the binary expansion i = sum_k i_k 2^(d-1-k) of Sec. 4.

Parity: pinned in tests/test_oracle_tt.py against dense numpy arrays, known
exact ranks (the index function i -> i has rank 2, Sec. 5.1) and LAPACK.
"""
from __future__ import annotations

import numpy as np


# ----------------------------------------------------------------------------- dense views

def tt_full(cores):
    """Dense vector of a TT (row-major over the core indices)."""
    v = np.ones((1, 1))
    for C in cores:
        r, n, r2 = C.shape
        v = (v @ C.reshape(r, n * r2)).reshape(-1, r2)
    return v.reshape(-1)


def mpo_full(cores):
    """Dense matrix of a TT operator: rows = flattened output indices."""
    T = np.ones((1, 1, 1))  # [rows, cols, rank]
    for C in cores:
        R, m, n, R2 = C.shape
        T = np.einsum("abr,rmns->ambns", T, C).reshape(T.shape[0] * m, T.shape[1] * n, R2)
    return T[:, :, 0]


def tt_shape(cores):
    return [C.shape[1] for C in cores], [C.shape[0] for C in cores] + [cores[-1].shape[2]]


# ----------------------------------------------------------------------------- decompositions

def _trunc_rank(s, delta, rmax):
    """Smallest rank r with sum_{j>=r} s_j^2 <= delta^2 (at least 1, at most rmax)."""
    tail = np.sqrt(np.cumsum((s ** 2)[::-1]))[::-1]  # tail[j] = ||s[j:]||
    r = len(s)
    for j in range(len(s)):
        if tail[j] <= delta:
            r = j
            break
    r = max(r, 1)
    if rmax is not None:
        r = min(r, rmax)
    return r


def tt_svd(tensor, modes, eps=1e-14, rmax=None):
    """TT-SVD of a dense tensor with the given mode sizes (Oseledets 2011).

    Relative Frobenius accuracy eps: each of the K-1 truncations drops at most
    eps / sqrt(K-1) of the norm.
    """
    K = len(modes)
    A = np.asarray(tensor, dtype=np.float64).reshape(modes)
    delta = eps * np.linalg.norm(A) / np.sqrt(max(K - 1, 1))
    cores = []
    r = 1
    rest = A.reshape(1, -1)
    for k in range(K - 1):
        mat = rest.reshape(r * modes[k], -1)
        U, s, Vt = np.linalg.svd(mat, full_matrices=False)
        rk = _trunc_rank(s, delta, rmax)
        cores.append(U[:, :rk].reshape(r, modes[k], rk))
        rest = s[:rk, None] * Vt[:rk]
        r = rk
    cores.append(rest.reshape(r, modes[-1], 1))
    return cores


def tt_orthogonalize_right(cores):
    """Right-to-left sweep of LQ steps: cores 1.. become right-orthogonal."""
    cores = [C.copy() for C in cores]
    for k in range(len(cores) - 1, 0, -1):
        r, n, r2 = cores[k].shape
        Q, R = np.linalg.qr(cores[k].reshape(r, n * r2).T)
        cores[k] = Q.T.reshape(-1, n, r2)
        cores[k - 1] = np.tensordot(cores[k - 1], R, axes=([2], [1]))  # [a, n, c] = sum_b core[a, n, b] R[c, b]
    return cores


def tt_round(cores, eps=1e-14, rmax=None):
    """TT rounding: right-orthogonalize, then truncated SVDs left to right."""
    K = len(cores)
    cores = tt_orthogonalize_right(cores)
    nrm = np.linalg.norm(cores[0])
    delta = eps * nrm / np.sqrt(max(K - 1, 1))
    for k in range(K - 1):
        r, n, r2 = cores[k].shape
        U, s, Vt = np.linalg.svd(cores[k].reshape(r * n, r2), full_matrices=False)
        rk = _trunc_rank(s, delta, rmax)
        cores[k] = U[:, :rk].reshape(r, n, rk)
        cores[k + 1] = np.tensordot(s[:rk, None] * Vt[:rk], cores[k + 1], axes=([1], [0]))
    return cores


# ----------------------------------------------------------------------------- algebra

def tt_add(x, y, alpha=1.0, beta=1.0):
    """alpha x + beta y as a TT whose ranks are the sums of the ranks."""
    K = len(x)
    if K == 1:
        return [alpha * x[0] + beta * y[0]]
    out = []
    for k in range(K):
        a, b = x[k], y[k]
        if k == 0:
            out.append(np.concatenate([alpha * a, beta * b], axis=2))
        elif k == K - 1:
            out.append(np.concatenate([a, b], axis=0))
        else:
            C = np.zeros((a.shape[0] + b.shape[0], a.shape[1], a.shape[2] + b.shape[2]))
            C[: a.shape[0], :, : a.shape[2]] = a
            C[a.shape[0]:, :, a.shape[2]:] = b
            out.append(C)
    return out


def mpo_as_tt(A):
    """View an operator as a TT vector over the fused (out, in) index."""
    return [C.reshape(C.shape[0], C.shape[1] * C.shape[2], C.shape[3]) for C in A]


def tt_as_mpo(cores, m_modes, n_modes):
    return [C.reshape(C.shape[0], m, n, C.shape[2]) for C, m, n in zip(cores, m_modes, n_modes)]


def mpo_add(A, B, alpha=1.0, beta=1.0):
    m = [C.shape[1] for C in A]
    n = [C.shape[2] for C in A]
    return tt_as_mpo(tt_add(mpo_as_tt(A), mpo_as_tt(B), alpha, beta), m, n)


def mpo_round(A, eps=1e-14, rmax=None):
    m = [C.shape[1] for C in A]
    n = [C.shape[2] for C in A]
    return tt_as_mpo(tt_round(mpo_as_tt(A), eps, rmax), m, n)


def tt_dot(x, y):
    """Euclidean inner product <x, y> of two TTs, by left-to-right contraction."""
    E = np.ones((1, 1))
    for a, b in zip(x, y):
        T = np.tensordot(E, a, axes=([0], [0]))           # [b, n, c]
        E = np.tensordot(T, b, axes=([0, 1], [0, 1]))     # [c, d]
    return float(E[0, 0])


def tt_norm(x):
    return float(np.sqrt(max(tt_dot(x, x), 0.0)))


def mpo_matvec(A, x):
    """Exact product A x as a TT with ranks R_k r_k."""
    out = []
    for C, X in zip(A, x):
        R, m, n, R2 = C.shape
        r, _, r2 = X.shape
        Y = np.tensordot(C, X, axes=([2], [1]))            # [R, m, R2, r, r2]
        Y = Y.transpose(0, 3, 1, 2, 4).reshape(R * r, m, R2 * r2)
        out.append(Y)
    return out


def tt_scale(x, alpha):
    out = [C.copy() for C in x]
    out[0] = out[0] * alpha
    return out


def tt_rel_diff(x, y):
    """||x - y|| / ||y|| computed in TT format (no densification)."""
    diff = tt_round(tt_add(x, y, 1.0, -1.0), eps=1e-15)
    ny = tt_norm(y)
    return tt_norm(diff) / ny if ny > 0 else tt_norm(diff)


def tt_eval(cores, idx):
    """Entries of a TT at integer multi-indices idx[num, K]."""
    idx = np.asarray(idx)
    v = np.ones((idx.shape[0], 1))
    for k, C in enumerate(cores):
        v = np.einsum("pa,pab->pb", v, C[:, idx[:, k], :].transpose(1, 0, 2))
    return v[:, 0]
