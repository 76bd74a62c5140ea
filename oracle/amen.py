"""O2 -- a plain alternating minimal-energy (AMEn) sweep for A u = b (oracle).

Alg. 2 of the paper solves A u = M f0 with the AMEn solver of Dolgov and
Savostyanov (2014); the paper names the method and no parameters.  This module
writes the method out step by step with numpy tensor contractions and LAPACK, in the order
below, which the GPU library follows as well (the readings of every constant
the paper leaves open are listed in the design doc):

  * start: X = random rank-2 TT, Z = random rank-rho TT (SplitMix64 draws);
    orthogonalise both from the right and build the right interfaces;
  * half-sweep over the cores k = 0 .. K-1 (a "sweep" alternates direction;
    the right-to-left half-sweep is the same step on the reversed chain):
      g   = local right-hand side  (Phi_b,L  B_k  Phi_b,R)
      B   = local operator          (Phi_A,L  A_k  Phi_A,R), symmetric
      res = ||g - B x_k|| / ||g||
      if res > tol/2: preconditioned CG from x_k until
            ||g - B x|| <= max(0.1 res, tol/2) ||g||; the preconditioner is
            block Jacobi over the mode index: for every pair (a, c) of left and
            right interface indices the n x n diagonal block B[(a,:,c),(a,:,c)]
            is inverted
      if k < K-1:
        SVD of the (r_k n_k) x r_{k+1} unfolding, keep the smallest rank whose
            discarded tail is <= tol/sqrt(K-1) of the norm, at most rank_cap;
        z_k = projection of the residual b - A x~ on the Z interfaces, QR;
        e   = residual b - A x~ projected on (left X, right Z) interfaces;
        [U | e] -> QR -> new core X_k, carry Q^T x~ into X_{k+1}
            (at most rank_cap columns in total);
        update the four left interfaces.
  * stop after a half-sweep with max_k res_k <= tol, or after max_sweeps.

Parity: tests/test_oracle_amen.py pins it to the sparse direct solve of
oracle.fem on small grids (unconstrained rank), to the scaling law
u(sE) = u(E)/s, to superposition of loads and to the mirror symmetry of a
symmetric problem; with a binding rank cap to ranks <= cap on every bond after
every step and to the energy J(x) = x^T A x / 2 - b^T x never rising across a
local solve (computed from the dense reconstruction on tiny grids).  pcg is
pinned to a dense solve, local_block to the blocks cut from the densely built
local operator.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import rng


# ----------------------------------------------------------------------------- local contractions
# Shapes: left interface L[p, R, q]; MPO core A[R, n_out, n_in, R']; x[q, n, s];
# right interface Rt[t, R', s]; result [p, n, t].

def local_apply(L, A, x, Rt):
    """y[p, j, t] = sum L[p, b, q] A[b, j, i, e] x[q, i, s] Rt[t, e, s], in three stages."""
    T1 = np.tensordot(L, x, axes=([2], [0]))            # [p, b, i, s]
    T2 = np.tensordot(T1, A, axes=([1, 2], [0, 2]))     # [p, s, j, e]
    return np.tensordot(T2, Rt, axes=([3, 1], [1, 2]))  # [p, j, t]


def local_rhs(Lb, B, Rb):
    """g[p, j, u] = sum Lb[p, s] B[s, j, t] Rb[u, t]."""
    return np.tensordot(np.tensordot(Lb, B, axes=([1], [0])), Rb, axes=([2], [1]))


def env_A(L, W, A, X):
    """Next left interface: sum W[p, j, t] L[p, b, q] A[b, j, i, e] X[q, i, s] -> [t, e, s]."""
    T1 = np.tensordot(L, X, axes=([2], [0]))             # [p, b, i, s]
    T2 = np.tensordot(T1, A, axes=([1, 2], [0, 2]))      # [p, s, j, e]
    return np.tensordot(W, T2, axes=([0, 1], [0, 2])).transpose(0, 2, 1)  # [t, e, s]


def env_b(Lb, W, B):
    """Next left load interface: sum W[p, j, t] Lb[p, s] B[s, j, u] -> [t, u]."""
    T = np.tensordot(Lb, B, axes=([1], [0]))             # [p, j, u]
    return np.tensordot(W, T, axes=([0, 1], [0, 1]))


def local_block(L, A, Rt):
    """Diagonal blocks of the local operator over the mode index:
    blk[a, c, j, i] = sum_{b,e} L[a, b, a] A[b, j, i, e] Rt[c, e, c]."""
    La = np.einsum("aba->ab", L)
    Rc = np.einsum("cec->ce", Rt)
    return np.einsum("ab,bjie,ce->acji", La, A, Rc)


def block_preconditioner(blk):
    """r -> z with z[a, :, c] = blk[a, c]^{-1} r[a, :, c] (blocks of an SPD operator are SPD)."""
    def apply(r):
        rr = r.transpose(0, 2, 1)[..., None]                # [p, t, n, 1]
        return np.linalg.solve(blk, rr)[..., 0].transpose(0, 2, 1)
    return apply


def pcg(apply, g, x, precond, thr, maxit):
    """Preconditioned conjugate gradients from x until ||g - B x|| <= thr.

    The textbook method (Hestenes and Stiefel, with a preconditioner):
    z = M^{-1} r, p = z + beta p, q = B p, alpha = (r, z) / (p, q),
    x += alpha p, r -= alpha q, beta = (r_new, z_new) / (r, z); one product with
    B per iteration.  precond(r) returns z.
    """
    r = g - apply(x)
    z = precond(r)
    p = np.zeros_like(r)
    beta = 0.0
    rz = float(np.vdot(r, z))
    it = 0
    while it < maxit and np.linalg.norm(r) > thr:
        p = z + beta * p
        q = apply(p)
        pq = float(np.vdot(p, q))
        if pq <= 0.0:
            break
        alpha = rz / pq
        x = x + alpha * p
        r = r - alpha * q
        z = precond(r)
        rz_new = float(np.vdot(r, z))
        beta = rz_new / rz
        rz = rz_new
        it += 1
    return x, it


def truncation_rank(s, tol_rel, cap):
    """Smallest r with ||s[r:]|| <= tol_rel ||s||, clipped to [1, cap]."""
    tot = float(np.sum(s ** 2))
    tail = 0.0
    r = len(s)
    for j in range(len(s) - 1, -1, -1):  # tail sums from the smallest value up
        if tail + s[j] ** 2 <= (tol_rel ** 2) * tot:
            tail += s[j] ** 2
            r = j
        else:
            break
    return max(1, min(r, cap))


# ----------------------------------------------------------------------------- state

@dataclasses.dataclass
class Options:
    tol: float = 1e-8
    rank_cap: int = 32
    rho: int = 4
    max_sweeps: int = 30
    init_rank: int = 2
    seed_x: int = 1
    seed_z: int = 2
    cg_maxit: int = 500


@dataclasses.dataclass
class Stats:
    sweeps: int = 0
    max_res: list = dataclasses.field(default_factory=list)
    cg_iters: int = 0
    applies: int = 0
    ranks: list = dataclasses.field(default_factory=list)


class _Chain:
    """Cores of A, b, X, Z and the interfaces on every bond, in one orientation."""

    def __init__(self, A, b, X, Z):
        self.A = [C.copy() for C in A]
        self.B = [C.copy() for C in b]
        self.X = [C.copy() for C in X]
        self.Z = [C.copy() for C in Z]
        K = len(A)
        one3 = np.ones((1, 1, 1))
        one2 = np.ones((1, 1))
        self.LA = [one3] + [None] * (K - 1) + [one3]
        self.Lb = [one2] + [None] * (K - 1) + [one2]
        self.LzA = [one3] + [None] * (K - 1) + [one3]
        self.Lzb = [one2] + [None] * (K - 1) + [one2]
        self.reversed = False

    def reverse(self):
        self.A = [C.transpose(3, 1, 2, 0) for C in self.A[::-1]]
        self.B = [C.transpose(2, 1, 0) for C in self.B[::-1]]
        self.X = [C.transpose(2, 1, 0) for C in self.X[::-1]]
        self.Z = [C.transpose(2, 1, 0) for C in self.Z[::-1]]
        self.LA, self.Lb = self.LA[::-1], self.Lb[::-1]
        self.LzA, self.Lzb = self.LzA[::-1], self.Lzb[::-1]
        self.reversed = not self.reversed

    def forward_cores(self):
        """Cores of the current iterate in the forward (unreversed) chain order."""
        if self.reversed:
            return [C.transpose(2, 1, 0).copy() for C in self.X[::-1]]
        return [C.copy() for C in self.X]

    def update_envs(self, k):
        A, B, X, Z = self.A[k], self.B[k], self.X[k], self.Z[k]
        self.LA[k + 1] = env_A(self.LA[k], X, A, X)
        self.Lb[k + 1] = env_b(self.Lb[k], X, B)
        self.LzA[k + 1] = env_A(self.LzA[k], Z, A, X)
        self.Lzb[k + 1] = env_b(self.Lzb[k], Z, B)

    def qr_pass(self):
        """Left-orthogonalise X and Z and build the left interfaces."""
        K = len(self.A)
        for k in range(K - 1):
            for T in (self.X, self.Z):
                r, n, r2 = T[k].shape
                Q, R = np.linalg.qr(T[k].reshape(r * n, r2))
                T[k] = Q.reshape(r, n, -1)
                T[k + 1] = np.einsum("ab,bnc->anc", R, T[k + 1])
            self.update_envs(k)


def _half_sweep(ch: _Chain, opt: Options, st: Stats, observe=None):
    K = len(ch.A)
    tol = opt.tol
    tr_tol = tol / np.sqrt(max(K - 1, 1))
    max_res = 0.0
    for k in range(K):
        L, A, Rt = ch.LA[k], ch.A[k], ch.LA[k + 1]
        g = local_rhs(ch.Lb[k], ch.B[k], ch.Lb[k + 1])
        x = ch.X[k]

        def apply(v):
            st.applies += 1
            return local_apply(L, A, v, Rt)

        gn = np.linalg.norm(g)
        res0 = np.linalg.norm(g - apply(x))
        res = res0 / gn if gn > 0 else (0.0 if res0 == 0 else 1.0)
        max_res = max(max_res, res)
        if observe is not None:
            observe("before_solve", k, ch.forward_cores())
        if res > 0.5 * tol:
            precond = block_preconditioner(local_block(L, A, Rt))
            thr = max(0.1 * res, 0.5 * tol) * gn
            x, it = pcg(apply, g, x, precond, thr, opt.cg_maxit)
            st.cg_iters += it
        if observe is not None:
            ch.X[k] = x
            observe("after_solve", k, ch.forward_cores())
        if k == K - 1:
            ch.X[k] = x
            break
        r, n, r2 = x.shape
        U, s, Vt = np.linalg.svd(x.reshape(r * n, r2), full_matrices=False)
        rk = truncation_rank(s, tr_tol, opt.rank_cap)
        xt = (U[:, :rk] * s[:rk]) @ Vt[:rk]
        xt3 = xt.reshape(r, n, r2)
        # residual projected on the Z interfaces -> new Z_k
        zt = local_rhs(ch.Lzb[k], ch.B[k], ch.Lzb[k + 1]) - local_apply(ch.LzA[k], A, xt3, ch.LzA[k + 1])
        rz, _, rz2 = zt.shape
        Qz, _ = np.linalg.qr(zt.reshape(rz * n, rz2))
        ch.Z[k] = Qz.reshape(rz, n, -1)
        # enrichment: residual on (left X, right Z) interfaces
        e = local_rhs(ch.Lb[k], ch.B[k], ch.Lzb[k + 1]) - local_apply(L, A, xt3, ch.LzA[k + 1])
        rho_eff = max(0, min(e.shape[2], opt.rank_cap - rk, r * n - rk))
        aug = np.concatenate([U[:, :rk], e.reshape(r * n, -1)[:, :rho_eff]], axis=1)
        Q, _ = np.linalg.qr(aug)
        ch.X[k] = Q.reshape(r, n, -1)
        W = Q.T @ xt
        ch.X[k + 1] = np.einsum("ab,bnc->anc", W, ch.X[k + 1])
        ch.update_envs(k)
    return max_res


def amen_solve(A, b, opt: Options | None = None, after_half_sweep=None, observe=None):
    """Solve A u = b in TT format.  Returns (list of cores of u, Stats).

    after_half_sweep(stats), if given, is called after every half-sweep; a true
    return value ends the sweep loop there (used to time bounded samples).
    observe(event, k, cores), if given, receives copies of the iterate's cores
    (forward order) before and after every local solve ("before_solve",
    "after_solve") and after every half-sweep ("half_sweep", k = -1); it only
    reads (used by the pins of the rank cap and the energy).
    """
    opt = opt or Options()
    modes = [C.shape[1] for C in A]
    X = rng.random_tt(modes, opt.init_rank, opt.seed_x)
    Z = rng.random_tt(modes, opt.rho, opt.seed_z)
    ch = _Chain(A, b, X, Z)
    st = Stats()
    ch.reverse()
    ch.qr_pass()
    ch.reverse()
    for _ in range(opt.max_sweeps):
        mr = _half_sweep(ch, opt, st, observe)
        st.sweeps += 1
        st.max_res.append(mr)
        if observe is not None:
            observe("half_sweep", -1, ch.forward_cores())
        ch.reverse()
        if mr <= opt.tol:
            break
        if after_half_sweep is not None and after_half_sweep(st):
            break
    if ch.reversed:
        ch.reverse()
    st.ranks = [C.shape[0] for C in ch.X] + [1]
    return ch.X, st
