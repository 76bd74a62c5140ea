"""Seeded problem descriptions (shapes of the paper's workloads; no solver arithmetic).

Every generator returns a plain dict understood by the library binding and by
any other consumer.  Random draws use numpy.random.default_rng(seed).
"""
from __future__ import annotations

import numpy as np


def small_2d():
    """2D plane strain on the unit square, 32 x 32 nodes (QTT level 5), E = 1, nu = 0.3,
    left edge clamped, uniform x-traction 1.0 on the right edge."""
    return dict(dim=2, level=5, E=1.0, nu=0.3, clamp=[(0, 0)], tractions=[(0, 1, [1.0, 0.0])])


def cube_body_force(level: int = 7):
    """3D unit cube, 2^level nodes per axis, E = 1, nu = 0.3, face x = 0 clamped,
    uniform body force (0, 0, -1)."""
    return dict(dim=3, level=level, E=1.0, nu=0.3, clamp=[(0, 0)], body_force=[0.0, 0.0, -1.0])


def cube_manufactured(level: int = 10, seed: int = 0):
    """3D unit cube, all faces clamped, load of the manufactured field
    u_i = c_i sin(pi x) sin(pi y) sin(pi z), c ~ N(0, 1) drawn from `seed`."""
    c = np.random.default_rng(seed).standard_normal(3)
    faces = [(a, s) for a in range(3) for s in (0, 1)]
    return dict(dim=3, level=level, E=1.0, nu=0.3, clamp=faces, manufactured_c=[float(v) for v in c])


def layered_cube(level: int = 9):
    """3D cube with 8 slabs along z alternating E = 1 and E = 10 (slab of element e_z is
    e_z // 2^(level-3)), nu = 0.3, base z = 0 clamped, top pressure 1.0."""
    ne = 2 ** level - 1
    slab = np.arange(ne) // (2 ** (level - 3))
    E = np.where(slab % 2 == 1, 10.0, 1.0)
    return dict(dim=3, level=level, E=1.0, nu=0.3, clamp=[(2, 0)], tractions=[(2, 1, [0.0, 0.0, -1.0])],
                layered_E=(2, E.tolist()))


def random_anisotropic_voigt(dim: int, seed: int = 0):
    """A seeded symmetric positive definite stiffness in Voigt notation (3 x 3 in 2D, 6 x 6 in
    3D): an isotropic part (E = 1, nu = 0.3 scale) plus a random symmetric perturbation that
    couples normal and shear components, as a fully anisotropic crystal does."""
    rng = np.random.default_rng(seed)
    nv = 3 if dim == 2 else 6
    Bm = rng.standard_normal((nv, nv))
    C = 0.3 * Bm @ Bm.T / nv + np.eye(nv)
    C[:dim, :dim] += 0.5
    return C.tolist()


def orthotropic_voigt(dim: int, E1: float, E2: float, E3: float = 1.0, nu: float = 0.25, G: float = 0.4):
    """Orthotropic stiffness aligned with the axes (Voigt), from its compliance: diagonal
    1/E_a, off-diagonal -nu/E_a, shear 1/G."""
    E = [E1, E2, E3][:dim]
    nv = 3 if dim == 2 else 6
    S = np.zeros((nv, nv))
    for a in range(dim):
        for b in range(dim):
            S[a, b] = 1.0 / E[a] if a == b else -nu / max(E[a], E[b])
    for k in range(dim, nv):
        S[k, k] = 1.0 / G
    return np.linalg.inv(S).tolist()


# aluminium cantilever of Sec. 6: density (kg/m^3), gravity (m/s^2)
CANTILEVER_RHO = 2700.0
CANTILEVER_G = 9.81


def cantilever(level: int = 8):
    """2D plane-stress cantilever of Sec. 6: 20 m x 1 m aluminium (E = 68 GPa, nu = 0.33),
    edge x = 0 clamped, loaded by its own weight f = (0, -rho g), 2^level nodes per axis."""
    return dict(dim=2, level=level, E=68e9, nu=0.33, plane_stress=True, extent=[20.0, 1.0], clamp=[(0, 0)],
                body_force=[0.0, -CANTILEVER_RHO * CANTILEVER_G])


def serving_stream(n: int = 256, seed: int = 0, rate: float = 1.0):
    """Requests: (arrival time, problem dict, rank cap).  2D/3D with p = 1/2, level
    uniform in 6..10, nu ~ U[0.2, 0.45], E log-uniform in [0.1, 10], face x = 0 clamped,
    traction t ~ N(0, 1)^D on x = 1, rank cap uniform in 32..64 rounded up to 16."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    out = []
    for i in range(n):
        D = 2 if rng.random() < 0.5 else 3
        level = int(rng.integers(6, 11))
        nu = float(rng.uniform(0.2, 0.45))
        E = float(10.0 ** rng.uniform(-1.0, 1.0))
        tr = rng.standard_normal(D)
        cap = int(rng.integers(32, 65))
        cap = int(-(-cap // 16) * 16)
        prob = dict(dim=D, level=level, E=E, nu=nu, clamp=[(0, 0)], tractions=[(0, 1, [float(v) for v in tr])])
        out.append((float(t[i]), prob, cap))
    return out
