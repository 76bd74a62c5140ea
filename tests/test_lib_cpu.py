"""Host-side checks of the C-ABI library (no GPU): exports, assembly parity, errors."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import fem, qtt, tt
from paper_2501_12151_amd import tnfem, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "tnfem.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tnfem_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = _declared_functions()
    assert len(names) >= 20
    lib = ctypes.CDLL(tnfem.LIB_PATH)
    for nm in names:
        assert hasattr(lib, nm), nm
    assert set(names) == set(tnfem.EXPORTED)


CASES = [
    dict(dim=2, level=3, E=1.0, nu=0.3, clamp=[(0, 0)], tractions=[(0, 1, [1.0, 0.0])]),
    dict(dim=2, level=4, E=68.0, nu=0.33, plane_stress=True, clamp=[(0, 0)], body_force=[0.0, -1.0], extent=[20.0, 1.0]),
    dict(dim=2, level=4, E=2.0, nu=0.25, clamp=[(0, 0), (0, 1), (1, 0), (1, 1)], manufactured_c=[0.7, -0.4]),
    dict(dim=2, level=2, E=1.0, nu=0.2, clamp=[], tractions=[(1, 0, [0.5, 1.0]), (1, 1, [0.5, -1.0])]),
    dict(dim=3, level=2, E=1.0, nu=0.3, clamp=[(0, 0)], body_force=[0.0, 0.0, -1.0]),
    dict(dim=3, level=3, E=0.5, nu=0.4, clamp=[(2, 0), (0, 1)], tractions=[(2, 1, [0, 0, -1.0]), (0, 1, [0.3, 0.2, 0.1])],
         body_force=[0.1, 0.2, 0.3], extent=[2.0, 1.0, 0.5]),
    dict(dim=3, level=2, E=1.0, nu=0.3, clamp=[(a, s) for a in range(3) for s in (0, 1)], manufactured_c=[0.5, 1.0, -0.3]),
    # anisotropic materials: constant Voigt stiffness (one with slabs of it)
    dict(dim=2, level=3, E=1.0, nu=0.3, clamp=[(0, 0)], tractions=[(0, 1, [1.0, 0.3])], extent=[2.0, 1.0],
         stiffness_voigt=workloads.random_anisotropic_voigt(2, 1)),
    dict(dim=3, level=3, E=1.0, nu=0.3, clamp=[(0, 0), (1, 1)], body_force=[0.0, 0.5, -1.0],
         stiffness_voigt=workloads.random_anisotropic_voigt(3, 2)),
    dict(dim=3, level=3, E=2.0, nu=0.3, clamp=[(2, 0)], tractions=[(2, 1, [0.0, 0.0, -1.0])],
         layered_E=(2, [2.0, 2.0, 20.0, 20.0, 2.0, 2.0, 20.0]), stiffness_voigt=workloads.orthotropic_voigt(3, 1.0, 3.0, 0.5)),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_library_assembly_equals_sparse_fem(case):
    """The library's QTT operator and load, reconstructed densely, equal the sparse assembly."""
    prob = CASES[case]
    A, b, grid, info = fem.build_system(prob)
    D, d = prob["dim"], prob["level"]
    Ac = tnfem.export_operator(prob)
    bc = tnfem.export_load(prob)
    Ap = qtt.matrix_to_qtt_order(A, D, d).toarray()
    assert np.abs(tt.mpo_full(Ac) - Ap).max() <= 1e-13 * np.abs(Ap).max()
    bp = qtt.to_qtt_order(b, D, d)
    assert np.abs(tt.tt_full(bc) - bp).max() <= 1e-13 * np.abs(bp).max()
    # exact automaton ranks: 5^D joint carry states in the middle (7 on a layered axis)
    assert max(C.shape[3] for C in Ac) <= (7 * 5 ** (D - 1) if "layered_E" in prob else 5 ** D)


def _random_nodal_tt(D, d, rank, seed):
    """Seeded TT of nodal force values in the solution layout (levels, then component)."""
    rng = np.random.default_rng(seed)
    modes = [2 ** D] * d + [D]
    ranks = [1] + [rank] * d + [1]
    return [rng.standard_normal((ranks[k], modes[k], ranks[k + 1])) for k in range(d + 1)]


NODAL_CASES = [
    dict(dim=2, level=4, E=1.0, nu=0.3, clamp=[(0, 0)]),
    dict(dim=2, level=3, E=2.0, nu=0.25, clamp=[(0, 0), (0, 1), (1, 0), (1, 1)], extent=[3.0, 0.5],
         body_force=[0.2, -1.0]),
    dict(dim=3, level=3, E=1.0, nu=0.3, clamp=[(2, 0), (1, 1)], tractions=[(2, 1, [0.0, 0.0, -1.0])]),
    dict(dim=3, level=2, E=1.0, nu=0.3, clamp=[], extent=[1.0, 2.0, 0.5]),
]


@pytest.mark.parametrize("case", range(len(NODAL_CASES)))
def test_nodal_load_through_the_c_abi_equals_sparse_mass_product(case):
    """A non-constant nodal load f0 (a random rank-3 TT; Alg. 2, Sec. 5.3) handed through
    the C ABI: the library's load equals P M f0 of the sparse assembly (plus the other
    loads of the case)."""
    prob = dict(NODAL_CASES[case])
    D, d = prob["dim"], prob["level"]
    prob["f_nodal_tt"] = _random_nodal_tt(D, d, 3, seed=case)
    _, b, _, _ = fem.build_system(prob)
    bp = qtt.to_qtt_order(b, D, d)
    bl = tt.tt_full(tnfem.export_load(prob))
    assert np.abs(bl - bp).max() <= 1e-12 * np.abs(bp).max()
    # the oracle's QTT load of the same description agrees as well
    assert np.abs(tt.tt_full(qtt.assemble_load(prob)) - bp).max() <= 1e-12 * np.abs(bp).max()


def test_constant_nodal_load_equals_body_force():
    """f0 = constant vector at every node reproduces the body-force load exactly."""
    f = [0.3, -1.0, 0.5]
    base = dict(dim=3, level=4, E=1.0, nu=0.3, clamp=[(0, 0), (2, 1)])
    ones = [np.ones((1, 8, 1)) for _ in range(4)] + [np.asarray(f).reshape(1, 3, 1)]
    b1 = tt.tt_full(tnfem.export_load(dict(base, body_force=f)))
    b2 = tt.tt_full(tnfem.export_load(dict(base, f_nodal_tt=ones)))
    assert np.abs(b1 - b2).max() <= 1e-13 * np.abs(b1).max()


@pytest.mark.parametrize("ranks", [[2, 1, 1, 1], [1, 0, 1, 1], [1, 5000, 1, 1], [1, 1, 1, 3]])
def test_nodal_load_rejects_bad_ranks(ranks):
    """Ranks are validated before any core is read (d + 2 = 4 ranks at level 2)."""
    prob = dict(dim=2, level=2, E=1.0, nu=0.3, clamp=[(0, 0)],
                f_nodal_tt=[np.ones((1, 4, 1)), np.ones((1, 4, 1)), np.ones((1, 2, 1))])
    desc = tnfem.make_desc(prob)
    r = (ctypes.c_int * 4)(*ranks)
    desc.f0_ranks = ctypes.cast(r, ctypes.POINTER(ctypes.c_int))
    nc, need = ctypes.c_int(), ctypes.c_size_t()
    modes, rk = (ctypes.c_int * 64)(), (ctypes.c_int * 65)()
    rc = tnfem._lib.tnfem_export_load(ctypes.byref(desc), ctypes.byref(nc), modes, rk, None, 0, ctypes.byref(need))
    assert rc == tnfem.EINVAL


TRAPEZOID = [[0.0, 0.0], [2.0, 0.0], [0.0, 1.0], [1.4, 0.7]]
QUAD_CASES = [
    dict(dim=2, level=2, E=1.0, nu=0.3, quad=TRAPEZOID, clamp=[], body_force=[0.0, -1.0]),
    dict(dim=2, level=3, E=1.0, nu=0.3, quad=TRAPEZOID, clamp=[(0, 0)], tractions=[(0, 1, [0.3, -1.0])],
         body_force=[0.1, -1.0]),
    dict(dim=2, level=3, E=68.0, nu=0.33, plane_stress=True, quad=[[0.0, 0.0], [4.0, 0.5], [0.2, 1.0], [3.6, 1.4]],
         clamp=[(0, 0), (1, 0)], tractions=[(1, 1, [0.0, -2.0])]),
    dict(dim=2, level=3, E=1.0, nu=0.3, quad=TRAPEZOID, clamp=[(0, 1)], stiffness_voigt=workloads.random_anisotropic_voigt(2, 4),
         f_nodal_tt=[np.full((1, 4, 1), 0.5), np.full((1, 4, 1), 1.0), np.full((1, 4, 1), -1.0), np.array([[[0.2], [1.0]]])]),
    dict(dim=2, level=4, E=2.0, nu=0.25, quad=TRAPEZOID, clamp=[(0, 0), (1, 1)], tractions=[(1, 0, [0.0, -1.0])]),
]


@pytest.mark.parametrize("case", range(len(QUAD_CASES)))
def test_quadrilateral_assembly_equals_sparse_fem(case):
    """Alg. 1 in full on a quadrilateral (element Jacobians at the centres, fields in QTT,
    corner-pair automata): the library's operator and load equal the oracle's
    element-by-element sparse assembly with the same rule."""
    prob = QUAD_CASES[case]
    A, b, grid, info = fem.build_system(prob)
    D, d = 2, prob["level"]
    Ac = tnfem.export_operator(prob)
    bc = tnfem.export_load(prob)
    Ap = qtt.matrix_to_qtt_order(A, D, d).toarray()
    assert np.abs(tt.mpo_full(Ac) - Ap).max() <= 1e-12 * np.abs(Ap).max()
    bp = qtt.to_qtt_order(b, D, d)
    assert np.abs(tt.tt_full(bc) - bp).max() <= 1e-12 * np.abs(bp).max()


def _inclusion(level, value=10.0):
    """Per-element weights: value inside a disk of radius 0.3 at (0.55, 0.45), 1 outside."""
    ne = 2 ** level - 1
    c = (np.arange(ne) + 0.5) / ne
    X, Y = np.meshgrid(c, c, indexing="ij")
    return np.where((X - 0.55) ** 2 + (Y - 0.45) ** 2 < 0.09, value, 1.0)


WEIGHT_CASES = [
    dict(dim=2, level=3, E=1.0, nu=0.3, clamp=[(0, 0)], tractions=[(0, 1, [1.0, 0.0])],
         elem_weight=np.random.default_rng(3).uniform(0.2, 5.0, (7, 7))),
    dict(dim=2, level=4, E=1.0, nu=0.3, clamp=[(1, 0)], body_force=[0.0, -1.0], extent=[2.0, 1.0],
         elem_weight=_inclusion(4)),
    dict(dim=2, level=3, E=1.0, nu=0.3, quad=TRAPEZOID, clamp=[(0, 0)], tractions=[(0, 1, [0.3, -1.0])],
         elem_weight=_inclusion(3, 4.0), stiffness_voigt=workloads.orthotropic_voigt(2, 1.0, 3.0)),
]


@pytest.mark.parametrize("case", range(len(WEIGHT_CASES)))
def test_element_field_assembly_equals_sparse_fem(case):
    """A general per-element material field (random, or a stiff disk inclusion) in 2D: the
    library's operator and load equal the oracle's element-by-element assembly."""
    prob = WEIGHT_CASES[case]
    A, b, grid, info = fem.build_system(prob)
    d = prob["level"]
    Ac = tnfem.export_operator(prob)
    Ap = qtt.matrix_to_qtt_order(A, 2, d).toarray()
    assert np.abs(tt.mpo_full(Ac) - Ap).max() <= 1e-12 * np.abs(Ap).max()
    bp = qtt.to_qtt_order(b, 2, d)
    assert np.abs(tt.tt_full(tnfem.export_load(prob)) - bp).max() <= 1e-12 * np.abs(bp).max()


@pytest.mark.parametrize("bad,msg", [
    (dict(quad=[[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]]), "det J"),  # P01 / P11 swapped: twisted
    (dict(quad=TRAPEZOID, dim=3), "2D"),
    (dict(quad=TRAPEZOID, layered_E=(0, [1.0] * 7)), "layer_E"),
    (dict(quad=TRAPEZOID, level=9), "level"),
    (dict(elem_weight=np.ones((6, 6))), "elem_weight"),
    (dict(elem_weight=-np.ones((7, 7))), "elem_weight"),
    (dict(elem_weight=np.ones(49), dim=3), "2D"),
])
def test_invalid_quadrilateral_rejected(bad, msg):
    prob = dict(dim=2, level=3, E=1.0, nu=0.3, clamp=[(0, 0)], body_force=[0.0, -1.0])
    prob.update(bad)
    with pytest.raises(tnfem.TnfemError) as e:
        tnfem.export_operator(prob)
    assert e.value.code == tnfem.EINVAL
    assert msg in str(e.value)


@pytest.mark.parametrize("prob", [dict(workloads.small_2d(), level=8), workloads.cube_body_force(4),
                                  workloads.layered_cube(5)])
def test_library_operator_matches_oracle_tt_at_larger_levels(prob):
    """Beyond dense sizes: bilinear forms w^T A x agree for random TT vectors w, x."""
    Ao = qtt.assemble_operator(prob)
    Al = tnfem.export_operator(prob)
    modes = [C.shape[1] for C in Ao]
    rng = np.random.default_rng(0)
    for trial in range(4):
        x = [rng.standard_normal((1 if k == 0 else 2, n, 1 if k == len(modes) - 1 else 2)) for k, n in enumerate(modes)]
        w = [rng.standard_normal((1 if k == 0 else 2, n, 1 if k == len(modes) - 1 else 2)) for k, n in enumerate(modes)]
        vo = tt.tt_dot(w, tt.mpo_matvec(Ao, x))
        vl = tt.tt_dot(w, tt.mpo_matvec(Al, x))
        scale = np.sqrt(abs(tt.tt_dot(tt.mpo_matvec(Ao, x), tt.mpo_matvec(Ao, x)))) * tt.tt_norm(w)
        assert abs(vo - vl) <= 1e-12 * scale
    bo = qtt.assemble_load(prob)
    bl = tnfem.export_load(prob)
    assert tt.tt_rel_diff(bl, bo) <= 1e-12


@pytest.mark.parametrize("bad,msg", [
    (dict(dim=4), "dim"),
    (dict(nu=0.5), "nu"),
    (dict(level=1), "level"),
    (dict(E=-1.0), "E"),
    (dict(extent=[1.0, 0.0]), "extent"),
    (dict(stiffness_voigt=[[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, -1.0]]), "positive definite"),
    (dict(stiffness_voigt=[[1.0, 0.5, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]]), "symmetric"),
    (dict(stiffness_voigt=[[2.0, 0.5, 0.0], [0.5, 2.0, 0.0], [0.0, 0.0, 1.0]], plane_stress=True), "plane_stress"),
    (dict(stiffness_voigt=[[2.0, 0.5, 0.0], [0.5, 2.0, 0.0], [0.0, 0.0, 1.0]], manufactured_c=[1.0, 0.0]),
     "manufactured"),
])
def test_invalid_descriptor_rejected(bad, msg):
    prob = dict(workloads.small_2d(), **bad)
    with pytest.raises(tnfem.TnfemError) as e:
        tnfem.export_operator(prob)
    assert e.value.code == tnfem.EINVAL
    assert msg in str(e.value)


def _layers(level, L, v0, v1):
    """Per-element weights of one bit (level L, most significant first) of the element index."""
    e = np.arange(2 ** level - 1)
    return np.where((e >> (level - 1 - L)) & 1, v1, v0).tolist()


LAYERED = [
    workloads.layered_cube(3),  # the slab pattern (bit 2 of 3: the last level)
    workloads.layered_cube(4),  # the slab pattern at a middle level
    dict(dim=3, level=3, E=2.0, nu=0.3, clamp=[(2, 0), (2, 1)], body_force=[0.0, 0.0, -1.0],
         layered_E=(2, _layers(3, 0, 2.0, 20.0))),  # first level; both ends of the layered axis clamped
    dict(dim=3, level=3, E=1.0, nu=0.25, clamp=[(0, 0)], tractions=[(0, 1, [0.2, 0.4, -1.0])],
         layered_E=(1, _layers(3, 1, 3.0, 0.5))),  # layered across y, clamp on another axis
    dict(dim=2, level=4, E=1.0, nu=0.3, clamp=[(1, 0)], tractions=[(1, 1, [0.0, -1.0])],
         layered_E=(1, _layers(4, 2, 1.0, 10.0))),
    dict(dim=2, level=4, E=1.0, nu=0.3, clamp=[(0, 0), (1, 1)], tractions=[(0, 1, [1.0, 0.0])],
         layered_E=(0, _layers(4, 3, 4.0, 1.5))),  # the last level, clamped at both ends of two axes
    dict(dim=2, level=3, E=1.0, nu=0.3, clamp=[(0, 0)], tractions=[(0, 1, [1.0, 0.0])],
         layered_E=(0, [2.5] * 7)),  # constant: a rescaled material
]


@pytest.mark.parametrize("case", range(len(LAYERED)))
def test_layered_assembly_equals_sparse_fem(case):
    """Young's modulus varying by one bit of the element index along an axis: the library's
    weighted automaton operator equals the sparse FEM assembly with per-element E."""
    prob = LAYERED[case]
    A, b, grid, info = fem.build_system(prob)
    D, d = prob["dim"], prob["level"]
    Ac = tnfem.export_operator(prob)
    Ap = qtt.matrix_to_qtt_order(A, D, d).toarray()
    assert np.abs(tt.mpo_full(Ac) - Ap).max() <= 1e-13 * np.abs(Ap).max()
    bp = qtt.to_qtt_order(b, D, d)
    assert np.abs(tt.tt_full(tnfem.export_load(prob)) - bp).max() <= 1e-13 * np.abs(bp).max()
    assert max(C.shape[3] for C in Ac) <= 7 * 5 ** (D - 1)  # two extra states on the layered axis


def test_unsupported_layering_rejected():
    prob = dict(workloads.layered_cube(3), layered_E=(2, [1.0, 2.0, 3.0, 1.0, 2.0, 3.0, 1.0]))
    with pytest.raises(tnfem.TnfemError) as e:
        tnfem.export_operator(prob)
    assert e.value.code == tnfem.EINVAL
    assert "one bit" in str(e.value)


def test_no_device_is_a_clean_error():
    import torch

    if torch.cuda.device_count() > 0:
        pytest.skip("a device is present")
    with pytest.raises(tnfem.TnfemError) as e:
        tnfem.Context(0)
    assert e.value.code == tnfem.EDEVICE


def test_default_options():
    o = tnfem.default_opts()
    assert (o.rank_cap, o.rho, o.init_rank, o.seed_x, o.seed_z, o.precision) == (32, 4, 2, 1, 2, 0)
    assert o.tol == 1e-8


def _random_tt(rng, modes, ranks):
    return [rng.standard_normal((ranks[k], n, ranks[k + 1])) for k, n in enumerate(modes)]


@pytest.mark.parametrize("seed", [0, 1])
def test_tt_norm_and_rel_diff_match_dense(seed):
    rng = np.random.default_rng(seed)
    modes = [3, 4, 2, 5]
    a = _random_tt(rng, modes, [1, 3, 5, 4, 1])
    b = _random_tt(rng, modes, [1, 2, 6, 3, 1])
    A, B = tnfem.TT.from_cores(a), tnfem.TT.from_cores(b)
    fa, fb = tt.tt_full(a), tt.tt_full(b)
    assert abs(A.norm() - np.linalg.norm(fa)) <= 1e-13 * np.linalg.norm(fa)
    ref = np.linalg.norm(fa - fb) / np.linalg.norm(fb)
    assert abs(A.rel_diff(B) - ref) <= 1e-13 * ref
    assert A.rel_diff(A) <= 1e-15


def test_tt_rel_diff_resolves_small_differences():
    # b = a + 1e-9 * c: the relative difference must come out to a few digits, where
    # ||a||^2 + ||b||^2 - 2 <a, b> would lose it to cancellation
    rng = np.random.default_rng(5)
    modes = [4] * 6
    a = _random_tt(rng, modes, [1, 4, 6, 6, 6, 4, 1])
    c = _random_tt(rng, modes, [1, 2, 2, 2, 2, 2, 1])
    b = tt.tt_add(a, c, 1.0, 1e-9)
    A, B = tnfem.TT.from_cores(a), tnfem.TT.from_cores(b)
    fa, fb = tt.tt_full(a), tt.tt_full(b)
    ref = np.linalg.norm(fa - fb) / np.linalg.norm(fb)
    assert abs(A.rel_diff(B) - ref) <= 1e-6 * ref


def test_interpreter_exit_with_open_library_objects():
    """TT objects left open at interpreter exit are destroyed cleanly (the binding closes
    live device objects from an exit handler, before the runtime's own teardown)."""
    import subprocess
    import sys

    code = ("import sys; sys.path.insert(0, %r)\n"
            "import numpy as np\n"
            "from paper_2501_12151_amd import tnfem\n"
            "a = tnfem.TT.from_cores([np.ones((1, 4, 2)), np.ones((2, 4, 1))])\n"
            "b = tnfem.TT.from_cores([np.ones((1, 4, 1)), np.ones((1, 4, 1))])\n"
            "print(a.rel_diff(b))\n") % ROOT
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
