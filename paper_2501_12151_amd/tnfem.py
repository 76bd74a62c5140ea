"""Python binding of libtnfem (ctypes; argument marshalling only).

Every computation happens in the HIP library behind include/tnfem.h.  If the
library has not been built (``python -m paper_2501_12151_amd.build`` or
``__graft_entry__.build()``) importing this module raises ImportError; there is
no fallback path.

Problem descriptions are plain dicts with the keys
    dim, level, E, nu, plane_stress (opt), extent (opt),
    clamp: [(axis, side), ...], tractions: [(axis, side, t), ...],
    body_force (opt), manufactured_c (opt)
so that the same dict can describe a workload to any consumer.

torch ships its own HIP runtime under the same library names (libamdhip64.so.7,
libhsa-runtime64.so.1) as the ROCm runtime the library links, and a process holds
whichever copy it loads first.  torch does not initialise on a runtime other than
its own, so this module imports torch (when it is installed) before loading the
library: the process then has one runtime, torch's, for both.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtnfem.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libtnfem.so is not built at {LIB_PATH}; run paper_2501_12151_amd/build.py")

try:  # load torch's HIP runtime first (see the module docstring)
    import torch  # noqa: F401
except ImportError:
    pass
_lib = C.CDLL(LIB_PATH)

OK, EINVAL, ENOMEM, EBUDGET, ENOTCONV, EDEVICE, ENAN, EBUSY = 0, -1, -2, -3, -4, -5, -6, -7


class ProblemDesc(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("level", C.c_int), ("extent", C.c_double * 3),
        ("E", C.c_double), ("nu", C.c_double), ("plane_stress", C.c_int),
        ("clamp_mask", C.c_uint32), ("n_tractions", C.c_int), ("traction_face", C.c_int * 6),
        ("traction", (C.c_double * 3) * 6), ("has_body_force", C.c_int), ("body_force", C.c_double * 3),
        ("has_manufactured", C.c_int), ("manufactured_c", C.c_double * 3),
        ("layer_axis", C.c_int), ("n_layer_E", C.c_int), ("layer_E", C.POINTER(C.c_double)),
        ("f0_ranks", C.POINTER(C.c_int)), ("f0_cores", C.POINTER(C.c_double)),
        ("has_stiffness", C.c_int), ("stiffness", (C.c_double * 6) * 6),
        ("has_quad", C.c_int), ("quad", (C.c_double * 2) * 4),
        ("n_elem_weight", C.c_int), ("elem_weight", C.POINTER(C.c_double)),
    ]


class SolveOpts(C.Structure):
    _fields_ = [
        ("rank_cap", C.c_int), ("tol", C.c_double), ("max_sweeps", C.c_int), ("rho", C.c_int),
        ("init_rank", C.c_int), ("seed_x", C.c_uint64), ("seed_z", C.c_uint64), ("cg_maxit", C.c_int),
        ("precision", C.c_int), ("profile", C.c_int),
        ("ir_max", C.c_int), ("ir_sweeps", C.c_int), ("ir_tol", C.c_double),
    ]


class SolveStats(C.Structure):
    _fields_ = [
        ("sweeps", C.c_int), ("converged", C.c_int), ("final_max_res", C.c_double),
        ("cg_iters", C.c_longlong), ("local_applies", C.c_longlong), ("flops", C.c_double),
        ("seconds", C.c_double), ("max_rank", C.c_int), ("refinements", C.c_longlong),
        ("low_precision_flops", C.c_double), ("precision_fallbacks", C.c_longlong),
        ("contraction_ms", C.c_double),
        ("contraction_flops", C.c_double), ("contraction_launches", C.c_longlong),
        ("apply_kernel_ms", C.c_double), ("apply_kernel_flops", C.c_double),
        ("apply_kernel_launches", C.c_longlong), ("peak_rank", C.c_int),
        ("ir_iters", C.c_int), ("ir_last_update", C.c_double), ("sweeps_total", C.c_int),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerInfo(C.Structure):
    _fields_ = [
        ("queued", C.c_int), ("running", C.c_int), ("peak_running", C.c_int), ("completed", C.c_longlong),
        ("bytes_in_use", C.c_size_t), ("peak_bytes", C.c_size_t), ("budget_bytes", C.c_size_t),
        ("peak_batch", C.c_int), ("batched_requests", C.c_longlong),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp = C.c_void_p
_ip = C.POINTER(C.c_int)
_dp = C.POINTER(C.c_double)
# device allocator hooks: alloc(bytes, stream, user) -> ptr, free(ptr, stream, user)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)
_sig = {
    "tnfem_last_error": (C.c_char_p, []),
    "tnfem_default_opts": (None, [C.POINTER(SolveOpts)]),
    "tnfem_ctx_create": (C.c_int, [C.POINTER(_vp), C.c_int, _vp]),
    "tnfem_ctx_destroy": (C.c_int, [_vp]),
    "tnfem_problem_create": (C.c_int, [_vp, C.POINTER(ProblemDesc), C.POINTER(_vp)]),
    "tnfem_problem_destroy": (C.c_int, [_vp]),
    "tnfem_problem_info": (C.c_int, [_vp, _ip, _ip, _ip, _ip]),
    "tnfem_solve": (C.c_int, [_vp, C.POINTER(SolveOpts), C.POINTER(_vp), C.POINTER(SolveStats)]),
    "tnfem_solve_batch": (C.c_int, [C.POINTER(_vp), C.c_int, _vp, C.POINTER(_vp), _vp, _ip]),
    "tnfem_server_set_max_batch": (C.c_int, [_vp, C.c_int]),
    "tnfem_tt_create": (C.c_int, [C.c_int, _ip, _ip, _dp, C.POINTER(_vp)]),
    "tnfem_tt_shape": (C.c_int, [_vp, _ip, _ip, _ip]),
    "tnfem_tt_size": (C.c_size_t, [_vp]),
    "tnfem_tt_copy_cores": (C.c_int, [_vp, _dp, C.c_size_t]),
    "tnfem_tt_eval": (C.c_int, [_vp, C.POINTER(C.c_int64), C.c_size_t, _dp]),
    "tnfem_tt_destroy": (C.c_int, [_vp]),
    "tnfem_tt_norm": (C.c_int, [_vp, _dp]),
    "tnfem_tt_rel_diff": (C.c_int, [_vp, _vp, _dp]),
    "tnfem_tt_dot": (C.c_int, [_vp, _vp, _dp]),
    "tnfem_export_operator": (C.c_int, [C.POINTER(ProblemDesc), _ip, _ip, _ip, _dp, C.c_size_t, C.POINTER(C.c_size_t)]),
    "tnfem_export_load": (C.c_int, [C.POINTER(ProblemDesc), _ip, _ip, _ip, _dp, C.c_size_t, C.POINTER(C.c_size_t)]),
    "tnfem_prim_local_apply": (C.c_int, [_vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _vp, _vp, _vp, _vp, _vp]),
    "tnfem_prim_local_apply_ex": (C.c_int, [_vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _vp, _vp, _vp,
                                             _vp, C.c_int, _vp]),
    "tnfem_prim_env_update": (C.c_int, [_vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _vp, _vp, _vp, _vp, _vp]),
    "tnfem_ctx_create_ex": (C.c_int, [C.POINTER(_vp), C.c_int, _vp, ALLOC_FN, FREE_FN, _vp]),
    "tnfem_prim_qr": (C.c_int, [_vp, C.c_int, C.c_int, _vp, _vp, _vp, _vp]),
    "tnfem_prim_svd": (C.c_int, [_vp, C.c_int, C.c_int, _vp, _vp, _vp, _vp, _vp]),
    "tnfem_prim_svd_noalloc": (C.c_int, [_vp, C.c_int, C.c_int, _vp, _vp, _vp, _vp, _vp]),
    "tnfem_prim_svd_noalloc_doubles": (C.c_size_t, [C.c_int, C.c_int]),
    "tnfem_server_create": (C.c_int, [C.c_int, C.c_int, C.c_size_t, C.POINTER(_vp)]),
    "tnfem_server_submit": (C.c_int, [_vp, C.POINTER(ProblemDesc), C.POINTER(SolveOpts), C.POINTER(C.c_longlong)]),
    "tnfem_server_poll": (C.c_int, [_vp, C.c_longlong, C.c_int, C.POINTER(_vp), C.POINTER(SolveStats),
                                    C.POINTER(C.c_double)]),
    "tnfem_server_info": (C.c_int, [_vp, C.POINTER(ServerInfo)]),
    "tnfem_server_destroy": (C.c_int, [_vp]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


class TnfemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tnfem error {code}: {msg}")
        self.code = code


def _check(rc, allow=()):
    if rc != OK and rc not in allow:
        raise TnfemError(rc, _lib.tnfem_last_error().decode())
    return rc


def make_desc(problem: dict) -> ProblemDesc:
    d = ProblemDesc()
    D = int(problem["dim"])
    d.dim = D
    d.level = int(problem["level"])
    ext = problem.get("extent") or [1.0, 1.0, 1.0]
    for a in range(3):
        d.extent[a] = float(ext[a]) if a < len(ext) else 1.0
    d.E = float(problem["E"])
    d.nu = float(problem["nu"])
    d.plane_stress = int(bool(problem.get("plane_stress", False)))
    mask = 0
    for axis, side in problem.get("clamp", []):
        mask |= 1 << (2 * int(axis) + int(side))
    d.clamp_mask = mask
    trs = problem.get("tractions", [])
    d.n_tractions = len(trs)
    for q, (axis, side, t) in enumerate(trs):
        d.traction_face[q] = 2 * int(axis) + int(side)
        for a in range(min(3, len(t))):
            d.traction[q][a] = float(t[a])
    if problem.get("body_force") is not None:
        d.has_body_force = 1
        for a, v in enumerate(problem["body_force"][:3]):
            d.body_force[a] = float(v)
    if problem.get("manufactured_c") is not None:
        d.has_manufactured = 1
        for a, v in enumerate(problem["manufactured_c"][:3]):
            d.manufactured_c[a] = float(v)
    if problem.get("layered_E") is not None:
        axis, vals = problem["layered_E"]
        arr = np.ascontiguousarray(vals, dtype=np.float64)
        d._layer_keep = arr
        d.layer_axis = int(axis)
        d.n_layer_E = arr.size
        d.layer_E = arr.ctypes.data_as(_dp)
    if problem.get("stiffness_voigt") is not None:
        Cv = np.asarray(problem["stiffness_voigt"], dtype=np.float64)
        d.has_stiffness = 1
        for i in range(Cv.shape[0]):
            for j in range(Cv.shape[1]):
                d.stiffness[i][j] = float(Cv[i, j])
    if problem.get("elem_weight") is not None:
        w = np.ascontiguousarray(problem["elem_weight"], dtype=np.float64).reshape(-1)
        d._ew_keep = w
        d.n_elem_weight = w.size
        d.elem_weight = w.ctypes.data_as(_dp)
    if problem.get("quad") is not None:
        Q = np.asarray(problem["quad"], dtype=np.float64).reshape(4, 2)
        d.has_quad = 1
        for c in range(4):
            for k in range(2):
                d.quad[c][k] = float(Q[c, k])
    if problem.get("f_nodal_tt") is not None:
        cores = [np.asarray(c, dtype=np.float64) for c in problem["f_nodal_tt"]]
        ranks = np.ascontiguousarray([c.shape[0] for c in cores] + [cores[-1].shape[2]], dtype=np.int32)
        flat = np.ascontiguousarray(np.concatenate([c.reshape(-1) for c in cores]))
        d._f0_keep = (ranks, flat)
        d.f0_ranks = ranks.ctypes.data_as(_ip)
        d.f0_cores = flat.ctypes.data_as(_dp)
    return d


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    _lib.tnfem_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _export(fn, problem):
    desc = make_desc(problem)
    nc = C.c_int()
    modes = (C.c_int * 64)()
    ranks = (C.c_int * 65)()
    need = C.c_size_t()
    _check(fn(C.byref(desc), C.byref(nc), modes, ranks, None, 0, C.byref(need)))
    buf = np.zeros(need.value, dtype=np.float64)
    _check(fn(C.byref(desc), C.byref(nc), modes, ranks, buf.ctypes.data_as(_dp), buf.size, C.byref(need)))
    return nc.value, list(modes[: nc.value]), list(ranks[: nc.value + 1]), buf


def export_operator(problem: dict):
    """Dense copies of the library's operator cores, [R_k, n, n, R_k+1] each (host only)."""
    K, modes, ranks, buf = _export(_lib.tnfem_export_operator, problem)
    cores, off = [], 0
    for k in range(K):
        cnt = ranks[k] * modes[k] * modes[k] * ranks[k + 1]
        cores.append(buf[off:off + cnt].reshape(ranks[k], modes[k], modes[k], ranks[k + 1]))
        off += cnt
    return cores


def export_load(problem: dict):
    """The library's load TT cores, [r_k, n, r_k+1] each (host only)."""
    K, modes, ranks, buf = _export(_lib.tnfem_export_load, problem)
    cores, off = [], 0
    for k in range(K):
        cnt = ranks[k] * modes[k] * ranks[k + 1]
        cores.append(buf[off:off + cnt].reshape(ranks[k], modes[k], ranks[k + 1]))
        off += cnt
    return cores


class TT:
    """Library-owned TT (host memory); .cores gives numpy copies."""

    def __init__(self, handle):
        self._h = handle

    def close(self):
        if getattr(self, "_h", None):
            _lib.tnfem_tt_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except (AttributeError, TypeError):  # interpreter shutdown: the library is already gone
            pass

    @classmethod
    def from_cores(cls, cores):
        """Library TT holding copies of the given cores ([r_k, n_k, r_{k+1}] arrays)."""
        modes = (C.c_int * len(cores))(*[int(c.shape[1]) for c in cores])
        ranks = (C.c_int * (len(cores) + 1))(*([int(cores[0].shape[0])] + [int(c.shape[2]) for c in cores]))
        flat = np.ascontiguousarray(np.concatenate([np.asarray(c, dtype=np.float64).reshape(-1) for c in cores]))
        h = _vp()
        _check(_lib.tnfem_tt_create(len(cores), modes, ranks, flat.ctypes.data_as(_dp), C.byref(h)))
        return cls(h)

    def shape(self):
        nc = C.c_int()
        modes = (C.c_int * 64)()
        ranks = (C.c_int * 65)()
        _check(_lib.tnfem_tt_shape(self._h, C.byref(nc), modes, ranks))
        return list(modes[: nc.value]), list(ranks[: nc.value + 1])

    @property
    def cores(self):
        modes, ranks = self.shape()
        buf = np.zeros(_lib.tnfem_tt_size(self._h), dtype=np.float64)
        _check(_lib.tnfem_tt_copy_cores(self._h, buf.ctypes.data_as(_dp), buf.size))
        out, off = [], 0
        for k, n in enumerate(modes):
            cnt = ranks[k] * n * ranks[k + 1]
            out.append(buf[off:off + cnt].reshape(ranks[k], n, ranks[k + 1]).copy())
            off += cnt
        return out

    def norm(self):
        out = C.c_double()
        _check(_lib.tnfem_tt_norm(self._h, C.byref(out)))
        return out.value

    def rel_diff(self, ref):
        """||self - ref|| / ||ref||, computed by the library in TT format."""
        out = C.c_double()
        _check(_lib.tnfem_tt_rel_diff(self._h, ref._h, C.byref(out)))
        return out.value

    def dot(self, other):
        """<self, other>, computed by the library in TT format."""
        out = C.c_double()
        _check(_lib.tnfem_tt_dot(self._h, other._h, C.byref(out)))
        return out.value

    def eval(self, idx):
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        out = np.zeros(idx.shape[0])
        _check(_lib.tnfem_tt_eval(self._h, idx.ctypes.data_as(C.POINTER(C.c_int64)), idx.shape[0],
                                  out.ctypes.data_as(_dp)))
        return out


# Device objects still open when the interpreter exits are closed by an exit handler, which
# runs before module teardown and before the HIP runtime's own destructors at process exit;
# left to garbage collection at shutdown, their hipFree calls could reach a runtime that is
# already gone.
_live = weakref.WeakSet()


@atexit.register
def _close_live_objects():
    for obj in list(_live):
        try:
            obj.close()
        except Exception:  # noqa: BLE001 -- best effort at exit
            pass


class Context:
    """A device context; stream may be a torch.cuda.Stream or a raw hipStream_t int.
    allocator="torch" hands the library's device allocations to torch's caching allocator."""

    def __init__(self, device: int = 0, stream=None, allocator=None):
        h = _vp()
        s = None
        if stream is not None:
            s = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        self._hooks = None
        if allocator == "torch":
            import torch

            dev = int(device)

            def _alloc(nbytes, stream_ptr, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), device=dev, stream=int(stream_ptr or 0))
                except Exception:  # noqa: BLE001 -- reported to the library as NULL (TNFEM_ENOMEM)
                    return None

            def _free(ptr, stream_ptr, user):
                torch.cuda.caching_allocator_delete(int(ptr))

            self._hooks = (ALLOC_FN(_alloc), FREE_FN(_free))
            _check(_lib.tnfem_ctx_create_ex(C.byref(h), dev, s, self._hooks[0], self._hooks[1], None))
        elif allocator is None:
            _check(_lib.tnfem_ctx_create(C.byref(h), int(device), s))
        else:
            raise ValueError("allocator must be None or 'torch'")
        self._h = h
        self._problems = weakref.WeakSet()
        _live.add(self)

    def close(self):
        """Destroys the context after every problem created on it."""
        if getattr(self, "_h", None):
            for p in list(self._problems):
                p.close()
            _lib.tnfem_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except (AttributeError, TypeError):  # interpreter shutdown: the library is already gone
            pass

    def qr(self, m, n, A, Q, R, stream=None):
        """Device QR on raw pointers (ints) or torch tensors."""
        _check(_lib.tnfem_prim_qr(self._h, m, n, _ptr(A), _ptr(Q), _ptr(R), _ptr(stream)))

    def svd(self, m, n, A, U, S, Vt, stream=None):
        _check(_lib.tnfem_prim_svd(self._h, m, n, _ptr(A), _ptr(U), _ptr(S), _ptr(Vt), _ptr(stream)))

    def svd_noalloc(self, m, n, A, U, S, Vt, stream=None):
        """The same SVD with the library's fixed device workspace (no allocation)."""
        _check(_lib.tnfem_prim_svd_noalloc(self._h, m, n, _ptr(A), _ptr(U), _ptr(S), _ptr(Vt), _ptr(stream)))


def svd_noalloc_doubles(m, n):
    """Workspace doubles of an m x n SVD (0 for an invalid shape)."""
    return int(_lib.tnfem_prim_svd_noalloc_doubles(int(m), int(n)))


NOALLOC_SCRATCH_BYTES = 16 << 20


def _ptr(x):
    if x is None:
        return None
    if hasattr(x, "cuda_stream"):
        return x.cuda_stream
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    return int(x)


def solve_batch(problems, **opts):
    """Lockstep solve of several problems of one dimension and level in one context (FP64,
    shared launches of the CG iterations).  Returns [(TT or None, stats dict, status)]."""
    n = len(problems)
    o = default_opts(**opts)
    hs = (_vp * n)(*[p._h for p in problems])
    outs = (_vp * n)()
    sts = (SolveStats * n)()
    status = (C.c_int * n)()
    _check(_lib.tnfem_solve_batch(hs, n, C.byref(o), outs, C.cast(sts, _vp), status))
    res = []
    for i in range(n):
        tt = TT(outs[i]) if outs[i] else None
        res.append((tt, sts[i].as_dict(), status[i]))
    return res


class Problem:
    def __init__(self, ctx: Context, problem: dict):
        self.ctx = ctx
        self.desc = make_desc(problem)
        h = _vp()
        _check(_lib.tnfem_problem_create(ctx._h, C.byref(self.desc), C.byref(h)))
        self._h = h
        ctx._problems.add(self)

    def close(self):
        if getattr(self, "_h", None):
            _lib.tnfem_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except (AttributeError, TypeError):  # interpreter shutdown: the library is already gone
            pass

    def info(self):
        nc = C.c_int()
        modes = (C.c_int * 64)()
        mr = (C.c_int * 65)()
        br = (C.c_int * 65)()
        _check(_lib.tnfem_problem_info(self._h, C.byref(nc), modes, mr, br))
        K = nc.value
        return dict(ncores=K, modes=list(modes[:K]), mpo_ranks=list(mr[:K + 1]), rhs_ranks=list(br[:K + 1]))

    def solve(self, **opts):
        """Blocking solve.  Returns (TT, stats dict, status code)."""
        o = default_opts(**opts)
        h = _vp()
        st = SolveStats()
        rc = _check(_lib.tnfem_solve(self._h, C.byref(o), C.byref(h), C.byref(st)), allow=(ENOTCONV,))
        return TT(h), st.as_dict(), rc

    def local_apply(self, k, reversed_, p, q, s, t, L, x, Rt, y, stream=None):
        _check(_lib.tnfem_prim_local_apply(self._h, k, int(reversed_), p, q, s, t, _ptr(L), _ptr(x), _ptr(Rt),
                                           _ptr(y), _ptr(stream)))

    def local_apply_ex(self, k, reversed_, p, q, s, t, L, x, Rt, y, precision=0, stream=None):
        _check(_lib.tnfem_prim_local_apply_ex(self._h, k, int(reversed_), p, q, s, t, _ptr(L), _ptr(x), _ptr(Rt),
                                              _ptr(y), int(precision), _ptr(stream)))

    def env_update(self, k, reversed_, p, q, s, t, W, L, X, Lnew, stream=None):
        _check(_lib.tnfem_prim_env_update(self._h, k, int(reversed_), p, q, s, t, _ptr(W), _ptr(L), _ptr(X),
                                          _ptr(Lnew), _ptr(stream)))


class Server:
    """Request server on one device (see tnfem_server_* in include/tnfem.h)."""

    def __init__(self, device: int = 0, slots: int = 4, hbm_budget_bytes: int = 0):
        h = _vp()
        _check(_lib.tnfem_server_create(int(device), int(slots), int(hbm_budget_bytes), C.byref(h)))
        self._h = h
        self._descs = {}
        _live.add(self)

    def submit(self, problem: dict, **opts) -> int:
        desc = make_desc(problem)
        o = default_opts(**opts)
        t = C.c_longlong()
        _check(_lib.tnfem_server_submit(self._h, C.byref(desc), C.byref(o), C.byref(t)))
        return t.value

    def poll(self, ticket: int, wait: bool = True):
        """None while running (wait=False); else (TT or None, stats, status, latency_s)."""
        h = _vp()
        st = SolveStats()
        lat = C.c_double()
        rc = _lib.tnfem_server_poll(self._h, int(ticket), int(bool(wait)), C.byref(h), C.byref(st), C.byref(lat))
        if rc == EBUSY:
            return None
        if rc not in (OK, ENOTCONV):
            raise TnfemError(rc, _lib.tnfem_last_error().decode())
        return TT(h), st.as_dict(), rc, lat.value

    def set_max_batch(self, n: int):
        _check(_lib.tnfem_server_set_max_batch(self._h, int(n)))

    def info(self):
        i = ServerInfo()
        _check(_lib.tnfem_server_info(self._h, C.byref(i)))
        return i.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            _lib.tnfem_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except (AttributeError, TypeError):  # interpreter shutdown: the library is already gone
            pass
