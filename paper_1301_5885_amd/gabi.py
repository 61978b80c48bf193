"""Python binding of libgabi (include/gabi.h): argument marshalling only.

Every computation runs in the HIP library; this module converts numpy arrays
and torch tensors to pointers and status codes to exceptions.  If the
library has not been built the import of ``load()`` fails loudly -- there is
no fallback.

Host entry points take numpy arrays and return numpy arrays.  ``*_dev``
entry points take float64 torch tensors on the GPU and run on torch's
current stream.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgabi.so")

OK, NOT_CONVERGED = 0, 1
EINVAL, ESTATE, EMESH, ENOMEM, EDEVICE, EBUSY = -1, -2, -3, -4, -5, -6
FP64, FP32_PAIR = 0, 1
SOLVE_FP64, SOLVE_MIXED_IR, SOLVE_TREE_IR = 0, 1, 2
SCHEME_SPLIT, SCHEME_SYMMETRIC = 0, 1
_NAMES = {0: "GABI_OK", 1: "GABI_NOT_CONVERGED", -1: "GABI_EINVAL",
          -2: "GABI_ESTATE", -3: "GABI_EMESH", -4: "GABI_ENOMEM",
          -5: "GABI_EDEVICE", -6: "GABI_EBUSY"}

# Every symbol declared in include/gabi.h.
EXPORTS = (
    "gabi_default_opts", "gabi_create", "gabi_destroy", "gabi_last_error",
    "gabi_set_stream", "gabi_mesh_elements", "gabi_set_surface",
    "gabi_set_surface_mesh", "gabi_set_charges", "gabi_set_params",
    "gabi_rhs", "gabi_rhs_dev", "gabi_matvec", "gabi_matvec_dev",
    "gabi_solve", "gabi_solve_dev", "gabi_energy", "gabi_energy_dev",
    "gabi_reaction_potential", "gabi_device_bytes", "gabi_set_kernel_timing",
    "gabi_kernel_time", "gabi_solve_footprint", "gabi_batch_solve",
    "gabi_server_create", "gabi_server_submit", "gabi_server_poll",
    "gabi_server_drain", "gabi_server_stats_get", "gabi_server_clock",
    "gabi_server_last_error", "gabi_server_destroy", "gabi_tune_set", "gabi_tune_get",
    "gabi_set_part_budget", "gabi_get_part_budget", "gabi_tree_matvec",
    "gabi_tree_matvec_dev", "gabi_tree_info_get", "gabi_tree_plan",
    "gabi_msms_counts", "gabi_msms_read", "gabi_msms_orient", "gabi_pqr_count",
    "gabi_pqr_read", "gabi_selftest_exp_neg", "gabi_server_set_round_cap",
    "gabi_matvec_noalloc",
)
TIMING_TREE = 2  # gabi_kernel_time kind of the treecode products

# Tuned decomposition table for gfx950, applied when the library is loaded
# (set GABI_TUNING=none to keep the built-in defaults, or to another path).
TUNING_PATH = os.path.join(HERE, "tuning_gfx950.json")


class GabiError(RuntimeError):
    def __init__(self, code, msg=""):
        self.code = code
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")


class SolveOpts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("maxit", C.c_int32), ("tol", C.c_double),
                ("mode", C.c_int32), ("inner_tol", C.c_double),
                ("max_outer", C.c_int32), ("use_graph", C.c_int32),
                ("x0_previous", C.c_int32), ("tree_theta", C.c_double),
                ("tree_degree", C.c_int32), ("tree_leaf", C.c_int32),
                ("tree_precision", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("matvecs_fp64", C.c_int64),
                ("matvecs_fp32", C.c_int64), ("restarts", C.c_int64),
                ("outer", C.c_int64), ("rel_residual", C.c_double),
                ("converged", C.c_int32), ("seconds", C.c_double),
                ("warm_start", C.c_int32), ("matvecs_tree", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ProblemC(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(k, C.c_void_p) for k in
                                     ("cx", "cy", "cz", "nx", "ny", "nz", "area")] + \
               [("nc", C.c_int64)] + [(k, C.c_void_p) for k in ("px", "py", "pz", "q")] + \
               [("eps1", C.c_double), ("eps2", C.c_double), ("kappa", C.c_double),
                ("u_out", C.c_void_p), ("tag", C.c_int64)]


class ResultC(C.Structure):
    _fields_ = [("tag", C.c_int64), ("status", C.c_int32), ("energy", C.c_double),
                ("info", SolveInfo), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double), ("device_bytes", C.c_int64),
                ("ticket", C.c_int64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "info"}
        d["info"] = self.info.as_dict()
        return d


class TreeOpts(C.Structure):
    _fields_ = [("theta", C.c_double), ("degree", C.c_int32), ("leaf_size", C.c_int32),
                ("precision", C.c_int32), ("reserved", C.c_int32)]


class TreeInfo(C.Structure):
    _fields_ = [(k, C.c_int64) for k in (
        "leaves", "clusters_with_proxies", "far_entries", "near_entries", "far_pairs",
        "near_pairs", "device_bytes")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def tree_opts(theta=0.7, degree=5, leaf_size=256, precision=0):
    """gabi_tree_opts; precision FP64 (0) or FP32_PAIR (1)."""
    return TreeOpts(float(theta), int(degree), int(leaf_size), int(precision), 0)


class ServerStats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in (
        "submitted", "admitted", "completed", "failed", "queued", "active", "rounds",
        "max_active", "bytes_in_use", "peak_bytes", "budget_bytes")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_dp = C.POINTER(C.c_double)
_vp = C.c_void_p
_i64 = C.c_int64


def load():
    """Load libgabi.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch ships its own HIP runtime; loading it first lets libgabi bind to
    # that same runtime (one runtime per process) instead of a second copy.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built; run __graft_entry__.build() "
            "(hipcc --offload-arch=gfx950) first")
    lib = C.CDLL(LIB_PATH)
    ctx = _vp
    lib.gabi_default_opts.argtypes = [C.POINTER(SolveOpts)]
    lib.gabi_default_opts.restype = None
    lib.gabi_create.argtypes = [C.POINTER(_vp), C.c_int]
    lib.gabi_destroy.argtypes = [ctx]
    lib.gabi_destroy.restype = None
    lib.gabi_last_error.argtypes = [ctx]
    lib.gabi_last_error.restype = C.c_char_p
    lib.gabi_set_stream.argtypes = [ctx, _vp]
    lib.gabi_mesh_elements.argtypes = [_i64, _dp, _i64, C.POINTER(C.c_int32)] + [_dp] * 7
    lib.gabi_set_surface.argtypes = [ctx, _i64] + [_dp] * 7
    lib.gabi_set_surface_mesh.argtypes = [ctx, _i64, _dp, _i64, C.POINTER(C.c_int32)]
    lib.gabi_set_charges.argtypes = [ctx, _i64] + [_dp] * 4
    lib.gabi_set_params.argtypes = [ctx, C.c_double, C.c_double, C.c_double]
    lib.gabi_rhs.argtypes = [ctx, _dp]
    lib.gabi_rhs_dev.argtypes = [ctx, _vp]
    lib.gabi_matvec.argtypes = [ctx, C.c_int, _dp, _dp]
    lib.gabi_matvec_dev.argtypes = [ctx, C.c_int, _vp, _vp]
    lib.gabi_matvec_noalloc.argtypes = [ctx, _i64, _vp, _vp, _vp]
    lib.gabi_solve.argtypes = [ctx, C.POINTER(SolveOpts), _dp, _dp, C.POINTER(SolveInfo)]
    lib.gabi_solve_dev.argtypes = [ctx, C.POINTER(SolveOpts), _vp, _vp, C.POINTER(SolveInfo)]
    lib.gabi_energy.argtypes = [ctx, _dp, _dp]
    lib.gabi_energy_dev.argtypes = [ctx, _vp, _dp]
    lib.gabi_reaction_potential.argtypes = [ctx, _dp, _dp]
    lib.gabi_device_bytes.argtypes = [ctx]
    lib.gabi_device_bytes.restype = C.c_int64
    lib.gabi_set_kernel_timing.argtypes = [ctx, C.c_int]
    lib.gabi_kernel_time.argtypes = [ctx, C.c_int, _dp, C.POINTER(C.c_int64), C.c_int]
    lib.gabi_set_part_budget.argtypes = [_i64]
    lib.gabi_get_part_budget.argtypes = []
    lib.gabi_get_part_budget.restype = C.c_int64
    lib.gabi_tree_matvec.argtypes = [ctx, C.POINTER(TreeOpts), _dp, _dp]
    lib.gabi_tree_matvec_dev.argtypes = [ctx, C.POINTER(TreeOpts), _vp, _vp]
    lib.gabi_tree_info_get.argtypes = [ctx, C.POINTER(TreeOpts), C.POINTER(TreeInfo)]
    lib.gabi_tree_plan.argtypes = [_i64, _dp, _dp, _dp, C.POINTER(TreeOpts),
                                   C.POINTER(TreeInfo)]
    lib.gabi_msms_counts.argtypes = [C.c_char_p, C.c_char_p, C.POINTER(_i64),
                                     C.POINTER(_i64)]
    lib.gabi_msms_read.argtypes = [C.c_char_p, C.c_char_p, _i64, _dp, _dp, _i64,
                                   C.POINTER(C.c_int32)]
    lib.gabi_msms_orient.argtypes = [_i64, _dp, _dp, _i64, C.POINTER(C.c_int32),
                                     C.POINTER(_i64)]
    lib.gabi_pqr_count.argtypes = [C.c_char_p, C.POINTER(_i64)]
    lib.gabi_selftest_exp_neg.argtypes = [C.c_int, _i64, _dp, _dp]
    lib.gabi_pqr_read.argtypes = [C.c_char_p, _i64, _dp, _dp, _dp]
    lib.gabi_tune_set.argtypes = [C.c_int] * 6
    lib.gabi_tune_get.argtypes = [C.c_int, C.c_int] + [C.POINTER(C.c_int)] * 4
    lib.gabi_solve_footprint.argtypes = [_i64, _i64, C.c_int32]
    lib.gabi_solve_footprint.restype = C.c_int64
    lib.gabi_batch_solve.argtypes = [C.c_int, _i64, C.POINTER(ProblemC),
                                     C.POINTER(SolveOpts), C.POINTER(ResultC)]
    lib.gabi_server_create.argtypes = [C.POINTER(_vp), C.c_int, _i64, C.c_int32,
                                       C.POINTER(SolveOpts), C.c_double]
    lib.gabi_server_submit.argtypes = [_vp, C.POINTER(ProblemC), C.POINTER(C.c_int64)]
    lib.gabi_server_poll.argtypes = [_vp, C.POINTER(ResultC), C.c_int32,
                                     C.POINTER(C.c_int32)]
    lib.gabi_server_drain.argtypes = [_vp, C.c_double]
    lib.gabi_server_set_round_cap.argtypes = [_vp, C.c_double, _i64]
    lib.gabi_server_stats_get.argtypes = [_vp, C.POINTER(ServerStats)]
    lib.gabi_server_clock.argtypes = [_vp]
    lib.gabi_server_clock.restype = C.c_double
    lib.gabi_server_last_error.argtypes = [_vp]
    lib.gabi_server_last_error.restype = C.c_char_p
    lib.gabi_server_destroy.argtypes = [_vp]
    lib.gabi_server_destroy.restype = None
    for name in EXPORTS:
        if name not in ("gabi_default_opts", "gabi_destroy", "gabi_last_error",
                        "gabi_device_bytes", "gabi_solve_footprint", "gabi_server_clock",
                        "gabi_server_last_error", "gabi_server_destroy",
                        "gabi_get_part_budget"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    _apply_tuning(lib)
    return lib


def _apply_tuning(lib):
    import json
    path = os.environ.get("GABI_TUNING", TUNING_PATH)
    if path == "none" or not os.path.exists(path):
        return
    with open(path) as f:
        table = json.load(f)
    for key, prec in (("fp64", FP64), ("fp32", FP32_PAIR)):
        for bucket, e in table.get("entries", {}).get(key, {}).items():
            rc = lib.gabi_tune_set(prec, int(bucket), int(e.get("scheme", SCHEME_SPLIT)),
                                   int(e["rows_per_thread"]), int(e["target_blocks"]),
                                   int(e.get("tail_pieces", 0)))
            if rc != OK:
                raise GabiError(rc, f"bad tuning entry {key}/{bucket} in {path}")


def tune_set(precision, bucket, scheme, rows_per_thread, target_blocks, tail_pieces=0):
    rc = load().gabi_tune_set(int(precision), int(bucket), int(scheme), int(rows_per_thread),
                              int(target_blocks), int(tail_pieces))
    if rc != OK:
        raise GabiError(rc, "gabi_tune_set")


def tune_get(precision, bucket):
    """(scheme, rows_per_thread, target_blocks, tail_pieces) of a table entry."""
    sc, r, t, p = C.c_int(), C.c_int(), C.c_int(), C.c_int()
    rc = load().gabi_tune_get(int(precision), int(bucket), C.byref(sc), C.byref(r), C.byref(t),
                              C.byref(p))
    if rc != OK:
        raise GabiError(rc, "gabi_tune_get")
    return sc.value, r.value, t.value, p.value


def set_part_budget(nbytes):
    """Partial-sum budget per molecule and precision, in bytes (see gabi.h)."""
    rc = load().gabi_set_part_budget(int(nbytes))
    if rc != OK:
        raise GabiError(rc, "gabi_set_part_budget")


def get_part_budget():
    return int(load().gabi_get_part_budget())


def read_msms(vert_path, face_path, orient=True):
    """An MSMS triangulation: (V (nv, 3), F (nf, 3) 0-based int32, vertex
    normals (nv, 3), number of faces rewound to counter-clockwise)."""
    lib = load()
    nv, nf = _i64(), _i64()
    vp, fp = os.fsencode(vert_path), os.fsencode(face_path)
    rc = lib.gabi_msms_counts(vp, fp, C.byref(nv), C.byref(nf))
    if rc != OK:
        raise GabiError(rc, f"gabi_msms_counts({vert_path}, {face_path})")
    V = np.empty((nv.value, 3))
    N = np.empty((nv.value, 3))
    F = np.empty((nf.value, 3), dtype=np.int32)
    tp = F.ctypes.data_as(C.POINTER(C.c_int32))
    rc = lib.gabi_msms_read(vp, fp, nv.value, _p(V), _p(N), nf.value, tp)
    if rc != OK:
        raise GabiError(rc, f"gabi_msms_read({vert_path}, {face_path})")
    flipped = _i64(0)
    if orient:
        rc = lib.gabi_msms_orient(nv.value, _p(V), _p(N), nf.value, tp, C.byref(flipped))
        if rc != OK:
            raise GabiError(rc, "gabi_msms_orient")
    return V, F, N, flipped.value


def selftest_exp_neg(t, device=0):
    """The device's FP64 e^{-t} of the pair kernels at host values t >= 0."""
    t = _f64(t).ravel()
    out = np.empty_like(t)
    rc = load().gabi_selftest_exp_neg(int(device), t.size, _p(t), _p(out))
    if rc != OK:
        raise GabiError(rc, "gabi_selftest_exp_neg")
    return out


def read_pqr(path):
    """Atom records of a PQR file: (positions (n, 3), charges, radii)."""
    lib = load()
    n = _i64()
    p = os.fsencode(path)
    rc = lib.gabi_pqr_count(p, C.byref(n))
    if rc != OK:
        raise GabiError(rc, f"gabi_pqr_count({path})")
    xyz, q, r = np.empty((n.value, 3)), np.empty(n.value), np.empty(n.value)
    rc = lib.gabi_pqr_read(p, n.value, _p(xyz), _p(q), _p(r))
    if rc != OK:
        raise GabiError(rc, f"gabi_pqr_read({path})")
    return xyz, q, r


def tree_plan(centroids, theta=0.7, degree=5, leaf_size=256):
    """Treecode statistics from centroids alone (host only, no device)."""
    c = _f64(centroids).reshape(-1, 3)
    cols = [np.ascontiguousarray(c[:, k]) for k in range(3)]
    info = TreeInfo()
    o = tree_opts(theta, degree, leaf_size)
    rc = load().gabi_tree_plan(c.shape[0], *[_p(x) for x in cols], C.byref(o), C.byref(info))
    if rc != OK:
        raise GabiError(rc, "gabi_tree_plan")
    return info.as_dict()


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def mesh_elements(V, F):
    """Element data of a mesh computed by the library (host utility)."""
    lib = load()
    V = _f64(V).reshape(-1, 3)
    F = np.ascontiguousarray(F, dtype=np.int32).reshape(-1, 3)
    n = F.shape[0]
    out = [np.empty(n) for _ in range(7)]
    rc = lib.gabi_mesh_elements(V.shape[0], _p(V), n,
                                F.ctypes.data_as(C.POINTER(C.c_int32)),
                                *[_p(a) for a in out])
    if rc != OK:
        raise GabiError(rc, "gabi_mesh_elements")
    keys = ("cx", "cy", "cz", "nx", "ny", "nz", "area")
    return dict(zip(keys, out))


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    load().gabi_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown solve option {k}")
        setattr(o, k, v)
    return o


def _torch_ptr(t, numel=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA/HIP torch tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float64")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


@dataclass
class Problem:
    """Host-side description handed to a context in one call."""
    V: np.ndarray
    F: np.ndarray
    pos: np.ndarray
    q: np.ndarray
    eps1: float = 1.0
    eps2: float = 80.0
    kappa: float = 0.1257


class Context:
    """One libgabi context on one device (not thread-safe)."""

    def __init__(self, device: int = 0):
        self._lib = load()
        h = _vp()
        rc = self._lib.gabi_create(C.byref(h), int(device))
        if rc != OK:
            raise GabiError(rc, f"gabi_create(device={device})")
        self._h = h
        self.n = 0
        self.nc = 0

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None):
            self._lib.gabi_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc, what, allow_warning=False):
        if rc == OK or (allow_warning and rc == NOT_CONVERGED):
            return rc
        msg = self._lib.gabi_last_error(self._h).decode()
        raise GabiError(rc, f"{what}: {msg}")

    # -- configuration
    def set_stream(self, stream=None):
        """Use a hipStream_t handle (int), a torch stream, or torch's current."""
        if stream is None:
            import torch
            stream = torch.cuda.current_stream()
        handle = getattr(stream, "cuda_stream", stream)
        self._check(self._lib.gabi_set_stream(self._h, C.c_void_p(int(handle))),
                    "gabi_set_stream")

    def set_surface(self, centroids, normals, area):
        c = _f64(centroids).reshape(-1, 3)
        nrm = _f64(normals).reshape(-1, 3)
        a = _f64(area)
        cols = [np.ascontiguousarray(c[:, k]) for k in range(3)] + \
               [np.ascontiguousarray(nrm[:, k]) for k in range(3)] + [a]
        self._check(self._lib.gabi_set_surface(self._h, c.shape[0], *[_p(x) for x in cols]),
                    "gabi_set_surface")
        self.n = c.shape[0]

    def set_surface_mesh(self, V, F):
        V = _f64(V).reshape(-1, 3)
        F = np.ascontiguousarray(F, dtype=np.int32).reshape(-1, 3)
        self._check(self._lib.gabi_set_surface_mesh(
            self._h, V.shape[0], _p(V), F.shape[0],
            F.ctypes.data_as(C.POINTER(C.c_int32))), "gabi_set_surface_mesh")
        self.n = F.shape[0]

    def set_charges(self, pos, q):
        pos = _f64(pos).reshape(-1, 3)
        q = _f64(q)
        cols = [np.ascontiguousarray(pos[:, k]) for k in range(3)] + [q]
        self._check(self._lib.gabi_set_charges(self._h, q.shape[0], *[_p(x) for x in cols]),
                    "gabi_set_charges")
        self.nc = q.shape[0]

    def set_params(self, eps1=1.0, eps2=80.0, kappa=0.1257):
        self._check(self._lib.gabi_set_params(self._h, eps1, eps2, kappa), "gabi_set_params")

    def load_problem(self, p):
        self.set_surface_mesh(p.V, p.F)
        self.set_charges(p.pos, p.q)
        self.set_params(p.eps1, p.eps2, p.kappa)

    def load_request(self, req):
        """Surface, charges and parameters of a Request (element arrays)."""
        self._check(self._lib.gabi_set_surface(self._h, req.n, *[_p(x) for x in req.cols]),
                    "gabi_set_surface")
        self.n = req.n
        self._check(self._lib.gabi_set_charges(self._h, req.nc,
                                               *[_p(x) if req.nc else None
                                                 for x in req.charges]),
                    "gabi_set_charges")
        self.nc = req.nc
        self.set_params(req.c.eps1, req.c.eps2, req.c.kappa)

    # -- host entry points
    def rhs(self):
        b = np.empty(2 * self.n)
        self._check(self._lib.gabi_rhs(self._h, _p(b)), "gabi_rhs")
        return b

    def matvec(self, u, precision=FP64):
        u = _f64(u)
        if u.shape != (2 * self.n,):
            raise ValueError("u must have length 2N")
        y = np.empty(2 * self.n)
        self._check(self._lib.gabi_matvec(self._h, int(precision), _p(u), _p(y)),
                    "gabi_matvec")
        return y

    def solve(self, x0=None, **opts):
        o = default_opts(**opts)
        info = SolveInfo()
        u = np.empty(2 * self.n)
        x0a = None if x0 is None else _f64(x0)
        rc = self._lib.gabi_solve(self._h, C.byref(o), _p(x0a), _p(u), C.byref(info))
        self._check(rc, "gabi_solve", allow_warning=True)
        return u, info.as_dict()

    def energy(self, u=None):
        e = C.c_double()
        ua = None if u is None else _f64(u)
        self._check(self._lib.gabi_energy(self._h, _p(ua), C.byref(e)), "gabi_energy")
        return e.value

    def reaction_potential(self, u=None):
        phi = np.empty(self.nc)
        ua = None if u is None else _f64(u)
        self._check(self._lib.gabi_reaction_potential(self._h, _p(ua), _p(phi)),
                    "gabi_reaction_potential")
        return phi

    # -- device entry points (torch tensors, current stream)
    def rhs_dev(self, b):
        self.set_stream()
        self._check(self._lib.gabi_rhs_dev(self._h, _torch_ptr(b, 2 * self.n, "b")),
                    "gabi_rhs_dev")

    def matvec_dev(self, u, y, precision=FP64):
        self.set_stream()
        self._check(self._lib.gabi_matvec_dev(
            self._h, int(precision), _torch_ptr(u, 2 * self.n, "u"),
            _torch_ptr(y, 2 * self.n, "y")), "gabi_matvec_dev")

    def matvec_noalloc(self, elem, u, y):
        """FP64 product through the allocation-free entry point: elem is a
        contiguous float64 device tensor of 8 n values ((cx, cy, cz, area)
        per element, then (nx, ny, nz, 0) per element); u, y of 2 n."""
        n = elem.numel() // 8
        self.set_stream()
        self._check(self._lib.gabi_matvec_noalloc(
            self._h, n, _torch_ptr(elem, 8 * n, "elem"), _torch_ptr(u, 2 * n, "u"),
            _torch_ptr(y, 2 * n, "y")), "gabi_matvec_noalloc")

    def solve_dev(self, u, x0=None, **opts):
        self.set_stream()
        o = default_opts(**opts)
        info = SolveInfo()
        x0p = None if x0 is None else _torch_ptr(x0, 2 * self.n, "x0")
        rc = self._lib.gabi_solve_dev(self._h, C.byref(o), x0p,
                                      _torch_ptr(u, 2 * self.n, "u"), C.byref(info))
        self._check(rc, "gabi_solve_dev", allow_warning=True)
        return info.as_dict()

    def energy_dev(self, u=None):
        self.set_stream()
        e = C.c_double()
        up = None if u is None else _torch_ptr(u, 2 * self.n, "u")
        self._check(self._lib.gabi_energy_dev(self._h, up, C.byref(e)), "gabi_energy_dev")
        return e.value

    # -- treecode product
    def tree_matvec(self, u, theta=0.7, degree=5, leaf_size=256, precision=0):
        o = tree_opts(theta, degree, leaf_size, precision)
        ua = _f64(u)
        y = np.empty(2 * self.n)
        self._check(self._lib.gabi_tree_matvec(self._h, C.byref(o), _p(ua), _p(y)),
                    "gabi_tree_matvec")
        return y

    def tree_matvec_dev(self, u, y, theta=0.7, degree=5, leaf_size=256, precision=0):
        self.set_stream()
        o = tree_opts(theta, degree, leaf_size, precision)
        self._check(self._lib.gabi_tree_matvec_dev(self._h, C.byref(o),
                                                   _torch_ptr(u, 2 * self.n, "u"),
                                                   _torch_ptr(y, 2 * self.n, "y")),
                    "gabi_tree_matvec_dev")

    def tree_info(self, theta=0.7, degree=5, leaf_size=256):
        o = tree_opts(theta, degree, leaf_size)
        info = TreeInfo()
        self._check(self._lib.gabi_tree_info_get(self._h, C.byref(o), C.byref(info)),
                    "gabi_tree_info_get")
        return info.as_dict()

    # -- accounting and timing
    def device_bytes(self):
        return int(self._lib.gabi_device_bytes(self._h))

    def set_kernel_timing(self, enable=True):
        self._check(self._lib.gabi_set_kernel_timing(self._h, int(bool(enable))),
                    "gabi_set_kernel_timing")

    def kernel_time(self, precision=FP64, reset=False):
        ms = C.c_double()
        cnt = C.c_int64()
        self._check(self._lib.gabi_kernel_time(self._h, int(precision), C.byref(ms),
                                               C.byref(cnt), int(bool(reset))),
                    "gabi_kernel_time")
        return ms.value, cnt.value


# ---------------------------------------------------------------------------
# many molecules
# ---------------------------------------------------------------------------
def solve_footprint(n, nc, restart=20):
    """Device bytes one solve holds (the unit of admission)."""
    return int(load().gabi_solve_footprint(int(n), int(nc), int(restart)))


class Request:
    """One solve request: element arrays, charges, parameters.

    Keeps the numpy arrays alive for as long as the C side may read them."""

    def __init__(self, centroids, normals, area, pos, q, eps1=1.0, eps2=80.0,
                 kappa=0.1257, tag=0, want_solution=False):
        c = _f64(centroids).reshape(-1, 3)
        nrm = _f64(normals).reshape(-1, 3)
        self.cols = [np.ascontiguousarray(c[:, k]) for k in range(3)] + \
                    [np.ascontiguousarray(nrm[:, k]) for k in range(3)] + [_f64(area)]
        pos = _f64(pos).reshape(-1, 3)
        self.charges = [np.ascontiguousarray(pos[:, k]) for k in range(3)] + [_f64(q)]
        self.n = c.shape[0]
        self.nc = pos.shape[0]
        self.u = np.empty(2 * self.n) if want_solution else None
        self.c = ProblemC(self.n, *[a.ctypes.data for a in self.cols], self.nc,
                          *[a.ctypes.data if self.nc else None for a in self.charges],
                          eps1, eps2, kappa,
                          self.u.ctypes.data if self.u is not None else None, int(tag))

    @staticmethod
    def from_mesh(V, F, pos, q, **kw):
        el = mesh_elements(V, F)
        c = np.stack([el["cx"], el["cy"], el["cz"]], axis=1)
        nrm = np.stack([el["nx"], el["ny"], el["nz"]], axis=1)
        return Request(c, nrm, el["area"], pos, q, **kw)


def batch_solve(requests, device=0, **opts):
    """Solve all requests together; returns one result dict per request."""
    lib = load()
    arr = (ProblemC * len(requests))(*[r.c for r in requests])
    res = (ResultC * len(requests))()
    o = default_opts(**opts)
    rc = lib.gabi_batch_solve(int(device), len(requests), arr, C.byref(o), res)
    if rc != OK:
        raise GabiError(rc, "gabi_batch_solve")
    return [r.as_dict() for r in res]


class Server:
    """Serving loop (see include/gabi.h): FIFO admission by device-memory
    footprint, continuous batching at round boundaries.  device=-1 runs the
    scheduler with the host-only executor (no arithmetic)."""

    def __init__(self, device=0, budget_bytes=1 << 30, max_slots=64,
                 mock_round_seconds=0.0, **opts):
        self._lib = load()
        h = _vp()
        o = default_opts(**opts)
        rc = self._lib.gabi_server_create(C.byref(h), int(device), int(budget_bytes),
                                          int(max_slots), C.byref(o),
                                          float(mock_round_seconds))
        if rc != OK:
            raise GabiError(rc, "gabi_server_create")
        self._h = h
        # requests in flight by ticket: the worker may still copy a solution
        # into req.u, so each Request stays alive until its result is polled
        self._keep = {}

    def submit(self, req):
        """Queues req; returns its ticket (results carry it back)."""
        t = C.c_int64()
        rc = self._lib.gabi_server_submit(self._h, C.byref(req.c), C.byref(t))
        if rc != OK:
            raise GabiError(rc, self._lib.gabi_server_last_error(self._h).decode())
        self._keep[t.value] = req
        return t.value

    def in_flight(self):
        """Tickets submitted whose results have not been polled yet."""
        return sorted(self._keep)

    def poll(self, max_results=256):
        buf = (ResultC * max_results)()
        cnt = C.c_int32()
        rc = self._lib.gabi_server_poll(self._h, buf, max_results, C.byref(cnt))
        if rc != OK:
            raise GabiError(rc, "gabi_server_poll")
        out = [buf[i].as_dict() for i in range(cnt.value)]
        for r in out:
            self._keep.pop(r["ticket"], None)
        return out

    def set_round_cap(self, slack, floor_elements=0):
        """Oldest-first round cap (see include/gabi.h); slack < 0 disables."""
        rc = self._lib.gabi_server_set_round_cap(self._h, float(slack), int(floor_elements))
        if rc != OK:
            raise GabiError(rc, "gabi_server_set_round_cap")

    def drain(self, timeout_s=600.0):
        return self._lib.gabi_server_drain(self._h, float(timeout_s)) == OK

    def stats(self):
        st = ServerStats()
        rc = self._lib.gabi_server_stats_get(self._h, C.byref(st))
        if rc != OK:
            raise GabiError(rc, "gabi_server_stats_get")
        return st.as_dict()

    def clock(self):
        return float(self._lib.gabi_server_clock(self._h))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.gabi_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
