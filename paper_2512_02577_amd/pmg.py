"""Python binding of libpmg.so: argument marshalling only.

Every function has the name of the C entry point it wraps (without the pmg_ prefix) and
calls it once; all work runs in the library's HIP kernels.  Device vectors are
contiguous torch tensors on the current HIP device (float64 for PMG_FP64 calls,
float32 for PMG_FP32), passed by pointer together with torch's current stream.  The
library must have been built (python -m paper_2512_02577_amd.build); there is no
fallback: a missing library raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpmg.so")

OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_OUT_OF_MEMORY, ERR_DEVICE, ERR_NOT_CONVERGED, ERR_BREAKDOWN, ERR_STATE = (
    0, -1, -2, -3, -4, -5, -6, -7)
FP64, FP32, FP32_BF16 = 0, 1, 2
LOCAL_HALF_V, LOCAL_FULL_V, LOCAL_DIRECT = 0, 1, 2
SMOOTHER_JACOBI, SMOOTHER_REINFORCED = 0, 1
LANES_AUTO, LANES_NARROW, LANES_WIDE, LANES_HALF = 0, 1, 2, 3


class PmgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"pmg status {status}: {message}")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [("local_solver", ctypes.c_int), ("n_local_iter", ctypes.c_int), ("n_pre", ctypes.c_int),
                ("n_post", ctypes.c_int), ("max_iter", ctypes.c_int), ("rtol", ctypes.c_double),
                ("n_omega", ctypes.c_int), ("omega", ctypes.c_double * 8), ("patch_lanes", ctypes.c_int),
                ("local_smoother", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("rel_residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("status", ctypes.c_int)]


_lib = None
_vp, _ip, _dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_double


def lib() -> ctypes.CDLL:
    """The loaded libpmg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2512_02577_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        sig = {
            "pmg_last_error": (ctypes.c_char_p, []),
            "pmg_default_config": (None, [P(Config)]),
            "pmg_setup_mesh": (_ip, [_ip, P(ctypes.c_int32), _ip, P(_dp), P(_vp)]),
            "pmg_mesh_levels": (_ip, [_vp, P(_ip), P(_ip), P(ctypes.c_int32)]),
            "pmg_destroy_mesh": (None, [_vp]),
            "pmg_setup_dofmap": (_ip, [_vp, _ip, P(ctypes.c_int32), _ip, P(Config), P(_vp)]),
            "pmg_problem_sizes": (_ip, [_vp, P(_ip), P(_ip), P(_ip), P(ctypes.c_int32), P(ctypes.c_int64),
                                        P(ctypes.c_int64), P(ctypes.c_int32), P(_dp)]),
            "pmg_export_maps": (_ip, [_vp, _ip, _ip, P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_int32),
                                      P(ctypes.c_uint8)]),
            "pmg_get_qpoints": (_ip, [_vp, _ip, _ip, P(_dp)]),
            "pmg_set_coefficient": (_ip, [_vp, _ip, _ip, P(_dp)]),
            "pmg_device_init": (_ip, [_vp]),
            "pmg_apply_operator": (_ip, [_vp, _ip, _ip, _vp, _vp, _vp]),
            "pmg_mass_operator": (_ip, [_vp, _ip, _ip, _vp, _vp, _vp]),
            "pmg_residual": (_ip, [_vp, _ip, _ip, _vp, _vp, _vp, _vp]),
            "pmg_smooth": (_ip, [_vp, _ip, _ip, _ip, _vp, _vp, _vp]),
            "pmg_local_solve": (_ip, [_vp, _ip, _ip, _ip, _ip, _vp, _vp, _vp]),
            "pmg_restrict": (_ip, [_vp, _ip, _ip, _vp, _vp, _vp]),
            "pmg_prolongate_add": (_ip, [_vp, _ip, _ip, _vp, _vp, _vp]),
            "pmg_coarse_solve": (_ip, [_vp, _ip, _vp, _vp, _vp]),
            "pmg_vcycle": (_ip, [_vp, _ip, _vp, _vp, _vp]),
            "pmg_vcycle_noalloc": (_ip, [_vp, _ip, _vp, _vp, _vp]),
            "pmg_solve": (_ip, [_vp, _ip, _vp, _vp, _ip, P(SolveInfo), _vp]),
            "pmg_destroy_problem": (None, [_vp]),
            "pmg_batch_create": (_ip, [P(_vp), _ip, ctypes.c_char_p, P(_vp)]),
            "pmg_batch_stats": (_ip, [_vp, _ip, P(_ip), P(_ip)]),
            "pmg_batch_vcycle": (_ip, [_vp, _ip, P(_vp), P(_vp), _vp]),
            "pmg_batch_solve": (_ip, [_vp, _ip, P(_vp), P(_vp), P(SolveInfo), _vp]),
            "pmg_destroy_batch": (None, [_vp]),
            "pmg_setup_hex": (_ip, [_ip, _ip, ctypes.c_int64, P(_dp), ctypes.c_int64, P(ctypes.c_int32),
                                    ctypes.c_int64, P(ctypes.c_int32), P(Config), P(_vp)]),
            "pmg_hex_sizes": (_ip, [_vp, P(ctypes.c_int64), P(_ip), P(_ip), P(_ip), P(ctypes.c_int32), P(_dp)]),
            "pmg_hex_export": (_ip, [_vp, P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_int32),
                                     P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_uint8)]),
            "pmg_hex_device_init": (_ip, [_vp]),
            "pmg_hex_apply": (_ip, [_vp, _ip, _vp, _vp, _vp]),
            "pmg_hex_residual": (_ip, [_vp, _ip, _vp, _vp, _vp, _vp]),
            "pmg_hex_smooth": (_ip, [_vp, _ip, _ip, _vp, _vp, _vp]),
            "pmg_hex_destroy": (None, [_vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().pmg_last_error().decode()


def _check(rc: int) -> int:
    if rc != OK:
        raise PmgError(rc, last_error())
    return rc


def default_config() -> Config:
    c = Config()
    lib().pmg_default_config(ctypes.byref(c))
    return c


def _stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _prec_of(t, bf16: bool = False) -> int:
    import torch

    if t.dtype == torch.float64:
        return FP64
    if t.dtype == torch.float32:
        return FP32_BF16 if bf16 else FP32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _nodes(pr: "Problem", hlevel: int):
    """Expected vector length on an h-level, or None when the level is out of range
    (the library then rejects the call with its own error)."""
    return pr.n_nodes[hlevel] if 0 <= hlevel < len(pr.n_nodes) else None


def _ptr(t, n: int | None = None, dtype=None):
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("vectors must be contiguous device tensors")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} entries, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


class Mesh:
    """Handle of a pmg_mesh (setup_mesh)."""

    def __init__(self, handle: ctypes.c_void_p):
        self.handle = handle

    def levels(self) -> list[int]:
        nh = ctypes.c_int()
        _check(lib().pmg_mesh_levels(self.handle, None, ctypes.byref(nh), None))
        out = (ctypes.c_int32 * nh.value)()
        _check(lib().pmg_mesh_levels(self.handle, None, None, out))
        return list(out)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.pmg_destroy_mesh(self.handle)
            self.handle = None


class Problem:
    """Handle of a pmg_problem (setup_dofmap) with its sizes."""

    def __init__(self, handle: ctypes.c_void_p, degree: int):
        self.handle = handle
        self.p = degree
        dim, nh, npl = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().pmg_problem_sizes(handle, ctypes.byref(dim), ctypes.byref(nh), ctypes.byref(npl), None, None,
                                       None, None, None))
        self.dim, self.n_hlevels, self.n_plevels = dim.value, nh.value, npl.value
        cells = (ctypes.c_int32 * nh.value)()
        nodes = (ctypes.c_int64 * nh.value)()
        patches = (ctypes.c_int64 * nh.value)()
        deg = (ctypes.c_int32 * npl.value)()
        om = (ctypes.c_double * npl.value)()
        _check(lib().pmg_problem_sizes(handle, None, None, None, cells, nodes, patches, deg, om))
        self.cells, self.n_nodes, self.n_patches = list(cells), list(nodes), list(patches)
        self.degrees, self.omega = list(deg), list(om)
        self.finest = nh.value - 1

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.pmg_destroy_problem(self.handle)
            self.handle = None


def setup_mesh(dim: int, n, n_hlevels: int = 0, vertices: np.ndarray | None = None) -> Mesh:
    """n: cells per direction (an int, or a sequence of dim counts)."""
    h = ctypes.c_void_p()
    vp = None
    if vertices is not None:
        vertices = np.ascontiguousarray(vertices, dtype=np.float64)
        vp = vertices.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    cells = [int(n)] * 3 if np.isscalar(n) else [int(x) for x in n] + [0] * (3 - len(n))
    _check(lib().pmg_setup_mesh(dim, (ctypes.c_int32 * 3)(*cells), n_hlevels, vp, ctypes.byref(h)))
    return Mesh(h)


def setup_dofmap(mesh: Mesh, degree: int, p_levels=None, config: Config | None = None) -> Problem:
    h = ctypes.c_void_p()
    lv, nl = None, 0
    if p_levels is not None:
        nl = len(p_levels)
        lv = (ctypes.c_int32 * nl)(*p_levels)
    cfg = ctypes.byref(config) if config is not None else None
    _check(lib().pmg_setup_dofmap(mesh.handle, degree, lv, nl, cfg, ctypes.byref(h)))
    return Problem(h, degree)


def export_maps(pr: Problem, hlevel: int, plevel: int) -> dict[str, np.ndarray]:
    n = pr.cells[hlevel]
    q = pr.degrees[plevel]
    d = pr.dim
    cd = np.empty((n ** d, (q + 1) ** d), dtype=np.int32)
    npch = (n - 1) ** d
    pi = np.empty((npch, (2 * q - 1) ** d), dtype=np.int32)
    pc = np.empty((npch, (2 * q + 1) ** d), dtype=np.int32)
    col = np.empty(npch, dtype=np.uint8)
    P32 = ctypes.POINTER(ctypes.c_int32)
    _check(lib().pmg_export_maps(pr.handle, hlevel, plevel, cd.ctypes.data_as(P32), pi.ctypes.data_as(P32),
                                 pc.ctypes.data_as(P32), col.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
    return {"cell_dofs": cd, "patch_interior": pi, "patch_closure": pc, "patch_color": col}


def get_qpoints(pr: Problem, hlevel: int, plevel: int) -> np.ndarray:
    """Physical Gauss points, shape (cells, (q+1)^dim, dim)."""
    q = pr.degrees[plevel]
    out = np.empty((pr.cells[hlevel] ** pr.dim, (q + 1) ** pr.dim, pr.dim), dtype=np.float64)
    _check(lib().pmg_get_qpoints(pr.handle, hlevel, plevel, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def set_coefficient(pr: Problem, hlevel: int, plevel: int, a_q: np.ndarray | None) -> None:
    ptr = None
    if a_q is not None:
        a_q = np.ascontiguousarray(a_q, dtype=np.float64)
        q = pr.degrees[plevel]
        if a_q.size != pr.cells[hlevel] ** pr.dim * (q + 1) ** pr.dim:
            raise ValueError("one coefficient value per Gauss point expected")
        ptr = a_q.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    _check(lib().pmg_set_coefficient(pr.handle, hlevel, plevel, ptr))


def set_coefficient_field(pr: Problem, field) -> None:
    """Evaluates field(x) (x: (npoints, dim) array) at the Gauss points of every h- and
    p-level and passes the values to the library."""
    for hl in range(pr.n_hlevels):
        for pl in range(pr.n_plevels):
            x = get_qpoints(pr, hl, pl)
            set_coefficient(pr, hl, pl, field(x.reshape(-1, pr.dim)))


def device_init(pr: Problem) -> None:
    _check(lib().pmg_device_init(pr.handle))


def apply_operator(pr: Problem, hlevel: int, u, v, bf16: bool = False) -> None:
    n = _nodes(pr, hlevel)
    _check(lib().pmg_apply_operator(pr.handle, hlevel, _prec_of(u, bf16), _ptr(u, n), _ptr(v, n, u.dtype),
                                    _stream()))


def mass_operator(pr: Problem, hlevel: int, u, v) -> None:
    """v = M u (consistent mass matrix, zero Dirichlet rows and columns; Cartesian mesh)."""
    n = _nodes(pr, hlevel)
    _check(lib().pmg_mass_operator(pr.handle, hlevel, _prec_of(u), _ptr(u, n), _ptr(v, n, u.dtype), _stream()))


def residual(pr: Problem, hlevel: int, b, u, r) -> None:
    n = _nodes(pr, hlevel)
    _check(lib().pmg_residual(pr.handle, hlevel, _prec_of(u), _ptr(b, n, u.dtype), _ptr(u, n), _ptr(r, n, u.dtype),
                              _stream()))


def smooth(pr: Problem, hlevel: int, u, b, color_dir: int = 1, bf16: bool = False) -> None:
    n = _nodes(pr, hlevel)
    _check(lib().pmg_smooth(pr.handle, hlevel, _prec_of(u, bf16), color_dir, _ptr(u, n), _ptr(b, n, u.dtype),
                            _stream()))


def local_solve(pr: Problem, hlevel: int, r, d, first_patch: int = 0) -> None:
    blk = (2 * pr.p - 1) ** pr.dim
    if r.numel() % blk or d.numel() != r.numel():
        raise ValueError("r and d must hold whole patch-interior blocks")
    _check(lib().pmg_local_solve(pr.handle, hlevel, _prec_of(r), first_patch, r.numel() // blk, _ptr(r),
                                 _ptr(d, dtype=r.dtype), _stream()))


def restrict(pr: Problem, hlevel: int, fine, coarse) -> None:
    _check(lib().pmg_restrict(pr.handle, hlevel, _prec_of(fine), _ptr(fine, _nodes(pr, hlevel)),
                              _ptr(coarse, _nodes(pr, hlevel - 1), fine.dtype), _stream()))


def prolongate_add(pr: Problem, hlevel: int, coarse, fine) -> None:
    _check(lib().pmg_prolongate_add(pr.handle, hlevel, _prec_of(fine),
                                    _ptr(coarse, _nodes(pr, hlevel - 1), fine.dtype),
                                    _ptr(fine, _nodes(pr, hlevel)), _stream()))


def coarse_solve(pr: Problem, r, z) -> None:
    n = pr.n_nodes[0]
    _check(lib().pmg_coarse_solve(pr.handle, _prec_of(r), _ptr(r, n), _ptr(z, n, r.dtype), _stream()))


def vcycle(pr: Problem, r, z, mg_prec: int = FP64) -> None:
    import torch

    n = pr.n_nodes[pr.finest]
    _check(lib().pmg_vcycle(pr.handle, mg_prec, _ptr(r, n, torch.float64), _ptr(z, n, torch.float64), _stream()))


def vcycle_noalloc(pr: Problem, r, z, mg_prec: int = FP64) -> None:
    import torch

    n = pr.n_nodes[pr.finest]
    _check(lib().pmg_vcycle_noalloc(pr.handle, mg_prec, _ptr(r, n, torch.float64), _ptr(z, n, torch.float64),
                                    _stream()))


NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024


def solve(pr: Problem, b, x, mg_prec: int = FP64, x_is_initial_guess: bool = False,
          raise_on_failure: bool = True) -> SolveInfo:
    import torch

    n = pr.n_nodes[pr.finest]
    info = SolveInfo()
    rc = lib().pmg_solve(pr.handle, mg_prec, _ptr(b, n, torch.float64), _ptr(x, n, torch.float64),
                         int(x_is_initial_guess), ctypes.byref(info), _stream())
    if rc != OK and raise_on_failure:
        raise PmgError(rc, last_error())
    return info


def make_problem(dim: int, n: int, p: int, p_levels=None, n_hlevels: int = 0, config: Config | None = None,
                 device: bool = True, vertices: np.ndarray | None = None, coefficient=None) -> Problem:
    """setup_mesh + setup_dofmap (+ coefficient at every level's Gauss points) (+ device_init)."""
    mesh = setup_mesh(dim, n, n_hlevels, vertices)
    pr = setup_dofmap(mesh, p, p_levels, config)
    pr._mesh = mesh
    if coefficient is not None:
        set_coefficient_field(pr, coefficient)
    if device:
        device_init(pr)
    return pr


BATCH_MAX = 16


class Batch:
    """Handle of a batch of problems (pmg_batch_create); keeps its problems alive."""

    def __init__(self, handle: ctypes.c_void_p, problems: list[Problem]):
        self.handle = handle
        self.problems = problems

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.pmg_destroy_batch(self.handle)
            self.handle = None


def batch_create(problems: list[Problem], tuning_cache: str | None = None) -> Batch:
    arr = (ctypes.c_void_p * len(problems))(*[pr.handle.value if isinstance(pr.handle, ctypes.c_void_p)
                                              else pr.handle for pr in problems])
    h = ctypes.c_void_p()
    path = tuning_cache.encode() if tuning_cache else None
    _check(lib().pmg_batch_create(arr, len(problems), path, ctypes.byref(h)))
    return Batch(h, list(problems))


def batch_stats(bt: Batch, mg_prec: int = FP32) -> tuple[int, int]:
    st, la = ctypes.c_int(), ctypes.c_int()
    _check(lib().pmg_batch_stats(bt.handle, mg_prec, ctypes.byref(st), ctypes.byref(la)))
    return st.value, la.value


def _vec_array(bt: Batch, ts) -> ctypes.Array:
    import torch

    if len(ts) != len(bt.problems):
        raise ValueError(f"expected {len(bt.problems)} vectors, got {len(ts)}")
    return (ctypes.c_void_p * len(ts))(*[_ptr(t, pr.n_nodes[pr.finest], torch.float64).value
                                         for t, pr in zip(ts, bt.problems)])


def batch_vcycle(bt: Batch, r, z, mg_prec: int = FP32) -> None:
    _check(lib().pmg_batch_vcycle(bt.handle, mg_prec, _vec_array(bt, r), _vec_array(bt, z), _stream()))


def batch_solve(bt: Batch, b, x, mg_prec: int = FP32, raise_on_failure: bool = True) -> list[SolveInfo]:
    infos = (SolveInfo * len(bt.problems))()
    rc = lib().pmg_batch_solve(bt.handle, mg_prec, _vec_array(bt, b), _vec_array(bt, x), infos, _stream())
    if rc != OK and raise_on_failure:
        raise PmgError(rc, last_error())
    return list(infos)


# ---------------------------------------------------------------------------------------
# General hex meshes with stored maps
# ---------------------------------------------------------------------------------------
class HexProblem:
    """Handle of a pmg_hex (setup_hex) with its sizes."""

    def __init__(self, handle: ctypes.c_void_p, dim: int, degree: int, n_cells: int, n_dofs: int):
        self.handle = handle
        self.dim, self.p, self.n_cells, self.n_dofs = dim, degree, n_cells, n_dofs
        npat, npc, ncc, npl = ctypes.c_int64(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().pmg_hex_sizes(handle, ctypes.byref(npat), ctypes.byref(npc), ctypes.byref(ncc),
                                   ctypes.byref(npl), None, None))
        self.n_patches, self.n_patch_colors, self.n_cell_colors = npat.value, npc.value, ncc.value
        deg = (ctypes.c_int32 * npl.value)()
        om = (ctypes.c_double * npl.value)()
        _check(lib().pmg_hex_sizes(handle, None, None, None, None, deg, om))
        self.degrees, self.omega = list(deg), list(om)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.pmg_hex_destroy(self.handle)
            self.handle = None


def setup_hex(dim: int, degree: int, vertices, cell_vertices, cell_dofs, n_dofs: int,
              config: Config | None = None) -> HexProblem:
    P = ctypes.POINTER
    v = np.ascontiguousarray(vertices, dtype=np.float64)
    cv = np.ascontiguousarray(cell_vertices, dtype=np.int32)
    cd = np.ascontiguousarray(cell_dofs, dtype=np.int32)
    h = ctypes.c_void_p()
    _check(lib().pmg_setup_hex(dim, degree, len(v), v.ctypes.data_as(P(ctypes.c_double)), len(cv),
                               cv.ctypes.data_as(P(ctypes.c_int32)), int(n_dofs), cd.ctypes.data_as(P(ctypes.c_int32)),
                               ctypes.byref(config) if config is not None else None, ctypes.byref(h)))
    return HexProblem(h, dim, degree, len(cv), int(n_dofs))


def hex_export(hp: HexProblem) -> dict:
    P = ctypes.POINTER
    ncn, N = 2 ** hp.dim, (2 * hp.p + 1) ** hp.dim
    out = {"patch_vertex": np.empty(hp.n_patches, np.int32), "patch_color": np.empty(hp.n_patches, np.int32),
           "patch_cells": np.empty((hp.n_patches, ncn), np.int32),
           "patch_closure": np.empty((hp.n_patches, N), np.int32), "cell_color": np.empty(hp.n_cells, np.int32),
           "boundary": np.empty(hp.n_dofs, np.uint8)}
    i32 = lambda a: a.ctypes.data_as(P(ctypes.c_int32))  # noqa: E731
    _check(lib().pmg_hex_export(hp.handle, i32(out["patch_vertex"]), i32(out["patch_color"]),
                                i32(out["patch_cells"]), i32(out["patch_closure"]), i32(out["cell_color"]),
                                out["boundary"].ctypes.data_as(P(ctypes.c_uint8))))
    return out


def hex_device_init(hp: HexProblem) -> None:
    _check(lib().pmg_hex_device_init(hp.handle))


def hex_apply(hp: HexProblem, u, v) -> None:
    _check(lib().pmg_hex_apply(hp.handle, _prec_of(u), _ptr(u, hp.n_dofs), _ptr(v, hp.n_dofs, u.dtype), _stream()))


def hex_residual(hp: HexProblem, b, u, r) -> None:
    _check(lib().pmg_hex_residual(hp.handle, _prec_of(u), _ptr(b, hp.n_dofs, u.dtype), _ptr(u, hp.n_dofs),
                                  _ptr(r, hp.n_dofs, u.dtype), _stream()))


def hex_smooth(hp: HexProblem, u, b, color_dir: int = 1) -> None:
    _check(lib().pmg_hex_smooth(hp.handle, _prec_of(u), color_dir, _ptr(u, hp.n_dofs), _ptr(b, hp.n_dofs, u.dtype),
                                _stream()))
