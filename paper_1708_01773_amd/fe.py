"""Thin ctypes binding of the C ABI in include/fe.h (argument marshalling only).

Every step of the finite element path runs in the HIP kernels of libfe.so;
PyTorch is used here only to own device buffers and to provide streams.  If the
library is missing the import fails loudly: there is no CPU fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfe.so")

FE_OK, FE_EINVAL, FE_ENOMEM, FE_EMESH, FE_ENOTCONV, FE_EBREAKDOWN, FE_EDEVICE = range(7)
STATUS_NAMES = {0: "FE_OK", 1: "FE_EINVAL", 2: "FE_ENOMEM", 3: "FE_EMESH", 4: "FE_ENOTCONV",
                5: "FE_EBREAKDOWN", 6: "FE_EDEVICE"}
FE_POISSON, FE_ELASTICITY = 0, 1
FE_FP64, FE_FP32, FE_FP16, FE_BF16 = 0, 1, 2, 3
PRECISIONS = {"fp64": FE_FP64, "fp32": FE_FP32, "fp16": FE_FP16, "bf16": FE_BF16}
FE_SOURCE_NONE, FE_SOURCE_CONST, FE_SOURCE_SINPROD = 0, 1, 2
FE_DIRICHLET_ZERO, FE_DIRICHLET_AFFINE = 0, 1
FE_NEDELEC, FE_RAVIART_THOMAS, FE_NEDELEC2, FE_RAVIART_THOMAS2 = 1, 2, 3, 4
FAMILIES = {"nedelec": FE_NEDELEC, "raviart_thomas": FE_RAVIART_THOMAS, "nedelec2": FE_NEDELEC2,
            "raviart_thomas2": FE_RAVIART_THOMAS2}

# every entry point include/fe.h declares
EXPORTS = [
    "fe_last_error", "fe_version", "fe_create_mesh", "fe_destroy_mesh", "fe_set_coefficients",
    "fe_assemble_query", "fe_pattern", "fe_assemble", "fe_integrate", "fe_element_layout", "fe_scatter",
    "fe_cell_dofs", "fe_permutation", "fe_get_status", "fe_pcg_query", "fe_pcg_solve", "fe_spmv",
    "fe_set_timing", "fe_get_timing", "fe_csr_to_fp32", "fe_refine_query", "fe_refine_solve",
    "fe_pcg_batch_query", "fe_pcg_solve_batch", "fe_assemble_batch_query", "fe_assemble_batch",
    "fe_spmv_autotune_query", "fe_spmv_autotune", "fe_spmv_tuning_reset", "fe_spmv_plan_of",
    "fe_server_create", "fe_server_submit", "fe_server_poll", "fe_server_wait", "fe_server_solution",
    "fe_server_release", "fe_server_get_stats", "fe_server_clock", "fe_server_destroy",
    "fe_spmv_mesh", "fe_pcg_solve_mesh", "fe_pcg_solve_batch_mesh", "fe_spmv_autotune_mesh", "fe_spmv_plan_of_mesh",
    "fe_spmv_plan_set_mesh", "fe_sym_query", "fe_sym_from_csr", "fe_spmv_sym", "fe_pcg_solve_sym",
    "fe_sym_fp32_from_csr", "fe_refine_solve_sym", "fe_spmv_plan_set", "fe_pcg_solve_noalloc",
    "fe_refine_solve_mesh", "fe_refine_batch_query", "fe_refine_solve_batch_mesh", "fe_integrate_autotune",
    "fe_integrate_plan_of", "fe_dg_query", "fe_dg_pattern", "fe_dg_assemble", "fe_dg_spmv", "fe_dg_pcg_solve",
    "fe_stokes_create", "fe_stokes_destroy", "fe_stokes_query", "fe_stokes_assemble", "fe_stokes_system",
    "fe_stokes_solve", "fe_simplex_create", "fe_simplex_destroy", "fe_simplex_query", "fe_simplex_cell_dofs",
    "fe_simplex_pattern", "fe_simplex_assemble", "fe_simplex_elements", "fe_simplex_create_vector",
]

FE_REQ_QUEUED, FE_REQ_SETUP, FE_REQ_SOLVING, FE_REQ_DONE, FE_REQ_FAILED = 0, 1, 2, 3, 4

_c = ctypes
_P = _c.c_void_p


class FeError(RuntimeError):
    def __init__(self, status, where, text):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {text}")


class MeshDesc(_c.Structure):
    _fields_ = [("dim", _c.c_int32), ("n", _c.c_int32 * 3), ("vertex_xyz", _P), ("cell_coeff", _P)]


class Coeff(_c.Structure):
    _fields_ = [("problem", _c.c_int32), ("precision", _c.c_int32), ("young", _c.c_double),
                ("poisson_ratio", _c.c_double), ("source_kind", _c.c_int32), ("source", _c.c_double * 3),
                ("dirichlet_faces", _c.c_uint32), ("dirichlet_kind", _c.c_int32),
                ("dirichlet_affine", _c.c_double * 12)]


class SimplexDesc(_c.Structure):
    _fields_ = [("dim", _c.c_int32), ("nverts", _c.c_int64), ("ncells", _c.c_int64), ("vertex_xyz", _P),
                ("cells", _P), ("cell_coeff", _P)]


class Csr(_c.Structure):
    _fields_ = [("n_rows", _c.c_int64), ("nnz", _c.c_int64), ("rowptr", _P), ("colind", _P), ("values", _P),
                ("rhs", _P), ("dinv", _P)]


class SolveInfo(_c.Structure):
    _fields_ = [("iters", _c.c_int32), ("status", _c.c_int32), ("relres", _c.c_double),
                ("true_relres", _c.c_double), ("lambda_min_est", _c.c_double), ("lambda_max_est", _c.c_double)]


class Request(_c.Structure):
    _fields_ = [("mesh", MeshDesc), ("order", _c.c_int32), ("coeff", Coeff), ("rtol", _c.c_double),
                ("maxit", _c.c_int32)]


class Result(_c.Structure):
    _fields_ = [("state", _c.c_int32), ("status", _c.c_int32), ("n_rows", _c.c_int64), ("nnz", _c.c_int64),
                ("bytes", _c.c_int64), ("iters", _c.c_int32), ("relres", _c.c_double),
                ("true_relres", _c.c_double), ("t_submit", _c.c_double), ("t_admit", _c.c_double),
                ("t_ready", _c.c_double), ("t_done", _c.c_double)]


class ServerStats(_c.Structure):
    _fields_ = [("budget", _c.c_int64), ("arena_bytes", _c.c_int64), ("mesh_reserve", _c.c_int64),
                ("in_use", _c.c_int64), ("peak_in_use", _c.c_int64), ("peak_arena", _c.c_int64),
                ("queued", _c.c_int32), ("setting_up", _c.c_int32), ("solving", _c.c_int32),
                ("peak_solving", _c.c_int32), ("submitted", _c.c_int64), ("admitted", _c.c_int64),
                ("completed", _c.c_int64), ("rejected", _c.c_int64), ("chunks", _c.c_int64),
                ("admission_waits", _c.c_int64)]


class SpmvPlan(_c.Structure):
    _fields_ = [("mode", _c.c_int32), ("rows_per_wave", _c.c_int32), ("us", _c.c_double)]


class K3Plan(_c.Structure):
    _fields_ = [("pairs_per_wave", _c.c_int32), ("parts", _c.c_int32), ("us", _c.c_double)]


class RefineInfo(_c.Structure):
    _fields_ = [("outer_iters", _c.c_int32), ("inner_iters", _c.c_int32), ("status", _c.c_int32),
                ("relres", _c.c_double)]


class Timing(_c.Structure):
    _fields_ = [("integrate_ms", _c.c_double), ("scatter_ms", _c.c_double), ("spmv_ms", _c.c_double),
                ("integrate_calls", _c.c_int64), ("scatter_calls", _c.c_int64), ("spmv_calls", _c.c_int64)]


_lib = None


def lib():
    """Load libfe.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        # torch first: libfe.so then binds to the HIP runtime torch already
        # loaded (same soname), so the process holds a single HIP runtime
        import torch  # noqa: F401
        L = _c.CDLL(LIB_PATH)
        L.fe_last_error.restype = _c.c_char_p
        L.fe_version.restype = _c.c_int32
        sigs = {
            "fe_create_mesh": [_c.POINTER(MeshDesc), _c.POINTER(_P)],
            "fe_destroy_mesh": [_P],
            "fe_set_coefficients": [_P, _P],
            "fe_assemble_query": [_P, _c.c_int32, _c.POINTER(Coeff), _c.POINTER(_c.c_int64),
                                  _c.POINTER(_c.c_int64), _c.POINTER(_c.c_size_t)],
            "fe_pattern": [_P, _c.c_int32, _c.POINTER(Coeff), _c.POINTER(Csr), _P],
            "fe_assemble": [_P, _c.c_int32, _c.POINTER(Coeff), _c.POINTER(Csr), _P, _c.c_size_t, _P],
            "fe_integrate": [_P, _c.c_int32, _c.POINTER(Coeff), _P, _c.c_size_t, _P],
            "fe_element_layout": [_P, _c.c_int32, _c.POINTER(Coeff), _c.POINTER(_c.c_int32),
                                  _c.POINTER(_c.c_int32), _c.POINTER(_c.c_int32), _c.POINTER(_c.c_size_t),
                                  _c.POINTER(_c.c_int32)],
            "fe_scatter": [_P, _c.c_int32, _c.POINTER(Coeff), _c.POINTER(Csr), _P, _c.c_size_t, _P],
            "fe_cell_dofs": [_P, _c.c_int32, _c.POINTER(Coeff), _P, _P],
            "fe_permutation": [_P, _c.c_int32, _c.POINTER(Coeff), _P, _P],
            "fe_get_status": [_P],
            "fe_pcg_query": [_c.c_int64, _c.POINTER(_c.c_size_t)],
            "fe_pcg_solve": [_c.POINTER(Csr), _P, _P, _c.c_double, _c.c_int32, _P, _c.c_size_t,
                             _c.POINTER(SolveInfo), _P],
            "fe_pcg_solve_noalloc": [_c.POINTER(Csr), _P, _P, _c.c_double, _c.c_int32, _c.POINTER(SolveInfo), _P],
            "fe_spmv": [_c.POINTER(Csr), _P, _P, _P],
            "fe_set_timing": [_c.c_int32],
            "fe_csr_to_fp32": [_c.POINTER(Csr), _P, _P],
            "fe_refine_query": [_c.c_int64, _c.POINTER(_c.c_size_t)],
            "fe_refine_solve": [_c.POINTER(Csr), _c.POINTER(Csr), _P, _P, _P, _c.c_double, _c.c_double, _c.c_int32,
                                _c.c_int32, _P, _c.c_size_t, _c.POINTER(RefineInfo), _P],
            "fe_get_timing": [_c.POINTER(Timing), _c.c_int32],
            "fe_assemble_batch_query": [_c.c_int32, _c.POINTER(_P), _c.POINTER(_c.c_int32), _c.POINTER(Coeff),
                                        _c.POINTER(_c.c_int64), _c.POINTER(_c.c_int64), _c.POINTER(_c.c_size_t)],
            "fe_assemble_batch": [_c.c_int32, _c.POINTER(_P), _c.POINTER(_c.c_int32), _c.POINTER(Coeff),
                                  _c.POINTER(Csr), _P, _c.c_size_t, _P],
            "fe_spmv_autotune_query": [_c.c_int64, _c.POINTER(_c.c_size_t)],
            "fe_spmv_autotune": [_c.POINTER(Csr), _c.c_int32, _P, _c.c_size_t, _c.POINTER(SpmvPlan), _c.c_int32,
                                 _c.POINTER(_c.c_int32), _c.POINTER(SpmvPlan), _P],
            "fe_spmv_tuning_reset": [],
            "fe_spmv_plan_of": [_c.c_int64, _c.c_int64, _c.POINTER(SpmvPlan), _c.POINTER(_c.c_int32)],
            "fe_spmv_plan_set": [_c.c_int64, _c.c_int64, _c.POINTER(SpmvPlan)],
            "fe_spmv_mesh": [_P, _c.c_int32, _c.POINTER(Coeff), _c.POINTER(Csr), _P, _P, _P],
            "fe_pcg_solve_mesh": [_P, _c.c_int32, _c.POINTER(Coeff), _c.POINTER(Csr), _P, _P, _c.c_double,
                                  _c.c_int32, _P, _c.c_size_t, _c.POINTER(SolveInfo), _P],
            "fe_pcg_solve_batch_mesh": [_c.c_int32, _c.POINTER(_P), _c.POINTER(_c.c_int32), _c.POINTER(Coeff),
                                        _c.POINTER(Csr), _c.POINTER(_P), _c.POINTER(_P), _c.c_double, _c.c_int32,
                                        _P, _c.c_size_t, _c.POINTER(SolveInfo), _P],
            "fe_spmv_autotune_mesh": [_P, _c.c_int32, _c.POINTER(Coeff), _c.POINTER(Csr), _c.c_int32, _P, _c.c_size_t,
                                      _c.POINTER(SpmvPlan), _c.c_int32, _c.POINTER(_c.c_int32), _c.POINTER(SpmvPlan), _P],
            "fe_spmv_plan_of_mesh": [_P, _c.c_int32, _c.POINTER(Coeff), _c.POINTER(SpmvPlan), _c.POINTER(_c.c_int32)],
            "fe_spmv_plan_set_mesh": [_P, _c.c_int32, _c.POINTER(Coeff), _c.POINTER(SpmvPlan)],
            "fe_sym_query": [_P, _c.c_int32, _c.POINTER(Coeff), _c.POINTER(_c.c_size_t)],
            "fe_sym_fp32_from_csr": [_P, _c.c_int32, _c.POINTER(Coeff), _c.POINTER(Csr), _P, _c.c_size_t, _P],
            "fe_integrate_autotune": [_P, _c.c_int32, _c.POINTER(Coeff), _P, _c.c_size_t, _c.c_int32,
                                      _c.POINTER(K3Plan), _c.c_int32, _c.POINTER(_c.c_int32), _c.POINTER(K3Plan), _P],
            "fe_integrate_plan_of": [_P, _c.c_int32, _c.POINTER(Coeff), _c.POINTER(K3Plan)],
            "fe_dg_query": [_P, _c.c_int32, _c.POINTER(_c.c_int64), _c.POINTER(_c.c_int64), _c.POINTER(_c.c_size_t)],
            "fe_dg_pattern": [_P, _c.c_int32, _c.POINTER(Csr), _P],
            "fe_dg_assemble": [_P, _c.c_int32, _c.POINTER(Coeff), _c.c_double, _c.c_double, _c.POINTER(Csr), _P,
                               _c.c_size_t, _P],
            "fe_dg_spmv": [_P, _c.c_int32, _c.POINTER(Csr), _P, _P, _P],
            "fe_stokes_create": [_P, _c.c_int32, _c.c_double, _c.POINTER(Coeff), _c.POINTER(_P)],
            "fe_stokes_destroy": [_P],
            "fe_simplex_create": [_c.POINTER(SimplexDesc), _c.c_int32, _c.POINTER(Coeff), _c.POINTER(_P)],
            "fe_simplex_destroy": [_P],
            "fe_simplex_create_vector": [_c.POINTER(SimplexDesc), _c.c_int32, _c.c_double, _c.POINTER(Coeff),
                                         _c.POINTER(_P)],
            "fe_simplex_query": [_P, _c.POINTER(_c.c_int64), _c.POINTER(_c.c_int64), _c.POINTER(_c.c_int64),
                                 _c.POINTER(_c.c_int64)],
            "fe_simplex_cell_dofs": [_P, _P, _P],
            "fe_simplex_pattern": [_P, _c.POINTER(Csr), _P],
            "fe_simplex_assemble": [_P, _c.POINTER(Csr), _P],
            "fe_simplex_elements": [_P, _c.POINTER(_P), _c.POINTER(_P)],
            "fe_stokes_query": [_P, _c.POINTER(_c.c_int64), _c.POINTER(_c.c_int64), _c.POINTER(_c.c_int64),
                                _c.POINTER(_c.c_int64)],
            "fe_stokes_assemble": [_P, _P],
            "fe_stokes_system": [_P, _c.POINTER(Csr), _c.POINTER(Csr), _c.POINTER(Csr), _c.POINTER(_P),
                                 _c.POINTER(_P)],
            "fe_stokes_solve": [_P, _c.c_double, _c.c_int32, _P, _P, _c.POINTER(SolveInfo), _P],
            "fe_dg_pcg_solve": [_P, _c.c_int32, _c.POINTER(Csr), _P, _P, _c.c_double, _c.c_int32, _P, _c.c_size_t,
                                _c.POINTER(SolveInfo), _P],
            "fe_refine_batch_query": [_c.c_int32, _c.POINTER(_c.c_int64), _c.POINTER(_c.c_size_t)],
            "fe_refine_solve_batch_mesh": [_c.c_int32, _c.POINTER(_P), _c.POINTER(_c.c_int32), _c.POINTER(Coeff),
                                           _c.POINTER(Csr), _c.POINTER(Csr), _c.POINTER(_P), _c.POINTER(_P),
                                           _c.c_double, _c.c_double, _c.c_int32, _c.c_int32, _P, _c.c_size_t,
                                           _c.POINTER(RefineInfo), _P],
            "fe_refine_solve_mesh": [_P, _c.c_int32, _c.POINTER(Coeff), _c.POINTER(Csr), _c.POINTER(Csr), _P, _P, _P,
                                     _c.c_double, _c.c_double, _c.c_int32, _c.c_int32, _P, _c.c_size_t,
                                     _c.POINTER(RefineInfo), _P],
            "fe_refine_solve_sym": [_P, _c.c_int32, _c.POINTER(Coeff), _c.POINTER(Csr), _c.POINTER(Csr), _P,
                                    _c.c_size_t, _P, _P, _c.c_double, _c.c_double, _c.c_int32, _c.c_int32, _P,
                                    _c.c_size_t, _c.POINTER(RefineInfo), _P],
            "fe_sym_from_csr": [_P, _c.c_int32, _c.POINTER(Coeff), _c.POINTER(Csr), _P, _c.c_size_t, _P],
            "fe_spmv_sym": [_P, _c.c_int32, _c.POINTER(Coeff), _P, _c.c_size_t, _P, _P, _P],
            "fe_pcg_solve_sym": [_P, _c.c_int32, _c.POINTER(Coeff), _c.POINTER(Csr), _P, _c.c_size_t, _P, _P,
                                 _c.c_double, _c.c_int32, _P, _c.c_size_t, _c.POINTER(SolveInfo), _P],
            "fe_server_create": [_c.c_size_t, _c.c_int32, _c.POINTER(_P)],
            "fe_server_submit": [_P, _c.POINTER(Request), _c.POINTER(_c.c_uint64)],
            "fe_server_poll": [_P, _c.c_uint64, _c.POINTER(Result)],
            "fe_server_wait": [_P, _c.c_uint64, _c.c_double, _c.POINTER(Result)],
            "fe_server_solution": [_P, _c.c_uint64, _P, _c.c_int64],
            "fe_server_release": [_P, _c.c_uint64],
            "fe_server_get_stats": [_P, _c.POINTER(ServerStats)],
            "fe_server_destroy": [_P],
            "fe_pcg_batch_query": [_c.c_int32, _c.POINTER(_c.c_int64), _c.POINTER(_c.c_size_t)],
            "fe_pcg_solve_batch": [_c.c_int32, _c.POINTER(Csr), _c.POINTER(_P), _c.POINTER(_P), _c.c_double,
                                   _c.c_int32, _P, _c.c_size_t, _c.POINTER(SolveInfo), _P],
        }
        for name, args in sigs.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = _c.c_int
        L.fe_server_clock.argtypes = [_P]
        L.fe_server_clock.restype = _c.c_double
        _lib = L
    return _lib


def _check(st, where):
    if st != FE_OK:
        raise FeError(st, where, lib().fe_last_error().decode())
    return st


def _stream(stream):
    """hipStream_t of a torch stream (None: torch's current stream)."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return _P(s.cuda_stream)


def _ptr(t):
    return None if t is None else _P(t.data_ptr())


def make_coeff(problem="poisson", precision="fp64", young=1.0, nu=0.3, source_kind=FE_SOURCE_NONE,
               source=(0.0, 0.0, 0.0), faces=None, dim=3, dirichlet_kind=FE_DIRICHLET_ZERO, affine=None):
    c = Coeff()
    c.problem = FE_ELASTICITY if problem == "elasticity" else FE_POISSON
    c.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    c.young, c.poisson_ratio = float(young), float(nu)
    c.source_kind = int(source_kind)
    src = list(source) + [0.0] * (3 - len(source))
    for i in range(3):
        c.source[i] = float(src[i])
    c.dirichlet_faces = ((1 << (2 * dim)) - 1) if faces is None else int(faces)
    c.dirichlet_kind = int(dirichlet_kind)
    aff = list(affine) if affine is not None else []
    aff = aff + [0.0] * (12 - len(aff))
    for i in range(12):
        c.dirichlet_affine[i] = float(aff[i])
    return c


class Mesh:
    """Owning wrapper of an fe_mesh handle."""

    def __init__(self, dim, n, vertices=None, coeff=None):
        import numpy as np
        d = MeshDesc()
        d.dim = int(dim)
        n = list(n) if hasattr(n, "__len__") else [int(n)] * dim
        n = n + [1] * (3 - len(n))
        for i in range(3):
            d.n[i] = int(n[i])
        self._v = None if vertices is None else np.ascontiguousarray(vertices, dtype=np.float64)
        self._k = None if coeff is None else np.ascontiguousarray(coeff, dtype=np.float64)
        d.vertex_xyz = None if self._v is None else self._v.ctypes.data_as(_P)
        d.cell_coeff = None if self._k is None else self._k.ctypes.data_as(_P)
        h = _P()
        _check(lib().fe_create_mesh(_c.byref(d), _c.byref(h)), "fe_create_mesh")
        self.handle = h
        self.dim = int(dim)
        self.n = n[:dim]
        self._v = self._k = None

    def close(self):
        if self.handle is not None and self.handle.value:
            lib().fe_destroy_mesh(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def create_mesh(dim, n, vertices=None, coeff=None):
    return Mesh(dim, n, vertices, coeff)


def set_coefficients(mesh, coeff):
    import numpy as np
    k = np.ascontiguousarray(coeff, dtype=np.float64)
    _check(lib().fe_set_coefficients(mesh.handle, k.ctypes.data_as(_P)), "fe_set_coefficients")


def assemble_query(mesh, order, coeff):
    nr, nz, ws = _c.c_int64(), _c.c_int64(), _c.c_size_t()
    _check(lib().fe_assemble_query(mesh.handle, int(order), _c.byref(coeff), _c.byref(nr), _c.byref(nz),
                                   _c.byref(ws)), "fe_assemble_query")
    return nr.value, nz.value, ws.value


def element_layout(mesh, order, coeff):
    """(nloc, cells per block, element bytes, load offset, packed upper triangle)."""
    nloc, cb, eb, off, pk = _c.c_int32(), _c.c_int32(), _c.c_int32(), _c.c_size_t(), _c.c_int32()
    _check(lib().fe_element_layout(mesh.handle, int(order), _c.byref(coeff), _c.byref(nloc), _c.byref(cb),
                                   _c.byref(eb), _c.byref(off), _c.byref(pk)), "fe_element_layout")
    return nloc.value, cb.value, eb.value, off.value, pk.value


def csr_struct(n_rows, nnz, rowptr=None, colind=None, values=None, rhs=None, dinv=None):
    c = Csr()
    c.n_rows, c.nnz = int(n_rows), int(nnz)
    c.rowptr, c.colind, c.values, c.rhs, c.dinv = (_ptr(rowptr), _ptr(colind), _ptr(values), _ptr(rhs),
                                                   _ptr(dinv))
    return c


def pattern(mesh, order, coeff, csr, stream=None):
    _check(lib().fe_pattern(mesh.handle, int(order), _c.byref(coeff), _c.byref(csr), _stream(stream)), "fe_pattern")


def assemble(mesh, order, coeff, csr, ws, stream=None):
    _check(lib().fe_assemble(mesh.handle, int(order), _c.byref(coeff), _c.byref(csr), _ptr(ws),
                             ws.numel() * ws.element_size(), _stream(stream)), "fe_assemble")


def dg_query(mesh, order):
    """(n_rows, nnz, workspace bytes) of the interior-penalty DG system."""
    nr, nz, ws = _c.c_int64(), _c.c_int64(), _c.c_size_t()
    _check(lib().fe_dg_query(mesh.handle, int(order), _c.byref(nr), _c.byref(nz), _c.byref(ws)), "fe_dg_query")
    return nr.value, nz.value, ws.value


def dg_pattern(mesh, order, csr, stream=None):
    _check(lib().fe_dg_pattern(mesh.handle, int(order), _c.byref(csr), _stream(stream)), "fe_dg_pattern")


def dg_assemble(mesh, order, coeff, gamma, tau, csr, ws, stream=None):
    _check(lib().fe_dg_assemble(mesh.handle, int(order), _c.byref(coeff), float(gamma), float(tau), _c.byref(csr),
                                _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)), "fe_dg_assemble")


def dg_spmv(mesh, order, csr, x, y, stream=None):
    _check(lib().fe_dg_spmv(mesh.handle, int(order), _c.byref(csr), _ptr(x), _ptr(y), _stream(stream)), "fe_dg_spmv")


def dg_pcg_solve(mesh, order, csr, b, x, rtol, maxit, ws, stream=None, check=True):
    """Jacobi-PCG on a DG system with the cell-block SpMV; returns the info dict of pcg_solve."""
    info = SolveInfo()
    st = lib().fe_dg_pcg_solve(mesh.handle, int(order), _c.byref(csr), _ptr(b), _ptr(x), float(rtol), int(maxit),
                               _ptr(ws), ws.numel() * ws.element_size(), _c.byref(info), _stream(stream))
    out = dict(iters=info.iters, status=info.status, relres=info.relres, true_relres=info.true_relres,
               lambda_min_est=info.lambda_min_est, lambda_max_est=info.lambda_max_est)
    if check and st not in (FE_OK, FE_ENOTCONV, FE_EBREAKDOWN):
        _check(st, "fe_dg_pcg_solve")
    return out


def integrate(mesh, order, coeff, ws, stream=None):
    _check(lib().fe_integrate(mesh.handle, int(order), _c.byref(coeff), _ptr(ws), ws.numel() * ws.element_size(),
                              _stream(stream)), "fe_integrate")


def scatter(mesh, order, coeff, csr, ws, stream=None):
    _check(lib().fe_scatter(mesh.handle, int(order), _c.byref(coeff), _c.byref(csr), _ptr(ws),
                            ws.numel() * ws.element_size(), _stream(stream)), "fe_scatter")


def cell_dofs(mesh, order, coeff, out, stream=None):
    _check(lib().fe_cell_dofs(mesh.handle, int(order), _c.byref(coeff), _ptr(out), _stream(stream)), "fe_cell_dofs")


def permutation(mesh, order, coeff, out, stream=None):
    _check(lib().fe_permutation(mesh.handle, int(order), _c.byref(coeff), _ptr(out), _stream(stream)),
           "fe_permutation")


def get_status(mesh):
    return lib().fe_get_status(mesh.handle)


def pcg_query(n_rows):
    ws = _c.c_size_t()
    _check(lib().fe_pcg_query(int(n_rows), _c.byref(ws)), "fe_pcg_query")
    return ws.value


def pcg_solve(csr, b, x, rtol, maxit, ws, stream=None, check=True):
    """Returns a dict with iters, status, relres, true_relres, lambda_min_est, lambda_max_est."""
    info = SolveInfo()
    st = lib().fe_pcg_solve(_c.byref(csr), _ptr(b), _ptr(x), float(rtol), int(maxit), _ptr(ws),
                            ws.numel() * ws.element_size(), _c.byref(info), _stream(stream))
    out = dict(iters=info.iters, status=info.status, relres=info.relres, true_relres=info.true_relres,
               lambda_min_est=info.lambda_min_est, lambda_max_est=info.lambda_max_est)
    if check and st not in (FE_OK, FE_ENOTCONV, FE_EBREAKDOWN):
        _check(st, "fe_pcg_solve")
    return out


def pcg_solve_noalloc(csr, b, x, rtol, maxit, stream=None, check=True):
    """fe_pcg_solve with the library's static device workspace (no allocation)."""
    info = SolveInfo()
    st = lib().fe_pcg_solve_noalloc(_c.byref(csr), _ptr(b), _ptr(x), float(rtol), int(maxit), _c.byref(info),
                                    _stream(stream))
    out = _info_dict(info)
    if check and st not in (FE_OK, FE_ENOTCONV, FE_EBREAKDOWN):
        _check(st, "fe_pcg_solve_noalloc")
    return out


PCG_NOALLOC_MAX_ROWS = 2700000


def pcg_batch_query(n_rows):
    arr = (_c.c_int64 * max(1, len(n_rows)))(*[int(v) for v in n_rows])
    ws = _c.c_size_t()
    _check(lib().fe_pcg_batch_query(len(n_rows), arr, _c.byref(ws)), "fe_pcg_batch_query")
    return ws.value


def pcg_solve_batch(csrs, bs, xs, rtol, maxit, ws, stream=None, check=True):
    """Solves len(csrs) systems in one engine pass; returns (status, [info dicts])."""
    n = len(csrs)
    A = (Csr * max(1, n))(*csrs)
    B = (_P * max(1, n))(*[_ptr(b) for b in bs])
    X = (_P * max(1, n))(*[_ptr(x) for x in xs])
    infos = (SolveInfo * max(1, n))()
    st = lib().fe_pcg_solve_batch(n, A, B, X, float(rtol), int(maxit), _ptr(ws), ws.numel() * ws.element_size(),
                                  infos, _stream(stream))
    if check and st not in (FE_OK, FE_ENOTCONV, FE_EBREAKDOWN):
        _check(st, "fe_pcg_solve_batch")
    out = [dict(iters=i.iters, status=i.status, relres=i.relres, true_relres=i.true_relres) for i in infos[:n]]
    return st, out


def spmv_autotune(csr, reps=20, stream=None):
    """Times every SpMV plan on csr and keeps the fastest for its row-length
    class; returns (chosen, tried) as dicts (mode, rows_per_wave, us)."""
    import torch
    q = _c.c_size_t()
    _check(lib().fe_spmv_autotune_query(int(csr.n_rows), _c.byref(q)), "fe_spmv_autotune_query")
    ws = torch.empty(max(q.value, 8), dtype=torch.uint8, device="cuda")
    tried = (SpmvPlan * 32)()
    nt = _c.c_int32()
    ch = SpmvPlan()
    _check(lib().fe_spmv_autotune(_c.byref(csr), int(reps), _ptr(ws), q.value, tried, 32, _c.byref(nt),
                                  _c.byref(ch), _stream(stream)), "fe_spmv_autotune")
    d = lambda p: dict(mode=p.mode, rows_per_wave=p.rows_per_wave, us=p.us)
    return d(ch), [d(t) for t in tried[: nt.value]]


def spmv_autotune_mesh(mesh, order, coeff, csr, reps=20, stream=None):
    """Times every evaluated-pattern plan on csr (assembled on mesh) and keeps
    the fastest for its row class; returns (chosen, tried)."""
    import torch
    q = _c.c_size_t()
    _check(lib().fe_spmv_autotune_query(int(csr.n_rows), _c.byref(q)), "fe_spmv_autotune_query")
    ws = torch.empty(max(q.value, 8), dtype=torch.uint8, device="cuda")
    tried = (SpmvPlan * 32)()
    nt = _c.c_int32()
    ch = SpmvPlan()
    _check(lib().fe_spmv_autotune_mesh(mesh.handle, int(order), _c.byref(coeff), _c.byref(csr), int(reps), _ptr(ws),
                                       q.value, tried, 32, _c.byref(nt), _c.byref(ch), _stream(stream)),
           "fe_spmv_autotune_mesh")
    d = lambda p: dict(mode=p.mode, rows_per_wave=p.rows_per_wave, us=p.us)
    return d(ch), [d(t) for t in tried[: nt.value]]


def spmv_plan_set_mesh(mesh, order, coeff, mode, rows_per_wave):
    """Make (mode, rows_per_wave) the evaluated-pattern plan of this system's row class."""
    p = SpmvPlan(int(mode), int(rows_per_wave), 0.0)
    _check(lib().fe_spmv_plan_set_mesh(mesh.handle, int(order), _c.byref(coeff), _c.byref(p)),
           "fe_spmv_plan_set_mesh")


def spmv_plan_of_mesh(mesh, order, coeff):
    """(mode, rows_per_wave, row_class) of the evaluated-pattern traversal now."""
    p = SpmvPlan()
    c = _c.c_int32()
    _check(lib().fe_spmv_plan_of_mesh(mesh.handle, int(order), _c.byref(coeff), _c.byref(p), _c.byref(c)),
           "fe_spmv_plan_of_mesh")
    return p.mode, p.rows_per_wave, c.value


def integrate_autotune(mesh, order, coeff, ws, reps=5, stream=None):
    """Times every tile shape of the matrix-core integration of this class and
    keeps the fastest; returns (chosen, tried) as dicts (pairs_per_wave, parts, us)."""
    tried = (K3Plan * 8)()
    nt = _c.c_int32()
    ch = K3Plan()
    _check(lib().fe_integrate_autotune(mesh.handle, int(order), _c.byref(coeff), _ptr(ws), _nbytes(ws), int(reps),
                                       tried, 8, _c.byref(nt), _c.byref(ch), _stream(stream)), "fe_integrate_autotune")
    d = lambda p: dict(pairs_per_wave=p.pairs_per_wave, parts=p.parts, us=p.us)
    return d(ch), [d(t) for t in tried[: nt.value]]


def integrate_plan_of(mesh, order, coeff):
    """(pairs_per_wave, parts) of the class's matrix-core integration now."""
    p = K3Plan()
    _check(lib().fe_integrate_plan_of(mesh.handle, int(order), _c.byref(coeff), _c.byref(p)), "fe_integrate_plan_of")
    return p.pairs_per_wave, p.parts


def spmv_tuning_reset():
    _check(lib().fe_spmv_tuning_reset(), "fe_spmv_tuning_reset")


def spmv_plan_of(n_rows, nnz):
    """(mode, rows_per_wave, row_class) a matrix of this size gets now."""
    p = SpmvPlan()
    c = _c.c_int32()
    _check(lib().fe_spmv_plan_of(int(n_rows), int(nnz), _c.byref(p), _c.byref(c)), "fe_spmv_plan_of")
    return p.mode, p.rows_per_wave, c.value


def spmv_plan_set(n_rows, nnz, mode, rows_per_wave):
    """Make (mode, rows_per_wave) the CSR plan of the row-length class of an n_rows x nnz matrix."""
    p = SpmvPlan(int(mode), int(rows_per_wave), 0.0)
    _check(lib().fe_spmv_plan_set(int(n_rows), int(nnz), _c.byref(p)), "fe_spmv_plan_set")


def _info_dict(info):
    return dict(iters=info.iters, status=info.status, relres=info.relres, true_relres=info.true_relres,
                lambda_min_est=info.lambda_min_est, lambda_max_est=info.lambda_max_est)


def pcg_solve_mesh(mesh, order, coeff, csr, b, x, rtol, maxit, ws, stream=None, check=True):
    """Jacobi-PCG of a system assembled on mesh, with the pattern evaluated from the mesh."""
    info = SolveInfo()
    st = lib().fe_pcg_solve_mesh(mesh.handle, int(order), _c.byref(coeff), _c.byref(csr), _ptr(b), _ptr(x),
                                 float(rtol), int(maxit), _ptr(ws), ws.numel() * ws.element_size(), _c.byref(info),
                                 _stream(stream))
    if check and st not in (FE_OK, FE_ENOTCONV, FE_EBREAKDOWN):
        _check(st, "fe_pcg_solve_mesh")
    return _info_dict(info)


def spmv_mesh(mesh, order, coeff, csr, x, y, stream=None):
    _check(lib().fe_spmv_mesh(mesh.handle, int(order), _c.byref(coeff), _c.byref(csr), _ptr(x), _ptr(y),
                              _stream(stream)), "fe_spmv_mesh")


def sym_query(mesh, order, coeff):
    """Bytes of the symmetric storage (upper triangle, slot-major) of a Q1 scalar system."""
    nb = _c.c_size_t()
    _check(lib().fe_sym_query(mesh.handle, int(order), _c.byref(coeff), _c.byref(nb)), "fe_sym_query")
    return nb.value


def _nbytes(t):
    return t.numel() * t.element_size()


def sym_from_csr(mesh, order, coeff, csr, sym, stream=None):
    """sym (float64 device tensor of sym_query bytes) = upper triangle of csr."""
    _check(lib().fe_sym_from_csr(mesh.handle, int(order), _c.byref(coeff), _c.byref(csr), _ptr(sym), _nbytes(sym),
                                 _stream(stream)), "fe_sym_from_csr")


def spmv_sym(mesh, order, coeff, sym, x, y, stream=None):
    _check(lib().fe_spmv_sym(mesh.handle, int(order), _c.byref(coeff), _ptr(sym), _nbytes(sym), _ptr(x), _ptr(y),
                             _stream(stream)), "fe_spmv_sym")


def pcg_solve_sym(mesh, order, coeff, csr, sym, b, x, rtol, maxit, ws, stream=None, check=True):
    """Jacobi-PCG with the operator applied from its symmetric storage."""
    info = SolveInfo()
    st = lib().fe_pcg_solve_sym(mesh.handle, int(order), _c.byref(coeff), _c.byref(csr), _ptr(sym), _nbytes(sym),
                                _ptr(b), _ptr(x), float(rtol), int(maxit), _ptr(ws), _nbytes(ws), _c.byref(info),
                                _stream(stream))
    if check and st not in (FE_OK, FE_ENOTCONV, FE_EBREAKDOWN):
        _check(st, "fe_pcg_solve_sym")
    return _info_dict(info)


def pcg_solve_batch_mesh(meshes, orders, coeffs, csrs, bs, xs, rtol, maxit, ws, stream=None, check=True):
    n = len(csrs)
    M = (_P * max(1, n))(*[m.handle for m in meshes])
    O = (_c.c_int32 * max(1, n))(*[int(k) for k in orders])
    C = (Coeff * max(1, n))(*coeffs)
    A = (Csr * max(1, n))(*csrs)
    B = (_P * max(1, n))(*[_ptr(b) for b in bs])
    X = (_P * max(1, n))(*[_ptr(x) for x in xs])
    infos = (SolveInfo * max(1, n))()
    st = lib().fe_pcg_solve_batch_mesh(n, M, O, C, A, B, X, float(rtol), int(maxit), _ptr(ws),
                                       ws.numel() * ws.element_size(), infos, _stream(stream))
    if check and st not in (FE_OK, FE_ENOTCONV, FE_EBREAKDOWN):
        _check(st, "fe_pcg_solve_batch_mesh")
    return st, [dict(iters=i.iters, status=i.status, relres=i.relres, true_relres=i.true_relres) for i in infos[:n]]


def spmv(csr, x, y, stream=None):
    _check(lib().fe_spmv(_c.byref(csr), _ptr(x), _ptr(y), _stream(stream)), "fe_spmv")


def csr_to_fp32(csr, values32, stream=None):
    _check(lib().fe_csr_to_fp32(_c.byref(csr), _ptr(values32), _stream(stream)), "fe_csr_to_fp32")


def refine_query(n_rows):
    ws = _c.c_size_t()
    _check(lib().fe_refine_query(int(n_rows), _c.byref(ws)), "fe_refine_query")
    return ws.value


def refine_solve(A_hi, A_lo, b, x, rtol, inner_rtol, max_outer, max_inner, ws, values32=None, stream=None):
    """Iterative refinement; returns dict(outer_iters, inner_iters, status, relres)."""
    info = RefineInfo()
    st = lib().fe_refine_solve(_c.byref(A_hi), _c.byref(A_lo), _ptr(values32), _ptr(b), _ptr(x), float(rtol),
                               float(inner_rtol), int(max_outer), int(max_inner), _ptr(ws),
                               ws.numel() * ws.element_size(), _c.byref(info), _stream(stream))
    if st not in (FE_OK, FE_ENOTCONV):
        _check(st, "fe_refine_solve")
    return dict(outer_iters=info.outer_iters, inner_iters=info.inner_iters, status=info.status, relres=info.relres)


def refine_solve_mesh(mesh, order, coeff, A_hi, A_lo, b, x, rtol, inner_rtol, max_outer, max_inner, ws,
                      values32=None, stream=None):
    """Iterative refinement whose inner PCG evaluates the pattern from the mesh
    (FP32 values32, or A_lo's FP64 values); returns dict(outer_iters, inner_iters, status, relres)."""
    info = RefineInfo()
    st = lib().fe_refine_solve_mesh(mesh.handle, int(order), _c.byref(coeff), _c.byref(A_hi), _c.byref(A_lo),
                                    _ptr(values32), _ptr(b), _ptr(x), float(rtol), float(inner_rtol), int(max_outer),
                                    int(max_inner), _ptr(ws), ws.numel() * ws.element_size(), _c.byref(info),
                                    _stream(stream))
    if st not in (FE_OK, FE_ENOTCONV):
        _check(st, "fe_refine_solve_mesh")
    return dict(outer_iters=info.outer_iters, inner_iters=info.inner_iters, status=info.status, relres=info.relres)


def refine_batch_query(n_rows):
    n = len(n_rows)
    arr = (_c.c_int64 * max(1, n))(*[int(v) for v in n_rows])
    ws = _c.c_size_t()
    _check(lib().fe_refine_batch_query(n, arr, _c.byref(ws)), "fe_refine_batch_query")
    return ws.value


def refine_solve_batch_mesh(meshes, orders, coeffs, csrs_hi, csrs_lo, bs, xs, rtol, inner_rtol, max_outer, max_inner,
                            ws, stream=None, check=True):
    """Batched iterative refinement (FP64 residuals with csrs_hi, batched inner
    PCG on csrs_lo); returns (status, [dict(outer_iters, inner_iters, status, relres)])."""
    n = len(meshes)
    M = (_P * max(1, n))(*[m.handle for m in meshes])
    O = (_c.c_int32 * max(1, n))(*[int(k) for k in orders])
    C = (Coeff * max(1, n))(*coeffs)
    H = (Csr * max(1, n))(*csrs_hi)
    L = (Csr * max(1, n))(*csrs_lo)
    B = (_P * max(1, n))(*[_ptr(b) for b in bs])
    X = (_P * max(1, n))(*[_ptr(x) for x in xs])
    infos = (RefineInfo * max(1, n))()
    st = lib().fe_refine_solve_batch_mesh(n, M, O, C, H, L, B, X, float(rtol), float(inner_rtol), int(max_outer),
                                          int(max_inner), _ptr(ws), ws.numel() * ws.element_size(), infos,
                                          _stream(stream))
    if check and st not in (FE_OK, FE_ENOTCONV, FE_EBREAKDOWN):
        _check(st, "fe_refine_solve_batch_mesh")
    return st, [dict(outer_iters=i.outer_iters, inner_iters=i.inner_iters, status=i.status, relres=i.relres)
                for i in infos[:n]]


def sym_fp32_from_csr(mesh, order, coeff, csr, sym32, stream=None):
    """sym32 (float32 device tensor of sym_query / 2 bytes) = upper triangle of csr in FP32."""
    _check(lib().fe_sym_fp32_from_csr(mesh.handle, int(order), _c.byref(coeff), _c.byref(csr), _ptr(sym32),
                                      _nbytes(sym32), _stream(stream)), "fe_sym_fp32_from_csr")


def refine_solve_sym(mesh, order, coeff, A_hi, A_lo, sym32, b, x, rtol, inner_rtol, max_outer, max_inner, ws,
                     stream=None):
    """Iterative refinement with the inner PCG on the FP32 symmetric storage of A_lo."""
    info = RefineInfo()
    st = lib().fe_refine_solve_sym(mesh.handle, int(order), _c.byref(coeff), _c.byref(A_hi), _c.byref(A_lo),
                                   _ptr(sym32), _nbytes(sym32), _ptr(b), _ptr(x), float(rtol), float(inner_rtol),
                                   int(max_outer), int(max_inner), _ptr(ws), _nbytes(ws), _c.byref(info),
                                   _stream(stream))
    if st not in (FE_OK, FE_ENOTCONV):
        _check(st, "fe_refine_solve_sym")
    return dict(outer_iters=info.outer_iters, inner_iters=info.inner_iters, status=info.status, relres=info.relres)


def set_timing(enable):
    _check(lib().fe_set_timing(1 if enable else 0), "fe_set_timing")


def get_timing(reset=True):
    t = Timing()
    _check(lib().fe_get_timing(_c.byref(t), 1 if reset else 0), "fe_get_timing")
    return {f: getattr(t, f) for f, _ in Timing._fields_}


class Assembly:
    """Device buffers (torch tensors) of one assembled system plus its workspace."""

    def __init__(self, mesh, order, coeff, device="cuda"):
        import torch
        self.mesh, self.order, self.coeff = mesh, int(order), coeff
        self.n_rows, self.nnz, ws_bytes = assemble_query(mesh, order, coeff)
        dev = torch.device(device)
        self.rowptr = torch.empty(self.n_rows + 1, dtype=torch.int64, device=dev)
        self.colind = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=dev)
        self.values = torch.empty(max(self.nnz, 1), dtype=torch.float64, device=dev)
        self.rhs = torch.empty(max(self.n_rows, 1), dtype=torch.float64, device=dev)
        self.dinv = torch.empty(max(self.n_rows, 1), dtype=torch.float64, device=dev)
        self.ws = torch.empty(max(ws_bytes, 8), dtype=torch.uint8, device=dev)
        self.csr = csr_struct(self.n_rows, self.nnz, self.rowptr, self.colind, self.values, self.rhs, self.dinv)

    def pattern(self, stream=None):
        pattern(self.mesh, self.order, self.coeff, self.csr, stream)

    def assemble(self, stream=None):
        assemble(self.mesh, self.order, self.coeff, self.csr, self.ws, stream)

    def integrate(self, stream=None):
        integrate(self.mesh, self.order, self.coeff, self.ws, stream)

    def scatter(self, stream=None):
        scatter(self.mesh, self.order, self.coeff, self.csr, self.ws, stream)

    def solve(self, x, rtol, maxit, ws, stream=None):
        """Jacobi-PCG with the pattern evaluated from the mesh (fe_pcg_solve_mesh)."""
        return pcg_solve_mesh(self.mesh, self.order, self.coeff, self.csr, self.rhs, x, rtol, maxit, ws, stream)


class DGAssembly:
    """Device buffers (torch tensors) of one interior-penalty DG system plus its
    workspace; the pattern is written at construction."""

    def __init__(self, mesh, order, coeff, gamma, tau=1.0, device="cuda", stream=None):
        import torch
        self.mesh, self.order, self.coeff = mesh, int(order), coeff
        self.gamma, self.tau = float(gamma), float(tau)
        self.n_rows, self.nnz, ws_bytes = dg_query(mesh, order)
        dev = torch.device(device)
        self.rowptr = torch.empty(self.n_rows + 1, dtype=torch.int64, device=dev)
        self.colind = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=dev)
        self.values = torch.empty(max(self.nnz, 1), dtype=torch.float64, device=dev)
        self.rhs = torch.empty(max(self.n_rows, 1), dtype=torch.float64, device=dev)
        self.dinv = torch.empty(max(self.n_rows, 1), dtype=torch.float64, device=dev)
        self.ws = torch.empty(max(ws_bytes, 8), dtype=torch.uint8, device=dev)
        self.csr = csr_struct(self.n_rows, self.nnz, self.rowptr, self.colind, self.values, self.rhs, self.dinv)
        dg_pattern(mesh, order, self.csr, stream)

    def assemble(self, stream=None):
        dg_assemble(self.mesh, self.order, self.coeff, self.gamma, self.tau, self.csr, self.ws, stream)

    def spmv(self, x, y, stream=None):
        dg_spmv(self.mesh, self.order, self.csr, x, y, stream)

    def solve(self, x, rtol, maxit, ws, stream=None):
        """Jacobi-PCG with the cell-block SpMV (fe_dg_pcg_solve)."""
        return dg_pcg_solve(self.mesh, self.order, self.csr, self.rhs, x, rtol, maxit, ws, stream)


def _copy_to_host(out, ptr):
    """Copies device memory at ptr into the numpy array out (hipMemcpy through
    the HIP runtime libfe.so is linked against)."""
    L = lib()
    f = L.hipMemcpy
    f.argtypes = [_P, _P, _c.c_size_t, _c.c_int]
    f.restype = _c.c_int
    if f(out.ctypes.data_as(_P), _c.c_void_p(ptr), out.nbytes, 2) != 0:  # hipMemcpyDeviceToHost
        raise FeError(FE_EDEVICE, "hipMemcpy", "copy to the host failed")


class Stokes:
    """Owning wrapper of an fe_stokes handle (Taylor-Hood Q_{k+1}^d x Q_k on a
    mesh): assemble(), system() device views as torch tensors, solve()."""

    def __init__(self, mesh, order, mu=1.0, source_kind=FE_SOURCE_NONE, source=(0.0, 0.0, 0.0)):
        self.mesh, self.order, self.mu = mesh, int(order), float(mu)
        c = make_coeff("elasticity", "fp64", source_kind=source_kind, source=source, dim=mesh.dim)
        h = _P()
        _check(lib().fe_stokes_create(mesh.handle, self.order, self.mu, _c.byref(c), _c.byref(h)),
               "fe_stokes_create")
        self.handle = h
        nu, np_, na, nb = _c.c_int64(), _c.c_int64(), _c.c_int64(), _c.c_int64()
        _check(lib().fe_stokes_query(h, _c.byref(nu), _c.byref(np_), _c.byref(na), _c.byref(nb)), "fe_stokes_query")
        self.n_u, self.n_p, self.nnz_a, self.nnz_b = nu.value, np_.value, na.value, nb.value

    def assemble(self, stream=None):
        _check(lib().fe_stokes_assemble(self.handle, _stream(stream)), "fe_stokes_assemble")

    def system(self):
        """Host copies (numpy) of A (CSR arrays), B, B^T, md and the rhs."""
        import numpy as np
        import torch
        A, B, Bt = Csr(), Csr(), Csr()
        md, rhs = _P(), _P()
        _check(lib().fe_stokes_system(self.handle, _c.byref(A), _c.byref(B), _c.byref(Bt), _c.byref(md),
                                      _c.byref(rhs)), "fe_stokes_system")
        torch.cuda.synchronize()

        def dev(ptr, n, dtype):
            out = np.empty(n, dtype=dtype)
            if n > 0:
                _copy_to_host(out, ptr)
            return out

        def csr(C):
            return (dev(C.rowptr, C.n_rows + 1, np.int64), dev(C.colind, C.nnz, np.int32),
                    dev(C.values, C.nnz, np.float64))
        return dict(A=csr(A), B=csr(B), Bt=csr(Bt), md=dev(md.value, self.n_p, np.float64),
                    rhs=dev(rhs.value, self.n_u + self.n_p, np.float64), dinv=dev(A.dinv, self.n_u, np.float64))

    def solve(self, u, p, rtol, maxit, stream=None, check=True):
        info = SolveInfo()
        st = lib().fe_stokes_solve(self.handle, float(rtol), int(maxit), _ptr(u), _ptr(p), _c.byref(info),
                                   _stream(stream))
        out = dict(iters=info.iters, status=info.status, relres=info.relres, true_relres=info.true_relres)
        if check and st not in (FE_OK, FE_ENOTCONV, FE_EBREAKDOWN):
            _check(st, "fe_stokes_solve")
        return out

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            lib().fe_stokes_destroy(h)
            self.handle = None


def assemble_batch_query(meshes, orders, coeffs):
    """Per-problem (n_rows, nnz) lists and the batch workspace bytes."""
    n = len(meshes)
    M = (_P * max(1, n))(*[m.handle for m in meshes])
    O = (_c.c_int32 * max(1, n))(*[int(k) for k in orders])
    C = (Coeff * max(1, n))(*coeffs)
    nr = (_c.c_int64 * max(1, n))()
    nz = (_c.c_int64 * max(1, n))()
    ws = _c.c_size_t()
    _check(lib().fe_assemble_batch_query(n, M, O, C, nr, nz, _c.byref(ws)), "fe_assemble_batch_query")
    return list(nr[:n]), list(nz[:n]), ws.value


def assemble_batch(meshes, orders, coeffs, csrs, ws, stream=None):
    n = len(meshes)
    M = (_P * max(1, n))(*[m.handle for m in meshes])
    O = (_c.c_int32 * max(1, n))(*[int(k) for k in orders])
    C = (Coeff * max(1, n))(*coeffs)
    A = (Csr * max(1, n))(*csrs)
    _check(lib().fe_assemble_batch(n, M, O, C, A, _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)),
           "fe_assemble_batch")


class BatchAssembly:
    """Device buffers of a batch of independent systems: one CSR (pattern
    written once at construction), right-hand side, diagonal inverse and
    solution per problem, the batched assembly workspace and the batched
    solver workspace."""

    def __init__(self, meshes, orders, coeffs, device="cuda", stream=None):
        import torch
        self.meshes, self.orders, self.coeffs = list(meshes), [int(k) for k in orders], list(coeffs)
        self.n_rows, self.nnz, ws_bytes = assemble_batch_query(self.meshes, self.orders, self.coeffs)
        dev = torch.device(device)
        self.rowptr, self.colind, self.values, self.rhs, self.dinv, self.x, self.csrs = [], [], [], [], [], [], []
        for m, k, c, nr, nz in zip(self.meshes, self.orders, self.coeffs, self.n_rows, self.nnz):
            rp = torch.empty(nr + 1, dtype=torch.int64, device=dev)
            ci = torch.empty(max(nz, 1), dtype=torch.int32, device=dev)
            va = torch.empty(max(nz, 1), dtype=torch.float64, device=dev)
            rh = torch.empty(max(nr, 1), dtype=torch.float64, device=dev)
            di = torch.empty(max(nr, 1), dtype=torch.float64, device=dev)
            csr = csr_struct(nr, nz, rp, ci, va, rh, di)
            pattern(m, k, c, csr, stream)
            self.rowptr.append(rp)
            self.colind.append(ci)
            self.values.append(va)
            self.rhs.append(rh)
            self.dinv.append(di)
            self.x.append(torch.zeros(max(nr, 1), dtype=torch.float64, device=dev))
            self.csrs.append(csr)
        self.ws = torch.empty(max(ws_bytes, 8), dtype=torch.uint8, device=dev)
        self.solve_ws = torch.empty(max(pcg_batch_query(self.n_rows), 8), dtype=torch.uint8, device=dev)

    def assemble(self, stream=None):
        assemble_batch(self.meshes, self.orders, self.coeffs, self.csrs, self.ws, stream)

    def solve(self, rtol, maxit, stream=None, zero_x=True, structured=True):
        """Batched Jacobi-PCG from x = 0 (or the current x); returns (status, infos).
        structured: evaluate the pattern from the meshes (fe_pcg_solve_batch_mesh)."""
        if zero_x:
            for x in self.x:
                x.zero_()
        if structured:
            return pcg_solve_batch_mesh(self.meshes, self.orders, self.coeffs, self.csrs, self.rhs, self.x, rtol,
                                        maxit, self.solve_ws, stream)
        return pcg_solve_batch(self.csrs, self.rhs, self.x, rtol, maxit, self.solve_ws, stream)

    def device_bytes(self):
        t = [self.ws, self.solve_ws] + self.rowptr + self.colind + self.values + self.rhs + self.dinv + self.x
        return sum(v.numel() * v.element_size() for v in t)


def _result_dict(r):
    return {f: getattr(r, f) for f, _ in Result._fields_}


class Server:
    """Owning wrapper of an fe_server: budget in bytes, max_active requests in flight."""

    def __init__(self, budget, max_active=64):
        h = _P()
        _check(lib().fe_server_create(int(budget), int(max_active), _c.byref(h)), "fe_server_create")
        self.handle = h

    def submit(self, dim, n, order, coeff, rtol, maxit, vertices=None, cell_coeff=None):
        import numpy as np
        q = Request()
        q.mesh.dim = int(dim)
        n = list(n) + [1] * (3 - len(n))
        for i in range(3):
            q.mesh.n[i] = int(n[i])
        v = None if vertices is None else np.ascontiguousarray(vertices, dtype=np.float64)
        k = None if cell_coeff is None else np.ascontiguousarray(cell_coeff, dtype=np.float64)
        q.mesh.vertex_xyz = None if v is None else v.ctypes.data_as(_P)
        q.mesh.cell_coeff = None if k is None else k.ctypes.data_as(_P)
        q.order = int(order)
        q.coeff = coeff
        q.rtol = float(rtol)
        q.maxit = int(maxit)
        t = _c.c_uint64()
        _check(lib().fe_server_submit(self.handle, _c.byref(q), _c.byref(t)), "fe_server_submit")
        return t.value

    def poll(self, ticket):
        r = Result()
        st = lib().fe_server_poll(self.handle, int(ticket), _c.byref(r))
        d = _result_dict(r)
        d["error"] = lib().fe_last_error().decode() if st != FE_OK else ""
        return d

    def wait(self, ticket, timeout=600.0):
        r = Result()
        st = lib().fe_server_wait(self.handle, int(ticket), float(timeout), _c.byref(r))
        d = _result_dict(r)
        d["error"] = lib().fe_last_error().decode() if st != FE_OK else ""
        return d

    def solution(self, ticket, out):
        _check(lib().fe_server_solution(self.handle, int(ticket), _ptr(out), int(out.numel())), "fe_server_solution")

    def release(self, ticket):
        _check(lib().fe_server_release(self.handle, int(ticket)), "fe_server_release")

    def stats(self):
        s = ServerStats()
        _check(lib().fe_server_get_stats(self.handle, _c.byref(s)), "fe_server_get_stats")
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def clock(self):
        return lib().fe_server_clock(self.handle)

    def close(self):
        if self.handle:
            _check(lib().fe_server_destroy(self.handle), "fe_server_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Simplex:
    """Owning wrapper of an fe_simplex handle (P_k on a simplicial mesh) with
    the device CSR of its free-free system (torch tensors); the pattern is
    written at construction."""

    def __init__(self, dim, vertices, cells, order, coeff, cell_coeff=None, device="cuda", stream=None, family=None,
                 kappa=1.0):
        """family None: Lagrange P_order; "nedelec" / "raviart_thomas": the
        lowest-order vector element (order ignored) with mass coefficient kappa."""
        import numpy as np
        import torch
        self.dim, self.order = int(dim), int(order)
        v = np.ascontiguousarray(vertices, dtype=np.float64)
        c = np.ascontiguousarray(cells, dtype=np.int32)
        k = None if cell_coeff is None else np.ascontiguousarray(cell_coeff, dtype=np.float64)
        d = SimplexDesc()
        d.dim = self.dim
        d.nverts, d.ncells = v.shape[0], c.shape[0]
        d.vertex_xyz = v.ctypes.data_as(_P)
        d.cells = c.ctypes.data_as(_P)
        d.cell_coeff = None if k is None else k.ctypes.data_as(_P)
        h = _P()
        if family is None:
            _check(lib().fe_simplex_create(_c.byref(d), self.order, _c.byref(coeff), _c.byref(h)), "fe_simplex_create")
        else:
            _check(lib().fe_simplex_create_vector(_c.byref(d), FAMILIES[family], float(kappa), _c.byref(coeff),
                                                  _c.byref(h)), "fe_simplex_create_vector")
        self.handle = h
        self.ncells = c.shape[0]
        nr, nz, nn, nc = _c.c_int64(), _c.c_int64(), _c.c_int64(), _c.c_int64()
        _check(lib().fe_simplex_query(h, _c.byref(nr), _c.byref(nz), _c.byref(nn), _c.byref(nc)), "fe_simplex_query")
        self.n_rows, self.nnz, self.n_nodes, self.n_contrib = nr.value, nz.value, nn.value, nc.value
        if family is None:
            ncomp = self.dim if coeff.problem == FE_ELASTICITY else 1
            nnode = (order + 1) * (order + 2) // 2 if dim == 2 else (order + 1) * (order + 2) * (order + 3) // 6
            self.nloc = nnode * ncomp
        else:
            self.nloc = {"nedelec": 6 if dim == 3 else 3, "nedelec2": 20 if dim == 3 else 8,
                         "raviart_thomas2": 15 if dim == 3 else 8}.get(family, dim + 1)
        self.ntri = self.nloc * (self.nloc + 1) // 2
        dev = torch.device(device)
        self.rowptr = torch.empty(self.n_rows + 1, dtype=torch.int64, device=dev)
        self.colind = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=dev)
        self.values = torch.empty(max(self.nnz, 1), dtype=torch.float64, device=dev)
        self.rhs = torch.empty(max(self.n_rows, 1), dtype=torch.float64, device=dev)
        self.dinv = torch.empty(max(self.n_rows, 1), dtype=torch.float64, device=dev)
        self.csr = csr_struct(self.n_rows, self.nnz, self.rowptr, self.colind, self.values, self.rhs, self.dinv)
        _check(lib().fe_simplex_pattern(h, _c.byref(self.csr), _stream(stream)), "fe_simplex_pattern")

    def assemble(self, stream=None):
        _check(lib().fe_simplex_assemble(self.handle, _c.byref(self.csr), _stream(stream)), "fe_simplex_assemble")

    def cell_dofs(self, stream=None):
        import torch
        out = torch.empty((self.ncells, self.nloc), dtype=torch.int32, device="cuda")
        _check(lib().fe_simplex_cell_dofs(self.handle, _ptr(out), _stream(stream)), "fe_simplex_cell_dofs")
        return out

    def elements(self):
        """Host copies (numpy) of the last assembly's element upper triangles
        (ncells x ntri) and loads (ncells x nloc)."""
        import numpy as np
        import torch
        torch.cuda.synchronize()
        e, f = _P(), _P()
        _check(lib().fe_simplex_elements(self.handle, _c.byref(e), _c.byref(f)), "fe_simplex_elements")
        E = np.empty((self.ncells, self.ntri))
        F = np.empty((self.ncells, self.nloc))
        if self.ncells:
            _copy_to_host(E, e.value)
            _copy_to_host(F, f.value)
        return E, F

    def close(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            lib().fe_simplex_destroy(h)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
