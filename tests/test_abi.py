"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/fe.h declares, and rejects invalid arguments before
touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1708_01773_amd import fe as F
from fe_inputs import structured_vertices

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "fe.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fe_[a-z_0-9]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert header_functions() == sorted(F.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(F.LIB_PATH)
    for name in header_functions():
        assert hasattr(L, name), name
    assert F.lib().fe_version() >= 1


def test_struct_sizes_match_header_layout():
    # int32 dim, int32 n[3], two pointers
    assert ctypes.sizeof(F.MeshDesc) == 32
    assert ctypes.sizeof(F.Csr) == 56
    assert ctypes.sizeof(F.SolveInfo) == 40
    assert ctypes.sizeof(F.K3Plan) == 16 and ctypes.sizeof(F.SpmvPlan) == 16
    assert F.Coeff.dirichlet_affine.offset + 96 == ctypes.sizeof(F.Coeff)


def test_invalid_mesh_arguments_rejected_on_host():
    d = F.MeshDesc()
    d.dim = 4
    h = ctypes.c_void_p()
    assert F.lib().fe_create_mesh(ctypes.byref(d), ctypes.byref(h)) == F.FE_EINVAL
    assert "dim" in F.lib().fe_last_error().decode()
    d.dim = 3
    d.n[0], d.n[1], d.n[2] = 2, 0, 2
    assert F.lib().fe_create_mesh(ctypes.byref(d), ctypes.byref(h)) == F.FE_EINVAL
    with pytest.raises(F.FeError):
        F.create_mesh(3, [2, 2, 2], coeff=np.array([1.0] * 7 + [np.nan]))


def test_inverted_cell_rejected_on_host():
    v = structured_vertices(3, 2)
    # move the centre vertex far beyond its neighbours so a corner Jacobian flips
    centre = 1 + 3 * (1 + 3 * 1)
    v[centre] = [1.2, 1.2, 1.2]
    with pytest.raises(F.FeError) as e:
        F.create_mesh(3, [2, 2, 2], v)
    assert e.value.status == F.FE_EMESH


def test_null_and_bad_arguments_rejected():
    L = F.lib()
    c = F.make_coeff()
    n_rows, nnz, ws = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t()
    assert L.fe_assemble_query(None, 1, ctypes.byref(c), ctypes.byref(n_rows), ctypes.byref(nnz),
                               ctypes.byref(ws)) == F.FE_EINVAL
    assert L.fe_pcg_query(-1, ctypes.byref(ws)) == F.FE_EINVAL
    assert L.fe_pcg_query(1000, ctypes.byref(ws)) == F.FE_OK and ws.value > 3 * 8000
    assert L.fe_pcg_solve(None, None, None, 1e-8, 10, None, 0, None, None) == F.FE_EINVAL
    assert L.fe_spmv(None, None, None, None) == F.FE_EINVAL


def test_batch_and_tuning_entry_points_validate_on_host():
    L = F.lib()
    ws = ctypes.c_size_t()
    assert ctypes.sizeof(F.SpmvPlan) == 16
    assert L.fe_pcg_batch_query(-1, None, ctypes.byref(ws)) == F.FE_EINVAL
    rows = (ctypes.c_int64 * 2)(1000, -5)
    assert L.fe_pcg_batch_query(2, rows, ctypes.byref(ws)) == F.FE_EINVAL
    rows[1] = 10
    assert L.fe_pcg_batch_query(2, rows, ctypes.byref(ws)) == F.FE_OK
    one = ctypes.c_size_t()
    assert L.fe_pcg_query(1000, ctypes.byref(one)) == F.FE_OK
    assert ws.value > one.value  # two systems need more than one
    assert L.fe_pcg_solve_batch(0, None, None, None, 1e-8, 10, None, 0, None, None) == F.FE_OK
    assert L.fe_pcg_solve_batch(-1, None, None, None, 1e-8, 10, None, 0, None, None) == F.FE_EINVAL
    assert L.fe_assemble_batch_query(-1, None, None, None, None, None, ctypes.byref(ws)) == F.FE_EINVAL
    assert L.fe_assemble_batch_query(0, None, None, None, None, None, ctypes.byref(ws)) == F.FE_OK
    assert L.fe_assemble_batch_query(2, None, None, None, None, None, ctypes.byref(ws)) == F.FE_EINVAL
    assert L.fe_spmv_autotune(None, 5, None, 0, None, 0, None, None, None) == F.FE_EINVAL
    assert L.fe_spmv_autotune_query(-1, ctypes.byref(ws)) == F.FE_EINVAL
    # untuned plans follow the row length: block tiles of as many rows (a power
    # of two) as hold at most 6144 entries, 4 rows at least
    assert L.fe_spmv_tuning_reset() == F.FE_OK
    mode, rpw, cls = F.spmv_plan_of(1000, 27000)
    assert mode == 9 and rpw * 27 <= 6144 and rpw * 2 * 27 > 6144
    mode, rpw, cls2 = F.spmv_plan_of(1000, 343000)
    assert mode == 9 and rpw == 16 and cls2 > cls


def test_symmetric_storage_entry_points_validate_on_host():
    L = F.lib()
    c = F.make_coeff()
    nb = ctypes.c_size_t(123)
    assert L.fe_sym_query(None, 1, ctypes.byref(c), None) == F.FE_EINVAL
    assert L.fe_sym_query(None, 1, ctypes.byref(c), ctypes.byref(nb)) == F.FE_EINVAL and nb.value == 0
    assert L.fe_sym_from_csr(None, 1, ctypes.byref(c), None, None, 0, None) == F.FE_EINVAL
    assert L.fe_sym_fp32_from_csr(None, 1, ctypes.byref(c), None, None, 0, None) == F.FE_EINVAL
    assert L.fe_spmv_sym(None, 1, ctypes.byref(c), None, 0, None, None, None) == F.FE_EINVAL
    assert L.fe_pcg_solve_sym(None, 1, ctypes.byref(c), None, None, 0, None, None, 1e-8, 10, None, 0, None,
                              None) == F.FE_EINVAL
    assert L.fe_refine_solve_sym(None, 1, ctypes.byref(c), None, None, None, 0, None, None, 1e-10, 1e-5, 5, 100,
                                 None, 0, None, None) == F.FE_EINVAL


def test_csr_plans_can_be_pinned_per_row_class_on_host():
    # the CSR plans the autotuner times: stream runs of 1..32 rows per wave,
    # and one wave per row; each can be made the plan of a row-length class
    plans = [(0, 1), (0, 2), (0, 4), (0, 8), (0, 16), (0, 32), (1, 1), (9, 4), (9, 8), (9, 16), (9, 32), (9, 64),
             (9, 128), (9, 256)]
    try:
        for mode, rpw in plans:
            F.spmv_plan_set(1000, 250000, mode, rpw)
            assert F.spmv_plan_of(1000, 250000)[:2] == (mode, rpw)
            assert F.spmv_plan_of(1000, 251000)[:2] == (mode, rpw)  # same half-octave class
        for mode, rpw in [(0, 3), (0, 64), (1, 2), (2, 8), (9, 2), (9, 512), (10, 64), (11, 1)]:
            with pytest.raises(F.FeError, match="not a CSR plan"):
                F.spmv_plan_set(1000, 250000, mode, rpw)
    finally:
        F.spmv_tuning_reset()
    # the heuristic again: block tiles of the most rows (a power of two, 4..256) with at most 6144 entries
    assert F.spmv_plan_of(1000, 250000)[:2] == (9, 16)
    assert F.spmv_plan_of(2048383, 54439939)[:2] == (9, 128)
    assert F.spmv_plan_of(2572125, 1572091911)[:2] == (9, 8)
    assert F.spmv_plan_of(1000, 3000)[:2] == (9, 256)


def test_dg_entry_points_validate_on_host():
    L = F.lib()
    nr, nz, ws = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t()
    assert L.fe_dg_query(None, 2, ctypes.byref(nr), ctypes.byref(nz), ctypes.byref(ws)) == F.FE_EINVAL
    assert "mesh" in L.fe_last_error().decode()
    assert L.fe_dg_pattern(None, 2, None, None) == F.FE_EINVAL
    c = F.make_coeff()
    assert L.fe_dg_assemble(None, 2, ctypes.byref(c), 36.0, 1.0, None, None, 0, None) == F.FE_EINVAL


def _simplex_create(dim, verts, cells, order=2, problem="poisson", precision="fp64"):
    L = F.lib()
    v = np.ascontiguousarray(verts, dtype=np.float64)
    c = np.ascontiguousarray(cells, dtype=np.int32)
    d = F.SimplexDesc()
    d.dim, d.nverts, d.ncells = dim, v.shape[0], c.shape[0]
    d.vertex_xyz = v.ctypes.data_as(ctypes.c_void_p)
    d.cells = c.ctypes.data_as(ctypes.c_void_p)
    d.cell_coeff = None
    h = ctypes.c_void_p()
    coeff = F.make_coeff(problem, precision, dim=dim)
    st = L.fe_simplex_create(ctypes.byref(d), order, ctypes.byref(coeff), ctypes.byref(h))
    return st, L.fe_last_error().decode()


def test_simplex_entry_points_validate_on_host():
    """Argument and mesh checks of fe_simplex_create run before any device
    call: bad dimension or order, reduced precision, vertex ids out of range,
    degenerate cells, a facet shared by three cells."""
    L = F.lib()
    h = ctypes.c_void_p()
    c = F.make_coeff()
    assert L.fe_simplex_create(None, 1, ctypes.byref(c), ctypes.byref(h)) == F.FE_EINVAL
    tet = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float64)
    assert _simplex_create(4, tet, [[0, 1, 2, 3]])[0] == F.FE_EINVAL
    assert _simplex_create(3, tet, [[0, 1, 2, 3]], order=5)[0] == F.FE_EINVAL
    assert _simplex_create(3, tet, [[0, 1, 2, 3]], order=4, problem="elasticity")[0] == F.FE_EINVAL
    assert _simplex_create(3, tet, [[0, 1, 2, 3]], precision="fp32")[0] == F.FE_EINVAL
    st, msg = _simplex_create(3, tet, [[0, 1, 2, 4]])
    assert st == F.FE_EMESH and "range" in msg
    flat = tet.copy()
    flat[3] = [0.5, 0.5, 0.0]  # coplanar with the first three
    st, msg = _simplex_create(3, flat, [[0, 1, 2, 3]])
    assert st == F.FE_EMESH and "degenerate" in msg
    tri = np.array([[0, 0], [1, 0], [0, 1], [1, 1], [-1, -1]], dtype=np.float64)
    st, msg = _simplex_create(2, tri, [[0, 1, 2], [1, 2, 3], [2, 1, 4]])
    assert st == F.FE_EMESH and "more than two" in msg
    for name in ("fe_simplex_destroy",):
        assert getattr(L, name)(None) == F.FE_EINVAL
    assert L.fe_simplex_query(None, None, None, None, None) == F.FE_EINVAL
    assert L.fe_simplex_pattern(None, None, None) == F.FE_EINVAL
    assert L.fe_simplex_assemble(None, None, None) == F.FE_EINVAL
