"""Oracle: plain FP64 CPU reference of the finite element pipeline.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the HIP library (``paper_1708_01773_amd``) and never imports it.

The numerical work lives in ``fe_oracle.c`` (single-threaded, FP64, written
from the definitions in arXiv 1708.01773: Sect. 3.4 Lagrange bases, Sect. 3.6
cell-wise assembly, Sect. 3.7 numerical integration, Sect. 10.4 strong
Dirichlet elimination, Sect. 11.1 COO compression).  This module marshals
numpy arrays to it through ctypes and adds two pure-Python pieces:

* :func:`coo_compress` -- the paper's build-up in COO form followed by the
  "compression" that sums duplicate entries and converts to CSR (Sect. 11.1),
  used as a self-check of the symbolic/numeric CSR path on small inputs;
* :func:`lanczos_extremes` -- extremal eigenvalue estimates of the
  preconditioned operator from the CG coefficients (the Lanczos tridiagonal
  built from CG's alpha/beta, Saad Sect. 6.7.3).
"""
import ctypes
import os
import time

import numpy as np

from . import build as _build

_lib = None

_d = ctypes.c_double
_i = ctypes.c_int
_i64 = ctypes.c_int64
_P = ctypes.c_void_p


class OrcProblem(ctypes.Structure):
    _fields_ = [
        ("dim", _i),
        ("n", _i * 3),
        ("k", _i),
        ("problem", _i),
        ("lam", _d),
        ("mu", _d),
        ("source_kind", _i),
        ("source", _d * 3),
        ("dirichlet_kind", _i),
        ("dirichlet_affine", _d * 12),
    ]


class OrcSxProblem(ctypes.Structure):
    _fields_ = [
        ("dim", _i),
        ("k", _i),
        ("problem", _i),
        ("lam", _d),
        ("mu", _d),
        ("source_kind", _i),
        ("source", _d * 3),
        ("dirichlet_kind", _i),
        ("dirichlet_affine", _d * 12),
    ]


def lib():
    """Load (building on first use) the oracle shared library."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.orc_gauss_legendre.argtypes = [_i, _P, _P]
        L.orc_gauss_legendre.restype = _i
        L.orc_lagrange_1d.argtypes = [_i, _d, _P, _P]
        L.orc_lagrange_1d.restype = None
        L.orc_element_matrix.argtypes = [_i, _i, _i, _P, _d, _d, _d, _P]
        L.orc_element_matrix.restype = _i
        L.orc_element_load.argtypes = [_i, _i, _i, _P, _i, _P, _P]
        L.orc_element_load.restype = _i
        L.orc_cell_vertices.argtypes = [_i, _P, _P, _i64, _P]
        L.orc_cell_vertices.restype = None
        L.orc_number_nodes.argtypes = [_i, _P, _i, ctypes.c_uint, _P, _P, _P]
        L.orc_number_nodes.restype = None
        L.orc_cell_dofs.argtypes = [_i, _P, _i, _i, _P, _i64, _P]
        L.orc_cell_dofs.restype = None
        L.orc_csr_pattern.argtypes = [_i64, _i, _P, _i64, _P, ctypes.POINTER(ctypes.POINTER(ctypes.c_int32))]
        L.orc_csr_pattern.restype = _i64
        L.orc_free.argtypes = [_P]
        L.orc_free.restype = None
        L.orc_assemble.argtypes = [ctypes.POINTER(OrcProblem), _P, _P, _P, _i64, _P, _P, _P, _P]
        L.orc_assemble.restype = _i
        L.orc_assemble_row.argtypes = [ctypes.POINTER(OrcProblem), _P, _P, _P, _i64, _i64, _P, _P, _P]
        L.orc_assemble_row.restype = _i64
        L.orc_spmv.argtypes = [_i64, _P, _P, _P, _P, _P]
        L.orc_spmv.restype = None
        L.orc_pcg.argtypes = [_i64, _P, _P, _P, _P, _P, _d, _i, _P, _P, _P, _P]
        L.orc_pcg.restype = _i
        L.orc_l2_error.argtypes = [ctypes.POINTER(OrcProblem), _P, _P, _P, _i, _i, _P]
        L.orc_l2_error.restype = _d
        L.orc_fixed_values.argtypes = [ctypes.POINTER(OrcProblem), _P, _P, _i64, _P]
        L.orc_fixed_values.restype = None
        L.orc_dg_pattern.argtypes = [ctypes.POINTER(OrcProblem), _P, ctypes.POINTER(ctypes.POINTER(ctypes.c_int32))]
        L.orc_dg_pattern.restype = _i64
        L.orc_dg_assemble.argtypes = [ctypes.POINTER(OrcProblem), _P, _d, _d, _P, _P, _P, _P]
        L.orc_dg_assemble.restype = _i
        L.orc_stokes_b_element.argtypes = [_i, _i, _P, _P, _P]
        L.orc_stokes_b_element.restype = _i
        L.orc_sx_nodes.argtypes = [_i, _i, _P]
        L.orc_sx_nodes.restype = _i
        L.orc_sx_basis.argtypes = [_i, _i, _P]
        L.orc_sx_basis.restype = _i
        L.orc_sx_shape.argtypes = [_i, _i, _P, _P, _P]
        L.orc_sx_shape.restype = _i
        L.orc_sx_quadrature.argtypes = [_i, _i, _P, _P]
        L.orc_sx_quadrature.restype = _i
        L.orc_sx_element_matrix.argtypes = [_i, _i, _i, _P, _d, _d, _d, _P]
        L.orc_sx_element_matrix.restype = _i
        L.orc_sx_element_load.argtypes = [_i, _i, _i, _P, _i, _P, _P]
        L.orc_sx_element_load.restype = _i
        L.orc_sx_number.argtypes = [_i, _i, _i64, _i64, _P, _i, _P, _P, _P, _P, _P]
        L.orc_sx_number.restype = _i
        L.orc_sx_cell_dofs.argtypes = [_i, _i, _i, _i64, _P, _P, _P]
        L.orc_sx_cell_dofs.restype = None
        L.orc_sx_node_positions.argtypes = [_i, _i, _i64, _P, _P, _P, _P]
        L.orc_sx_node_positions.restype = None
        L.orc_sx_assemble.argtypes = [ctypes.POINTER(OrcSxProblem), _P, _i64, _P, _P, _P, _i64, _P, _P, _P, _P]
        L.orc_sx_assemble.restype = _i
        L.orc_sx_l2_error.argtypes = [ctypes.POINTER(OrcSxProblem), _P, _i64, _P, _P, _P, _i, _i, _P]
        L.orc_sx_l2_error.restype = _d
        L.orc_vx_basis.argtypes = [_i, _i, _P]
        L.orc_vx_basis.restype = _i
        L.orc_vx_shape.argtypes = [_i, _i, _P, _P, _P, _P]
        L.orc_vx_shape.restype = _i
        L.orc_vx_element.argtypes = [_i, _i, _P, _P, _d, _d, _i, _P, _P, _P]
        L.orc_vx_element.restype = _i
        L.orc_vx_number.argtypes = [_i, _i, _i64, _i64, _P, _i, _P, _P, _P, _P, _P]
        L.orc_vx_number.restype = _i
        L.orc_vx_assemble.argtypes = [_i, _i, _P, _i64, _P, _P, _d, _i, _P, _P, _i64, _P, _P, _P, _P]
        L.orc_vx_assemble.restype = _i
        L.orc_vx_l2_error.argtypes = [_i, _i, _P, _i64, _P, _P, _P, _d, _i]
        L.orc_vx_l2_error.restype = _d
        _lib = L
    return _lib


_omp = None


def omp_lib():
    """The all-cores (OpenMP) build of the oracle: the CPU baseline only."""
    global _omp
    if _omp is None:
        if not os.path.exists(_build.LIB_OMP):
            _build.build()
        L = ctypes.CDLL(_build.LIB_OMP)
        L.orc_omp_threads.argtypes = []
        L.orc_omp_threads.restype = _i
        L.orc_omp_csr_pattern.argtypes = [_i64, _i, _P, _i64, _P, ctypes.POINTER(ctypes.POINTER(ctypes.c_int32))]
        L.orc_omp_csr_pattern.restype = _i64
        L.orc_omp_assemble.argtypes = [ctypes.POINTER(OrcProblem), _P, _P, _P, _i64, _P, _P, _P, _P]
        L.orc_omp_assemble.restype = _i
        L.orc_omp_pcg.argtypes = [_i64, _P, _P, _P, _P, _P, _d, _i, _P, _P]
        L.orc_omp_pcg.restype = _i
        L.orc_free.argtypes = [_P]
        L.orc_free.restype = None
        _omp = L
    return _omp


def omp_threads():
    return omp_lib().orc_omp_threads()


def omp_csr_pattern(cdofs, nfree):
    cdofs = _c(cdofs, np.int64)
    rowptr = np.zeros(nfree + 1, dtype=np.int64)
    cptr = ctypes.POINTER(ctypes.c_int32)()
    L = omp_lib()
    nnz = L.orc_omp_csr_pattern(cdofs.shape[0], cdofs.shape[1], _ptr(cdofs), nfree, _ptr(rowptr), ctypes.byref(cptr))
    colind = np.ctypeslib.as_array(cptr, shape=(max(nnz, 1),))[:nnz].copy()
    L.orc_free(ctypes.cast(cptr, _P))
    return rowptr, colind


def omp_assemble(P, vxyz, coef, cdofs, nfree, rowptr, colind):
    s = P.c_struct()
    values = np.zeros(int(rowptr[-1]))
    rhs = np.zeros(nfree)
    coef = None if coef is None else _c(coef, np.float64)
    rc = omp_lib().orc_omp_assemble(ctypes.byref(s), _ptr(_c(vxyz, np.float64)), _ptr(coef),
                                    _ptr(_c(cdofs, np.int64)), nfree, _ptr(_c(rowptr, np.int64)),
                                    _ptr(_c(colind, np.int32)), _ptr(values), _ptr(rhs))
    return values, rhs, rc == 0


def omp_pcg(rowptr, colind, values, b, rtol, maxit):
    n = len(rowptr) - 1
    x = np.zeros(n)
    it = _i()
    rr = _d()
    st = omp_lib().orc_omp_pcg(n, _ptr(_c(rowptr, np.int64)), _ptr(_c(colind, np.int32)),
                               _ptr(_c(values, np.float64)), _ptr(_c(b, np.float64)), _ptr(x), float(rtol),
                               int(maxit), ctypes.byref(it), ctypes.byref(rr))
    return dict(x=x, status=st, iters=it.value, relres=rr.value)


def _ptr(a):
    return a.ctypes.data_as(_P) if a is not None else None


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def lame(young, nu):
    """Lame parameters of isotropic elasticity from Young's modulus and Poisson's ratio."""
    lam = young * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = young / (2.0 * (1.0 + nu))
    return lam, mu


class Problem:
    """Description of one assembly problem (all fields are plain numbers).

    problem: 'poisson' or 'elasticity'; faces: Dirichlet face bitmask
    (bit 2r: x_r = 0, bit 2r+1: x_r = 1); source_kind 0 none, 1 constant
    vector, 2 manufactured sin-product load; dirichlet_kind 0 zero, 1 affine
    (u_D,c = aff[4c] + sum_r aff[4c+1+r] x_r).
    """

    def __init__(self, dim, n, k, problem="poisson", young=1.0, nu=0.3,
                 source_kind=0, source=(0.0, 0.0, 0.0), faces=None,
                 dirichlet_kind=0, dirichlet_affine=None):
        self.dim = int(dim)
        n = [int(v) for v in (n if hasattr(n, "__len__") else [n] * dim)]
        self.n = n + [1] * (3 - len(n))
        if self.dim == 2:
            self.n[2] = 1
        self.k = int(k)
        self.problem = problem
        self.young, self.nu = float(young), float(nu)
        self.source_kind = int(source_kind)
        self.source = [float(s) for s in source] + [0.0] * (3 - len(source))
        self.faces = (1 << (2 * dim)) - 1 if faces is None else int(faces)
        self.dirichlet_kind = int(dirichlet_kind)
        aff = list(dirichlet_affine) if dirichlet_affine is not None else []
        self.dirichlet_affine = [float(v) for v in aff] + [0.0] * (12 - len(aff))

    @property
    def ncomp(self):
        return self.dim if self.problem == "elasticity" else 1

    @property
    def ncells(self):
        return self.n[0] * self.n[1] * (self.n[2] if self.dim == 3 else 1)

    @property
    def nn(self):
        return (self.k + 1) ** self.dim

    @property
    def nloc(self):
        return self.nn * self.ncomp

    def c_struct(self):
        s = OrcProblem()
        s.dim = self.dim
        for r in range(3):
            s.n[r] = self.n[r]
        s.k = self.k
        s.problem = 1 if self.problem == "elasticity" else 0
        s.lam, s.mu = lame(self.young, self.nu) if self.problem == "elasticity" else (0.0, 0.0)
        s.source_kind = self.source_kind
        for r in range(3):
            s.source[r] = self.source[r]
        s.dirichlet_kind = self.dirichlet_kind
        for r in range(12):
            s.dirichlet_affine[r] = self.dirichlet_affine[r]
        return s


def gauss_legendre(n):
    x = np.zeros(n)
    w = np.zeros(n)
    if lib().orc_gauss_legendre(n, _ptr(x), _ptr(w)) != 0:
        raise ValueError("unsupported number of Gauss points")
    return x, w


def lagrange_1d(k, x):
    v = np.zeros(k + 1)
    d = np.zeros(k + 1)
    lib().orc_lagrange_1d(k, float(x), _ptr(v), _ptr(d))
    return v, d


def element_matrix(dim, k, X, coef=1.0, problem="poisson", young=1.0, nu=0.3):
    """Element matrix of one cell with vertex coordinates X (2^d x d).

    Returns (A, ok); ok is False if det J <= 0 at a quadrature point."""
    X = _c(X, np.float64).reshape(-1)
    ncomp = dim if problem == "elasticity" else 1
    nloc = (k + 1) ** dim * ncomp
    A = np.zeros((nloc, nloc))
    lam, mu = lame(young, nu) if problem == "elasticity" else (0.0, 0.0)
    rc = lib().orc_element_matrix(dim, k, 1 if problem == "elasticity" else 0, _ptr(X),
                                  float(coef), lam, mu, _ptr(A))
    if rc == -2:
        raise ValueError("unsupported dim/order")
    return A, rc == 0


def element_load(dim, k, ncomp, X, source_kind, source):
    X = _c(X, np.float64).reshape(-1)
    src = _c(list(source) + [0.0] * (3 - len(source)), np.float64)
    f = np.zeros((k + 1) ** dim * ncomp)
    lib().orc_element_load(dim, k, ncomp, _ptr(X), int(source_kind), _ptr(src), _ptr(f))
    return f


def cell_vertices(dim, n, vxyz, cell):
    nn = _c(list(n) + [1] * (3 - len(n)), np.int32)
    v = _c(vxyz, np.float64)
    X = np.zeros((1 << dim, dim))
    lib().orc_cell_vertices(dim, _ptr(nn), _ptr(v), int(cell), _ptr(X))
    return X


def number_nodes(dim, n, k, faces):
    nn = _c(list(n) + [1] * (3 - len(n)), np.int32)
    nnodes = 1
    for r in range(dim):
        nnodes *= n[r] * k + 1
    code = np.zeros(nnodes, dtype=np.int64)
    nf = _i64()
    nx = _i64()
    lib().orc_number_nodes(dim, _ptr(nn), k, faces, _ptr(code), ctypes.byref(nf), ctypes.byref(nx))
    return code, nf.value, nx.value


def cell_dofs(P: Problem, node_code):
    nn = _c(P.n, np.int32)
    out = np.zeros((P.ncells, P.nloc), dtype=np.int64)
    lib().orc_cell_dofs(P.dim, _ptr(nn), P.k, P.ncomp, _ptr(_c(node_code, np.int64)), P.ncells, _ptr(out))
    return out


def csr_pattern(cdofs, nfree):
    cdofs = _c(cdofs, np.int64)
    rowptr = np.zeros(nfree + 1, dtype=np.int64)
    cptr = ctypes.POINTER(ctypes.c_int32)()
    nnz = lib().orc_csr_pattern(cdofs.shape[0], cdofs.shape[1], _ptr(cdofs), nfree, _ptr(rowptr),
                                ctypes.byref(cptr))
    colind = np.ctypeslib.as_array(cptr, shape=(max(nnz, 1),))[:nnz].copy()
    lib().orc_free(ctypes.cast(cptr, _P))
    return rowptr, colind


def assemble(P: Problem, vxyz, coef, cdofs, nfree, rowptr, colind):
    """Numeric assembly; returns (values, rhs, ok)."""
    s = P.c_struct()
    vxyz = _c(vxyz, np.float64)
    coef = None if coef is None else _c(coef, np.float64)
    cdofs = _c(cdofs, np.int64)
    values = np.zeros(int(rowptr[-1]))
    rhs = np.zeros(nfree)
    rc = lib().orc_assemble(ctypes.byref(s), _ptr(vxyz), _ptr(coef), _ptr(cdofs), nfree,
                            _ptr(_c(rowptr, np.int64)), _ptr(_c(colind, np.int32)), _ptr(values), _ptr(rhs))
    return values, rhs, rc == 0


def assemble_row(P: Problem, vxyz, coef, cdofs, row, maxlen=4096):
    """One row (columns, values, rhs entry) of the assembled free-free system."""
    s = P.c_struct()
    cols = np.zeros(maxlen, dtype=np.int64)
    vals = np.zeros(maxlen)
    rhs = _d()
    coef = None if coef is None else _c(coef, np.float64)
    ln = lib().orc_assemble_row(ctypes.byref(s), _ptr(_c(vxyz, np.float64)), _ptr(coef),
                                _ptr(_c(cdofs, np.int64)), int(row), maxlen, _ptr(cols), _ptr(vals),
                                ctypes.byref(rhs))
    if ln < 0:
        raise ValueError("row longer than maxlen")
    return cols[:ln].copy(), vals[:ln].copy(), rhs.value


def spmv(rowptr, colind, values, x):
    n = len(rowptr) - 1
    y = np.zeros(n)
    lib().orc_spmv(n, _ptr(_c(rowptr, np.int64)), _ptr(_c(colind, np.int32)), _ptr(_c(values, np.float64)),
                   _ptr(_c(x, np.float64)), _ptr(y))
    return y


def pcg(rowptr, colind, values, b, rtol, maxit, x0=None):
    """Jacobi PCG.  Returns dict(x, status, iters, relres, alphas, betas)."""
    n = len(rowptr) - 1
    x = np.zeros(n) if x0 is None else _c(x0, np.float64).copy()
    al = np.zeros(max(maxit, 1))
    be = np.zeros(max(maxit, 1))
    it = _i()
    rr = _d()
    st = lib().orc_pcg(n, _ptr(_c(rowptr, np.int64)), _ptr(_c(colind, np.int32)), _ptr(_c(values, np.float64)),
                       _ptr(_c(b, np.float64)), _ptr(x), float(rtol), int(maxit), ctypes.byref(it),
                       ctypes.byref(rr), _ptr(al), _ptr(be))
    return dict(x=x, status=st, iters=it.value, relres=rr.value, alphas=al[:it.value].copy(),
                betas=be[:it.value].copy())


def l2_error(P: Problem, vxyz, cdofs, xfree, kq, exact_kind, exact):
    s = P.c_struct()
    ex = _c(list(exact) + [0.0] * (12 - len(exact)), np.float64)
    return lib().orc_l2_error(ctypes.byref(s), _ptr(_c(vxyz, np.float64)), _ptr(_c(cdofs, np.int64)),
                              _ptr(_c(xfree, np.float64)), int(kq), int(exact_kind), _ptr(ex))


def fixed_values(P: Problem, vxyz, cdofs, nfixed_dofs):
    s = P.c_struct()
    out = np.zeros(max(nfixed_dofs, 1))
    lib().orc_fixed_values(ctypes.byref(s), _ptr(_c(vxyz, np.float64)), _ptr(_c(cdofs, np.int64)),
                           int(nfixed_dofs), _ptr(out))
    return out[:nfixed_dofs]


class System:
    """The whole assembled free-free system of a problem on a given mesh."""

    def __init__(self, P: Problem, vxyz, coef=None):
        self.P = P
        self.vxyz = _c(vxyz, np.float64)
        self.coef = None if coef is None else _c(coef, np.float64)
        self.node_code, nfree_nodes, nfixed_nodes = number_nodes(P.dim, P.n, P.k, P.faces)
        self.nfree = nfree_nodes * P.ncomp
        self.nfixed = nfixed_nodes * P.ncomp
        self.cell_dofs = cell_dofs(P, self.node_code)
        self.rowptr, self.colind = csr_pattern(self.cell_dofs, self.nfree)
        self.values, self.rhs, self.ok = assemble(P, self.vxyz, self.coef, self.cell_dofs, self.nfree,
                                                  self.rowptr, self.colind)

    @property
    def nnz(self):
        return int(self.rowptr[-1])

    def dense(self):
        A = np.zeros((self.nfree, self.nfree))
        for i in range(self.nfree):
            for j in range(self.rowptr[i], self.rowptr[i + 1]):
                A[i, self.colind[j]] = self.values[j]
        return A

    def scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.values, self.colind, self.rowptr), shape=(self.nfree, self.nfree))


def _cell_vefs(dim, k):
    """The vefs (vertices, edges, faces, the cell itself) of a Q_k cell and the
    local nodes each one owns (the nodes in its relative interior).

    A vef is given per axis by a side: 0 or 1 (the vef lies on that side of
    the cell) or None (the vef spans the axis).  Local vef order: by
    dimension (vertices first), then by the set of spanned axes in binary
    order, then by the sides in the vertex order v0 + 2 v1 + 4 v2 of the paper's
    hexahedron (Sect. 3.14).  Within a vef, nodes keep their local
    lexicographic order.  Returns a list of (sides, local node list)."""
    vefs = []
    for vdim in range(dim + 1):
        for mask in range(1 << dim):
            if bin(mask).count("1") != vdim:
                continue
            fixed_axes = [r for r in range(dim) if not (mask >> r) & 1]
            for code in range(1 << len(fixed_axes)):
                sides = [None] * dim
                for t, r in enumerate(fixed_axes):
                    sides[r] = (code >> t) & 1
                nodes = []
                for a in range((k + 1) ** dim):
                    ar = [(a // (k + 1) ** r) % (k + 1) for r in range(dim)]
                    on = True
                    for r in range(dim):
                        if sides[r] is None:
                            on = on and 0 < ar[r] < k
                        else:
                            on = on and ar[r] == sides[r] * k
                    if on:
                        nodes.append(a)
                vefs.append((tuple(sides), nodes))
    return vefs


def owner_cell_numbering(P: Problem):
    """Cell-to-DOF map in the paper's owner-cell numbering (Sect. 10.3).

    One sweep over the cells in the iterator's order (lexicographic): a cell
    first numbers the DOFs in its own interior, then visits its vefs; the
    first cell that reaches a vef owning at least one DOF becomes its owner
    and numbers the DOFs on it from the next free identifier, and every later
    cell fetches the identifiers of that vef from its owner.  Free and fixed
    DOFs are numbered separately (Sect. 10.4): free ones 0, 1, ..., fixed ones
    -1, -2, ... (a DOF is fixed if its node lies on a Dirichlet face).  Vector
    fields number the components of a node consecutively.

    On the structured brick the vefs of neighbouring cells are aligned, so the
    fetch from the owner maps a node of the vef to the same lattice node; it is
    done here through a table from lattice node to the identifier its owner
    gave it.  Pure Python: small meshes only.  Returns (cell_dofs, nfree,
    nfixed) with cell_dofs[cell, ncomp*a + c]."""
    dim, k, nc = P.dim, P.k, P.ncomp
    n = P.n[:dim]
    N = [n[r] * k + 1 for r in range(dim)]
    vefs = _cell_vefs(dim, k)
    # the cell interior (its last vef) is numbered first, then the others
    order = [vefs[-1]] + vefs[:-1]
    out = np.zeros((P.ncells, P.nloc), dtype=np.int64)
    owner_ids = {}  # lattice node -> list of ncomp identifiers from its owner
    visited = set()  # global vefs that already have an owner
    nfree = nfixed = 0
    for cell in range(P.ncells):
        ci = [(cell // int(np.prod(n[:r]))) % n[r] for r in range(dim)]
        for sides, nodes in order:
            if not nodes:
                continue  # a vef with no DOF gets no owner
            gvef = (tuple(ci[r] if sides[r] is None else ci[r] + sides[r] for r in range(dim)),
                    tuple(s is None for s in sides))
            first = gvef not in visited
            visited.add(gvef)
            for a in nodes:
                ar = [(a // (k + 1) ** r) % (k + 1) for r in range(dim)]
                I = tuple(ci[r] * k + ar[r] for r in range(dim))
                if first:
                    fixed = any((I[r] == 0 and (P.faces >> (2 * r)) & 1) or
                                (I[r] == N[r] - 1 and (P.faces >> (2 * r + 1)) & 1) for r in range(dim))
                    ids = []
                    for c in range(nc):
                        if fixed:
                            ids.append(-1 - nfixed)
                            nfixed += 1
                        else:
                            ids.append(nfree)
                            nfree += 1
                    owner_ids[I] = ids
                for c in range(nc):
                    out[cell, nc * a + c] = owner_ids[I][c]
    return out, nfree, nfixed


class DGSystem:
    """The interior-penalty DG system of -Laplace(u) = f (Sect. 3.12) on a
    mesh: DOF K nn + a, every facet integrated, Dirichlet data weak.  gamma is
    the penalty parameter, tau = 1 the symmetric method.  The problem's
    source and Dirichlet datum (kinds as in Problem) are used; its faces are
    ignored (every boundary facet carries the datum)."""

    def __init__(self, P: Problem, vxyz, gamma, tau=1.0):
        assert P.problem == "poisson"
        self.P, self.gamma, self.tau = P, float(gamma), float(tau)
        self.vxyz = _c(vxyz, np.float64)
        self.nfree = P.ncells * P.nn
        s = P.c_struct()
        self.rowptr = np.zeros(self.nfree + 1, dtype=np.int64)
        cptr = ctypes.POINTER(ctypes.c_int32)()
        nnz = lib().orc_dg_pattern(ctypes.byref(s), _ptr(self.rowptr), ctypes.byref(cptr))
        self.colind = np.ctypeslib.as_array(cptr, shape=(max(nnz, 1),))[:nnz].copy()
        lib().orc_free(ctypes.cast(cptr, _P))
        self.values = np.zeros(nnz)
        self.rhs = np.zeros(self.nfree)
        rc = lib().orc_dg_assemble(ctypes.byref(s), _ptr(self.vxyz), self.gamma, self.tau, _ptr(self.rowptr),
                                   _ptr(self.colind), _ptr(self.values), _ptr(self.rhs))
        self.ok = rc == 0
        self.cell_dofs = np.arange(self.nfree, dtype=np.int64).reshape(P.ncells, P.nn)

    @property
    def nnz(self):
        return int(self.rowptr[-1])

    def dense(self):
        A = np.zeros((self.nfree, self.nfree))
        for i in range(self.nfree):
            A[i, self.colind[self.rowptr[i]:self.rowptr[i + 1]]] = self.values[self.rowptr[i]:self.rowptr[i + 1]]
        return A

    def scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.values, self.colind, self.rowptr), shape=(self.nfree, self.nfree))


def stokes_b_element(dim, k, X):
    """Divergence block (pressure order k, velocity order k+1; rows pressure
    nodes, columns local velocity DOFs dim b + c) and pressure mass diagonal
    of one cell.  Returns (B, md, ok)."""
    X = _c(X, np.float64).reshape(-1)
    nnp, nlu = (k + 1) ** dim, dim * (k + 2) ** dim
    B = np.zeros((nnp, nlu))
    md = np.zeros(nnp)
    rc = lib().orc_stokes_b_element(dim, k, _ptr(X), _ptr(B), _ptr(md))
    if rc == -2:
        raise ValueError("unsupported dim/order")
    return B, md, rc == 0


class StokesSystem:
    """Taylor-Hood Stokes on a mesh (the Stokes example of Sect. 3.1):
    velocity Q_{k+1}^d with zero Dirichlet data on the whole boundary,
    pressure Q_k with every node free, viscous term mu eps(u):eps(v) (the
    elasticity system with lambda = 0, its mu = mu / 2: Young's modulus mu,
    Poisson ratio 0), b(v, q) = -int q div v, body force from source_kind /
    source.  The system [[A, B^T], [B, 0]] [u; p] = [f; 0] is symmetric and
    indefinite; the pressure is fixed up to a constant."""

    def __init__(self, dim, n, k, vxyz, mu=1.0, source_kind=1, source=(1.0, 0.0, 0.0)):
        import scipy.sparse as sp
        self.dim, self.k, self.mu = int(dim), int(k), float(mu)
        self.vxyz = _c(vxyz, np.float64)
        self.Pu = Problem(dim, n, k + 1, problem="elasticity", young=mu, nu=0.0, source_kind=source_kind,
                          source=source)
        self.A = System(self.Pu, self.vxyz)
        self.Pp = Problem(dim, n, k, problem="poisson", faces=0)
        code, nfp, _ = number_nodes(dim, self.Pp.n, k, 0)
        self.cdp = cell_dofs(self.Pp, code)
        self.nu, self.np = self.A.nfree, nfp
        rows, cols, vals = [], [], []
        self.md = np.zeros(self.np)
        self.ok = self.A.ok
        for K in range(self.Pp.ncells):
            X = cell_vertices(dim, self.Pp.n, self.vxyz, K)
            Bk, mdk, ok = stokes_b_element(dim, k, X)
            self.ok &= ok
            gp, gu = self.cdp[K], self.A.cell_dofs[K]
            np.add.at(self.md, gp, mdk)
            free = gu >= 0
            R, C = np.meshgrid(gp, gu[free], indexing="ij")
            rows.append(R.ravel())
            cols.append(C.ravel())
            vals.append(Bk[:, free].ravel())
        self.B = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                               shape=(self.np, self.nu)).tocsr()
        self.B.sort_indices()

    def matrix(self):
        import scipy.sparse as sp
        return sp.bmat([[self.A.scipy(), self.B.T], [self.B, None]]).tocsr()

    def rhs(self):
        return np.concatenate([self.A.rhs, np.zeros(self.np)])

    def solve(self):
        """Direct solve with the pressure's DOF sum set to zero (a bordered
        system).  Returns (u, p)."""
        import scipy.sparse as sp
        import scipy.sparse.linalg as spla
        e = np.concatenate([np.zeros(self.nu), np.ones(self.np)])[:, None]
        Kb = sp.bmat([[self.matrix(), sp.csr_matrix(e)], [sp.csr_matrix(e.T), None]]).tocsc()
        x = spla.spsolve(Kb, np.concatenate([self.rhs(), [0.0]]))
        return x[:self.nu], x[self.nu:self.nu + self.np]

    def pressure_nodes(self):
        """Physical coordinates of the pressure nodes (order-1 map of each cell)."""
        k, dim = self.k, self.dim
        out = np.zeros((self.np, dim))
        for K in range(self.Pp.ncells):
            X = cell_vertices(dim, self.Pp.n, self.vxyz, K)
            for a in range(self.Pp.nn):
                xi = [((a // (k + 1) ** r) % (k + 1)) / k for r in range(dim)]
                w = np.array([np.prod([xi[r] if (v >> r) & 1 else 1 - xi[r] for r in range(dim)])
                              for v in range(1 << dim)])
                out[self.cdp[K][a]] = w @ X
        return out


def coo_compress(rows, cols, vals, n):
    """The paper's COO build-up followed by compression (Sect. 11.1): sort the
    pushed-back (row, col, value) triplets and sum duplicates, giving CSR."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    order = np.lexsort((cols, rows))
    r, c, v = rows[order], cols[order], vals[order]
    out_c, out_v, out_r = [], [], []
    for i in range(len(r)):
        if out_r and out_r[-1] == r[i] and out_c[-1] == c[i]:
            out_v[-1] += v[i]
        else:
            out_r.append(r[i])
            out_c.append(c[i])
            out_v.append(v[i])
    rowptr = np.zeros(n + 1, dtype=np.int64)
    for rr in out_r:
        rowptr[rr + 1] += 1
    rowptr = np.cumsum(rowptr)
    return rowptr, np.asarray(out_c, dtype=np.int32), np.asarray(out_v)


def lanczos_extremes(alphas, betas):
    """Extremal Ritz values of the preconditioned operator from CG
    coefficients: T has diagonal 1/a_j + b_{j-1}/a_{j-1} and off-diagonal
    sqrt(b_j)/a_j (Saad, Sect. 6.7.3)."""
    m = len(alphas)
    if m == 0:
        return float("nan"), float("nan")
    T = np.zeros((m, m))
    for j in range(m):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < m:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(betas[j]) / alphas[j]
    ev = np.linalg.eigvalsh(T)
    return float(ev[0]), float(ev[-1])


# ---------------------------------------------------------------------------
# Lagrangian P_k on simplicial meshes (fe_oracle_simplex.c)
# ---------------------------------------------------------------------------
def simplex_nn(dim, k):
    """Number of nodes of P_k on the d-simplex."""
    return (k + 1) * (k + 2) // 2 if dim == 2 else (k + 1) * (k + 2) * (k + 3) // 6


def simplex_nodes(dim, k):
    """Lattice points s (nn x dim, integers) of the local nodes, in local order."""
    s = np.zeros(3 * 64, dtype=np.int32)
    nn = lib().orc_sx_nodes(dim, k, _ptr(s))
    return s[: 3 * nn].reshape(nn, 3)[:, :dim].copy()


def simplex_basis(dim, k):
    """Change-of-basis matrix Phi (nn x nn): phi_a = sum_b Phi_ab xi^(alpha_b)."""
    nn = simplex_nn(dim, k)
    Phi = np.zeros((nn, nn))
    if lib().orc_sx_basis(dim, k, _ptr(Phi)) != nn:
        raise ValueError("unsupported dim/order")
    return Phi


def simplex_shape(dim, k, xi):
    """Reference shape values (nn) and gradients (nn x dim) at xi."""
    nn = simplex_nn(dim, k)
    x = _c(list(xi) + [0.0] * (3 - len(xi)), np.float64)
    phi = np.zeros(nn)
    d = np.zeros((nn, dim))
    lib().orc_sx_shape(dim, k, _ptr(x), _ptr(phi), _ptr(d))
    return phi, d


def simplex_quadrature(dim, n):
    """Collapsed Gauss rule: points (n^d x dim) and weights on the reference simplex."""
    nq = n ** dim
    xi = np.zeros((nq, 3))
    w = np.zeros(nq)
    lib().orc_sx_quadrature(dim, n, _ptr(xi), _ptr(w))
    return xi[:, :dim].copy(), w


def simplex_element_matrix(dim, k, X, coef=1.0, problem="poisson", young=1.0, nu=0.3):
    """Element matrix on the simplex with vertices X ((d+1) x d); (A, ok)."""
    X = _c(X, np.float64).reshape(-1)
    ncomp = dim if problem == "elasticity" else 1
    nloc = simplex_nn(dim, k) * ncomp
    A = np.zeros((nloc, nloc))
    lam, mu = lame(young, nu) if problem == "elasticity" else (0.0, 0.0)
    rc = lib().orc_sx_element_matrix(dim, k, 1 if problem == "elasticity" else 0, _ptr(X), float(coef), lam, mu,
                                     _ptr(A))
    if rc == -2:
        raise ValueError("unsupported dim/order")
    return A, rc == 0


def simplex_element_load(dim, k, ncomp, X, source_kind, source):
    X = _c(X, np.float64).reshape(-1)
    src = _c(list(source) + [0.0] * (3 - len(source)), np.float64)
    f = np.zeros(simplex_nn(dim, k) * ncomp)
    lib().orc_sx_element_load(dim, k, ncomp, _ptr(X), int(source_kind), _ptr(src), _ptr(f))
    return f


def simplex_number(dim, k, nverts, cells, dirichlet=True):
    """(node_of (ncells x nn), node_code (nnodes), nfree, nfixed)."""
    cells = _c(cells, np.int32)
    nc = cells.shape[0]
    nn = simplex_nn(dim, k)
    node_of = np.zeros((nc, nn), dtype=np.int64)
    code = np.zeros(max(nc * nn, 1), dtype=np.int64)
    nnodes, nf, nx = _i64(), _i64(), _i64()
    rc = lib().orc_sx_number(dim, k, int(nverts), nc, _ptr(cells), 1 if dirichlet else 0, _ptr(node_of),
                             _ptr(code), ctypes.byref(nnodes), ctypes.byref(nf), ctypes.byref(nx))
    if rc != 0:
        raise ValueError(f"orc_sx_number failed ({rc})")
    return node_of, code[: nnodes.value].copy(), nf.value, nx.value


class SimplexSystem:
    """The oracle's free-free system of P_k on a simplicial mesh.

    verts (nverts x dim), cells (ncells x (dim+1)) int; coef per cell or None;
    problem 'poisson' / 'elasticity'; dirichlet: fix every boundary node;
    dirichlet_kind 0 zero, 1 affine (u_D,c = aff[4c] + sum_r aff[4c+1+r] x_r)."""

    def __init__(self, dim, k, verts, cells, coef=None, problem="poisson", young=1.0, nu=0.3, source_kind=0,
                 source=(0.0, 0.0, 0.0), dirichlet=True, dirichlet_kind=0, dirichlet_affine=None):
        self.dim, self.k, self.problem = int(dim), int(k), problem
        self.verts = _c(verts, np.float64)
        self.cells = _c(cells, np.int32)
        self.coef = None if coef is None else _c(coef, np.float64)
        self.ncomp = dim if problem == "elasticity" else 1
        self.nn = simplex_nn(dim, k)
        self.nloc = self.nn * self.ncomp
        t0 = time.perf_counter()
        self.node_of, self.node_code, self.nfree_nodes, self.nfixed_nodes = simplex_number(
            dim, k, self.verts.shape[0], self.cells, dirichlet)
        self.nnodes = len(self.node_code)
        nc = self.cells.shape[0]
        self.cell_dofs = np.zeros((nc, self.nloc), dtype=np.int64)
        lib().orc_sx_cell_dofs(dim, k, self.ncomp, nc, _ptr(_c(self.node_of, np.int64)), _ptr(self.node_code),
                               _ptr(self.cell_dofs))
        self.nfree = self.nfree_nodes * self.ncomp
        self.rowptr, self.colind = csr_pattern(self.cell_dofs, self.nfree)
        self.nnz = int(self.rowptr[-1])
        self.t_setup = time.perf_counter() - t0  # numbering and pattern (seconds)
        s = OrcSxProblem()
        s.dim, s.k = self.dim, self.k
        s.problem = 1 if problem == "elasticity" else 0
        s.lam, s.mu = lame(young, nu) if problem == "elasticity" else (0.0, 0.0)
        s.source_kind = int(source_kind)
        src = list(source) + [0.0] * (3 - len(source))
        for r in range(3):
            s.source[r] = float(src[r])
        s.dirichlet_kind = int(dirichlet_kind)
        aff = list(dirichlet_affine) if dirichlet_affine is not None else []
        aff = aff + [0.0] * (12 - len(aff))
        for r in range(12):
            s.dirichlet_affine[r] = float(aff[r])
        self._s = s
        self.values = np.zeros(self.nnz)
        self.rhs = np.zeros(self.nfree)
        t0 = time.perf_counter()
        rc = lib().orc_sx_assemble(ctypes.byref(s), _ptr(self.verts), nc, _ptr(self.cells), _ptr(self.coef),
                                   _ptr(self.cell_dofs), self.nfree, _ptr(self.rowptr), _ptr(_c(self.colind, np.int32)),
                                   _ptr(self.values), _ptr(self.rhs))
        self.t_assemble = time.perf_counter() - t0  # numeric assembly (seconds)
        self.ok = rc == 0
        rows = np.repeat(np.arange(self.nfree), np.diff(self.rowptr))
        diag = self.values[self.colind == rows]
        self.dinv = 1.0 / diag if self.nfree else diag

    def node_positions(self):
        xyz = np.zeros((self.nnodes, self.dim))
        lib().orc_sx_node_positions(self.dim, self.k, self.cells.shape[0], _ptr(self.cells), _ptr(self.verts),
                                    _ptr(_c(self.node_of, np.int64)), _ptr(xyz))
        return xyz

    def scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.values, self.colind, self.rowptr), shape=(self.nfree, self.nfree))

    def dense(self):
        return self.scipy().toarray()

    def solve(self):
        import scipy.sparse.linalg as spla
        return spla.spsolve(self.scipy().tocsc(), self.rhs)

    def l2_error(self, x, exact_kind, exact, nq1=None):
        nq1 = nq1 or self.k + 3
        ex = _c(list(exact) + [0.0] * (12 - len(exact)), np.float64)
        return lib().orc_sx_l2_error(ctypes.byref(self._s), _ptr(self.verts), self.cells.shape[0], _ptr(self.cells),
                                     _ptr(self.cell_dofs), _ptr(_c(x, np.float64)), int(nq1), int(exact_kind),
                                     _ptr(ex))


# ---------------------------------------------------------------------------
# Lowest-order Nedelec (edges, covariant Piola) and Raviart-Thomas (facets,
# contravariant Piola) elements on simplices (fe_oracle_simplex.c)
# ---------------------------------------------------------------------------
FAMILIES = {"nedelec": 1, "raviart_thomas": 2, "nedelec2": 3, "raviart_thomas2": 4}


def vector_ndof(family, dim):
    if family == "nedelec2":
        return 20 if dim == 3 else 8
    if family == "raviart_thomas2":
        return 15 if dim == 3 else 8
    return (6 if dim == 3 else 3) if family == "nedelec" else dim + 1


def vector_basis(family, dim):
    nd = vector_ndof(family, dim)
    Phi = np.zeros((nd, nd))
    if lib().orc_vx_basis(FAMILIES[family], dim, _ptr(Phi)) != nd:
        raise ValueError("unsupported family/dim")
    return Phi


def vector_shape(family, dim, xi):
    """Reference shape functions (nd x dim), curls (nd x 3 in 3D, nd in 2D), divergences (nd)."""
    nd = vector_ndof(family, dim)
    x = _c(list(xi) + [0.0] * (3 - len(xi)), np.float64)
    phi = np.zeros((nd, dim))
    curl = np.zeros((nd, 3)) if dim == 3 else np.zeros(nd)
    div = np.zeros(nd)
    lib().orc_vx_shape(FAMILIES[family], dim, _ptr(x), _ptr(phi), _ptr(curl), _ptr(div))
    return phi, curl, div


def vector_element(family, dim, X, g, coef=1.0, kappa=1.0, source_kind=0, source=(0.0, 0.0, 0.0)):
    """Element matrix and load (global orientation signs applied); (A, f, ok)."""
    nd = vector_ndof(family, dim)
    A = np.zeros((nd, nd))
    f = np.zeros(nd)
    src = _c(list(source) + [0.0] * (12 - len(source)), np.float64)
    rc = lib().orc_vx_element(FAMILIES[family], dim, _ptr(_c(X, np.float64).reshape(-1)), _ptr(_c(g, np.int32)),
                              float(coef), float(kappa), int(source_kind), _ptr(src), _ptr(A), _ptr(f))
    return A, f, rc == 0


def vector_number(family, dim, nverts, cells, dirichlet=True):
    cells = _c(cells, np.int32)
    nc = cells.shape[0]
    nd = vector_ndof(family, dim)
    dof_of = np.zeros((nc, nd), dtype=np.int64)
    code = np.zeros(max(nc * nd, 1), dtype=np.int64)
    ne, nf, nx = _i64(), _i64(), _i64()
    rc = lib().orc_vx_number(FAMILIES[family], dim, int(nverts), nc, _ptr(cells), 1 if dirichlet else 0,
                             _ptr(dof_of), _ptr(code), ctypes.byref(ne), ctypes.byref(nf), ctypes.byref(nx))
    if rc != 0:
        raise ValueError(f"orc_vx_number failed ({rc})")
    return dof_of, code[: ne.value].copy(), nf.value, nx.value


class VectorSystem:
    """The oracle's free-free system of a vector element on a simplicial mesh
    ("nedelec", "raviart_thomas": lowest order; "nedelec2", "raviart_thomas2":
    second order): int coef curl.curl (div div) + kappa u.v, zero tangential
    (normal) trace on the boundary when dirichlet.  source_kind 1 constant,
    2 the manufactured field, 3 affine (12 coefficients, as a Dirichlet datum)."""

    def __init__(self, family, dim, verts, cells, coef=None, kappa=1.0, source_kind=0, source=(0.0, 0.0, 0.0),
                 dirichlet=True):
        self.family, self.dim = family, int(dim)
        self.verts = _c(verts, np.float64)
        self.cells = _c(cells, np.int32)
        self.coef = None if coef is None else _c(coef, np.float64)
        self.kappa = float(kappa)
        self.nd = vector_ndof(family, dim)
        self.dof_of, self.code, self.nfree, self.nfixed = vector_number(family, dim, self.verts.shape[0], self.cells,
                                                                        dirichlet)
        self.nent = len(self.code)
        self.cell_dofs = self.code[self.dof_of]
        self.rowptr, self.colind = csr_pattern(self.cell_dofs, self.nfree)
        self.nnz = int(self.rowptr[-1])
        self.values = np.zeros(self.nnz)
        self.rhs = np.zeros(self.nfree)
        src = _c(list(source) + [0.0] * (12 - len(source)), np.float64)
        t0 = time.perf_counter()
        rc = lib().orc_vx_assemble(FAMILIES[family], self.dim, _ptr(self.verts), self.cells.shape[0], _ptr(self.cells),
                                   _ptr(self.coef), self.kappa, int(source_kind), _ptr(src), _ptr(self.cell_dofs),
                                   self.nfree, _ptr(self.rowptr), _ptr(_c(self.colind, np.int32)), _ptr(self.values),
                                   _ptr(self.rhs))
        self.t_assemble = time.perf_counter() - t0
        self.ok = rc == 0
        rows = np.repeat(np.arange(self.nfree), np.diff(self.rowptr))
        diag = self.values[self.colind == rows]
        self.dinv = 1.0 / diag if self.nfree else diag

    def scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.values, self.colind, self.rowptr), shape=(self.nfree, self.nfree))

    def solve(self):
        import scipy.sparse.linalg as spla
        return spla.spsolve(self.scipy().tocsc(), self.rhs)

    def l2_error(self, x, scale, nq1=4):
        return lib().orc_vx_l2_error(FAMILIES[self.family], self.dim, _ptr(self.verts), self.cells.shape[0],
                                     _ptr(self.cells), _ptr(_c(self.cell_dofs, np.int64)), _ptr(_c(x, np.float64)),
                                     float(scale), int(nq1))
