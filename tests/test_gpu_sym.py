"""GPU parity of the symmetric storage of Q1 scalar systems (upper triangle,
slot-major): its layout against the oracle's pattern, its SpMV bitwise
against the CSR value traversal of the same matrix and against the oracle,
its PCG against the CSR-value PCG and a direct solve."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import oracle as O
from paper_1708_01773_amd import fe as F
from tests.gpu_util import Pair, rel, say

pytestmark = pytest.mark.gpu

# (dim, cells per axis, Dirichlet faces): all-Dirichlet, mixed Neumann faces
# (rows on a Neumann face keep their outer neighbours' slots empty), ragged
# row counts (not multiples of 32 or 64), and a single free line.
CASES = [(3, [7, 6, 5], None), (3, [9, 4, 6], 0b011010), (3, [5, 5, 5], 0b000001), (2, [33, 17], None),
         (2, [5, 40], 0b0110), (3, [40, 2, 2], None), (2, [64, 3], 0b1111)]


def _free_coords(dim, n, faces):
    """Lattice coordinates of the oracle's free nodes, by free index."""
    code, nfree, _ = O.number_nodes(dim, n, 1, faces)
    N = [c + 1 for c in n] + [1] * (3 - dim)
    ids = np.nonzero(code >= 0)[0]
    out = np.zeros((nfree, 3), dtype=np.int64)
    out[code[ids]] = np.stack([ids % N[0], (ids // N[0]) % N[1], ids // (N[0] * N[1])], axis=1)
    return out


def _expected_sym(S, coords, dim, values):
    """The slot-major upper triangle built from the oracle's pattern: slot
    g - C of row r holds the entry of the column whose node sits at offset d
    (g = 9 (dz+1) + 3 (dy+1) + (dx+1), C = 13; 2D: g = 3 (dy+1) + (dx+1), C = 4)."""
    n = S.nfree
    ns = (n + 63) // 64 * 64
    C = 13 if dim == 3 else 4
    out = np.zeros((C + 1) * ns)
    for r in range(n):
        for p in range(S.rowptr[r], S.rowptr[r + 1]):
            c = S.colind[p]
            if c < r:
                continue
            d = coords[c] - coords[r]
            assert np.all(np.abs(d) <= 1)
            g = 9 * (d[2] + 1) + 3 * (d[1] + 1) + (d[0] + 1) if dim == 3 else 3 * (d[1] + 1) + (d[0] + 1)
            assert g >= C
            out[(g - C) * ns + r] = values[p]
    return out


def _sym_of(pair, A):
    nb = F.sym_query(pair.mesh, 1, pair.coeff)
    sym = torch.full((nb // 8,), float("nan"), dtype=torch.float64, device="cuda")
    F.sym_from_csr(pair.mesh, 1, pair.coeff, A.csr, sym)
    return sym


@pytest.mark.parametrize("dim,n,faces", CASES)
def test_symmetric_storage_layout_and_spmv(dim, n, faces):
    pair = Pair(dim, n, 1, faces=faces, seed=51)
    A = pair.gpu_assembly()
    say(f"[sym] dim {dim} n {n} faces {faces} rows {A.n_rows}")
    S = pair.system
    coords = _free_coords(dim, n, pair.P.faces)
    vals = A.values[: A.nnz].cpu().numpy()
    # the assembled matrix is bitwise symmetric (same element entries, same cell order)
    M = S.scipy().tocsr()
    M.data = vals.copy()
    assert (M != M.T).nnz == 0
    sym = _sym_of(pair, A)
    torch.cuda.synchronize()
    got = sym.cpu().numpy()
    # placement: bit-exact against the layout built from the oracle's pattern
    # and the assembled values; every slot entry written (empty ones are 0)
    assert np.array_equal(got, _expected_sym(S, coords, dim, vals))
    # values: the oracle's upper triangle to 1e-12
    want = _expected_sym(S, coords, dim, S.values)
    assert np.all(np.abs(got - want) <= 1e-12 * np.abs(want).max())
    # SpMV: bitwise the Q1 value traversal, and the oracle's product to 1e-12
    x = torch.from_numpy(np.random.Generator(np.random.PCG64(52)).standard_normal(A.n_rows)).cuda()
    y = torch.empty_like(x)
    ym = torch.empty_like(x)
    F.spmv_sym(pair.mesh, 1, pair.coeff, sym, x, y)
    F.spmv_mesh(pair.mesh, 1, pair.coeff, A.csr, x, ym)
    torch.cuda.synchronize()
    assert torch.equal(y, ym)
    xo = x.cpu().numpy()
    yo = O.spmv(S.rowptr, S.colind, S.values, xo)
    scale = O.spmv(S.rowptr, S.colind, np.abs(S.values), np.abs(xo))
    assert np.all(np.abs(y.cpu().numpy() - yo) <= 1e-12 * scale + 1e-300)


def _solve_pair(pair, A, sym, rtol):
    """Symmetric-storage solve (twice: bitwise reproducible) and the CSR-value solve."""
    ws = torch.empty(F.pcg_query(A.n_rows), dtype=torch.uint8, device="cuda")
    u = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
    info = F.pcg_solve_sym(pair.mesh, 1, pair.coeff, A.csr, sym, A.rhs, u, rtol, 20000, ws)
    u2 = torch.zeros_like(u)
    info2 = F.pcg_solve_sym(pair.mesh, 1, pair.coeff, A.csr, sym, A.rhs, u2, rtol, 20000, ws)
    um = torch.zeros_like(u)
    im = A.solve(um, rtol, 20000, ws)
    torch.cuda.synchronize()
    say(f"   iters sym {info['iters']} mesh {im['iters']}")
    assert info["status"] == info2["status"] == im["status"] == F.FE_OK
    assert info2["iters"] == info["iters"] and torch.equal(u, u2)
    # same rows and products; the fused p.q partials group 256 rows instead of
    # 128, so the iterates agree to rounding (amplified by the CG recurrences)
    assert abs(info["iters"] - im["iters"]) <= 2 and info["relres"] <= rtol
    assert float(torch.linalg.vector_norm(u - um) / torch.linalg.vector_norm(um)) <= 1e3 * rtol
    return u


@pytest.mark.parametrize("dim,n,faces", CASES)
def test_symmetric_storage_pcg(dim, n, faces):
    pair = Pair(dim, n, 1, faces=faces, seed=53)
    A = pair.gpu_assembly()
    say(f"[sym pcg] dim {dim} n {n} faces {faces} rows {A.n_rows}")
    u = _solve_pair(pair, A, _sym_of(pair, A), 1e-10)
    S = pair.system
    assert rel(u.cpu().numpy(), spla.spsolve(S.scipy().tocsc(), S.rhs)) <= 1e-8


def test_symmetric_storage_with_wave_strided_steps():
    """Above 256 x 32768 rows the blocks take several steps each (mode 7, the
    looping form): SpMV bitwise that of the Q1 value traversal, PCG as above."""
    n = 205  # 204^3 = 8.49M free nodes
    pair = Pair(3, [n, n, n], 1, seed=13)
    A = pair.gpu_assembly()
    assert A.n_rows > 256 * 32768
    say(f"[sym strided] rows {A.n_rows} nnz {A.nnz}")
    sym = _sym_of(pair, A)
    g = torch.Generator(device="cuda").manual_seed(54)
    x = torch.rand(A.n_rows, dtype=torch.float64, device="cuda", generator=g) - 0.5
    y = torch.empty_like(x)
    ym = torch.empty_like(x)
    F.spmv_sym(pair.mesh, 1, pair.coeff, sym, x, y)
    F.spmv_mesh(pair.mesh, 1, pair.coeff, A.csr, x, ym)
    torch.cuda.synchronize()
    assert torch.equal(y, ym)
    _solve_pair(pair, A, sym, 1e-8)


def test_symmetric_storage_refuses_other_spaces_and_bad_buffers():
    q2 = Pair(3, [3, 3, 2], 2, seed=55)
    with pytest.raises(F.FeError, match="Q1 scalar"):
        F.sym_query(q2.mesh, 2, q2.coeff)
    el = Pair(3, [3, 3, 2], 1, "elasticity", seed=56)
    with pytest.raises(F.FeError, match="Q1 scalar"):
        F.sym_query(el.mesh, 1, el.coeff)
    pair = Pair(3, [4, 4, 4], 1, seed=57)
    A = pair.gpu_assembly()
    nb = F.sym_query(pair.mesh, 1, pair.coeff)
    assert nb == 14 * ((A.n_rows + 63) // 64 * 64) * 8
    small = torch.empty(nb // 8 - 1, dtype=torch.float64, device="cuda")
    with pytest.raises(F.FeError, match="too small"):
        F.sym_from_csr(pair.mesh, 1, pair.coeff, A.csr, small)
    raw = torch.empty(nb + 8, dtype=torch.uint8, device="cuda")
    with pytest.raises(F.FeError, match="8-byte"):
        F.sym_from_csr(pair.mesh, 1, pair.coeff, A.csr, raw[4: 4 + nb])


@pytest.mark.parametrize("dim,n", [(3, [1, 1, 1]), (3, [2, 2, 2]), (2, [2, 2]), (2, [1, 3])])
def test_symmetric_storage_of_empty_and_single_row_systems(dim, n):
    """All-Dirichlet meshes with no free node (nothing launched, FE_OK) or one
    free node (a 1 x 1 system: the diagonal slot only)."""
    pair = Pair(dim, n, 1, seed=58)
    A = pair.gpu_assembly()
    say(f"[sym edge] dim {dim} n {n} rows {A.n_rows}")
    nb = F.sym_query(pair.mesh, 1, pair.coeff)
    assert nb == (14 if dim == 3 else 5) * ((A.n_rows + 63) // 64 * 64) * 8
    sym = torch.full((max(nb // 8, 1),), float("nan"), dtype=torch.float64, device="cuda")
    F.sym_from_csr(pair.mesh, 1, pair.coeff, A.csr, sym)
    x = torch.ones(max(A.n_rows, 1), dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    F.spmv_sym(pair.mesh, 1, pair.coeff, sym, x, y)
    ws = torch.empty(F.pcg_query(A.n_rows), dtype=torch.uint8, device="cuda")
    u = torch.zeros_like(x)
    info = F.pcg_solve_sym(pair.mesh, 1, pair.coeff, A.csr, sym, A.rhs, u, 1e-10, 100, ws)
    torch.cuda.synchronize()
    assert info["status"] == F.FE_OK
    if A.n_rows == 0:
        assert nb == 0 and info["iters"] == 0
    else:
        assert A.n_rows == 1
        d = float(A.values[0])
        assert float(sym[0]) == d and bool(torch.all(sym[1:] == 0.0))
        assert float(y[0]) == d
        assert abs(float(u[0]) - float(A.rhs[0]) / d) <= 1e-14 * abs(float(A.rhs[0]) / d)


@pytest.mark.parametrize("dim,n", [(3, [7, 6, 5]), (2, [33, 17])])
def test_symmetric_storage_with_vectors_off_16_byte_boundaries(dim, n):
    """x is staged with 16-byte loads when it is 16-byte aligned, else with
    8-byte loads into the same slots: an x (and a workspace, which holds the
    PCG's direction) 8 bytes off a 16-byte boundary give bitwise the same."""
    pair = Pair(dim, n, 1, seed=59)
    A = pair.gpu_assembly()
    say(f"[sym unaligned] dim {dim} n {n} rows {A.n_rows}")
    sym = _sym_of(pair, A)
    x = torch.from_numpy(np.random.Generator(np.random.PCG64(60)).standard_normal(A.n_rows)).cuda()
    xb = torch.empty(A.n_rows + 1, dtype=torch.float64, device="cuda")
    xb[1:] = x
    xm = xb[1:]
    assert xm.data_ptr() % 16 == 8
    y, ym = torch.empty_like(x), torch.empty_like(x)
    F.spmv_sym(pair.mesh, 1, pair.coeff, sym, x, y)
    F.spmv_sym(pair.mesh, 1, pair.coeff, sym, xm, ym)
    nbw = F.pcg_query(A.n_rows)
    ws = torch.empty(nbw, dtype=torch.uint8, device="cuda")
    wb = torch.empty(nbw + 16, dtype=torch.uint8, device="cuda")
    w8 = wb[8: 8 + nbw]
    assert w8.data_ptr() % 16 == 8
    u, u8 = torch.zeros_like(x), torch.zeros_like(x)
    info = F.pcg_solve_sym(pair.mesh, 1, pair.coeff, A.csr, sym, A.rhs, u, 1e-10, 20000, ws)
    info8 = F.pcg_solve_sym(pair.mesh, 1, pair.coeff, A.csr, sym, A.rhs, u8, 1e-10, 20000, w8)
    torch.cuda.synchronize()
    assert torch.equal(y, ym)
    assert info["status"] == info8["status"] == F.FE_OK and info["iters"] == info8["iters"] and torch.equal(u, u8)


def _views_above_bit_31(sizes):
    """Byte views of one allocation of 4 GiB and a little more, each starting
    at an address whose low 32 bits have the top bit set (256-byte aligned).
    Kernels that take a buffer's base in scalar registers rebuild it from two
    32-bit halves; a low half read back as a signed int would corrupt the
    high half exactly at such addresses."""
    spans = [(s + 255) // 256 * 256 for s in sizes]
    assert sum(spans) <= 2**30
    buf = torch.empty(2**32 + sum(spans) + 256, dtype=torch.uint8, device="cuda")
    off = ((2**31 + 2**20) - (buf.data_ptr() & 0xFFFFFFFF)) % 2**32
    views = []
    for s, sp in zip(sizes, spans):
        v = buf[off: off + s]
        assert v.data_ptr() & 0x80000000 and (v.data_ptr() & 0xFFFFFFFF) + s < 2**32
        views.append(v)
        off += sp
    return buf, views


@pytest.mark.parametrize("dim,n", [(3, [7, 6, 5]), (2, [33, 17])])
def test_symmetric_storage_at_addresses_with_bit_31_set(dim, n):
    """The symmetric storage (FP64 and FP32), x and the workspace placed where
    the low word of the address has its top bit set: the same storage, the
    same products and bitwise the same solves as at ordinary addresses."""
    pair = Pair(dim, n, 1, seed=62)
    A = pair.gpu_assembly()
    say(f"[sym bit 31] dim {dim} n {n} rows {A.n_rows}")
    nb = F.sym_query(pair.mesh, 1, pair.coeff)
    nbw, nbr = F.pcg_query(A.n_rows), F.refine_query(A.n_rows)
    buf, (b64, b32, bx, bw, br) = _views_above_bit_31([nb, nb // 2, 8 * A.n_rows, nbw, nbr])
    sym, sym_h = _sym_of(pair, A), b64.view(torch.float64)
    F.sym_from_csr(pair.mesh, 1, pair.coeff, A.csr, sym_h)
    sym32 = torch.empty(nb // 8, dtype=torch.float32, device="cuda")
    sym32_h = b32.view(torch.float32)
    F.sym_fp32_from_csr(pair.mesh, 1, pair.coeff, A.csr, sym32)
    F.sym_fp32_from_csr(pair.mesh, 1, pair.coeff, A.csr, sym32_h)
    x = torch.from_numpy(np.random.Generator(np.random.PCG64(63)).standard_normal(A.n_rows)).cuda()
    x_h = bx.view(torch.float64)
    x_h.copy_(x)
    y, y_h = torch.empty_like(x), torch.empty_like(x)
    F.spmv_sym(pair.mesh, 1, pair.coeff, sym, x, y)
    F.spmv_sym(pair.mesh, 1, pair.coeff, sym_h, x_h, y_h)
    ws, wr = (torch.empty(k, dtype=torch.uint8, device="cuda") for k in (nbw, nbr))
    u, u_h = torch.zeros_like(x), torch.zeros_like(x)
    info = F.pcg_solve_sym(pair.mesh, 1, pair.coeff, A.csr, sym, A.rhs, u, 1e-10, 20000, ws)
    info_h = F.pcg_solve_sym(pair.mesh, 1, pair.coeff, A.csr, sym_h, A.rhs, u_h, 1e-10, 20000, bw)
    v, v_h = torch.zeros_like(x), torch.zeros_like(x)
    rinfo = F.refine_solve_sym(pair.mesh, 1, pair.coeff, A.csr, A.csr, sym32, A.rhs, v, 1e-12, 1e-4, 50, 5000, wr)
    rinfo_h = F.refine_solve_sym(pair.mesh, 1, pair.coeff, A.csr, A.csr, sym32_h, A.rhs, v_h, 1e-12, 1e-4, 50, 5000,
                                 br)
    torch.cuda.synchronize()
    assert torch.equal(sym_h, sym) and torch.equal(sym32_h, sym32) and torch.equal(y_h, y)
    assert info["status"] == info_h["status"] == F.FE_OK and info_h["iters"] == info["iters"]
    assert torch.equal(u_h, u)
    assert rinfo["status"] == F.FE_OK and rinfo_h == rinfo and torch.equal(v_h, v)
    del buf
    torch.cuda.empty_cache()
