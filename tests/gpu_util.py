"""Shared helpers of the GPU parity tests: build one problem on both sides
(HIP library through the C ABI, and the oracle) from the same seeded inputs."""
import numpy as np

import oracle as O
from fe_inputs import lognormal_coefficients, structured_vertices
from paper_1708_01773_amd import fe as F

MATRIX_RTOL = 1e-12  # relative Frobenius tolerance of FP64 matrices and vectors


def say(*a):
    print(*a, flush=True)


class Pair:
    def __init__(self, dim, n, k, prob="poisson", jitter=0.2, lognormal=True, faces=None, source_kind=1,
                 source=(1.0, 0.0, -1.0), dirichlet_kind=0, affine=None, seed=0, precision="fp64"):
        n = list(n) if hasattr(n, "__len__") else [n] * dim
        self.dim, self.n, self.k, self.prob = dim, n, k, prob
        self.v = structured_vertices(dim, n, jitter=jitter, seed=17080 + seed)
        self.P = O.Problem(dim, n, k, problem=prob, faces=faces, source_kind=source_kind, source=source,
                           dirichlet_kind=dirichlet_kind, dirichlet_affine=affine)
        self.coef = lognormal_coefficients(self.P.ncells, seed=17081 + seed) if lognormal else None
        self.mesh = F.create_mesh(dim, n, self.v, self.coef)
        self.coeff = F.make_coeff(prob, precision, source_kind=source_kind, source=source, faces=self.P.faces,
                                  dim=dim, dirichlet_kind=dirichlet_kind, affine=affine)
        self._sys = None

    @property
    def system(self):
        """The oracle's full system (only for sizes it finishes in seconds)."""
        if self._sys is None:
            self._sys = O.System(self.P, self.v, self.coef)
        return self._sys

    def gpu_assembly(self):
        import torch
        A = F.Assembly(self.mesh, self.k, self.coeff)
        A.pattern()
        A.assemble()
        torch.cuda.synchronize()
        return A

    def oracle_element(self, cell):
        X = O.cell_vertices(self.dim, self.n, self.v, cell)
        coef = 1.0 if self.coef is None else self.coef[cell]
        A, ok = O.element_matrix(self.dim, self.k, X, coef=coef, problem=self.prob)
        return A


def element_matrices(pair, A, cells):
    """Element matrices of the given cells read from the K3 workspace."""
    import torch
    nloc, cb, eb, off, packed = F.element_layout(pair.mesh, pair.k, pair.coeff)
    dt = torch.float64 if eb == 8 else torch.float32
    ncells = pair.P.ncells
    ncells_pad = (ncells + cb - 1) // cb * cb
    ne = nloc * (nloc + 1) // 2 if packed else nloc * nloc
    E = A.ws[: ncells_pad * ne * eb].view(dt).view(ncells_pad // cb, ne, cb)
    out = []
    for c in cells:
        e = E[c // cb, :, c % cb].double().cpu().numpy()
        if packed:  # upper triangle, row-major
            M = np.zeros((nloc, nloc))
            iu = np.triu_indices(nloc)
            M[iu] = e
            M = M + np.triu(M, 1).T
            out.append(M)
        else:
            out.append(e.reshape(nloc, nloc))
    Fl = A.ws[off: off + ncells * nloc * 8].view(torch.float64).view(ncells, nloc)
    return out, Fl.cpu().numpy()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
