"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no finite element arithmetic: it only draws meshes and
coefficients.  Both the HIP library and the oracle receive the arrays it
returns.  Recipe (stated once here, used everywhere):

* RNG: ``numpy.random.Generator(numpy.random.PCG64(seed))``.
* Mesh: structured brick of n_0 x n_1 (x n_2) cells on the unit square/cube.
  Vertex (i, j, l) sits at (i h_0, j h_1, l h_2), h_r = 1/n_r, numbered
  lexicographically with x fastest; coordinates are returned as an
  (n_vertices, d) float64 array.  With ``jitter > 0`` every interior vertex
  (not on the boundary) moves by ``rng.uniform(-jitter, jitter, size=(n_int, d)) * h``
  drawn in vertex-lexicographic order, one row per interior vertex; boundary
  vertices stay put.  The workloads use jitter 0.2 (i.e. +-0.2 h).
* Simplicial mesh (``simplex_mesh``): the Kuhn (Freudenthal) subdivision of
  the brick above, with the jittered vertices: every cell (lexicographic
  order) splits into d! simplices, one per permutation pi of the axes (in
  ``itertools.permutations`` order), with vertices c, c + e_pi0,
  c + e_pi0 + e_pi1, ... (the cell's lower corner c).  With ``shuffle`` the
  vertex labels, the cell order and each cell's local vertex order are
  permuted at random (seed 17084): the same mesh as general connectivity.
* Coefficients: per-cell ``exp(rng.standard_normal(ncells))`` (lognormal,
  cell-lexicographic order), or all ones.
* Seeds: jitter 17080, coefficients 17081, batch sampling 17082, arrivals
  17083; problem i of a batch or request stream uses 17080 + 1000 (i + 1)
  and 17081 + 1000 (i + 1).
"""
import numpy as np

SEED_JITTER = 17080
SEED_COEF = 17081
SEED_BATCH = 17082
SEED_ARRIVALS = 17083
SEED_SHUFFLE = 17084


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _dims(dim, n):
    if np.isscalar(n):
        n = [int(n)] * dim
    n = [int(v) for v in n][:dim]
    if len(n) != dim:
        raise ValueError("n must have one entry per dimension")
    return n


def structured_vertices(dim, n, jitter=0.0, seed=SEED_JITTER):
    """Vertex coordinates (n_vertices, dim) of an n^d brick on [0,1]^d."""
    n = _dims(dim, n)
    axes = [np.arange(nr + 1, dtype=np.float64) / nr for nr in n]
    if dim == 2:
        Y, X = np.meshgrid(axes[1], axes[0], indexing="ij")
        v = np.stack([X.ravel(), Y.ravel()], axis=1)
        idx = np.meshgrid(np.arange(n[1] + 1), np.arange(n[0] + 1), indexing="ij")
        interior = ((idx[1] > 0) & (idx[1] < n[0]) & (idx[0] > 0) & (idx[0] < n[1])).ravel()
    else:
        Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
        v = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
        I2, I1, I0 = np.meshgrid(np.arange(n[2] + 1), np.arange(n[1] + 1), np.arange(n[0] + 1), indexing="ij")
        interior = ((I0 > 0) & (I0 < n[0]) & (I1 > 0) & (I1 < n[1]) & (I2 > 0) & (I2 < n[2])).ravel()
    if jitter > 0.0:
        h = np.array([1.0 / nr for nr in n])
        g = rng(seed)
        nint = int(interior.sum())
        d = g.uniform(-jitter, jitter, size=(nint, dim)) * h
        v[interior] += d
    return np.ascontiguousarray(v)


def lognormal_coefficients(ncells, seed=SEED_COEF):
    """Per-cell coefficient k_K = exp(g), g ~ N(0, 1) i.i.d."""
    return np.exp(rng(seed).standard_normal(int(ncells)))


def ncells_of(dim, n):
    n = _dims(dim, n)
    out = 1
    for v in n:
        out *= v
    return out


def problem_seeds(i):
    """(jitter seed, coefficient seed) of problem i in a batch or request stream."""
    return SEED_JITTER + 1000 * (i + 1), SEED_COEF + 1000 * (i + 1)


def batch_specs(nprob=512, seed=SEED_BATCH, nmin=8, nmax=64, orders=(1, 2, 3)):
    """Sizes and orders of a batch of independent 3D Poisson problems:
    n_i uniform in [nmin, nmax], order uniform in ``orders``."""
    g = rng(seed)
    ns = g.integers(nmin, nmax + 1, size=nprob)
    ks = g.integers(min(orders), max(orders) + 1, size=nprob)
    return [(int(a), int(b)) for a, b in zip(ns, ks)]


def serving_requests(nreq, rate, seed=SEED_ARRIVALS, nmin=8, nmax=96, kmax=4):
    """Poisson-process arrivals: (arrival time s, n, order) per request; n is
    log-uniform in [nmin, nmax], order uniform in 1..kmax."""
    g = rng(seed)
    gaps = g.exponential(1.0 / rate, size=nreq)
    t = np.cumsum(gaps) - gaps[0]
    ns = np.rint(np.exp(g.uniform(np.log(nmin), np.log(nmax), size=nreq))).astype(int)
    ks = g.integers(1, kmax + 1, size=nreq)
    return [(float(a), int(b), int(c)) for a, b, c in zip(t, ns, ks)]


def simplex_mesh(dim, n, jitter=0.0, seed=SEED_JITTER, shuffle=False, shuffle_seed=SEED_SHUFFLE):
    """(vertices (nverts x dim) float64, cells (ncells x (dim+1)) int32) of the
    Kuhn subdivision of the n^d brick."""
    import itertools
    n = _dims(dim, n)
    v = structured_vertices(dim, n, jitter, seed)
    perms = list(itertools.permutations(range(dim)))
    if dim == 2:
        j, i = np.meshgrid(np.arange(n[1]), np.arange(n[0]), indexing="ij")
        base = (i + (n[0] + 1) * j).ravel()
        stride = [1, n[0] + 1]
    else:
        l, j, i = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
        base = (i + (n[0] + 1) * (j + (n[1] + 1) * l)).ravel()
        stride = [1, n[0] + 1, (n[0] + 1) * (n[1] + 1)]
    cells = np.zeros((base.size, len(perms), dim + 1), dtype=np.int64)
    for p, pi in enumerate(perms):
        off = 0
        cells[:, p, 0] = base
        for t, axis in enumerate(pi):
            off += stride[axis]
            cells[:, p, t + 1] = base + off
    cells = cells.reshape(-1, dim + 1)
    if shuffle:
        g = rng(shuffle_seed)
        relabel = g.permutation(v.shape[0])
        v2 = np.empty_like(v)
        v2[relabel] = v
        v = v2
        cells = relabel[cells]
        cells = cells[g.permutation(cells.shape[0])]
        order = np.argsort(g.random(cells.shape), axis=1)
        cells = np.take_along_axis(cells, order, axis=1)
    return np.ascontiguousarray(v), np.ascontiguousarray(cells.astype(np.int32))
