"""Batched form: many independent 3D Poisson problems of uneven size and
order assembled and solved together through the batched C ABI calls, in
waves whose device memory fits a budget.  With reduced-precision element
integration the problems are solved by batched iterative refinement: each is
also assembled in FP64, whose residuals the corrections are taken against, so
the batched solutions reach those of the plain FP64 path.

Every problem is the scalar problem -div(k grad u) = 1 on the unit cube with
u = 0 on the boundary, on an n^3 brick with interior vertices jittered by
+-0.2 h and lognormal per-cell coefficients; problem i draws its jitter and
coefficients from its own seeds, so a problem is the same whichever batch or
wave it lands in.
"""
import time

from fe_inputs import lognormal_coefficients, problem_seeds, structured_vertices

from . import fe as F


def make_problem(i, n, k, precision="fp32"):
    """(mesh, order, coeff) of problem i of a batch.  A jitter draw of +-0.2 h
    can invert a cell (about one mesh in a few hundred of 64^3 cells); the
    library refuses such a mesh, and the problem then takes the next draw
    (jitter seed + 1 for every attempt), so it stays the same in every run."""
    sj, sc = problem_seeds(i)
    coef = lognormal_coefficients(n ** 3, seed=sc)
    for attempt in range(16):
        v = structured_vertices(3, n, jitter=0.2, seed=sj + attempt)
        try:
            mesh = F.create_mesh(3, [n, n, n], v, coef)
            break
        except F.FeError as e:
            if e.status != F.FE_EMESH or attempt == 15:
                raise
    coeff = F.make_coeff("poisson", precision, source_kind=F.FE_SOURCE_CONST, source=(1.0,), dim=3)
    return mesh, int(k), coeff


def problem_bytes(n_rows, nnz, asm_ws_bytes, refine=False):
    """Device bytes one problem holds while its wave runs: CSR (int64 row
    pointers, int32 columns, FP64 values), rhs, Jacobi diagonal, solution,
    the PCG vectors (r, p, q) and its element workspace; with refinement a
    second system (the FP64 one) and the correction vectors r, d."""
    one = 8 * (n_rows + 1) + 12 * nnz + 3 * 8 * n_rows + 3 * 8 * n_rows + 256 * 1024 + asm_ws_bytes
    return 2 * one + 2 * 8 * n_rows if refine else one


def plan_waves(sizes, budget):
    """Greedy waves in problem order: a wave takes problems while their bytes
    fit the budget.  A problem larger than the budget cannot run."""
    waves, cur, used = [], [], 0
    for i, b in enumerate(sizes):
        if b > budget:
            raise ValueError(f"problem {i} needs {b} bytes, more than the budget {budget}")
        if cur and used + b > budget:
            waves.append(cur)
            cur, used = [], 0
        cur.append(i)
        used += b
    if cur:
        waves.append(cur)
    return waves


class BatchRun:
    """Meshes of a list of (n, k) specs, their sizes and wave plan."""

    def __init__(self, specs, precision="fp32", budget=160 << 30, first_index=0, refine=None):
        self.specs = list(specs)
        self.precision = precision
        # reduced-precision integration is refined against FP64 unless told otherwise
        self.refine = precision != "fp64" if refine is None else bool(refine)
        self.problems = [make_problem(first_index + i, n, k, precision) for i, (n, k) in enumerate(self.specs)]
        self.coeffs_hi = [F.make_coeff("poisson", "fp64", source_kind=F.FE_SOURCE_CONST, source=(1.0,), dim=3)
                          for _ in self.problems] if self.refine else None
        self.sizes, self.n_rows, self.nnz = [], [], []
        for mesh, k, coeff in self.problems:
            nr, nz, ws = F.assemble_query(mesh, k, coeff)
            self.n_rows.append(nr)
            self.nnz.append(nz)
            self.sizes.append(problem_bytes(nr, nz, ws, self.refine))
        self.waves = plan_waves(self.sizes, budget)
        self.cells = sum(n ** 3 for n, _ in self.specs)

    def autotune(self, reps=10):
        """Tunes the evaluated-pattern SpMV plan of every row class in the batch
        (longest row, components) on its largest matrix, assembled alone for
        the purpose; the batched solve then uses the tuned plans."""
        best = {}
        for i, (mesh, k, coeff) in enumerate(self.problems):
            if self.n_rows[i] == 0:
                continue
            cls = F.spmv_plan_of_mesh(mesh, k, coeff)[2]
            if cls not in best or self.nnz[i] > self.nnz[best[cls]]:
                best[cls] = i
        chosen = {}
        for cls, i in sorted(best.items()):
            mesh, k, coeff = self.problems[i]
            A = F.Assembly(mesh, k, coeff)
            A.pattern()
            A.assemble()
            ch, tried = F.spmv_autotune_mesh(mesh, k, coeff, A.csr, reps)
            chosen[cls] = dict(chosen=ch, tried=tried,
                               matrix=dict(problem=i, order=k, n_rows=self.n_rows[i], nnz=self.nnz[i]))
            del A
        return chosen

    def run(self, rtol, maxit, keep=None, stream=None, progress=None, inner_rtol=1e-4, max_outer=50):
        """Assembles and solves every wave; returns per-phase times and the
        per-problem solver infos.  keep(i, x) is called with each solution,
        progress(w, nwaves, assemble_s, solve_s) after each wave.  With
        refinement both systems of every problem are assembled and the wave is
        solved by batched iterative refinement (maxit bounds each inner solve)."""
        import torch
        infos = [None] * len(self.specs)
        t_setup = t_asm = t_solve = 0.0
        status = F.FE_OK
        for wave in self.waves:
            ts = time.perf_counter()
            probs = [self.problems[i] for i in wave]
            meshes, orders = [p[0] for p in probs], [p[1] for p in probs]
            B = F.BatchAssembly(meshes, orders, [p[2] for p in probs], stream=stream)
            Bh = F.BatchAssembly(meshes, orders, [self.coeffs_hi[i] for i in wave], stream=stream) \
                if self.refine else None
            rws = torch.empty(max(F.refine_batch_query(B.n_rows), 8), dtype=torch.uint8, device="cuda") \
                if self.refine else None
            torch.cuda.synchronize()
            ta = time.perf_counter()
            B.assemble(stream)
            if Bh is not None:
                Bh.assemble(stream)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            if Bh is not None:
                for x in Bh.x:
                    x.zero_()
                st, inf = F.refine_solve_batch_mesh(meshes, orders, Bh.coeffs, Bh.csrs, B.csrs, Bh.rhs, Bh.x, rtol,
                                                    inner_rtol, max_outer, maxit, rws, stream)
                B.x = Bh.x
            else:
                st, inf = B.solve(rtol, maxit, stream)
            torch.cuda.synchronize()
            tc = time.perf_counter()
            t_setup += ta - ts
            t_asm += tb - ta
            t_solve += tc - tb
            if st != F.FE_OK and status == F.FE_OK:
                status = st
            for j, i in enumerate(wave):
                infos[i] = inf[j]
                if keep is not None:
                    keep(i, B.x[j][: B.n_rows[j]])
            del B, Bh, rws
            if progress is not None:
                progress(self.waves.index(wave), len(self.waves), tb - ta, tc - tb)
            torch.cuda.empty_cache()
        return dict(status=status, setup_s=t_setup, assemble_s=t_asm, solve_s=t_solve, infos=infos)


def run_sequential(problems, rtol, maxit, keep=None, stream=None, coeffs_hi=None, inner_rtol=1e-4, max_outer=50):
    """The plain path, one problem at a time: fe_assemble then
    fe_pcg_solve_mesh (set-up outside the timed part); with coeffs_hi (the
    FP64 coefficients of every problem) both systems are assembled and the
    problem is solved by fe_refine_solve_mesh on A_lo's values."""
    import torch
    t_asm = t_solve = 0.0
    infos = []
    for i, (mesh, k, coeff) in enumerate(problems):
        A = F.Assembly(mesh, k, coeff)
        A.pattern()
        Ah = None
        if coeffs_hi is not None:
            Ah = F.Assembly(mesh, k, coeffs_hi[i])
            Ah.pattern()
        nws = F.refine_query(A.n_rows) if Ah is not None else F.pcg_query(A.n_rows)
        ws = torch.empty(max(nws, 8), dtype=torch.uint8, device="cuda")
        x = torch.zeros(max(A.n_rows, 1), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        ta = time.perf_counter()
        A.assemble(stream)
        if Ah is not None:
            Ah.assemble(stream)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        if not A.n_rows:
            info = dict(iters=0, status=F.FE_OK)
        elif Ah is not None:
            info = F.refine_solve_mesh(mesh, k, Ah.coeff, Ah.csr, A.csr, Ah.rhs, x, rtol, inner_rtol, max_outer, maxit,
                                       ws, stream=stream)
        else:
            info = A.solve(x, rtol, maxit, ws, stream)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        t_asm += tb - ta
        t_solve += tc - tb
        infos.append(info)
        if keep is not None:
            keep(i, x[: A.n_rows])
        del A, Ah, ws, x
    return dict(assemble_s=t_asm, solve_s=t_solve, infos=infos)
