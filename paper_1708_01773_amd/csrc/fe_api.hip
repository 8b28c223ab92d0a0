// fe_api.hip -- the extern "C" entry points declared in include/fe.h:
// argument validation, the mesh handle and its cached set-up, and the
// dispatch to the kernels of fe_setup / fe_integrate / fe_scatter / fe_solve.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fe_internal.h"

namespace fe {

static thread_local std::string g_last_error;

fe_status set_error(fe_status st, const std::string &msg)
{
    if (st != FE_OK) g_last_error = msg;
    return st;
}

fe_status hip_error(hipError_t e, const char *what)
{
    return set_error(FE_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

static hipStream_t as_stream(fe_stream s) { return reinterpret_cast<hipStream_t>(s); }

// ---------------------------------------------------------------------------
// Kernel timing
// ---------------------------------------------------------------------------
struct PendingTime {
    hipEvent_t a, b;
    TimedKind kind;
};
static std::atomic<bool> g_timing{false};
static std::mutex g_timing_mu;
static std::vector<hipEvent_t> g_event_pool;
static std::vector<PendingTime> g_pending;
static double g_ms[3] = {0, 0, 0};
static int64_t g_calls[3] = {0, 0, 0};

static hipEvent_t pooled_event()
{
    std::lock_guard<std::mutex> lk(g_timing_mu);
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

bool timing_on() { return g_timing.load(); }

hipEvent_t timing_begin(hipStream_t s)
{
    if (!g_timing.load()) return nullptr;
    hipEvent_t e = pooled_event();
    if (e && hipEventRecord(e, s) != hipSuccess) return nullptr;
    return e;
}

hipEvent_t timing_mark(hipStream_t s) { return timing_begin(s); }

void timing_commit(hipEvent_t a, hipEvent_t b, TimedKind kind)
{
    if (!a || !b) return;
    std::lock_guard<std::mutex> lk(g_timing_mu);
    g_pending.push_back({a, b, kind});
}

void timing_release(hipEvent_t e)
{
    if (!e) return;
    (void)hipEventSynchronize(e);
    std::lock_guard<std::mutex> lk(g_timing_mu);
    g_event_pool.push_back(e);
}

void timing_end(hipEvent_t begin, TimedKind kind, hipStream_t s)
{
    if (!begin) return;
    hipEvent_t e = pooled_event();
    if (!e || hipEventRecord(e, s) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_timing_mu);
    g_pending.push_back({begin, e, kind});
}

// Corner Jacobians of the order-1 map: at corner v the columns of J are the
// cell edges leaving that corner.  det J > 0 at every corner is necessary for
// a valid cell; the kernels check every quadrature point as well.
static bool corners_valid(int dim, const int *n, const double *v, int64_t &bad_cell)
{
    const int64_t nx = n[0] + 1, ny = n[1] + 1;
    const int64_t ncells = int64_t(n[0]) * n[1] * (dim == 3 ? n[2] : 1);
    for (int64_t c = 0; c < ncells; c++) {
        const int64_t e0 = c % n[0], e1 = (c / n[0]) % n[1], e2 = dim == 3 ? c / (int64_t(n[0]) * n[1]) : 0;
        auto vid = [&](int vv) {
            return (e0 + (vv & 1)) + nx * ((e1 + ((vv >> 1) & 1)) + ny * (dim == 3 ? e2 + ((vv >> 2) & 1) : 0));
        };
        for (int vv = 0; vv < (1 << dim); vv++) {
            double J[3][3];
            for (int sdir = 0; sdir < dim; sdir++) {
                const int64_t hi = vid(vv | (1 << sdir)), lo = vid(vv & ~(1 << sdir));
                for (int r = 0; r < dim; r++) J[r][sdir] = v[hi * dim + r] - v[lo * dim + r];
            }
            double det;
            if (dim == 2)
                det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
            else
                det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                      J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
            if (!(det > 0.0)) {
                bad_cell = c;
                return false;
            }
        }
    }
    return true;
}

static fe_status check_coeff(const fe_mesh m, int32_t order, const fe_coeff *c)
{
    if (!m) return set_error(FE_EINVAL, "null mesh");
    if (!c) return set_error(FE_EINVAL, "null coeff");
    if (order < 1 || order > kMaxOrder) return set_error(FE_EINVAL, "order must be in 1..4");
    if (c->problem != FE_POISSON && c->problem != FE_ELASTICITY) return set_error(FE_EINVAL, "unknown problem");
    if (c->precision < FE_FP64 || c->precision > FE_BF16) return set_error(FE_EINVAL, "unknown precision");
    if (c->source_kind < FE_SOURCE_NONE || c->source_kind > FE_SOURCE_SINPROD)
        return set_error(FE_EINVAL, "unknown source kind");
    if (c->dirichlet_kind != FE_DIRICHLET_ZERO && c->dirichlet_kind != FE_DIRICHLET_AFFINE)
        return set_error(FE_EINVAL, "unknown dirichlet kind");
    if (c->dirichlet_faces >= (1u << (2 * m->dim))) return set_error(FE_EINVAL, "dirichlet face bit out of range");
    if (c->problem == FE_ELASTICITY) {
        if (!(c->poisson_ratio > -1.0 && c->poisson_ratio < 0.5)) return set_error(FE_EINVAL, "poisson ratio out of range");
        if (!(c->young > 0.0)) return set_error(FE_EINVAL, "young modulus must be positive");
    }
    return FE_OK;
}

static ProblemArgs problem_args(const fe_coeff *c)
{
    ProblemArgs p{};
    p.problem = c->problem;
    p.precision = c->precision;
    if (c->problem == FE_ELASTICITY) {
        const double E = c->young, nu = c->poisson_ratio;
        p.lambda = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
        p.mu = E / (2.0 * (1.0 + nu));
    }
    p.source_kind = c->source_kind;
    for (int i = 0; i < 3; i++) p.source[i] = c->source[i];
    p.dirichlet_kind = c->dirichlet_kind;
    for (int i = 0; i < 12; i++) p.aff[i] = c->dirichlet_affine[i];
    return p;
}

static MeshArgs mesh_args(const fe_mesh m)
{
    MeshArgs a{};
    a.x = m->d_xyz;
    a.y = m->d_xyz + m->nverts;
    a.z = m->dim == 3 ? m->d_xyz + 2 * m->nverts : nullptr;
    a.coef = m->d_coef;
    a.n0 = m->n[0];
    a.n1 = m->n[1];
    a.n2 = m->dim == 3 ? m->n[2] : 1;
    a.status = m->d_status;
    return a;
}

// Builds (or reuses) the cached set-up for (order, problem, faces).
static fe_status ensure_space(fe_mesh m, int32_t order, const fe_coeff *c, hipStream_t s = nullptr)
{
    const int ncomp = c->problem == FE_ELASTICITY ? m->dim : 1;
    Space &sp = m->space;
    if (sp.valid && sp.k == order && sp.ncomp == ncomp && sp.faces == c->dirichlet_faces) return FE_OK;
    return build_space(m, order, ncomp, c->dirichlet_faces, sp, s);
}

fe_status prepare_space(fe_mesh m, int32_t order, const fe_coeff *c, hipStream_t s)
{
    fe_status st = check_coeff(m, order, c);
    if (st != FE_OK) return st;
    return ensure_space(m, order, c, s);
}

static fe_status check_csr(const fe_csr *out, const SpaceArgs &sa, bool need_values)
{
    if (!out) return set_error(FE_EINVAL, "null csr");
    if (out->n_rows != sa.n_rows || out->nnz != sa.nnz)
        return set_error(FE_EINVAL, "csr sizes differ from fe_assemble_query");
    if (need_values && sa.n_rows > 0 && (!out->values || !out->rhs || !out->dinv))
        return set_error(FE_EINVAL, "null csr values/rhs/dinv");
    return FE_OK;
}

}  // namespace fe

using namespace fe;

extern "C" {

const char *fe_last_error(void) { return g_last_error.c_str(); }

int32_t fe_version(void) { return 1; }

fe_status fe_create_mesh(const fe_mesh_desc *desc, fe_mesh *out)
{
    if (!desc || !out) return set_error(FE_EINVAL, "null argument");
    *out = nullptr;
    const int dim = desc->dim;
    if (dim != 2 && dim != 3) return set_error(FE_EINVAL, "dim must be 2 or 3");
    int n[3] = {desc->n[0], desc->n[1], dim == 3 ? desc->n[2] : 1};
    for (int r = 0; r < dim; r++)
        if (n[r] < 1 || n[r] > (1 << 20)) return set_error(FE_EINVAL, "cells per axis must be in 1..2^20");
    const int64_t ncells = int64_t(n[0]) * n[1] * n[2];
    const int64_t nverts = int64_t(n[0] + 1) * (n[1] + 1) * (dim == 3 ? n[2] + 1 : 1);
    std::vector<double> uni;
    const double *v = desc->vertex_xyz;
    if (!v) {
        uni.resize(size_t(nverts) * dim);
        for (int64_t id = 0; id < nverts; id++) {
            const int64_t i = id % (n[0] + 1), j = (id / (n[0] + 1)) % (n[1] + 1), l = id / (int64_t(n[0] + 1) * (n[1] + 1));
            uni[id * dim + 0] = double(i) / n[0];
            uni[id * dim + 1] = double(j) / n[1];
            if (dim == 3) uni[id * dim + 2] = double(l) / n[2];
        }
        v = uni.data();
    }
    int64_t bad = -1;
    if (!corners_valid(dim, n, v, bad))
        return set_error(FE_EMESH, "cell " + std::to_string(bad) + " has det J <= 0 at a corner");
    if (desc->cell_coeff)
        for (int64_t c = 0; c < ncells; c++)
            if (!std::isfinite(desc->cell_coeff[c])) return set_error(FE_EINVAL, "non-finite cell coefficient");
    fe_mesh m = new fe_mesh_s();
    m->dim = dim;
    for (int r = 0; r < 3; r++) m->n[r] = n[r];
    m->ncells = ncells;
    m->nverts = nverts;
    (void)hipGetDevice(&m->device);
    std::vector<double> soa(size_t(nverts) * dim);
    for (int64_t id = 0; id < nverts; id++)
        for (int r = 0; r < dim; r++) soa[size_t(r) * nverts + id] = v[id * dim + r];
    std::vector<double> coef(size_t(ncells), 1.0);
    if (desc->cell_coeff) std::memcpy(coef.data(), desc->cell_coeff, sizeof(double) * ncells);
    hipError_t e = hipMalloc(&m->d_xyz, sizeof(double) * soa.size());
    if (e == hipSuccess) e = hipMalloc(&m->d_coef, sizeof(double) * ncells);
    if (e == hipSuccess) e = hipMalloc(&m->d_status, sizeof(int32_t));
    if (e == hipSuccess) e = hipMemcpy(m->d_xyz, soa.data(), sizeof(double) * soa.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->d_coef, coef.data(), sizeof(double) * ncells, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(m->d_status, 0, sizeof(int32_t));
    if (e != hipSuccess) {
        fe_destroy_mesh(m);
        return e == hipErrorOutOfMemory ? set_error(FE_ENOMEM, "device allocation failed")
                                        : hip_error(e, "fe_create_mesh");
    }
    *out = m;
    return FE_OK;
}

fe_status fe_destroy_mesh(fe_mesh m)
{
    if (!m) return FE_OK;
    (void)hipDeviceSynchronize();
    free_space(m->space);
    if (m->d_xyz) (void)hipFree(m->d_xyz);
    if (m->d_coef) (void)hipFree(m->d_coef);
    if (m->d_status) (void)hipFree(m->d_status);
    delete m;
    return FE_OK;
}

fe_status fe_set_coefficients(fe_mesh m, const double *cell_coeff)
{
    if (!m || !cell_coeff) return set_error(FE_EINVAL, "null argument");
    for (int64_t c = 0; c < m->ncells; c++)
        if (!std::isfinite(cell_coeff[c])) return set_error(FE_EINVAL, "non-finite cell coefficient");
    FE_HIP(hipDeviceSynchronize());
    FE_HIP(hipMemcpy(m->d_coef, cell_coeff, sizeof(double) * m->ncells, hipMemcpyHostToDevice));
    return FE_OK;
}

fe_status fe_assemble_query(fe_mesh m, int32_t order, const fe_coeff *c, int64_t *n_rows, int64_t *nnz,
                            size_t *ws_bytes)
{
    fe_status st = check_coeff(m, order, c);
    if (st != FE_OK) return st;
    st = ensure_space(m, order, c);
    if (st != FE_OK) return st;
    const SpaceArgs &sa = m->space.args;
    if (n_rows) *n_rows = sa.n_rows;
    if (nnz) *nnz = sa.nnz;
    if (ws_bytes) *ws_bytes = elem_layout(sa, c->precision).total;
    return FE_OK;
}

fe_status fe_element_layout(fe_mesh m, int32_t order, const fe_coeff *c, int32_t *nloc, int32_t *cell_block,
                            int32_t *elem_bytes, size_t *load_offset, int32_t *packed)
{
    fe_status st = check_coeff(m, order, c);
    if (st != FE_OK) return st;
    st = ensure_space(m, order, c);
    if (st != FE_OK) return st;
    const ElemLayout el = elem_layout(m->space.args, c->precision);
    if (nloc) *nloc = m->space.args.nloc;
    if (cell_block) *cell_block = el.cb;
    if (elem_bytes) *elem_bytes = el.elem_bytes;
    if (load_offset) *load_offset = el.f_offset;
    if (packed) *packed = el.packed;
    return FE_OK;
}

fe_status fe_pattern(fe_mesh m, int32_t order, const fe_coeff *c, fe_csr *out, fe_stream stream)
{
    fe_status st = check_coeff(m, order, c);
    if (st != FE_OK) return st;
    st = ensure_space(m, order, c);
    if (st != FE_OK) return st;
    st = check_csr(out, m->space.args, false);
    if (st != FE_OK) return st;
    if (!out->rowptr || (m->space.args.nnz > 0 && !out->colind)) return set_error(FE_EINVAL, "null rowptr/colind");
    m->last_stream = as_stream(stream);
    return launch_pattern(m->space.args, out->rowptr, out->colind, as_stream(stream));
}

fe_status fe_integrate(fe_mesh m, int32_t order, const fe_coeff *c, void *ws, size_t ws_bytes, fe_stream stream)
{
    fe_status st = check_coeff(m, order, c);
    if (st != FE_OK) return st;
    st = ensure_space(m, order, c);
    if (st != FE_OK) return st;
    const SpaceArgs &sa = m->space.args;
    const ElemLayout el = elem_layout(sa, c->precision);
    if (!ws || ws_bytes < el.total) return set_error(FE_EINVAL, "workspace too small (see fe_assemble_query)");
    RefTables rt;
    ref_tables(order, rt);
    const ProblemArgs pa = problem_args(c);
    const MeshArgs ma = mesh_args(m);
    m->last_stream = as_stream(stream);
    hipEvent_t t0 = timing_begin(as_stream(stream));
    st = launch_integrate(sa, ma, pa, rt, el, ws, as_stream(stream));
    if (st == FE_OK) st = launch_lift(sa, ma, pa, m->space.d_cell_dofs, el, ws, as_stream(stream));
    timing_end(t0, kTimeIntegrate, as_stream(stream));
    return st;
}

fe_status fe_integrate_autotune(fe_mesh m, int32_t order, const fe_coeff *c, void *ws, size_t ws_bytes, int32_t reps,
                                fe_k3_plan *tried, int32_t max_tried, int32_t *n_tried, fe_k3_plan *chosen,
                                fe_stream stream)
{
    if (reps < 1 || max_tried < 0 || (max_tried > 0 && !tried)) return set_error(FE_EINVAL, "bad reps/max_tried");
    fe_status st = check_coeff(m, order, c);
    if (st != FE_OK) return st;
    st = ensure_space(m, order, c);
    if (st != FE_OK) return st;
    const SpaceArgs &sa = m->space.args;
    if (sa.dim != 3 || order < 2) return set_error(FE_EINVAL, "no tile shapes to tune for this space");
    const ElemLayout el = elem_layout(sa, c->precision);
    if (!ws || ws_bytes < el.total) return set_error(FE_EINVAL, "workspace too small (see fe_assemble_query)");
    RefTables rt;
    ref_tables(order, rt);
    m->last_stream = as_stream(stream);
    int nt = 0;
    st = integrate_autotune(sa, mesh_args(m), problem_args(c), rt, ws,
                            reinterpret_cast<double *>(static_cast<char *>(ws) + el.f_offset), reps, tried, max_tried,
                            &nt, chosen, as_stream(stream));
    if (n_tried) *n_tried = nt;
    return st;
}

fe_status fe_integrate_plan_of(fe_mesh m, int32_t order, const fe_coeff *c, fe_k3_plan *plan)
{
    if (!plan) return set_error(FE_EINVAL, "null plan");
    fe_status st = check_coeff(m, order, c);
    if (st != FE_OK) return st;
    st = ensure_space(m, order, c);
    if (st != FE_OK) return st;
    integrate_plan_of(m->space.args, problem_args(c), plan);
    return FE_OK;
}

fe_status fe_scatter(fe_mesh m, int32_t order, const fe_coeff *c, fe_csr *out, const void *ws, size_t ws_bytes,
                     fe_stream stream)
{
    fe_status st = check_coeff(m, order, c);
    if (st != FE_OK) return st;
    st = ensure_space(m, order, c);
    if (st != FE_OK) return st;
    const SpaceArgs &sa = m->space.args;
    st = check_csr(out, sa, true);
    if (st != FE_OK) return st;
    const ElemLayout el = elem_layout(sa, c->precision);
    if (!ws || ws_bytes < el.total) return set_error(FE_EINVAL, "workspace too small (see fe_assemble_query)");
    m->last_stream = as_stream(stream);
    hipEvent_t t0 = timing_begin(as_stream(stream));
    st = launch_scatter(sa, el, ws, out->values, out->rhs, out->dinv, as_stream(stream));
    timing_end(t0, kTimeScatter, as_stream(stream));
    return st;
}

fe_status fe_assemble(fe_mesh m, int32_t order, const fe_coeff *c, fe_csr *out, void *ws, size_t ws_bytes,
                      fe_stream stream)
{
    fe_status st = fe_integrate(m, order, c, ws, ws_bytes, stream);
    if (st != FE_OK) return st;
    return fe_scatter(m, order, c, out, ws, ws_bytes, stream);
}

// ---------------------------------------------------------------------------
// Batched assembly: problems grouped by kernel class, one launch per class
// ---------------------------------------------------------------------------
}  // extern "C"

namespace fe {

struct BatchLayout {
    size_t table, boff, total;
    std::vector<size_t> ws_off;
    std::vector<ElemLayout> el;
};

static fe_status batch_prepare(int32_t nprob, const fe_mesh *meshes, const int32_t *orders, const fe_coeff *coeffs,
                               BatchLayout &L)
{
    if (nprob < 0) return set_error(FE_EINVAL, "negative nprob");
    if (nprob > 0 && (!meshes || !orders || !coeffs)) return set_error(FE_EINVAL, "null argument");
    for (int i = 0; i < nprob; i++) {
        fe_status st = check_coeff(meshes[i], orders[i], &coeffs[i]);
        if (st != FE_OK) return st;
    }
    // a mesh may appear more than once only with the same space
    for (int i = 0; i < nprob; i++)
        for (int j = 0; j < i; j++)
            if (meshes[i] == meshes[j]) {
                const int nci = coeffs[i].problem == FE_ELASTICITY ? meshes[i]->dim : 1;
                const int ncj = coeffs[j].problem == FE_ELASTICITY ? meshes[j]->dim : 1;
                if (orders[i] != orders[j] || nci != ncj || coeffs[i].dirichlet_faces != coeffs[j].dirichlet_faces)
                    return set_error(FE_EINVAL, "a mesh repeated in a batch needs the same order, problem and faces");
            }
    L.el.resize(nprob);
    L.ws_off.resize(nprob);
    L.table = 0;
    L.boff = align256(sizeof(AsmJob) * 2 * size_t(std::max(nprob, 1)));
    size_t off = L.boff + align256(sizeof(int32_t) * (4 * size_t(nprob) + 16));
    for (int i = 0; i < nprob; i++) {
        fe_status st = ensure_space(meshes[i], orders[i], &coeffs[i]);
        if (st != FE_OK) return st;
        L.el[i] = elem_layout(meshes[i]->space.args, coeffs[i].precision);
        L.ws_off[i] = off;
        off += align256(L.el[i].total);
    }
    L.total = off;
    return FE_OK;
}

}  // namespace fe

extern "C" {

fe_status fe_assemble_batch_query(int32_t nprob, const fe_mesh *meshes, const int32_t *orders,
                                  const fe_coeff *coeffs, int64_t *n_rows, int64_t *nnz, size_t *ws_bytes)
{
    BatchLayout L;
    fe_status st = batch_prepare(nprob, meshes, orders, coeffs, L);
    if (st != FE_OK) return st;
    for (int i = 0; i < nprob; i++) {
        if (n_rows) n_rows[i] = meshes[i]->space.args.n_rows;
        if (nnz) nnz[i] = meshes[i]->space.args.nnz;
    }
    if (ws_bytes) *ws_bytes = L.total;
    return FE_OK;
}

fe_status fe_assemble_batch(int32_t nprob, const fe_mesh *meshes, const int32_t *orders, const fe_coeff *coeffs,
                            fe_csr *out, void *ws, size_t ws_bytes, fe_stream stream)
{
    BatchLayout L;
    fe_status st = batch_prepare(nprob, meshes, orders, coeffs, L);
    if (st != FE_OK) return st;
    if (nprob == 0) return FE_OK;
    if (!out) return set_error(FE_EINVAL, "null csr array");
    if (!ws || ws_bytes < L.total) return set_error(FE_EINVAL, "workspace too small (see fe_assemble_batch_query)");
    for (int i = 0; i < nprob; i++) {
        st = check_csr(&out[i], meshes[i]->space.args, true);
        if (st != FE_OK) return st;
    }
    hipStream_t s = as_stream(stream);
    char *base = static_cast<char *>(ws);
    std::vector<AsmJob> jobs(nprob);
    for (int i = 0; i < nprob; i++) {
        AsmJob &J = jobs[i];
        fe_mesh m = meshes[i];
        m->last_stream = s;
        J.s = m->space.args;
        J.m = mesh_args(m);
        J.p = problem_args(&coeffs[i]);
        ref_tables(orders[i], J.rt);
        J.E = base + L.ws_off[i];
        J.F = reinterpret_cast<double *>(base + L.ws_off[i] + L.el[i].f_offset);
        J.values = out[i].values;
        J.rhs = out[i].rhs;
        J.dinv = out[i].dinv;
        J.parts = 1;
    }
    // classes: integration by (dim, order, components, precision) for the
    // batchable kernels; scatter by (element layout, components)
    std::vector<int> iorder, sorder, single;
    for (int i = 0; i < nprob; i++) {
        if (jobs[i].s.ncells == 0) continue;
        if (integrate_batchable(jobs[i].s, jobs[i].p)) iorder.push_back(i);
        else single.push_back(i);
    }
    auto ikey = [&](int i) {
        const AsmJob &J = jobs[i];
        return ((J.s.dim * 8 + J.s.k) * 4 + J.s.ncomp) * 4 + J.p.precision;
    };
    auto skey = [&](int i) {
        return (L.el[i].cb > 1 ? 1000 : 0) + jobs[i].s.dim * 100 + L.el[i].elem_bytes * 10 + jobs[i].s.ncomp;
    };
    std::stable_sort(iorder.begin(), iorder.end(), [&](int a, int b) { return ikey(a) < ikey(b); });
    for (int i = 0; i < nprob; i++)
        if (jobs[i].s.n_rows > 0) sorder.push_back(i);
    std::stable_sort(sorder.begin(), sorder.end(), [&](int a, int b) { return skey(a) < skey(b); });
    // device table in the order: integration classes, then scatter classes
    struct Launch {
        int first, count, grid;
        size_t boff_pos;
        int job0;  // host job index of the class
    };
    std::vector<AsmJob> table;
    std::vector<int32_t> boff;
    std::vector<Launch> il, sl;
    auto build = [&](const std::vector<int> &ord, auto key, bool integ, std::vector<Launch> &ls) -> fe_status {
        size_t t = 0;
        while (t < ord.size()) {
            size_t u = t;
            while (u < ord.size() && key(ord[u]) == key(ord[t])) u++;
            Launch l{int(table.size()), int(u - t), 0, boff.size(), ord[t]};
            int64_t acc = 0;
            for (size_t v = t; v < u; v++) {
                AsmJob J = jobs[ord[v]];
                int32_t parts = 1;
                const int64_t nb = integ ? integrate_blocks(J.s, J.p, parts) : scatter_blocks(J.s, L.el[ord[v]]);
                J.parts = parts;
                boff.push_back(int32_t(acc));
                acc += nb;
                if (acc > int64_t(INT32_MAX)) return set_error(FE_EINVAL, "batch class exceeds 2^31 workgroups");
                table.push_back(J);
            }
            boff.push_back(int32_t(acc));
            l.grid = int(acc);
            ls.push_back(l);
            t = u;
        }
        return FE_OK;
    };
    st = build(iorder, ikey, true, il);
    if (st != FE_OK) return st;
    st = build(sorder, skey, false, sl);
    if (st != FE_OK) return st;
    if (sizeof(int32_t) * boff.size() > align256(sizeof(int32_t) * (4 * size_t(nprob) + 16)) ||
        table.size() > size_t(2 * nprob))
        return set_error(FE_EINVAL, "internal batch table overflow");
    AsmJob *d_table = reinterpret_cast<AsmJob *>(base + L.table);
    int32_t *d_boff = reinterpret_cast<int32_t *>(base + L.boff);
    if (!table.empty()) {
        FE_HIP(hipMemcpyAsync(d_table, table.data(), sizeof(AsmJob) * table.size(), hipMemcpyHostToDevice, s));
        FE_HIP(hipMemcpyAsync(d_boff, boff.data(), sizeof(int32_t) * boff.size(), hipMemcpyHostToDevice, s));
        // the host vectors go away on return: wait for the staged copies
        FE_HIP(hipStreamSynchronize(s));
    }
    hipEvent_t t0 = timing_begin(s);
    for (const Launch &l : il) {
        st = launch_integrate_batch(jobs[l.job0], d_table + l.first, d_boff + l.boff_pos, l.count, l.grid, s);
        if (st != FE_OK) return st;
    }
    for (int i : single) {
        st = launch_integrate(jobs[i].s, jobs[i].m, jobs[i].p, jobs[i].rt, L.el[i], jobs[i].E, s);
        if (st != FE_OK) return st;
    }
    for (int i = 0; i < nprob; i++) {
        st = launch_lift(jobs[i].s, jobs[i].m, jobs[i].p, meshes[i]->space.d_cell_dofs, L.el[i], jobs[i].E, s);
        if (st != FE_OK) return st;
    }
    timing_end(t0, kTimeIntegrate, s);
    t0 = timing_begin(s);
    for (const Launch &l : sl) {
        st = launch_scatter_batch(jobs[l.job0], L.el[l.job0], d_table + l.first, d_boff + l.boff_pos, l.count,
                                  l.grid, s);
        if (st != FE_OK) return st;
    }
    timing_end(t0, kTimeScatter, s);
    return FE_OK;
}

// ---------------------------------------------------------------------------
// Interior-penalty discontinuous Galerkin (fe_dg.hip)
// ---------------------------------------------------------------------------
static fe_status dg_check(fe_mesh m, int32_t order, int64_t &n_rows, int64_t &nnz)
{
    if (!m) return set_error(FE_EINVAL, "null mesh");
    if (order < 1 || order > kMaxOrder) return set_error(FE_EINVAL, "order must be in 1..4");
    dg_sizes(m->dim, m->n, order, n_rows, nnz);
    if (n_rows >= (int64_t(1) << 31)) return set_error(FE_EINVAL, "too many rows for int32 column indices");
    return FE_OK;
}

fe_status fe_dg_query(fe_mesh m, int32_t order, int64_t *n_rows, int64_t *nnz, size_t *ws_bytes)
{
    int64_t nr, nz;
    fe_status st = dg_check(m, order, nr, nz);
    if (st != FE_OK) return st;
    if (n_rows) *n_rows = nr;
    if (nnz) *nnz = nz;
    if (ws_bytes) *ws_bytes = elem_layout(dg_space(m->dim, m->n, order), FE_FP64).total;
    return FE_OK;
}

fe_status fe_dg_pattern(fe_mesh m, int32_t order, fe_csr *out, fe_stream stream)
{
    int64_t nr, nz;
    fe_status st = dg_check(m, order, nr, nz);
    if (st != FE_OK) return st;
    if (!out) return set_error(FE_EINVAL, "null csr");
    if (out->n_rows != nr || out->nnz != nz) return set_error(FE_EINVAL, "csr sizes differ from fe_dg_query");
    if (!out->rowptr || !out->colind) return set_error(FE_EINVAL, "null rowptr/colind");
    m->last_stream = as_stream(stream);
    return launch_dg_pattern(m->dim, m->n, order, out->rowptr, out->colind, as_stream(stream));
}

fe_status fe_dg_assemble(fe_mesh m, int32_t order, const fe_coeff *c, double gamma, double tau, fe_csr *out,
                         void *ws, size_t ws_bytes, fe_stream stream)
{
    int64_t nr, nz;
    fe_status st = dg_check(m, order, nr, nz);
    if (st != FE_OK) return st;
    if (!c) return set_error(FE_EINVAL, "null coeff");
    if (c->problem != FE_POISSON) return set_error(FE_EINVAL, "the DG form is built for the Poisson problem only");
    if (c->precision != FE_FP64) return set_error(FE_EINVAL, "the DG form is assembled in FP64 only");
    if (c->source_kind < FE_SOURCE_NONE || c->source_kind > FE_SOURCE_SINPROD)
        return set_error(FE_EINVAL, "unknown source kind");
    if (c->dirichlet_kind != FE_DIRICHLET_ZERO && c->dirichlet_kind != FE_DIRICHLET_AFFINE)
        return set_error(FE_EINVAL, "unknown dirichlet kind");
    if (c->dirichlet_faces != (1u << (2 * m->dim)) - 1u)
        return set_error(FE_EINVAL, "the DG form imposes Dirichlet data weakly on every boundary face");
    if (!(gamma > 0.0) || !std::isfinite(gamma) || !std::isfinite(tau))
        return set_error(FE_EINVAL, "gamma must be positive and finite, tau finite");
    if (!out) return set_error(FE_EINVAL, "null csr");
    if (out->n_rows != nr || out->nnz != nz) return set_error(FE_EINVAL, "csr sizes differ from fe_dg_query");
    if (!out->rowptr || !out->colind || !out->values || !out->rhs || !out->dinv)
        return set_error(FE_EINVAL, "null csr array");
    const SpaceArgs sa = dg_space(m->dim, m->n, order);
    const ElemLayout el = elem_layout(sa, FE_FP64);
    if (!ws || ws_bytes < el.total) return set_error(FE_EINVAL, "workspace too small (see fe_dg_query)");
    RefTables rt;
    ref_tables(order, rt);
    ProblemArgs pa = problem_args(c);
    MeshArgs ma = mesh_args(m);
    ma.coef = nullptr;  // coefficient 1 in the volume term
    hipStream_t s = as_stream(stream);
    m->last_stream = s;
    hipEvent_t t0 = timing_begin(s);
    st = launch_integrate(sa, ma, pa, rt, el, ws, s);
    timing_end(t0, kTimeIntegrate, s);
    if (st != FE_OK) return st;
    hipEvent_t t1 = timing_begin(s);
    st = launch_dg_facets(m->dim, m->n, order, gamma, tau, ma, pa, el, ws, out->rowptr, out->values, out->rhs,
                          out->dinv, s);
    timing_end(t1, kTimeScatter, s);
    return st;
}

fe_status fe_dg_spmv(fe_mesh m, int32_t order, const fe_csr *A, const double *x, double *y, fe_stream stream)
{
    int64_t nr, nz;
    fe_status st = dg_check(m, order, nr, nz);
    if (st != FE_OK) return st;
    if (!A || !x || !y) return set_error(FE_EINVAL, "null argument");
    if (A->n_rows != nr || A->nnz != nz) return set_error(FE_EINVAL, "csr sizes differ from fe_dg_query");
    if (nz > 0 && !A->values) return set_error(FE_EINVAL, "null csr values");
    if (reinterpret_cast<uintptr_t>(A->values) & 15u) return set_error(FE_EINVAL, "csr values not 16-byte aligned");
    m->last_stream = as_stream(stream);
    return launch_spmv_dg(dg_space(m->dim, m->n, order), A->values, x, y, as_stream(stream));
}

fe_status fe_dg_pcg_solve(fe_mesh m, int32_t order, const fe_csr *A, const double *b, double *x, double rtol,
                          int32_t maxit, void *ws, size_t ws_bytes, fe_solve_info *info, fe_stream stream)
{
    int64_t nr, nz;
    fe_status st = dg_check(m, order, nr, nz);
    if (st != FE_OK) return st;
    if (!A || !b || !x || !ws || !info) return set_error(FE_EINVAL, "null argument");
    if (A->n_rows != nr || A->nnz != nz) return set_error(FE_EINVAL, "csr sizes differ from fe_dg_query");
    if (nr > 0 && (!A->values || !A->dinv)) return set_error(FE_EINVAL, "null csr values/dinv");
    if (reinterpret_cast<uintptr_t>(A->values) & 15u) return set_error(FE_EINVAL, "csr values not 16-byte aligned");
    if (!(rtol >= 0.0) || maxit < 0) return set_error(FE_EINVAL, "bad rtol/maxit");
    m->last_stream = as_stream(stream);
    const SpaceArgs sa = dg_space(m->dim, m->n, order);
    return pcg_solve_dg(A, sa, b, x, rtol, maxit, ws, ws_bytes, info, as_stream(stream));
}

fe_status fe_cell_dofs(fe_mesh m, int32_t order, const fe_coeff *c, int32_t *out, fe_stream stream)
{
    fe_status st = check_coeff(m, order, c);
    if (st != FE_OK) return st;
    st = ensure_space(m, order, c);
    if (st != FE_OK) return st;
    if (!out) return set_error(FE_EINVAL, "null output");
    const SpaceArgs &sa = m->space.args;
    FE_HIP(hipMemcpyAsync(out, m->space.d_cell_dofs, sizeof(int32_t) * size_t(sa.ncells) * sa.nloc,
                          hipMemcpyDeviceToDevice, as_stream(stream)));
    return FE_OK;
}

fe_status fe_permutation(fe_mesh m, int32_t order, const fe_coeff *c, int64_t *perm, fe_stream stream)
{
    fe_status st = check_coeff(m, order, c);
    if (st != FE_OK) return st;
    st = ensure_space(m, order, c);
    if (st != FE_OK) return st;
    if (!perm) return set_error(FE_EINVAL, "null output");
    return launch_permutation(m->space.args, mesh_args(m), perm, as_stream(stream));
}

fe_status fe_get_status(fe_mesh m)
{
    if (!m) return set_error(FE_EINVAL, "null mesh");
    FE_HIP(hipStreamSynchronize(m->last_stream));
    int32_t h = 0;
    FE_HIP(hipMemcpy(&h, m->d_status, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (h) {
        FE_HIP(hipMemset(m->d_status, 0, sizeof(int32_t)));
        return set_error(FE_EMESH, "det J <= 0 at a quadrature point");
    }
    return FE_OK;
}

fe_status fe_pcg_query(int64_t n_rows, size_t *ws_bytes)
{
    if (n_rows < 0 || !ws_bytes) return set_error(FE_EINVAL, "bad argument");
    *ws_bytes = pcg_solve_ws_bytes(n_rows);
    return FE_OK;
}

fe_status fe_pcg_solve(const fe_csr *A, const double *b, double *x, double rtol, int32_t maxit, void *ws,
                       size_t ws_bytes, fe_solve_info *info, fe_stream stream)
{
    if (!A || !b || !x || !ws || !info) return set_error(FE_EINVAL, "null argument");
    if (!A->rowptr || !A->colind || !A->values || !A->dinv) return set_error(FE_EINVAL, "incomplete csr");
    if (!(rtol >= 0.0) || maxit < 0) return set_error(FE_EINVAL, "bad rtol/maxit");
    return pcg_solve(A, b, x, rtol, maxit, ws, ws_bytes, info, as_stream(stream));
}

fe_status fe_pcg_solve_noalloc(const fe_csr *A, const double *b, double *x, double rtol, int32_t maxit,
                               fe_solve_info *info, fe_stream stream)
{
    static_assert(FE_PCG_NOALLOC_BYTES == (64u << 20), "header and library disagree on the scratch size");
    if (!A || !b || !x || !info) return set_error(FE_EINVAL, "null argument");
    if (!A->rowptr || !A->colind || !A->values || !A->dinv) return set_error(FE_EINVAL, "incomplete csr");
    if (!(rtol >= 0.0) || maxit < 0) return set_error(FE_EINVAL, "bad rtol/maxit");
    if (A->n_rows < 0 || A->nnz < 0) return set_error(FE_EINVAL, "negative size");
    if (A->n_rows > FE_PCG_NOALLOC_MAX_ROWS)
        return set_error(FE_EINVAL, "system too large for the allocation-free solve (at most 2,700,000 rows)");
    return pcg_solve_noalloc(A, b, x, rtol, maxit, info, as_stream(stream));
}

fe_status fe_pcg_batch_query(int32_t nprob, const int64_t *n_rows, size_t *ws_bytes)
{
    if (nprob < 0 || (nprob > 0 && !n_rows) || !ws_bytes) return set_error(FE_EINVAL, "bad argument");
    for (int i = 0; i < nprob; i++)
        if (n_rows[i] < 0) return set_error(FE_EINVAL, "negative n_rows");
    *ws_bytes = pcg_batch_ws_bytes(nprob, n_rows);
    return FE_OK;
}

fe_status fe_pcg_solve_batch(int32_t nprob, const fe_csr *A, const double *const *b, double *const *x, double rtol,
                             int32_t maxit, void *ws, size_t ws_bytes, fe_solve_info *infos, fe_stream stream)
{
    if (nprob < 0) return set_error(FE_EINVAL, "negative nprob");
    if (nprob == 0) return FE_OK;
    if (!A || !b || !x || !ws || !infos) return set_error(FE_EINVAL, "null argument");
    if (!(rtol >= 0.0) || maxit < 0) return set_error(FE_EINVAL, "bad rtol/maxit");
    for (int i = 0; i < nprob; i++) {
        if (A[i].n_rows < 0 || A[i].nnz < 0) return set_error(FE_EINVAL, "negative size");
        if (A[i].n_rows > 0 && (!A[i].rowptr || !A[i].colind || !A[i].values || !A[i].dinv || !b[i] || !x[i]))
            return set_error(FE_EINVAL, "incomplete csr or null vector");
    }
    return pcg_solve_batch(nprob, A, b, x, rtol, maxit, ws, ws_bytes, infos, as_stream(stream));
}

fe_status fe_spmv_autotune_query(int64_t n_rows, size_t *ws_bytes)
{
    if (n_rows < 0 || !ws_bytes) return set_error(FE_EINVAL, "bad argument");
    *ws_bytes = autotune_ws_bytes(n_rows);
    return FE_OK;
}

fe_status fe_spmv_autotune(const fe_csr *A, int32_t reps, void *ws, size_t ws_bytes, fe_spmv_plan *tried,
                           int32_t max_tried, int32_t *n_tried, fe_spmv_plan *chosen, fe_stream stream)
{
    if (!A || !ws || !A->rowptr || !A->colind || !A->values) return set_error(FE_EINVAL, "null argument");
    if (reps < 1 || max_tried < 0 || (max_tried > 0 && !tried)) return set_error(FE_EINVAL, "bad reps/max_tried");
    int nt = 0;
    const fe_status st = spmv_autotune(A, reps, ws, ws_bytes, tried, max_tried, &nt, chosen, as_stream(stream));
    if (n_tried) *n_tried = nt;
    return st;
}

fe_status fe_spmv_autotune_mesh(fe_mesh m, int32_t order, const fe_coeff *c, const fe_csr *A, int32_t reps, void *ws,
                                size_t ws_bytes, fe_spmv_plan *tried, int32_t max_tried, int32_t *n_tried,
                                fe_spmv_plan *chosen, fe_stream stream)
{
    if (!A || !ws) return set_error(FE_EINVAL, "null argument");
    if (reps < 1 || max_tried < 0 || (max_tried > 0 && !tried)) return set_error(FE_EINVAL, "bad reps/max_tried");
    fe_status st = prepare_space(m, order, c, nullptr);
    if (st != FE_OK) return st;
    st = check_csr(A, m->space.args, false);
    if (st != FE_OK) return st;
    if (A->nnz > 0 && !A->values) return set_error(FE_EINVAL, "null csr values");
    m->last_stream = as_stream(stream);
    int nt = 0;
    st = spmv_autotune_struct(m->space.args, A->values, reps, ws, ws_bytes, tried, max_tried, &nt, chosen,
                              as_stream(stream));
    if (n_tried) *n_tried = nt;
    return st;
}

fe_status fe_spmv_plan_of_mesh(fe_mesh m, int32_t order, const fe_coeff *c, fe_spmv_plan *plan, int32_t *row_class)
{
    fe_status st = prepare_space(m, order, c, nullptr);
    if (st != FE_OK) return st;
    spmv_plan_of_struct(m->space.args, plan, row_class);
    return FE_OK;
}

fe_status fe_spmv_plan_set_mesh(fe_mesh m, int32_t order, const fe_coeff *c, const fe_spmv_plan *plan)
{
    if (!plan) return set_error(FE_EINVAL, "null plan");
    fe_status st = prepare_space(m, order, c, nullptr);
    if (st != FE_OK) return st;
    return spmv_plan_set_struct(m->space.args, *plan);
}

fe_status fe_spmv_tuning_reset(void)
{
    spmv_tuning_reset();
    integrate_tuning_reset();
    return FE_OK;
}

fe_status fe_spmv_plan_of(int64_t n_rows, int64_t nnz, fe_spmv_plan *plan, int32_t *row_class)
{
    if (n_rows < 0 || nnz < 0) return set_error(FE_EINVAL, "negative size");
    spmv_plan_of(n_rows, nnz, plan, row_class);
    return FE_OK;
}

fe_status fe_spmv_plan_set(int64_t n_rows, int64_t nnz, const fe_spmv_plan *plan)
{
    if (!plan) return set_error(FE_EINVAL, "null plan");
    if (n_rows < 0 || nnz < 0) return set_error(FE_EINVAL, "negative size");
    return spmv_plan_set(n_rows, nnz, *plan);
}

fe_status fe_pcg_solve_mesh(fe_mesh m, int32_t order, const fe_coeff *c, const fe_csr *A, const double *b, double *x,
                            double rtol, int32_t maxit, void *ws, size_t ws_bytes, fe_solve_info *info,
                            fe_stream stream)
{
    if (!A || !b || !x || !ws || !info) return set_error(FE_EINVAL, "null argument");
    fe_status st = prepare_space(m, order, c, nullptr);
    if (st != FE_OK) return st;
    st = check_csr(A, m->space.args, true);
    if (st != FE_OK) return st;
    if (!(rtol >= 0.0) || maxit < 0) return set_error(FE_EINVAL, "bad rtol/maxit");
    m->last_stream = as_stream(stream);
    return pcg_solve_mesh(A, m->space.args, b, x, rtol, maxit, ws, ws_bytes, info, as_stream(stream));
}

fe_status fe_spmv_mesh(fe_mesh m, int32_t order, const fe_coeff *c, const fe_csr *A, const double *x, double *y,
                       fe_stream stream)
{
    if (!A || !x || !y) return set_error(FE_EINVAL, "null argument");
    fe_status st = prepare_space(m, order, c, nullptr);
    if (st != FE_OK) return st;
    st = check_csr(A, m->space.args, false);
    if (st != FE_OK) return st;
    if (A->nnz > 0 && !A->values) return set_error(FE_EINVAL, "null csr values");
    m->last_stream = as_stream(stream);
    return launch_spmv_struct(m->space.args, A->values, x, y, as_stream(stream));
}

fe_status fe_sym_query(fe_mesh m, int32_t order, const fe_coeff *c, size_t *bytes)
{
    if (!bytes) return set_error(FE_EINVAL, "null argument");
    *bytes = 0;
    fe_status st = prepare_space(m, order, c, nullptr);
    if (st != FE_OK) return st;
    if (!sym_supported(m->space.args)) return set_error(FE_EINVAL, "symmetric storage needs a Q1 scalar space");
    *bytes = sym_bytes(m->space.args);
    return FE_OK;
}

// The symmetric-storage calls share their checks: a Q1 scalar space, a buffer
// of fe_sym_query's size (FP64 slots), aligned to its element size.
static fe_status check_sym(fe_mesh m, int32_t order, const fe_coeff *c, const void *sym, size_t sym_bytes_given,
                           size_t elem = sizeof(double))
{
    fe_status st = prepare_space(m, order, c, nullptr);
    if (st != FE_OK) return st;
    const SpaceArgs &sa = m->space.args;
    if (!sym_supported(sa)) return set_error(FE_EINVAL, "symmetric storage needs a Q1 scalar space");
    if (sym_bytes_given < sym_bytes(sa)) return set_error(FE_EINVAL, "symmetric storage buffer too small");
    if (sa.n_rows > 0 && !sym) return set_error(FE_EINVAL, "null symmetric storage");
    if (reinterpret_cast<uintptr_t>(sym) & (elem - 1))
        return set_error(FE_EINVAL, elem == 8 ? "symmetric storage not 8-byte aligned" : "symmetric storage not 4-byte aligned");
    return FE_OK;
}

fe_status fe_sym_from_csr(fe_mesh m, int32_t order, const fe_coeff *c, const fe_csr *A, double *sym,
                          size_t sym_bytes_given, fe_stream stream)
{
    if (!A) return set_error(FE_EINVAL, "null argument");
    fe_status st = check_sym(m, order, c, sym, sym_bytes_given);
    if (st != FE_OK) return st;
    st = check_csr(A, m->space.args, false);
    if (st != FE_OK) return st;
    if (A->nnz > 0 && !A->values) return set_error(FE_EINVAL, "null csr values");
    m->last_stream = as_stream(stream);
    return launch_sym_fill(m->space.args, A->values, sym, as_stream(stream));
}

fe_status fe_spmv_sym(fe_mesh m, int32_t order, const fe_coeff *c, const double *sym, size_t sym_bytes_given,
                      const double *x, double *y, fe_stream stream)
{
    fe_status st = check_sym(m, order, c, sym, sym_bytes_given);
    if (st != FE_OK) return st;
    if (m->space.args.n_rows > 0 && (!x || !y)) return set_error(FE_EINVAL, "null argument");
    m->last_stream = as_stream(stream);
    return launch_spmv_sym(m->space.args, sym, x, y, as_stream(stream));
}

fe_status fe_pcg_solve_sym(fe_mesh m, int32_t order, const fe_coeff *c, const fe_csr *A, const double *sym,
                           size_t sym_bytes_given, const double *b, double *x, double rtol, int32_t maxit, void *ws,
                           size_t ws_bytes, fe_solve_info *info, fe_stream stream)
{
    if (!A || !b || !x || !ws || !info) return set_error(FE_EINVAL, "null argument");
    fe_status st = check_sym(m, order, c, sym, sym_bytes_given);
    if (st != FE_OK) return st;
    st = check_csr(A, m->space.args, false);
    if (st != FE_OK) return st;
    if (A->n_rows > 0 && !A->dinv) return set_error(FE_EINVAL, "null csr dinv");
    if (!(rtol >= 0.0) || maxit < 0) return set_error(FE_EINVAL, "bad rtol/maxit");
    m->last_stream = as_stream(stream);
    return pcg_solve_sym(A, m->space.args, sym, b, x, rtol, maxit, ws, ws_bytes, info, as_stream(stream));
}

fe_status fe_pcg_solve_batch_mesh(int32_t nprob, const fe_mesh *meshes, const int32_t *orders, const fe_coeff *coeffs,
                                  const fe_csr *A, const double *const *b, double *const *x, double rtol,
                                  int32_t maxit, void *ws, size_t ws_bytes, fe_solve_info *infos, fe_stream stream)
{
    BatchLayout L;
    fe_status st = batch_prepare(nprob, meshes, orders, coeffs, L);
    if (st != FE_OK) return st;
    if (nprob == 0) return FE_OK;
    if (!A || !b || !x || !ws || !infos) return set_error(FE_EINVAL, "null argument");
    if (!(rtol >= 0.0) || maxit < 0) return set_error(FE_EINVAL, "bad rtol/maxit");
    std::vector<const SpaceArgs *> sas(nprob);
    for (int i = 0; i < nprob; i++) {
        st = check_csr(&A[i], meshes[i]->space.args, true);
        if (st != FE_OK) return st;
        if (A[i].n_rows > 0 && (!b[i] || !x[i])) return set_error(FE_EINVAL, "null vector");
        sas[i] = &meshes[i]->space.args;
        meshes[i]->last_stream = as_stream(stream);
    }
    return pcg_solve_batch(nprob, A, b, x, rtol, maxit, ws, ws_bytes, infos, as_stream(stream), sas.data());
}

fe_status fe_spmv(const fe_csr *A, const double *x, double *y, fe_stream stream)
{
    if (!A || !x || !y || !A->rowptr || !A->colind || !A->values) return set_error(FE_EINVAL, "null argument");
    if (A->n_rows < 0 || A->nnz < 0) return set_error(FE_EINVAL, "negative size");
    return launch_spmv(A->n_rows, A->rowptr, A->colind, A->values, x, y, A->nnz, as_stream(stream));
}

fe_status fe_csr_to_fp32(const fe_csr *A, float *values32, fe_stream stream)
{
    if (!A || !values32 || (A->nnz > 0 && !A->values)) return set_error(FE_EINVAL, "null argument");
    return csr_to_fp32(A, values32, as_stream(stream));
}

fe_status fe_refine_query(int64_t n_rows, size_t *ws_bytes)
{
    if (n_rows < 0 || !ws_bytes) return set_error(FE_EINVAL, "bad argument");
    *ws_bytes = refine_ws_bytes(n_rows);
    return FE_OK;
}

fe_status fe_refine_solve(const fe_csr *A_hi, const fe_csr *A_lo, const float *values32, const double *b, double *x,
                          double rtol, double inner_rtol, int32_t max_outer, int32_t max_inner, void *ws,
                          size_t ws_bytes, fe_refine_info *info, fe_stream stream)
{
    if (!A_hi || !A_lo || !b || !x || !ws || !info) return set_error(FE_EINVAL, "null argument");
    if (!A_hi->rowptr || !A_hi->colind || !A_hi->values || !A_lo->rowptr || !A_lo->colind || !A_lo->dinv ||
        (!values32 && !A_lo->values))
        return set_error(FE_EINVAL, "incomplete csr");
    if (!(rtol >= 0.0) || !(inner_rtol > 0.0) || max_outer < 0 || max_inner < 1)
        return set_error(FE_EINVAL, "bad tolerances or iteration limits");
    return refine_solve(A_hi, A_lo, values32, b, x, rtol, inner_rtol, max_outer, max_inner, ws, ws_bytes, info,
                        as_stream(stream));
}

fe_status fe_refine_solve_mesh(fe_mesh m, int32_t order, const fe_coeff *c, const fe_csr *A_hi, const fe_csr *A_lo,
                               const float *values32, const double *b, double *x, double rtol, double inner_rtol,
                               int32_t max_outer, int32_t max_inner, void *ws, size_t ws_bytes, fe_refine_info *info,
                               fe_stream stream)
{
    if (!A_hi || !A_lo || !b || !x || !ws || !info) return set_error(FE_EINVAL, "null argument");
    fe_status st = prepare_space(m, order, c, nullptr);
    if (st != FE_OK) return st;
    st = check_csr(A_hi, m->space.args, true);
    if (st != FE_OK) return st;
    st = check_csr(A_lo, m->space.args, false);
    if (st != FE_OK) return st;
    if (!A_hi->rowptr || !A_hi->colind || (A_lo->n_rows > 0 && !A_lo->dinv)) return set_error(FE_EINVAL, "incomplete csr");
    if (A_lo->nnz > 0 && !values32 && !A_lo->values) return set_error(FE_EINVAL, "no A_lo values");
    if (values32 && (reinterpret_cast<uintptr_t>(values32) & 3u)) return set_error(FE_EINVAL, "values32 not 4-byte aligned");
    if (!(rtol >= 0.0) || !(inner_rtol > 0.0) || max_outer < 0 || max_inner < 1)
        return set_error(FE_EINVAL, "bad tolerances or iteration limits");
    m->last_stream = as_stream(stream);
    return refine_solve(A_hi, A_lo, values32, b, x, rtol, inner_rtol, max_outer, max_inner, ws, ws_bytes, info,
                        as_stream(stream), &m->space.args, nullptr);
}

fe_status fe_refine_batch_query(int32_t nprob, const int64_t *n_rows, size_t *ws_bytes)
{
    if (nprob < 0 || (nprob > 0 && !n_rows) || !ws_bytes) return set_error(FE_EINVAL, "bad argument");
    for (int i = 0; i < nprob; i++)
        if (n_rows[i] < 0) return set_error(FE_EINVAL, "negative n_rows");
    *ws_bytes = refine_batch_ws_bytes(nprob, n_rows);
    return FE_OK;
}

fe_status fe_refine_solve_batch_mesh(int32_t nprob, const fe_mesh *meshes, const int32_t *orders,
                                     const fe_coeff *coeffs, const fe_csr *A_hi, const fe_csr *A_lo,
                                     const double *const *b, double *const *x, double rtol, double inner_rtol,
                                     int32_t max_outer, int32_t max_inner, void *ws, size_t ws_bytes,
                                     fe_refine_info *infos, fe_stream stream)
{
    BatchLayout L;
    fe_status st = batch_prepare(nprob, meshes, orders, coeffs, L);
    if (st != FE_OK) return st;
    if (nprob == 0) return FE_OK;
    if (!A_hi || !A_lo || !b || !x || !ws || !infos) return set_error(FE_EINVAL, "null argument");
    if (!(rtol >= 0.0) || !(inner_rtol > 0.0) || max_outer < 0 || max_inner < 1)
        return set_error(FE_EINVAL, "bad tolerances or iteration limits");
    std::vector<const SpaceArgs *> sas(nprob);
    for (int i = 0; i < nprob; i++) {
        st = check_csr(&A_hi[i], meshes[i]->space.args, true);
        if (st != FE_OK) return st;
        st = check_csr(&A_lo[i], meshes[i]->space.args, true);
        if (st != FE_OK) return st;
        if (A_hi[i].n_rows > 0 && (!b[i] || !x[i] || !A_hi[i].rowptr || !A_hi[i].colind || !A_hi[i].values))
            return set_error(FE_EINVAL, "null vector or incomplete csr");
        sas[i] = &meshes[i]->space.args;
        meshes[i]->last_stream = as_stream(stream);
    }
    return refine_solve_batch(nprob, A_hi, A_lo, b, x, rtol, inner_rtol, max_outer, max_inner, ws, ws_bytes, infos,
                              as_stream(stream), sas.data());
}

fe_status fe_sym_fp32_from_csr(fe_mesh m, int32_t order, const fe_coeff *c, const fe_csr *A, float *sym32,
                               size_t sym32_bytes, fe_stream stream)
{
    if (!A) return set_error(FE_EINVAL, "null argument");
    fe_status st = check_sym(m, order, c, sym32, 2 * sym32_bytes, sizeof(float));
    if (st != FE_OK) return st;
    st = check_csr(A, m->space.args, false);
    if (st != FE_OK) return st;
    if (A->nnz > 0 && !A->values) return set_error(FE_EINVAL, "null csr values");
    m->last_stream = as_stream(stream);
    return launch_sym_fill_fp32(m->space.args, A->values, sym32, as_stream(stream));
}

fe_status fe_refine_solve_sym(fe_mesh m, int32_t order, const fe_coeff *c, const fe_csr *A_hi, const fe_csr *A_lo,
                              const float *sym32, size_t sym32_bytes, const double *b, double *x, double rtol,
                              double inner_rtol, int32_t max_outer, int32_t max_inner, void *ws, size_t ws_bytes,
                              fe_refine_info *info, fe_stream stream)
{
    if (!A_hi || !A_lo || !b || !x || !ws || !info) return set_error(FE_EINVAL, "null argument");
    fe_status st = check_sym(m, order, c, sym32, 2 * sym32_bytes, sizeof(float));
    if (st != FE_OK) return st;
    st = check_csr(A_hi, m->space.args, true);
    if (st != FE_OK) return st;
    st = check_csr(A_lo, m->space.args, false);
    if (st != FE_OK) return st;
    if (!A_hi->rowptr || !A_hi->colind || (A_lo->n_rows > 0 && !A_lo->dinv)) return set_error(FE_EINVAL, "incomplete csr");
    if (!(rtol >= 0.0) || !(inner_rtol > 0.0) || max_outer < 0 || max_inner < 1)
        return set_error(FE_EINVAL, "bad tolerances or iteration limits");
    m->last_stream = as_stream(stream);
    return refine_solve(A_hi, A_lo, nullptr, b, x, rtol, inner_rtol, max_outer, max_inner, ws, ws_bytes, info,
                        as_stream(stream), &m->space.args, sym32);
}

fe_status fe_set_timing(int32_t enable)
{
    g_timing.store(enable != 0);
    return FE_OK;
}

fe_status fe_get_timing(fe_timing *out, int32_t reset)
{
    std::vector<PendingTime> pend;
    {
        std::lock_guard<std::mutex> lk(g_timing_mu);
        pend.swap(g_pending);
    }
    fe_status st = FE_OK;
    for (const PendingTime &p : pend) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(p.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.a, p.b);
        if (e != hipSuccess) st = hip_error(e, "fe_get_timing");
        std::lock_guard<std::mutex> lk(g_timing_mu);
        g_ms[p.kind] += ms;
        g_calls[p.kind] += 1;
        g_event_pool.push_back(p.a);
        g_event_pool.push_back(p.b);
    }
    std::lock_guard<std::mutex> lk(g_timing_mu);
    if (out) {
        out->integrate_ms = g_ms[0];
        out->scatter_ms = g_ms[1];
        out->spmv_ms = g_ms[2];
        out->integrate_calls = g_calls[0];
        out->scatter_calls = g_calls[1];
        out->spmv_calls = g_calls[2];
    }
    if (reset)
        for (int i = 0; i < 3; i++) {
            g_ms[i] = 0;
            g_calls[i] = 0;
        }
    return st;
}

}  // extern "C"
