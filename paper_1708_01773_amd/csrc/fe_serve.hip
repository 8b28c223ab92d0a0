// fe_serve.hip -- request server: assemble-and-solve requests admitted by a
// device-memory budget, continuous batching of the Jacobi-PCG iterations of
// every request in flight.
//
// Two host threads drive one device:
//  - the set-up thread takes queued requests in arrival order, waits until
//    the request's bytes fit the budget and a slot is free, then builds the
//    mesh, the CSR pattern, the assembled system and the first PCG state on
//    its own stream;
//  - the solve thread repeatedly takes every request whose set-up finished,
//    runs a chunk of CG iterations for all of them in one sequence of launches
//    (one launch per kernel type over a table of the requests), and retires
//    the requests that stopped.
// A request's arithmetic does not depend on the others in flight: the same
// kernels, plans and per-request reduction order as fe_assemble and
// fe_pcg_solve_mesh, so its result is bitwise that of the request served
// alone.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "fe_internal.h"

namespace fe {

// First-fit allocator over one device block, 256-byte granules.
class Arena {
public:
    ~Arena()
    {
        if (base_) (void)hipFree(base_);
    }
    fe_status init(size_t bytes)
    {
        bytes = bytes / 256 * 256;
        if (bytes == 0) return set_error(FE_EINVAL, "arena of zero bytes");
        hipError_t e = hipMalloc(&base_, bytes);
        if (e != hipSuccess) {
            base_ = nullptr;
            return e == hipErrorOutOfMemory ? set_error(FE_ENOMEM, "budget exceeds free device memory")
                                            : hip_error(e, "arena");
        }
        size_ = bytes;
        free_[0] = bytes;
        return FE_OK;
    }
    bool alloc(size_t bytes, size_t &off)
    {
        bytes = align256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            off = it->first;
            const size_t rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align256(bytes);
        if (bytes == 0) return;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    char *ptr(size_t off) const { return static_cast<char *>(base_) + off; }
    size_t size() const { return size_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

private:
    void *base_ = nullptr;
    size_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

struct Req {
    uint64_t ticket = 0;
    // inputs (host copies)
    int32_t dim = 3, n[3] = {1, 1, 1};
    std::vector<double> xyz, coef;
    int32_t order = 1;
    fe_coeff coeff{};
    double rtol = 0.0;
    int32_t maxit = 0;
    // sizes
    int64_t n_rows = 0, nnz = 0;
    size_t keep_bytes = 0, asm_bytes = 0, mesh_bytes = 0;
    // resources
    fe_mesh mesh = nullptr;
    size_t off = 0, held = 0;  // arena block and the bytes still held
    fe_csr csr{};
    double *x = nullptr;
    void *pcg_ws = nullptr;
    PcgJob job{};
    fe_solve_info info{};
    fe_result res{};
    bool admitted = false;
    std::string err;
};

// Bytes of a request's arena block: CSR, rhs, diagonal inverse, solution and
// PCG state first (kept while solving), then the element workspace and the
// set-up table (returned once the system is assembled).
static void request_sizes(Req &R)
{
    const int ncomp = R.coeff.problem == FE_ELASTICITY ? R.dim : 1;
    space_sizes(R.dim, R.n, R.order, ncomp, R.coeff.dirichlet_faces, R.n_rows, R.nnz);
    const size_t n = size_t(R.n_rows), z = size_t(R.nnz);
    R.keep_bytes = align256(8 * (n + 1)) + align256(4 * z) + align256(8 * z) + 3 * align256(8 * n) +
                   align256(pcg_ws_bytes(R.n_rows));
    SpaceArgs sa{};
    sa.dim = R.dim;
    sa.k = R.order;
    sa.ncomp = ncomp;
    sa.nn = 1;
    for (int r = 0; r < R.dim; r++) sa.nn *= R.order + 1;
    sa.nloc = sa.nn * ncomp;
    sa.ncells = int64_t(R.n[0]) * R.n[1] * (R.dim == 3 ? R.n[2] : 1);
    R.asm_bytes = align256(elem_layout(sa, R.coeff.precision).total) + align256(engine_table_bytes(1));
    // mesh-owned device arrays: vertices, coefficients, axis tables, cell-to-DOF map
    const int64_t nverts = int64_t(R.n[0] + 1) * (R.n[1] + 1) * (R.dim == 3 ? R.n[2] + 1 : 1);
    int64_t axis = 0;
    for (int r = 0; r < R.dim; r++) axis += 3 * (int64_t(R.n[r]) * R.order + 1);
    auto page = [](size_t b) { return (b + 4095) / 4096 * 4096; };
    R.mesh_bytes = page(8 * size_t(nverts) * R.dim) + page(8 * size_t(sa.ncells)) + page(4) + page(8 * size_t(axis)) +
                   page(4 * size_t(sa.ncells) * sa.nloc);
}

}  // namespace fe

using namespace fe;

struct fe_server_s {
    int device = 0;
    size_t budget = 0, mesh_reserve = 0, mesh_used = 0;
    int max_active = 1;
    Arena arena;
    void *tables = nullptr;  // two engine tables of max_active entries
    size_t table_bytes = 0;
    hipStream_t setup_stream = nullptr, solve_stream = nullptr;
    std::mutex mu;
    std::condition_variable cv_setup, cv_solve, cv_done;
    std::deque<Req *> queue;
    std::vector<Req *> ready, active;
    int setting_up = 0;
    std::map<uint64_t, std::unique_ptr<Req>> reqs;
    std::vector<fe_mesh> graveyard;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread setup_thr, solve_thr;
    std::chrono::steady_clock::time_point t0;
    fe_server_stats st{};

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace fe {

static void fail_request(fe_server S, Req *R, fe_status status, const std::string &why)
{
    R->res.state = FE_REQ_FAILED;
    R->res.status = status;
    R->res.t_done = S->now();
    R->err = why;
}

// Set-up of one admitted request on the set-up stream; returns when its
// system is assembled and its PCG state initialised.
static fe_status setup_request(fe_server S, Req &R)
{
    fe_mesh_desc d{};
    d.dim = R.dim;
    for (int r = 0; r < 3; r++) d.n[r] = R.n[r];
    d.vertex_xyz = R.xyz.empty() ? nullptr : R.xyz.data();
    d.cell_coeff = R.coef.empty() ? nullptr : R.coef.data();
    fe_status st = fe_create_mesh(&d, &R.mesh);
    if (st != FE_OK) return st;
    std::vector<double>().swap(R.xyz);
    std::vector<double>().swap(R.coef);
    hipStream_t s = S->setup_stream;
    st = prepare_space(R.mesh, R.order, &R.coeff, s);
    if (st != FE_OK) return st;
    if (R.mesh->space.args.n_rows != R.n_rows || R.mesh->space.args.nnz != R.nnz)
        return set_error(FE_EINVAL, "internal: request sizes differ from the space");
    char *p = S->arena.ptr(R.off);
    const size_t n = size_t(R.n_rows), z = size_t(R.nnz);
    R.csr.n_rows = R.n_rows;
    R.csr.nnz = R.nnz;
    R.csr.rowptr = reinterpret_cast<int64_t *>(p);
    p += align256(8 * (n + 1));
    R.csr.colind = reinterpret_cast<int32_t *>(p);
    p += align256(4 * z);
    R.csr.values = reinterpret_cast<double *>(p);
    p += align256(8 * z);
    R.csr.rhs = reinterpret_cast<double *>(p);
    p += align256(8 * n);
    R.csr.dinv = reinterpret_cast<double *>(p);
    p += align256(8 * n);
    R.x = reinterpret_cast<double *>(p);
    p += align256(8 * n);
    R.pcg_ws = p;
    p += align256(pcg_ws_bytes(R.n_rows));
    void *asm_ws = p;
    const size_t asm_ws_bytes = R.asm_bytes - align256(engine_table_bytes(1));
    void *table = p + asm_ws_bytes;
    st = fe_pattern(R.mesh, R.order, &R.coeff, &R.csr, s);
    if (st != FE_OK) return st;
    st = fe_assemble(R.mesh, R.order, &R.coeff, &R.csr, asm_ws, asm_ws_bytes, s);
    if (st != FE_OK) return st;
    if (R.n_rows > 0) {
        FE_HIP(hipMemsetAsync(R.x, 0, sizeof(double) * n, s));
        R.job = PcgJob{R.n_rows, R.nnz, R.csr.rowptr, R.csr.colind, R.csr.values, false, R.csr.dinv, R.csr.rhs,
                       R.x, R.pcg_ws, &R.info, R.rtol, R.maxit, &R.mesh->space.args};
        std::unique_ptr<EngineSet, void (*)(EngineSet *)> E(engine_create(), engine_destroy);
        st = engine_build(*E, &R.job, 1, table, s);
        if (st != FE_OK) return st;
        st = engine_init(*E, s);
        if (st != FE_OK) return st;
        FE_HIP(hipStreamSynchronize(s));
    }
    return fe_get_status(R.mesh);  // synchronizes the set-up stream; FE_EMESH on det J <= 0
}

static void setup_loop(fe_server S)
{
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        // destroy the meshes of released requests (may wait for the device)
        if (!S->graveyard.empty()) {
            std::vector<fe_mesh> g;
            g.swap(S->graveyard);
            lk.unlock();
            for (fe_mesh m : g) (void)fe_destroy_mesh(m);
            lk.lock();
            continue;
        }
        if (S->stop) {
            for (Req *R : S->queue) fail_request(S, R, FE_EINVAL, "server stopped before admission");
            S->queue.clear();
            S->cv_done.notify_all();
            break;
        }
        if (S->queue.empty()) {
            S->cv_setup.wait(lk);
            continue;
        }
        Req *R = S->queue.front();
        const int in_flight = S->setting_up + int(S->ready.size()) + int(S->active.size());
        size_t off = 0;
        const bool slot = in_flight < S->max_active;
        const bool mesh_fits = S->mesh_used + R->mesh_bytes <= S->mesh_reserve;
        if (!(slot && mesh_fits && S->arena.alloc(R->keep_bytes + R->asm_bytes, off))) {
            S->st.admission_waits++;
            S->cv_setup.wait(lk);  // a retirement, release or stop wakes us
            continue;
        }
        S->queue.pop_front();
        R->admitted = true;
        R->off = off;
        R->held = R->keep_bytes + R->asm_bytes;
        S->mesh_used += R->mesh_bytes;
        S->setting_up++;
        S->st.admitted++;
        S->st.in_use = int64_t(S->arena.used() + S->mesh_used);
        S->st.peak_in_use = std::max(S->st.peak_in_use, S->st.in_use);
        R->res.state = FE_REQ_SETUP;
        R->res.t_admit = S->now();
        R->res.bytes = int64_t(R->held + R->mesh_bytes);
        lk.unlock();
        const fe_status status = setup_request(S, *R);
        const std::string why = status == FE_OK ? std::string() : std::string(fe_last_error());
        lk.lock();
        S->setting_up--;
        // the element workspace and set-up table go back to the arena
        S->arena.release(R->off + R->keep_bytes, R->asm_bytes);
        R->held = R->keep_bytes;
        S->st.in_use = int64_t(S->arena.used() + S->mesh_used);
        if (status != FE_OK) {
            fail_request(S, R, status, why);
            S->cv_done.notify_all();
            continue;
        }
        R->res.t_ready = S->now();
        if (R->n_rows == 0) {
            R->res.state = FE_REQ_DONE;
            R->res.status = FE_OK;
            R->res.t_done = R->res.t_ready;
            S->st.completed++;
            S->cv_done.notify_all();
            continue;
        }
        R->res.state = FE_REQ_SOLVING;
        S->ready.push_back(R);
        S->cv_solve.notify_one();
    }
}

static void solve_loop(fe_server S)
{
    (void)hipSetDevice(S->device);
    std::unique_ptr<EngineSet, void (*)(EngineSet *)> E(engine_create(), engine_destroy);
    std::unique_ptr<EngineSet, void (*)(EngineSet *)> Fin(engine_create(), engine_destroy);
    char *tab0 = static_cast<char *>(S->tables), *tab1 = tab0 + S->table_bytes;
    int chunk = 4;
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        for (Req *R : S->ready) S->active.push_back(R);
        S->ready.clear();
        if (S->active.empty()) {
            if (S->stop && S->setting_up == 0 && S->queue.empty()) break;
            S->cv_solve.wait(lk);
            continue;
        }
        std::vector<PcgJob> jobs;
        for (Req *R : S->active) jobs.push_back(R->job);
        S->st.peak_solving = std::max(S->st.peak_solving, int32_t(jobs.size()));
        S->st.chunks++;
        lk.unlock();
        const auto c0 = std::chrono::steady_clock::now();
        hipStream_t s = S->solve_stream;
        fe_status status = engine_build(*E, jobs.data(), int(jobs.size()), tab0, s);
        if (status == FE_OK) status = engine_iterate(*E, chunk, s);
        if (status == FE_OK) status = engine_states(*E, s);
        std::vector<PcgJob> fin;
        if (status == FE_OK) {
            for (int t = 0; t < engine_size(*E); t++)
                if (engine_done(*E, t)) fin.push_back(engine_job(*E, t));
            if (!fin.empty()) {
                status = engine_build(*Fin, fin.data(), int(fin.size()), tab1, s);
                if (status == FE_OK) status = engine_finish(*Fin, s);
            }
        }
        const std::string why = status == FE_OK ? std::string() : std::string(fe_last_error());
        // chunks of about 4 ms keep the admission delay of new requests short
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - c0).count();
        const double per = ms / chunk;
        chunk = std::max(1, std::min(64, int(4.0 / std::max(per, 1e-3))));
        lk.lock();
        const double t = S->now();
        if (status != FE_OK) {
            for (Req *R : S->active) fail_request(S, R, status, why);
            S->active.clear();
        } else {
            for (const PcgJob &j : fin) {
                Req *R = nullptr;
                for (Req *A : S->active)
                    if (A->job.info == j.info) R = A;
                if (!R) continue;
                R->res.iters = R->info.iters;
                R->res.relres = R->info.relres;
                R->res.true_relres = R->info.true_relres;
                R->res.status = R->info.status;
                R->res.state = FE_REQ_DONE;
                R->res.t_done = t;
                S->st.completed++;
                S->active.erase(std::find(S->active.begin(), S->active.end(), R));
            }
        }
        if (!fin.empty() || status != FE_OK) {
            S->cv_done.notify_all();
            S->cv_setup.notify_all();
        }
    }
}

}  // namespace fe

extern "C" {

fe_status fe_server_create(size_t hbm_budget, int32_t max_active, fe_server *out)
{
    if (!out) return set_error(FE_EINVAL, "null argument");
    *out = nullptr;
    if (max_active < 1 || max_active > 4096) return set_error(FE_EINVAL, "max_active must be in 1..4096");
    if (hbm_budget < (size_t(64) << 20)) return set_error(FE_EINVAL, "budget below 64 MiB");
    std::unique_ptr<fe_server_s> S(new fe_server_s());
    FE_HIP(hipGetDevice(&S->device));
    S->budget = hbm_budget;
    S->max_active = max_active;
    S->table_bytes = align256(engine_table_bytes(max_active));
    S->mesh_reserve = hbm_budget / 8;
    const size_t overhead = 2 * S->table_bytes;
    if (S->mesh_reserve + overhead >= hbm_budget) return set_error(FE_EINVAL, "budget too small");
    fe_status st = S->arena.init(hbm_budget - S->mesh_reserve - overhead);
    if (st != FE_OK) return st;
    FE_HIP(hipMalloc(&S->tables, overhead));
    FE_HIP(hipStreamCreateWithFlags(&S->setup_stream, hipStreamNonBlocking));
    FE_HIP(hipStreamCreateWithFlags(&S->solve_stream, hipStreamNonBlocking));
    S->t0 = std::chrono::steady_clock::now();
    S->st.budget = int64_t(hbm_budget);
    S->st.arena_bytes = int64_t(S->arena.size());
    S->st.mesh_reserve = int64_t(S->mesh_reserve);
    fe_server raw = S.get();
    S->setup_thr = std::thread(setup_loop, raw);
    S->solve_thr = std::thread(solve_loop, raw);
    *out = S.release();
    return FE_OK;
}

fe_status fe_server_submit(fe_server S, const fe_request *q, uint64_t *ticket)
{
    if (!S || !q || !ticket) return set_error(FE_EINVAL, "null argument");
    const fe_mesh_desc &d = q->mesh;
    if (d.dim != 3 && d.dim != 2) return set_error(FE_EINVAL, "dim must be 2 or 3");
    for (int r = 0; r < d.dim; r++)
        if (d.n[r] < 1 || d.n[r] > (1 << 20)) return set_error(FE_EINVAL, "cells per axis must be in 1..2^20");
    if (q->order < 1 || q->order > kMaxOrder) return set_error(FE_EINVAL, "order must be in 1..4");
    if (q->coeff.problem != FE_POISSON && q->coeff.problem != FE_ELASTICITY)
        return set_error(FE_EINVAL, "unknown problem");
    if (q->coeff.precision < FE_FP64 || q->coeff.precision > FE_BF16) return set_error(FE_EINVAL, "unknown precision");
    if (q->coeff.dirichlet_faces >= (1u << (2 * d.dim))) return set_error(FE_EINVAL, "dirichlet face bit out of range");
    if (!(q->rtol >= 0.0) || q->maxit < 0) return set_error(FE_EINVAL, "bad rtol/maxit");
    std::unique_ptr<Req> R(new Req());
    R->dim = d.dim;
    R->n[0] = d.n[0];
    R->n[1] = d.n[1];
    R->n[2] = d.dim == 3 ? d.n[2] : 1;
    R->order = q->order;
    R->coeff = q->coeff;
    R->rtol = q->rtol;
    R->maxit = q->maxit;
    request_sizes(*R);
    if (R->n_rows >= (int64_t(1) << 31)) return set_error(FE_EINVAL, "system has 2^31 or more rows");
    if (R->keep_bytes + R->asm_bytes > S->arena.size() || R->mesh_bytes > S->mesh_reserve) {
        std::lock_guard<std::mutex> lk(S->mu);
        S->st.rejected++;
        return set_error(FE_ENOMEM, "request needs more device memory than the server budget");
    }
    const int64_t nverts = int64_t(R->n[0] + 1) * (R->n[1] + 1) * (d.dim == 3 ? R->n[2] + 1 : 1);
    const int64_t ncells = int64_t(R->n[0]) * R->n[1] * R->n[2];
    if (d.vertex_xyz) R->xyz.assign(d.vertex_xyz, d.vertex_xyz + nverts * d.dim);
    if (d.cell_coeff) R->coef.assign(d.cell_coeff, d.cell_coeff + ncells);
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return set_error(FE_EINVAL, "server is stopping");
    R->ticket = S->next_ticket++;
    R->res.state = FE_REQ_QUEUED;
    R->res.status = FE_OK;
    R->res.n_rows = R->n_rows;
    R->res.nnz = R->nnz;
    R->res.bytes = int64_t(R->keep_bytes + R->asm_bytes + R->mesh_bytes);
    R->res.t_submit = S->now();
    *ticket = R->ticket;
    S->queue.push_back(R.get());
    S->reqs[R->ticket] = std::move(R);
    S->st.submitted++;
    S->cv_setup.notify_one();
    return FE_OK;
}

static fe_status result_of(fe_server S, uint64_t ticket, fe_result *out)
{
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return set_error(FE_EINVAL, "unknown ticket");
    *out = it->second->res;
    if (out->state == FE_REQ_FAILED) return set_error(fe_status(out->status), it->second->err);
    return FE_OK;
}

fe_status fe_server_poll(fe_server S, uint64_t ticket, fe_result *out)
{
    if (!S || !out) return set_error(FE_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    return result_of(S, ticket, out);
}

fe_status fe_server_wait(fe_server S, uint64_t ticket, double timeout_s, fe_result *out)
{
    if (!S || !out) return set_error(FE_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(S->mu);
    const auto until = std::chrono::steady_clock::now() + std::chrono::duration<double>(std::max(timeout_s, 0.0));
    for (;;) {
        auto it = S->reqs.find(ticket);
        if (it == S->reqs.end()) return set_error(FE_EINVAL, "unknown ticket");
        const int state = it->second->res.state;
        if (state == FE_REQ_DONE || state == FE_REQ_FAILED) return result_of(S, ticket, out);
        if (S->cv_done.wait_until(lk, until) == std::cv_status::timeout) return result_of(S, ticket, out);
    }
}

fe_status fe_server_solution(fe_server S, uint64_t ticket, double *x, int64_t n)
{
    if (!S || (!x && n > 0)) return set_error(FE_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return set_error(FE_EINVAL, "unknown ticket");
    Req *R = it->second.get();
    if (R->res.state != FE_REQ_DONE) return set_error(FE_EINVAL, "request has no solution (not done or failed)");
    if (n != R->n_rows) return set_error(FE_EINVAL, "n differs from the request's n_rows");
    lk.unlock();  // a done request's buffers change only through fe_server_release
    if (n > 0) FE_HIP(hipMemcpy(x, R->x, sizeof(double) * size_t(n), hipMemcpyDefault));
    return FE_OK;
}

fe_status fe_server_release(fe_server S, uint64_t ticket)
{
    if (!S) return set_error(FE_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return set_error(FE_EINVAL, "unknown ticket");
    Req *R = it->second.get();
    if (R->res.state != FE_REQ_DONE && R->res.state != FE_REQ_FAILED)
        return set_error(FE_EINVAL, "request still in flight");
    if (R->held) S->arena.release(R->off, R->held);
    if (R->mesh) S->graveyard.push_back(R->mesh);
    if (R->admitted) S->mesh_used -= R->mesh_bytes;
    S->st.in_use = int64_t(S->arena.used() + S->mesh_used);
    S->reqs.erase(it);
    S->cv_setup.notify_all();
    return FE_OK;
}

fe_status fe_server_get_stats(fe_server S, fe_server_stats *out)
{
    if (!S || !out) return set_error(FE_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->st;
    out->queued = int32_t(S->queue.size());
    out->setting_up = S->setting_up;
    out->solving = int32_t(S->ready.size() + S->active.size());
    out->in_use = int64_t(S->arena.used() + S->mesh_used);
    out->peak_arena = int64_t(S->arena.peak());
    return FE_OK;
}

double fe_server_clock(fe_server S) { return S ? S->now() : 0.0; }

fe_status fe_server_destroy(fe_server S)
{
    if (!S) return FE_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_setup.notify_all();
    S->cv_solve.notify_all();
    if (S->setup_thr.joinable()) S->setup_thr.join();
    {
        std::lock_guard<std::mutex> lk(S->mu);
    }
    S->cv_solve.notify_all();
    if (S->solve_thr.joinable()) S->solve_thr.join();
    for (auto &kv : S->reqs)
        if (kv.second->mesh) (void)fe_destroy_mesh(kv.second->mesh);
    for (fe_mesh m : S->graveyard) (void)fe_destroy_mesh(m);
    if (S->setup_stream) (void)hipStreamDestroy(S->setup_stream);
    if (S->solve_stream) (void)hipStreamDestroy(S->solve_stream);
    if (S->tables) (void)hipFree(S->tables);
    delete S;
    return FE_OK;
}

}  // extern "C"
