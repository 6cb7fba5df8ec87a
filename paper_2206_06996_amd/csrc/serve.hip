// serve.hip -- continuous-batching server over the SCR and mesh-motion solves (srv_* in scr.h).
//
// A FIFO queue feeds max_slots worker threads, each owning one HIP stream.  Admission is by
// device-memory footprint: a request starts only when a slot is free and its footprint estimate
// fits next to the requests already running; requests that arrive meanwhile wait in order and
// start as soon as a finishing request releases its slot and memory.  Kernels of different
// requests overlap on the device through the slots' streams.  Each request builds its
// hierarchies once and reuses them for all of its successive corrections, re-set up numerically
// when a correction brings new matrix values (given, or assembled on the device from the
// request's mesh at a new advective velocity).
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>

#include "../../include/scr.h"
#include "common.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Job {
    int64_t id = 0;
    scr_bsr K{};
    const double* coords = nullptr;
    std::vector<const double*> b, bm, vals, u;
    scr_assembler* tangent = nullptr;   // tangents assembled on the device at u[c]
    std::vector<double*> x, xm;
    bool has_L = false;
    scr_bsr L{};
    int64_t footprint = 0;
    Clock::time_point t_submit, t_admit;
    bool done = false;
    srv_result res{};
};

}  // namespace

struct scr_server {
    scr_ctx* ctx = nullptr;
    int device = 0;
    int64_t budget = 0;
    scr_amg_opts amg{};
    scr_solve_opts solve{};
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Job*> queue;
    std::map<int64_t, Job*> jobs;
    int64_t next_id = 1, reserved = 0;
    int active = 0, max_active = 0, pending = 0;
    bool stop = false;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
};

namespace {

void run_job(scr_server* S, Job* j, hipStream_t st) {
    srv_result& r = j->res;
    r.status = SCR_OK;
    scr_handle* h = nullptr;
    scr_handle* hm = nullptr;
    double* kval = nullptr;            // assembled tangent values (16 nnzb), if j->tangent
    const int64_t kbytes = j->K.nnzb * 16 * (int64_t)sizeof(double);
    auto t0 = Clock::now();
    scr_bsr K0 = j->K;
    scr_status rc = SCR_OK;
    if (j->tangent) {
        if (hipMallocAsync(reinterpret_cast<void**>(&kval), (size_t)j->K.nnzb * 16 * sizeof(double), st) != hipSuccess) {
            (void)hipGetLastError();
            kval = nullptr;
            rc = SCR_E_OOM;
        } else {
            rc = scr_assemble_tangent(j->tangent, j->u.empty() ? nullptr : j->u[0], kval, st);
            K0.val = kval;
        }
    }
    if (rc == SCR_OK) rc = amg_setup(S->ctx, SCR_SYSTEM, &K0, j->coords, &S->amg, st, &h);
    if (rc == SCR_OK && j->has_L) rc = amg_setup(S->ctx, MESH_SYSTEM, &j->L, nullptr, &S->amg, st, &hm);
    r.setup_ms = std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
    if (rc != SCR_OK) {
        r.status = rc;
    } else {
        r.device_bytes = scr_handle_peak_bytes(h) + (hm ? scr_handle_peak_bytes(hm) : 0) + (kval ? kbytes : 0);
        auto t1 = Clock::now();
        for (size_t c = 0; c < j->b.size(); ++c) {
            const double* newval = nullptr;
            auto tu = Clock::now();
            scr_status ru = SCR_OK;
            if (c > 0 && j->tangent && !j->u.empty() && j->u[c]) {
                ru = scr_assemble_tangent(j->tangent, j->u[c], kval, st);
                newval = kval;
            } else if (c > 0 && !j->tangent && !j->vals.empty() && j->vals[c]) {
                newval = j->vals[c];
            }
            if (ru == SCR_OK && newval) {
                // a new tangent for this correction: numeric re-setup on the same pattern
                scr_bsr Kc = j->K;
                Kc.val = newval;
                ru = amg_update(h, &Kc, nullptr, st);
            }
            if (newval || ru != SCR_OK) {
                r.setup_ms += std::chrono::duration<double, std::milli>(Clock::now() - tu).count();
                if (ru != SCR_OK) {
                    r.status = ru;
                    break;
                }
            }
            scr_stats stt{};
            scr_status rs = scr_solve(h, j->b[c], j->x[c], &S->solve, st, &stt);
            r.last = stt;
            ++r.n_solves;
            if (rs != SCR_OK && (r.status == SCR_OK || rs < 0)) r.status = rs;
            if (rs < 0) break;
            if (hm) {
                scr_stats sm{};
                scr_status rm = mesh_motion_solve(hm, j->bm[c], j->xm[c], &S->solve, st, &sm);
                if (rm != SCR_OK && (r.status == SCR_OK || rm < 0)) r.status = rm;
                if (rm < 0) break;
            }
            int64_t by = scr_handle_peak_bytes(h) + (hm ? scr_handle_peak_bytes(hm) : 0) + (kval ? kbytes : 0);
            if (by > r.device_bytes) r.device_bytes = by;
        }
        r.solve_ms = std::chrono::duration<double, std::milli>(Clock::now() - t1).count();
    }
    if (h) scr_handle_destroy(h);
    if (hm) scr_handle_destroy(hm);
    if (kval) {
        (void)hipFreeAsync(kval, st);
        (void)hipStreamSynchronize(st);
    }
}

void worker(scr_server* S, int slot) {
    (void)hipSetDevice(S->device);
    hipStream_t st = S->streams[slot];
    for (;;) {
        Job* j = nullptr;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            // the budget holds on the way out too: srv_destroy lets the queue drain, in order
            S->cv_work.wait(lk, [&] {
                if (S->queue.empty()) return S->stop;
                Job* h = S->queue.front();
                return S->reserved + h->footprint <= S->budget || S->active == 0 || S->budget <= 0;
            });
            if (S->queue.empty()) return;     // stop requested and nothing left
            j = S->queue.front();
            S->queue.pop_front();
            S->reserved += j->footprint;
            ++S->active;
            if (S->active > S->max_active) S->max_active = S->active;
            j->t_admit = Clock::now();
        }
        run_job(S, j, st);
        {
            std::lock_guard<std::mutex> lk(S->mu);
            auto now = Clock::now();
            j->res.latency_ms = std::chrono::duration<double, std::milli>(now - j->t_submit).count();
            j->res.queue_ms = std::chrono::duration<double, std::milli>(j->t_admit - j->t_submit).count();
            j->res.footprint = j->footprint;
            j->done = true;
            S->reserved -= j->footprint;
            --S->active;
            --S->pending;
        }
        S->cv_work.notify_all();
        S->cv_done.notify_all();
    }
}

}  // namespace

extern "C" {

scr_status srv_create(scr_ctx* ctx, int max_slots, int64_t hbm_budget, const scr_amg_opts* amg,
                      const scr_solve_opts* solve, scr_server** out) {
    if (!ctx || !out || max_slots < 1 || max_slots > 64) {
        scr::set_last_error("srv_create: NULL argument or max_slots outside [1, 64]");
        return SCR_E_INVALID;
    }
    auto* S = new scr_server();
    S->ctx = ctx;
    S->device = ctx->c.device;
    S->budget = hbm_budget > 0 ? hbm_budget : ctx->c.budget;
    if (amg) S->amg = *amg; else scr_default_amg_opts(&S->amg);
    if (solve) S->solve = *solve; else scr_default_solve_opts(&S->solve);
    if (hipSetDevice(S->device) != hipSuccess) {
        delete S;
        scr::set_last_error("srv_create: hipSetDevice failed");
        return SCR_E_HIP;
    }
    for (int i = 0; i < max_slots; ++i) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (auto q : S->streams) (void)hipStreamDestroy(q);
            delete S;
            scr::set_last_error("srv_create: hipStreamCreate failed");
            return SCR_E_HIP;
        }
        S->streams.push_back(st);
    }
    for (int i = 0; i < max_slots; ++i) S->workers.emplace_back(worker, S, i);
    *out = S;
    return SCR_OK;
}

scr_status srv_submit(scr_server* S, const scr_request* r, int64_t* id) {
    if (!S || !r || !id || r->n_rhs < 1 || r->n_rhs > 64 || !r->b || !r->x || !r->coords) {
        scr::set_last_error("srv_submit: NULL argument or n_rhs outside [1, 64]");
        return SCR_E_INVALID;
    }
    if (r->L && (!r->bm || !r->xm)) {
        scr::set_last_error("srv_submit: mesh right-hand sides and outputs are required with L");
        return SCR_E_INVALID;
    }
    if (r->tangent && (scr_assembler_nnzb(r->tangent) != r->K.nnzb ||
                       scr_assembler_nbrows(r->tangent) != r->K.n_brows)) {
        scr::set_last_error("srv_submit: the assembler was not created on K's pattern");
        return SCR_E_INVALID;
    }
    auto* j = new Job();
    j->K = r->K;
    j->tangent = r->tangent;
    j->coords = r->coords;
    for (int c = 0; c < r->n_rhs; ++c) {
        j->b.push_back(r->b[c]);
        j->x.push_back(r->x[c]);
        if (r->L) { j->bm.push_back(r->bm[c]); j->xm.push_back(r->xm[c]); }
        if (r->vals) j->vals.push_back(r->vals[c]);
        if (r->tangent && r->u) j->u.push_back(r->u[c]);
    }
    if (r->L) { j->has_L = true; j->L = *r->L; }
    j->footprint = scr_footprint_estimate(SCR_SYSTEM, r->K.n_brows, r->K.nnzb, &S->amg, &S->solve);
    if (r->L) j->footprint += scr_footprint_estimate(MESH_SYSTEM, r->L->n_brows, r->L->nnzb, &S->amg, &S->solve);
    if (r->tangent) j->footprint += r->K.nnzb * 16 * (int64_t)sizeof(double);
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->budget > 0 && j->footprint > S->budget) {
        delete j;
        scr::set_last_error("srv_submit: request footprint exceeds the server budget");
        return SCR_E_OOM;
    }
    j->id = S->next_id++;
    j->t_submit = Clock::now();
    S->jobs[j->id] = j;
    S->queue.push_back(j);
    ++S->pending;
    *id = j->id;
    S->cv_work.notify_all();
    return SCR_OK;
}

scr_status srv_poll(scr_server* S, int64_t id, int* done, srv_result* res) {
    if (!S || !done) { scr::set_last_error("srv_poll: NULL argument"); return SCR_E_INVALID; }
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(id);
    if (it == S->jobs.end()) { scr::set_last_error("srv_poll: unknown request id"); return SCR_E_INVALID; }
    *done = it->second->done ? 1 : 0;
    if (*done && res) *res = it->second->res;
    return SCR_OK;
}

scr_status srv_wait(scr_server* S, int64_t id, srv_result* res) {
    if (!S) { scr::set_last_error("srv_wait: NULL server"); return SCR_E_INVALID; }
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->jobs.find(id);
    if (it == S->jobs.end()) { scr::set_last_error("srv_wait: unknown request id"); return SCR_E_INVALID; }
    Job* j = it->second;
    S->cv_done.wait(lk, [&] { return j->done; });
    if (res) *res = j->res;
    return SCR_OK;
}

scr_status srv_drain(scr_server* S, int* max_active) {
    if (!S) { scr::set_last_error("srv_drain: NULL server"); return SCR_E_INVALID; }
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->pending == 0; });
    if (max_active) *max_active = S->max_active;
    return SCR_OK;
}

void srv_destroy(scr_server* S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    for (auto& t : S->workers) t.join();
    for (auto q : S->streams) (void)hipStreamDestroy(q);
    for (auto& kv : S->jobs) delete kv.second;
    delete S;
}

}  // extern "C"
