// Serving core on the GPU (nao.h, nao_server_*): the scheduling logic of scheduler.cpp driven by a
// HIP executor.  A session's structure lives in a system of the home context plus device
// buffers for D, v, H and n; every launch is one nao_run_many on a slot's context and stream.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "internal.h"
#include "nao.h"
#include "scheduler.h"

using namespace nao;

namespace {

size_t matrix_bytes(int64_t nb) { return (size_t)std::max<int64_t>(1, nb * nb) * sizeof(double); }
size_t points_bytes(int64_t np) { return (size_t)std::max<int64_t>(1, np) * sizeof(double); }

struct HipSession {
    nao_system sys = nullptr;
    double *D = nullptr, *v = nullptr, *H = nullptr, *n = nullptr;
    bool v_staged = false;  // a v has been staged by an earlier launch
};

struct HipSlot {
    nao_ctx ctx = nullptr;
    hipEvent_t done = nullptr;
};

class HipExec : public SchedExec {
public:
    nao_ctx home = nullptr;
    nao_precision prec = NAO_FP64;
    int32_t group_max = 256;
    std::vector<HipSlot> slots;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    nao_status admit(const HostStructure& h, SessionRes& res, std::string& err) override
    {
        nao_system sys = nullptr;
        nao_status st = nao_build_batches(home, &h.desc, h.n_points(), h.xyz.data(), h.w.data(), h.max_batch, &sys);
        if (st == NAO_OK && group_max != 256) {
            st = nao_system_set_group_max(sys, group_max);
            if (st != NAO_OK) {
                nao_system_destroy(sys);
                sys = nullptr;
            }
        }
        if (st != NAO_OK) {
            err = nao_last_error(home);
            return st;
        }
        int64_t nb = 0;
        nao_system_info(sys, &nb, nullptr, nullptr, nullptr);
        const int64_t np = h.n_points();
        HipSession* hs = new (std::nothrow) HipSession();
        if (!hs) {
            nao_system_destroy(sys);
            err = "host allocation failed";
            return NAO_ERR_OUT_OF_MEMORY;
        }
        void *D = nullptr, *H = nullptr, *v = nullptr, *n = nullptr;
        const size_t mb = matrix_bytes(nb), pb = points_bytes(np);
        if ((st = ctx_alloc(home, mb, &D)) == NAO_OK && (st = ctx_alloc(home, mb, &H)) == NAO_OK &&
            (st = ctx_alloc(home, pb, &v)) == NAO_OK && (st = ctx_alloc(home, pb, &n)) == NAO_OK) {
            hs->sys = sys;
            hs->D = static_cast<double*>(D);
            hs->H = static_cast<double*>(H);
            hs->v = static_cast<double*>(v);
            hs->n = static_cast<double*>(n);
            res.handle = hs;
            res.n_basis = nb;
            res.n_points = np;
            res.bytes = system_device_bytes(sys) + 2 * mb + 2 * pb;
            return NAO_OK;
        }
        err = nao_last_error(home);
        ctx_free(home, D, mb);
        ctx_free(home, H, mb);
        ctx_free(home, v, pb);
        ctx_free(home, n, pb);
        nao_system_destroy(sys);
        delete hs;
        return st;
    }

    void release(SessionRes& res) override
    {
        HipSession* hs = static_cast<HipSession*>(res.handle);
        if (!hs) return;
        if (hs->sys) nao_system_destroy(hs->sys);
        ctx_free(home, hs->D, matrix_bytes(res.n_basis));
        ctx_free(home, hs->H, matrix_bytes(res.n_basis));
        ctx_free(home, hs->v, points_bytes(res.n_points));
        ctx_free(home, hs->n, points_bytes(res.n_points));
        delete hs;
        res = SessionRes();
    }

    nao_status launch(int slot, const std::vector<LaunchItem>& items, std::string& err) override
    {
        HipSlot& sl = slots[slot];
        hipStream_t st = ctx_stream(sl.ctx);
        std::vector<nao_work> work;
        nao_status s = NAO_OK;
        for (const LaunchItem& it : items) {
            HipSession* hs = static_cast<HipSession*>(it.res->handle);
            // stage this iteration's inputs into the session's buffers on the slot's stream
            const size_t mb = (size_t)it.res->n_basis * it.res->n_basis * sizeof(double);
            hipError_t e = hipSuccess;
            if (mb) {
                const hipMemcpyKind k = it.D_space == NAO_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
                e = hipMemcpyAsync(hs->D, it.D, mb, k, st);
            }
            if (e == hipSuccess && it.v && it.res->n_points) {
                const hipMemcpyKind k = it.v_space == NAO_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
                e = hipMemcpyAsync(hs->v, it.v, it.res->n_points * sizeof(double), k, st);
            }
            if (e != hipSuccess) {
                err = std::string("staging inputs: ") + hipGetErrorString(e);
                s = NAO_ERR_HIP;
                break;
            }
            if (it.v) hs->v_staged = true;
            if (!hs->v_staged) {
                err = "no potential staged for this session (its first request failed)";
                s = NAO_ERR_INVALID_ARG;
                break;
            }
            work.push_back(nao_work{hs->sys, 1, hs->D, hs->n, nullptr});
            work.push_back(nao_work{hs->sys, 0, hs->v, hs->H, nullptr});
        }
        if (s == NAO_OK) {
            s = nao_run_many(sl.ctx, work.data(), (int64_t)work.size(), prec, nullptr, 0);
            if (s != NAO_OK) err = nao_last_error(sl.ctx);
        }
        if (s == NAO_OK) {
            const hipError_t e = hipEventRecord(sl.done, st);
            if (e == hipSuccess) return NAO_OK;
            err = std::string("slot event: ") + hipGetErrorString(e);
            s = NAO_ERR_HIP;
        }
        (void)hipStreamSynchronize(st);  // nothing of a failed launch may still run
        return s;
    }

    int poll(int slot, std::string& err) override
    {
        const hipError_t e = hipEventQuery(slots[slot].done);
        if (e == hipErrorNotReady) return 0;
        if (e == hipSuccess) return 1;
        err = hipGetErrorString(e);
        return NAO_ERR_HIP;
    }

    void retired(int slot) override { (void)nao_ctx_synchronize(slots[slot].ctx); }  // frees its launch plan

    nao_status copy_out(const SessionRes& res, double* H, double* n, nao_memspace space, std::string& err) override
    {
        const HipSession* hs = static_cast<const HipSession*>(res.handle);
        const hipMemcpyKind k = space == NAO_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        hipError_t e = hipSuccess;
        if (H && res.n_basis) e = hipMemcpy(H, hs->H, res.n_basis * res.n_basis * sizeof(double), k);
        if (e == hipSuccess && n && res.n_points) e = hipMemcpy(n, hs->n, res.n_points * sizeof(double), k);
        if (e == hipSuccess) return NAO_OK;
        err = hipGetErrorString(e);
        return NAO_ERR_HIP;
    }

    double now() override
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    void report(const std::string& msg) override { ctx_set_error(home, msg); }
};

}  // namespace

struct nao_server_s {
    HipExec exec;
    Scheduler* sched = nullptr;
};

extern "C" {

void nao_server_destroy(nao_server srv)
{
    if (!srv) return;
    delete srv->sched;  // stops the builder, waits for launches, releases the sessions
    for (HipSlot& sl : srv->exec.slots) {
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.ctx) nao_ctx_destroy(sl.ctx);
    }
    delete srv;
}

nao_status nao_server_create(nao_ctx home, int32_t n_slots, int32_t max_per_launch, int32_t group_max,
                             nao_precision precision, nao_server* out)
{
    if (!out || !home) return NAO_ERR_INVALID_ARG;
    *out = nullptr;
    if (n_slots < 1 || n_slots > 16 || max_per_launch < 1 || max_per_launch > 256)
        return (ctx_set_error(home, "n_slots outside [1, 16] or max_per_launch outside [1, 256]"), NAO_ERR_INVALID_ARG);
    if (precision < NAO_FP64 || precision > NAO_BF16X6) return (ctx_set_error(home, "bad precision"), NAO_ERR_INVALID_ARG);
    if (group_max != 0 && (group_max < 16 || group_max > 256))
        return (ctx_set_error(home, "group_max must be 0 or in [16, 256]"), NAO_ERR_INVALID_ARG);
    nao_server srv = new (std::nothrow) nao_server_s();
    if (!srv) return NAO_ERR_OUT_OF_MEMORY;
    srv->exec.home = home;
    srv->exec.prec = precision;
    srv->exec.group_max = group_max;
    srv->exec.slots.resize(n_slots);
    for (HipSlot& sl : srv->exec.slots) {
        nao_status st = nao_ctx_create(ctx_device(home), nullptr, 0, &sl.ctx);
        if (st == NAO_OK && hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) st = NAO_ERR_HIP;
        if (st != NAO_OK) {
            nao_server_destroy(srv);
            return st;
        }
    }
    srv->sched = new (std::nothrow) Scheduler(&srv->exec, n_slots, max_per_launch);
    if (!srv->sched || srv->sched->start() != NAO_OK) {
        nao_server_destroy(srv);
        return NAO_ERR_INTERNAL;
    }
    *out = srv;
    return NAO_OK;
}

nao_status nao_server_open_session(nao_server srv, const nao_basis_desc* basis, int64_t n_points,
                                   const double* point_xyz, const double* point_w, int32_t max_batch, int64_t* session)
{
    if (!srv) return NAO_ERR_INVALID_ARG;
    return srv->sched->open_session(basis, n_points, point_xyz, point_w, max_batch, session);
}

nao_status nao_server_close_session(nao_server srv, int64_t session)
{
    if (!srv) return NAO_ERR_INVALID_ARG;
    return srv->sched->close_session(session);
}

nao_status nao_server_session_info(nao_server srv, int64_t session, int32_t* state, size_t* bytes, int64_t* n_basis,
                                   int64_t* n_points)
{
    if (!srv) return NAO_ERR_INVALID_ARG;
    return srv->sched->session_info(session, state, bytes, n_basis, n_points);
}

nao_status nao_server_submit(nao_server srv, int64_t session, const double* D, nao_memspace D_space, const double* v,
                             nao_memspace v_space, uint64_t* ticket)
{
    if (!srv) return NAO_ERR_INVALID_ARG;
    return srv->sched->submit(session, D, D_space, v, v_space, ticket);
}

nao_status nao_server_step(nao_server srv, int32_t* n_running, int32_t* n_waiting)
{
    if (!srv) return NAO_ERR_INVALID_ARG;
    return srv->sched->step(n_running, n_waiting);
}

nao_status nao_server_poll(nao_server srv, uint64_t ticket, int32_t* state, double* t_submit, double* t_start,
                           double* t_end)
{
    if (!srv) return NAO_ERR_INVALID_ARG;
    return srv->sched->poll(ticket, state, t_submit, t_start, t_end);
}

nao_status nao_server_result(nao_server srv, uint64_t ticket, double* H, double* n, nao_memspace space)
{
    if (!srv) return NAO_ERR_INVALID_ARG;
    return srv->sched->result(ticket, H, n, space);
}

}  // extern "C"
