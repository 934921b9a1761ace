// Serving core (nao.h, nao_server_*): sessions admitted by HBM footprint, a FIFO of ready
// requests, execution slots (one context and stream each) and continuous batching through
// nao_run_many.  Host-side only; every GPU step is a library call on a slot's stream.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "internal.h"
#include "nao.h"

using namespace nao;

namespace {

struct HostStructure {
    // deep copy of a basis description
    std::vector<double> atom_xyz, rmin, rcut, samples;
    std::vector<int32_t> atom_species, shell_ptr, shell_l, shell_radial;
    nao_basis_desc desc{};
    std::vector<double> xyz, w;
    int32_t max_batch = 0;

    void take(const nao_basis_desc* d, int64_t np, const double* px, const double* pw, int32_t mb)
    {
        const int32_t n_shells = d->species_shell_ptr[d->n_species];
        atom_xyz.assign(d->atom_xyz, d->atom_xyz + 3 * d->n_atoms);
        atom_species.assign(d->atom_species, d->atom_species + d->n_atoms);
        shell_ptr.assign(d->species_shell_ptr, d->species_shell_ptr + d->n_species + 1);
        shell_l.assign(d->shell_l, d->shell_l + n_shells);
        shell_radial.assign(d->shell_radial, d->shell_radial + n_shells);
        rmin.assign(d->radial_rmin, d->radial_rmin + d->n_radial);
        rcut.assign(d->radial_rcut, d->radial_rcut + d->n_radial);
        samples.assign(d->radial_samples, d->radial_samples + (size_t)d->n_radial * d->n_knots);
        desc = *d;
        desc.atom_xyz = atom_xyz.data();
        desc.atom_species = atom_species.data();
        desc.species_shell_ptr = shell_ptr.data();
        desc.shell_l = shell_l.data();
        desc.shell_radial = shell_radial.data();
        desc.radial_rmin = rmin.data();
        desc.radial_rcut = rcut.data();
        desc.radial_samples = samples.data();
        xyz.assign(px, px + 3 * np);
        w.assign(pw, pw + np);
        max_batch = mb;
    }
};

// PENDING -> BUILDING -> RESIDENT -> RELEASING -> GONE; the builder thread owns BUILDING and
// RELEASING (it alone uses the home context), the scheduler dispatches RESIDENT sessions.
enum SessionState { S_PENDING, S_BUILDING, S_RESIDENT, S_RELEASING, S_GONE };

struct Session {
    SessionState state = S_PENDING;
    HostStructure host;
    nao_system sys = nullptr;
    int64_t n_basis = 0, n_points = 0;
    double *D = nullptr, *v = nullptr, *H = nullptr, *n = nullptr;
    size_t bytes = 0;
    bool close_requested = false;
    bool busy = false;        // a request of this session is running
    bool have_v = false;
    bool no_memory = false;   // the last admission attempt did not fit the budget
    bool failed = false;      // admission failed for another reason
};

struct Request {
    int64_t session;
    int32_t state = NAO_REQ_WAITING;
    double t_submit = 0, t_start = 0, t_end = 0;
    const double* D;
    nao_memspace D_space;
    const double* v;
    nao_memspace v_space;
    int slot = -1;
};

struct Slot {
    nao_ctx ctx = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<uint64_t> tickets;
};

}  // namespace

struct nao_server_s {
    std::mutex mu;                      // sessions, queues, requests
    std::condition_variable cv;         // wakes the builder
    std::thread builder;
    bool stop = false;
    uint64_t releases = 0;              // sessions released so far (budget waits on it)
    nao_ctx home = nullptr;
    nao_precision prec = NAO_FP64;
    int32_t max_per_launch = 8;
    int32_t group_max = 256;
    std::vector<Slot> slots;
    std::map<int64_t, Session> sessions;
    std::deque<int64_t> pending;            // sessions waiting for admission, in open order
    std::deque<uint64_t> ready;             // waiting requests, in submit order
    std::unordered_map<uint64_t, Request> reqs;
    uint64_t next_ticket = 1;
    int64_t next_session = 1;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

nao_status fail(nao_server s, nao_status st, const std::string& m)
{
    ctx_set_error(s->home, m);
    return st;
}

size_t matrix_bytes(int64_t nb) { return (size_t)std::max<int64_t>(1, nb * nb) * sizeof(double); }
size_t points_bytes(int64_t np) { return (size_t)std::max<int64_t>(1, np) * sizeof(double); }

// Builder thread only: frees a session's system and buffers through the home context.
void release_session(nao_server srv, Session& se)
{
    if (se.sys) nao_system_destroy(se.sys);
    se.sys = nullptr;
    ctx_free(srv->home, se.D, matrix_bytes(se.n_basis));
    ctx_free(srv->home, se.H, matrix_bytes(se.n_basis));
    ctx_free(srv->home, se.v, points_bytes(se.n_points));
    ctx_free(srv->home, se.n, points_bytes(se.n_points));
    se.D = se.H = se.v = se.n = nullptr;
    se.bytes = 0;
}

// Builder thread only: makes a session resident; NAO_ERR_BUDGET means "not now".
nao_status admit(nao_server srv, Session& se)
{
    nao_system sys = nullptr;
    nao_status st = nao_build_batches(srv->home, &se.host.desc, (int64_t)se.host.w.size(), se.host.xyz.data(),
                                      se.host.w.data(), se.host.max_batch, &sys);
    if (st != NAO_OK) return st;
    if (srv->group_max != 256 && (st = nao_system_set_group_max(sys, srv->group_max)) != NAO_OK) {
        nao_system_destroy(sys);
        return st;
    }
    int64_t nb = 0, np = (int64_t)se.host.w.size();
    nao_system_info(sys, &nb, nullptr, nullptr, nullptr);
    void *D = nullptr, *H = nullptr, *v = nullptr, *n = nullptr;
    const size_t mb = matrix_bytes(nb), pb = points_bytes(np);
    if ((st = ctx_alloc(srv->home, mb, &D)) == NAO_OK && (st = ctx_alloc(srv->home, mb, &H)) == NAO_OK &&
        (st = ctx_alloc(srv->home, pb, &v)) == NAO_OK && (st = ctx_alloc(srv->home, pb, &n)) == NAO_OK) {
        se.sys = sys;
        se.n_basis = nb;
        se.n_points = np;
        se.D = static_cast<double*>(D);
        se.H = static_cast<double*>(H);
        se.v = static_cast<double*>(v);
        se.n = static_cast<double*>(n);
        se.bytes = system_device_bytes(sys) + 2 * mb + 2 * pb;
        se.host.xyz.clear();
        se.host.xyz.shrink_to_fit();
        se.host.w.clear();
        se.host.w.shrink_to_fit();
        return NAO_OK;
    }
    ctx_free(srv->home, D, mb);
    ctx_free(srv->home, H, mb);
    ctx_free(srv->home, v, pb);
    ctx_free(srv->home, n, pb);
    nao_system_destroy(sys);
    return st;
}

bool queued_for(nao_server srv, int64_t sid)
{
    for (uint64_t tk : srv->ready)
        if (srv->reqs[tk].session == sid) return true;
    return false;
}

// The builder: releases closed sessions and admits pending ones in open order, off the
// scheduler's path.  A session that does not fit waits (and blocks those behind it) until
// another one has been released.
void builder_loop(nao_server srv)
{
    std::unique_lock<std::mutex> lk(srv->mu);
    uint64_t seen_releases = srv->releases;
    bool blocked = false;
    for (;;) {
        srv->cv.wait(lk, [&] {
            if (srv->stop) return true;
            for (auto& kv : srv->sessions)
                if (kv.second.state == S_RELEASING) return true;
            return !srv->pending.empty() && (!blocked || srv->releases != seen_releases);
        });
        if (srv->stop) return;
        // releases first: they make room
        for (auto& kv : srv->sessions) {
            Session& se = kv.second;
            if (se.state != S_RELEASING) continue;
            lk.unlock();
            release_session(srv, se);
            lk.lock();
            se.state = S_GONE;
            ++srv->releases;
        }
        while (!srv->pending.empty()) {
            const int64_t id = srv->pending.front();
            Session& se = srv->sessions[id];
            if (se.state != S_PENDING) {
                srv->pending.pop_front();
                continue;
            }
            se.state = S_BUILDING;
            lk.unlock();
            const nao_status st = admit(srv, se);
            lk.lock();
            if (st == NAO_OK) {
                se.state = S_RESIDENT;
                se.no_memory = false;
                srv->pending.pop_front();
                blocked = false;
                continue;
            }
            bool others = false;  // resident sessions whose release could make room
            for (auto& kv : srv->sessions)
                others = others || (kv.first != id && (kv.second.state == S_RESIDENT || kv.second.state == S_RELEASING));
            if (st == NAO_ERR_BUDGET && others) {
                se.state = S_PENDING;
                se.no_memory = true;
                blocked = true;
                seen_releases = srv->releases;
                break;
            }
            if (st == NAO_ERR_BUDGET) ctx_set_error(srv->home, "session does not fit the budget of the home context");
            // any other failure (or a session larger than the whole budget): it and its requests fail
            se.state = S_GONE;
            se.failed = true;
            srv->pending.pop_front();
            for (auto& kv : srv->reqs)
                if (kv.second.session == id && kv.second.state == NAO_REQ_WAITING) kv.second.state = NAO_REQ_FAILED;
            std::deque<uint64_t> keep;
            for (uint64_t tk : srv->ready)
                if (srv->reqs[tk].session != id) keep.push_back(tk);
            srv->ready.swap(keep);
        }
    }
}

// Scheduler side (caller holds mu): finished launches, then sessions that can be released.
nao_status retire(nao_server srv)
{
    bool released = false;
    for (Slot& sl : srv->slots) {
        if (!sl.busy) continue;
        const hipError_t e = hipEventQuery(sl.done);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) return fail(srv, NAO_ERR_HIP, std::string("slot completion: ") + hipGetErrorString(e));
        const double t = srv->now();
        for (uint64_t tk : sl.tickets) {
            Request& r = srv->reqs[tk];
            r.state = NAO_REQ_DONE;
            r.t_end = t;
            srv->sessions[r.session].busy = false;
        }
        sl.tickets.clear();
        sl.busy = false;
        nao_ctx_synchronize(sl.ctx);  // frees the finished launch plan of this slot
    }
    for (auto& kv : srv->sessions) {
        Session& se = kv.second;
        if (se.close_requested && !se.busy && se.state == S_RESIDENT && !queued_for(srv, kv.first)) {
            se.state = S_RELEASING;
            released = true;
        }
    }
    if (released) srv->cv.notify_all();
    return NAO_OK;
}

nao_status dispatch(nao_server srv, Slot& sl)
{
    std::vector<uint64_t> take;
    std::vector<int64_t> used;
    for (auto it = srv->ready.begin(); it != srv->ready.end() && (int32_t)take.size() < srv->max_per_launch;) {
        Request& r = srv->reqs[*it];
        Session& se = srv->sessions[r.session];
        const bool dup = std::find(used.begin(), used.end(), r.session) != used.end();
        if (se.state == S_RESIDENT && !se.busy && !dup) {
            take.push_back(*it);
            used.push_back(r.session);
            it = srv->ready.erase(it);
        } else {
            ++it;
        }
    }
    if (take.empty()) return NAO_OK;
    hipStream_t st = ctx_stream(sl.ctx);
    std::vector<nao_work> work;
    const double t = srv->now();
    for (uint64_t tk : take) {
        Request& r = srv->reqs[tk];
        Session& se = srv->sessions[r.session];
        // stage this iteration's inputs into the session's buffers on the slot's stream
        const size_t mb = (size_t)se.n_basis * se.n_basis * sizeof(double);
        if (mb) {
            const hipMemcpyKind k = r.D_space == NAO_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
            const hipError_t e = hipMemcpyAsync(se.D, r.D, mb, k, st);
            if (e != hipSuccess) return fail(srv, NAO_ERR_HIP, std::string("staging D: ") + hipGetErrorString(e));
        }
        if (r.v && se.n_points) {
            const hipMemcpyKind k = r.v_space == NAO_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
            const hipError_t e = hipMemcpyAsync(se.v, r.v, se.n_points * sizeof(double), k, st);
            if (e != hipSuccess) return fail(srv, NAO_ERR_HIP, std::string("staging v: ") + hipGetErrorString(e));
            se.have_v = true;
        }
        se.busy = true;
        r.state = NAO_REQ_RUNNING;
        r.t_start = t;
        r.slot = (int)(&sl - srv->slots.data());
        work.push_back(nao_work{se.sys, 1, se.D, se.n});
        work.push_back(nao_work{se.sys, 0, se.v, se.H});
    }
    nao_status s = nao_run_many(sl.ctx, work.data(), (int64_t)work.size(), srv->prec, 0);
    if (s != NAO_OK) return fail(srv, s, std::string("slot launch: ") + nao_last_error(sl.ctx));
    const hipError_t e = hipEventRecord(sl.done, st);
    if (e != hipSuccess) return fail(srv, NAO_ERR_HIP, std::string("slot event: ") + hipGetErrorString(e));
    sl.tickets = take;
    sl.busy = true;
    return NAO_OK;
}

}  // namespace

extern "C" {

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
    srv->home = home;
    srv->prec = precision;
    srv->max_per_launch = max_per_launch;
    srv->group_max = group_max;
    srv->slots.resize(n_slots);
    for (Slot& sl : srv->slots) {
        nao_status st = nao_ctx_create(ctx_device(home), nullptr, 0, &sl.ctx);
        if (st == NAO_OK && hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) st = NAO_ERR_HIP;
        if (st != NAO_OK) {
            nao_server_destroy(srv);
            return st;
        }
    }
    try {
        srv->builder = std::thread(builder_loop, srv);
    } catch (...) {
        nao_server_destroy(srv);
        return NAO_ERR_INTERNAL;
    }
    *out = srv;
    return NAO_OK;
}

nao_status nao_server_open_session(nao_server srv, const nao_basis_desc* basis, int64_t n_points,
                                   const double* point_xyz, const double* point_w, int32_t max_batch, int64_t* session)
{
    if (!srv || !basis || !session || n_points < 0 || (n_points > 0 && (!point_xyz || !point_w)))
        return NAO_ERR_INVALID_ARG;
    if (!basis->species_shell_ptr || basis->n_species < 1) return fail(srv, NAO_ERR_INVALID_ARG, "bad basis");
    try {
        HostStructure host;
        host.take(basis, n_points, point_xyz, point_w, max_batch);
        std::lock_guard<std::mutex> lk(srv->mu);
        const int64_t id = srv->next_session++;
        Session& se = srv->sessions[id];
        se.host = std::move(host);
        se.host.desc.atom_xyz = se.host.atom_xyz.data();  // re-point the copy after the move
        se.host.desc.atom_species = se.host.atom_species.data();
        se.host.desc.species_shell_ptr = se.host.shell_ptr.data();
        se.host.desc.shell_l = se.host.shell_l.data();
        se.host.desc.shell_radial = se.host.shell_radial.data();
        se.host.desc.radial_rmin = se.host.rmin.data();
        se.host.desc.radial_rcut = se.host.rcut.data();
        se.host.desc.radial_samples = se.host.samples.data();
        se.n_points = n_points;
        srv->pending.push_back(id);
        *session = id;
    } catch (const std::bad_alloc&) {
        return fail(srv, NAO_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
    srv->cv.notify_all();
    return NAO_OK;
}

nao_status nao_server_close_session(nao_server srv, int64_t session)
{
    if (!srv) return NAO_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->sessions.find(session);
    if (it == srv->sessions.end() || it->second.state == S_GONE || it->second.close_requested)
        return fail(srv, NAO_ERR_INVALID_ARG, "unknown or closed session");
    it->second.close_requested = true;
    if (it->second.state == S_PENDING && !queued_for(srv, session)) {
        srv->pending.erase(std::remove(srv->pending.begin(), srv->pending.end(), session), srv->pending.end());
        it->second.state = S_GONE;
    }
    return NAO_OK;
}

nao_status nao_server_session_info(nao_server srv, int64_t session, int32_t* state, size_t* bytes, int64_t* n_basis,
                                   int64_t* n_points)
{
    if (!srv) return NAO_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->sessions.find(session);
    if (it == srv->sessions.end()) return fail(srv, NAO_ERR_INVALID_ARG, "unknown session");
    const Session& se = it->second;
    if (state) {
        if (se.state == S_RESIDENT) *state = NAO_SESSION_RESIDENT;
        else if (se.failed) *state = NAO_SESSION_FAILED;
        else if (se.state == S_GONE || se.state == S_RELEASING) *state = NAO_SESSION_CLOSED;
        else *state = se.no_memory ? NAO_SESSION_NO_MEMORY : NAO_SESSION_QUEUED;
    }
    if (bytes) *bytes = it->second.bytes;
    if (n_basis) *n_basis = it->second.n_basis;
    if (n_points) *n_points = it->second.n_points;
    return NAO_OK;
}

nao_status nao_server_submit(nao_server srv, int64_t session, const double* D, nao_memspace D_space, const double* v,
                             nao_memspace v_space, uint64_t* ticket)
{
    if (!srv || !ticket) return NAO_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->sessions.find(session);
    if (it == srv->sessions.end() || it->second.state == S_GONE || it->second.close_requested)
        return fail(srv, NAO_ERR_INVALID_ARG, "unknown or closed session");
    if (!D) return fail(srv, NAO_ERR_INVALID_ARG, "D is NULL");
    if (!v && !it->second.have_v) {
        bool earlier = false;  // an earlier queued request may bring v
        for (uint64_t tk : srv->ready) earlier = earlier || (srv->reqs[tk].session == session && srv->reqs[tk].v);
        if (!earlier) return fail(srv, NAO_ERR_INVALID_ARG, "first request of a session needs v");
    }
    const uint64_t tk = srv->next_ticket++;
    Request r;
    r.session = session;
    r.t_submit = srv->now();
    r.D = D;
    r.D_space = D_space;
    r.v = v;
    r.v_space = v_space;
    srv->reqs[tk] = r;
    srv->ready.push_back(tk);
    *ticket = tk;
    return NAO_OK;
}

nao_status nao_server_step(nao_server srv, int32_t* n_running, int32_t* n_waiting)
{
    if (!srv) return NAO_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    nao_status st = retire(srv);
    if (st != NAO_OK) return st;
    for (Slot& sl : srv->slots)
        if (!sl.busy && (st = dispatch(srv, sl)) != NAO_OK) return st;
    int32_t run = 0, wait = (int32_t)srv->ready.size();
    for (const Slot& sl : srv->slots) run += (int32_t)sl.tickets.size();
    if (n_running) *n_running = run;
    if (n_waiting) *n_waiting = wait;
    return NAO_OK;
}

nao_status nao_server_poll(nao_server srv, uint64_t ticket, int32_t* state, double* t_submit, double* t_start,
                           double* t_end)
{
    if (!srv) return NAO_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return fail(srv, NAO_ERR_INVALID_ARG, "unknown ticket");
    if (state) *state = it->second.state;
    if (t_submit) *t_submit = it->second.t_submit;
    if (t_start) *t_start = it->second.t_start;
    if (t_end) *t_end = it->second.t_end;
    return NAO_OK;
}

nao_status nao_server_result(nao_server srv, uint64_t ticket, double* H, double* n, nao_memspace space)
{
    if (!srv) return NAO_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end() || it->second.state != NAO_REQ_DONE) return fail(srv, NAO_ERR_NOT_READY, "request not done");
    Session& se = srv->sessions[it->second.session];
    if (se.state != S_RESIDENT) return fail(srv, NAO_ERR_INVALID_ARG, "session no longer resident");
    const hipMemcpyKind k = space == NAO_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    hipError_t e = hipSuccess;
    if (H && se.n_basis) e = hipMemcpy(H, se.H, se.n_basis * se.n_basis * sizeof(double), k);
    if (e == hipSuccess && n && se.n_points) e = hipMemcpy(n, se.n, se.n_points * sizeof(double), k);
    if (e != hipSuccess) return fail(srv, NAO_ERR_HIP, std::string("result copy: ") + hipGetErrorString(e));
    return NAO_OK;
}

void nao_server_destroy(nao_server srv)
{
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv.notify_all();
    if (srv->builder.joinable()) srv->builder.join();
    for (Slot& sl : srv->slots)
        if (sl.ctx) nao_ctx_synchronize(sl.ctx);
    for (auto& kv : srv->sessions)
        if (kv.second.state == S_RESIDENT || kv.second.state == S_RELEASING) release_session(srv, kv.second);
    for (Slot& sl : srv->slots) {
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.ctx) nao_ctx_destroy(sl.ctx);
    }
    delete srv;
}

}  // extern "C"
