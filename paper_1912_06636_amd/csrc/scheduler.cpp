// Scheduling core of the serving loop; see scheduler.h.  Pure C++: the device is reached only
// through the SchedExec interface.
#include "scheduler.h"

#include <algorithm>
#include <new>

namespace nao {

bool HostStructure::take(const nao_basis_desc* d, int64_t np, const double* px, const double* pw, int32_t mb)
{
    if (!d || d->n_atoms < 0 || d->n_species < 1 || d->n_radial < 0 || d->n_knots < 0 || !d->species_shell_ptr ||
        np < 0 || (np > 0 && (!px || !pw)))
        return false;
    const int32_t n_shells = d->species_shell_ptr[d->n_species];
    if (n_shells < 0 || (d->n_atoms > 0 && (!d->atom_xyz || !d->atom_species)) ||
        (n_shells > 0 && (!d->shell_l || !d->shell_radial)) ||
        (d->n_radial > 0 && (!d->radial_rmin || !d->radial_rcut || (d->n_knots > 0 && !d->radial_samples))))
        return false;
    atom_xyz.assign(d->atom_xyz, d->atom_xyz + 3 * d->n_atoms);
    atom_species.assign(d->atom_species, d->atom_species + d->n_atoms);
    shell_ptr.assign(d->species_shell_ptr, d->species_shell_ptr + d->n_species + 1);
    shell_l.assign(d->shell_l, d->shell_l + n_shells);
    shell_radial.assign(d->shell_radial, d->shell_radial + n_shells);
    rmin.assign(d->radial_rmin, d->radial_rmin + d->n_radial);
    rcut.assign(d->radial_rcut, d->radial_rcut + d->n_radial);
    samples.assign(d->radial_samples, d->radial_samples + (size_t)d->n_radial * d->n_knots);
    desc = *d;
    xyz.assign(px, px + 3 * np);
    w.assign(pw, pw + np);
    max_batch = mb;
    reseat();
    return true;
}

void HostStructure::reseat()
{
    desc.atom_xyz = atom_xyz.data();
    desc.atom_species = atom_species.data();
    desc.species_shell_ptr = shell_ptr.data();
    desc.shell_l = shell_l.data();
    desc.shell_radial = shell_radial.data();
    desc.radial_rmin = rmin.data();
    desc.radial_rcut = rcut.data();
    desc.radial_samples = samples.data();
}

Scheduler::Scheduler(SchedExec* exec, int n_slots, int max_per_launch)
    : exec_(exec), max_per_launch_(max_per_launch), slots_(n_slots)
{
}

nao_status Scheduler::start()
{
    try {
        builder_ = std::thread(&Scheduler::builder_loop, this);
    } catch (...) {
        return NAO_ERR_INTERNAL;
    }
    return NAO_OK;
}

Scheduler::~Scheduler()
{
    {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
    }
    cv_.notify_all();
    if (builder_.joinable()) builder_.join();
    // launches still in flight finish before their sessions' memory goes
    for (size_t k = 0; k < slots_.size(); ++k) {
        if (!slots_[k].busy) continue;
        std::string err;
        while (exec_->poll((int)k, err) == 0) std::this_thread::yield();
        exec_->retired((int)k);
    }
    for (auto& kv : sessions_)
        if (kv.second.state == S_RESIDENT || kv.second.state == S_RELEASING) exec_->release(kv.second.res);
}

nao_status Scheduler::fail(nao_status st, const std::string& msg)
{
    exec_->report(msg);
    return st;
}

bool Scheduler::queued_for(int64_t sid) const
{
    for (uint64_t tk : ready_) {
        auto it = reqs_.find(tk);
        if (it != reqs_.end() && it->second.session == sid) return true;
    }
    return false;
}

// Caller holds mu_: the requests end as failed and their sessions become free again.
void Scheduler::fail_requests(const std::vector<uint64_t>& tickets, double t)
{
    for (uint64_t tk : tickets) {
        Request& r = reqs_[tk];
        r.state = NAO_REQ_FAILED;
        r.t_end = t;
        sessions_[r.session].busy = false;
    }
}

// The builder: releases closed sessions and admits pending ones in open order, off the
// scheduler's path.  A session that does not fit waits (and holds those behind it) until
// another one has been released.
void Scheduler::builder_loop()
{
    std::unique_lock<std::mutex> lk(mu_);
    uint64_t seen_releases = releases_;
    bool blocked = false;
    for (;;) {
        cv_.wait(lk, [&] {
            if (stop_) return true;
            for (auto& kv : sessions_)
                if (kv.second.state == S_RELEASING) return true;
            return !pending_.empty() && (!blocked || releases_ != seen_releases);
        });
        if (stop_) return;
        for (auto& kv : sessions_) {  // releases first: they make room
            Session& se = kv.second;
            if (se.state != S_RELEASING) continue;
            SessionRes res = se.res;
            lk.unlock();
            exec_->release(res);
            lk.lock();
            se.res = SessionRes();
            se.state = S_GONE;
            ++releases_;
        }
        while (!pending_.empty() && !stop_) {
            const int64_t id = pending_.front();
            Session& se = sessions_[id];
            if (se.state != S_PENDING) {
                pending_.pop_front();
                continue;
            }
            se.state = S_BUILDING;
            lk.unlock();
            SessionRes res;
            std::string err;
            const nao_status st = exec_->admit(se.host, res, err);  // se.host is not touched by others while BUILDING
            lk.lock();
            if (st == NAO_OK) {
                se.res = res;
                se.state = S_RESIDENT;
                se.no_memory = false;
                se.host.xyz.clear();
                se.host.xyz.shrink_to_fit();
                se.host.w.clear();
                se.host.w.shrink_to_fit();
                pending_.pop_front();
                blocked = false;
                continue;
            }
            bool others = false;  // resident sessions whose release could make room
            for (auto& kv : sessions_)
                others = others || (kv.first != id && (kv.second.state == S_RESIDENT || kv.second.state == S_RELEASING));
            if (st == NAO_ERR_BUDGET && others) {
                se.state = S_PENDING;
                se.no_memory = true;
                blocked = true;
                seen_releases = releases_;
                break;
            }
            exec_->report(st == NAO_ERR_BUDGET ? "session does not fit the budget of the home context" : err);
            // any other failure (or a session larger than the whole budget): it and its requests fail
            se.state = S_GONE;
            se.failed = true;
            pending_.pop_front();
            const double t = exec_->now();
            std::deque<uint64_t> keep;
            for (uint64_t tk : ready_) {
                Request& r = reqs_[tk];
                if (r.session == id) {
                    r.state = NAO_REQ_FAILED;
                    r.t_end = t;
                } else {
                    keep.push_back(tk);
                }
            }
            ready_.swap(keep);
        }
    }
}

// Caller holds mu_: finished launches, then sessions that can be released.
nao_status Scheduler::retire()
{
    nao_status out = NAO_OK;
    bool released = false;
    for (size_t k = 0; k < slots_.size(); ++k) {
        Slot& sl = slots_[k];
        if (!sl.busy) continue;
        std::string err;
        const int q = exec_->poll((int)k, err);
        if (q == 0) continue;
        const double t = exec_->now();
        if (q < 0) {  // the launch failed: its requests fail, their sessions are free again
            fail_requests(sl.tickets, t);
            out = fail((nao_status)q, "slot completion: " + err);
        } else {
            for (uint64_t tk : sl.tickets) {
                Request& r = reqs_[tk];
                r.state = NAO_REQ_DONE;
                r.t_end = t;
                sessions_[r.session].busy = false;
            }
        }
        sl.tickets.clear();
        sl.busy = false;
        exec_->retired((int)k);
    }
    for (auto& kv : sessions_) {
        Session& se = kv.second;
        if (se.close_requested && !se.busy && se.state == S_RESIDENT && !queued_for(kv.first)) {
            se.state = S_RELEASING;
            released = true;
        }
    }
    if (released) cv_.notify_all();
    return out;
}

// Caller holds mu_: the oldest ready requests of distinct resident, idle sessions, up to
// max_per_launch, go to the slot as one launch.
nao_status Scheduler::dispatch(int slot)
{
    std::vector<uint64_t> take;
    std::vector<int64_t> used;
    for (auto it = ready_.begin(); it != ready_.end() && (int)take.size() < max_per_launch_;) {
        Request& r = reqs_[*it];
        Session& se = sessions_[r.session];
        const bool dup = std::find(used.begin(), used.end(), r.session) != used.end();
        if (se.state == S_RESIDENT && !se.busy && !dup) {
            take.push_back(*it);
            used.push_back(r.session);
            it = ready_.erase(it);
        } else {
            ++it;
        }
    }
    if (take.empty()) return NAO_OK;
    std::vector<LaunchItem> items;
    const double t = exec_->now();
    for (uint64_t tk : take) {
        Request& r = reqs_[tk];
        Session& se = sessions_[r.session];
        se.busy = true;
        se.last_started = tk;
        r.state = NAO_REQ_RUNNING;
        r.t_start = t;
        items.push_back(LaunchItem{&se.res, r.D, r.D_space, r.v, r.v_space});
    }
    std::string err;
    const nao_status s = exec_->launch(slot, items, err);
    if (s != NAO_OK) {
        fail_requests(take, exec_->now());
        return fail(s, "slot launch: " + err);
    }
    slots_[slot].tickets = take;
    slots_[slot].busy = true;
    return NAO_OK;
}

nao_status Scheduler::open_session(const nao_basis_desc* basis, int64_t n_points, const double* xyz, const double* w,
                                   int32_t max_batch, int64_t* session)
{
    if (!session) return fail(NAO_ERR_INVALID_ARG, "session is NULL");
    try {
        HostStructure host;
        if (!host.take(basis, n_points, xyz, w, max_batch)) return fail(NAO_ERR_INVALID_ARG, "bad structure description");
        std::lock_guard<std::mutex> lk(mu_);
        const int64_t id = next_session_++;
        Session& se = sessions_[id];
        se.host = std::move(host);
        se.host.reseat();
        se.n_points = n_points;
        pending_.push_back(id);
        *session = id;
    } catch (const std::bad_alloc&) {
        return fail(NAO_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
    cv_.notify_all();
    return NAO_OK;
}

nao_status Scheduler::close_session(int64_t session)
{
    std::lock_guard<std::mutex> lk(mu_);
    auto it = sessions_.find(session);
    if (it == sessions_.end() || it->second.state == S_GONE || it->second.close_requested)
        return fail(NAO_ERR_INVALID_ARG, "unknown or closed session");
    it->second.close_requested = true;
    if (it->second.state == S_PENDING && !queued_for(session)) {
        pending_.erase(std::remove(pending_.begin(), pending_.end(), session), pending_.end());
        it->second.state = S_GONE;
    }
    return NAO_OK;
}

nao_status Scheduler::session_info(int64_t session, int32_t* state, size_t* bytes, int64_t* n_basis, int64_t* n_points)
{
    std::lock_guard<std::mutex> lk(mu_);
    auto it = sessions_.find(session);
    if (it == sessions_.end()) return fail(NAO_ERR_INVALID_ARG, "unknown session");
    const Session& se = it->second;
    if (state) {
        if (se.state == S_RESIDENT) *state = NAO_SESSION_RESIDENT;
        else if (se.failed) *state = NAO_SESSION_FAILED;
        else if (se.state == S_GONE || se.state == S_RELEASING) *state = NAO_SESSION_CLOSED;
        else *state = se.no_memory ? NAO_SESSION_NO_MEMORY : NAO_SESSION_QUEUED;
    }
    if (bytes) *bytes = se.res.bytes;
    if (n_basis) *n_basis = se.res.n_basis;
    if (n_points) *n_points = se.n_points;
    return NAO_OK;
}

nao_status Scheduler::submit(int64_t session, const double* D, nao_memspace D_space, const double* v,
                             nao_memspace v_space, uint64_t* ticket)
{
    if (!ticket) return fail(NAO_ERR_INVALID_ARG, "ticket is NULL");
    if ((D_space != NAO_MEM_HOST && D_space != NAO_MEM_DEVICE) || (v_space != NAO_MEM_HOST && v_space != NAO_MEM_DEVICE))
        return fail(NAO_ERR_INVALID_ARG, "bad memspace");
    std::lock_guard<std::mutex> lk(mu_);
    auto it = sessions_.find(session);
    if (it == sessions_.end() || it->second.state == S_GONE || it->second.close_requested)
        return fail(NAO_ERR_INVALID_ARG, "unknown or closed session");
    if (!D) return fail(NAO_ERR_INVALID_ARG, "D is NULL");
    if (!v && !it->second.have_v) return fail(NAO_ERR_INVALID_ARG, "first request of a session needs v");
    if (v) it->second.have_v = true;  // requests of a session run in submit order
    try {
        const uint64_t tk = next_ticket_++;
        Request r;
        r.session = session;
        r.t_submit = exec_->now();
        r.D = D;
        r.D_space = D_space;
        r.v = v;
        r.v_space = v_space;
        reqs_[tk] = r;
        ready_.push_back(tk);
        *ticket = tk;
    } catch (const std::bad_alloc&) {
        return fail(NAO_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
    return NAO_OK;
}

nao_status Scheduler::step(int32_t* n_running, int32_t* n_waiting)
{
    std::lock_guard<std::mutex> lk(mu_);
    nao_status st = retire();
    for (size_t k = 0; k < slots_.size(); ++k) {
        if (slots_[k].busy) continue;
        const nao_status s = dispatch((int)k);
        if (s != NAO_OK && st == NAO_OK) st = s;
        if (s != NAO_OK) break;
    }
    int32_t run = 0;
    for (const Slot& sl : slots_) run += (int32_t)sl.tickets.size();
    if (n_running) *n_running = run;
    if (n_waiting) *n_waiting = (int32_t)ready_.size();
    return st;
}

nao_status Scheduler::poll(uint64_t ticket, int32_t* state, double* t_submit, double* t_start, double* t_end)
{
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return fail(NAO_ERR_INVALID_ARG, "unknown ticket");
    if (state) *state = it->second.state;
    if (t_submit) *t_submit = it->second.t_submit;
    if (t_start) *t_start = it->second.t_start;
    if (t_end) *t_end = it->second.t_end;
    return NAO_OK;
}

nao_status Scheduler::result(uint64_t ticket, double* H, double* n, nao_memspace space)
{
    if (space != NAO_MEM_HOST && space != NAO_MEM_DEVICE) return fail(NAO_ERR_INVALID_ARG, "bad memspace");
    std::lock_guard<std::mutex> lk(mu_);  // no request of the session can start during the copy
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return fail(NAO_ERR_INVALID_ARG, "unknown ticket");
    if (it->second.state != NAO_REQ_DONE) return fail(NAO_ERR_NOT_READY, "request not done");
    Session& se = sessions_[it->second.session];
    if (se.state != S_RESIDENT) return fail(NAO_ERR_INVALID_ARG, "session no longer resident");
    if (se.last_started != ticket)
        return fail(NAO_ERR_INVALID_ARG, "a later request of this session has started: its result replaced this one");
    std::string err;
    const nao_status st = exec_->copy_out(se.res, H, n, space, err);
    if (st != NAO_OK) return fail(st, "result copy: " + err);
    return NAO_OK;
}

}  // namespace nao
