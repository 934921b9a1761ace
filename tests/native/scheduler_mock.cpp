// CPU test of the serving scheduler (scheduler.cpp) with a mock executor and a virtual clock:
// admission in open order by footprint, budget waits and releases, continuous batching over
// slots (at most one request per session in flight, at most max_per_launch requests of distinct
// sessions per launch, FIFO among eligible requests), result validity, forced launch and
// completion failures, shutdown with launches in flight.  Built with sanitizers by
// tests/test_host_native.py; exits non-zero on the first failed check.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "nao.h"
#include "scheduler.h"

using namespace nao;

#define CHECK(cond)                                                                  \
    do {                                                                             \
        if (!(cond)) {                                                               \
            std::fprintf(stderr, "CHECK failed at %s:%d: %s\n", __FILE__, __LINE__, #cond); \
            std::exit(1);                                                            \
        }                                                                            \
    } while (0)

// Inputs carry a tag: D[0] = the iteration's number, v[0] = the potential's number.  The mock
// "result" of a request is H[0] = 1000 v + D, n[0] = D.
struct MockSession {
    double H = -1.0, n = -1.0;
    double v = -1.0;          // staged potential tag (< 0: none staged)
    double last_D = -1e300;   // iterations of a session must arrive in submit order
    bool running = false;
};

class MockExec : public SchedExec {
public:
    std::mutex mu;
    double t = 0.0;                 // virtual clock
    size_t budget = 0, used = 0, peak = 0;
    int max_per_launch = 1;
    int launches = 0;
    int fail_next_launch = 0;       // status returned by the next launch (0: none)
    int fail_next_poll = 0;         // status returned by the next completed poll (0: none)
    bool finish_all = false;        // shutdown: every launch counts as done
    std::string last_report;
    std::vector<std::vector<double>> launch_tags;  // D tags of every launch, in launch order
    struct SlotState {
        bool running = false;
        double t_done = 0.0;
        std::vector<const SessionRes*> items;
        std::vector<double> D, v;
    };
    std::vector<SlotState> slots;
    std::atomic<int> admissions{0};

    explicit MockExec(int n_slots) : slots(n_slots) {}

    nao_status admit(const HostStructure& h, SessionRes& res, std::string& err) override
    {
        std::lock_guard<std::mutex> lk(mu);
        admissions++;
        if (h.max_batch < 1) {
            err = "max_batch outside [1, 4096]";
            return NAO_ERR_INVALID_ARG;
        }
        const size_t bytes = 100 * (size_t)h.n_points();
        if (budget && used + bytes > budget) {
            err = "HBM budget exceeded";
            return NAO_ERR_BUDGET;
        }
        used += bytes;
        peak = std::max(peak, used);
        res.handle = new MockSession();
        res.bytes = bytes;
        res.n_basis = 1;
        res.n_points = h.n_points();
        return NAO_OK;
    }
    void release(SessionRes& res) override
    {
        std::lock_guard<std::mutex> lk(mu);
        MockSession* ms = static_cast<MockSession*>(res.handle);
        CHECK(ms && !ms->running);
        CHECK(used >= res.bytes);
        used -= res.bytes;
        delete ms;
        res = SessionRes();
    }
    nao_status launch(int slot, const std::vector<LaunchItem>& items, std::string& err) override
    {
        std::lock_guard<std::mutex> lk(mu);
        SlotState& s = slots[slot];
        CHECK(!s.running);
        CHECK(!items.empty() && (int)items.size() <= max_per_launch);
        if (fail_next_launch) {
            const int st = fail_next_launch;
            fail_next_launch = 0;
            err = "injected launch failure";
            return (nao_status)st;
        }
        std::set<const SessionRes*> seen;
        std::vector<double> tags;
        for (const LaunchItem& it : items) {
            CHECK(seen.insert(it.res).second);  // distinct sessions
            MockSession* ms = static_cast<MockSession*>(it.res->handle);
            CHECK(!ms->running);                 // one request per session in flight
            CHECK(it.D && it.D[0] > ms->last_D); // submit order within a session
            if (it.v) ms->v = it.v[0];
            if (ms->v < 0) {
                err = "no potential staged for this session";
                return NAO_ERR_INVALID_ARG;
            }
            tags.push_back(it.D[0]);
        }
        s.items.clear();
        s.D.clear();
        for (const LaunchItem& it : items) {
            MockSession* ms = static_cast<MockSession*>(it.res->handle);
            ms->running = true;
            ms->last_D = it.D[0];
            s.items.push_back(it.res);
            s.D.push_back(it.D[0]);
        }
        launch_tags.push_back(tags);
        s.running = true;
        s.t_done = t + (double)items.size();
        launches++;
        return NAO_OK;
    }
    int poll(int slot, std::string& err) override
    {
        std::lock_guard<std::mutex> lk(mu);
        SlotState& s = slots[slot];
        CHECK(s.running);
        if (!finish_all && t < s.t_done) return 0;
        for (size_t k = 0; k < s.items.size(); ++k) {
            MockSession* ms = static_cast<MockSession*>(s.items[k]->handle);
            ms->running = false;
            ms->H = 1000.0 * ms->v + s.D[k];
            ms->n = s.D[k];
        }
        if (fail_next_poll && !finish_all) {
            const int st = fail_next_poll;
            fail_next_poll = 0;
            err = "injected completion failure";
            return st;
        }
        return 1;
    }
    void retired(int slot) override
    {
        std::lock_guard<std::mutex> lk(mu);
        slots[slot].running = false;
        slots[slot].items.clear();
    }
    nao_status copy_out(const SessionRes& res, double* H, double* n, nao_memspace, std::string&) override
    {
        std::lock_guard<std::mutex> lk(mu);
        const MockSession* ms = static_cast<const MockSession*>(res.handle);
        CHECK(!ms->running);
        if (H) H[0] = ms->H;
        if (n) n[0] = ms->n;
        return NAO_OK;
    }
    double now() override
    {
        std::lock_guard<std::mutex> lk(mu);
        return t;
    }
    void report(const std::string& msg) override
    {
        std::lock_guard<std::mutex> lk(mu);
        last_report = msg;
    }
    void advance(double dt)
    {
        std::lock_guard<std::mutex> lk(mu);
        t += dt;
    }
    size_t used_now()
    {
        std::lock_guard<std::mutex> lk(mu);
        return used;
    }
};

// A structure of n_points points (the mock's footprint is 100 bytes per point).
struct Structure {
    double xyz[3] = {0.0, 0.0, 0.0};
    int32_t species = 0, shell_ptr[2] = {0, 1}, shell_l = 0, shell_rad = 0;
    double rmin = 1e-4, rcut = 4.0, samples[4] = {1.0, 0.5, 0.25, 0.0};
    std::vector<double> pxyz, pw;
    nao_basis_desc d{};
    explicit Structure(int64_t np)
    {
        pxyz.assign(3 * np, 0.5);
        pw.assign(np, 1.0);
        d.n_atoms = 1;
        d.atom_xyz = xyz;
        d.atom_species = &species;
        d.n_species = 1;
        d.species_shell_ptr = shell_ptr;
        d.shell_l = &shell_l;
        d.shell_radial = &shell_rad;
        d.n_radial = 1;
        d.n_knots = 4;
        d.radial_rmin = &rmin;
        d.radial_rcut = &rcut;
        d.radial_samples = samples;
    }
};

int32_t state_of(Scheduler& s, int64_t sid)
{
    int32_t st = -1;
    CHECK(s.session_info(sid, &st, nullptr, nullptr, nullptr) == NAO_OK);
    return st;
}

// Wait (real time) until the builder has settled the session out of QUEUED.
int32_t settle(Scheduler& s, int64_t sid)
{
    for (int k = 0; k < 20000; ++k) {
        const int32_t st = state_of(s, sid);
        if (st != NAO_SESSION_QUEUED) return st;
        std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
    CHECK(!"session did not settle");
    return -1;
}

int32_t req_state(Scheduler& s, uint64_t tk)
{
    int32_t st = -1;
    CHECK(s.poll(tk, &st, nullptr, nullptr, nullptr) == NAO_OK);
    return st;
}

// Drive the scheduler (steps, virtual time) until every ticket has ended.
void drain(Scheduler& s, MockExec& ex, const std::vector<uint64_t>& tks, int max_steps = 100000)
{
    for (int k = 0; k < max_steps; ++k) {
        bool all = true;
        for (uint64_t tk : tks) {
            const int32_t st = req_state(s, tk);
            all = all && (st == NAO_REQ_DONE || st == NAO_REQ_FAILED);
        }
        if (all) return;
        (void)s.step(nullptr, nullptr);
        ex.advance(0.25);
        if (k % 64 == 63) std::this_thread::sleep_for(std::chrono::microseconds(50));  // let the builder run
    }
    CHECK(!"requests did not finish");
}

void test_admission_and_budget()
{
    MockExec ex(1);
    ex.budget = 25000;  // two sessions of 100 points, not a third
    ex.max_per_launch = 1;
    {
        Scheduler s(&ex, 1, 1);
        CHECK(s.start() == NAO_OK);
        Structure a(100), big(1000);
        int64_t sid[4], huge;
        for (int k = 0; k < 4; ++k) CHECK(s.open_session(&a.d, 100, a.pxyz.data(), a.pw.data(), 256, &sid[k]) == NAO_OK);
        CHECK(settle(s, sid[0]) == NAO_SESSION_RESIDENT);
        CHECK(settle(s, sid[1]) == NAO_SESSION_RESIDENT);
        CHECK(settle(s, sid[2]) == NAO_SESSION_NO_MEMORY);
        CHECK(state_of(s, sid[3]) == NAO_SESSION_QUEUED);  // behind sid[2], in open order
        size_t bytes = 0;
        CHECK(s.session_info(sid[0], nullptr, &bytes, nullptr, nullptr) == NAO_OK && bytes == 10000);
        CHECK(ex.used_now() == 20000);
        // releasing one session admits the next in open order, not the one behind it
        CHECK(s.close_session(sid[0]) == NAO_OK);
        CHECK(s.close_session(sid[0]) == NAO_ERR_INVALID_ARG);
        for (int k = 0; k < 20000 && state_of(s, sid[2]) != NAO_SESSION_RESIDENT; ++k) {
            (void)s.step(nullptr, nullptr);
            std::this_thread::sleep_for(std::chrono::microseconds(100));
        }
        CHECK(state_of(s, sid[2]) == NAO_SESSION_RESIDENT);
        CHECK(state_of(s, sid[0]) == NAO_SESSION_CLOSED);
        CHECK(state_of(s, sid[3]) == NAO_SESSION_NO_MEMORY || state_of(s, sid[3]) == NAO_SESSION_QUEUED);
        // a session larger than the whole budget fails with its requests
        CHECK(s.close_session(sid[3]) == NAO_OK);  // queued, no requests: gone at once
        CHECK(state_of(s, sid[3]) == NAO_SESSION_CLOSED);
        CHECK(s.open_session(&big.d, 1000, big.pxyz.data(), big.pw.data(), 256, &huge) == NAO_OK);
        double D = 1.0, v = 1.0;
        uint64_t tk = 0;
        const nao_status sst = s.submit(huge, &D, NAO_MEM_HOST, &v, NAO_MEM_HOST, &tk);
        // it waits while resident sessions could make room; once none is left it fails
        for (int k = 0; k < 200; ++k) {
            (void)s.step(nullptr, nullptr);
            std::this_thread::sleep_for(std::chrono::microseconds(100));
        }
        CHECK(state_of(s, huge) == NAO_SESSION_NO_MEMORY || state_of(s, huge) == NAO_SESSION_QUEUED);
        CHECK(s.close_session(sid[1]) == NAO_OK);
        CHECK(s.close_session(sid[2]) == NAO_OK);
        for (int k = 0; k < 20000 && state_of(s, huge) != NAO_SESSION_FAILED; ++k) {
            (void)s.step(nullptr, nullptr);
            std::this_thread::sleep_for(std::chrono::microseconds(100));
        }
        CHECK(state_of(s, huge) == NAO_SESSION_FAILED);
        if (sst == NAO_OK) CHECK(req_state(s, tk) == NAO_REQ_FAILED);
        // a session whose admission fails for another reason fails too
        int64_t bad;
        CHECK(s.open_session(&a.d, 100, a.pxyz.data(), a.pw.data(), 0, &bad) == NAO_OK);
        CHECK(settle(s, bad) == NAO_SESSION_FAILED);
        CHECK(ex.peak <= ex.budget);
    }
    CHECK(ex.used_now() == 0);  // every admitted session was released
    std::printf("admission and budget: ok (%d admission attempts)\n", ex.admissions.load());
}

void test_continuous_batching()
{
    const int n_slots = 2, per_launch = 3, n_sess = 7, iters = 5;
    MockExec ex(n_slots);
    ex.max_per_launch = per_launch;
    std::vector<uint64_t> all;
    std::vector<std::vector<uint64_t>> by_sess(n_sess);
    std::vector<double> Ds(n_sess * iters), vs(n_sess);
    {
        Scheduler s(&ex, n_slots, per_launch);
        CHECK(s.start() == NAO_OK);
        Structure a(50);
        std::vector<int64_t> sid(n_sess);
        for (int k = 0; k < n_sess; ++k) CHECK(s.open_session(&a.d, 50, a.pxyz.data(), a.pw.data(), 256, &sid[k]) == NAO_OK);
        for (int k = 0; k < n_sess; ++k) CHECK(settle(s, sid[k]) == NAO_SESSION_RESIDENT);
        // iteration i of every session is submitted before iteration i + 1 of any
        for (int i = 0; i < iters; ++i)
            for (int k = 0; k < n_sess; ++k) {
                Ds[k * iters + i] = i + 1;
                vs[k] = k + 1;
                uint64_t tk;
                CHECK(s.submit(sid[k], &Ds[k * iters + i], NAO_MEM_HOST, i == 0 ? &vs[k] : nullptr, NAO_MEM_HOST, &tk) ==
                      NAO_OK);
                all.push_back(tk);
                by_sess[k].push_back(tk);
            }
        int32_t run = -1, wait = -1;
        CHECK(s.step(&run, &wait) == NAO_OK);
        CHECK(run == n_slots * per_launch && wait == n_sess * iters - run);
        drain(s, ex, all);
        for (int k = 0; k < n_sess; ++k) {
            double prev_end = -1.0;
            for (int i = 0; i < iters; ++i) {
                double ts, t0, t1;
                int32_t st;
                CHECK(s.poll(by_sess[k][i], &st, &ts, &t0, &t1) == NAO_OK);
                CHECK(st == NAO_REQ_DONE && ts <= t0 && t0 < t1);
                CHECK(t0 >= prev_end);  // iterations of a session never overlap
                prev_end = t1;
            }
            // the last request's result is readable; an earlier one's was replaced
            double H = 0, n = 0;
            CHECK(s.result(by_sess[k][iters - 1], &H, &n, NAO_MEM_HOST) == NAO_OK);
            CHECK(H == 1000.0 * (k + 1) + iters && n == iters);  // kept v of the first request
            CHECK(s.result(by_sess[k][0], &H, &n, NAO_MEM_HOST) == NAO_ERR_INVALID_ARG);
        }
        // FIFO: the first launch takes the oldest requests (iteration 1 of the first sessions)
        CHECK(ex.launch_tags.size() >= 2);
        for (double tg : ex.launch_tags[0]) CHECK(tg == 1.0);
        for (int k = 0; k < n_sess; ++k) CHECK(s.close_session(sid[k]) == NAO_OK);
        for (int k = 0; k < 20000 && ex.used_now() > 0; ++k) {
            (void)s.step(nullptr, nullptr);
            std::this_thread::sleep_for(std::chrono::microseconds(100));
        }
        CHECK(ex.used_now() == 0);
    }
    std::printf("continuous batching: ok (%d launches for %d requests)\n", ex.launches, n_sess * iters);
}

void test_failures()
{
    MockExec ex(1);
    ex.max_per_launch = 2;
    {
        Scheduler s(&ex, 1, 2);
        CHECK(s.start() == NAO_OK);
        Structure a(10);
        int64_t s1, s2;
        CHECK(s.open_session(&a.d, 10, a.pxyz.data(), a.pw.data(), 256, &s1) == NAO_OK);
        CHECK(s.open_session(&a.d, 10, a.pxyz.data(), a.pw.data(), 256, &s2) == NAO_OK);
        CHECK(settle(s, s1) == NAO_SESSION_RESIDENT && settle(s, s2) == NAO_SESSION_RESIDENT);
        double D[4] = {1, 2, 3, 4}, v = 7;
        uint64_t t1, t2, t3, t4;
        // the first request of a session must bring v
        CHECK(s.submit(s1, &D[0], NAO_MEM_HOST, nullptr, NAO_MEM_HOST, &t1) == NAO_ERR_INVALID_ARG);
        // a launch that fails: its requests fail and their sessions are free again
        CHECK(s.submit(s1, &D[0], NAO_MEM_HOST, &v, NAO_MEM_HOST, &t1) == NAO_OK);
        CHECK(s.submit(s2, &D[0], NAO_MEM_HOST, &v, NAO_MEM_HOST, &t2) == NAO_OK);
        ex.fail_next_launch = NAO_ERR_OUT_OF_MEMORY;
        CHECK(s.step(nullptr, nullptr) == NAO_ERR_OUT_OF_MEMORY);
        CHECK(req_state(s, t1) == NAO_REQ_FAILED && req_state(s, t2) == NAO_REQ_FAILED);
        double H = 0;
        CHECK(s.result(t1, &H, nullptr, NAO_MEM_HOST) == NAO_ERR_NOT_READY);
        // the sessions run again; the failed request's v never reached the device, so a request
        // of s1 without its own v fails at launch, one with v runs
        CHECK(s.submit(s1, &D[1], NAO_MEM_HOST, nullptr, NAO_MEM_HOST, &t3) == NAO_OK);
        CHECK(s.step(nullptr, nullptr) == NAO_ERR_INVALID_ARG);
        CHECK(req_state(s, t3) == NAO_REQ_FAILED);
        CHECK(s.submit(s1, &D[1], NAO_MEM_HOST, &v, NAO_MEM_HOST, &t3) == NAO_OK);
        drain(s, ex, {t3});
        CHECK(req_state(s, t3) == NAO_REQ_DONE);
        CHECK(s.result(t3, &H, nullptr, NAO_MEM_HOST) == NAO_OK && H == 7002.0);
        // a launch whose completion reports a failure
        CHECK(s.submit(s2, &D[2], NAO_MEM_HOST, &v, NAO_MEM_HOST, &t4) == NAO_OK);
        ex.fail_next_poll = NAO_ERR_HIP;
        nao_status last = NAO_OK;
        for (int k = 0; k < 1000 && (req_state(s, t4) == NAO_REQ_WAITING || req_state(s, t4) == NAO_REQ_RUNNING); ++k) {
            const nao_status st = s.step(nullptr, nullptr);
            if (st != NAO_OK) last = st;
            ex.advance(0.25);
        }
        CHECK(req_state(s, t4) == NAO_REQ_FAILED && last == NAO_ERR_HIP);
        CHECK(ex.last_report.find("injected completion failure") != std::string::npos);
        // close with a request queued: it still runs, then the session is released
        uint64_t t5;
        CHECK(s.submit(s2, &D[3], NAO_MEM_HOST, &v, NAO_MEM_HOST, &t5) == NAO_OK);
        CHECK(s.close_session(s2) == NAO_OK);
        CHECK(s.submit(s2, &D[3], NAO_MEM_HOST, &v, NAO_MEM_HOST, &t5) == NAO_ERR_INVALID_ARG);
        drain(s, ex, {t5});
        CHECK(req_state(s, t5) == NAO_REQ_DONE);
        for (int k = 0; k < 20000 && state_of(s, s2) != NAO_SESSION_CLOSED; ++k) {
            (void)s.step(nullptr, nullptr);
            std::this_thread::sleep_for(std::chrono::microseconds(100));
        }
        CHECK(state_of(s, s2) == NAO_SESSION_CLOSED);
        // unknown tickets and sessions, bad arguments
        CHECK(s.poll(999999, nullptr, nullptr, nullptr, nullptr) == NAO_ERR_INVALID_ARG);
        CHECK(s.submit(424242, &D[0], NAO_MEM_HOST, &v, NAO_MEM_HOST, &t5) == NAO_ERR_INVALID_ARG);
        CHECK(s.submit(s1, nullptr, NAO_MEM_HOST, &v, NAO_MEM_HOST, &t5) == NAO_ERR_INVALID_ARG);
        CHECK(s.open_session(nullptr, 10, a.pxyz.data(), a.pw.data(), 256, &s2) == NAO_ERR_INVALID_ARG);
        // shutdown with a launch in flight: the destructor waits for it, then releases s1
        uint64_t t6;
        CHECK(s.submit(s1, &D[2], NAO_MEM_HOST, nullptr, NAO_MEM_HOST, &t6) == NAO_OK);
        CHECK(s.step(nullptr, nullptr) == NAO_OK);
        CHECK(req_state(s, t6) == NAO_REQ_RUNNING);
        ex.finish_all = true;
    }
    CHECK(ex.used_now() == 0);
    std::printf("failures: ok\n");
}

int main()
{
    test_admission_and_budget();
    test_continuous_batching();
    test_failures();
    std::printf("scheduler mock: all ok\n");
    return 0;
}
