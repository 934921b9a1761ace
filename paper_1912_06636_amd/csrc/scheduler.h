// Scheduling core of the serving loop (nao.h, nao_server_*): sessions admitted in open order by
// device footprint, a FIFO of ready requests, execution slots and continuous batching.  Pure
// C++ (no HIP): every device step goes through an executor interface, implemented on the GPU by
// server.cpp and by a mock executor with a virtual clock in the CPU tests.
#pragma once

#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "nao.h"

namespace nao {

// Deep copy of a structure handed to open_session (basis description, points, weights).
struct HostStructure {
    std::vector<double> atom_xyz, rmin, rcut, samples;
    std::vector<int32_t> atom_species, shell_ptr, shell_l, shell_radial;
    nao_basis_desc desc{};
    std::vector<double> xyz, w;
    int32_t max_batch = 0;

    // Copies every array the descriptor points to; false when the descriptor is malformed.
    bool take(const nao_basis_desc* d, int64_t n_points, const double* xyz, const double* w, int32_t max_batch);
    // Points desc at this object's own arrays (after a copy or move).
    void reseat();
    int64_t n_points() const { return (int64_t)w.size(); }
};

// Device resources of a resident session, owned by the executor.
struct SessionRes {
    void* handle = nullptr;  // executor state (system and buffers)
    size_t bytes = 0;        // device footprint
    int64_t n_basis = 0;
    int64_t n_points = 0;
};

// One request of a launch: the session's resources and this iteration's inputs.
struct LaunchItem {
    const SessionRes* res;
    const double* D;
    nao_memspace D_space;
    const double* v;          // NULL: keep the session's last v
    nao_memspace v_space;
};

// The device side as the scheduler sees it.  admit/release run on the builder thread, the
// rest on the thread that drives the scheduler; the two never touch the same slot.
class SchedExec {
public:
    virtual ~SchedExec() = default;
    // Make a structure resident.  NAO_ERR_BUDGET: does not fit now (the scheduler retries after
    // a release); any other failure fails the session.
    virtual nao_status admit(const HostStructure& host, SessionRes& res, std::string& err) = 0;
    virtual void release(SessionRes& res) = 0;
    // Stage the inputs of every item and enqueue one launch for all of them on the slot.  On
    // failure nothing of the launch may still be running when it returns.
    virtual nao_status launch(int slot, const std::vector<LaunchItem>& items, std::string& err) = 0;
    // 1: the slot's launch is done, 0: still running, < 0: a nao_status of a failed launch.
    virtual int poll(int slot, std::string& err) = 0;
    // The slot's launch is done and its requests retired: release per-launch state.
    virtual void retired(int slot) = 0;
    // Copy the session's H and/or n (either may be NULL) to the caller.
    virtual nao_status copy_out(const SessionRes& res, double* H, double* n, nao_memspace space,
                                std::string& err) = 0;
    virtual double now() = 0;
    virtual void report(const std::string& msg) = 0;  // message of the last failing call
};

class Scheduler {
public:
    Scheduler(SchedExec* exec, int n_slots, int max_per_launch);
    ~Scheduler();  // stops the builder and releases every resident session
    nao_status start();  // starts the builder thread

    nao_status open_session(const nao_basis_desc* basis, int64_t n_points, const double* xyz, const double* w,
                            int32_t max_batch, int64_t* session);
    nao_status close_session(int64_t session);
    nao_status session_info(int64_t session, int32_t* state, size_t* bytes, int64_t* n_basis, int64_t* n_points);
    nao_status submit(int64_t session, const double* D, nao_memspace D_space, const double* v, nao_memspace v_space,
                      uint64_t* ticket);
    nao_status step(int32_t* n_running, int32_t* n_waiting);
    nao_status poll(uint64_t ticket, int32_t* state, double* t_submit, double* t_start, double* t_end);
    nao_status result(uint64_t ticket, double* H, double* n, nao_memspace space);

private:
    // PENDING -> BUILDING -> RESIDENT -> RELEASING -> GONE; the builder thread owns BUILDING and
    // RELEASING, the scheduler dispatches RESIDENT sessions.
    enum State { S_PENDING, S_BUILDING, S_RESIDENT, S_RELEASING, S_GONE };
    struct Session {
        State state = S_PENDING;
        HostStructure host;
        SessionRes res;
        int64_t n_points = 0;
        bool close_requested = false;
        bool busy = false;           // a request of this session is running
        bool have_v = false;
        bool no_memory = false;      // its last admission attempt did not fit
        bool failed = false;         // admission failed for another reason
        uint64_t last_started = 0;   // ticket of its latest request that started running
    };
    struct Request {
        int64_t session = 0;
        int32_t state = NAO_REQ_WAITING;
        double t_submit = 0, t_start = 0, t_end = 0;
        const double* D = nullptr;
        nao_memspace D_space = NAO_MEM_HOST;
        const double* v = nullptr;
        nao_memspace v_space = NAO_MEM_HOST;
    };
    struct Slot {
        bool busy = false;
        std::vector<uint64_t> tickets;
    };

    nao_status fail(nao_status st, const std::string& msg);
    bool queued_for(int64_t session) const;
    void fail_requests(const std::vector<uint64_t>& tickets, double t);
    nao_status retire();
    nao_status dispatch(int slot);
    void builder_loop();

    SchedExec* exec_;
    int max_per_launch_;
    std::mutex mu_;
    std::condition_variable cv_;
    std::thread builder_;
    bool stop_ = false;
    uint64_t releases_ = 0;
    std::vector<Slot> slots_;
    std::map<int64_t, Session> sessions_;
    std::deque<int64_t> pending_;   // sessions waiting for admission, in open order
    std::deque<uint64_t> ready_;    // waiting requests, in submit order
    std::unordered_map<uint64_t, Request> reqs_;
    uint64_t next_ticket_ = 1;
    int64_t next_session_ = 1;
};

}  // namespace nao
