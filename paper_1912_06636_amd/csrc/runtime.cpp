// Host runtime behind the C ABI (nao.h): contexts with an HBM budget, resident systems,
// execution groups and blocks, and the launch sequences of the API calls.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include <hip/hip_runtime_api.h>
#include <sys/stat.h>
#include <unistd.h>

#include "devtypes.h"
#include "internal.h"
#include "nao.h"
#include "plan.h"

using namespace nao;

namespace {

thread_local std::string g_thread_error;

struct Fail {
    nao_status st;
    std::string msg;
};

}  // namespace

// ------------------------------------------------------------------------------------------
// context

struct nao_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    size_t budget = 0;
    size_t used = 0;
    bool failed = false;
    std::mutex err_mu;           // err may be set from a server's builder thread
    std::string err;
    double* scratch = nullptr;   // basis values of one block of units
    size_t scratch_elems = 0;
    void* gscratch = nullptr;    // gradients of the basis values of one block (density gradient)
    size_t gscratch_bytes = 0;
    size_t scratch_cap_elems = 0;
    double* wsum = nullptr;      // WSUM_BLOCKS partials + 1 result
    // Overlap of the basis evaluation of block k + 1 with the contraction of block k (density
    // update and Hamiltonian): odd blocks take their basis values in a second buffer, the basis
    // launches run on a second stream (default priority), and events order the two (see
    // run_blocks).  Off with NAO_OVERLAP=0, or when the second buffer does not fit the budget.
    bool overlap = true;
    hipStream_t stream2 = nullptr;
    double* scratch2 = nullptr;
    size_t scratch2_elems = 0;
    void* gscratch2 = nullptr;           // second buffer of gscratch (the extended operations)
    size_t gscratch2_bytes = 0;
    hipEvent_t ev_start = nullptr;       // the context stream's work before the operation
    hipEvent_t ev_ready[2] = {};         // basis values of the last block of each buffer written
    hipEvent_t ev_done[2] = {};          // contraction of the last block of each buffer done
    int n_systems = 0;
    // per-kernel timing
    bool prof = false;
    struct Rec {
        const char* name;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    int n_cu = 256;
    int64_t persistent_per_cu = 0;       // workgroups per CU of a multi-structure launch (0 = one
                                         // workgroup per item, dispatched by the hardware)
    std::vector<std::pair<void*, size_t>> spare;  // device buffers of retired launch plans, for reuse
    std::vector<struct ManyPlan*> many;  // launch plans of nao_run_many (captured graphs)
    std::vector<std::pair<hipEvent_t, struct ManyPlan*>> inflight;  // eager plans still running
};

namespace {

void set_err(nao_ctx c, const std::string& m)
{
    if (c) {
        std::lock_guard<std::mutex> lk(c->err_mu);
        c->err = m;
    }
    g_thread_error = m;
}

nao_status hip_fail(nao_ctx c, hipError_t e, const char* what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    if (c) c->failed = true;
    set_err(c, m);
    return NAO_ERR_HIP;
}

#define HIP_TRY(ctx, expr)                                   \
    do {                                                     \
        hipError_t e__ = (expr);                             \
        if (e__ != hipSuccess) return hip_fail(ctx, e__, #expr); \
    } while (0)

hipEvent_t take_event(nao_ctx c)
{
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch through f(); when profiling, bracket it with events on the stream it launches on.
template <typename F>
hipError_t timed(nao_ctx c, const char* name, hipStream_t st, F&& f)
{
    if (!c->prof) return f();
    hipEvent_t a = take_event(c), b = take_event(c);
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, st);
    if (e != hipSuccess) return e;
    e = f();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, st);
    c->recs.push_back({name, a, b});
    return e;
}

#define LAUNCH(ctx, name, call) HIP_TRY(ctx, timed(ctx, name, (ctx)->stream, [&]() { return (call); }))
#define LAUNCH_ON(ctx, name, st, call) HIP_TRY(ctx, timed(ctx, name, st, [&]() { return (call); }))

nao_status dev_alloc(nao_ctx c, size_t bytes, void** out)
{
    *out = nullptr;
    if (bytes == 0) return NAO_OK;
    if (c->budget && c->used + bytes > c->budget) {
        set_err(c, "HBM budget exceeded: need " + std::to_string(bytes) + " B, used " + std::to_string(c->used) +
                       " of " + std::to_string(c->budget));
        return NAO_ERR_BUDGET;
    }
    hipError_t e = hipMalloc(out, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *out = nullptr;
        set_err(c, std::string("hipMalloc of ") + std::to_string(bytes) + " B failed: " + hipGetErrorString(e));
        return NAO_ERR_OUT_OF_MEMORY;
    }
    c->used += bytes;
    return NAO_OK;
}

void dev_free(nao_ctx c, void* p, size_t bytes)
{
    if (!p) return;
    (void)hipFree(p);
    c->used -= std::min(c->used, bytes);
}

struct DevArray {
    void* p = nullptr;
    size_t bytes = 0;
    template <typename T> T* as() const { return static_cast<T*>(p); }
};

nao_status upload(nao_ctx c, DevArray& a, const void* src, size_t bytes)
{
    if (a.bytes != bytes) {
        dev_free(c, a.p, a.bytes);
        a.p = nullptr;
        a.bytes = 0;
        nao_status s = dev_alloc(c, bytes, &a.p);
        if (s != NAO_OK) return s;
        a.bytes = bytes;
    }
    if (bytes) HIP_TRY(c, hipMemcpyAsync(a.p, src, bytes, hipMemcpyHostToDevice, c->stream));
    return NAO_OK;
}

nao_status ensure(nao_ctx c, DevArray& a, size_t bytes)
{
    if (a.bytes >= bytes && a.p) return NAO_OK;
    dev_free(c, a.p, a.bytes);
    a.p = nullptr;
    a.bytes = 0;
    nao_status s = dev_alloc(c, bytes, &a.p);
    if (s == NAO_OK) a.bytes = bytes;
    return s;
}

// Launch-plan buffers come from a per-context pool: hipMalloc is slow and hipFree may wait
// for the whole device, which would stall the work other streams have in flight.
nao_status pool_take(nao_ctx c, DevArray& a, size_t bytes)
{
    bytes = std::max<size_t>(bytes, 256);
    int best = -1;
    for (size_t i = 0; i < c->spare.size(); ++i)
        if (c->spare[i].second >= bytes && (best < 0 || c->spare[i].second < c->spare[best].second)) best = (int)i;
    if (best >= 0) {
        a.p = c->spare[best].first;
        a.bytes = c->spare[best].second;
        c->spare.erase(c->spare.begin() + best);
        return NAO_OK;
    }
    size_t r = 256;  // powers of two make reuse likely
    while (r < bytes) r <<= 1;
    nao_status s = dev_alloc(c, r, &a.p);
    a.bytes = s == NAO_OK ? r : 0;
    return s;
}

// Return a buffer whose work has completed (or is ordered before any later use on the stream).
void pool_give(nao_ctx c, DevArray& a)
{
    if (!a.p) return;
    c->spare.push_back({a.p, a.bytes});
    a.p = nullptr;
    a.bytes = 0;
    while (c->spare.size() > 32) {
        dev_free(c, c->spare.front().first, c->spare.front().second);
        c->spare.erase(c->spare.begin());
    }
}

nao_status check_ctx(nao_ctx c)
{
    if (!c) {
        g_thread_error = "context is NULL";
        return NAO_ERR_INVALID_ARG;
    }
    if (c->failed) {
        std::string first;
        {
            std::lock_guard<std::mutex> lk(c->err_mu);
            first = c->err;
        }
        set_err(c, "context is unusable after an earlier HIP failure: " + first);
        return NAO_ERR_HIP;
    }
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    return NAO_OK;
}

size_t scratch_cap_from_env()
{
    size_t mb = 2048;
    if (const char* s = std::getenv("NAO_SCRATCH_MB")) {
        long v = std::atol(s);
        if (v >= 16) mb = (size_t)v;
    }
    return mb * (size_t)1024 * 1024 / sizeof(double);
}

}  // namespace

// ------------------------------------------------------------------------------------------
// system

namespace {

struct Block {
    int64_t unit_begin = 0, unit_count = 0;
    int64_t h_begin = 0, h_count = 0;    // Hamiltonian items over 64-wide tiles
    int64_t hw_begin = 0, hw_count = 0;  // ... over 128-wide tiles (systems with h_tile 128)
    int64_t n_begin = 0, n_count = 0;
    int64_t phi_elems = 0;
};

}  // namespace

struct nao_system_s {
    nao_ctx ctx = nullptr;
    HostBasis basis;
    int64_t n_points = 0;
    int32_t max_batch = 0;
    int32_t batcher = NAO_BATCH_OCTREE;
    int32_t group_max = MAX_UNIT_POINTS;
    int32_t h_tile = TILE;  // width of the Hamiltonian kernel's tiles (64 or 128)
    std::vector<int64_t> perm, batch_ptr, atom_ptr;
    std::vector<int32_t> atoms;
    double work_units = 0.0;
    // groups
    std::vector<Block> blocks;
    int64_t n_units = 0, n_h_items = 0, n_n_items = 0;
    // host copies for the allocation-free Hamiltonian call: every unit, the first 64-wide
    // Hamiltonian item of every unit (n_units + 1 entries), and that call's segment table
    std::vector<DevUnit> h_units;
    std::vector<int64_t> h_item_first;
    std::vector<DevSeg> na_segs;
    // device state
    DevSys dsys{};
    DevArray d_sys, d_px, d_py, d_pz, d_pw, d_perm, d_atoms, d_species, d_shell_ptr, d_shell_l, d_shell_rad,
        d_radial_par, d_spline, d_fn_ptr, d_fn_code;
    DevArray d_units, d_unit_atoms, d_unit_cols, d_unit_fn, d_h_items, d_hw_items, d_n_items;
    DevArray d_wv, d_v, d_D, d_H, d_n, d_gn, d_a, d_wa, d_segs, d_Q, d_fb, d_atom_first, d_F;
    // resident basis values (opt-in): every block's values kept across operations
    bool resident = false;
    int res_kind = -1;              // -1: not evaluated, 0: FP64 values, 1: FP32 values
    std::vector<int64_t> res_off;   // element offset of every block
    DevArray d_phi_res;
    int spline_lds = 0;  // doubles of spline table staged in LDS by the basis kernel (0 = not staged)
};

nao_status grow_scratch(nao_ctx c, size_t elems);

namespace {

size_t system_bytes(const nao_system_s* s)
{
    const DevArray* arr[] = {&s->d_sys, &s->d_px, &s->d_py, &s->d_pz, &s->d_pw, &s->d_perm, &s->d_atoms,
                             &s->d_species, &s->d_shell_ptr, &s->d_shell_l, &s->d_shell_rad, &s->d_radial_par,
                             &s->d_spline, &s->d_fn_ptr, &s->d_fn_code, &s->d_units, &s->d_unit_atoms, &s->d_unit_cols, &s->d_unit_fn,
                             &s->d_h_items, &s->d_hw_items, &s->d_n_items, &s->d_wv, &s->d_v, &s->d_D, &s->d_H, &s->d_n,
                             &s->d_gn, &s->d_a, &s->d_wa, &s->d_segs, &s->d_Q, &s->d_fb, &s->d_atom_first,
                             &s->d_F, &s->d_phi_res};
    size_t t = 0;
    for (auto* a : arr) t += a->bytes;
    return t;
}

void free_all(nao_system_s* s)
{
    DevArray* arr[] = {&s->d_sys, &s->d_px, &s->d_py, &s->d_pz, &s->d_pw, &s->d_perm, &s->d_atoms,
                       &s->d_species, &s->d_shell_ptr, &s->d_shell_l, &s->d_shell_rad, &s->d_radial_par,
                       &s->d_spline, &s->d_fn_ptr, &s->d_fn_code, &s->d_units, &s->d_unit_atoms, &s->d_unit_cols, &s->d_unit_fn,
                       &s->d_h_items, &s->d_hw_items, &s->d_n_items, &s->d_wv, &s->d_v, &s->d_D, &s->d_H, &s->d_n, &s->d_gn, &s->d_a, &s->d_wa, &s->d_segs,
                       &s->d_Q, &s->d_fb, &s->d_atom_first, &s->d_F, &s->d_phi_res};
    for (auto* a : arr) {
        dev_free(s->ctx, a->p, a->bytes);
        a->p = nullptr;
        a->bytes = 0;
    }
}

int32_t round_up(int32_t x, int32_t m) { return (x + m - 1) / m * m; }

// Resident basis values: one slot per block (8 bytes per value, FP32 modes use half), marked
// not evaluated.  When the new layout does not fit the budget the mode turns off and the status
// is returned.
nao_status resident_layout(nao_system_s* s)
{
    s->res_kind = -1;
    if (!s->resident) return NAO_OK;
    s->res_off.clear();
    int64_t total = 0;
    for (const Block& b : s->blocks) {
        s->res_off.push_back(total);
        total += b.phi_elems;
    }
    const nao_status st = ensure(s->ctx, s->d_phi_res, (size_t)std::max<int64_t>(1, total) * sizeof(double));
    if (st != NAO_OK) {
        dev_free(s->ctx, s->d_phi_res.p, s->d_phi_res.bytes);
        s->d_phi_res.p = nullptr;
        s->d_phi_res.bytes = 0;
        s->resident = false;
        s->res_off.clear();
    }
    return st;
}

// Build execution groups, split them into scratch-sized blocks and upload units and items.
nao_status build_groups(nao_system_s* s)
{
    nao_ctx c = s->ctx;
    std::vector<Unit> units;
    std::vector<int32_t> uat, ucol;
    make_groups(s->basis, s->batch_ptr, s->atom_ptr, s->atoms, s->group_max, units, uat, ucol);
    std::vector<DevUnit> du(units.size());
    std::vector<int32_t> ufn;
    std::vector<HItem> hitems, hwitems;
    std::vector<NItem> nitems;
    std::vector<int64_t> item_first;
    s->blocks.clear();
    Block cur;
    int64_t off = 0;
    const int64_t cap = (int64_t)c->scratch_cap_elems;
    for (size_t k = 0; k < units.size(); ++k) {
        const Unit& u = units[k];
        DevUnit& d = du[k];
        d.point_begin = u.point_begin;
        d.atom_begin = u.atom_begin;
        d.fn_begin = (int64_t)ufn.size();
        d.n_points = u.n_points;
        d.n_atoms = u.n_atoms;
        d.m = u.m;
        d.ld = round_up(u.m, std::max<int32_t>(TILE, s->h_tile));
        for (int32_t q = 0; q < u.n_atoms; ++q) {
            const int32_t a = uat[u.atom_begin + q];
            for (int64_t f = s->basis.atom_first[a]; f < s->basis.atom_first[a + 1]; ++f) ufn.push_back((int32_t)f);
        }
        const int64_t elems = (int64_t)d.n_points * d.ld;
        if (elems > cap) return (set_err(c, "one execution group exceeds the scratch size"), NAO_ERR_INTERNAL);
        if (off + elems > cap) {
            s->blocks.push_back(cur);
            cur = Block();
            cur.unit_begin = (int64_t)k;
            cur.h_begin = (int64_t)hitems.size();
            cur.hw_begin = (int64_t)hwitems.size();
            cur.n_begin = (int64_t)nitems.size();
            off = 0;
        }
        d.out_offset = off;
        off += elems;
        cur.phi_elems = off;
        cur.unit_count++;
        item_first.push_back((int64_t)hitems.size());
        const int nt = (d.m + TILE - 1) / TILE;  // tiles that hold at least one column
        for (int tj = 0; tj < nt; ++tj) {
            for (int ti = 0; ti <= tj; ++ti) hitems.push_back(HItem{(int32_t)k, (int16_t)ti, (int16_t)tj});
            nitems.push_back(NItem{(int32_t)k, tj});
        }
        if (s->h_tile == 128) {
            const int ntw = (d.m + 127) / 128;
            for (int tj = 0; tj < ntw; ++tj)
                for (int ti = 0; ti <= tj; ++ti) hwitems.push_back(HItem{(int32_t)k, (int16_t)ti, (int16_t)tj});
        }
        cur.h_count = (int64_t)hitems.size() - cur.h_begin;
        cur.hw_count = (int64_t)hwitems.size() - cur.hw_begin;
        cur.n_count = (int64_t)nitems.size() - cur.n_begin;
    }
    if (cur.unit_count) s->blocks.push_back(cur);
    item_first.push_back((int64_t)hitems.size());
    s->n_units = (int64_t)units.size();
    s->n_h_items = (int64_t)hitems.size();
    s->n_n_items = (int64_t)nitems.size();
    if (hitems.size() > 0x7fffffffu) return (set_err(c, "too many work items"), NAO_ERR_INTERNAL);
    nao_status st;
    if ((st = upload(c, s->d_units, du.data(), du.size() * sizeof(DevUnit))) != NAO_OK) return st;
    if ((st = upload(c, s->d_unit_atoms, uat.data(), uat.size() * sizeof(int32_t))) != NAO_OK) return st;
    if ((st = upload(c, s->d_unit_cols, ucol.data(), ucol.size() * sizeof(int32_t))) != NAO_OK) return st;
    if ((st = upload(c, s->d_unit_fn, ufn.data(), ufn.size() * sizeof(int32_t))) != NAO_OK) return st;
    if ((st = upload(c, s->d_h_items, hitems.data(), hitems.size() * sizeof(HItem))) != NAO_OK) return st;
    if ((st = upload(c, s->d_hw_items, hwitems.data(), hwitems.size() * sizeof(HItem))) != NAO_OK) return st;
    if ((st = upload(c, s->d_n_items, nitems.data(), nitems.size() * sizeof(NItem))) != NAO_OK) return st;
    if ((st = ensure(c, s->d_segs, std::max<size_t>(1, s->blocks.size()) * sizeof(DevSeg))) != NAO_OK) return st;
    size_t need = 0;
    for (const Block& b : s->blocks) need = std::max(need, (size_t)b.phi_elems);
    if ((st = grow_scratch(c, need)) != NAO_OK) return st;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    s->h_units = std::move(du);
    s->h_item_first = std::move(item_first);
    return resident_layout(s);
}

// Hamiltonian segments use the 128-wide items when wide is set (FP64 / FP32 on systems with
// h_tile 128), else the 64-wide ones.
DevSeg make_seg(const nao_system_s* s, const Block& b, bool ham, bool wide = false)
{
    DevSeg g{};
    g.sys = s->d_sys.as<DevSys>();
    g.units = s->d_units.as<DevUnit>();
    g.unit_atoms = s->d_unit_atoms.as<int32_t>();
    g.unit_cols = s->d_unit_cols.as<int32_t>();
    g.unit_fn = s->d_unit_fn.as<int32_t>();
    g.items = ham ? (wide ? (const void*)s->d_hw_items.p : (const void*)s->d_h_items.p) : (const void*)s->d_n_items.p;
    g.phi = s->ctx->scratch;
    g.ld = s->basis.n_basis;
    g.unit_begin = b.unit_begin;
    g.unit_count = b.unit_count;
    g.unit_prefix = 0;
    g.item_begin = ham ? (wide ? b.hw_begin : b.h_begin) : b.n_begin;
    g.item_count = ham ? (wide ? b.hw_count : b.h_count) : b.n_count;
    g.item_prefix = 0;
    return g;
}

bool finite_all(const double* p, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

}  // namespace


// ------------------------------------------------------------------------------------------
// many structures per launch sequence

static Mode exec_mode(nao_ctx, nao_precision p) { return (Mode)p; }

static const char* kname(bool ham, nao_precision p)
{
    static const char* h[] = {"h_f64", "h_f32", "h_bf16x3", "h_bf16x6"};
    static const char* n[] = {"n_f64", "n_f32", "n_bf16x3", "n_bf16x6"};
    return ham ? h[p] : n[p];
}


struct ManyPlan {
    std::vector<const void*> key;  // precision, then (sys, op, in, out) per entry
    struct Chunk {
        size_t all_off = 0, all_n = 0, h_off[2] = {0, 0}, h_n[2] = {0, 0}, n_off = 0, n_n = 0;
        int64_t units = 0, h_items[2] = {0, 0}, n_items = 0;  // H lists: 64- and 128-wide tiles
    };
    std::vector<Chunk> chunks;
    std::vector<DevSeg> segs;
    std::vector<nao_work> entries;
    std::vector<int64_t> wv_off;  // per entry: offset into the w*v arena (H entries)
    nao_precision prec = NAO_FP64;
    bool overlap = false;  // odd chunks in the second buffer, basis launches on the second stream
    DevArray d_segs, d_wv;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

void many_free(nao_ctx c, ManyPlan* m)
{
    if (m->exec) (void)hipGraphExecDestroy(m->exec);
    if (m->graph) (void)hipGraphDestroy(m->graph);
    pool_give(c, m->d_segs);
    pool_give(c, m->d_wv);
    delete m;
}

// Free eager launch plans whose work has finished (all of them when wait is set).
void many_retire(nao_ctx c, bool wait)
{
    std::vector<std::pair<hipEvent_t, ManyPlan*>> keep;
    for (auto& f : c->inflight) {
        if (wait) (void)hipEventSynchronize(f.first);
        if (wait || hipEventQuery(f.first) == hipSuccess) {
            many_free(c, f.second);
            c->pool.push_back(f.first);
        } else {
            keep.push_back(f);
        }
    }
    c->inflight.swap(keep);
}

// Drop cached launch plans that mention sys (or all of them for sys = NULL).
void many_forget(nao_ctx c, const nao_system_s* sys)
{
    (void)hipStreamSynchronize(c->stream);
    many_retire(c, true);
    std::vector<ManyPlan*> keep;
    for (ManyPlan* m : c->many) {
        bool uses = sys == nullptr;
        for (const nao_work& w : m->entries) uses = uses || w.sys == sys;
        if (uses) many_free(c, m);
        else keep.push_back(m);
    }
    c->many.swap(keep);
}

}  // namespace

// Replace the context's basis scratch by one of at least `elems` values.  Captured launch plans
// hold the old buffer's address, so they are dropped first (after the work in flight is done).
nao_status grow_scratch(nao_ctx c, size_t elems)
{
    if (elems <= c->scratch_elems) return NAO_OK;
    many_forget(c, nullptr);
    dev_free(c, c->scratch, c->scratch_elems * sizeof(double));
    c->scratch = nullptr;
    c->scratch_elems = 0;
    void* p = nullptr;
    const nao_status st = dev_alloc(c, elems * sizeof(double), &p);
    if (st != NAO_OK) return st;
    c->scratch = static_cast<double*>(p);
    c->scratch_elems = elems;
    return NAO_OK;
}

// Second stream, events and a second basis buffer of `elems` values for the overlapped block
// loops (run_blocks, nao_run_many); false (and the loop runs on one stream) when overlap is off,
// the buffer would exceed the budget or a resource cannot be had.
static bool overlap_ready(nao_ctx c, size_t elems)
{
    if (!c->overlap) return false;
    if (!c->stream2) {
        bool ok = hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking) == hipSuccess;
        for (hipEvent_t* e : {&c->ev_start, &c->ev_ready[0], &c->ev_ready[1], &c->ev_done[0], &c->ev_done[1]})
            ok = ok && hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            c->overlap = false;
            return false;
        }
    }
    if (elems > c->scratch2_elems) {
        const size_t bytes = elems * sizeof(double), held = c->scratch2_elems * sizeof(double);
        if (c->budget && c->used - held + bytes > c->budget) return false;
        if (c->scratch2) {  // earlier operations may still read or write it, captured plans hold it
            many_forget(c, nullptr);
            (void)hipStreamSynchronize(c->stream2);
            (void)hipStreamSynchronize(c->stream);
        }
        dev_free(c, c->scratch2, held);
        c->scratch2 = nullptr;
        c->scratch2_elems = 0;
        void* p = nullptr;
        if (dev_alloc(c, bytes, &p) != NAO_OK) return false;
        c->scratch2 = static_cast<double*>(p);
        c->scratch2_elems = elems;
    }
    return true;
}

// A second extra-value buffer of `bytes` for the overlapped loops of the extended operations;
// false (serial loop) when it would exceed the budget or cannot be had.
static bool overlap_gscratch(nao_ctx c, size_t bytes)
{
    if (bytes <= c->gscratch2_bytes) return true;
    if (c->budget && c->used - c->gscratch2_bytes + bytes > c->budget) return false;
    if (c->gscratch2) {  // earlier operations may still read or write it
        (void)hipStreamSynchronize(c->stream2);
        (void)hipStreamSynchronize(c->stream);
    }
    dev_free(c, c->gscratch2, c->gscratch2_bytes);
    c->gscratch2 = nullptr;
    c->gscratch2_bytes = 0;
    void* p = nullptr;
    if (dev_alloc(c, bytes, &p) != NAO_OK) return false;
    c->gscratch2 = p;
    c->gscratch2_bytes = bytes;
    return true;
}

// The block loop of an operation: per block k, basis(k, stream) (skipped when bname is null)
// and then contract(k) on the context stream.  With ovl, block k's basis launch runs on the
// second stream, after the context stream's work before the loop and after the contraction of
// block k - 2 (the last reader of its buffers), and block k's contraction waits for it; the
// context stream thus ends after every launch of the loop.
template <typename FB, typename FC>
static nao_status block_loop(nao_ctx c, size_t n_blocks, bool ovl, const char* bname, const char* cname, FB&& basis,
                             FC&& contract)
{
    if (ovl) {
        HIP_TRY(c, hipEventRecord(c->ev_start, c->stream));
        HIP_TRY(c, hipStreamWaitEvent(c->stream2, c->ev_start, 0));
    }
    for (size_t k = 0; k < n_blocks; ++k) {
        const int buf = (int)(k & 1);
        if (ovl) {
            if (k >= 2) HIP_TRY(c, hipStreamWaitEvent(c->stream2, c->ev_done[buf], 0));
            LAUNCH_ON(c, bname, c->stream2, basis(k, c->stream2));
            HIP_TRY(c, hipEventRecord(c->ev_ready[buf], c->stream2));
            HIP_TRY(c, hipStreamWaitEvent(c->stream, c->ev_ready[buf], 0));
        } else if (bname) {
            LAUNCH(c, bname, basis(k, c->stream));
        }
        LAUNCH(c, cname, contract(k));
        if (ovl) HIP_TRY(c, hipEventRecord(c->ev_done[buf], c->stream));
    }
    return NAO_OK;
}

namespace {

nao_status many_build(nao_ctx c, const nao_work* work, int64_t n_work, nao_precision prec, ManyPlan* m)
{
    m->prec = prec;
    m->entries.assign(work, work + n_work);
    int64_t wv_total = 0;
    for (const nao_work& w : m->entries) {
        m->wv_off.push_back(wv_total);
        if (w.op == 0) wv_total += w.sys->n_points;
    }
    nao_status st = pool_take(c, m->d_wv, std::max<int64_t>(1, wv_total) * sizeof(double));
    if (st != NAO_OK) return st;
    // the scratch must hold the largest block of every system (systems may come from other
    // contexts on this device)
    int64_t need = 0;
    for (const nao_work& w : m->entries)
        for (const Block& b : w.sys->blocks) need = std::max(need, b.phi_elems);
    if ((st = grow_scratch(c, (size_t)need)) != NAO_OK) return st;
    // one segment per (entry, block); consecutive segments share a chunk while their basis
    // values fit the scratch
    struct Pending { DevSeg g; bool ham; int64_t phi; int32_t h_tile; };
    std::vector<std::vector<Pending>> chunks(1);
    int64_t off = 0;
    for (size_t e = 0; e < m->entries.size(); ++e) {
        const nao_work& w = m->entries[e];
        nao_system_s* s = w.sys;
        const bool ham = w.op == 0;
        for (const Block& b : s->blocks) {
            if (off + b.phi_elems > (int64_t)c->scratch_elems && off > 0) {
                chunks.emplace_back();
                off = 0;
            }
            const bool wide = ham && s->h_tile == 128 && (prec == NAO_FP64 || prec == NAO_FP32);
            DevSeg g = make_seg(s, b, ham, wide);
            if (ham) {
                g.wv = m->d_wv.as<double>() + m->wv_off[e];
                g.H = const_cast<double*>(w.out);
            } else {
                g.D = w.in;
                g.n = w.out;
            }
            chunks.back().push_back(Pending{g, ham, off, wide ? 128 : TILE});
            off += b.phi_elems;
        }
    }
    const bool f32 = prec != NAO_FP64;
    const size_t esz = f32 ? sizeof(float) : sizeof(double);
    size_t n_chunks = 0;
    for (auto& ch : chunks) n_chunks += !ch.empty();
    m->overlap = n_chunks > 1 && overlap_ready(c, c->scratch_elems);
    for (auto& ch : chunks) {
        if (ch.empty()) continue;
        ManyPlan::Chunk k;
        k.all_off = m->segs.size();
        double* buf = m->overlap && (m->chunks.size() & 1) ? c->scratch2 : c->scratch;
        for (Pending& p : ch) {
            DevSeg g = p.g;
            g.phi = static_cast<char*>(static_cast<void*>(buf)) + p.phi * esz;
            g.unit_prefix = k.units;
            k.units += g.unit_count;
            m->segs.push_back(g);
        }
        k.all_n = m->segs.size() - k.all_off;
        for (int pass = 0; pass < 3; ++pass) {  // H with 64-wide tiles, H with 128-wide, density
            const bool ham = pass < 2;
            const int want_tile = pass == 1 ? 128 : TILE;
            const size_t o = m->segs.size();
            int64_t items = 0;
            for (size_t q = 0; q < k.all_n; ++q) {
                if (ch[q].ham != ham || (ham && ch[q].h_tile != want_tile)) continue;
                DevSeg g = m->segs[k.all_off + q];
                g.item_prefix = items;
                items += g.item_count;
                m->segs.push_back(g);
            }
            if (ham) {
                k.h_off[pass] = o;
                k.h_n[pass] = m->segs.size() - o;
                k.h_items[pass] = items;
            } else {
                k.n_off = o;
                k.n_n = m->segs.size() - o;
                k.n_items = items;
            }
        }
        m->chunks.push_back(k);
    }
    const size_t seg_bytes = std::max<size_t>(1, m->segs.size()) * sizeof(DevSeg);
    if ((st = pool_take(c, m->d_segs, seg_bytes)) != NAO_OK) return st;
    // the host table lives as long as the plan; the copy is ordered before the plan's kernels
    if (!m->segs.empty())
        HIP_TRY(c, hipMemcpyAsync(m->d_segs.p, m->segs.data(), m->segs.size() * sizeof(DevSeg), hipMemcpyHostToDevice,
                                  c->stream));
    return NAO_OK;
}

nao_status many_enqueue(nao_ctx c, ManyPlan* m)
{
    const Mode mode = exec_mode(c, m->prec);
    const bool f32 = m->prec != NAO_FP64;
    const bool staged = true;
    const int64_t grid = (int64_t)c->n_cu * c->persistent_per_cu;
    for (size_t e = 0; e < m->entries.size(); ++e) {
        const nao_work& w = m->entries[e];
        nao_system_s* s = w.sys;
        if (w.op == 0) {
            LAUNCH(c, "fill", launch_fill(w.out, s->basis.n_basis * s->basis.n_basis, 0.0, c->stream));
            LAUNCH(c, "wv", launch_wv(s->d_pw.as<double>(), s->d_perm.as<int32_t>(), w.in,
                                      m->d_wv.as<double>() + m->wv_off[e], s->n_points, c->stream));
        } else {
            LAUNCH(c, "fill", launch_fill(w.out, s->n_points, 0.0, c->stream));
        }
    }
    const DevSeg* d = m->d_segs.as<DevSeg>();
    // stage the spline tables in LDS only if every system's table fits
    int lds = 0;
    bool all_fit = true;
    for (const nao_work& w : m->entries) {
        all_fit = all_fit && w.sys->spline_lds > 0;
        lds = std::max(lds, w.sys->spline_lds);
    }
    if (!all_fit) lds = 0;
    // with overlap, as in run_blocks: chunk k's basis launch on the second stream after the
    // contraction of chunk k - 2 (the last reader of its buffer), its contractions after it (the
    // fork and join are events, which a captured graph records as dependencies)
    const bool ovl = m->overlap;
    if (ovl) {
        HIP_TRY(c, hipEventRecord(c->ev_start, c->stream));
        HIP_TRY(c, hipStreamWaitEvent(c->stream2, c->ev_start, 0));
    }
    for (size_t ki = 0; ki < m->chunks.size(); ++ki) {
        const auto& k = m->chunks[ki];
        const int buf = (int)(ki & 1);
        if (ovl) {
            if (ki >= 2) HIP_TRY(c, hipStreamWaitEvent(c->stream2, c->ev_done[buf], 0));
            LAUNCH_ON(c, f32 ? "basis_f32" : "basis_f64", c->stream2,
                      launch_basis(d + k.all_off, (int)k.all_n, k.units, lds, f32, c->stream2, grid));
            HIP_TRY(c, hipEventRecord(c->ev_ready[buf], c->stream2));
            HIP_TRY(c, hipStreamWaitEvent(c->stream, c->ev_ready[buf], 0));
        } else if (staged) {
            LAUNCH(c, f32 ? "basis_f32" : "basis_f64",
                   launch_basis(d + k.all_off, (int)k.all_n, k.units, lds, f32, c->stream, grid));
        }
        for (int t = 0; t < 2; ++t)
            if (k.h_n[t])
                LAUNCH(c, kname(true, m->prec), launch_h(mode, d + k.h_off[t], (int)k.h_n[t], k.h_items[t], c->stream,
                                                         grid, t == 0 ? TILE : 128));
        if (k.n_n) LAUNCH(c, kname(false, m->prec), launch_n(mode, d + k.n_off, (int)k.n_n, k.n_items, c->stream, grid));
        if (ovl) HIP_TRY(c, hipEventRecord(c->ev_done[buf], c->stream));
    }
    for (const nao_work& w : m->entries)
        if (w.op == 0) LAUNCH(c, "mirror", launch_mirror(w.out, w.sys->basis.n_basis, c->stream));
    return NAO_OK;
}

nao_status run_many_impl(nao_ctx c, const nao_work* work, int64_t n_work, nao_precision prec, bool capture)
{
    many_retire(c, false);
    std::vector<const void*> key;
    key.push_back(reinterpret_cast<const void*>((uintptr_t)prec + 1));
    for (int64_t k = 0; k < n_work; ++k) {
        key.push_back(work[k].sys);
        key.push_back(reinterpret_cast<const void*>((uintptr_t)work[k].op));
        key.push_back(work[k].in);
        key.push_back(work[k].out);
    }
    if (capture) {
        for (ManyPlan* m : c->many)
            if (m->key == key && m->exec) {
                HIP_TRY(c, timed(c, "graph", c->stream, [&]() { return hipGraphLaunch(m->exec, c->stream); }));
                return NAO_OK;
            }
    }
    ManyPlan* m = new ManyPlan();
    m->key = key;
    nao_status st = many_build(c, work, n_work, prec, m);
    if (st != NAO_OK) {
        many_free(c, m);
        return st;
    }
    if (!capture) {
        st = many_enqueue(c, m);
        if (st != NAO_OK) {
            (void)hipStreamSynchronize(c->stream);
            many_free(c, m);
            return st;
        }
        // the plan's device arrays must outlive the enqueued work: retire it once its event fires
        hipEvent_t ev = take_event(c);
        if (!ev) {
            (void)hipStreamSynchronize(c->stream);
            many_free(c, m);
            return NAO_OK;
        }
        HIP_TRY(c, hipEventRecord(ev, c->stream));
        c->inflight.push_back({ev, m});
        return NAO_OK;
    }
    const bool prof = c->prof;
    c->prof = false;  // no event records inside a captured graph
    hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        st = many_enqueue(c, m);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(c->stream, &g);
        m->graph = g;
        if (st == NAO_OK && e2 != hipSuccess) st = hip_fail(c, e2, "hipStreamEndCapture");
        if (st == NAO_OK) {
            e = hipGraphInstantiate(&m->exec, m->graph, nullptr, nullptr, 0);
            if (e != hipSuccess) st = hip_fail(c, e, "hipGraphInstantiate");
        }
    } else {
        st = hip_fail(c, e, "hipStreamBeginCapture");
    }
    c->prof = prof;
    if (st != NAO_OK) {
        many_free(c, m);
        return st;
    }
    if (c->many.size() >= 8) {
        (void)hipStreamSynchronize(c->stream);
        many_free(c, c->many.front());
        c->many.erase(c->many.begin());
    }
    c->many.push_back(m);
    HIP_TRY(c, timed(c, "graph", c->stream, [&]() { return hipGraphLaunch(m->exec, c->stream); }));
    return NAO_OK;
}

}  // namespace

// ------------------------------------------------------------------------------------------
// helpers for the serving core

namespace nao {

nao_status ctx_alloc(nao_ctx c, size_t bytes, void** out) { return dev_alloc(c, bytes, out); }
void ctx_free(nao_ctx c, void* p, size_t bytes) { dev_free(c, p, bytes); }
hipStream_t ctx_stream(nao_ctx c) { return c->stream; }
int ctx_device(nao_ctx c) { return c->device; }
void ctx_set_error(nao_ctx c, const std::string& msg) { set_err(c, msg); }
size_t system_device_bytes(nao_system s) { return system_bytes(s); }

}  // namespace nao

// ------------------------------------------------------------------------------------------
// C ABI

extern "C" {

nao_status nao_ctx_create(int device, void* hip_stream, size_t hbm_budget_bytes, nao_ctx* out)
{
    if (!out) {
        g_thread_error = "out is NULL";
        return NAO_ERR_INVALID_ARG;
    }
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        g_thread_error = "no HIP device available";
        return NAO_ERR_NOT_READY;
    }
    if (device < 0 || device >= count) {
        g_thread_error = "device ordinal out of range";
        return NAO_ERR_INVALID_ARG;
    }
    nao_ctx c = new (std::nothrow) nao_ctx_s();
    if (!c) return NAO_ERR_OUT_OF_MEMORY;
    c->device = device;
    c->budget = hbm_budget_bytes;
    {
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cu > 0)
            c->n_cu = cu;
    }
    if (const char* e = std::getenv("NAO_PERSISTENT_PER_CU")) {
        const long v = std::atol(e);
        if (v >= 0 && v <= 64) c->persistent_per_cu = v;
    }
    if (const char* e = std::getenv("NAO_OVERLAP")) c->overlap = std::atol(e) != 0;
    c->scratch_cap_elems = scratch_cap_from_env();
    e = hipSetDevice(device);
    if (e == hipSuccess) e = noalloc_scratch_init(device);  // the device address of the fixed scratch
    if (e == hipSuccess) {
        if (hip_stream) {
            c->stream = static_cast<hipStream_t>(hip_stream);
        } else {
            e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
            c->own_stream = e == hipSuccess;
        }
    }
    if (e == hipSuccess) {
        void* p = nullptr;
        nao_status s = dev_alloc(c, (WSUM_BLOCKS + 1) * sizeof(double), &p);
        if (s != NAO_OK) {
            g_thread_error = c->err;
            if (c->own_stream) (void)hipStreamDestroy(c->stream);
            delete c;
            return s;
        }
        c->wsum = static_cast<double*>(p);
    }
    if (e != hipSuccess) {
        g_thread_error = std::string("context setup failed: ") + hipGetErrorString(e);
        delete c;
        return NAO_ERR_HIP;
    }
    *out = c;
    return NAO_OK;
}

void nao_ctx_destroy(nao_ctx c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    many_forget(c, nullptr);
    (void)hipStreamSynchronize(c->stream);
    for (auto& sp : c->spare) dev_free(c, sp.first, sp.second);
    c->spare.clear();
    if (c->stream2) (void)hipStreamSynchronize(c->stream2);
    dev_free(c, c->scratch, c->scratch_elems * sizeof(double));
    dev_free(c, c->scratch2, c->scratch2_elems * sizeof(double));
    dev_free(c, c->gscratch, c->gscratch_bytes);
    dev_free(c, c->gscratch2, c->gscratch2_bytes);
    dev_free(c, c->wsum, (WSUM_BLOCKS + 1) * sizeof(double));
    for (hipEvent_t e : {c->ev_start, c->ev_ready[0], c->ev_ready[1], c->ev_done[0], c->ev_done[1]})
        if (e) (void)hipEventDestroy(e);
    if (c->stream2) (void)hipStreamDestroy(c->stream2);
    for (auto& r : c->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : c->pool) (void)hipEventDestroy(e);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char* nao_last_error(nao_ctx c)
{
    if (!c) return g_thread_error.c_str();
    static thread_local std::string copy;  // the caller's view stays valid until its next call
    std::lock_guard<std::mutex> lk(c->err_mu);
    copy = c->err;
    return copy.c_str();
}

nao_status nao_ctx_set_stream(nao_ctx c, void* hip_stream)
{
    nao_status st = check_ctx(c);
    if (st != NAO_OK) return st;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->own_stream) HIP_TRY(c, hipStreamDestroy(c->stream));
    c->own_stream = false;
    if (hip_stream) {
        c->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        HIP_TRY(c, hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        c->own_stream = true;
    }
    return NAO_OK;
}

void* nao_ctx_stream(nao_ctx c) { return c ? (void*)c->stream : nullptr; }

nao_status nao_ctx_synchronize(nao_ctx c)
{
    nao_status st = check_ctx(c);
    if (st != NAO_OK) return st;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    many_retire(c, false);
    return NAO_OK;
}

nao_status nao_ctx_memory(nao_ctx c, size_t* used, size_t* budget)
{
    if (!c) {
        g_thread_error = "context is NULL";
        return NAO_ERR_INVALID_ARG;
    }
    if (used) *used = c->used;
    if (budget) *budget = c->budget;
    return NAO_OK;
}

nao_status nao_ctx_set_overlap(nao_ctx c, int enable)
{
    nao_status st = check_ctx(c);
    if (st != NAO_OK) return st;
    c->overlap = enable != 0;
    if (!c->overlap && c->scratch2) {
        many_forget(c, nullptr);  // captured plans hold the buffer
        HIP_TRY(c, hipStreamSynchronize(c->stream2));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        dev_free(c, c->scratch2, c->scratch2_elems * sizeof(double));
        c->scratch2 = nullptr;
        c->scratch2_elems = 0;
    }
    if (!c->overlap && c->gscratch2) {
        HIP_TRY(c, hipStreamSynchronize(c->stream2));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        dev_free(c, c->gscratch2, c->gscratch2_bytes);
        c->gscratch2 = nullptr;
        c->gscratch2_bytes = 0;
    }
    return NAO_OK;
}

nao_status nao_ctx_profile(nao_ctx c, int enable)
{
    nao_status st = check_ctx(c);
    if (st != NAO_OK) return st;
    if (enable) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        for (auto& r : c->recs) {
            c->pool.push_back(r.a);
            c->pool.push_back(r.b);
        }
        c->recs.clear();
    }
    c->prof = enable != 0;
    return NAO_OK;
}

nao_status nao_ctx_profile_read(nao_ctx c, int32_t max_entries, char* names, int64_t* launches, double* total_ms,
                                int32_t* n_entries)
{
    nao_status st = check_ctx(c);
    if (st != NAO_OK) return st;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    std::vector<std::string> keys;
    std::vector<int64_t> cnt;
    std::vector<double> ms;
    for (auto& r : c->recs) {
        float t = 0.0f;
        HIP_TRY(c, hipEventElapsedTime(&t, r.a, r.b));
        size_t k = 0;
        while (k < keys.size() && keys[k] != r.name) ++k;
        if (k == keys.size()) {
            keys.push_back(r.name);
            cnt.push_back(0);
            ms.push_back(0.0);
        }
        cnt[k]++;
        ms[k] += t;
    }
    const int32_t n = (int32_t)std::min<size_t>(keys.size(), max_entries > 0 ? (size_t)max_entries : 0);
    for (int32_t k = 0; k < n; ++k) {
        if (names) {
            std::memset(names + 32 * k, 0, 32);
            std::strncpy(names + 32 * k, keys[k].c_str(), 31);
        }
        if (launches) launches[k] = cnt[k];
        if (total_ms) total_ms[k] = ms[k];
    }
    if (n_entries) *n_entries = (int32_t)keys.size();
    return NAO_OK;
}

// ---------------------------------------------------------------------------------- plans

struct nao_plan_s {
    HostBasis basis;
    int64_t n_points = 0;
    std::vector<int64_t> perm, batch_ptr, atom_ptr;
    std::vector<int32_t> atoms;
    std::vector<int64_t> basis_ptr;
    std::vector<int32_t> basis_idx;
};

static nao_status check_points(const double* xyz, int64_t n, int32_t max_batch, std::string& why)
{
    if (n < 0 || n > 0x7fffffffLL) return (why = "n_points outside [0, 2^31-1]", NAO_ERR_INVALID_ARG);
    if (n > 0 && !xyz) return (why = "point_xyz is NULL", NAO_ERR_INVALID_ARG);
    if (max_batch < 1 || max_batch > 4096) return (why = "max_batch outside [1, 4096]", NAO_ERR_INVALID_ARG);
    if (!finite_all(xyz, 3 * n)) return (why = "non-finite point coordinate", NAO_ERR_INVALID_ARG);
    return NAO_OK;
}

nao_status nao_plan_create(const nao_basis_desc* basis, int64_t n_points, const double* point_xyz,
                           int32_t max_batch, nao_plan* out)
{
    return nao_plan_create_ex(basis, n_points, point_xyz, max_batch, NAO_BATCH_OCTREE, out);
}

nao_status nao_plan_create_ex(const nao_basis_desc* basis, int64_t n_points, const double* point_xyz,
                              int32_t max_batch, nao_batcher batcher, nao_plan* out)
{
    if (!out) return (g_thread_error = "out is NULL", NAO_ERR_INVALID_ARG);
    *out = nullptr;
    if (batcher != NAO_BATCH_OCTREE && batcher != NAO_BATCH_CUTPLANE)
        return (g_thread_error = "unknown batcher", NAO_ERR_INVALID_ARG);
    std::string why;
    nao_status st = check_points(point_xyz, n_points, max_batch, why);
    if (st != NAO_OK) return (g_thread_error = why, st);
    try {
        nao_plan p = new nao_plan_s();
        why = load_basis(basis, p->basis);
        if (!why.empty()) {
            delete p;
            g_thread_error = why;
            return NAO_ERR_INVALID_ARG;
        }
        p->n_points = n_points;
        make_batches(batcher, point_xyz, n_points, max_batch, p->perm, p->batch_ptr);
        relevant_atoms(p->basis, point_xyz, p->perm, p->batch_ptr, p->atom_ptr, p->atoms);
        expand_lists(p->basis, p->atom_ptr, p->atoms, p->basis_ptr, p->basis_idx);
        *out = p;
        return NAO_OK;
    } catch (const std::bad_alloc&) {
        g_thread_error = "host allocation failed";
        return NAO_ERR_OUT_OF_MEMORY;
    } catch (...) {
        g_thread_error = "internal error in planning";
        return NAO_ERR_INTERNAL;
    }
}

nao_status nao_plan_info(nao_plan p, int64_t* n_basis, int64_t* n_batches, int64_t* n_list)
{
    if (!p) return (g_thread_error = "plan is NULL", NAO_ERR_INVALID_ARG);
    if (n_basis) *n_basis = p->basis.n_basis;
    if (n_batches) *n_batches = (int64_t)p->batch_ptr.size() - 1;
    if (n_list) *n_list = (int64_t)p->basis_idx.size();
    return NAO_OK;
}

nao_status nao_plan_get_batches(nao_plan p, int64_t* perm, int64_t* batch_ptr, int64_t* basis_ptr,
                                int32_t* basis_idx)
{
    if (!p) return (g_thread_error = "plan is NULL", NAO_ERR_INVALID_ARG);
    if (perm) std::copy(p->perm.begin(), p->perm.end(), perm);
    if (batch_ptr) std::copy(p->batch_ptr.begin(), p->batch_ptr.end(), batch_ptr);
    if (basis_ptr) std::copy(p->basis_ptr.begin(), p->basis_ptr.end(), basis_ptr);
    if (basis_idx) std::copy(p->basis_idx.begin(), p->basis_idx.end(), basis_idx);
    return NAO_OK;
}

void nao_plan_destroy(nao_plan p) { delete p; }

// -------------------------------------------------------------------------------- systems

static nao_status setup_system(nao_system s, const double* xyz, const double* w)
{
    nao_ctx c = s->ctx;
    const HostBasis& B = s->basis;
    const int64_t n = s->n_points;
    make_batches(s->batcher, xyz, n, s->max_batch, s->perm, s->batch_ptr);
    relevant_atoms(B, xyz, s->perm, s->batch_ptr, s->atom_ptr, s->atoms);
    s->work_units = 0.0;
    for (size_t b = 0; b + 1 < s->batch_ptr.size(); ++b) {
        double m = 0.0;
        for (int64_t q = s->atom_ptr[b]; q < s->atom_ptr[b + 1]; ++q)
            m += (double)(B.atom_first[s->atoms[q] + 1] - B.atom_first[s->atoms[q]]);
        s->work_units += (double)(s->batch_ptr[b + 1] - s->batch_ptr[b]) * m * m;
    }
    // batch-ordered points
    std::vector<double> px(n), py(n), pz(n), pw(n);
    std::vector<int32_t> perm32(n);
    for (int64_t k = 0; k < n; ++k) {
        const int64_t p = s->perm[k];
        px[k] = xyz[3 * p];
        py[k] = xyz[3 * p + 1];
        pz[k] = xyz[3 * p + 2];
        pw[k] = w[p];
        perm32[k] = (int32_t)p;
    }
    std::vector<double> axyzr(4 * B.n_atoms);
    for (int64_t a = 0; a < B.n_atoms; ++a) {
        axyzr[4 * a] = B.atom_xyz[3 * a];
        axyzr[4 * a + 1] = B.atom_xyz[3 * a + 1];
        axyzr[4 * a + 2] = B.atom_xyz[3 * a + 2];
        axyzr[4 * a + 3] = B.atom_rcut[a] * B.atom_rcut[a];
    }
    std::vector<double> rpar(4 * B.n_radial);
    for (int32_t r = 0; r < B.n_radial; ++r) {
        rpar[4 * r] = B.rmin[r];
        rpar[4 * r + 1] = B.rcut[r] * B.rcut[r];
        rpar[4 * r + 2] = (double)(B.n_knots - 1) / std::log(B.rcut[r] / B.rmin[r]);
        rpar[4 * r + 3] = std::log(B.rmin[r]);
    }
    std::vector<double> spl = spline_knots(B);
    s->spline_lds = spl.size() <= (size_t)MAX_SPLINE_LDS ? (int)spl.size() : 0;
    nao_status st;
#define UP(arr, vec) \
    if ((st = upload(c, s->arr, (vec).data(), (vec).size() * sizeof((vec)[0]))) != NAO_OK) return st
    UP(d_px, px);
    UP(d_py, py);
    UP(d_pz, pz);
    UP(d_pw, pw);
    UP(d_perm, perm32);
    UP(d_atoms, axyzr);
    UP(d_species, B.atom_species);
    UP(d_shell_ptr, B.shell_ptr);
    UP(d_shell_l, B.shell_l);
    UP(d_shell_rad, B.shell_radial);
    UP(d_radial_par, rpar);
    UP(d_spline, spl);
    std::vector<int32_t> fn_ptr(1, 0), fn_code;
    for (int32_t sp = 0; sp < B.n_species; ++sp) {
        for (int32_t j = B.shell_ptr[sp]; j < B.shell_ptr[sp + 1]; ++j)
            for (int32_t mm = 0; mm < 2 * B.shell_l[j] + 1; ++mm)
                fn_code.push_back(((j - B.shell_ptr[sp]) << 4) | (B.shell_l[j] * B.shell_l[j] + mm));
        fn_ptr.push_back((int32_t)fn_code.size());
    }
    UP(d_fn_ptr, fn_ptr);
    UP(d_fn_code, fn_code);
#undef UP
    DevSys& d = s->dsys;
    d.px = s->d_px.as<double>();
    d.py = s->d_py.as<double>();
    d.pz = s->d_pz.as<double>();
    d.pw = s->d_pw.as<double>();
    d.perm = s->d_perm.as<int32_t>();
    d.atom_xyzr = s->d_atoms.as<double>();
    d.atom_species = s->d_species.as<int32_t>();
    d.species_shell_ptr = s->d_shell_ptr.as<int32_t>();
    d.shell_l = s->d_shell_l.as<int32_t>();
    d.shell_radial = s->d_shell_rad.as<int32_t>();
    d.radial_par = s->d_radial_par.as<double>();
    d.spline = s->d_spline.as<double>();
    d.species_fn_ptr = s->d_fn_ptr.as<int32_t>();
    d.fn_code = s->d_fn_code.as<int32_t>();
    d.n_species = B.n_species;
    d.n_shells = B.shell_ptr[B.n_species];
    d.n_radial = B.n_radial;
    d.n_knots = B.n_knots;
    d.n_basis = B.n_basis;
    d.n_points = n;
    if ((st = upload(c, s->d_sys, &d, sizeof(DevSys))) != NAO_OK) return st;
    if ((st = ensure(c, s->d_wv, std::max<int64_t>(1, n) * sizeof(double))) != NAO_OK) return st;
    HIP_TRY(c, hipStreamSynchronize(c->stream));  // host vectors above go out of scope
    return build_groups(s);
}

nao_status nao_build_batches(nao_ctx c, const nao_basis_desc* basis, int64_t n_points, const double* point_xyz,
                             const double* point_w, int32_t max_batch, nao_system* out)
{
    return nao_build_batches_ex(c, basis, n_points, point_xyz, point_w, max_batch, NAO_BATCH_OCTREE, out);
}

nao_status nao_build_batches_ex(nao_ctx c, const nao_basis_desc* basis, int64_t n_points, const double* point_xyz,
                                const double* point_w, int32_t max_batch, nao_batcher batcher, nao_system* out)
{
    if (!out) return (set_err(c, "out is NULL"), NAO_ERR_INVALID_ARG);
    *out = nullptr;
    nao_status st = check_ctx(c);
    if (st != NAO_OK) return st;
    if (batcher != NAO_BATCH_OCTREE && batcher != NAO_BATCH_CUTPLANE)
        return (set_err(c, "unknown batcher"), NAO_ERR_INVALID_ARG);
    std::string why;
    if ((st = check_points(point_xyz, n_points, max_batch, why)) != NAO_OK) return (set_err(c, why), st);
    if (n_points > 0 && !point_w) return (set_err(c, "point_w is NULL"), NAO_ERR_INVALID_ARG);
    for (int64_t k = 0; k < n_points; ++k)
        if (!std::isfinite(point_w[k]) || point_w[k] < 0.0)
            return (set_err(c, "point weights must be finite and >= 0"), NAO_ERR_INVALID_ARG);
    nao_system s = nullptr;
    try {
        s = new nao_system_s();
        s->ctx = c;
        why = load_basis(basis, s->basis);
        if (!why.empty()) {
            delete s;
            set_err(c, why);
            return NAO_ERR_INVALID_ARG;
        }
        s->n_points = n_points;
        s->max_batch = max_batch;
        s->batcher = batcher;
        st = setup_system(s, point_xyz, point_w);
    } catch (const std::bad_alloc&) {
        set_err(c, "host allocation failed");
        st = NAO_ERR_OUT_OF_MEMORY;
    } catch (...) {
        set_err(c, "internal error in nao_build_batches");
        st = NAO_ERR_INTERNAL;
    }
    if (st != NAO_OK) {
        if (s) {
            free_all(s);
            delete s;
        }
        return st;
    }
    c->n_systems++;
    *out = s;
    return NAO_OK;
}

nao_status nao_system_set_group_max(nao_system s, int32_t group_max)
{
    if (!s) return (g_thread_error = "system is NULL", NAO_ERR_INVALID_ARG);
    nao_status st = check_ctx(s->ctx);
    if (st != NAO_OK) return st;
    if (group_max != 0 && (group_max < 16 || group_max > MAX_UNIT_POINTS))
        return (set_err(s->ctx, "group_max must be 0 or in [16, 256]"), NAO_ERR_INVALID_ARG);
    HIP_TRY(s->ctx, hipStreamSynchronize(s->ctx->stream));
    many_forget(s->ctx, s);
    s->group_max = group_max;
    try {
        return build_groups(s);
    } catch (...) {
        set_err(s->ctx, "internal error in nao_system_set_group_max");
        return NAO_ERR_INTERNAL;
    }
}

nao_status nao_system_set_resident_basis(nao_system s, int enable)
{
    if (!s) return (g_thread_error = "system is NULL", NAO_ERR_INVALID_ARG);
    nao_status st = check_ctx(s->ctx);
    if (st != NAO_OK) return st;
    if (enable != 0 && enable != 1) return (set_err(s->ctx, "enable must be 0 or 1"), NAO_ERR_INVALID_ARG);
    HIP_TRY(s->ctx, hipStreamSynchronize(s->ctx->stream));
    if (!enable) {
        dev_free(s->ctx, s->d_phi_res.p, s->d_phi_res.bytes);
        s->d_phi_res.p = nullptr;
        s->d_phi_res.bytes = 0;
        s->resident = false;
        s->res_kind = -1;
        s->res_off.clear();
        return NAO_OK;
    }
    s->resident = true;
    st = resident_layout(s);
    return st;  // the allocation's own message says what did not fit
}

nao_status nao_system_set_h_tile(nao_system s, int32_t h_tile)
{
    if (!s) return (g_thread_error = "system is NULL", NAO_ERR_INVALID_ARG);
    nao_status st = check_ctx(s->ctx);
    if (st != NAO_OK) return st;
    if (h_tile != 64 && h_tile != 128) return (set_err(s->ctx, "h_tile must be 64 or 128"), NAO_ERR_INVALID_ARG);
    if (h_tile == s->h_tile) return NAO_OK;
    HIP_TRY(s->ctx, hipStreamSynchronize(s->ctx->stream));
    many_forget(s->ctx, s);
    s->h_tile = h_tile;
    try {
        return build_groups(s);
    } catch (...) {
        set_err(s->ctx, "internal error in nao_system_set_h_tile");
        return NAO_ERR_INTERNAL;
    }
}

nao_status nao_system_info(nao_system s, int64_t* n_basis, int64_t* n_batches, int64_t* n_list, size_t* dev_bytes)
{
    if (!s) return (g_thread_error = "system is NULL", NAO_ERR_INVALID_ARG);
    if (n_basis) *n_basis = s->basis.n_basis;
    if (n_batches) *n_batches = (int64_t)s->batch_ptr.size() - 1;
    if (n_list) {
        int64_t t = 0;
        for (size_t b = 0; b + 1 < s->atom_ptr.size(); ++b)
            for (int64_t q = s->atom_ptr[b]; q < s->atom_ptr[b + 1]; ++q)
                t += s->basis.atom_first[s->atoms[q] + 1] - s->basis.atom_first[s->atoms[q]];
        *n_list = t;
    }
    if (dev_bytes) *dev_bytes = system_bytes(s);
    return NAO_OK;
}

nao_status nao_get_batches(nao_system s, int64_t* perm, int64_t* batch_ptr, int64_t* basis_ptr, int32_t* basis_idx)
{
    if (!s) return (g_thread_error = "system is NULL", NAO_ERR_INVALID_ARG);
    try {
        if (perm) std::copy(s->perm.begin(), s->perm.end(), perm);
        if (batch_ptr) std::copy(s->batch_ptr.begin(), s->batch_ptr.end(), batch_ptr);
        if (basis_ptr || basis_idx) {
            std::vector<int64_t> bp;
            std::vector<int32_t> bi;
            expand_lists(s->basis, s->atom_ptr, s->atoms, bp, bi);
            if (basis_ptr) std::copy(bp.begin(), bp.end(), basis_ptr);
            if (basis_idx) std::copy(bi.begin(), bi.end(), basis_idx);
        }
    } catch (...) {
        set_err(s->ctx, "host allocation failed");
        return NAO_ERR_OUT_OF_MEMORY;
    }
    return NAO_OK;
}

nao_status nao_system_work(nao_system s, double* units)
{
    if (!s || !units) return (g_thread_error = "NULL argument", NAO_ERR_INVALID_ARG);
    *units = s->work_units;
    return NAO_OK;
}

void nao_system_destroy(nao_system s)
{
    if (!s) return;
    (void)hipSetDevice(s->ctx->device);
    many_forget(s->ctx, s);
    (void)hipStreamSynchronize(s->ctx->stream);
    free_all(s);
    s->ctx->n_systems--;
    delete s;
}

// ------------------------------------------------------------------------------ basis values

nao_status nao_eval_basis(nao_system s, int64_t b0, int64_t b1, double* phi, nao_memspace phi_space,
                          int64_t* phi_ptr)
{
    if (!s) return (g_thread_error = "system is NULL", NAO_ERR_INVALID_ARG);
    nao_ctx c = s->ctx;
    nao_status st = check_ctx(c);
    if (st != NAO_OK) return st;
    const int64_t nb = (int64_t)s->batch_ptr.size() - 1;
    if (b0 < 0 || b1 < b0 || b1 > nb) return (set_err(c, "batch range out of bounds"), NAO_ERR_INVALID_ARG);
    if (!phi_ptr) return (set_err(c, "phi_ptr is NULL"), NAO_ERR_INVALID_ARG);
    if (phi_space != NAO_MEM_HOST && phi_space != NAO_MEM_DEVICE) return (set_err(c, "bad memspace"), NAO_ERR_INVALID_ARG);
    std::vector<Unit> units;
    std::vector<int32_t> uat, ucol;
    try {
        batch_units(s->basis, s->batch_ptr, s->atom_ptr, s->atoms, b0, b1, units, uat, ucol);
    } catch (...) {
        return (set_err(c, "host allocation failed"), NAO_ERR_OUT_OF_MEMORY);
    }
    phi_ptr[0] = 0;
    std::vector<DevUnit> du;
    for (size_t k = 0; k < units.size(); ++k) {
        const Unit& u = units[k];
        phi_ptr[k + 1] = phi_ptr[k] + (int64_t)u.n_points * u.m;
        if (u.m == 0 || u.n_points == 0) continue;
        DevUnit d{};
        d.point_begin = u.point_begin;
        d.atom_begin = u.atom_begin;
        d.fn_begin = 0;
        d.out_offset = phi_ptr[k];
        d.n_points = u.n_points;
        d.n_atoms = u.n_atoms;
        d.m = u.m;
        d.ld = u.m;
        du.push_back(d);
    }
    if (!phi || du.empty()) return NAO_OK;
    const int64_t total = phi_ptr[units.size()];
    DevArray t_units, t_at, t_col, t_out, t_seg;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(c->stream);
        for (DevArray* a : {&t_units, &t_at, &t_col, &t_out, &t_seg}) dev_free(c, a->p, a->bytes);
    };
    if ((st = upload(c, t_units, du.data(), du.size() * sizeof(DevUnit))) != NAO_OK) return cleanup(), st;
    if ((st = upload(c, t_at, uat.data(), uat.size() * sizeof(int32_t))) != NAO_OK) return cleanup(), st;
    if ((st = upload(c, t_col, ucol.data(), ucol.size() * sizeof(int32_t))) != NAO_OK) return cleanup(), st;
    double* out = phi;
    if (phi_space == NAO_MEM_HOST) {
        if ((st = ensure(c, t_out, (size_t)total * sizeof(double))) != NAO_OK) return cleanup(), st;
        out = t_out.as<double>();
    }
    DevSeg g{};
    g.sys = s->d_sys.as<DevSys>();
    g.units = t_units.as<DevUnit>();
    g.unit_atoms = t_at.as<int32_t>();
    g.unit_cols = t_col.as<int32_t>();
    g.phi = out;
    g.unit_begin = 0;
    g.unit_count = (int64_t)du.size();
    g.unit_prefix = 0;
    if ((st = upload(c, t_seg, &g, sizeof(DevSeg))) != NAO_OK) return cleanup(), st;
    hipError_t e = launch_basis(t_seg.as<DevSeg>(), 1, (int64_t)du.size(), s->spline_lds, false, c->stream);
    if (e == hipSuccess && phi_space == NAO_MEM_HOST)
        e = hipMemcpyAsync(phi, out, (size_t)total * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    cleanup();
    if (e != hipSuccess) return hip_fail(c, e, "nao_eval_basis");
    return NAO_OK;
}

// ------------------------------------------------------------------------------ contractions

static nao_status check_prec(nao_ctx c, nao_precision p)
{
    if (p == NAO_FP64 || p == NAO_FP32 || p == NAO_BF16X3 || p == NAO_BF16X6) return NAO_OK;
    return (set_err(c, "unknown precision"), NAO_ERR_INVALID_ARG);
}

// The block loop of a density update or Hamiltonian integration: per block, the basis values of
// its units (unless resident), then the contraction.  With more than one block and overlap on,
// block k's basis values go to buffer k % 2 and its basis launch to the second stream, which
// waits for the contraction of block k - 2 (the last reader of that buffer); the contraction of
// block k waits for its basis launch.  The context stream thus ends after every launch of the
// operation, so callers synchronize on it alone.
static nao_status run_blocks(nao_system s, bool ham, nao_precision prec, const double* wv, const double* D, double* H,
                             double* n)
{
    const Mode mode = exec_mode(s->ctx, prec);
    const bool f32 = prec != NAO_FP64;
    const bool staged = true;  // every mode reads its basis values from the scratch block
    nao_ctx c = s->ctx;
    std::vector<DevSeg> segs;
    const bool wide = ham && s->h_tile == 128 && (prec == NAO_FP64 || prec == NAO_FP32);
    // resident mode: each block reads its own slot, evaluated once per value type
    const bool res = s->resident && s->d_phi_res.p && s->res_off.size() == s->blocks.size();
    const int kind = f32 ? 1 : 0;
    const bool evaluate = !res || s->res_kind != kind;
    size_t need = 0;
    for (const Block& b : s->blocks) need = std::max(need, (size_t)b.phi_elems);
    const bool ovl = !res && s->blocks.size() > 1 && overlap_ready(c, need);
    for (size_t k = 0; k < s->blocks.size(); ++k) {
        DevSeg g = make_seg(s, s->blocks[k], ham, wide);
        if (ovl && (k & 1)) g.phi = c->scratch2;
        if (res) g.phi = static_cast<char*>(s->d_phi_res.p) + s->res_off[k] * (f32 ? sizeof(float) : sizeof(double));
        g.wv = wv;
        g.D = D;
        g.H = H;
        g.n = n;
        segs.push_back(g);
    }
    if (segs.empty()) return NAO_OK;
    HIP_TRY(c, hipMemcpyAsync(s->d_segs.p, segs.data(), segs.size() * sizeof(DevSeg), hipMemcpyHostToDevice,
                              c->stream));
    DevSeg* dseg = s->d_segs.as<DevSeg>();
    if (res && evaluate) s->res_kind = -1;  // marked valid only once every block is enqueued
    nao_status st = block_loop(
        c, segs.size(), ovl, staged && evaluate ? (f32 ? "basis_f32" : "basis_f64") : nullptr, kname(ham, prec),
        [&](size_t k, hipStream_t q) { return launch_basis(dseg + k, 1, segs[k].unit_count, s->spline_lds, f32, q); },
        [&](size_t k) {
            return ham ? launch_h(mode, dseg + k, 1, segs[k].item_count, c->stream, 0, wide ? 128 : TILE)
                       : launch_n(mode, dseg + k, 1, segs[k].item_count, c->stream);
        });
    if (st != NAO_OK) return st;
    if (res) s->res_kind = kind;
    return NAO_OK;
}

nao_status nao_integrate_h(nao_system s, const double* v, nao_memspace v_space, nao_precision prec, double* H,
                           nao_memspace H_space)
{
    if (!s) return (g_thread_error = "system is NULL", NAO_ERR_INVALID_ARG);
    nao_ctx c = s->ctx;
    nao_status st = check_ctx(c);
    if (st != NAO_OK) return st;
    if ((st = check_prec(c, prec)) != NAO_OK) return st;
    if (!H || (s->n_points > 0 && !v)) return (set_err(c, "NULL v or H"), NAO_ERR_INVALID_ARG);
    if ((v_space != NAO_MEM_HOST && v_space != NAO_MEM_DEVICE) || (H_space != NAO_MEM_HOST && H_space != NAO_MEM_DEVICE))
        return (set_err(c, "bad memspace"), NAO_ERR_INVALID_ARG);
    const int64_t n = s->n_points, nb = s->basis.n_basis;
    const double* vd = v;
    if (v_space == NAO_MEM_HOST && n > 0) {
        if ((st = ensure(c, s->d_v, n * sizeof(double))) != NAO_OK) return st;
        HIP_TRY(c, hipMemcpyAsync(s->d_v.p, v, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
        vd = s->d_v.as<double>();
    }
    double* Hd = H;
    if (H_space == NAO_MEM_HOST) {
        if ((st = ensure(c, s->d_H, std::max<int64_t>(1, nb * nb) * sizeof(double))) != NAO_OK) return st;
        Hd = s->d_H.as<double>();
    }
    LAUNCH(c, "fill", launch_fill(Hd, nb * nb, 0.0, c->stream));
    LAUNCH(c, "wv", launch_wv(s->d_pw.as<double>(), s->d_perm.as<int32_t>(), vd, s->d_wv.as<double>(), n, c->stream));
    if ((st = run_blocks(s, true, prec, s->d_wv.as<double>(), nullptr, Hd, nullptr)) != NAO_OK) return st;
    LAUNCH(c, "mirror", launch_mirror(Hd, nb, c->stream));
    if (H_space == NAO_MEM_HOST) {
        HIP_TRY(c, hipMemcpyAsync(H, Hd, nb * nb * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    if (v_space == NAO_MEM_HOST) HIP_TRY(c, hipStreamSynchronize(c->stream));
    return NAO_OK;
}

nao_status nao_integrate_h_noalloc(nao_system s, const double* v, nao_precision prec, double* H)
{
    if (!s) return (g_thread_error = "system is NULL", NAO_ERR_INVALID_ARG);
    nao_ctx c = s->ctx;
    nao_status st = check_ctx(c);
    if (st != NAO_OK) return st;
    if ((st = check_prec(c, prec)) != NAO_OK) return st;
    const int64_t n = s->n_points, nb = s->basis.n_basis;
    if (!H || (n > 0 && !v)) return (set_err(c, "NULL v or H"), NAO_ERR_INVALID_ARG);
    char* base = static_cast<char*>(noalloc_scratch(c->device));
    if (!base) return (set_err(c, "the fixed scratch of this device was not set up"), NAO_ERR_NOT_READY);
    // layout of the fixed scratch: segment table | w*v | basis values of one sub-block
    const size_t wv_bytes = ((size_t)std::max<int64_t>(1, n) * sizeof(double) + 255) / 256 * 256;
    if (NOALLOC_SEG_BYTES + wv_bytes >= NOALLOC_SCRATCH_BYTES)
        return (set_err(c, "n_points = " + std::to_string(n) + " needs " + std::to_string(wv_bytes) +
                               " B of w*v, more than the fixed scratch of " +
                               std::to_string(NOALLOC_SCRATCH_BYTES) + " B holds"),
                NAO_ERR_INVALID_ARG);
    const size_t esz = prec == NAO_FP64 ? sizeof(double) : sizeof(float);
    double* wv = reinterpret_cast<double*>(base + NOALLOC_SEG_BYTES);
    const uintptr_t phi0 = reinterpret_cast<uintptr_t>(base + NOALLOC_SEG_BYTES + wv_bytes);
    const int64_t cap = (int64_t)((NOALLOC_SCRATCH_BYTES - NOALLOC_SEG_BYTES - wv_bytes) / esz);
    if (s->h_units.size() != (size_t)s->n_units || s->h_item_first.size() != (size_t)s->n_units + 1)
        return (set_err(c, "system has no unit table"), NAO_ERR_INTERNAL);
    // sub-blocks: runs of consecutive units of one block whose basis values fit the fixed
    // scratch; phi of a sub-block is placed so that its first unit's values start at phi0
    std::vector<DevSeg>& segs = s->na_segs;
    segs.clear();
    for (const Block& b : s->blocks) {
        int64_t u = b.unit_begin;
        const int64_t uend = b.unit_begin + b.unit_count;
        while (u < uend) {
            const int64_t o0 = s->h_units[u].out_offset;
            int64_t u1 = u;
            while (u1 < uend) {
                const DevUnit& d = s->h_units[u1];
                if (d.out_offset + (int64_t)d.n_points * d.ld - o0 > cap) break;
                ++u1;
            }
            if (u1 == u)
                return (set_err(c, "an execution group's basis values (" +
                                       std::to_string((int64_t)s->h_units[u].n_points * s->h_units[u].ld * (int64_t)esz) +
                                       " B) exceed the fixed scratch"),
                        NAO_ERR_INVALID_ARG);
            DevSeg g = make_seg(s, b, true, false);
            g.phi = reinterpret_cast<void*>(phi0 - (uintptr_t)o0 * esz);
            g.unit_begin = u;
            g.unit_count = u1 - u;
            g.item_begin = s->h_item_first[u];
            g.item_count = s->h_item_first[u1] - s->h_item_first[u];
            g.wv = wv;
            g.H = H;
            segs.push_back(g);
            u = u1;
        }
    }
    if (segs.size() * sizeof(DevSeg) > NOALLOC_SEG_BYTES)
        return (set_err(c, std::to_string(segs.size()) + " sub-blocks exceed the segment table of the fixed scratch"),
                NAO_ERR_INVALID_ARG);
    // no profiling events here: nothing in this call creates or allocates anything
    const Mode mode = exec_mode(c, prec);
    HIP_TRY(c, launch_fill(H, nb * nb, 0.0, c->stream));
    if (n > 0) HIP_TRY(c, launch_wv(s->d_pw.as<double>(), s->d_perm.as<int32_t>(), v, wv, n, c->stream));
    if (!segs.empty()) {
        HIP_TRY(c, hipMemcpyAsync(base, segs.data(), segs.size() * sizeof(DevSeg), hipMemcpyHostToDevice, c->stream));
        const DevSeg* dseg = reinterpret_cast<const DevSeg*>(base);
        for (size_t k = 0; k < segs.size(); ++k) {
            HIP_TRY(c, launch_basis(dseg + k, 1, segs[k].unit_count, s->spline_lds, prec != NAO_FP64, c->stream));
            HIP_TRY(c, launch_h(mode, dseg + k, 1, segs[k].item_count, c->stream, 0, TILE));
        }
    }
    HIP_TRY(c, launch_mirror(H, nb, c->stream));
    return NAO_OK;
}

nao_status nao_update_density(nao_system s, const double* D, nao_memspace D_space, nao_precision prec, double* nout,
                              nao_memspace n_space, double* n_electrons)
{
    if (!s) return (g_thread_error = "system is NULL", NAO_ERR_INVALID_ARG);
    nao_ctx c = s->ctx;
    nao_status st = check_ctx(c);
    if (st != NAO_OK) return st;
    if ((st = check_prec(c, prec)) != NAO_OK) return st;
    const int64_t n = s->n_points, nb = s->basis.n_basis;
    if ((nb > 0 && !D) || (n > 0 && !nout)) return (set_err(c, "NULL D or n"), NAO_ERR_INVALID_ARG);
    if ((D_space != NAO_MEM_HOST && D_space != NAO_MEM_DEVICE) || (n_space != NAO_MEM_HOST && n_space != NAO_MEM_DEVICE))
        return (set_err(c, "bad memspace"), NAO_ERR_INVALID_ARG);
    const double* Dd = D;
    if (D_space == NAO_MEM_HOST && nb > 0) {
        if ((st = ensure(c, s->d_D, nb * nb * sizeof(double))) != NAO_OK) return st;
        HIP_TRY(c, hipMemcpyAsync(s->d_D.p, D, nb * nb * sizeof(double), hipMemcpyHostToDevice, c->stream));
        Dd = s->d_D.as<double>();
    }
    double* nd = nout;
    if (n_space == NAO_MEM_HOST) {
        if ((st = ensure(c, s->d_n, std::max<int64_t>(1, n) * sizeof(double))) != NAO_OK) return st;
        nd = s->d_n.as<double>();
    }
    LAUNCH(c, "fill", launch_fill(nd, n, 0.0, c->stream));
    if ((st = run_blocks(s, false, prec, nullptr, Dd, nullptr, nd)) != NAO_OK) return st;
    if (n_electrons) {
        LAUNCH(c, "electron_count", launch_weighted_sum(s->d_pw.as<double>(), s->d_perm.as<int32_t>(), nd, n,
                                                         c->wsum, c->wsum + WSUM_BLOCKS, c->stream));
        HIP_TRY(c, hipMemcpyAsync(n_electrons, c->wsum + WSUM_BLOCKS, sizeof(double), hipMemcpyDeviceToHost,
                                  c->stream));
    }
    if (n_space == NAO_MEM_HOST && n > 0)
        HIP_TRY(c, hipMemcpyAsync(nout, nd, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (n_space == NAO_MEM_HOST || n_electrons || D_space == NAO_MEM_HOST) HIP_TRY(c, hipStreamSynchronize(c->stream));
    return NAO_OK;
}

// Extra per-block scratch beside the basis values: `per_value` FP64 slots per basis value.
// Both second buffers for an overlapped extended operation whose extra block holds per_value
// values per basis value (call after ensure_gscratch).
static bool overlap_ext(nao_system s, int per_value)
{
    nao_ctx c = s->ctx;
    if (s->blocks.size() < 2) return false;
    size_t need = 0;
    for (const Block& b : s->blocks) need = std::max(need, (size_t)b.phi_elems);
    return overlap_ready(c, need) && overlap_gscratch(c, need * per_value * sizeof(double));
}

static nao_status ensure_gscratch(nao_system s, int per_value)
{
    nao_ctx c = s->ctx;
    size_t need = 0;
    for (const Block& b : s->blocks) need = std::max(need, (size_t)b.phi_elems * per_value * sizeof(double));
    if (need <= c->gscratch_bytes) return NAO_OK;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    dev_free(c, c->gscratch, c->gscratch_bytes);
    c->gscratch = nullptr;
    c->gscratch_bytes = 0;
    nao_status st = dev_alloc(c, need, &c->gscratch);
    if (st == NAO_OK) c->gscratch_bytes = need;
    return st;
}

// H = K^T L + L^T K over the upper-triangle tile pairs, L written by the basis launch in mode
// `extra` (EXTRA_GGA_L, or EXTRA_KS_L with an optional field a), then mirrored.
static nao_status integrate_h_with_l(nao_system s, const double* v, const double* a, nao_memspace in_space,
                                     nao_precision prec, double* H, nao_memspace H_space, int extra)
{
    nao_ctx c = s->ctx;
    const bool ks = extra == EXTRA_KS_L;
    const int64_t n = s->n_points, nb = s->basis.n_basis;
    if (!H || (n > 0 && (!v || (!ks && !a)))) return (set_err(c, "NULL v, a or H"), NAO_ERR_INVALID_ARG);
    if ((in_space != NAO_MEM_HOST && in_space != NAO_MEM_DEVICE) || (H_space != NAO_MEM_HOST && H_space != NAO_MEM_DEVICE))
        return (set_err(c, "bad memspace"), NAO_ERR_INVALID_ARG);
    nao_status st;
    if ((st = ensure_gscratch(s, 1)) != NAO_OK) return st;  // L: one value per basis value
    const bool has_a = a != nullptr && n > 0;
    const double* vd = v;
    const double* ad = a;
    if (in_space == NAO_MEM_HOST && n > 0) {
        if ((st = ensure(c, s->d_v, n * sizeof(double))) != NAO_OK) return st;
        HIP_TRY(c, hipMemcpyAsync(s->d_v.p, v, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
        vd = s->d_v.as<double>();
        if (has_a) {
            if ((st = ensure(c, s->d_a, 3 * n * sizeof(double))) != NAO_OK) return st;
            HIP_TRY(c, hipMemcpyAsync(s->d_a.p, a, 3 * n * sizeof(double), hipMemcpyHostToDevice, c->stream));
            ad = s->d_a.as<double>();
        }
    }
    if (has_a && (st = ensure(c, s->d_wa, std::max<int64_t>(1, 3 * n) * sizeof(double))) != NAO_OK) return st;
    double* Hd = H;
    if (H_space == NAO_MEM_HOST) {
        if ((st = ensure(c, s->d_H, std::max<int64_t>(1, nb * nb) * sizeof(double))) != NAO_OK) return st;
        Hd = s->d_H.as<double>();
    }
    LAUNCH(c, "fill", launch_fill(Hd, nb * nb, 0.0, c->stream));
    LAUNCH(c, "wv", launch_wv(s->d_pw.as<double>(), s->d_perm.as<int32_t>(), vd, s->d_wv.as<double>(), n, c->stream));
    if (has_a)
        LAUNCH(c, "wa", launch_wa(s->d_pw.as<double>(), s->d_perm.as<int32_t>(), ad, s->d_wa.as<double>(), n, c->stream));
    const Mode mode = exec_mode(c, prec);
    const bool f32 = prec != NAO_FP64;
    const bool ovl = overlap_ext(s, 1);
    std::vector<DevSeg> segs;
    for (const Block& b : s->blocks) {
        DevSeg g = make_seg(s, b, true, false);
        g.wv = s->d_wv.as<double>();
        g.wa = has_a ? s->d_wa.as<double>() : nullptr;
        g.H = Hd;
        g.gphi = c->gscratch;
        if (ovl && (segs.size() & 1)) {
            g.phi = c->scratch2;
            g.gphi = c->gscratch2;
        }
        segs.push_back(g);
    }
    if (!segs.empty()) {
        HIP_TRY(c, hipMemcpyAsync(s->d_segs.p, segs.data(), segs.size() * sizeof(DevSeg), hipMemcpyHostToDevice,
                                  c->stream));
        DevSeg* dseg = s->d_segs.as<DevSeg>();
        const char* bname = ks ? (f32 ? "basis_ks_f32" : "basis_ks_f64") : (f32 ? "basis_gga_f32" : "basis_gga_f64");
        const char* hname = ks ? (f32 ? "hks_f32" : "hks_f64") : (f32 ? "hgga_f32" : "hgga_f64");
        st = block_loop(
            c, segs.size(), ovl, bname, hname,
            [&](size_t k, hipStream_t q) { return launch_basis(dseg + k, 1, segs[k].unit_count, s->spline_lds, f32, q, 0, extra); },
            [&](size_t k) { return launch_h_gga(mode, dseg + k, 1, segs[k].item_count, c->stream); });
        if (st != NAO_OK) return st;
    }
    LAUNCH(c, "mirror", launch_mirror(Hd, nb, c->stream));
    if (H_space == NAO_MEM_HOST) {
        HIP_TRY(c, hipMemcpyAsync(H, Hd, nb * nb * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    if (in_space == NAO_MEM_HOST) HIP_TRY(c, hipStreamSynchronize(c->stream));
    return NAO_OK;
}

nao_status nao_integrate_h_gga(nao_system s, const double* v, const double* a, nao_memspace in_space,
                               nao_precision prec, double* H, nao_memspace H_space)
{
    if (!s) return (g_thread_error = "system is NULL", NAO_ERR_INVALID_ARG);
    nao_ctx c = s->ctx;
    nao_status st = check_ctx(c);
    if (st != NAO_OK) return st;
    if (prec != NAO_FP64 && prec != NAO_FP32)
        return (set_err(c, "the Hamiltonian with a vector field runs in FP64 or FP32"), NAO_ERR_INVALID_ARG);
    return integrate_h_with_l(s, v, a, in_space, prec, H, H_space, EXTRA_GGA_L);
}

nao_status nao_integrate_h_ks(nao_system s, const double* v, const double* a, nao_memspace in_space,
                              nao_precision prec, double* H, nao_memspace H_space)
{
    if (!s) return (g_thread_error = "system is NULL", NAO_ERR_INVALID_ARG);
    nao_ctx c = s->ctx;
    nao_status st = check_ctx(c);
    if (st != NAO_OK) return st;
    if (prec != NAO_FP64 && prec != NAO_FP32)
        return (set_err(c, "the Kohn-Sham Hamiltonian runs in FP64 or FP32"), NAO_ERR_INVALID_ARG);
    return integrate_h_with_l(s, v, a, in_space, prec, H, H_space, EXTRA_KS_L);
}

nao_status nao_update_density_gradient(nao_system s, const double* D, nao_memspace D_space, nao_precision prec,
                                       double* nout, double* gout, nao_memspace out_space)
{
    if (!s) return (g_thread_error = "system is NULL", NAO_ERR_INVALID_ARG);
    nao_ctx c = s->ctx;
    nao_status st = check_ctx(c);
    if (st != NAO_OK) return st;
    if (prec != NAO_FP64 && prec != NAO_FP32)
        return (set_err(c, "the density gradient runs in FP64 or FP32"), NAO_ERR_INVALID_ARG);
    const int64_t n = s->n_points, nb = s->basis.n_basis;
    if ((nb > 0 && !D) || (n > 0 && (!nout || !gout))) return (set_err(c, "NULL D, n or grad_n"), NAO_ERR_INVALID_ARG);
    if ((D_space != NAO_MEM_HOST && D_space != NAO_MEM_DEVICE) || (out_space != NAO_MEM_HOST && out_space != NAO_MEM_DEVICE))
        return (set_err(c, "bad memspace"), NAO_ERR_INVALID_ARG);
    // gradients of one block's basis values: 3 per value
    if ((st = ensure_gscratch(s, 3)) != NAO_OK) return st;
    const double* Dd = D;
    if (D_space == NAO_MEM_HOST && nb > 0) {
        if ((st = ensure(c, s->d_D, nb * nb * sizeof(double))) != NAO_OK) return st;
        HIP_TRY(c, hipMemcpyAsync(s->d_D.p, D, nb * nb * sizeof(double), hipMemcpyHostToDevice, c->stream));
        Dd = s->d_D.as<double>();
    }
    double* nd = nout;
    double* gd = gout;
    if (out_space == NAO_MEM_HOST) {
        if ((st = ensure(c, s->d_n, std::max<int64_t>(1, n) * sizeof(double))) != NAO_OK) return st;
        if ((st = ensure(c, s->d_gn, std::max<int64_t>(1, 3 * n) * sizeof(double))) != NAO_OK) return st;
        nd = s->d_n.as<double>();
        gd = s->d_gn.as<double>();
    }
    LAUNCH(c, "fill", launch_fill(nd, n, 0.0, c->stream));
    LAUNCH(c, "fill", launch_fill(gd, 3 * n, 0.0, c->stream));
    const Mode mode = exec_mode(c, prec);
    const bool f32 = prec != NAO_FP64;
    const bool ovl = overlap_ext(s, 3);
    std::vector<DevSeg> segs;
    for (const Block& b : s->blocks) {
        DevSeg g = make_seg(s, b, false);
        g.D = Dd;
        g.n = nd;
        g.gn = gd;
        g.gphi = c->gscratch;
        if (ovl && (segs.size() & 1)) {
            g.phi = c->scratch2;
            g.gphi = c->gscratch2;
        }
        segs.push_back(g);
    }
    if (!segs.empty()) {
        HIP_TRY(c, hipMemcpyAsync(s->d_segs.p, segs.data(), segs.size() * sizeof(DevSeg), hipMemcpyHostToDevice,
                                  c->stream));
        DevSeg* dseg = s->d_segs.as<DevSeg>();
        st = block_loop(
            c, segs.size(), ovl, f32 ? "basis_grad_f32" : "basis_grad_f64", f32 ? "ngrad_f32" : "ngrad_f64",
            [&](size_t k, hipStream_t q) {
                return launch_basis(dseg + k, 1, segs[k].unit_count, s->spline_lds, f32, q, 0, EXTRA_GRAD);
            },
            [&](size_t k) { return launch_n_grad(mode, dseg + k, 1, segs[k].item_count, c->stream); });
        if (st != NAO_OK) return st;
    }
    if (out_space == NAO_MEM_HOST && n > 0) {
        HIP_TRY(c, hipMemcpyAsync(nout, nd, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipMemcpyAsync(gout, gd, 3 * n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    }
    if (out_space == NAO_MEM_HOST || D_space == NAO_MEM_HOST) HIP_TRY(c, hipStreamSynchronize(c->stream));
    return NAO_OK;
}

nao_status nao_pulay_forces(nao_system s, const double* D, const double* Q, const double* v, nao_memspace in_space,
                            nao_precision prec, double* F, nao_memspace F_space)
{
    if (!s) return (g_thread_error = "system is NULL", NAO_ERR_INVALID_ARG);
    nao_ctx c = s->ctx;
    nao_status st = check_ctx(c);
    if (st != NAO_OK) return st;
    if (prec != NAO_FP64 && prec != NAO_FP32)
        return (set_err(c, "the forces run in FP64 or FP32"), NAO_ERR_INVALID_ARG);
    const int64_t n = s->n_points, nb = s->basis.n_basis, na = s->basis.n_atoms;
    if (!F || (nb > 0 && (!D || !Q)) || (n > 0 && !v)) return (set_err(c, "NULL D, Q, v or F"), NAO_ERR_INVALID_ARG);
    if ((in_space != NAO_MEM_HOST && in_space != NAO_MEM_DEVICE) || (F_space != NAO_MEM_HOST && F_space != NAO_MEM_DEVICE))
        return (set_err(c, "bad memspace"), NAO_ERR_INVALID_ARG);
    if ((st = ensure_gscratch(s, 4)) != NAO_OK) return st;  // gradient and lap phi: 4 per basis value
    const double* Dd = D;
    const double* Qd = Q;
    const double* vd = v;
    if (in_space == NAO_MEM_HOST) {
        if (nb > 0) {
            if ((st = ensure(c, s->d_D, nb * nb * sizeof(double))) != NAO_OK) return st;
            if ((st = ensure(c, s->d_Q, nb * nb * sizeof(double))) != NAO_OK) return st;
            HIP_TRY(c, hipMemcpyAsync(s->d_D.p, D, nb * nb * sizeof(double), hipMemcpyHostToDevice, c->stream));
            HIP_TRY(c, hipMemcpyAsync(s->d_Q.p, Q, nb * nb * sizeof(double), hipMemcpyHostToDevice, c->stream));
            Dd = s->d_D.as<double>();
            Qd = s->d_Q.as<double>();
        }
        if (n > 0) {
            if ((st = ensure(c, s->d_v, n * sizeof(double))) != NAO_OK) return st;
            HIP_TRY(c, hipMemcpyAsync(s->d_v.p, v, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
            vd = s->d_v.as<double>();
        }
    }
    if ((st = ensure(c, s->d_fb, std::max<int64_t>(1, 3 * nb) * sizeof(double))) != NAO_OK) return st;
    if ((st = ensure(c, s->d_atom_first, (na + 1) * sizeof(int64_t))) != NAO_OK) return st;
    HIP_TRY(c, hipMemcpyAsync(s->d_atom_first.p, s->basis.atom_first.data(), (na + 1) * sizeof(int64_t),
                              hipMemcpyHostToDevice, c->stream));
    double* Fd = F;
    if (F_space == NAO_MEM_HOST) {
        if ((st = ensure(c, s->d_F, std::max<int64_t>(1, 3 * na) * sizeof(double))) != NAO_OK) return st;
        Fd = s->d_F.as<double>();
    }
    LAUNCH(c, "fill", launch_fill(s->d_fb.as<double>(), 3 * nb, 0.0, c->stream));
    LAUNCH(c, "wv", launch_wv(s->d_pw.as<double>(), s->d_perm.as<int32_t>(), vd, s->d_wv.as<double>(), n, c->stream));
    const Mode mode = exec_mode(c, prec);
    const bool f32 = prec != NAO_FP64;
    const bool ovl = overlap_ext(s, 4);
    std::vector<DevSeg> segs;
    for (const Block& b : s->blocks) {
        DevSeg g = make_seg(s, b, false);
        g.D = Dd;
        g.Q = Qd;
        g.wv = s->d_wv.as<double>();
        g.fb = s->d_fb.as<double>();
        g.gphi = c->gscratch;
        if (ovl && (segs.size() & 1)) {
            g.phi = c->scratch2;
            g.gphi = c->gscratch2;
        }
        segs.push_back(g);
    }
    if (!segs.empty()) {
        HIP_TRY(c, hipMemcpyAsync(s->d_segs.p, segs.data(), segs.size() * sizeof(DevSeg), hipMemcpyHostToDevice,
                                  c->stream));
        DevSeg* dseg = s->d_segs.as<DevSeg>();
        st = block_loop(
            c, segs.size(), ovl, f32 ? "basis_gradlap_f32" : "basis_gradlap_f64", f32 ? "nforce_f32" : "nforce_f64",
            [&](size_t k, hipStream_t q) {
                return launch_basis(dseg + k, 1, segs[k].unit_count, s->spline_lds, f32, q, 0, EXTRA_GRAD_H);
            },
            [&](size_t k) { return launch_n_force(mode, dseg + k, 1, segs[k].item_count, c->stream); });
        if (st != NAO_OK) return st;
    }
    LAUNCH(c, "force_atoms", launch_force_atoms(s->d_fb.as<double>(), s->d_atom_first.as<int64_t>(), na, Fd, c->stream));
    if (F_space == NAO_MEM_HOST && na > 0)
        HIP_TRY(c, hipMemcpyAsync(F, Fd, 3 * na * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (F_space == NAO_MEM_HOST || in_space == NAO_MEM_HOST) HIP_TRY(c, hipStreamSynchronize(c->stream));
    return NAO_OK;
}

nao_status nao_run_many(nao_ctx c, const nao_work* work, int64_t n_work, nao_precision prec, void* hip_stream,
                        uint32_t flags)
{
    nao_status st = check_ctx(c);
    if (st != NAO_OK) return st;
    if ((st = check_prec(c, prec)) != NAO_OK) return st;
    if (n_work < 0 || (n_work > 0 && !work)) return (set_err(c, "bad work list"), NAO_ERR_INVALID_ARG);
    if (flags & ~NAO_RUN_CAPTURE_GRAPH) return (set_err(c, "unknown flags"), NAO_ERR_INVALID_ARG);
    const bool capture = (flags & NAO_RUN_CAPTURE_GRAPH) != 0;
    bool electrons = false;
    for (int64_t k = 0; k < n_work; ++k) {
        const nao_work& w = work[k];
        if (!w.sys || w.sys->ctx->device != c->device)
            return (set_err(c, "work entry with a system on another device"), NAO_ERR_INVALID_ARG);
        if (capture && w.sys->ctx != c)
            return (set_err(c, "graph capture needs every system to belong to the context"), NAO_ERR_INVALID_ARG);
        if (w.op != 0 && w.op != 1) return (set_err(c, "work op must be 0 (H) or 1 (density)"), NAO_ERR_INVALID_ARG);
        const bool need_in = w.op == 0 ? w.sys->n_points > 0 : w.sys->basis.n_basis > 0;
        if ((need_in && !w.in) || !w.out) return (set_err(c, "NULL work pointer"), NAO_ERR_INVALID_ARG);
        if (w.n_electrons && w.op != 1) return (set_err(c, "n_electrons is for density entries"), NAO_ERR_INVALID_ARG);
        electrons = electrons || w.n_electrons;
    }
    if (electrons && capture)
        return (set_err(c, "n_electrons cannot be written by a captured graph"), NAO_ERR_INVALID_ARG);
    if (n_work == 0) return NAO_OK;
    // another stream: it waits for the context's work, and the context's stream for it
    hipStream_t own = c->stream, user = hip_stream ? static_cast<hipStream_t>(hip_stream) : own;
    if (user != own) {
        hipEvent_t ev = take_event(c);
        if (!ev) return (set_err(c, "event creation failed"), NAO_ERR_HIP);
        HIP_TRY(c, hipEventRecord(ev, own));
        HIP_TRY(c, hipStreamWaitEvent(user, ev, 0));
        c->pool.push_back(ev);
        c->stream = user;
    }
    try {
        st = run_many_impl(c, work, n_work, prec, capture);
        for (int64_t k = 0; st == NAO_OK && k < n_work; ++k) {
            const nao_work& w = work[k];
            if (!w.n_electrons) continue;
            const hipError_t e = launch_weighted_sum(w.sys->d_pw.as<double>(), w.sys->d_perm.as<int32_t>(), w.out,
                                                     w.sys->n_points, c->wsum, c->wsum + WSUM_BLOCKS, c->stream);
            if (e == hipSuccess)
                (void)hipMemcpyAsync(w.n_electrons, c->wsum + WSUM_BLOCKS, sizeof(double), hipMemcpyDeviceToHost,
                                     c->stream);
            if (e != hipSuccess) st = hip_fail(c, e, "electron count");
        }
        if (st == NAO_OK && electrons) {
            const hipError_t e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) st = hip_fail(c, e, "nao_run_many");
        }
    } catch (const std::bad_alloc&) {
        set_err(c, "host allocation failed");
        st = NAO_ERR_OUT_OF_MEMORY;
    }
    if (user != own) {
        c->stream = own;
        hipEvent_t ev = take_event(c);
        if (!ev) return (set_err(c, "event creation failed"), NAO_ERR_HIP);
        HIP_TRY(c, hipEventRecord(ev, user));
        HIP_TRY(c, hipStreamWaitEvent(own, ev, 0));
        c->pool.push_back(ev);
    }
    return st;
}

}  // extern "C"

// ------------------------------------------------------------------------------------------
// autotuner: (Hamiltonian tile width, execution-group size) per device, precision and shape

namespace {

std::string tune_cache_path()
{
    if (const char* p = std::getenv("NAO_TUNE_CACHE")) return p;
    const char* home = std::getenv("HOME");
    return std::string(home ? home : "/tmp") + "/.cache/nao_tune.json";
}

// {"key": [h_tile, group_max], ...}, one entry per line
std::map<std::string, std::pair<int, int>> tune_load()
{
    std::map<std::string, std::pair<int, int>> out;
    std::ifstream f(tune_cache_path());
    std::string line;
    while (std::getline(f, line)) {
        const size_t q0 = line.find('"');
        if (q0 == std::string::npos) continue;
        const size_t q1 = line.find('"', q0 + 1);
        if (q1 == std::string::npos) continue;
        const size_t b0 = line.find('[', q1);
        if (b0 == std::string::npos) continue;
        int a = 0, b = 0;
        if (std::sscanf(line.c_str() + b0 + 1, "%d , %d", &a, &b) == 2) out[line.substr(q0 + 1, q1 - q0 - 1)] = {a, b};
    }
    return out;
}

void tune_save(const std::map<std::string, std::pair<int, int>>& c)
{
    const std::string path = tune_cache_path();
    for (size_t k = 1; k < path.size(); ++k)
        if (path[k] == '/') (void)::mkdir(path.substr(0, k).c_str(), 0755);
    const std::string tmp = path + ".tmp" + std::to_string((long)::getpid());
    {
        std::ofstream f(tmp);
        if (!f) return;
        f << "{\n";
        size_t k = 0;
        for (const auto& kv : c)
            f << "  \"" << kv.first << "\": [" << kv.second.first << ", " << kv.second.second << "]"
              << (++k < c.size() ? ",\n" : "\n");
        f << "}\n";
    }
    std::rename(tmp.c_str(), path.c_str());
}

// Shape class of a system: device, precision, work-weighted mean list length and mean batch
// size of its batches (both bucketed), batch-size limit.
std::string tune_key(nao_system s, nao_precision prec)
{
    hipDeviceProp_t prop;
    std::string dev = "gpu";
    if (hipGetDeviceProperties(&prop, s->ctx->device) == hipSuccess)
        dev = std::string(prop.gcnArchName).substr(0, std::string(prop.gcnArchName).find(':')) + "x" +
              std::to_string(prop.multiProcessorCount);
    double bm2 = 0.0, bm = 0.0, pts = 0.0, nb = 0.0;
    for (size_t b = 0; b + 1 < s->batch_ptr.size(); ++b) {
        double m = 0.0;
        for (int64_t q = s->atom_ptr[b]; q < s->atom_ptr[b + 1]; ++q)
            m += (double)(s->basis.atom_first[s->atoms[q] + 1] - s->basis.atom_first[s->atoms[q]]);
        if (m == 0.0) continue;
        const double B = (double)(s->batch_ptr[b + 1] - s->batch_ptr[b]);
        bm2 += B * m * m;
        bm += B * m;
        pts += B;
        nb += 1.0;
    }
    const int mclass = bm > 0 ? (int)std::lround(bm2 / bm / 32.0) * 32 : 0;
    const int bclass = nb > 0 ? (int)std::lround(pts / nb / 8.0) * 8 : 0;
    static const char* pn[] = {"fp64", "fp32", "bf16x3", "bf16x6"};
    return dev + "/" + pn[prec] + "/m" + std::to_string(mclass) + "/b" + std::to_string(bclass) + "/max" +
           std::to_string(s->max_batch);
}

nao_status tune_apply(nao_system s, int h_tile, int group_max)
{
    nao_status st = NAO_OK;
    if (s->group_max != group_max && (st = nao_system_set_group_max(s, group_max)) != NAO_OK) return st;
    if (s->h_tile != h_tile && (st = nao_system_set_h_tile(s, h_tile)) != NAO_OK) return st;
    return NAO_OK;
}

}  // namespace

extern "C" nao_status nao_system_autotune(nao_system s, nao_precision prec, const double* v, const double* D,
                                          nao_memspace space, uint32_t flags, int32_t* h_tile_out,
                                          int32_t* group_max_out, double* best_ms)
{
    if (!s) return (g_thread_error = "system is NULL", NAO_ERR_INVALID_ARG);
    nao_ctx c = s->ctx;
    nao_status st = check_ctx(c);
    if (st != NAO_OK) return st;
    if ((st = check_prec(c, prec)) != NAO_OK) return st;
    if (flags & ~NAO_TUNE_FORCE) return (set_err(c, "unknown flags"), NAO_ERR_INVALID_ARG);
    const int64_t nb = s->basis.n_basis, np = s->n_points;
    if ((np > 0 && !v) || (nb > 0 && !D)) return (set_err(c, "NULL v or D"), NAO_ERR_INVALID_ARG);
    std::string key;
    std::map<std::string, std::pair<int, int>> cache;
    try {
        key = tune_key(s, prec);
        cache = tune_load();
    } catch (...) {
        return (set_err(c, "host allocation failed"), NAO_ERR_OUT_OF_MEMORY);
    }
    auto report = [&](int ht, int gm, double ms) {
        if (h_tile_out) *h_tile_out = ht;
        if (group_max_out) *group_max_out = gm;
        if (best_ms) *best_ms = ms;
    };
    auto hit = cache.find(key);
    if (!(flags & NAO_TUNE_FORCE) && hit != cache.end()) {
        if ((st = tune_apply(s, hit->second.first, hit->second.second)) != NAO_OK) return st;
        report(hit->second.first, hit->second.second, -1.0);
        return NAO_OK;
    }
    // device-side inputs and outputs for the timing runs
    DevArray dv, dD, dH, dn;
    auto release = [&]() {
        (void)hipStreamSynchronize(c->stream);
        for (DevArray* a : {&dv, &dD, &dH, &dn}) dev_free(c, a->p, a->bytes);
    };
    const double* vin = v;
    const double* Din = D;
    if (space == NAO_MEM_HOST) {
        if ((st = upload(c, dv, v, np * sizeof(double))) != NAO_OK) return release(), st;
        if ((st = upload(c, dD, D, nb * nb * sizeof(double))) != NAO_OK) return release(), st;
        vin = dv.as<double>();
        Din = dD.as<double>();
    }
    if ((st = ensure(c, dH, std::max<int64_t>(1, nb * nb) * sizeof(double))) != NAO_OK) return release(), st;
    if ((st = ensure(c, dn, std::max<int64_t>(1, np) * sizeof(double))) != NAO_OK) return release(), st;
    std::vector<std::pair<int, int>> cand;
    const bool dense = prec == NAO_FP64 || prec == NAO_FP32;
    for (int gm : {256, 192, 128})
        for (int ht : {64, 128})
            if (dense || ht == 64) cand.push_back({ht, gm});
    hipEvent_t e0 = take_event(c), e1 = take_event(c);
    if (!e0 || !e1) return release(), (set_err(c, "event creation failed"), NAO_ERR_HIP);
    const bool prof = c->prof;
    c->prof = false;
    double best = 1e300;
    std::pair<int, int> pick = {s->h_tile, s->group_max};
    for (const auto& cf : cand) {
        if ((st = tune_apply(s, cf.first, cf.second)) != NAO_OK) break;
        // one warm-up, then one timed density + Hamiltonian pair
        if ((st = nao_update_density(s, Din, NAO_MEM_DEVICE, prec, dn.as<double>(), NAO_MEM_DEVICE, nullptr)) != NAO_OK ||
            (st = nao_integrate_h(s, vin, NAO_MEM_DEVICE, prec, dH.as<double>(), NAO_MEM_DEVICE)) != NAO_OK)
            break;
        if (hipEventRecord(e0, c->stream) != hipSuccess) { st = NAO_ERR_HIP; break; }
        if ((st = nao_update_density(s, Din, NAO_MEM_DEVICE, prec, dn.as<double>(), NAO_MEM_DEVICE, nullptr)) != NAO_OK ||
            (st = nao_integrate_h(s, vin, NAO_MEM_DEVICE, prec, dH.as<double>(), NAO_MEM_DEVICE)) != NAO_OK)
            break;
        float ms = 0.0f;
        if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            st = NAO_ERR_HIP;
            break;
        }
        if (ms < best) {
            best = ms;
            pick = cf;
        }
    }
    c->prof = prof;
    c->pool.push_back(e0);
    c->pool.push_back(e1);
    release();
    if (st == NAO_ERR_HIP) return hip_fail(c, hipGetLastError(), "autotune timing");
    if (st != NAO_OK) return st;
    if ((st = tune_apply(s, pick.first, pick.second)) != NAO_OK) return st;
    try {
        cache[key] = pick;
        tune_save(cache);
    } catch (...) {
    }
    report(pick.first, pick.second, best);
    return NAO_OK;
}
