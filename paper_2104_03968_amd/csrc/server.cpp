// Request server: a stream of independent FLD diffusion solves of mixed sizes
// (2D and 3D), continuously batched on one GPU.
//
//  * Memory: every device buffer of a request (its plan's tables and multigrid
//    fields, a copy of its inputs and its result) is carved out of one arena the
//    caller provides; a request is admitted only when a slot is free and the
//    arena has room (first fit, FIFO order, no overtaking), so a burst of
//    arrivals queues instead of failing.
//  * Work: a request's coefficient pass and initial residual run on its own
//    single-grid plan as it is admitted; its iterations run inside a composite
//    plan over every resident request, so each multigrid phase is one launch for
//    all of them.  The composite plan is rebuilt at iteration boundaries when
//    requests join or leave; each request's solver state carries over.
//  * Results: a finished request's iterate is copied to its result buffer,
//    which stays in the arena until fld_release.
// Per request, the kernels, tiles and reduction orders are those of a solve of
// that grid alone, so the result does not depend on what else is resident.
#include "fld_internal.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

namespace fld {
namespace {

constexpr size_t kNoOff = ~size_t(0);

// First-fit allocator over [0, bytes) of the arena, 256-byte granules.
class Arena {
public:
    void init(size_t bytes) {
        total_ = bytes / kAlign * kAlign;
        free_.clear();
        if (total_) free_[0] = total_;
        used_ = 0;
    }
    size_t alloc(size_t n) {
        n = align_up(std::max<size_t>(n, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const size_t off = it->first, sz = it->second;
            free_.erase(it);
            if (sz > n) free_[off + n] = sz - n;
            used_ += n;
            return off;
        }
        return kNoOff;
    }
    void release(size_t off, size_t n) {
        if (off == kNoOff) return;
        n = align_up(std::max<size_t>(n, 1));
        used_ -= n;
        auto it = free_.emplace(off, n).first;
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
    size_t total() const { return total_; }
    size_t free_bytes() const { return total_ - used_; }
    bool fits(size_t n) const {
        n = align_up(std::max<size_t>(n, 1));
        for (auto& kv : free_)
            if (kv.second >= n) return true;
        return false;
    }

private:
    size_t total_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;
};

double now_s() {
    using clk = std::chrono::steady_clock;
    static const clk::time_point t0 = clk::now();
    return std::chrono::duration<double>(clk::now() - t0).count();
}

enum Phase { PENDING = 0, RESIDENT = 1, DONE = 2 };

struct Request {
    uint64_t ticket = 0;
    fld_grid grid{};
    double dt = 0.0;
    int64_t n = 0;
    const double* E_dev = nullptr;            // device inputs (caller keeps them until done)
    const double* kr_dev = nullptr;
    hipEvent_t ready = nullptr;               // device inputs: written once this event completes
    std::vector<double> E_host, kr_host;      // host inputs, copied at submit
    size_t plan_bytes = 0;                    // single-grid plan workspace
    size_t off_ws = kNoOff, off_in = kNoOff, off_out = kNoOff;
    std::unique_ptr<Plan> plan;
    GridState state{};
    int phase = PENDING;
    int status = FLD_PENDING;
    fld_stats stats{};
    double t_submit = 0, t_admit = 0, t_start = 0, t_done = 0;

    ~Request() {
        if (ready) (void)hipEventDestroy(ready);
    }
};

}  // namespace

struct Server {
    int device = 0;
    fld_server_opts sopts{};
    fld_opts opts{};                          // solver options every request runs with
    char* arena_base = nullptr;
    Arena arena;
    size_t off_tables = kNoOff, tables_bytes = 0;   // composite plan tables
    size_t off_states = kNoOff;               // solver state of every slot (composite and request plans)
    GridState* d_states = nullptr;
    hipStream_t stream = nullptr;
    // pinned staging of the plans' table uploads: one region per slot for the request
    // plans, two alternating regions for the composite (an event guards each)
    static constexpr size_t kReqStage = 128 * 1024;
    char* pin_stage_req = nullptr;
    char* pin_stage_comp[2] = {nullptr, nullptr};
    hipEvent_t comp_ev[2] = {nullptr, nullptr};
    int comp_buf = 0;
    // pinned staging shared by the composite and the request plans
    StepIO* pin_io = nullptr;
    GridState* pin_req = nullptr;             // one state per slot (request plans)
    GridState* pin_comp = nullptr;            // composite states
    Control* pin_ctrl = nullptr;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> pending;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> all;
    std::vector<Request*> resident;           // order = composite grid order
    std::unique_ptr<Plan> comp;
    bool dirty = true;                        // composite must be rebuilt
    bool stop = false;
    int error = FLD_OK;
    uint64_t next_ticket = 1;
    std::vector<int> free_slots;
    std::unordered_map<uint64_t, int> slot_of;
    fld_server_info info{};
    std::thread worker;

    ~Server();
    void run();
    int admit_locked(std::vector<Request*>& admitted);
    int start_request(Request* r, int slot);
    int rebuild();
    int round();
    void fail_all(int code);
};

namespace {

int request_plan(const fld_opts& opts, const fld_grid& g, std::unique_ptr<Plan>& out) {
    out = std::make_unique<Plan>();
    return plan_init(*out, &g, 1, opts);
}

}  // namespace

Server::~Server() {
    {
        std::lock_guard<std::mutex> lk(mu);
        stop = true;
    }
    cv_work.notify_all();
    if (worker.joinable()) worker.join();
    comp.reset();
    all.clear();
    if (stream) (void)hipStreamDestroy(stream);
    if (pin_io) (void)hipHostFree(pin_io);
    if (pin_req) (void)hipHostFree(pin_req);
    if (pin_comp) (void)hipHostFree(pin_comp);
    if (pin_ctrl) (void)hipHostFree(pin_ctrl);
    if (pin_stage_req) (void)hipHostFree(pin_stage_req);
    for (int k = 0; k < 2; ++k) {
        if (pin_stage_comp[k]) (void)hipHostFree(pin_stage_comp[k]);
        if (comp_ev[k]) (void)hipEventDestroy(comp_ev[k]);
    }
}

void Server::fail_all(int code) {
    std::lock_guard<std::mutex> lk(mu);
    error = code;
    auto fail = [&](Request* r) {
        if (r->phase == DONE) return;
        r->phase = DONE;
        r->status = code;
        r->stats.status = code;
        r->t_done = now_s();
        r->plan.reset();
        arena.release(r->off_ws, r->plan_bytes);
        arena.release(r->off_in, 16 * (size_t)r->n);
        arena.release(r->off_out, 8 * (size_t)r->n);
        r->off_ws = r->off_in = r->off_out = kNoOff;
        info.failed++;
    };
    for (Request* r : pending) fail(r);
    pending.clear();
    for (Request* r : resident) fail(r);
    resident.clear();
    info.pending = 0;
    info.resident = 0;
    cv_done.notify_all();
}

// Admit pending requests in arrival order while a slot is free and the arena can
// hold the request's plan, input copy and result.  Called with `mu` held.
int Server::admit_locked(std::vector<Request*>& admitted) {
    while (!pending.empty() && !free_slots.empty()) {
        Request* r = pending.front();
        const size_t in_bytes = 16 * (size_t)r->n, out_bytes = 8 * (size_t)r->n;
        const size_t ws = arena.alloc(r->plan_bytes);
        if (ws == kNoOff) break;
        const size_t in = arena.alloc(in_bytes);
        if (in == kNoOff) { arena.release(ws, r->plan_bytes); break; }
        const size_t out = arena.alloc(out_bytes);
        if (out == kNoOff) {
            arena.release(ws, r->plan_bytes);
            arena.release(in, in_bytes);
            break;
        }
        pending.pop_front();
        r->off_ws = ws;
        r->off_in = in;
        r->off_out = out;
        r->phase = RESIDENT;
        r->t_admit = now_s();
        const int slot = free_slots.back();
        free_slots.pop_back();
        slot_of[r->ticket] = slot;
        admitted.push_back(r);
        info.admitted++;
    }
    info.pending = (int32_t)pending.size();
    return FLD_OK;
}

// Copy a newly admitted request's inputs into the arena and run its coefficient
// pass and initial residual on its own single-grid plan, whose solver state is the
// request's slot of the shared state array (asynchronous: the table upload, the input
// copies and the prologue are ordered on the server stream; nothing waits here).
int Server::start_request(Request* r, int slot) {
    Plan& p = *r->plan;
    p.own_pinned = false;
    p.hIO = pin_io + slot;
    p.hS = pin_req + slot;
    p.hCtrl = pin_ctrl;
    p.ext_state = d_states;
    p.grid_slot.assign(1, slot);
    p.ext_state_init = true;
    p.bind_stream = stream;
    p.bind_staging = pin_stage_req + (size_t)slot * kReqStage;   // free: the slot's last user is retired
    p.bind_staging_bytes = kReqStage;
    int rc = plan_bind(p, arena_base + r->off_ws, r->plan_bytes, nullptr);
    if (rc != FLD_OK) return rc;
    double* inE = reinterpret_cast<double*>(arena_base + r->off_in);
    double* inK = inE + r->n;
    double* out = reinterpret_cast<double*>(arena_base + r->off_out);
    const size_t nb = 8 * (size_t)r->n;
    if (r->E_dev) {
        // the caller's producer stream may still be writing the inputs
        if (r->ready) FLD_HIP(hipStreamWaitEvent(stream, r->ready, 0));
        FLD_HIP(hipMemcpyAsync(inE, r->E_dev, nb, hipMemcpyDeviceToDevice, stream));
        FLD_HIP(hipMemcpyAsync(inK, r->kr_dev, nb, hipMemcpyDeviceToDevice, stream));
    } else {
        FLD_HIP(hipMemcpyAsync(inE, r->E_host.data(), nb, hipMemcpyHostToDevice, stream));
        FLD_HIP(hipMemcpyAsync(inK, r->kr_host.data(), nb, hipMemcpyHostToDevice, stream));
    }
    const StepIO io{inE, inK, out, r->dt};
    if ((rc = plan_upload_io(p, &io, stream)) != FLD_OK) return rc;
    if ((rc = plan_prologue(p, stream)) != FLD_OK) return rc;
    r->t_start = now_s();
    return FLD_OK;
}

// Composite plan over the resident requests: fields stay where each request's plan
// put them and the solver states stay in their slots, so a rebuild is the host
// work of the descriptors and lists plus one asynchronous table upload, ordered on
// the stream after the rounds that used the previous tables.
int Server::rebuild() {
    comp.reset();
    dirty = false;
    if (resident.empty()) return FLD_OK;
    std::vector<fld_grid> grids;
    auto c = std::make_unique<Plan>();
    for (Request* r : resident) {
        grids.push_back(r->grid);
        c->grid_slot.push_back(slot_of[r->ticket]);
        c->field_base.push_back(reinterpret_cast<char*>(r->plan->ws) + r->plan->field_off[0]);
    }
    int rc = plan_init(*c, grids.data(), (int)grids.size(), opts);
    if (rc != FLD_OK) return rc;
    if (c->ws_bytes > tables_bytes) {
        g_last_error = "server: composite tables exceed their reserved region";
        return FLD_ERR_HIP;
    }
    c->own_pinned = false;
    c->hIO = pin_io;
    c->hS = pin_comp;
    c->hCtrl = pin_ctrl;
    c->ext_state = d_states;
    c->ext_state_init = false;                 // the states carry over
    comp_buf ^= 1;                             // the other staging region: its last copy is done
    FLD_HIP(hipEventSynchronize(comp_ev[comp_buf]));
    c->bind_stream = stream;
    c->bind_staging = pin_stage_comp[comp_buf];
    c->bind_staging_bytes = tables_bytes;
    if ((rc = plan_bind(*c, arena_base + off_tables, tables_bytes, nullptr)) != FLD_OK) return rc;
    FLD_HIP(hipEventRecord(comp_ev[comp_buf], stream));
    comp = std::move(c);
    return FLD_OK;
}

// Run the resident requests' iterations, then retire the finished ones.
int Server::round() {
    Plan& c = *comp;
    const int G = c.ngrids();
    const int k = std::max(1, sopts.cycles_per_round);
    for (int i = 0; i < k; ++i) plan_cycle(c, stream);
    if (c.krylov) plan_verify(c, stream);
    FLD_HIP(hipGetLastError());
    // every slot's state in one copy (the resident requests are a subset of the slots)
    FLD_HIP(hipMemcpyAsync(pin_comp, d_states, (size_t)sopts.max_slots * sizeof(GridState), hipMemcpyDeviceToHost,
                           stream));
    FLD_HIP(hipStreamSynchronize(stream));
    std::vector<Request*> finished;
    for (int g = 0; g < G; ++g) {
        Request* r = resident[g];
        r->state = pin_comp[slot_of[r->ticket]];
        if (!r->state.active) finished.push_back(r);
    }
    info.rounds++;
    if (finished.empty()) return FLD_OK;
    for (Request* r : finished) plan_output(*r->plan, stream);
    FLD_HIP(hipGetLastError());
    FLD_HIP(hipStreamSynchronize(stream));
    const double t = now_s();
    std::lock_guard<std::mutex> lk(mu);
    for (Request* r : finished) {
        plan_stats(*r->plan, r->state, 0, &r->stats);
        r->status = r->stats.status;
        r->t_done = t;
        r->phase = DONE;
        r->plan.reset();
        arena.release(r->off_ws, r->plan_bytes);
        arena.release(r->off_in, 16 * (size_t)r->n);
        r->off_ws = r->off_in = kNoOff;
        r->E_host.clear();
        r->E_host.shrink_to_fit();
        r->kr_host.clear();
        r->kr_host.shrink_to_fit();
        free_slots.push_back(slot_of[r->ticket]);
        slot_of.erase(r->ticket);
        info.completed++;
        if (r->status != FLD_OK) info.failed++;
        info.cells_done += r->n;
        resident.erase(std::find(resident.begin(), resident.end(), r));
    }
    info.resident = (int32_t)resident.size();
    dirty = true;
    cv_done.notify_all();
    return FLD_OK;
}

void Server::run() {
    if (hipSetDevice(device) != hipSuccess) {
        fail_all(FLD_ERR_HIP);
        return;
    }
    while (true) {
        std::vector<Request*> admitted;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stop || !pending.empty() || !resident.empty(); });
            if (stop) return;
            admit_locked(admitted);
        }
        int rc = FLD_OK;
        for (Request* r : admitted)
            if ((rc = start_request(r, slot_of[r->ticket])) != FLD_OK) break;
        if (rc == FLD_OK && !admitted.empty()) {
            // no wait: the prologues wrote the states into their slots in stream order
            std::lock_guard<std::mutex> lk(mu);
            for (Request* r : admitted) resident.push_back(r);
            info.resident = (int32_t)resident.size();
            dirty = true;
        }
        if (rc == FLD_OK && dirty) rc = rebuild();
        if (rc == FLD_OK && comp) rc = round();
        if (rc != FLD_OK) {
            fail_all(rc);
            return;
        }
    }
}

}  // namespace fld

// ============================================================================
// C ABI
// ============================================================================
struct fld_server_s {
    fld::Server s;
};

extern "C" {

void fld_server_opts_default(fld_server_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->max_slots = 64;
    o->precision = FLD_PREC_MIXED;
    o->rtol = 1e-10;
    o->max_cycles = 50;
    o->c = 1.0;
    o->limiter = FLD_LIMITER_LP;
    o->cycles_per_round = 2;
}

int32_t fld_server_create(const fld_server_opts* o, void* arena_dev, size_t arena_bytes, fld_server_t* out) {
    if (!o || !arena_dev || !out) return FLD_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(arena_dev) % fld::kAlign) != 0) return FLD_ERR_INVALID_ARG;
    if (o->max_slots < 1 || o->max_slots > 4096 || o->cycles_per_round < 1) return FLD_ERR_INVALID_ARG;
    *out = nullptr;
    try {
        auto h = std::make_unique<fld_server_s>();
        fld::Server& s = h->s;
        s.sopts = *o;
        fld_opts_default(&s.opts);
        s.opts.c = o->c;
        s.opts.limiter = o->limiter;
        s.opts.precision = o->precision;
        s.opts.rtol = o->rtol;
        s.opts.max_cycles = o->max_cycles;
        s.opts.use_graph = 0;
        s.opts.fmg = 0;                       // requests advance by rounds of V-cycles
        int rc = fld::validate_opts(s.opts);
        if (rc != FLD_OK) return rc;
        if (hipGetDevice(&s.device) != hipSuccess) return FLD_ERR_HIP;
        s.arena_base = static_cast<char*>(arena_dev);
        s.arena.init(arena_bytes);
        s.tables_bytes = fld::align_up((size_t)256 * 1024 + (size_t)o->max_slots * 24 * 1024);
        s.off_tables = s.arena.alloc(s.tables_bytes);
        if (s.off_tables == fld::kNoOff) return FLD_ERR_TOO_LARGE;
        const size_t M = (size_t)o->max_slots;
        s.off_states = s.arena.alloc(M * sizeof(fld::GridState));
        if (s.off_states == fld::kNoOff) return FLD_ERR_TOO_LARGE;
        s.d_states = reinterpret_cast<fld::GridState*>(s.arena_base + s.off_states);
        if (hipMemset(s.d_states, 0, M * sizeof(fld::GridState)) != hipSuccess) return FLD_ERR_HIP;
        if (hipHostMalloc((void**)&s.pin_stage_req, M * fld::Server::kReqStage, hipHostMallocDefault) != hipSuccess)
            return FLD_ERR_HIP;
        for (int k = 0; k < 2; ++k) {
            if (hipHostMalloc((void**)&s.pin_stage_comp[k], s.tables_bytes, hipHostMallocDefault) != hipSuccess)
                return FLD_ERR_HIP;
            if (hipEventCreateWithFlags(&s.comp_ev[k], hipEventDisableTiming) != hipSuccess) return FLD_ERR_HIP;
        }
        if (hipHostMalloc((void**)&s.pin_io, M * sizeof(fld::StepIO), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&s.pin_req, M * sizeof(fld::GridState), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&s.pin_comp, M * sizeof(fld::GridState), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&s.pin_ctrl, sizeof(fld::Control), hipHostMallocDefault) != hipSuccess)
            return FLD_ERR_HIP;
        if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess) return FLD_ERR_HIP;
        for (int dim = 2; dim <= 3; ++dim)
            if (fld::prepare_tail(dim, s.opts.precision == FLD_PREC_MIXED, fld::kTailLdsBudget) != 0)
                return FLD_ERR_HIP;
        for (int i = o->max_slots - 1; i >= 0; --i) s.free_slots.push_back(i);
        s.info.arena_bytes = s.arena.total();
        s.worker = std::thread([&s] { s.run(); });
        *out = h.release();
        return FLD_OK;
    } catch (...) {
        return FLD_ERR_INVALID_ARG;
    }
}

int32_t fld_server_destroy(fld_server_t server) {
    if (!server) return FLD_ERR_INVALID_ARG;
    delete server;
    return FLD_OK;
}

int32_t fld_submit(fld_server_t server, const fld_request* req, uint64_t* ticket) {
    if (!server || !req || !ticket) return FLD_ERR_INVALID_ARG;
    fld::Server& s = server->s;
    if (!req->E_in || !req->kappa_rho || !(req->dt > 0.0) || !std::isfinite(req->dt)) return FLD_ERR_INVALID_ARG;
    try {
        auto r = std::make_unique<fld::Request>();
        r->grid = req->grid;
        if (r->grid.ndim == 2) { r->grid.n[2] = 1; r->grid.h[2] = 1.0; }
        int rc = fld::validate_grid(r->grid);
        if (rc != FLD_OK) return rc;
        std::unique_ptr<fld::Plan> plan;
        if ((rc = fld::request_plan(s.opts, r->grid, plan)) != FLD_OK) return rc;
        r->n = plan->ncell[0];
        r->plan_bytes = plan->ws_bytes;
        r->plan = std::move(plan);
        r->dt = req->dt;
        const size_t need = fld::align_up(r->plan_bytes) + fld::align_up(16 * (size_t)r->n) +
                            fld::align_up(8 * (size_t)r->n);
        if (need > s.arena.total() - s.tables_bytes) return FLD_ERR_TOO_LARGE;
        if (req->inputs_on_device) {
            r->E_dev = req->E_in;
            r->kr_dev = req->kappa_rho;
            int cur = -1;
            if (hipGetDevice(&cur) != hipSuccess) return FLD_ERR_HIP;
            if (cur != s.device && hipSetDevice(s.device) != hipSuccess) return FLD_ERR_HIP;
            hipError_t e = hipEventCreateWithFlags(&r->ready, hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventRecord(r->ready, static_cast<hipStream_t>(req->stream));
            if (cur != s.device) (void)hipSetDevice(cur);
            if (e != hipSuccess) {
                fld::set_error("fld_submit: input event", e);
                return FLD_ERR_HIP;
            }
        } else {
            r->E_host.assign(req->E_in, req->E_in + r->n);
            r->kr_host.assign(req->kappa_rho, req->kappa_rho + r->n);
        }
        std::lock_guard<std::mutex> lk(s.mu);
        if (s.stop) return FLD_ERR_SHUTDOWN;
        if (s.error != FLD_OK) return s.error;
        r->ticket = s.next_ticket++;
        r->t_submit = fld::now_s();
        *ticket = r->ticket;
        s.pending.push_back(r.get());
        s.all[r->ticket] = std::move(r);
        s.info.submitted++;
        s.info.pending = (int32_t)s.pending.size();
    } catch (...) {
        return FLD_ERR_INVALID_ARG;
    }
    s.cv_work.notify_one();
    return FLD_OK;
}

static void fill_result(const fld::Request& r, fld_result* out, char* arena_base) {
    out->E_out = r.off_out != fld::kNoOff ? reinterpret_cast<double*>(arena_base + r.off_out) : nullptr;
    out->stats = r.stats;
    out->t_submit = r.t_submit;
    out->t_admit = r.t_admit;
    out->t_start = r.t_start;
    out->t_done = r.t_done;
}

int32_t fld_poll(fld_server_t server, uint64_t ticket, fld_result* out) {
    if (!server || !out) return FLD_ERR_INVALID_ARG;
    fld::Server& s = server->s;
    std::lock_guard<std::mutex> lk(s.mu);
    auto it = s.all.find(ticket);
    if (it == s.all.end()) return FLD_ERR_UNKNOWN_TICKET;
    const fld::Request& r = *it->second;
    if (r.phase != fld::DONE) return FLD_PENDING;
    fill_result(r, out, s.arena_base);
    return r.status;
}

int32_t fld_wait(fld_server_t server, uint64_t ticket, double timeout_s, fld_result* out) {
    if (!server || !out) return FLD_ERR_INVALID_ARG;
    fld::Server& s = server->s;
    std::unique_lock<std::mutex> lk(s.mu);
    auto it = s.all.find(ticket);
    if (it == s.all.end()) return FLD_ERR_UNKNOWN_TICKET;
    const fld::Request* r = it->second.get();
    const auto deadline = std::chrono::steady_clock::now() +
                          std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                              std::chrono::duration<double>(std::max(0.0, timeout_s)));
    s.cv_done.wait_until(lk, deadline, [&] { return r->phase == fld::DONE; });
    if (r->phase != fld::DONE) return FLD_PENDING;
    fill_result(*r, out, s.arena_base);
    return r->status;
}

int32_t fld_release(fld_server_t server, uint64_t ticket) {
    if (!server) return FLD_ERR_INVALID_ARG;
    fld::Server& s = server->s;
    {
        std::lock_guard<std::mutex> lk(s.mu);
        auto it = s.all.find(ticket);
        if (it == s.all.end()) return FLD_ERR_UNKNOWN_TICKET;
        fld::Request& r = *it->second;
        if (r.phase != fld::DONE) return FLD_PENDING;
        s.arena.release(r.off_out, 8 * (size_t)r.n);
        s.all.erase(it);
    }
    s.cv_work.notify_one();        // freed arena space may admit a waiting request
    return FLD_OK;
}

int32_t fld_server_info_get(fld_server_t server, fld_server_info* out) {
    if (!server || !out) return FLD_ERR_INVALID_ARG;
    fld::Server& s = server->s;
    std::lock_guard<std::mutex> lk(s.mu);
    *out = s.info;
    out->arena_free = s.arena.free_bytes();
    out->arena_bytes = s.arena.total();
    out->error = s.error;
    return FLD_OK;
}

}  // extern "C"
