// Host-side internals of the FLD runtime shared by the plan C ABI (runtime.cpp)
// and the request server (server.cpp): plans, work-lists, workspace layout and
// the step drivers.
#pragma once

#include "fld_device.hpp"
#include "fld.h"

#include <string>
#include <vector>

namespace fld {

extern thread_local std::string g_last_error;
void set_error(const char* where, hipError_t e);

#define FLD_HIP(call)                                   \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) {                         \
            ::fld::set_error(#call, e_);                \
            return FLD_ERR_HIP;                         \
        }                                               \
    } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Device-side work-list storage: levels[] and prefix[] of one JobList.
struct HostList {
    std::vector<int32_t> levels;
    std::vector<int32_t> prefix;   // size levels.size() + 1
    size_t off_levels = 0, off_prefix = 0;
    JobList dev{};                 // filled at bind

    bool empty() const { return levels.empty(); }
};

// One dimension's worth of work-lists (2D and 3D grids run in separate launches).
struct DimLists {
    int dim = 0;
    HostList l0_cell;                          // level 0, cell tiles
    std::vector<HostList> smooth;              // per depth, smoother tiles
    std::vector<HostList> restrict_;           // per depth, cell tiles of the coarse level
    std::vector<HostList> prolong;             // per depth, cell tiles of the fine level
    std::vector<HostList> coarsen;             // per depth, all levels with a coarser one
    std::vector<HostList> down2, up2;          // per depth, fused 2D tiles (same levels as smooth)
    std::vector<int> thr_dn, thr_up;           // per depth, workgroup size of those tiles (256 or 1024)
    std::vector<HostList> mdn, mup;            // per depth, row-marching windows (same levels)
    std::vector<char> march;                   // per depth: the passes march rows instead of tiles
    std::vector<int> mfz;                      // per depth, rows per marching window
    bool fused = false;
    std::vector<HostList> sw3, sr3;            // per depth, fused 3D sweep blocks (plain / restricting)
    std::vector<int> fz_r;                     // per depth, planes per block of the restricting sweep
    std::vector<int> fz_s;                     // per depth, planes per block of the plain sweeps
    bool fused3 = false;                       // fused 3D sweeps available (lists and xs laid out)
    int levels3 = 0;                           // leading depths that run fused sweeps
    HostList coarsest;                         // coarsest level of grids without a tail
    HostList tail;                             // first tail level of grids with a tail
    // per depth d: the tails / coarsest levels of the grids with wide levels below d
    // (the V-cycles of the full-multigrid start that begin at depth d)
    std::vector<HostList> tail_from, coarsest_from;
    size_t tail_smem = 0;                      // LDS bytes of the largest tail
    bool fin_fused = false;                    // finish reductions in the last block (small grids)
    bool fold = false;                         // CG scalars formed in the consuming kernels (mid-sized grids)
    HostList pq3;                              // level 0, marching CG tiles (zero-flux operators): z-march
                                               // (3D) or row march (2D, even rows)
    HostList rz3;                              // level 0, plain 3D sweep windows of kRz3Fz planes (the
                                               // last up sweep when it also forms r . z)
    int fz_pq = 16;                            // planes per z-march CG tile
    int maxdepth = 0;
};

struct Plan {
    int device = 0;
    fld_opts opts{};
    std::vector<fld_grid> grids;
    std::vector<LevelDesc> levels;             // host copy (device pointers after bind)
    std::vector<int32_t> level0;               // LevelDesc index of each grid's level 0
    std::vector<int32_t> nlev;                 // levels per grid
    std::vector<int64_t> ncell;                // cells per grid
    std::vector<int32_t> tail_lev;             // first tail level of each grid (-1: no tail)
    DimLists dl[2];                            // [0] = 2D, [1] = 3D
    bool mixed = false;
    bool krylov = true;
    bool has_dir = false;                      // some face is FLD_BC_DIRICHLET
    bool has_per = false;                      // some axis is periodic
    bool has_cont = false;                     // some face is continuous (linear extrapolation)
    // the operator differs from zero flux at some face (extra diagonal, wrapped or cut
    // neighbours): per-colour kernels and the boundary instantiation of the tail
    bool nb_bc() const { return has_dir || has_per || has_cont; }
    bool any_bc = false;                       // some face is not zero flux
    int nuc1 = 2, nuc2 = 2;                    // sweeps on the levels below the finest

    // workspace layout (byte offsets)
    size_t off_levels = 0, off_state = 0, off_stepio = 0, off_exio = 0, off_moio = 0, off_imio = 0, off_ctrl = 0;
    size_t ws_bytes = 0;
    static constexpr int kExSlots = 4;
    struct FieldOff {
        size_t x = 0, b = 0, w[3] = {0, 0, 0}, x32 = 0, b32 = 0, w32[3] = {0, 0, 0}, part = 0, scratch = 0;
        size_t X = 0, B0 = 0, R = 0, P[2] = {0, 0}, Q = 0, xs = 0;
        bool has_x = false, has_b = false, has_x32 = false, has_scratch = false, has_part = false;
        bool has_xs = false;
        bool lev0 = false, has_cg = false;
        size_t ad = 0, ad32 = 0;                // Dirichlet ghost couplings (plans with Dirichlet faces)
    };
    std::vector<FieldOff> foff;                // per level (relative to the grid's field base)
    std::vector<size_t> field_off;             // byte offset of each grid's fields in the workspace
    std::vector<size_t> field_bytes;           // bytes of each grid's fields
    std::vector<char*> field_base;             // if set: each grid's fields live here instead
    size_t table_bytes = 0;                    // descriptor / list region at the workspace start

    // bound state
    char* ws = nullptr;
    LevelDesc* dL = nullptr;
    GridState* dS = nullptr;
    StepIO* dIO = nullptr;
    ExchangeIO* dEx = nullptr;
    MomentsIO* dMo = nullptr;
    ImexIO* dIm = nullptr;                     // kImStages * ngrids stage tables
    Control* dCtrl = nullptr;
    StepIO* hIO = nullptr;                     // pinned staging
    ExchangeIO* hEx = nullptr;                 // pinned staging, kExSlots * ngrids
    MomentsIO* hMo = nullptr;                  // pinned staging, kExSlots * ngrids
    ImexIO* hIm = nullptr;                     // pinned staging, kImStages * ngrids
    static constexpr int kImStages = 3;
    Control* hCtrl = nullptr;                  // pinned
    GridState* hS = nullptr;                   // pinned
    bool own_pinned = true;                    // false: staging buffers belong to a server
    // staging in plain host memory for steps that must not allocate (fld_step_noalloc),
    // sized when the plan is built; io_host also carries every step's per-grid pointers
    std::vector<StepIO> io_host;
    std::vector<GridState> st_host;
    Control ctrl_host{};
    bool noalloc = false;                      // binding for one no-allocation step: no tuning, no graphs
    // Binding into shared state slots (the request server): the solver state of grid g
    // lives at ext_state[grid_slot[g]] instead of the workspace; ext_state_init: the bind
    // also writes fresh states there.  With bind_staging (pinned, bind_staging_bytes) the
    // bind's table upload is one asynchronous copy on bind_stream, else one synchronous copy.
    GridState* ext_state = nullptr;
    std::vector<int32_t> grid_slot;
    bool ext_state_init = true;
    hipStream_t bind_stream = nullptr;
    char* bind_staging = nullptr;
    size_t bind_staging_bytes = 0;
    hipEvent_t ex_done[kExSlots] = {};
    int ex_slot = 0;
    hipEvent_t mo_done[kExSlots] = {};
    int mo_slot = 0;
    int ex_last = -1;                          // slot of the last fld_exchange (profiling)
    int64_t max_n = 0;
    // launch shape: fused 2D tile (width class, rows) and the persistent-grid cap
    int tile_wide = 0;
    int tile_rows = 16;
    int tile_rows_c = 16;                      // fused 2D tile rows below the finest level
    int tile_rows_u = 16;                      // fused 2D tile rows of the finest level's up pass
    int nblk = 2048;
    int tile_depth = 32;                       // fused 3D sweep: planes per block
    int ncu = 256;                             // compute units of the plan's device (block balancing)
    int sweep3 = 1;                            // 1: fused 3D sweeps where available; 0: per colour
    int sweep3_levels = 0;                     // leading 3D depths with fused sweeps (0: by block count)
    int tune_source = 0;                       // 0 defaults / options, 1 timed at bind, 2 cache
    int tune_candidates = 0;
    double tune_us = 0.0;                      // timed multigrid part of one V-cycle
    bool tune_done = false;
    int last_cycles = 0;                       // cycles of the previous step (replay sizing)

    fld_gas last_gas{};                        // constants of the last fld_exchange (profiling)
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t fmg_graph = nullptr;            // the full-multigrid start (plans with fmg = 1)
    hipGraphExec_t fmg_graph_exec = nullptr;

    ~Plan();
    int ngrids() const { return (int)grids.size(); }
};

inline Plan::~Plan() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (fmg_graph_exec) (void)hipGraphExecDestroy(fmg_graph_exec);
    if (fmg_graph) (void)hipGraphDestroy(fmg_graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (auto& e : ex_done)
        if (e) (void)hipEventDestroy(e);
    for (auto& e : mo_done)
        if (e) (void)hipEventDestroy(e);
    if (own_pinned) {
        if (hIO) (void)hipHostFree(hIO);
        if (hEx) (void)hipHostFree(hEx);
        if (hMo) (void)hipHostFree(hMo);
        if (hCtrl) (void)hipHostFree(hCtrl);
        if (hS) (void)hipHostFree(hS);
    }
    if (hIm) (void)hipHostFree(hIm);           // only fld_imex_step allocates it
}


// Plan construction: hierarchy, work-lists and workspace layout (host only).
int validate_opts(const fld_opts& o);
int validate_grid(const fld_grid& g);
int plan_init(Plan& p, const fld_grid* grids, int ngrids, const fld_opts& opts);
// Bind device memory: tables at `dev`; fields at `dev` too unless field_base is set.
// init: initial per-grid solver states (nullptr: fresh).  Synchronous.
int plan_bind(Plan& p, void* dev, size_t bytes, const GridState* init);
// Per-step phases, asynchronous on s (the StepIO table must be on the device).
int plan_prologue(Plan& p, hipStream_t s);               // coefficients, norms, initial residual
void plan_cycle(Plan& p, hipStream_t s);                 // one V-cycle (+ CG update) for active grids
void plan_verify(Plan& p, hipStream_t s);                // true residual of grids CG reported converged
void plan_output(Plan& p, hipStream_t s);                // X -> E_out
void plan_stats(const Plan& p, const GridState& st, int g, fld_stats* out);
int plan_upload_io(Plan& p, const StepIO* io, hipStream_t s);
// The plan behind a C-ABI handle (NULL for NULL).
Plan* plan_of(fld_plan_t h);
// One fld_step on an unbound plan whose tables and fields are laid out in `dev` (bytes):
// binds without tuning or graph capture, stages through the plan's host arrays,
// steps, and leaves the plan unbound again.  Allocates nothing.
int plan_step_noalloc(Plan& p, void* dev, size_t bytes, const double* const* E_in, const double* const* kr,
                      double* const* E_out, const double* dt, hipStream_t s, fld_stats* stats);

// Autotuner (autotune.cpp): pick the launch shape of a bound plan by timing the
// multigrid part of a V-cycle for each candidate, or take it from the cache.
int plan_autotune(Plan& p);
void plan_vcycle_mg(Plan& p, hipStream_t s);             // the timed part: smoothing, transfers, tails
struct LaunchShape {
    int wide, rows, nblk, depth, sweep3, levels3, rows_c, rows_u;
};
int plan_set_shape(Plan& p, const LaunchShape& s);         // rebuild and upload the fused lists
LaunchShape plan_shape(const Plan& p);

}  // namespace fld
