// Device-side data structures shared by the HIP kernels and the host runtime.
//
// Every multigrid phase is one launch over a work-list of (level, tile) items
// drawn from any number of grids, so a single grid and a batch of uneven grids
// run through the same kernels.  A level descriptor (LevelDesc) names the
// arrays of one level of one grid inside the caller's workspace; a JobList
// names which levels a launch covers and where each level's tiles start.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fld {

// Cell-parallel kernels: one thread per cell, 64 x 4 (x 1) cell tiles.
constexpr int kTX = 64;
constexpr int kTY = 4;
constexpr int kBlock = 256;
// MI355X: 256 compute units on 8 dies (XCDs), each die with its own L2.
constexpr int kXcds = 8;
// Red-black smoother: one thread per cell of one colour, 128 x 4 (x 1) cell tiles.
constexpr int kSX = 128;
// Coarsest-level solve: one workgroup per grid, up to kCoarseCPT cells per thread.
constexpr int kCoarseThreads = 1024;
constexpr int kCoarseCPT = 4;
constexpr int kCoarseMaxLDS = kCoarseThreads * kCoarseCPT;   // 4096 cells
// LDS tail: one 512-thread workgroup per grid (measured ahead of 256 and 1024); its
// coarsest CG holds up to 4 cells a thread.
constexpr int kTailThreads = 512;
constexpr int kTailCPT = 4;
constexpr int kTailMaxCoarsest = kTailThreads * kTailCPT;    // 2048 cells
constexpr int kTailWaveCells = 256;                         // tail levels run by one wavefront
constexpr int kMarchNP = 128;                               // row-marching 2D window: positions (two a lane)
constexpr int kMarchFz = 32;                                // rows per row-marching window
constexpr int kMarchFzShort = 16;                           // rows where windows are few
// halo of a row-marching window (even, so that a lane's two columns pair up for the
// restriction): 2 nu + 2 on the down pass, 2 nu on the up pass; and its interior columns
__host__ __device__ constexpr int march_halo(int nu, bool down) { return 2 * nu + (down ? 2 : 0); }
__host__ __device__ constexpr int march_fx(int nu, bool down) { return kMarchNP - 2 * march_halo(nu, down); }
__host__ __device__ inline int32_t march_tiles(const int32_t n[3], int nu, bool down, int fz) {
    const int fx = march_fx(nu, down);
    return ((n[0] + fx - 1) / fx) * ((n[1] + fz - 1) / fz);
}

// Tile counts of one level for the two tilings (host and device agree on these).
__host__ __device__ inline int32_t cell_tiles(const int32_t n[3]) {
    return ((n[0] + kTX - 1) / kTX) * ((n[1] + kTY - 1) / kTY) * n[2];
}
// Level-0 cell tiles (coefficients, residuals, CG vectors, outputs): kTX x kCY0
// cells in 2D, kTX x kCY3 x kCZ3 in 3D; kCPT0 per thread, one reduction partial
// per tile.  A 2D level has n[2] = 1 (every axis of a 3D grid has >= 2 cells).
constexpr int kCY0 = 16;
constexpr int kCY3 = 4;
constexpr int kCZ3 = 4;
constexpr int kCPT0 = kTX * kCY0 / kBlock;
static_assert(kTX * kCY0 == kCPT0 * kBlock && kCY3 * kCZ3 == kCY0, "level-0 tiles of kCPT0 cells per thread");
__host__ __device__ inline int32_t l0_tiles(const int32_t n[3]) {
    if (n[2] == 1) return ((n[0] + kTX - 1) / kTX) * ((n[1] + kCY0 - 1) / kCY0);
    return ((n[0] + kTX - 1) / kTX) * ((n[1] + kCY3 - 1) / kCY3) * ((n[2] + kCZ3 - 1) / kCZ3);
}
__host__ __device__ inline int32_t smooth_tiles(const int32_t n[3]) {
    return ((n[0] + kSX - 1) / kSX) * ((n[1] + kTY - 1) / kTY) * n[2];
}
// Fused 2D level tiles: FX x FY interior cells staged in LDS with a halo of HALO
// cells.  Narrow tiles are 64 cells wide; wide tiles fill a whole 128-cell row
// (one colour cell per lane of a wave) with the halo included.  FY and the
// width class are the tunable tile shape.
__host__ __device__ constexpr int fused_fx(int halo, int wide) { return wide ? 128 - 2 * halo : 64; }
__host__ __device__ inline int32_t fused_tiles(const int32_t n[3], int fx, int fy) {
    return ((n[0] + fx - 1) / fx) * ((n[1] + fy - 1) / fy) * n[2];
}
// LDS bytes of one fused tile (x, b and the two face arrays).
__host__ __device__ constexpr size_t fused_lds(int word, int halo, int wide, int fy) {
    return (size_t)4 * word * (fused_fx(halo, wide) + 2 * halo) * (fy + 2 * halo);
}
constexpr size_t kFusedLdsMax = 160 * 1024;

// Fused 3D sweep blocks: a window of px x py xy positions, one per thread, holding
// 64 x FY interior columns and a halo of 2 positions (3 where the sweep also
// restricts), marched over fz planes (fz even, tunable).  The interior is 64 cells
// wide, so a 2^k-wide level splits into whole tiles; FY = 11 (8 restricting).
__host__ __device__ constexpr int sweep3_halo(bool restr) { return restr ? 3 : 2; }
__host__ __device__ constexpr int sweep3_fx(bool) { return 64; }
__host__ __device__ constexpr int sweep3_fy(bool restr) { return restr ? 8 : 11; }
__host__ __device__ constexpr int sweep3_px(bool restr) { return sweep3_fx(restr) + 2 * sweep3_halo(restr); }
__host__ __device__ constexpr int sweep3_py(bool restr) { return sweep3_fy(restr) + 2 * sweep3_halo(restr); }
__host__ __device__ constexpr int sweep3_threads(bool restr) { return sweep3_px(restr) * sweep3_py(restr); }
static_assert(sweep3_threads(false) <= 1024 && sweep3_threads(true) <= 1024, "one workgroup per window");
__host__ __device__ inline int32_t sweep3_tiles(const int32_t n[3], bool restr, int fz) {
    const int fx = sweep3_fx(restr), fy = sweep3_fy(restr);
    return ((n[0] + fx - 1) / fx) * ((n[1] + fy - 1) / fy) * ((n[2] + fz - 1) / fz);
}

// z-march CG direction update (3D level 0): a window of kPqPX x kPqPY positions, 64 x 13
// interior columns with one halo position around them, fz planes per block.
constexpr int kPqPX = 66;
constexpr int kPqPY = 15;
// row-march CG direction update (2D level 0): windows of kMarchNP - 4 interior columns
// and kPq2Rows rows
constexpr int kPq2Rows = 32;
// plane depth of the level-0 3D sweep that also forms r . z
constexpr int kRz3Fz = 32;
__host__ __device__ inline int32_t pq2_tiles(const int32_t n[3], int fz) {
    return ((n[0] + kMarchNP - 5) / (kMarchNP - 4)) * ((n[1] + fz - 1) / fz);
}
__host__ __device__ inline int32_t pq3_tiles(const int32_t n[3], int fz) {
    return ((n[0] + kPqPX - 3) / (kPqPX - 2)) * ((n[1] + kPqPY - 3) / (kPqPY - 2)) * ((n[2] + fz - 1) / fz);
}

struct LevelDesc {
    int32_t n[3];        // nx, ny, nz (nz = 1 in 2D)
    int32_t ndim;
    int32_t grid;        // owning grid (index of the plan's per-grid call tables)
    int32_t sidx;        // index of the grid's solver state in the state array (the grid, or
                         // a request server's slot)
    int32_t level;       // 0 = finest
    int32_t coarse;      // index of the next coarser level, -1 at the coarsest
    int32_t fine;        // index of the next finer level, -1 at level 0
    int32_t nlev;        // levels of the owning grid (a grid's levels are consecutive entries)
    double  hinv[3];     // 1/h per axis (level 0 values are the grid's)
    // level 0 only: prescribed gradient dE/dx_a at the faces x-, x+, y-, y+, z-, z+ (0 for
    // zero flux), and that gradient times the cell width (the ghosts' linear part)
    int32_t has_bc;      // any face with a nonzero prescribed gradient or a Dirichlet value
    double  bcg[6];
    double  bcgh[6];
    int32_t per_mask;    // every level: bit a set for periodic axes
    int32_t cont_mask;   // every level: bit f set for the continuous faces (linear extrapolation)
    int32_t dir_mask;    // level 0: bit f set for the Dirichlet faces
    double  bcv[6];      // level 0: the ghost value E_B of each Dirichlet face
    double* ad;          // every level of a plan with Dirichlet faces: the extra diagonal of
    float*  ad32;        //   the ghost couplings, dt D / h^2 per Dirichlet face (NULL without)
    double* x;           // FP64 solution (level 0) / correction (coarser)
    double* b;           // FP64 right-hand side
    double* w[3];        // FP64 lower-face weights dt*D_face/h^2
    float*  x32;
    float*  b32;
    float*  w32[3];
    double* xs;          // fused 2D levels: smoothed iterate left by the down pass, read by
    float*  xs32;        //   the up pass (which writes x), so no pass reads what it writes
    double* part;        // per-tile partial sums (level 0 only)
    double* scratch;     // coarse-solve vectors for levels too large for LDS
    // level 0 only: the outer FP64 iteration (x and b above are the arrays the
    // V-cycle works on: X/B0 for plain V-cycle iteration, Z/R for CG)
    double* X;           // iterate, E^{n+1}
    double* B0;          // right-hand side E^n
    double* R;           // FP64 residual B0 - A X
    double* P[2];        // CG search directions (ping-pong by iteration parity)
    double* Q;           // A p
};

// Per-grid solver state, updated on the device between V-cycles.
struct GridState {
    double  bnorm2;      // ||b||^2
    double  bsum;        // sum b
    double  rnorm2;      // last ||b - A x||^2 (recursive in CG, true after a check)
    double  rprev2;      // best ||r||^2 so far (stagnation test)
    double  tol2;        // rtol^2 ||b||^2
    double  rho[2];      // CG: r . z of the iterations of even / odd parity
    double  alpha;       // CG step length
    double  beta;        // CG direction update
    int32_t active;      // 1 while iterations are still needed
    int32_t cycles;      // V-cycles done (one per CG iteration)
    int32_t status;      // FLD_* status
    int32_t stall;       // consecutive iterations without 10 % progress
    int32_t bad;         // input-validation bits (atomicOr)
    int32_t ntiles0;     // cell-tiles of level 0 (number of partial sums)
    int32_t iter;        // CG iterations since the last (re)start
    int32_t done;        // tiles of the running reduction finished so far (last block resets)
};

// fin argument of k_cg_pq / k_cg_update: every block forms the CG scalar it needs
// (beta / alpha) from the previous kernel's tile partials itself, in place of a
// k_finalize launch between the two (grids of up to kFoldMaxTiles level-0 tiles);
// k_cg_pq then leaves its partials after the r.z ones.
constexpr int kFinFold = -2;
constexpr int kFoldMaxTiles = 2048;

// Finalization modes of k_finalize (one block per grid, fixed-order sums).
enum FinMode : int32_t {
    FIN_B = 0,           // ||b||^2, sum b from the coefficient pass; (re)start the step
    FIN_R_INIT = 1,      // initial true residual
    FIN_R_CYCLE = 2,     // true residual after a plain V-cycle
    FIN_R_VERIFY = 3,    // true residual after CG reported convergence
    FIN_RZ = 4,          // CG: rho = r . z, beta
    FIN_PQ = 5,          // CG: alpha = rho / p . q
    FIN_CG = 6,          // CG: recursive ||r||^2, stop test
    FIN_R_FMG = 7,       // true residual after the full-multigrid start: counts a cycle, (re)starts CG
};

// Which levels a launch covers.  Level j of the list is LevelDesc levels[j];
// its tiles occupy [prefix[j], prefix[j+1]) of the launch's tile range.
struct JobList {
    const int32_t* levels;
    const int32_t* prefix;
    int32_t njobs;
    int32_t total;       // prefix[njobs]
    int64_t cells;       // cells of the listed levels (host bookkeeping; kernels ignore it)
    int32_t lev0;        // levels[0] (-1 for an empty list): a one-job launch reads its level
    int32_t pad_;        // from the kernel arguments instead of memory
};

// The job-list lookups of a tile's kernel.  prefix[0] is 0 and prefix[njobs] is total,
// so a one-job list needs no load from the list at all: its level comes from lev0.
__host__ __device__ inline int job_level(const JobList& jl, int jb) { return jl.njobs == 1 ? jl.lev0 : jl.levels[jb]; }
__host__ __device__ inline int job_start(const JobList& jl, int jb) { return jb == 0 ? 0 : jl.prefix[jb]; }
__host__ __device__ inline int job_tiles(const JobList& jl, int jb) {
    return (jb + 1 == jl.njobs ? jl.total : jl.prefix[jb + 1]) - job_start(jl, jb);
}

// Algorithmic-byte accounting.  While a thread has an Acct installed (acct_set),
// every launch wrapper adds the bytes its kernel must move (each array it reads
// or writes counted once, per the kernel's own access pattern) and its launch to
// the Acct instead of launching, so a driver such as one outer iteration can be
// replayed on the host to count what it moves.
struct Acct {
    double bytes = 0.0;
    int64_t launches = 0;
};
void acct_set(Acct* a);      // nullptr: launch normally
Acct* acct_get();

// Per-call pointers of fld_step (one entry per grid).
struct StepIO {
    const double* E_in;
    const double* kr;
    double*       E_out;
    double        dt;
    const double* krd[3];   // per-direction kappa rho (diagonal-tensor D); NULL: kr for every direction
};

// Per-call pointers of fld_exchange (one entry per grid).
struct ExchangeIO {
    double*       E;
    double*       eps;
    const double* rho;
    const double* kappa;
    double        dt;
    int64_t       n;
};

// Per-call pointers of fld_radiation_moments (one entry per grid; NULL outputs are
// not written; v[0] == NULL: no velocity).
struct MomentsIO {
    const double* E;
    const double* kr;
    const double* v[3];
    double*       F[3];
    double*       fr[3];
    double*       edd;
    double*       P[6];
    double*       tiring;
    double*       E_out;
    double        dt;
};

// Per-grid pointers of one pointwise stage of fld_imex_step (NULL: not used):
// kr <- kappa rho; E_x = E + 2 (Em - Ep) - dt_tir tir; (E_out, eps_out) <- the
// exchange of (E_x, eps) over tau.  E_out NULL: kr only.
struct ImexIO {
    const double* E;
    const double* eps;
    const double* rho;
    const double* kappa;
    const double* Em;
    const double* Ep;
    const double* tir;
    double*       kr;
    double*       E_out;
    double*       eps_out;
    double        tau;
    double        dt_tir;
    int64_t       n;
};

struct Control {
    int32_t nactive;     // grids still iterating after the last count
    int32_t bad_exchange;
    int64_t bisected;    // exchange cells that used the bisection fallback
    int32_t bad_imex;    // an IMEX stage met an invalid cell
    int32_t pad_;
};

// ---- launch wrappers (kernels.hip) ------------------------------------------
// All launches are asynchronous on `s`.  `nblk` caps the persistent grid size.
// Reductions finish on the device: the block that completes a grid's last tile sums
// the grid's tile partials in a fixed order and applies the FinMode update.
// bc: the plan has faces other than zero flux (selects the instantiation that handles them).
void launch_coeff(int dim, bool mixed, int bc, const LevelDesc* L, GridState* S, JobList jl,
                  const StepIO* io, double c, int limiter, int fin, double rtol, int max_cycles, int nblk,
                  hipStream_t s);
void launch_finalize(const LevelDesc* L, GridState* S, JobList jl, int mode, double rtol,
                     int max_cycles, hipStream_t s);
// galerkin: coarse weights of R A P (piecewise-constant P, child-mean R); 0: rediscretised.
void launch_coarsen(int dim, bool mixed, const LevelDesc* L, JobList jl, int galerkin, int nblk, hipStream_t s);
void launch_smooth(int dim, bool fp32, const LevelDesc* L, const GridState* S, JobList jl,
                   int color, int nblk, hipStream_t s);
void launch_restrict(int dim, bool fp32, const LevelDesc* L, const GridState* S, JobList jl,
                     int nblk, hipStream_t s);
void launch_prolong(int dim, bool fp32, const LevelDesc* L, const GridState* S, JobList jl,
                    int nblk, hipStream_t s);
// Full-multigrid start.  restrict_rhs: the coarse right-hand side is the mean of the
// children's right-hand sides (restriction list of a depth) and the coarse iterate 0;
// fmg_interp: the fine iterate is the bilinear / trilinear interpolation of the coarse
// one, mirrored at domain faces and wrapped on periodic axes (prolongation list of a depth).
void launch_restrict_rhs(int dim, bool fp32, const LevelDesc* L, const GridState* S, JobList jl,
                         int nblk, hipStream_t s);
void launch_fmg_interp(int dim, bool fp32, const LevelDesc* L, const GridState* S, JobList jl,
                       int nblk, hipStream_t s);
void launch_coarse_solve(int dim, bool fp32, const LevelDesc* L, const GridState* S, JobList jl,
                         hipStream_t s);
// Tail: one workgroup per job runs the V-cycle of every level from the job's level down
// in `smem` bytes of LDS.  prepare_tail raises the kernel's dynamic-LDS limit (call once,
// outside stream capture).  plain64: level-0 tails iterate from the current x.
int prepare_tail(int dim, bool fp32, size_t smem);
// Fused 2D level kernels (nu in 1..3).  down: nu red-black sweeps from a zero (or, with
// load_x, the stored) iterate, then the residual restricted to the coarse right-hand
// side; up: add the prolonged coarse correction, then nu black-red sweeps.
// Tile shapes: wide in {0,1}, fy in {4,8,16,32}, as long as the tile fits the LDS.
bool fused2_supported(int nu);
bool fused2_shape_ok(bool fp32, int nu, int wide, int fy, bool down);
// threads: workgroup size of the fused 2D level kernels, kBlock or 1024 (more waves
// per tile: shorter per-wave chains on small levels)
void launch_down2(bool fp32, const LevelDesc* L, const GridState* S, JobList jl, int nu, int load_x,
                  int wide, int fy, int threads, int nblk, hipStream_t s);
void launch_up2(bool fp32, const LevelDesc* L, const GridState* S, JobList jl, int nu, int wide, int fy,
                int threads, int nblk, hipStream_t s);
// The row-marching form of the same passes (down: nu sweeps from zero or the stored
// iterate, restricting; up: prolongation and nu sweeps), for levels with many tiles.
// rz (FP64 up pass of level 0 under CG, where b is the residual): each window also
// leaves its partial of b . x (r . z) in the level's partials, for a k_finalize
void launch_march2(bool fp32, const LevelDesc* L, const GridState* S, JobList jl, int nu, int down, int load_x,
                   int fz, int nblk, hipStream_t s, int rz = 0);
// Fused 3D sweeps (one red-black sweep per launch, colour c0 first), reading x (or xs
// with from_xs) and writing the other; modes: 0 from the iterate, 1 from zero, 2 / 3 the
// same plus restriction of the final residual, 4 from the iterate plus the prolonged
// coarse correction.
bool fused3_supported(bool fp32);
// rz (the last up sweep of level 0 under FP64 CG, a plain SW_LOAD sweep, where b is the
// residual): each window also leaves its partial of b . x (r . z) in the level's partials
void launch_sweep3(bool fp32, const LevelDesc* L, const GridState* S, JobList jl, int mode, int c0,
                   int from_xs, int fz, int nblk, hipStream_t s, int rz = 0);
// bc: the plan has Dirichlet or periodic faces.
void launch_tail(int dim, bool fp32, int bc, const LevelDesc* L, const GridState* S, JobList jl, size_t smem,
                 int nu1, int nu2, int plain64, hipStream_t s);
// LDS bytes of a tail whose finest level has cells n0 and whose levels halve down to
// `levels` levels: x, b and DIM face arrays per level plus one coarsest vector.
constexpr size_t kTailLdsBudget = 150 * 1024;
// select: 0 = active grids, 1 = inactive grids whose status is FLD_OK (convergence check).
// zero_x: also clear the level-0 V-cycle iterate (FP64 or FP32 by `mixed`); mixed also
// writes the FP32 right-hand side.
// fin: FinMode applied by the block that finishes a grid's last tile (-1: none;
// a separate launch_finalize finishes the reduction).
void launch_residual(int dim, bool mixed, const LevelDesc* L, GridState* S, JobList jl,
                     int select, int zero_x, int fin, double rtol, int max_cycles, int nblk, hipStream_t s);
void launch_cg_rz(int dim, bool mixed, const LevelDesc* L, GridState* S, JobList jl, int fin, double rtol,
                  int max_cycles, int nblk, hipStream_t s);
void launch_cg_pq(int dim, bool mixed, const LevelDesc* L, GridState* S, JobList jl, int fin, double rtol,
                  int max_cycles, int nblk, hipStream_t s);
// zero_z: also clear the level-0 V-cycle iterate (needed where the V-cycle's first
// sweep of level 0 reads it: the per-colour kernels).
void launch_cg_update(int dim, bool mixed, const LevelDesc* L, GridState* S, JobList jl, int fin, double rtol,
                  int max_cycles, int zero_z, int nblk, hipStream_t s);
// The same on the z-march tiles of a pq3 list (3D grids without Dirichlet or periodic faces):
// each tile stores its partial of p . q; a launch_finalize over the same list finishes.
void launch_cg_pq3(bool mixed, const LevelDesc* L, GridState* S, JobList jl, int fz, int nblk, hipStream_t s);
void launch_cg_pq2m(bool mixed, const LevelDesc* L, GridState* S, JobList jl, int fz, hipStream_t s);
// X += the level-0 V-cycle iterate (FP32 when mixed, else FP64).
void launch_correct(int dim, bool mixed, const LevelDesc* L, const GridState* S, JobList jl, int nblk,
                    hipStream_t s);
void launch_output(int dim, const LevelDesc* L, JobList jl, const StepIO* io, int nblk,
                   hipStream_t s);
void launch_count(const GridState* S, int ngrids, Control* ctrl, hipStream_t s);
// Radiation moments of every level-0 cell of the listed grids (io indexed by grid).
void launch_moments(int dim, const LevelDesc* L, JobList jl, const MomentsIO* io, double c, int limiter,
                    int nblk, hipStream_t s);
void launch_set_active(GridState* S, int ngrids, int value, hipStream_t s);
void launch_exchange(const ExchangeIO* io, int ngrids, int64_t max_n, double c, double a_rad,
                     double c_v, int max_halley, double root_rtol, Control* ctrl, int nblk,
                     hipStream_t s);
void launch_imex_point(const ImexIO* io, int ngrids, int64_t max_n, double c, double a_rad, double c_v,
                       int max_halley, double root_rtol, Control* ctrl, int nblk, hipStream_t s);

}  // namespace fld
