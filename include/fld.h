/*
 * fld.h -- C ABI of the MI355X flux-limited-diffusion (FLD) radiation-energy step.
 *
 * The method is the one of Moens et al., "Radiation-hydrodynamics with
 * MPI-AMRVAC: flux-limited diffusion" (A&A 2022):
 *
 *   diffusion (Sec. 3.4):  E^{n+1}/dt - div(D^n grad E^{n+1}) = E^n/dt,
 *     D = c lambda(R) / (kappa rho)                (Sec. 2.2, eq. fld_F)
 *     R = |grad E| / (kappa rho E)                 (Sec. 2.2)
 *     lambda = (2+R)/(6+3R+R^2)                    (Sec. 2.2, eq. fld_lambda)
 *     grad E by the 4th-order central stencil      (Sec. 3.2, eq. ileyk_flux)
 *     face D by the harmonic mean of cell values   (Sec. 3.4)
 *     5-point (2D) / 7-point (3D) finite volumes   (Sec. 3.4, eq. discdiff)
 *   exchange (Sec. 3.3): the point-implicit gas/radiation energy exchange, a
 *     quartic for the new gas energy solved by Halley's method with a
 *     bisection fallback, then E^{n+1} = (a1 eps'^4 + E^n)/(1 + a2).
 *
 * Conventions shared by every call:
 *   - Grids are uniform Cartesian, 2D or 3D, every axis >= 2 cells.  A field
 *     is one contiguous FP64 array, x fastest: idx = i + nx*(j + ny*k).
 *   - Boundaries are zero flux (Neumann with zero gradient, Sec. 3.4): ghost
 *     values mirror the interior (E_{-1} = E_0, E_{-2} = E_1).
 *   - "device" pointers are HIP device memory on the device that was current
 *     when the plan was created; "host" pointers are ordinary host memory.
 *     The caller owns every buffer it passes; the library never frees or
 *     retains caller memory beyond the call, except the workspace bound to a
 *     plan (kept until fld_plan_destroy or the next bind) and the server arena.
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).  Work is
 *     enqueued on it; calls documented as synchronous also wait for it.
 *   - Every call returns FLD_OK (0), a positive status (FLD_PENDING) or a
 *     negative error code; fld_strerror() names it.  No C++ exception crosses
 *     the boundary.  A plan must not be used from two threads at once; a
 *     server may be.
 */
#ifndef FLD_H
#define FLD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define FLD_OK                   0
#define FLD_PENDING              1   /* fld_poll: the request is not finished  */
#define FLD_ERR_INVALID_ARG     -1   /* bad argument (null, size, option)      */
#define FLD_ERR_BAD_INPUT       -2   /* device-detected E <= 0, kappa*rho <= 0,
                                        rho <= 0, kappa < 0 or a non-finite value */
#define FLD_ERR_NOT_CONVERGED   -3   /* rtol not met within max_cycles (or the
                                        residual stagnated); the output holds the
                                        best iterate and the stats are filled   */
#define FLD_ERR_TOO_LARGE       -4   /* request larger than the server arena   */
#define FLD_ERR_UNKNOWN_TICKET  -5
#define FLD_ERR_HIP             -6   /* a HIP runtime call failed              */
#define FLD_ERR_NO_WORKSPACE    -7   /* plan has no (or too small) workspace   */
#define FLD_ERR_UNSUPPORTED     -8   /* option not built (a boundary code other than the
                                        five FLD_BC_* kinds)                       */
#define FLD_ERR_SHUTDOWN        -9   /* server is shutting down               */

/* ---- options ------------------------------------------------------------ */
#define FLD_LIMITER_LP          0    /* lambda = (2+R)/(6+3R+R^2)   (Sec. 2.2, eq. fld_lambda) */
#define FLD_LIMITER_DIFFUSION   1    /* lambda = 1/3, the optically thick limit (Sec. 2.2)   */
#define FLD_LIMITER_MINERBO     2    /* Minerbo (1978), the alternative Sec. 2.2 names:
                                        2/(3 + sqrt(9 + 12 R^2)) for R <= 3/2,
                                        1/(1 + R + sqrt(1 + 2R)) above                       */
#define FLD_LIMITER_LP_EXACT    3    /* Levermore-Pomraning's own (coth R - 1/R)/R, which
                                        eq. fld_lambda approximates to ~7 %                  */

#define FLD_BC_ZERO_FLUX        0    /* Neumann, zero gradient (Sec. 3.4)      */
#define FLD_BC_DIRICHLET        2    /* the ghost cells hold E_B = bc_value (Sec. 3.4):
                                        both ghost layers for the 4th-order gradient;
                                        the ghost couples to the boundary cell over one
                                        cell width with the cell's own D, adding
                                        dt D / h^2 to the diagonal and that times E_B
                                        to the right-hand side.  Plans with Dirichlet
                                        faces run one kernel per colour sweep (no
                                        fused level kernels)                        */
#define FLD_BC_PERIODIC         3    /* both faces of an axis: the ghosts are the cells at
                                        the other end and the face between the last
                                        and the first cell is an interior face (harmonic
                                        mean of their D).  One face of an axis periodic
                                        and the other not is INVALID_ARG.  Such plans
                                        also sweep per colour                       */
#define FLD_BC_FIXED_GRADIENT   1    /* Neumann with the gradient dE/dx_a given in
                                        bc_grad (Sec. 3.4): ghosts continue the mirror
                                        image with that slope, E_{-k} = E_{k-1} -
                                        (2k-1) h G below and E_{n-1+k} = E_{n-k} +
                                        (2k-1) h G above, for the 4th-order gradient;
                                        the face flux -D G, D the boundary cell's,
                                        enters the right-hand side                 */
#define FLD_BC_CONTINUOUS       4    /* E^{n+1} extrapolated linearly into the ghosts
                                        (Sec. 3.4, continuous conditions): E_{-k} =
                                        E_0 + k (E_0 - E_1), likewise above, for the
                                        4th-order gradient and for the implicit solve,
                                        where the boundary face carries the flux
                                        coefficient of the first interior face, so the
                                        boundary cell's row loses its coupling along
                                        that axis.  The operator is then not
                                        symmetric: such plans need krylov = 0 (plain
                                        V-cycles; INVALID_ARG otherwise) and sweep per
                                        colour                                      */

#define FLD_COARSE_REDISCRETISED 0   /* coarse faces: mean of the sub-face weights
                                        times 1/4 (the operator rebuilt at 2h)  */
#define FLD_COARSE_GALERKIN     1    /* coarse operator R A P of the piecewise-
                                        constant prolongation P and the child-mean
                                        restriction R = P^T / 2^d: sum of the sub-face
                                        weights over 2^d                          */

#define FLD_PREC_FP64           0    /* every step in FP64                     */
#define FLD_PREC_MIXED          1    /* FP32 V-cycles inside FP64 defect correction:
                                        residual, update and stop test in FP64 */

/* One grid: ndim in {2,3}; n[d] cells and h[d] cell width along x, y, z
   (n[2], h[2] ignored in 2D). */
typedef struct fld_grid {
    int32_t ndim;
    int32_t n[3];
    double  h[3];
} fld_grid;

/* Solver options (fld_opts_default fills the defaults given in brackets). */
typedef struct fld_opts {
    double  c;            /* speed of light in the caller's units [1]               */
    int32_t limiter;      /* FLD_LIMITER_* [LP]                                      */
    int32_t bc[6];        /* per face x-,x+,y-,y+,z-,z+: FLD_BC_* [ZERO_FLUX] (z faces
                             ignored in 2D)                                          */
    int32_t precision;    /* FLD_PREC_* [FP64]                                       */
    double  rtol;         /* stop when ||E^n - A E||_2 <= rtol ||E^n||_2 [1e-10]     */
    int32_t max_cycles;   /* V-cycles (= outer iterations) per step [50]            */
    int32_t nu1, nu2;     /* red-black Gauss-Seidel sweeps before / after the coarse
                             correction [2, 2]; 2D grids keep the fused level
                             kernels for counts 1..3 and sweep per colour otherwise */
    int32_t use_graph;    /* replay V-cycles from a captured hipGraph [1]           */
    int32_t autotune;     /* launch shape: 0 = from the tile fields below; 1 = from
                             the autotuner's cache, timed at bind time on a miss;
                             2 = always timed at bind time [0].  Timing zeroes the
                             workspace fields and runs V-cycles on them (about 30
                             V-cycles).  The cache is the file $FLD_AUTOTUNE_CACHE,
                             else $HOME/.cache/fld_autotune.txt                      */
    int32_t krylov;       /* 1: conjugate gradients preconditioned by one V-cycle per
                             iteration, stopped on the recursive residual and
                             confirmed on the true FP64 residual; 0: plain V-cycle
                             iteration (defect correction in mixed precision) [1]   */
    int32_t fused;        /* 2D: run each multigrid level as two fused kernels
                             (sweeps + restriction, prolongation + sweeps) when nu1,
                             nu2 are in 1..3: 1 = LDS tiles, or windows that march
                             along the rows on depths with at least four windows per
                             compute unit; 2 = tiles only; 3 = march wherever fused;
                             0: one kernel per colour sweep and per transfer.  Every
                             choice gives the same results bit for bit [1]         */
    int32_t tile_rows;    /* fused 2D tile rows: 4, 8, 16 or 32; 0 = 8 [0]          */
    int32_t tile_wide;    /* fused 2D tile width: 0 = 64 cells, 1 = 128 cells less
                             the halo (a colour cell per lane of a 64-lane wave) [0].
                             INVALID_ARG if the tile does not fit the 160 KB LDS   */
    int32_t max_blocks;   /* cap on workgroups per persistent launch; 0 = 2048 [0]   */
    int32_t tile_depth;   /* fused 3D sweeps: planes per block, 16, 32 or 64; 0 = 32 [0] */
    int32_t fused3_levels;/* 3D: the first k multigrid levels run fused sweeps, the
                             coarser ones per-colour kernels; 0 = the levels whose
                             sweep has at least 256 blocks [0].  3D grids use fused
                             sweeps when fused = 1, nu1, nu2 >= 1 and nu1 + nu2 is
                             even.  tile_rows, tile_wide, max_blocks, tile_depth and
                             fused3_levels must be 0 with autotune                  */
    double  bc_grad[6];   /* per face: the prescribed gradient of FLD_BC_FIXED_GRADIENT
                             faces (ignored on zero-flux faces) [0]                  */
    int32_t tile_rows_coarse; /* fused 2D tile rows of the levels below the finest: 4, 8,
                             16 or 32; 0 = as tile_rows [0].  Must be 0 with autotune */
    int32_t fmg;          /* 1: the first outer iteration of each step is a full-
                             multigrid cycle (Sec. 3.4: an FMG cycle first, then
                             V-cycles until the requested residual): the right-hand
                             side is averaged down the hierarchy, the coarsest
                             levels are solved, and on each finer level the
                             bilinear (trilinear) interpolation of the coarser
                             solution starts one V-cycle.  With krylov = 1 or mixed
                             precision it solves for the correction of the initial
                             residual and CG restarts from the corrected iterate;
                             with plain FP64 V-cycles it replaces E^n as the start.
                             It counts as one cycle in fld_stats.  Request servers
                             iterate V-cycles only [1]                            */
    int32_t coarse_op;    /* FLD_COARSE_* [REDISCRETISED]                          */
    int32_t fmg_depths;   /* with fmg: only the finest fmg_depths levels run the V-cycle
                             of their full-multigrid stage; coarser ones pass the
                             interpolated solution on as it is (0 = every level;
                             -1 = by dimension: the finest 2 in 2D, 3 in 3D) [-1]   */
    double  bc_value[6];  /* per face: the ghost value E_B of FLD_BC_DIRICHLET faces,
                             finite and >= 0 (ignored elsewhere) [0]                 */
    int32_t tile_rows_up; /* fused 2D tile rows of the finest level's up pass: 4, 8, 16
                             or 32; 0 = as tile_rows (which then sets the finest
                             level's down pass alone) [0].  Must be 0 with autotune  */
    int32_t nu_coarse;    /* red-black sweeps before and after the coarse correction on
                             the levels below the finest, and on every level of a
                             grid small enough to be cycled whole in one LDS block;
                             0..16, 0 = nu1 before and nu2 after [3].  As for nu1
                             and nu2, a count outside 1..3 sends the plan's 2D grids
                             to the per-colour sweeps on every level, the finest
                             included                                              */
} fld_opts;

/* Per-grid result of fld_step. */
typedef struct fld_stats {
    int32_t cycles;        /* V-cycles (outer iterations) performed                 */
    int32_t status;        /* FLD_OK, FLD_ERR_NOT_CONVERGED or FLD_ERR_BAD_INPUT    */
    double  rel_residual;  /* final ||b - A x||_2 / ||b||_2, FP64                   */
    double  q_b;           /* ||b||_2 / (sqrt(N) |mean b|): relative error of the
                              result <= q_b * rel_residual (A is SPD, lambda_min>=1,
                              and zero flux conserves the mean)                     */
    double  b_norm;        /* ||E^n||_2                                             */
    double  b_sum;         /* sum of E^n (conserved by the exact solution)          */
} fld_stats;

/* Gas/radiation exchange constants (Sec. 3.3).  c_v = k_b / ((gamma-1) mu m_p)
   so that T_g = eps / (rho c_v); a_rad = 4 sigma / c. */
typedef struct fld_gas {
    double  c;
    double  a_rad;
    double  c_v;
    int32_t max_halley;   /* Halley iterations before bisection [100] (0 forces bisection) */
    double  root_rtol;    /* Halley stop: |step| <= root_rtol * root [4 * 2^-52]   */
} fld_gas;

typedef struct fld_plan_s* fld_plan_t;

/* Device pointers into a bound workspace for one level of one grid's
   multigrid hierarchy (level 0 = the grid itself).  w[d] holds the lower-face
   weights dt * D_face / h_d^2 along d (entry 0 along d is the domain face: 0).
   Pointers that the plan's precision does not use are NULL. */
typedef struct fld_level_view {
    int32_t ndim;
    int32_t n[3];
    double* x;            /* FP64: level 0 the iterate E^{n+1}, coarser the correction */
    double* b;            /* FP64: level 0 E^n, coarser the restricted residual      */
    double* w[3];         /* FP64 face weights                                      */
    float*  x32;
    float*  b32;
    float*  w32[3];
    double* ad;           /* plans with Dirichlet faces: the extra diagonal dt D / h^2
                             of the ghost couplings (FP64), else NULL               */
} fld_level_view;

/* Library version, major*10000 + minor*100 + patch. */
int32_t fld_version(void);
/* Static string naming a status code; never NULL. */
const char* fld_strerror(int32_t code);
/* Text of the last HIP failure seen on the calling thread (empty if none);
   valid until the next failing call on that thread. */
const char* fld_last_error(void);
/* Fill *o with the defaults listed in fld_opts. */
void fld_opts_default(fld_opts* o);
void fld_gas_default(fld_gas* g);

/* Build a plan for ngrids independent grids solved together: the multigrid
   hierarchy of each grid (halve every axis while all are even and >= 4), the
   workspace layout and the launch work-lists.  Host only: no device memory
   is allocated.  Errors: INVALID_ARG (null, ngrids < 1, ndim not 2/3, an axis
   < 2, h <= 0, bad option, a periodic axis with one periodic face, continuous
   faces with krylov = 1), UNSUPPORTED (a boundary code that is not an FLD_BC_*
   kind). */
int32_t fld_plan_create(const fld_grid* grids, int32_t ngrids, const fld_opts* opts,
                        fld_plan_t* out);
int32_t fld_plan_destroy(fld_plan_t plan);

/* Bytes of device workspace the plan needs (256-byte aligned). */
int32_t fld_plan_workspace_bytes(fld_plan_t plan, size_t* bytes);
/* Bind caller-owned device memory of >= the size above (256-byte aligned).  The
   library keeps the pointer (never frees it) and writes its level tables there.
   Synchronous.  Errors: INVALID_ARG, NO_WORKSPACE (too small), HIP. */
int32_t fld_plan_bind_workspace(fld_plan_t plan, void* dev, size_t bytes);

/* Number of multigrid levels of grid g, and a view of one level (see above). */
int32_t fld_plan_levels(fld_plan_t plan, int32_t g, int32_t* nlevels);
int32_t fld_plan_level_view(fld_plan_t plan, int32_t g, int32_t level, fld_level_view* out);

/* Coefficients only (the first stage of fld_step), for every grid g:
   D from E_in[g] and kappa_rho[g] (device, N_g doubles each) with dt[g] (host
   array of ngrids), written as face weights into the workspace of every level
   (level 0 per Sec. 3.4; coarser levels average the sub-faces and scale by
   1/4 per halving).  Asynchronous on stream.  Errors: INVALID_ARG, NO_WORKSPACE, HIP. */
int32_t fld_coefficients(fld_plan_t plan, const double* const* E_in,
                         const double* const* kappa_rho, const double* dt, void* stream);

/* One implicit FLD diffusion step for every grid g of the plan:
     E_out[g] = (I + dt[g] L(D(E_in[g])))^{-1} E_in[g]
   with D lagged at E_in (Sec. 3.4).  E_in, kappa_rho, E_out: host arrays of
   ngrids device pointers to N_g doubles (caller-owned; E_out[g] may equal
   E_in[g]).  dt: host array of ngrids.  Solved by multigrid V-cycles to
   opts.rtol relative residual (FP64 residual in both precisions).
   Synchronous: returns after the stream has finished the step.  stats: host
   array of ngrids (may be NULL).  Returns FLD_OK, or the first non-OK grid
   status (NOT_CONVERGED, BAD_INPUT) -- every grid's output is still written --
   or INVALID_ARG / NO_WORKSPACE / HIP. */
int32_t fld_step(fld_plan_t plan, const double* const* E_in, const double* const* kappa_rho,
                 double* const* E_out, const double* dt, void* stream, fld_stats* stats);

/* fld_step with a diagonal-tensor diffusion coefficient (the anisotropic D the
   paper reports testing, Sec. 5, with the notation of Sec. 3 carried over per
   grid direction): the caller gives one kappa rho per direction, and the faces
   normal to direction a use
     R_a = |grad E| / ((kappa rho)_a E),  D_a = c lambda(R_a) / (kappa rho)_a,
   harmonic-mean face values of D_a and the weights dt D_a / h_a^2; the solve is
   that of fld_step.  kappa_rho_dir: host array of 3 * ngrids device pointers,
   kappa_rho_dir[3 g + a] for a < ndim of grid g (N_g doubles each; entries past
   ndim are ignored).  Equal arrays give fld_step's result.  Same ownership,
   synchronisation and status codes as fld_step (BAD_INPUT covers every
   direction's opacity). */
int32_t fld_step_aniso(fld_plan_t plan, const double* const* E_in, const double* const* kappa_rho_dir,
                       double* const* E_out, const double* dt, void* stream, fld_stats* stats);

/* Point-implicit gas-radiation energy exchange (Sec. 3.3), in place, per cell
   of every grid g: with a1 = c a_rad kappa dt / (rho^3 c_v^4) and
   a2 = c kappa rho dt, eps' is the unique root in ]0, eps + E[ of
   a1 x^4 + (1+a2) x - ((1+a2) eps + a2 E) = 0 and E' = (a1 eps'^4 + E)/(1+a2).
   E, eps (read/write), rho, kappa (read): host arrays of ngrids device
   pointers to N_g doubles.  dt: host array of ngrids.  Asynchronous on stream.
   Cells with rho <= 0, kappa < 0, E < 0, eps < 0 or non-finite values are left
   unchanged and reported by the next fld_exchange_status().
   Errors: INVALID_ARG, NO_WORKSPACE, HIP. */
int32_t fld_exchange(fld_plan_t plan, double* const* E, double* const* eps,
                     const double* const* rho, const double* const* kappa,
                     const double* dt, const fld_gas* gas, void* stream);
/* Synchronous: waits for stream, returns FLD_OK or FLD_ERR_BAD_INPUT if any
   cell of any earlier fld_exchange on this plan was rejected (and clears the flag);
   *bisected (may be NULL) receives the number of cells that needed the
   bisection fallback since the last call. */
int32_t fld_exchange_status(fld_plan_t plan, void* stream, int64_t* bisected);

/* Radiation moments of E, per cell of every grid g (Sec. 2.2, 2.1 and 3.2), with
   the 4th-order gradient and the plan's limiter and c (as in the coefficient pass):
     F   = -c lambda / (kappa rho) grad E                      (eq. fld_F)
     f_r = rho kappa F / c                                      (eq. rhd_force)
     f   = lambda + lambda^2 R^2                                (eq. fld_Edd_fac)
     P   = E (1/2 (1 - f) I + 1/2 (3 f - 1) n n), n = grad E / |grad E|
           (n = 0 where grad E = 0)                             (eq. fld_Edd)
   and, given the gas velocity v, the photon-tiring work
     P : grad v = sum_ij P_ij dv_i/dx_j  (4th-order gradients of v, mirrored ghosts)
   and the explicit update E_out = E - dt P : grad v (the term's sign in the
   radiation energy equation, Eq. 0th_cmf).  Each output array holds N_g doubles;
   NULL outputs are skipped.  P is stored as its upper triangle, row-major:
   xx, xy, yy (2D); xx, xy, xz, yy, yz, zz (3D). */
typedef struct fld_moments_out {
    double* F[3];         /* flux components x, y[, z]                              */
    double* f_r[3];       /* radiation force density components                     */
    double* edd;          /* scalar Eddington factor f                              */
    double* P[6];         /* pressure tensor components (see above)                 */
    double* tiring;       /* P : grad v (needs v)                                   */
    double* E_out;        /* E - dt P : grad v (needs v; must differ from E)        */
} fld_moments_out;
/* E, kappa_rho: host arrays of ngrids device pointers (N_g doubles each).  v: NULL,
   or a host array of 3 * ngrids device pointers, v[3 g + d] the d-th component of
   grid g's velocity (NULL entries: no velocity for that grid; all ndim or none).
   dt: host array of ngrids (read only where E_out is set; may be NULL otherwise).
   out: host array of ngrids.  Needs a bound workspace (nothing of a step is read).
   Asynchronous on stream.  Errors: INVALID_ARG (null inputs, partial velocity,
   tiring or E_out without velocity, E_out == E, non-finite dt), NO_WORKSPACE, HIP. */
int32_t fld_radiation_moments(fld_plan_t plan, const double* const* E, const double* const* kappa_rho,
                              const double* const* v, const double* dt, const fld_moments_out* out,
                              void* stream);

/* ---- IMEX time step of the radiation subsystem --------------------------- */
/* The paper's split of the radiation energy equation (Sec. 3.1, eqs. G_expl_1 -
   G_implexpl) into an explicit operator G_ex -- the photon-tiring source
   E <- E - tau P : grad v when a velocity is given (Sec. 3.2), then the
   point-implicit exchange over tau (Sec. 3.3) -- and the implicit diffusion G_im
   over tau (Sec. 3.4, D lagged at the stage input), with kappa rho = kappa * rho
   serving both.  kappa, rho, v stay fixed over the step.
     FLD_IMEX_EULER:    u* = G_ex(u^n, dt);  E^{n+1} = G_im(E*, dt);  eps^{n+1} = eps*.
     FLD_IMEX_MIDPOINT: u_+ = G_ex(u^n, dt/2);  E^{n+1/2} = G_im(E_+, dt/2);
                        E_x = E^n + 2 (E^{n+1/2} - E_+) - dt P(E^{n+1/2}) : grad v
                        (dt times the half step's implicit tendency, and the tiring
                        source at the midpoint state); (E, eps)^{n+1} = the exchange
                        of (E_x, eps^n) over dt.
   The midpoint scheme is second order where the exchange is inactive; the
   exchange stage is a backward-Euler step in both schemes. */
#define FLD_IMEX_EULER      0
#define FLD_IMEX_MIDPOINT   1

/* Bytes of device scratch fld_imex_step needs for `scheme` (256-byte multiple per
   grid: 2 (Euler) or 4 (midpoint) arrays of N_g doubles).  Errors: INVALID_ARG. */
int32_t fld_imex_scratch_bytes(fld_plan_t plan, int32_t scheme, size_t* bytes);

/* One IMEX step for every grid g of the plan, in place on E[g] and eps[g]
   (host arrays of ngrids device pointers to N_g doubles; E[g] != eps[g]).
   rho, kappa: host arrays of ngrids device pointers (N_g doubles, read only).
   v: NULL, or a host array of 3 * ngrids device pointers as for
   fld_radiation_moments (all ndim components of a grid or none).  dt: host
   array of ngrids, > 0.  gas: exchange constants; gas->c must equal the plan's c.
   scratch: caller-owned device memory of >= fld_imex_scratch_bytes(scheme)
   bytes, 256-byte aligned, not overlapping any input; its contents on return
   are unspecified.  Synchronous (the implicit stage reads back convergence).
   stats: host array of ngrids (may be NULL) receiving the implicit solve's
   statistics.  Returns FLD_OK, the first non-OK solve status (NOT_CONVERGED,
   BAD_INPUT; every output is still written), BAD_INPUT if an exchange stage met
   an invalid cell (that cell keeps its pre-exchange values), or INVALID_ARG /
   NO_WORKSPACE / HIP.  Exchange cells that fell back to bisection add to the
   count fld_exchange_status reports. */
int32_t fld_imex_step(fld_plan_t plan, double* const* E, double* const* eps,
                      const double* const* rho, const double* const* kappa, const double* const* v,
                      const double* dt, const fld_gas* gas, int32_t scheme, void* scratch,
                      size_t scratch_bytes, void* stream, fld_stats* stats);

/* ---- measurement -------------------------------------------------------- */
#define FLD_KERNEL_SMOOTH    0   /* one red-black half sweep over every grid's level `level` */
#define FLD_KERNEL_RESIDUAL  1   /* level-0 FP64 residual and its per-tile norms           */
#define FLD_KERNEL_RESTRICT  2   /* residual + restriction from level `level` to level+1   */
#define FLD_KERNEL_PROLONG   3   /* prolongation + correction from level+1 to `level`      */
#define FLD_KERNEL_COEFF     4   /* coefficients, on the inputs of the last fld_step        */
#define FLD_KERNEL_VCYCLE    5   /* one whole V-cycle with its residual test               */
#define FLD_KERNEL_EXCHANGE  6   /* exchange, on the arrays of the last fld_exchange (alters them) */
#define FLD_KERNEL_DOWN      7   /* fused 2D: nu1 sweeps + residual + restriction at `level` */
#define FLD_KERNEL_UP        8   /* fused 2D: prolongation + nu2 sweeps at `level`           */
#define FLD_KERNEL_TAIL      9   /* the LDS tail of every grid                             */
#define FLD_KERNEL_SWEEP3   10   /* fused 3D: one red-black sweep from the stored iterate at `level` */
#define FLD_KERNEL_MG       11   /* the multigrid part of one V-cycle (every level, no CG update) */

/* Launch shape of a bound plan, and where it came from. */
typedef struct fld_tuning {
    int32_t tile_rows;    /* fused 2D tile rows                                     */
    int32_t tile_wide;    /* fused 2D tile width class (see fld_opts)               */
    int32_t max_blocks;   /* workgroup cap of persistent launches                   */
    int32_t source;       /* 0 = options / defaults, 1 = timed at bind, 2 = cache   */
    int32_t candidates;   /* shapes timed (source 1)                                */
    double  vcycle_us;    /* timed multigrid V-cycle of the choice, microseconds
                             (source 1; 0 otherwise)                                */
    int32_t tile_depth;   /* fused 3D sweep planes per block                        */
    int32_t fused3;       /* 1 if 3D grids run fused sweeps (the tuner may prefer the
                             per-colour kernels)                                    */
    int32_t fused3_levels;/* leading 3D levels with fused sweeps                    */
    int32_t tile_rows_coarse; /* fused 2D tile rows below the finest level              */
    int32_t tile_rows_up; /* fused 2D tile rows of the finest level's up pass (tile_rows:
                             its down pass)                                          */
    int32_t march_levels; /* 2D depths whose passes march rows (fused = 1 or 3)      */
    int32_t march_rows;   /* rows per window of the finest marching depth (32, or 16
                             where 32-row windows would be too few); 0: none         */
    int32_t pq_rows;      /* rows (2D) or planes (3D) per window of the marching CG
                             direction update of level 0; 0 when the cell-tile kernel
                             runs it (few tiles, or Dirichlet / periodic faces, or a 2D
                             grid with an odd row length)                          */
} fld_tuning;
/* Errors: INVALID_ARG (null), NO_WORKSPACE (not bound yet). */
int32_t fld_plan_tuning(fld_plan_t plan, fld_tuning* out);

/* fld_step for callers that cannot allocate (code under HIP graph capture, tight
   serving loops, harnesses that forbid allocation): the same step with the same
   kernels and results, but the plan's tables and fields live in a fixed device
   array of the library, FLD_NOALLOC_MAX_BYTES per GPU, held from the first call
   on a GPU until the process ends, instead of a caller workspace.  The plan must
   not be bound to a workspace (INVALID_ARG otherwise) and its workspace size
   (fld_plan_workspace_bytes) must not exceed FLD_NOALLOC_MAX_BYTES (TOO_LARGE).
   It calls no allocating routine: no autotuning and no graph capture (use_graph
   and autotune are ignored), host staging in the plan's own host arrays.  All
   calls on one GPU share the array, so calls that overlap on one GPU race;
   each call rebinds its plan, and the plan is left unbound.  Synchronous, with
   stats as fld_step.  Errors: as fld_step, plus INVALID_ARG and TOO_LARGE above. */
#define FLD_NOALLOC_MAX_BYTES (64u << 20)
int32_t fld_step_noalloc(fld_plan_t plan, const double* const* E_in, const double* const* kappa_rho,
                         double* const* E_out, const double* dt, void* stream, fld_stats* stats);

/* Algorithmic bytes of one pass of a driver: each kernel it launches counted by
   the arrays it must read and write once per cell it covers (faces, iterates,
   right-hand sides, CG vectors; coarse levels at their own size), summed over
   the pass, without launching anything.  Dividing by the pass's measured time
   gives its effective bandwidth.  what: FLD_CYCLE_ITERATION one outer iteration
   as fld_step replays it (V-cycle, CG update or defect correction, FP64 stop
   test), FLD_CYCLE_MG its multigrid part (as FLD_KERNEL_MG times it),
   FLD_CYCLE_FMG the first outer iteration of a step with the full-multigrid
   start.  *launches (may be NULL) receives the kernel launches of the pass.
   Host only.  Errors: INVALID_ARG, NO_WORKSPACE. */
#define FLD_CYCLE_ITERATION 0
#define FLD_CYCLE_MG        1
#define FLD_CYCLE_FMG       2
int32_t fld_plan_cycle_bytes(fld_plan_t plan, int32_t what, double* bytes, int64_t* launches);

/* Time `reps` back-to-back launches of one kernel of the plan (launch shape
   as fld_step uses it) between two HIP events on `stream`; *avg_ms receives
   the mean time per launch (it includes the dispatch gap between launches)
   and *cells the cells one launch processes (the level's cells summed over
   the grids).  Every grid is made active for the measurement and inactive
   afterwards, so call it between steps only.  The level arrays are modified
   (smoothing further an already converged iterate); fld_step outputs are not.
   Synchronous.  Errors: INVALID_ARG (kernel, level or reps), NO_WORKSPACE, HIP. */
int32_t fld_profile_kernel(fld_plan_t plan, int32_t kernel, int32_t level, int32_t reps,
                           void* stream, double* avg_ms, int64_t* cells);

/* ---- request server: continuous batching of independent solves ---------- *
 * A server owns a worker thread and one HIP stream on the device current at
 * creation.  Requests (one diffusion step of one 2D or 3D grid each, the
 * operation of fld_step) are admitted in arrival order when a slot is free and
 * the caller's arena has room for the request's multigrid workspace, a copy of
 * its inputs and its result; until then they wait (no request is refused for a
 * full arena unless it could never fit).  Admitted requests iterate together:
 * every multigrid phase is one launch over all resident requests, and requests
 * join and leave at iteration boundaries.  A request's result is the same
 * whether it runs alone or among others (same kernels, tiles and reduction
 * orders per grid).  All server calls are thread-safe. */
typedef struct fld_server_s* fld_server_t;

typedef struct fld_server_opts {
    int32_t max_slots;        /* requests resident on the device at once [64]          */
    int32_t precision;        /* FLD_PREC_* for every request [MIXED]                  */
    double  rtol;             /* relative FP64 residual target [1e-10]                 */
    int32_t max_cycles;       /* V-cycles per request [50]                             */
    double  c;                /* speed of light [1]                                    */
    int32_t limiter;          /* FLD_LIMITER_* [LP]                                    */
    int32_t cycles_per_round; /* iterations between admission / retirement points [2]  */
} fld_server_opts;

typedef struct fld_request {
    fld_grid      grid;
    double        dt;
    const double* E_in;       /* N doubles: E^n                                        */
    const double* kappa_rho;  /* N doubles                                             */
    int32_t       inputs_on_device;  /* 1: device pointers, read when the request is
                                        admitted, so they must stay valid and unchanged
                                        until it is done; 0: host pointers, copied by
                                        fld_submit before it returns                    */
    void*         stream;     /* device inputs: the hipStream_t that writes them (NULL:
                                 the null stream).  fld_submit records an event on it,
                                 and the server's copy at admission waits for that
                                 event, so work the caller enqueued on this stream
                                 before fld_submit is complete when the inputs are
                                 read.  Ignored for host inputs.                       */
} fld_request;

typedef struct fld_result {
    double*   E_out;          /* device pointer to N doubles inside the arena, valid
                                 until fld_release                                     */
    fld_stats stats;
    double    t_submit;       /* seconds on the library's steady clock                 */
    double    t_admit;        /* slot and arena space granted                          */
    double    t_start;        /* first kernels enqueued                                */
    double    t_done;         /* result written                                        */
} fld_result;

typedef struct fld_server_info {
    int64_t submitted, admitted, completed, failed, rounds, cells_done;
    int32_t pending, resident;
    size_t  arena_bytes, arena_free;
    int32_t error;            /* FLD_OK, or the error that stopped the worker          */
} fld_server_info;

void fld_server_opts_default(fld_server_opts* o);
/* arena_dev: caller-owned device memory (256-byte aligned) the server carves all
   its device buffers from; kept until fld_server_destroy.  Errors: INVALID_ARG,
   TOO_LARGE (arena smaller than the server's tables), HIP. */
int32_t fld_server_create(const fld_server_opts* opts, void* arena_dev, size_t arena_bytes,
                          fld_server_t* out);
/* Stops the worker (requests in flight are abandoned) and frees host state.
   The arena is not touched afterwards. */
int32_t fld_server_destroy(fld_server_t server);
/* Queue one request; *ticket identifies it.  Errors: INVALID_ARG (grid, dt,
   pointers), TOO_LARGE (can never fit the arena), SHUTDOWN, HIP (worker failed). */
int32_t fld_submit(fld_server_t server, const fld_request* req, uint64_t* ticket);
/* FLD_PENDING while queued or running; otherwise the request's final status
   (FLD_OK, NOT_CONVERGED, BAD_INPUT, HIP) with *out filled.  UNKNOWN_TICKET for
   tickets never issued or already released. */
int32_t fld_poll(fld_server_t server, uint64_t ticket, fld_result* out);
/* As fld_poll, blocking up to timeout_s seconds for the request to finish. */
int32_t fld_wait(fld_server_t server, uint64_t ticket, double timeout_s, fld_result* out);
/* Return a finished request's result buffer to the arena (PENDING if not finished). */
int32_t fld_release(fld_server_t server, uint64_t ticket);
int32_t fld_server_info_get(fld_server_t server, fld_server_info* out);

#ifdef __cplusplus
}
#endif

#endif /* FLD_H */
