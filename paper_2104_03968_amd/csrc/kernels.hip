// HIP kernels of the FLD radiation-energy step for gfx950 (wave64, no MFMA:
// every kernel here is a stencil, a reduction or a pointwise update, bound by
// memory bandwidth, not a dense contraction).
//
// Method (Moens et al., "Radiation-hydrodynamics with MPI-AMRVAC:
// flux-limited diffusion"):
//   coefficients  Sec. 3.2 (4th-order gradient), Sec. 2.2 (R, lambda, D),
//                 Sec. 3.4 (harmonic face mean, eq. discdiff)
//   solve         Sec. 3.4 (backward Euler with lagged D, multigrid with a
//                 Gauss-Seidel smoother); the red-black ordering, the
//                 transfer operators and the coarsest-level CG are this
//                 library's own multigrid design
//   exchange      Sec. 3.3 (point-implicit heating/cooling quartic, Halley's
//                 method with a bisection fallback, back-substitution for E)
//
// Every kernel walks a JobList of (level, tile) items with a grid-stride
// loop, so one launch serves one grid or a batch of uneven grids.  Per-grid
// convergence flags (GridState::active) make kernels skip finished grids.
// Reductions are deterministic: fixed per-tile partial sums, fixed-order
// wave butterflies and fixed-order cross-wave sums; no floating-point atomics.
#include "fld_device.hpp"
#include "fld.h"

#include <math.h>

#include <type_traits>

namespace fld {

namespace {

__device__ __forceinline__ int find_job(const int32_t* __restrict__ prefix, int njobs, int t) {
    int lo = 0, hi = njobs;            // prefix[lo] <= t < prefix[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (prefix[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

// XCD-aware tile order for kernels whose tiles share halo data.  The blocks of
// a launch are dealt round-robin to the chip's kXcds dies (block b runs on die
// b % kXcds), each die with its own L2.  With a block count that is a multiple
// of kXcds, die x walks the contiguous tile range [x C, (x+1) C), C = total / kXcds
// rounded up, so neighbouring tiles meet in one L2; otherwise the plain grid-stride
// order is used.  XcdOrder o(total); for (int k = o.first(); o.more(k); k += o.step)
// visits tile o.tile(k).
struct XcdOrder {
    int per, x, chunk, total, start;
    __device__ explicit XcdOrder(int total_) : total(total_) {
        const int G = gridDim.x;
        if (G % kXcds == 0) {
            per = G / kXcds;
            x = blockIdx.x % kXcds;
            start = blockIdx.x / kXcds;
            chunk = (total + kXcds - 1) / kXcds;
        } else {
            per = G;
            x = 0;
            start = blockIdx.x;
            chunk = total;
        }
    }
    __device__ int first() const { return start; }
    __device__ int tile(int k) const { return x * chunk + k; }
    __device__ bool more(int k) const { return k < chunk && x * chunk + k < total; }
};

// The neighbour mask of a level's operator: periodic axes (bits 0-2) and continuous
// faces (bits 3-8).
__device__ __forceinline__ int nb_mask(const LevelDesc& d) { return d.per_mask | (d.cont_mask << 3); }

__device__ __forceinline__ int mirror(int i, int n) {
    // even reflection across a zero-flux face: -1 -> 0, -2 -> 1, n -> n-1, n+1 -> n-2
    return i < 0 ? -1 - i : (i >= n ? 2 * n - 1 - i : i);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Barrier of the NT threads that run a phase: the workgroup, or for NT = 64 the one
// wavefront (its LDS operations complete in order; the fences keep the compiler from
// moving memory accesses across the phase boundary).
template <int NT>
__device__ __forceinline__ void group_sync() {
    if constexpr (NT == 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Deterministic block sum of two values; every thread receives the totals.
template <int NT>
__device__ __forceinline__ void block_sum2(double& a, double& b, double* sh) {
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    group_sync<NT>();                      // sh may still be read from a previous call
    if (lane == 0) { sh[2 * wid] = a; sh[2 * wid + 1] = b; }
    group_sync<NT>();
    double sa = 0.0, sb = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) { sa += sh[2 * i]; sb += sh[2 * i + 1]; }
    a = sa;
    b = sb;
}

template <int DIM>
__device__ __forceinline__ void cell_of_tile(const int32_t n[3], int lt, int tid, int& i, int& j, int& k) {
    const int tx_n = (n[0] + kTX - 1) / kTX;
    const int ty_n = (n[1] + kTY - 1) / kTY;
    const int tx = lt % tx_n;
    const int rest = lt / tx_n;
    const int ty = rest % ty_n;
    k = (DIM == 3) ? rest / ty_n : 0;
    i = tx * kTX + (tid & (kTX - 1));
    j = ty * kTY + (tid / kTX);
}

// Level-0 cell tiles, kCPT0 cells per thread and one reduction partial per tile:
// in 2D kTX x kCY0 cells (x fastest), in 3D kTX x kCY3 x kCZ3 (a thread's cells are
// one column of kCZ3 planes, so the z-neighbours of its cells are its own loads).
template <int DIM>
__device__ __forceinline__ void cell_of_l0tile(const int32_t n[3], int lt, int e, int& i, int& j, int& k) {
    const int tx_n = (n[0] + kTX - 1) / kTX;
    const int tx = lt % tx_n;
    const int rest = lt / tx_n;
    i = tx * kTX + (e & (kTX - 1));
    if (DIM == 3) {
        const int ty_n = (n[1] + kCY3 - 1) / kCY3;
        j = (rest % ty_n) * kCY3 + ((e / kTX) % kCY3);
        k = (rest / ty_n) * kCZ3 + e / (kTX * kCY3);
    } else {
        const int ty_n = (n[1] + kCY0 - 1) / kCY0;
        j = (rest % ty_n) * kCY0 + e / kTX;
        k = rest / ty_n;
    }
}

// Cell m of level-0 tile lt for this thread: its flat index, clamped to the nearest
// cell inside the level so that loads never need a branch, and whether it is inside.
template <int DIM>
__device__ __forceinline__ long l0_cell(const LevelDesc& d, int lt, int m, int& i, int& j, int& k, bool& ok) {
    cell_of_l0tile<DIM>(d.n, lt, threadIdx.x + m * kBlock, i, j, k);
    ok = i < d.n[0] && j < d.n[1] && k < d.n[2];
    i = min(i, d.n[0] - 1);
    j = min(j, d.n[1] - 1);
    k = min(k, d.n[2] - 1);
    return i + (long)d.n[0] * (j + (long)d.n[1] * k);
}

// Sum the level-0 per-tile partials of one grid in a fixed order: thread t adds
// partials t, t + kBlock, t + 2 kBlock, ... in turn, then a fixed-order block sum.
// The loads are issued kSumBatch at a time so they overlap; the additions keep
// their order.  LOAD reads partial i (plain, or past the L1 for the last-block path).
constexpr int kSumBatch = 16;
template <typename LOAD>
__device__ __forceinline__ void sum_parts_with(LOAD load, int ntiles, int stride, double& a, double& b,
                                               double* sh) {
    a = 0.0;
    b = 0.0;
    for (int i0 = threadIdx.x; i0 < ntiles; i0 += kSumBatch * kBlock) {
        double va[kSumBatch], vb[kSumBatch];
#pragma unroll
        for (int u = 0; u < kSumBatch; ++u) {
            const int i = i0 + u * kBlock;
            va[u] = i < ntiles ? load(stride * i) : 0.0;
            vb[u] = (stride == 2 && i < ntiles) ? load(stride * i + 1) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kSumBatch; ++u) {
            if (i0 + u * kBlock < ntiles) {
                a += va[u];
                if (stride == 2) b += vb[u];
            }
        }
    }
    block_sum2<kBlock>(a, b, sh);
}

__device__ __forceinline__ void sum_parts(const double* __restrict__ part, int ntiles, int stride,
                                          double& a, double& b, double* sh) {
    sum_parts_with([&](int i) { return part[i]; }, ntiles, stride, a, b, sh);
}

// The CG scalars from a summed reduction: beta = r.z / (previous r.z) (0 on a restart)
// and alpha = r.z / p.q (0 when p.q is not a positive finite number: breakdown).  The
// iteration's r.z sits in rho[iter & 1] and the previous one in the other slot, so a
// kernel whose blocks form these scalars from the partials themselves can record the
// new r.z in one block while the others still read the previous one.
__device__ __forceinline__ double cg_beta(const GridState& g, double rz) {
    const double prev = g.rho[(g.iter + 1) & 1];
    return (g.iter > 0 && prev != 0.0) ? rz / prev : 0.0;
}
__device__ __forceinline__ double cg_alpha(const GridState& g, double pq) {
    return (pq > 0.0 && isfinite(pq)) ? g.rho[g.iter & 1] / pq : 0.0;
}

// Stop test / CG scalar update of one grid from the summed partials (thread 0).
__device__ void finalize_grid(GridState& g, double s2, double s1, int mode, double rtol, int max_cycles) {
    switch (mode) {
        case FIN_B:
            g.bnorm2 = s2;
            g.bsum = s1;
            g.tol2 = rtol * rtol * s2;
            g.cycles = 0;
            g.iter = 0;
            g.stall = 0;
            g.rnorm2 = s2;
            g.rprev2 = INFINITY;
            g.status = g.bad ? FLD_ERR_BAD_INPUT : FLD_OK;
            g.active = g.bad ? 0 : 1;
            g.bad = 0;                               // read once per step; cleared for the next one
            break;
        case FIN_R_FMG:
        case FIN_R_INIT:
        case FIN_R_VERIFY:
            if (mode == FIN_R_FMG) g.cycles += 1;
            g.rnorm2 = s2;
            g.iter = 0;                              // (re)start CG from this residual
            g.stall = 0;
            if (!(s2 == s2) || isinf(s2)) { g.active = 0; g.status = FLD_ERR_NOT_CONVERGED; }
            else g.active = (s2 > g.tol2 && g.cycles < max_cycles) ? 1 : 0;
            if (g.active == 0 && s2 > g.tol2 && g.status == FLD_OK) g.status = FLD_ERR_NOT_CONVERGED;
            g.rprev2 = s2;
            break;
        case FIN_R_CYCLE:
        case FIN_CG:
            g.rnorm2 = s2;
            g.cycles += 1;
            if (mode == FIN_CG) g.iter += 1;
            if (!(s2 == s2) || isinf(s2)) {
                g.active = 0;
                g.status = FLD_ERR_NOT_CONVERGED;
            } else if (s2 <= g.tol2) {
                g.active = 0;
                g.status = FLD_OK;
            } else if (g.cycles >= max_cycles) {
                g.active = 0;
                g.status = FLD_ERR_NOT_CONVERGED;
            } else {
                // stagnation: no 10 % gain in ||r|| over the best so far for 5 iterations
                if (s2 < 0.81 * g.rprev2) { g.rprev2 = s2; g.stall = 0; }
                else if (++g.stall >= 5) { g.active = 0; g.status = FLD_ERR_NOT_CONVERGED; }
            }
            break;
        case FIN_RZ:
            g.beta = cg_beta(g, s2);
            g.rho[g.iter & 1] = s2;
            break;
        case FIN_PQ:
            g.alpha = cg_alpha(g, s2);
            if (g.alpha == 0.0) {                    // breakdown: no descent direction left
                g.active = 0;
                g.status = (g.rnorm2 <= g.tol2) ? FLD_OK : FLD_ERR_NOT_CONVERGED;
            }
            break;
        default:
            break;
    }
}

// Called by every block after thread 0 stored its tile partial: count the tile
// and report whether it was the grid's last.  The counter is an integer atomic;
// the partials themselves are summed in a fixed order by the last block.
__device__ __forceinline__ bool grid_tile_done(GridState& g, int ntiles, int* flag) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();                             // publish this tile's partial
        const int prev = atomicAdd(&g.done, 1);
        const int last = (prev == ntiles - 1);
        if (last) g.done = 0;                        // every tile has counted: reset for the next
        *flag = last;
    }
    __syncthreads();
    return *flag != 0;
}

// Fixed-order sum of a grid's tile partials, read past the (non-coherent) L1.
__device__ __forceinline__ void sum_parts_coherent(const double* part, int ntiles, int stride, double& a,
                                                   double& b, double* sh) {
    __threadfence();
    sum_parts_with([&](int i) { return __hip_atomic_load(part + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); },
                   ntiles, stride, a, b, sh);
}

// End of a reducing kernel's tile: store the partial(s) and, if this was the
// grid's last tile, finish the reduction (fin < 0: store only, a k_finalize
// launch finishes).  Counting tiles costs one same-address atomic per tile, so
// the host uses it for grids of a few tiles only.
__device__ __forceinline__ void tile_reduce_finish(const LevelDesc& d, GridState& g, int lt, int ntiles,
                                                   double a, double b, int stride, int fin, double rtol,
                                                   int max_cycles, double* sh, int* flag, double* part = nullptr) {
    if (!part) part = d.part;
    block_sum2<kBlock>(a, b, sh);
    if (threadIdx.x == 0) {
        part[stride * lt] = a;
        if (stride == 2) part[stride * lt + 1] = b;
    }
    if (fin < 0) return;
    if (!grid_tile_done(g, ntiles, flag)) return;
    double s2, s1;
    sum_parts_coherent(part, ntiles, stride, s2, s1, sh);
    if (threadIdx.x == 0) finalize_grid(g, s2, s1, fin, rtol, max_cycles);
}

// One block per grid: the same finalization as a separate launch (kept for the
// plain V-cycle path's callers that reduce without finishing).
__global__ void __launch_bounds__(kBlock)
k_finalize(const LevelDesc* __restrict__ L, GridState* __restrict__ S, JobList jl, int mode, double rtol,
           int max_cycles) {
    __shared__ double sh[2 * kBlock / 64];
    const LevelDesc& d = L[job_level(jl, blockIdx.x)];
    GridState& g = S[d.sidx];
    const bool run = (mode == FIN_B) || (mode == FIN_R_VERIFY ? (g.status == FLD_OK && !g.active) : g.active);
    if (!run) return;                                // uniform per block
    double s2, s1;
    // the tiles of the list's reducing kernel (level-0 cell tiles, or the z-march tiles)
    sum_parts(d.part, job_tiles(jl, blockIdx.x), mode == FIN_B ? 2 : 1, s2, s1, sh);
    if (threadIdx.x == 0) finalize_grid(g, s2, s1, mode, rtol, max_cycles);
}

// ---------------------------------------------------------------------------
// K1: coefficients.  R = |grad E|/(kappa rho E) with the 4th-order central
// gradient (mirrored ghosts), lambda(R), D = c lambda/(kappa rho), and the
// lower-face weights dt * 2 D_L D_R/(D_L + D_R) / h^2.  A first pass stores each
// cell's D; the face pass reads the two D of each face (with a diagonal-tensor D
// the face pass recomputes the lower neighbour's from its own stencil).
// ---------------------------------------------------------------------------
// 4th-order central gradient of E at cell (i, j, k) with mirrored ghosts (Sec. 3.2,
// eq. ileyk_flux); c12 = 1 / (12 h) per axis.  g[2] is 0 in 2D.
template <int DIM>
__device__ __forceinline__ void grad4_at(const double* __restrict__ E, int i, int j, int k, const int32_t n[3],
                                         const double c12[3], double g[3]) {
    const long sy = n[0], sz = (long)n[0] * n[1];
    const long row = (long)j * sy + (long)k * sz;
    g[0] = ((E[mirror(i - 2, n[0]) + row] - E[mirror(i + 2, n[0]) + row]) +
            8.0 * (E[mirror(i + 1, n[0]) + row] - E[mirror(i - 1, n[0]) + row])) * c12[0];
    const long col = i + (long)k * sz;
    g[1] = ((E[col + mirror(j - 2, n[1]) * sy] - E[col + mirror(j + 2, n[1]) * sy]) +
            8.0 * (E[col + mirror(j + 1, n[1]) * sy] - E[col + mirror(j - 1, n[1]) * sy])) * c12[1];
    g[2] = 0.0;
    if (DIM == 3) {
        const long pil = i + (long)j * sy;
        g[2] = ((E[pil + mirror(k - 2, n[2]) * sz] - E[pil + mirror(k + 2, n[2]) * sz]) +
                8.0 * (E[pil + mirror(k + 1, n[2]) * sz] - E[pil + mirror(k - 1, n[2]) * sz])) * c12[2];
    }
}

// The same gradient where faces prescribe a gradient G: the ghost at index i
// outside [0, n) is the mirror image plus the linear part of slope G, -(2k-1) h G
// below (i = -k) and +(2k-1) h G above (i = n-1+k); gh = {h G_lo, h G_hi} per axis.
// Dirichlet faces (bit of dir_mask) put their value E_B in both ghost layers;
// periodic axes (bit of per_mask) take the cells at the other end; continuous faces
// (bit of cont_mask) continue the line through the two cells next to the face,
// E_{-k} = E_0 + k (E_0 - E_1) and E_{n-1+k} = E_{n-1} + k (E_{n-1} - E_{n-2}).
__device__ __forceinline__ double ghost_lin(int i, int n, double ghlo, double ghhi) {
    return i < 0 ? (double)(2 * i + 1) * ghlo : (i >= n ? (double)(2 * (i - n) + 1) * ghhi : 0.0);
}

template <int DIM>
__device__ __forceinline__ void grad4_bc_at(const double* __restrict__ E, int i, int j, int k, const int32_t n[3],
                                            const double c12[3], const LevelDesc& bc, double g[3]) {
    const long sy = n[0], sz = (long)n[0] * n[1];
    const double* gh = bc.bcgh;
    const int dm = bc.dir_mask;
    // ghost or interior value at index q of an axis of m cells whose faces are 2a, 2a+1
    const int pmask = bc.per_mask;
    const int cm = bc.cont_mask;
    auto val = [&](long base, long stride, int q, int m, int a) {
        if ((pmask >> a) & 1) return E[base + (q < 0 ? q + m : (q >= m ? q - m : q)) * stride];
        if (q < 0 && ((cm >> (2 * a)) & 1)) {
            const double e0 = E[base], e1 = E[base + stride];
            return e0 + (double)(-q) * (e0 - e1);
        }
        if (q >= m && ((cm >> (2 * a + 1)) & 1)) {
            const double e0 = E[base + (long)(m - 1) * stride], e1 = E[base + (long)(m - 2) * stride];
            return e0 + (double)(q - m + 1) * (e0 - e1);
        }
        const double in = E[base + mirror(q, m) * stride] + ghost_lin(q, m, gh[2 * a], gh[2 * a + 1]);
        if (q < 0 && (dm >> (2 * a)) & 1) return bc.bcv[2 * a];
        if (q >= m && (dm >> (2 * a + 1)) & 1) return bc.bcv[2 * a + 1];
        return in;
    };
    const long row = (long)j * sy + (long)k * sz;
    g[0] = ((val(row, 1, i - 2, n[0], 0) - val(row, 1, i + 2, n[0], 0)) +
            8.0 * (val(row, 1, i + 1, n[0], 0) - val(row, 1, i - 1, n[0], 0))) * c12[0];
    const long col = i + (long)k * sz;
    g[1] = ((val(col, sy, j - 2, n[1], 1) - val(col, sy, j + 2, n[1], 1)) +
            8.0 * (val(col, sy, j + 1, n[1], 1) - val(col, sy, j - 1, n[1], 1))) * c12[1];
    g[2] = 0.0;
    if (DIM == 3) {
        const long pil = i + (long)j * sy;
        g[2] = ((val(pil, sz, k - 2, n[2], 2) - val(pil, sz, k + 2, n[2], 2)) +
                8.0 * (val(pil, sz, k + 1, n[2], 2) - val(pil, sz, k - 1, n[2], 2))) * c12[2];
    }
}

// The 4th-order gradient of a field with mirrored ghosts, wrapped on the periodic
// axes of pmask (the velocity of the photon-tiring term, whose own boundary values
// are not the radiation's).
template <int DIM>
__device__ __forceinline__ void grad4_per_at(const double* __restrict__ F, int i, int j, int k, const int32_t n[3],
                                             const double c12[3], int pmask, double g[3]) {
    const long sy = n[0], sz = (long)n[0] * n[1];
    auto at = [&](long base, long stride, int q, int m, int a) {
        const int qq = ((pmask >> a) & 1) ? (q < 0 ? q + m : (q >= m ? q - m : q)) : mirror(q, m);
        return F[base + qq * stride];
    };
    const long row = (long)j * sy + (long)k * sz;
    g[0] = ((at(row, 1, i - 2, n[0], 0) - at(row, 1, i + 2, n[0], 0)) +
            8.0 * (at(row, 1, i + 1, n[0], 0) - at(row, 1, i - 1, n[0], 0))) * c12[0];
    const long col = i + (long)k * sz;
    g[1] = ((at(col, sy, j - 2, n[1], 1) - at(col, sy, j + 2, n[1], 1)) +
            8.0 * (at(col, sy, j + 1, n[1], 1) - at(col, sy, j - 1, n[1], 1))) * c12[1];
    g[2] = 0.0;
    if (DIM == 3) {
        const long pil = i + (long)j * sy;
        g[2] = ((at(pil, sz, k - 2, n[2], 2) - at(pil, sz, k + 2, n[2], 2)) +
                8.0 * (at(pil, sz, k + 1, n[2], 2) - at(pil, sz, k - 1, n[2], 2))) * c12[2];
    }
}

// Flux limiter lambda(R) (Sec. 2.2): the rational bridging law of eq. fld_lambda,
// 1/3, Minerbo's two branches (meeting with equal value and slope at R = 3/2), or
// Levermore and Pomraning's (coth R - 1/R)/R, by its series below R = 0.1 where
// the difference cancels (the series truncation there is below 1e-16).
__device__ __forceinline__ double limiter_of(double R, int limiter) {
    if (limiter == FLD_LIMITER_DIFFUSION) return 1.0 / 3.0;
    if (limiter == FLD_LIMITER_MINERBO) {
        if (R <= 1.5) return 2.0 / (3.0 + sqrt(9.0 + 12.0 * R * R));
        return 1.0 / (1.0 + R + sqrt(1.0 + 2.0 * R));
    }
    if (limiter == FLD_LIMITER_LP_EXACT) {
        if (R < 0.1) {
            const double r2 = R * R;
            return 1.0 / 3.0 +
                   r2 * (-1.0 / 45.0 + r2 * (2.0 / 945.0 + r2 * (-1.0 / 4725.0 + r2 * (2.0 / 93555.0))));
        }
        return (1.0 / tanh(R) - 1.0 / R) / R;
    }
    if (R < 1e100) return (2.0 + R) / (6.0 + R * (3.0 + R));
    return 1.0 / R;                         // free-streaming limit, avoids inf/inf
}

template <int DIM>
__device__ __forceinline__ double cell_D(const double* __restrict__ E, const double* __restrict__ kr,
                                         int i, int j, int k, const int32_t n[3], const double c12[3],
                                         double c, int limiter, const LevelDesc* bc = nullptr) {
    const long idx = i + (long)n[0] * (j + (long)n[1] * k);
    const double e = E[idx];
    const double kk = kr[idx];
    double g[3];
    if (bc) grad4_bc_at<DIM>(E, i, j, k, n, c12, *bc, g);
    else grad4_at<DIM>(E, i, j, k, n, c12, g);
    double g2 = g[0] * g[0] + g[1] * g[1];
    if (DIM == 3) g2 += g[2] * g[2];
    const double R = sqrt(g2) / (kk * e);
    return c * limiter_of(R, limiter) / kk;
}

__device__ __forceinline__ double face_w(double DL, double DR, double dt, double hinv) {
    return dt * (2.0 * DL * DR / (DL + DR)) * (hinv * hinv);
}

// First pass of the coefficients: D = c lambda(R) / (kappa rho) once per level-0 cell,
// stored in the level's residual array (free until the initial residual), so the face
// pass reads each face's two D instead of recomputing the neighbour's stencil.  Grids
// with a diagonal-tensor D compute theirs in the face pass.
template <int DIM, bool BC>
__global__ void __launch_bounds__(kBlock)
k_cell_D(const LevelDesc* __restrict__ L, JobList jl, const StepIO* __restrict__ io, double c, int limiter) {
    const XcdOrder order(jl.total);
    for (int k_ = order.first(); order.more(k_); k_ += order.per) {
        const int t = order.tile(k_);
        const int jb = find_job(jl.prefix, jl.njobs, t);
        const LevelDesc& d = L[job_level(jl, jb)];
        const StepIO& p = io[d.grid];
        if (p.krd[0]) continue;                                  // uniform per tile
        const int lt = t - job_start(jl, jb);
        const LevelDesc* gh = (BC && d.has_bc) ? &d : nullptr;
        const double c12[3] = {d.hinv[0] / 12.0, d.hinv[1] / 12.0, d.hinv[2] / 12.0};
#pragma unroll
        for (int m_ = 0; m_ < kCPT0; ++m_) {
            int i, j, k;
            cell_of_l0tile<DIM>(d.n, lt, threadIdx.x + m_ * kBlock, i, j, k);
            if (i < d.n[0] && j < d.n[1] && k < d.n[2]) {
                const long idx = i + (long)d.n[0] * (j + (long)d.n[1] * k);
                d.R[idx] = cell_D<DIM>(p.E_in, p.kr, i, j, k, d.n, c12, c, limiter, gh);
            }
        }
    }
}

// BC: the plan has faces other than zero flux (fixed gradient, Dirichlet, periodic); the
// zero-flux instantiation carries none of their code.
template <int DIM, bool MIXED, bool BC>
__global__ void __launch_bounds__(kBlock)
k_coeff(const LevelDesc* __restrict__ L, GridState* __restrict__ S, JobList jl,
        const StepIO* __restrict__ io, double c, int limiter, int fin, double rtol, int max_cycles) {
    __shared__ double sh[2 * kBlock / 64];
    __shared__ int flag;
    const XcdOrder order(jl.total);
    for (int k_ = order.first(); order.more(k_); k_ += order.per) {
        const int t = order.tile(k_);
        const int jb = find_job(jl.prefix, jl.njobs, t);
        const LevelDesc& d = L[job_level(jl, jb)];
        const int lt = t - job_start(jl, jb);
        const StepIO& p = io[d.grid];
        const double dt = p.dt;
        double s2 = 0.0, s1 = 0.0;
#pragma unroll
        for (int m_ = 0; m_ < kCPT0; ++m_) {
            int i, j, k;
            cell_of_l0tile<DIM>(d.n, lt, threadIdx.x + m_ * kBlock, i, j, k);
            if (i < d.n[0] && j < d.n[1] && k < d.n[2]) {
                const double c12[3] = {d.hinv[0] / 12.0, d.hinv[1] / 12.0, d.hinv[2] / 12.0};
                const long idx = i + (long)d.n[0] * (j + (long)d.n[1] * k);
                const double e = p.E_in[idx];
                double wx = 0.0, wy = 0.0, wz = 0.0;
                const LevelDesc* gh = (BC && d.has_bc) ? &d : nullptr;
                const int pm = BC ? d.per_mask : 0;
                double Da[3] = {0.0, 0.0, 0.0};               // the cell's D along each direction
                if (!p.krd[0]) {
                    const double kk = p.kr[idx];
                    const bool ok = (e > 0.0) && isfinite(e) && (kk > 0.0) && isfinite(kk);
                    if (!ok) atomicOr(&S[d.sidx].bad, 1);
                    // cell D from the pass before (k_cell_D, kept in the residual array)
                    const double* Dg = d.R;
                    const double Dc = Dg[idx];
                    Da[0] = Da[1] = Da[2] = Dc;
                    // the face below; on a periodic axis the first cell's is the wrap face
                    const long sy = d.n[0], sz = (long)d.n[0] * d.n[1];
                    const long ixm = i > 0 ? idx - 1 : idx + (d.n[0] - 1);
                    const long iym = j > 0 ? idx - sy : idx + (d.n[1] - 1) * sy;
                    const long izm = k > 0 ? idx - sz : idx + (d.n[2] - 1) * sz;
                    if (i > 0 || (pm & 1)) wx = face_w(Dg[ixm], Dc, dt, d.hinv[0]);
                    if (j > 0 || (pm & 2)) wy = face_w(Dg[iym], Dc, dt, d.hinv[1]);
                    if (DIM == 3 && (k > 0 || (pm & 4))) wz = face_w(Dg[izm], Dc, dt, d.hinv[2]);
                } else {
                    // diagonal-tensor D: the faces normal to direction a use (kappa rho)_a
                    bool ok = (e > 0.0) && isfinite(e);
                    for (int a = 0; a < DIM; ++a) {
                        const double kk = p.krd[a][idx];
                        ok = ok && (kk > 0.0) && isfinite(kk);
                    }
                    if (!ok) atomicOr(&S[d.sidx].bad, 1);
                    for (int a = 0; a < DIM; ++a) Da[a] = cell_D<DIM>(p.E_in, p.krd[a], i, j, k, d.n, c12, c, limiter, gh);
                    const int im = i > 0 ? i - 1 : d.n[0] - 1, jm = j > 0 ? j - 1 : d.n[1] - 1;
                    const int km = k > 0 ? k - 1 : d.n[2] - 1;
                    if (i > 0 || (pm & 1))
                        wx = face_w(cell_D<DIM>(p.E_in, p.krd[0], im, j, k, d.n, c12, c, limiter, gh), Da[0], dt,
                                    d.hinv[0]);
                    if (j > 0 || (pm & 2))
                        wy = face_w(cell_D<DIM>(p.E_in, p.krd[1], i, jm, k, d.n, c12, c, limiter, gh), Da[1], dt,
                                    d.hinv[1]);
                    if (DIM == 3 && (k > 0 || (pm & 4)))
                        wz = face_w(cell_D<DIM>(p.E_in, p.krd[2], i, j, km, d.n, c12, c, limiter, gh), Da[2], dt,
                                    d.hinv[2]);
                }
                d.w[0][idx] = wx;
                d.w[1][idx] = wy;
                if (DIM == 3) d.w[2][idx] = wz;
                if (MIXED) {
                    d.w32[0][idx] = (float)wx;
                    d.w32[1][idx] = (float)wy;
                    if (DIM == 3) d.w32[2][idx] = (float)wz;
                }
                // fixed-gradient faces: the flux -D G through the face, D the cell's own, enters b;
                // Dirichlet faces couple the cell to its ghost (value E_B, one cell width away,
                // the cell's own D): alpha = dt D / h^2 on the diagonal, alpha E_B in b
                double bsrc = e;
                double al = 0.0;
                if (BC && d.has_bc) {
                    const int ci[3] = {i, j, k};
                    for (int a = 0; a < DIM; ++a) {
                        const double wa = dt * Da[a] * d.hinv[a] * d.hinv[a];
                        if (ci[a] == 0) {
                            if ((d.dir_mask >> (2 * a)) & 1) { al += wa; bsrc += wa * d.bcv[2 * a]; }
                            else bsrc += dt * d.hinv[a] * (-Da[a] * d.bcg[2 * a]);
                        }
                        if (ci[a] == d.n[a] - 1) {
                            if ((d.dir_mask >> (2 * a + 1)) & 1) { al += wa; bsrc += wa * d.bcv[2 * a + 1]; }
                            else bsrc += dt * d.hinv[a] * (Da[a] * d.bcg[2 * a + 1]);
                        }
                    }
                }
                if (BC && d.ad) {                           // every cell: coarsening reads them all
                    d.ad[idx] = al;
                    if (MIXED) d.ad32[idx] = (float)al;
                }
                d.B0[idx] = bsrc;
                d.X[idx] = e;
                s2 += bsrc * bsrc;
                s1 += bsrc;
            }
        }
        tile_reduce_finish(d, S[d.sidx], lt, job_tiles(jl, jb), s2, s1, 2, fin, rtol,
                           max_cycles, sh, &flag);
    }
}

// ---------------------------------------------------------------------------
// Coarse-level face weights.  Rediscretised: average the fine weights of the
// sub-faces that make up a coarse face, and scale by 1/4 for the doubled cell
// width.  Galerkin: the coarse operator R A P of the piecewise-constant
// prolongation P and the child-mean restriction R = P^T / 2^DIM, which keeps the
// unit diagonal and gives each coarse face the sum of its sub-face weights over
// 2^DIM (faces inside a coarse cell cancel), twice the rediscretised weight.
// ---------------------------------------------------------------------------
template <int DIM, bool MIXED>
__global__ void __launch_bounds__(kBlock)
k_coarsen(const LevelDesc* __restrict__ L, JobList jl, int galerkin) {
    const XcdOrder order(jl.total);
    for (int k_ = order.first(); order.more(k_); k_ += order.per) {
        const int t = order.tile(k_);
        const int jb = find_job(jl.prefix, jl.njobs, t);
        const LevelDesc& f = L[job_level(jl, jb)];
        const LevelDesc& cL = L[f.coarse];
        int I, J, K;
        cell_of_tile<DIM>(cL.n, t - job_start(jl, jb), threadIdx.x, I, J, K);
        if (I >= cL.n[0] || J >= cL.n[1]) continue;
        const long cidx = I + (long)cL.n[0] * (J + (long)cL.n[1] * K);
        const long fsy = f.n[0], fsz = (long)f.n[0] * f.n[1];
        const long f0 = 2 * I + 2 * J * fsy + (DIM == 3 ? 2 * K * fsz : 0);
        // 1/2^(DIM-1) * 1/4, or 1/2^DIM for the Galerkin product
        const double sc = galerkin ? ((DIM == 3) ? 0.125 : 0.25) : ((DIM == 3) ? 0.0625 : 0.125);
        double wc[3] = {0.0, 0.0, 0.0};
        // x faces: sub-faces at fine x = 2I over (j, j+1) [and (k, k+1)]
        const int pm = f.per_mask;                        // periodic: the wrap faces coarsen too
        if (I > 0 || (pm & 1)) {
            double s = f.w[0][f0] + f.w[0][f0 + fsy];
            if (DIM == 3) s += f.w[0][f0 + fsz] + f.w[0][f0 + fsy + fsz];
            wc[0] = s * sc;
        }
        if (J > 0 || (pm & 2)) {
            double s = f.w[1][f0] + f.w[1][f0 + 1];
            if (DIM == 3) s += f.w[1][f0 + fsz] + f.w[1][f0 + 1 + fsz];
            wc[1] = s * sc;
        }
        if (DIM == 3 && (K > 0 || (pm & 4))) {
            wc[2] = (f.w[2][f0] + f.w[2][f0 + 1] + f.w[2][f0 + fsy] + f.w[2][f0 + 1 + fsy]) * sc;
        }
        for (int a = 0; a < DIM; ++a) {
            cL.w[a][cidx] = wc[a];
            if (MIXED) cL.w32[a][cidx] = (float)wc[a];
        }
        // Dirichlet couplings: the 2^(DIM-1) children on a face carry alpha each; the
        // rediscretised coarse coupling is their mean over 4 (ghost two fine widths away),
        // the Galerkin one their sum over 2^DIM
        if (cL.ad) {
            const double* a = f.ad;
            double sa = a[f0] + a[f0 + 1] + a[f0 + fsy] + a[f0 + fsy + 1];
            if (DIM == 3) sa += a[f0 + fsz] + a[f0 + fsz + 1] + a[f0 + fsz + fsy] + a[f0 + fsz + fsy + 1];
            const double ac = sa * (galerkin ? ((DIM == 3) ? 0.125 : 0.25) : ((DIM == 3) ? 0.0625 : 0.125));
            cL.ad[cidx] = ac;
            if (MIXED) cL.ad32[cidx] = (float)ac;
        }
    }
}

// ---------------------------------------------------------------------------
// Stencil helpers over one level, in precision T.  The operator is
// (A x)_i = x_i + sum_faces w_f (x_i - x_nb); the residual is formed as
// b - x - sum w (x - x_nb), so nearly equal neighbours cancel before scaling.
// ---------------------------------------------------------------------------
// Level arrays live in global memory, but pointers read from a LevelDesc carry no
// address space, so accesses through them compile to flat loads and stores, which
// also count against the LDS wait counter: a kernel that keeps global loads in
// flight while it works on LDS must access them through global pointers.
template <typename T> using gptr = __attribute__((address_space(1))) T*;
template <typename T> __device__ __forceinline__ gptr<T> as_global(T* p) { return (gptr<T>)p; }

template <typename T> struct Arr;
template <> struct Arr<double> {
    __device__ static double* x(const LevelDesc& d) { return d.x; }
    __device__ static double* xs(const LevelDesc& d) { return d.xs; }
    __device__ static double* b(const LevelDesc& d) { return d.b; }
    __device__ static double* w(const LevelDesc& d, int a) { return d.w[a]; }
    __device__ static double* ad(const LevelDesc& d) { return d.ad; }
};
template <> struct Arr<float> {
    __device__ static float* x(const LevelDesc& d) { return d.x32; }
    __device__ static float* xs(const LevelDesc& d) { return d.xs32; }
    __device__ static float* b(const LevelDesc& d) { return d.b32; }
    __device__ static float* w(const LevelDesc& d, int a) { return d.w32[a]; }
    __device__ static float* ad(const LevelDesc& d) { return d.ad32; }
};

// Neighbour access without branches: a neighbour across the domain boundary is
// read from the cell itself and enters with weight 0, so every load is issued
// together (x - x and 0 * x add exactly zero).  nb_lo / nb_hi give the neighbour
// below / above a cell at coordinate i of n along an axis of stride s, wrapped when
// the axis is periodic (the face between the last and the first cell sits in the
// first cell's lower-face slot).  The face below a cell is its own slot, the face
// above is the upper neighbour's.
// bm holds the periodic axes (bit a) and the continuous faces (bit 3 + f, face f = 2a
// below, 2a + 1 above): a continuous face takes the boundary cell's coupling to its
// inner neighbour out of that cell's row (the linearly extrapolated ghost cancels it).
template <typename T, typename P>
__device__ __forceinline__ void nb_lo(P w, P x, long idx, int i, int n, long s, int bm, int a, T& wn, T& xn) {
    const bool per = (bm >> a) & 1;
    const bool cut = i == n - 1 && ((bm >> (4 + 2 * a)) & 1);
    const bool has = (i > 0 || per) && !cut;
    const long nb = i > 0 ? idx - s : (per ? idx + (long)(n - 1) * s : idx);
    const T wv = w[idx];
    wn = has ? wv : T(0);
    xn = x[nb];
}
template <typename T, typename P>
__device__ __forceinline__ void nb_hi(P w, P x, long idx, int i, int n, long s, int bm, int a, T& wn, T& xn) {
    const bool per = (bm >> a) & 1;
    const bool cut = i == 0 && ((bm >> (3 + 2 * a)) & 1);
    const bool has = (i + 1 < n || per) && !cut;
    const long nb = i + 1 < n ? idx + s : (per ? idx - (long)(n - 1) * s : idx);
    const T wv = w[nb];
    wn = has ? wv : T(0);
    xn = x[nb];
}

template <int DIM, typename T, typename P>
__device__ __forceinline__ T residual_at(P x, P b, P w0, P w1, P w2, const int32_t n[3], int i, int j, int k,
                                         P a = nullptr, bool has_a = false, int pm = 0) {
    const long sy = n[0], sz = (long)n[0] * n[1];
    const long idx = i + j * sy + k * sz;
    const T xc = x[idx];
    T r = b[idx] - xc;
    T wl, xl, wr, xr, wd, xd, wu, xu;
    nb_lo(w0, x, idx, i, n[0], 1, pm, 0, wl, xl);
    nb_hi(w0, x, idx, i, n[0], 1, pm, 0, wr, xr);
    nb_lo(w1, x, idx, j, n[1], sy, pm, 1, wd, xd);
    nb_hi(w1, x, idx, j, n[1], sy, pm, 1, wu, xu);
    r -= wl * (xc - xl);
    r -= wr * (xc - xr);
    r -= wd * (xc - xd);
    r -= wu * (xc - xu);
    if (DIM == 3) {
        T wb, xb, wf, xf;
        nb_lo(w2, x, idx, k, n[2], sz, pm, 2, wb, xb);
        nb_hi(w2, x, idx, k, n[2], sz, pm, 2, wf, xf);
        r -= wb * (xc - xb);
        r -= wf * (xc - xf);
    }
    if (has_a) r -= a[idx] * xc;                 // Dirichlet ghost coupling (ghost value 0)
    return r;
}

// Red-black Gauss-Seidel half sweep: update the cells with (i+j+k) % 2 == color
// to x_i = (b_i + sum w_f x_nb) / (1 + sum w_f).
template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock)
k_smooth(const LevelDesc* __restrict__ L, const GridState* __restrict__ S, JobList jl, int color) {
    const XcdOrder order(jl.total);
    for (int k_ = order.first(); order.more(k_); k_ += order.per) {
        const int t = order.tile(k_);
        const int jb = find_job(jl.prefix, jl.njobs, t);
        const LevelDesc& d = L[job_level(jl, jb)];
        if (!S[d.sidx].active) continue;
        const int lt = t - job_start(jl, jb);
        const int tx_n = (d.n[0] + kSX - 1) / kSX;
        const int ty_n = (d.n[1] + kTY - 1) / kTY;
        const int tx = lt % tx_n;
        const int rest = lt / tx_n;
        const int j = (rest % ty_n) * kTY + (threadIdx.x >> 6);
        const int k = (DIM == 3) ? rest / ty_n : 0;
        const int i = tx * kSX + 2 * (threadIdx.x & 63) + ((j + k + color) & 1);
        if (i >= d.n[0] || j >= d.n[1]) continue;
        const gptr<T> x = as_global(Arr<T>::x(d));
        const gptr<T> b = as_global(Arr<T>::b(d));
        const gptr<T> w0 = as_global(Arr<T>::w(d, 0));
        const gptr<T> w1 = as_global(Arr<T>::w(d, 1));
        const long sy = d.n[0], sz = (long)d.n[0] * d.n[1];
        const long idx = i + j * sy + k * sz;
        const int pm = nb_mask(d);
        T s = b[idx], dg = T(1);
        T wl, xl, wr, xr, wd, xd, wu, xu;
        nb_lo(w0, x, idx, i, d.n[0], 1, pm, 0, wl, xl);
        nb_hi(w0, x, idx, i, d.n[0], 1, pm, 0, wr, xr);
        nb_lo(w1, x, idx, j, d.n[1], sy, pm, 1, wd, xd);
        nb_hi(w1, x, idx, j, d.n[1], sy, pm, 1, wu, xu);
        s += wl * xl; dg += wl;
        s += wr * xr; dg += wr;
        s += wd * xd; dg += wd;
        s += wu * xu; dg += wu;
        if (DIM == 3) {
            const gptr<T> w2 = as_global(Arr<T>::w(d, 2));
            T wb, xb, wf, xf;
            nb_lo(w2, x, idx, k, d.n[2], sz, pm, 2, wb, xb);
            nb_hi(w2, x, idx, k, d.n[2], sz, pm, 2, wf, xf);
            s += wb * xb; dg += wb;
            s += wf * xf; dg += wf;
        }
        if (Arr<T>::ad(d)) dg += as_global(Arr<T>::ad(d))[idx];
        x[idx] = s / dg;
    }
}

// Residual of the 2^DIM children, averaged into the coarse right-hand side;
// the coarse correction starts from zero.
template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock)
k_restrict(const LevelDesc* __restrict__ L, const GridState* __restrict__ S, JobList jl) {
    const XcdOrder order(jl.total);
    for (int k_ = order.first(); order.more(k_); k_ += order.per) {
        const int t = order.tile(k_);
        const int jb = find_job(jl.prefix, jl.njobs, t);
        const LevelDesc& f = L[job_level(jl, jb)];
        if (!S[f.sidx].active) continue;
        const LevelDesc& cL = L[f.coarse];
        int I, J, K;
        cell_of_tile<DIM>(cL.n, t - job_start(jl, jb), threadIdx.x, I, J, K);
        if (I >= cL.n[0] || J >= cL.n[1]) continue;
        const gptr<T> x = as_global(Arr<T>::x(f));
        const gptr<T> b = as_global(Arr<T>::b(f));
        const gptr<T> w0 = as_global(Arr<T>::w(f, 0));
        const gptr<T> w1 = as_global(Arr<T>::w(f, 1));
        const gptr<T> w2 = as_global((DIM == 3) ? Arr<T>::w(f, 2) : Arr<T>::w(f, 0));
        T s = T(0);
#pragma unroll
        for (int c = 0; c < (1 << DIM); ++c) {
            s += residual_at<DIM, T>(x, b, w0, w1, w2, f.n, 2 * I + (c & 1), 2 * J + ((c >> 1) & 1),
                                     DIM == 3 ? 2 * K + (c >> 2) : 0, as_global(Arr<T>::ad(f)),
                                     Arr<T>::ad(f) != nullptr, nb_mask(f));
        }
        const long cidx = I + (long)cL.n[0] * (J + (long)cL.n[1] * K);
        as_global(Arr<T>::b(cL))[cidx] = s * T(DIM == 3 ? 0.125 : 0.25);
        as_global(Arr<T>::x(cL))[cidx] = T(0);
    }
}

// Piecewise-constant prolongation of the coarse correction, added to the fine level.
template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock)
k_prolong(const LevelDesc* __restrict__ L, const GridState* __restrict__ S, JobList jl) {
    const XcdOrder order(jl.total);
    for (int k_ = order.first(); order.more(k_); k_ += order.per) {
        const int t = order.tile(k_);
        const int jb = find_job(jl.prefix, jl.njobs, t);
        const LevelDesc& f = L[job_level(jl, jb)];
        if (!S[f.sidx].active) continue;
        const LevelDesc& cL = L[f.coarse];
        int i, j, k;
        cell_of_tile<DIM>(f.n, t - job_start(jl, jb), threadIdx.x, i, j, k);
        if (i >= f.n[0] || j >= f.n[1]) continue;
        const long idx = i + (long)f.n[0] * (j + (long)f.n[1] * k);
        const long cidx = (i >> 1) + (long)cL.n[0] * ((j >> 1) + (long)cL.n[1] * (k >> 1));
        as_global(Arr<T>::x(f))[idx] += as_global(Arr<T>::x(cL))[cidx];
    }
}

// Full-multigrid start, first half: the coarse right-hand side is the mean of the
// 2^DIM children's right-hand sides (the restriction of the V-cycle applied to b
// itself), and the coarse iterate starts from zero.
template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock)
k_restrict_rhs(const LevelDesc* __restrict__ L, const GridState* __restrict__ S, JobList jl) {
    const XcdOrder order(jl.total);
    for (int k_ = order.first(); order.more(k_); k_ += order.per) {
        const int t = order.tile(k_);
        const int jb = find_job(jl.prefix, jl.njobs, t);
        const LevelDesc& f = L[job_level(jl, jb)];
        if (!S[f.sidx].active) continue;
        const LevelDesc& cL = L[f.coarse];
        int I, J, K;
        cell_of_tile<DIM>(cL.n, t - job_start(jl, jb), threadIdx.x, I, J, K);
        if (I >= cL.n[0] || J >= cL.n[1]) continue;
        const gptr<T> b = as_global(Arr<T>::b(f));
        const long sy = f.n[0], sz = (long)f.n[0] * f.n[1];
        const long f0 = 2 * I + 2 * J * sy + (DIM == 3 ? 2 * K * sz : 0);
        T s = b[f0] + b[f0 + 1] + b[f0 + sy] + b[f0 + sy + 1];
        if (DIM == 3) s += b[f0 + sz] + b[f0 + sz + 1] + b[f0 + sz + sy] + b[f0 + sz + sy + 1];
        const long cidx = I + (long)cL.n[0] * (J + (long)cL.n[1] * K);
        as_global(Arr<T>::b(cL))[cidx] = s * T(DIM == 3 ? 0.125 : 0.25);
        as_global(Arr<T>::x(cL))[cidx] = T(0);
    }
}

// Full-multigrid start, second half: the fine iterate is the linear interpolation
// of the coarse solution between coarse cell centres, per axis weight 3/4 on the
// parent and 1/4 on the coarse neighbour on the child's side (that neighbour is
// the parent itself at a domain face, the mirror image of zero flux).
template <int DIM, typename T>
__global__ void __launch_bounds__(kBlock)
k_fmg_interp(const LevelDesc* __restrict__ L, const GridState* __restrict__ S, JobList jl) {
    const XcdOrder order(jl.total);
    for (int k_ = order.first(); order.more(k_); k_ += order.per) {
        const int t = order.tile(k_);
        const int jb = find_job(jl.prefix, jl.njobs, t);
        const LevelDesc& f = L[job_level(jl, jb)];
        if (!S[f.sidx].active) continue;
        const LevelDesc& cL = L[f.coarse];
        int i, j, k;
        cell_of_tile<DIM>(f.n, t - job_start(jl, jb), threadIdx.x, i, j, k);
        if (i >= f.n[0] || j >= f.n[1]) continue;
        const gptr<T> xc = as_global(Arr<T>::x(cL));
        const int I0 = i >> 1, J0 = j >> 1, K0 = k >> 1;
        // the coarse neighbour on the child's side, clamped into the grid
        // (wrapped on periodic axes)
        const int pm = f.per_mask;
        auto side = [&](int c0, int odd, int nc, int per) {
            const int c1 = c0 + (odd ? 1 : -1);
            return per ? (c1 + nc) % nc : min(max(c1, 0), nc - 1);
        };
        const int I1 = side(I0, i & 1, cL.n[0], pm & 1);
        const int J1 = side(J0, j & 1, cL.n[1], (pm >> 1) & 1);
        const int K1 = (DIM == 3) ? side(K0, k & 1, cL.n[2], (pm >> 2) & 1) : 0;
        const long sy = cL.n[0], sz = (long)cL.n[0] * cL.n[1];
        const T w0 = T(0.75), w1 = T(0.25);
        auto row = [&](int jj, int kk) {
            const long r = jj * sy + kk * sz;
            return w0 * xc[I0 + r] + w1 * xc[I1 + r];
        };
        T v = w0 * row(J0, K0) + w1 * row(J1, K0);
        if (DIM == 3) v = w0 * v + w1 * (w0 * row(J0, K1) + w1 * row(J1, K1));
        as_global(Arr<T>::x(f))[i + (long)f.n[0] * (j + (long)f.n[1] * k)] = v;
    }
}

// ---------------------------------------------------------------------------
// Coarsest level: Jacobi-preconditioned conjugate gradients in one workgroup
// per grid, from a zero start, to a 1e-6 relative residual (or n iterations).
// Up to kCoarseMaxLDS cells the search direction lives in LDS and every other
// vector in registers; larger coarsest levels use workspace scratch vectors.
// ---------------------------------------------------------------------------
template <int DIM, typename T>
__device__ __forceinline__ void cell_coords(const int32_t n[3], int c, int& i, int& j, int& k) {
    i = c % n[0];
    const int r = c / n[0];
    j = r % n[1];
    k = (DIM == 3) ? r / n[1] : 0;
}

template <int DIM, typename T>
__device__ __forceinline__ T apply_at(const T* __restrict__ p, const T* __restrict__ w0,
                                      const T* __restrict__ w1, const T* __restrict__ w2,
                                      const int32_t n[3], int c, T& dg, const T* a, bool has_a, int pm) {
    int i, j, k;
    cell_coords<DIM, T>(n, c, i, j, k);
    const long sy = n[0], sz = (long)n[0] * n[1];
    const T pc = p[c];
    T q = pc;
    dg = T(1);
    T wl, pl, wr, pr, wd, pd, wu, pu;
    nb_lo(w0, p, c, i, n[0], 1, pm, 0, wl, pl);
    nb_hi(w0, p, c, i, n[0], 1, pm, 0, wr, pr);
    nb_lo(w1, p, c, j, n[1], sy, pm, 1, wd, pd);
    nb_hi(w1, p, c, j, n[1], sy, pm, 1, wu, pu);
    q += wl * (pc - pl); dg += wl;
    q += wr * (pc - pr); dg += wr;
    q += wd * (pc - pd); dg += wd;
    q += wu * (pc - pu); dg += wu;
    if (DIM == 3) {
        T wb, pb, wf, pf;
        nb_lo(w2, p, c, k, n[2], sz, pm, 2, wb, pb);
        nb_hi(w2, p, c, k, n[2], sz, pm, 2, wf, pf);
        q += wb * (pc - pb); dg += wb;
        q += wf * (pc - pf); dg += wf;
    }
    if (has_a) {
        q += a[c] * pc;
        dg += a[c];
    }
    return q;
}

template <int DIM, typename T>
__device__ __forceinline__ T diag_at(const T* __restrict__ w0, const T* __restrict__ w1,
                                     const T* __restrict__ w2, const int32_t n[3], int c, const T* a, bool has_a,
                                     int pm) {
    int i, j, k;
    cell_coords<DIM, T>(n, c, i, j, k);
    const long sy = n[0], sz = (long)n[0] * n[1];
    T dg = T(1);
    T wn, unused;
    nb_lo(w0, w0, c, i, n[0], 1, pm, 0, wn, unused); dg += wn;
    nb_hi(w0, w0, c, i, n[0], 1, pm, 0, wn, unused); dg += wn;
    nb_lo(w1, w1, c, j, n[1], sy, pm, 1, wn, unused); dg += wn;
    nb_hi(w1, w1, c, j, n[1], sy, pm, 1, wn, unused); dg += wn;
    if (DIM == 3) {
        nb_lo(w2, w2, c, k, n[2], sz, pm, 2, wn, unused); dg += wn;
        nb_hi(w2, w2, c, k, n[2], sz, pm, 2, wn, unused); dg += wn;
    }
    if (has_a) dg += a[c];
    return dg;
}

// Block-wide red-black Gauss-Seidel on one level of up to NT * CPT cells, iterate in
// p_sh (LDS): each colour update x_c += (b_c - (A x)_c) / A_cc, the residual norm checked
// every 8 sweeps against tol2 (squared, relative to the starting residual).
template <int DIM, typename T, int NT, int CPT>
__device__ __forceinline__ void block_rbgs(const int32_t n[3], const T* w0, const T* w1, const T* w2, const T* b,
                                           T* x, bool warm, T* p_sh, double* red, const T* a, bool has_a, int pm,
                                           int maxit, double tol2) {
    const int ncell = n[0] * n[1] * n[2];
    T dinv[CPT];
    int col[CPT];
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int c = threadIdx.x + m * NT;
        dinv[m] = T(0);
        col[m] = -1;
        if (c < ncell) {
            int i, j, k;
            cell_coords<DIM, T>(n, c, i, j, k);
            col[m] = (i + j + k) & 1;
            dinv[m] = T(1) / diag_at<DIM, T>(w0, w1, w2, n, c, a, has_a, pm);
            p_sh[c] = warm ? x[c] : T(0);
        }
    }
    group_sync<NT>();
    double rr0 = -1.0;
    for (int it = 0; it < 4 * maxit; ++it) {
        for (int color = 0; color < 2; ++color) {
#pragma unroll
            for (int m = 0; m < CPT; ++m) {
                const int c = threadIdx.x + m * NT;
                if (col[m] == color) {
                    T dg;
                    const T ax = apply_at<DIM, T>(p_sh, w0, w1, w2, n, c, dg, a, has_a, pm);
                    p_sh[c] += (b[c] - ax) * dinv[m];
                }
            }
            group_sync<NT>();
        }
        if ((it & 7) == 7 || it == 0) {
            double rr = 0.0, unused = 0.0;
#pragma unroll
            for (int m = 0; m < CPT; ++m) {
                const int c = threadIdx.x + m * NT;
                if (c < ncell) {
                    T dg;
                    const double r = (double)b[c] - (double)apply_at<DIM, T>(p_sh, w0, w1, w2, n, c, dg, a, has_a, pm);
                    rr += r * r;
                }
            }
            block_sum2<NT>(rr, unused, red);
            if (rr0 < 0.0) rr0 = rr;
            if (!(rr > tol2 * rr0)) break;
        }
    }
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int c = threadIdx.x + m * NT;
        if (c < ncell) x[c] = p_sh[c];
    }
    group_sync<NT>();
}

// Block-wide Jacobi-preconditioned CG on one level of up to NT * CPT cells.
// Starts from x (read from `x` when warm, else zero), runs until the residual
// falls by 1e-6 (or maxit iterations) and writes the result back to `x`.  The
// search direction lives in p_sh (LDS); x, r and the inverse diagonal live in
// registers of the thread owning the cell.  w, b and x may be global or LDS.
template <int DIM, typename T, int NT, int CPT>
__device__ __forceinline__ void block_cg(const int32_t n[3], const T* w0, const T* w1, const T* w2, const T* b, T* x,
                         bool warm, T* p_sh, double* red, const T* a, bool has_a, int pm) {
    const int ncell = n[0] * n[1] * n[2];
    const int maxit = ncell < 2000 ? ncell + 4 : 2000;
    const double tol2 = 1e-12;                 // (1e-6)^2 relative
    if ((pm >> 3) != 0) {
        // continuous faces (a single-level grid's level 0): the operator is not symmetric,
        // so conjugate gradients do not apply; red-black Gauss-Seidel to the same
        // tolerance instead (the operator is an M-matrix with unit row sums)
        block_rbgs<DIM, T, NT, CPT>(n, w0, w1, w2, b, x, warm, p_sh, red, a, has_a, pm, maxit, tol2);
        return;
    }
    T xr[CPT], r[CPT], dinv[CPT];
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int c = threadIdx.x + m * NT;
        xr[m] = T(0);
        r[m] = T(0);
        dinv[m] = T(0);
        if (c < ncell) {
            dinv[m] = T(1) / diag_at<DIM, T>(w0, w1, w2, n, c, a, has_a, pm);
            xr[m] = warm ? x[c] : T(0);
            p_sh[c] = xr[m];
        }
    }
    group_sync<NT>();
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int c = threadIdx.x + m * NT;
        if (c < ncell) {
            T dg;
            r[m] = b[c];
            if (warm) r[m] -= apply_at<DIM, T>(p_sh, w0, w1, w2, n, c, dg, a, has_a, pm);
        }
    }
    group_sync<NT>();
    double rz = 0.0, rr0 = 0.0;
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int c = threadIdx.x + m * NT;
        if (c < ncell) {
            const T z = r[m] * dinv[m];
            p_sh[c] = z;
            rz += (double)r[m] * (double)z;
            rr0 += (double)r[m] * (double)r[m];
        }
    }
    block_sum2<NT>(rz, rr0, red);     // also orders the p_sh writes
    if (rr0 > 0.0) {
        for (int it = 0; it < maxit; ++it) {
            T q[CPT];
            double pq = 0.0, unused = 0.0;
#pragma unroll
            for (int m = 0; m < CPT; ++m) {
                const int c = threadIdx.x + m * NT;
                q[m] = T(0);
                if (c < ncell) {
                    T dg;
                    q[m] = apply_at<DIM, T>(p_sh, w0, w1, w2, n, c, dg, a, has_a, pm);
                    pq += (double)p_sh[c] * (double)q[m];
                }
            }
            block_sum2<NT>(pq, unused, red);
            if (!(pq > 0.0)) break;
            const T alpha = (T)(rz / pq);
            double rz_new = 0.0, rr = 0.0;
#pragma unroll
            for (int m = 0; m < CPT; ++m) {
                const int c = threadIdx.x + m * NT;
                if (c < ncell) {
                    xr[m] += alpha * p_sh[c];
                    r[m] -= alpha * q[m];
                    const T z = r[m] * dinv[m];
                    rz_new += (double)r[m] * (double)z;
                    rr += (double)r[m] * (double)r[m];
                }
            }
            block_sum2<NT>(rz_new, rr, red);   // every thread is done reading p_sh
            if (rr <= tol2 * rr0) break;
            const T beta = (T)(rz_new / rz);
            rz = rz_new;
#pragma unroll
            for (int m = 0; m < CPT; ++m) {
                const int c = threadIdx.x + m * NT;
                if (c < ncell) p_sh[c] = r[m] * dinv[m] + beta * p_sh[c];
            }
            group_sync<NT>();
        }
    }
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int c = threadIdx.x + m * NT;
        if (c < ncell) x[c] = xr[m];
    }
    group_sync<NT>();
}

template <int DIM, typename T>
__global__ void __launch_bounds__(kCoarseThreads)
k_coarse_solve(const LevelDesc* __restrict__ L, const GridState* __restrict__ S, JobList jl) {
    __shared__ T p_sh[kCoarseMaxLDS];
    __shared__ double red[2 * kCoarseThreads / 64];
    const LevelDesc& d = L[job_level(jl, blockIdx.x)];
    if (!S[d.sidx].active) return;
    const int ncell = d.n[0] * d.n[1] * d.n[2];
    const T* w0 = Arr<T>::w(d, 0);
    const T* w1 = Arr<T>::w(d, 1);
    const T* w2 = (DIM == 3) ? Arr<T>::w(d, 2) : nullptr;
    T* xg = Arr<T>::x(d);
    const T* bg = Arr<T>::b(d);
    const T* ag = Arr<T>::ad(d);
    const bool has_a = ag != nullptr;
    // The finest level of a single-level FP64 grid holds the solution itself: iterate
    // from it.  Every other coarsest level solves for a correction from zero.
    const bool warm = (d.level == 0) && (sizeof(T) == sizeof(double));
    if (ncell <= kCoarseMaxLDS) {
        block_cg<DIM, T, kCoarseThreads, kCoarseCPT>(d.n, w0, w1, w2, bg, xg, warm, p_sh, red, ag, has_a,
                                                     nb_mask(d));
        return;
    }
    const int maxit = 2000;
    const double tol2 = 1e-12;
    // Large coarsest level: vectors in workspace scratch (x lives in the level itself).
    T* r = reinterpret_cast<T*>(d.scratch);
    T* p = r + ncell;
    T* q = p + ncell;
    T* dv = q + ncell;
    double rz = 0.0, rr0 = 0.0;
    if (!warm)
        for (int c = threadIdx.x; c < ncell; c += kCoarseThreads) xg[c] = T(0);
    __syncthreads();
    for (int c = threadIdx.x; c < ncell; c += kCoarseThreads) {
        T dg;
        const T ax = apply_at<DIM, T>(xg, w0, w1, w2, d.n, c, dg, ag, has_a, nb_mask(d));
        const T rc = bg[c] - ax;
        const T z = rc / dg;
        r[c] = rc;
        dv[c] = T(1) / dg;
        p[c] = z;
        rz += (double)rc * (double)z;
        rr0 += (double)rc * (double)rc;
    }
    block_sum2<kCoarseThreads>(rz, rr0, red);
    if (rr0 <= 0.0) return;
    for (int it = 0; it < maxit; ++it) {
        double pq = 0.0, unused = 0.0;
        for (int c = threadIdx.x; c < ncell; c += kCoarseThreads) {
            T dg;
            const T qc = apply_at<DIM, T>(p, w0, w1, w2, d.n, c, dg, ag, has_a, nb_mask(d));
            q[c] = qc;
            pq += (double)p[c] * (double)qc;
        }
        block_sum2<kCoarseThreads>(pq, unused, red);
        if (!(pq > 0.0)) break;
        const T alpha = (T)(rz / pq);
        double rz_new = 0.0, rr = 0.0;
        for (int c = threadIdx.x; c < ncell; c += kCoarseThreads) {
            xg[c] += alpha * p[c];
            const T rc = r[c] - alpha * q[c];
            r[c] = rc;
            rz_new += (double)rc * (double)(rc * dv[c]);
            rr += (double)rc * (double)rc;
        }
        block_sum2<kCoarseThreads>(rz_new, rr, red);
        if (rr <= tol2 * rr0) break;
        const T beta = (T)(rz_new / rz);
        rz = rz_new;
        for (int c = threadIdx.x; c < ncell; c += kCoarseThreads) p[c] = r[c] * dv[c] + beta * p[c];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Fused 2D level kernels.  A tile of FX x FY cells is staged in LDS with a halo
// of width HALO and every half sweep is computed on a region that shrinks by one
// ring, so the tile's cells come out exactly as a global red-black sweep would
// leave them (the halo recomputes what neighbouring tiles compute).  Cells
// outside the domain hold x = b = 0 and zero face weights, so updating them
// keeps them 0 and no boundary test is needed inside the sweep.  A pass never
// reads the array it writes (tiles overlap through their halos): down reads x
// (when it starts from a stored iterate) and writes xs; up reads xs and writes x.
//
// The tile is stored by colour: plane q holds the cells of global parity
// (i + j) % 2 = q, row by row, cell li of row lj at index li / 2.  A half sweep
// then reads its operands at unit stride (its neighbours are all in the other
// plane: left at k + s - 1, right at k + s, up and down at k, where the cell
// is li = 2k + s), so all lanes of a wave work and LDS accesses do not collide.
// ---------------------------------------------------------------------------
template <typename T, int W_, int H_>
struct Tile2 {
    static constexpr int W = W_;
    static constexpr int H = H_;
    static constexpr int KW = W_ / 2;      // cells of one colour per row
    static_assert(W_ % 2 == 0, "tile width must be even");
    T x[2][H][KW];
    T b[2][H][KW];
    T w0[2][H][KW];
    T w1[2][H][KW];
    // cell (li, lj) of a tile whose corner has parity G = (gx0 + gy0) & 1
    __device__ T& X(int li, int lj, int G) { return x[(li + lj + G) & 1][lj][li >> 1]; }
    __device__ T& B(int li, int lj, int G) { return b[(li + lj + G) & 1][lj][li >> 1]; }
    __device__ T& W0(int li, int lj, int G) { return w0[(li + lj + G) & 1][lj][li >> 1]; }
    __device__ T& W1(int li, int lj, int G) { return w1[(li + lj + G) & 1][lj][li >> 1]; }
};

template <int NT, typename Tl>
__device__ __forceinline__ void tile2_half_sweep(Tl& t, int G, int color, int m) {
    // update the cells of `color` with local coordinates in [m, W-m) x [m, H-m)
    constexpr int KW = Tl::KW;
    const int o = color ^ 1;
    const int n = (Tl::H - 2 * m) * KW;
    for (int e = threadIdx.x; e < n; e += NT) {
        const int r = e / KW;
        const int k = e - r * KW;
        const int lj = m + r;
        const int sft = (color + lj + G) & 1;          // this colour's cells in row lj: li = 2k + sft
        const int li = 2 * k + sft;
        if (li < m || li >= Tl::W - m) continue;
        const auto wl = t.w0[color][lj][k], wr = t.w0[o][lj][k + sft], wd = t.w1[color][lj][k],
                   wu = t.w1[o][lj + 1][k];
        const auto s = t.b[color][lj][k] + wl * t.x[o][lj][k + sft - 1] + wr * t.x[o][lj][k + sft] +
                       wd * t.x[o][lj - 1][k] + wu * t.x[o][lj + 1][k];
        t.x[color][lj][k] = s / (decltype(s)(1) + wl + wr + wd + wu);
    }
    __syncthreads();
}

// A tile's operands in registers between their loads and their LDS stores.  The
// loads are branch-free (a cell outside the level loads its nearest in-level cell
// and is stored as 0), so a block can issue the next tile's loads and sweep the
// current one while they are in flight.
template <typename T, int NE>
struct Tile2Regs {
    T x[NE], c[NE], b[NE], w0[NE], w1[NE];
    uint32_t ok;          // bit r: element r lies inside the level
};

template <typename T, typename Tl, int NE, int NT>
__device__ __forceinline__ void tile2_fetch(Tile2Regs<T, NE>& v, const LevelDesc& d, const gptr<T> xs, int gx0,
                                            int gy0, bool load_x, const gptr<T> cx, int ncx) {
    static_assert(NE <= 32, "ok mask");
    const gptr<T> bs = as_global(Arr<T>::b(d));
    const gptr<T> w0 = as_global(Arr<T>::w(d, 0));
    const gptr<T> w1 = as_global(Arr<T>::w(d, 1));
    constexpr int W = Tl::W, H = Tl::H;
    v.ok = 0;
#pragma unroll
    for (int r = 0; r < NE; ++r) {
        const int e = threadIdx.x + r * NT;
        const int ec = min(e, W * H - 1);
        const int lj = ec / W, li = ec - lj * W;
        const int gi = gx0 + li, gj = gy0 + lj;
        const bool ok = e < W * H && gi >= 0 && gi < d.n[0] && gj >= 0 && gj < d.n[1];
        const int ic = min(max(gi, 0), d.n[0] - 1), jc = min(max(gj, 0), d.n[1] - 1);
        const long idx = ic + (long)d.n[0] * jc;
        v.ok |= (ok ? 1u : 0u) << r;
        v.b[r] = bs[idx];
        v.w0[r] = w0[idx];
        v.w1[r] = w1[idx];
        v.x[r] = load_x ? xs[idx] : T(0);
        v.c[r] = cx ? cx[(ic >> 1) + (long)ncx * (jc >> 1)] : T(0);
    }
}

// Store fetched operands to the tile (x plus the prolonged coarse correction when
// add_c); cells outside the level hold x = b = 0 and zero face weights.
template <typename T, typename Tl, int NE, int NT>
__device__ __forceinline__ void tile2_put(Tl& t, const Tile2Regs<T, NE>& v, int gx0, int gy0, bool add_c) {
    constexpr int W = Tl::W, H = Tl::H;
    const int G = (gx0 + gy0) & 1;
#pragma unroll
    for (int r = 0; r < NE; ++r) {
        const int e = threadIdx.x + r * NT;
        if (e < W * H) {
            const int lj = e / W, li = e - lj * W;
            const bool ok = (v.ok >> r) & 1u;
            T xx = v.x[r];
            if (add_c) xx += v.c[r];
            t.X(li, lj, G) = ok ? xx : T(0);
            t.B(li, lj, G) = ok ? v.b[r] : T(0);
            t.W0(li, lj, G) = ok ? v.w0[r] : T(0);
            t.W1(li, lj, G) = ok ? v.w1[r] : T(0);
        }
    }
    __syncthreads();
}

// One tile of a fused 2D launch: its level, the coarser level, its corner and
// whether its grid is still iterating.
struct Tile2Job {
    const LevelDesc* d;
    const LevelDesc* c;
    int gx0, gy0;
    bool act;
};

template <int FX, int FY, int HALO>
__device__ __forceinline__ Tile2Job tile2_job(const LevelDesc* __restrict__ L, const GridState* __restrict__ S,
                                              const JobList& jl, int tt) {
    Tile2Job j;
    const int jb = find_job(jl.prefix, jl.njobs, tt);
    j.d = &L[job_level(jl, jb)];
    j.c = &L[j.d->coarse];
    j.act = S[j.d->sidx].active != 0;
    const int lt = tt - job_start(jl, jb);
    const int tx_n = (j.d->n[0] + FX - 1) / FX;
    j.gx0 = (lt % tx_n) * FX - HALO;
    j.gy0 = (lt / tx_n) * FY - HALO;
    return j;
}

template <typename T, int NU, int WIDE, int FY, int NT>
__global__ void __launch_bounds__(NT)
k_down2(const LevelDesc* __restrict__ L, const GridState* __restrict__ S, JobList jl, int load_x) {
    constexpr int HALO = 2 * NU + 1;
    constexpr int FX = fused_fx(HALO, WIDE);
    using Tl = Tile2<T, FX + 2 * HALO, FY + 2 * HALO>;
    constexpr int NE = (Tl::W * Tl::H + NT - 1) / NT;
    __shared__ Tl t;
    const XcdOrder order(jl.total);
    int k = order.first();
    if (!order.more(k)) return;
    Tile2Job cj = tile2_job<FX, FY, HALO>(L, S, jl, order.tile(k));
    Tile2Regs<T, NE> v;
    tile2_fetch<T, Tl, NE, NT>(v, *cj.d, as_global(Arr<T>::x(*cj.d)), cj.gx0, cj.gy0, load_x != 0, nullptr, 0);
    // the current tile's job, kept in scalars (an aggregate copied across iterations
    // would be placed in LDS by the compiler)
    const LevelDesc* cd = cj.d;
    const LevelDesc* cc = cj.c;
    int cgx = cj.gx0, cgy = cj.gy0, cact = cj.act ? 1 : 0;
    while (true) {
        if (cact) tile2_put<T, Tl, NE, NT>(t, v, cgx, cgy, false);
        // the next tile's loads are in flight while this one is swept
        const int kn = k + order.per;
        const bool more = order.more(kn);
        const LevelDesc* nd = cd;
        const LevelDesc* nc = cc;
        int ngx = cgx, ngy = cgy, nact = cact;
        if (more) {
            const Tile2Job nj = tile2_job<FX, FY, HALO>(L, S, jl, order.tile(kn));
            nd = nj.d;
            nc = nj.c;
            ngx = nj.gx0;
            ngy = nj.gy0;
            nact = nj.act ? 1 : 0;
            tile2_fetch<T, Tl, NE, NT>(v, *nd, as_global(Arr<T>::x(*nd)), ngx, ngy, load_x != 0, nullptr, 0);
        }
        if (cact) {
            const LevelDesc& d = *cd;
            const LevelDesc& cL = *cc;
            const int gx0 = cgx, gy0 = cgy;
            const int G = (gx0 + gy0) & 1;
            for (int it = 0; it < NU; ++it) {
                tile2_half_sweep<NT>(t, G, 0, 2 * it + 1);
                tile2_half_sweep<NT>(t, G, 1, 2 * it + 2);
            }
            // smoothed iterate of the interior (to xs: other tiles may still read x), and the
            // residual averaged onto the coarse cells
            const gptr<T> xo = as_global(Arr<T>::xs(d));
            for (int e = threadIdx.x; e < FX * FY; e += NT) {
                const int lj = e / FX, li = e - lj * FX;
                const int gi = gx0 + HALO + li, gj = gy0 + HALO + lj;
                if (gi < d.n[0] && gj < d.n[1]) xo[gi + (long)d.n[0] * gj] = t.X(HALO + li, HALO + lj, G);
            }
            const gptr<T> cb = as_global(Arr<T>::b(cL));
            for (int e = threadIdx.x; e < (FX / 2) * (FY / 2); e += NT) {
                const int cj_ = e / (FX / 2), ci = e - cj_ * (FX / 2);
                const int CI = (gx0 + HALO) / 2 + ci, CJ = (gy0 + HALO) / 2 + cj_;
                if (CI < cL.n[0] && CJ < cL.n[1]) {
                    T sum = T(0);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int li = HALO + 2 * ci + (q & 1), lj = HALO + 2 * cj_ + (q >> 1);
                        const T xc = t.X(li, lj, G);
                        sum += t.B(li, lj, G) - xc - t.W0(li, lj, G) * (xc - t.X(li - 1, lj, G)) -
                               t.W0(li + 1, lj, G) * (xc - t.X(li + 1, lj, G)) -
                               t.W1(li, lj, G) * (xc - t.X(li, lj - 1, G)) -
                               t.W1(li, lj + 1, G) * (xc - t.X(li, lj + 1, G));
                    }
                    cb[CI + (long)cL.n[0] * CJ] = sum * T(0.25);
                }
            }
            __syncthreads();                           // t is rewritten by the next tile
        }
        if (!more) break;
        k = kn;
        cd = nd;
        cc = nc;
        cgx = ngx;
        cgy = ngy;
        cact = nact;
    }
}

template <typename T, int NU, int WIDE, int FY, int NT>
__global__ void __launch_bounds__(NT)
k_up2(const LevelDesc* __restrict__ L, const GridState* __restrict__ S, JobList jl) {
    constexpr int HALO = 2 * NU;
    constexpr int FX = fused_fx(HALO, WIDE);
    using Tl = Tile2<T, FX + 2 * HALO, FY + 2 * HALO>;
    constexpr int NE = (Tl::W * Tl::H + NT - 1) / NT;
    __shared__ Tl t;
    const XcdOrder order(jl.total);
    int k = order.first();
    if (!order.more(k)) return;
    // the down pass's iterate plus the prolonged coarse correction
    Tile2Job cj = tile2_job<FX, FY, HALO>(L, S, jl, order.tile(k));
    Tile2Regs<T, NE> v;
    tile2_fetch<T, Tl, NE, NT>(v, *cj.d, as_global(Arr<T>::xs(*cj.d)), cj.gx0, cj.gy0, true,
                           as_global(Arr<T>::x(*cj.c)), cj.c->n[0]);
    const LevelDesc* cd = cj.d;
    int cgx = cj.gx0, cgy = cj.gy0, cact = cj.act ? 1 : 0;
    while (true) {
        if (cact) tile2_put<T, Tl, NE, NT>(t, v, cgx, cgy, true);
        const int kn = k + order.per;
        const bool more = order.more(kn);
        const LevelDesc* nd = cd;
        int ngx = cgx, ngy = cgy, nact = cact;
        if (more) {
            const Tile2Job nj = tile2_job<FX, FY, HALO>(L, S, jl, order.tile(kn));
            nd = nj.d;
            ngx = nj.gx0;
            ngy = nj.gy0;
            nact = nj.act ? 1 : 0;
            tile2_fetch<T, Tl, NE, NT>(v, *nd, as_global(Arr<T>::xs(*nd)), ngx, ngy, true,
                                   as_global(Arr<T>::x(*nj.c)), nj.c->n[0]);
        }
        if (cact) {
            const LevelDesc& d = *cd;
            const int gx0 = cgx, gy0 = cgy;
            const int G = (gx0 + gy0) & 1;
            for (int it = 0; it < NU; ++it) {
                tile2_half_sweep<NT>(t, G, 1, 2 * it + 1);
                tile2_half_sweep<NT>(t, G, 0, 2 * it + 2);
            }
            const gptr<T> xo = as_global(Arr<T>::x(d));
            for (int e = threadIdx.x; e < FX * FY; e += NT) {
                const int lj = e / FX, li = e - lj * FX;
                const int gi = gx0 + HALO + li, gj = gy0 + HALO + lj;
                if (gi < d.n[0] && gj < d.n[1]) xo[gi + (long)d.n[0] * gj] = t.X(HALO + li, HALO + lj, G);
            }
            __syncthreads();
        }
        if (!more) break;
        k = kn;
        cd = nd;
        cgx = ngx;
        cgy = ngy;
        cact = nact;
    }
}

// Calls f(std::integral_constant<int, 0>{}) .. f(std::integral_constant<int, N - 1>{}) in order.
template <int N, typename F>
__device__ __forceinline__ void unroll(F&& f) {
    if constexpr (N > 0) {
        unroll<N - 1>(f);
        f(std::integral_constant<int, N - 1>{});
    }
}

// Value of v on lane l - 1 (LEFT) or l + 1 of the wavefront, 0 on lane 0 / 63: DPP
// whole-wavefront shifts (every lane must be active).
__device__ __forceinline__ uint32_t lane_shift(uint32_t v, bool left) {
    return left ? __builtin_amdgcn_update_dpp(0u, v, 0x138, 0xF, 0xF, true)     // wave_shr:1
                : __builtin_amdgcn_update_dpp(0u, v, 0x130, 0xF, 0xF, true);    // wave_shl:1
}
template <bool LEFT>
__device__ __forceinline__ float lane_nb(float v) {
    return __builtin_bit_cast(float, lane_shift(__builtin_bit_cast(uint32_t, v), LEFT));
}
template <bool LEFT>
__device__ __forceinline__ double lane_nb(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint64_t lo = lane_shift((uint32_t)u, LEFT), hi = lane_shift((uint32_t)(u >> 32), LEFT);
    return __builtin_bit_cast(double, (hi << 32) | lo);
}

// ---------------------------------------------------------------------------
// Row-marching fused 2D level kernels for levels with many windows.  One wavefront
// owns a window of kMarchNP x positions (FX interior columns and an even halo of H
// on each side), two adjacent columns a lane, and fz rows, and marches along y with
// all 2 nu half sweeps of the pass in flight at once: at step zt, half sweep k
// (k = 1 .. 2 nu, in order) updates row zt - k.  Row zt - k + 1 went through half
// sweep k - 1 earlier in the same step and row zt - k - 1 through half sweep k one
// step earlier, so every cell sees its neighbours exactly as a global red-black
// sweep leaves them.  In a step every half sweep updates the same one of a lane's two
// columns (the colour flips with both k and the row), the even one on every other
// step, so no lane idles: the y-neighbours are the lane's own registers (a ring of
// rows), the x-neighbours its other column and, across the pair boundary, the
// neighbouring lane's, taken by a DPP lane shift.  No LDS and no barrier.  Each cell
// update and residual keeps the operand order of the LDS tile kernels (k_down2 /
// k_up2), which gives bitwise equal results.  Rows and positions near the window's
// edge take wrong neighbours (zero rows before the march, the shifted-in zero at the
// wavefront's ends); that error moves inward one position or row per half sweep and
// stays in the halo.  Cells outside the level hold x = b = 0 and zero faces, and
// the level's boundary faces are zero, so they stay zero.  The down pass (halo 2 nu
// + 2) starts from zero or the stored iterate, writes the smoothed iterate to xs and
// averages the final residual of each row pair onto the coarse right-hand side (the
// residual of row r one step after its last update; a lane's two columns are the
// two fine columns of one coarse cell); the up pass (halo 2 nu) starts from xs plus
// the prolonged coarse correction and writes x; on level 0 under CG (FP64, b = r) it
// can also sum b . x over the window's interior (each lane's rows in turn, even
// column first, then a butterfly) into one partial of r . z.  A window recomputes no
// rows, only the x halo and its march's halo rows.
// ---------------------------------------------------------------------------
template <typename T, int NU, bool DOWN, bool LOADX>
__global__ void __launch_bounds__(64)
k_march2(const LevelDesc* __restrict__ L, const GridState* __restrict__ S, JobList jl, int fz, int rz) {
    constexpr int NP = kMarchNP;
    constexpr int SS = 2 * NU;                       // half sweeps of the pass
    constexpr int H = march_halo(NU, DOWN);
    constexpr int FX = march_fx(NU, DOWN);
    constexpr int PF = 2;                            // rows loaded ahead
    constexpr int NB = SS + PF + 4;                  // register ring: rows zt + PF .. zt - SS - 2 (and one spare)
    static_assert(H % 2 == 0 && FX % 2 == 0 && NB % 2 == 0, "pairs of columns, steps of known parity");
    using V2 = T __attribute__((ext_vector_type(2)));
    const int l = threadIdx.x;
    const XcdOrder order(jl.total);
    for (int kk = order.first(); order.more(kk); kk += order.per) {
        const int tt = order.tile(kk);
        const int jb = find_job(jl.prefix, jl.njobs, tt);
        const LevelDesc& d = L[job_level(jl, jb)];
        if (!S[d.sidx].active) continue;                              // uniform per window
        const int lt = tt - job_start(jl, jb);
        const int nx = d.n[0], ny = d.n[1];                           // even: the level has a coarse one
        const int tx_n = (nx + FX - 1) / FX;
        const int gx0 = (lt % tx_n) * FX - H;                         // even
        const int z0 = (lt / tx_n) * fz, z1 = min(z0 + fz, ny);
        const int zs = z0 - H;                                        // even: step zt has zt's parity
        const int ze = z1 + SS + (DOWN ? 1 : 0);
        const int ge = gx0 + 2 * l;                                   // the lane's even column
        const bool inx = ge >= 0 && ge < nx;                          // both columns in the level, or neither
        const int pc = min(max(ge, 0), nx - 2);
        const bool own = inx && l >= H / 2 && l < (NP - H) / 2;       // an interior pair
        const gptr<T> xin = as_global(DOWN ? Arr<T>::x(d) : Arr<T>::xs(d));
        const gptr<T> xout = as_global(DOWN ? Arr<T>::xs(d) : Arr<T>::x(d));
        const gptr<T> bg = as_global(Arr<T>::b(d));
        const gptr<T> w0g = as_global(Arr<T>::w(d, 0));
        const gptr<T> w1g = as_global(Arr<T>::w(d, 1));
        const LevelDesc& cL = L[d.coarse];
        const gptr<T> cxg = as_global(Arr<T>::x(cL));
        const gptr<T> cbg = as_global(Arr<T>::b(cL));
        const int cn0 = cL.n[0], cn1 = cL.n[1];
        T Xe[NB], Xo[NB], Be[NB], Bo[NB], W0e[NB], W0o[NB], W1e[NB], W1o[NB], C[NB];
        unroll<NB>([&](auto Qc) {
            constexpr int q = decltype(Qc)::value;
            Xe[q] = Xo[q] = Be[q] = Bo[q] = W0e[q] = W0o[q] = W1e[q] = W1o[q] = C[q] = T(0);
        });
        // loads of row gj (clamped) at the lane's two columns (clamped), masked when
        // committed; issued on every step whatever the row, so that the compiler's wait
        // before a row's first use leaves the next row's loads in flight
        auto load = [&](auto Sl, int gj) {
            constexpr int q = decltype(Sl)::value;
            const int jc = min(max(min(gj, ze - 1), 0), ny - 1);   // rows past the march: its last (cached)
            const long idx = pc + (long)nx * jc;
            const V2 b2 = *(const gptr<V2>)(bg + idx);
            const V2 u2 = *(const gptr<V2>)(w0g + idx);
            const V2 v2 = *(const gptr<V2>)(w1g + idx);
            Be[q] = b2.x;
            Bo[q] = b2.y;
            W0e[q] = u2.x;
            W0o[q] = u2.y;
            W1e[q] = v2.x;
            W1o[q] = v2.y;
            if constexpr (!DOWN) C[q] = cxg[(pc >> 1) + (long)cn0 * (jc >> 1)];
            if constexpr (LOADX) {
                const V2 x2 = *(const gptr<V2>)(xin + idx);
                Xe[q] = x2.x;
                Xo[q] = x2.y;
            } else {
                Xe[q] = Xo[q] = T(0);
            }
        };
        T acc = T(0);                                 // the lane's coarse cell of a row pair
        double rzacc = 0.0;                           // up pass, rz: the lane's b . x
        auto step = [&](auto Qc, int zt) {
            constexpr int q = decltype(Qc)::value;   // register slot of row zt; zt = q (mod 2)
            // the column that updates: down passes take colour 0 first, so cell (i, r) of
            // half sweep k updates when i + r + k is odd, i.e. i + zt is odd; up passes
            // take colour 1 first (i + zt even)
            constexpr bool AE = DOWN ? (q & 1) != 0 : (q & 1) == 0;
            {
                // row zt enters the window (zero outside the level)
                const bool in = inx && zt >= 0 && zt < ny;
                T xe = Xe[q], xo = Xo[q];
                if constexpr (!DOWN) {
                    xe += C[q];
                    xo += C[q];
                }
                Xe[q] = in ? xe : T(0);
                Xo[q] = in ? xo : T(0);
                Be[q] = in ? Be[q] : T(0);
                Bo[q] = in ? Bo[q] : T(0);
                W0e[q] = in ? W0e[q] : T(0);
                W0o[q] = in ? W0o[q] : T(0);
                W1e[q] = in ? W1e[q] : T(0);
                W1o[q] = in ? W1o[q] : T(0);
            }
            load(std::integral_constant<int, (q + PF) % NB>{}, zt + PF);
            unroll<SS>([&](auto Kc) {
                constexpr int k = decltype(Kc)::value + 1;
                constexpr int qk = (q + NB - k) % NB, qd = (q + NB - k - 1) % NB, qu = (q + NB - k + 1) % NB;
                if constexpr (AE) {
                    const T xl = lane_nb<true>(Xo[qk]);
                    const T wl = W0e[qk], wr = W0o[qk], wd = W1e[qk], wu = W1e[qu];
                    const T s = Be[qk] + wl * xl + wr * Xo[qk] + wd * Xe[qd] + wu * Xe[qu];
                    Xe[qk] = s / (T(1) + wl + wr + wd + wu);
                } else {
                    const T xr = lane_nb<false>(Xe[qk]);
                    const T wl = W0o[qk], wr = lane_nb<false>(W0e[qk]), wd = W1o[qk], wu = W1o[qu];
                    const T s = Bo[qk] + wl * Xe[qk] + wr * xr + wd * Xo[qd] + wu * Xo[qu];
                    Xo[qk] = s / (T(1) + wl + wr + wd + wu);
                }
            });
            // row zt - SS is final
            {
                constexpr int qf = (q + NB - SS) % NB;
                const int rf = zt - SS;
                if (own && rf >= z0 && rf < z1) {
                    V2 o2;
                    o2.x = Xe[qf];
                    o2.y = Xo[qf];
                    *(gptr<V2>)(xout + ge + (long)nx * rf) = o2;
                    if constexpr (!DOWN && std::is_same_v<T, double>) {
                        if (rz) {
                            rzacc += Be[qf] * Xe[qf];
                            rzacc += Bo[qf] * Xo[qf];
                        }
                    }
                }
            }
            if constexpr (DOWN) {
                // the residual of row zt - SS - 1 (final, as are its neighbours) at both
                // columns, added into the coarse cell in the tile kernels' order
                constexpr int q3 = (q + NB - SS - 1) % NB, q2 = (q + NB - SS) % NB, q4 = (q + NB - SS - 2) % NB;
                const T xe = Xe[q3], xo = Xo[q3];
                const T xl = lane_nb<true>(xo), xr = lane_nb<false>(xe), wr = lane_nb<false>(W0e[q3]);
                const T re = Be[q3] - xe - W0e[q3] * (xe - xl) - W0o[q3] * (xe - xo) - W1e[q3] * (xe - Xe[q4]) -
                             W1e[q2] * (xe - Xe[q2]);
                const T ro = Bo[q3] - xo - W0o[q3] * (xo - xe) - wr * (xo - xr) - W1o[q3] * (xo - Xo[q4]) -
                             W1o[q2] * (xo - Xo[q2]);
                const int rr = zt - SS - 1;
                if (own && rr >= z0 && rr < z1) {
                    if (((rr - z0) & 1) == 0) acc = T(0);
                    acc += re;
                    acc += ro;
                    if ((rr - z0) & 1) {
                        const int CI = ge >> 1, CJ = rr >> 1;
                        if (CI < cn0 && CJ < cn1) cbg[CI + (long)cn0 * CJ] = acc * T(0.25);
                    }
                }
            }
        };
        static_assert(PF == 2, "the prologue below loads two rows");
        load(std::integral_constant<int, 0>{}, zs);
        load(std::integral_constant<int, 1>{}, zs + 1);
        // whole rounds of NB steps without a branch between them, then the last steps
        int zb = zs;
        for (; zb + NB <= ze; zb += NB) unroll<NB>([&](auto Qc) { step(Qc, zb + decltype(Qc)::value); });
        unroll<NB - 1>([&](auto Qc) {
            if (zb + decltype(Qc)::value < ze) step(Qc, zb + decltype(Qc)::value);
        });
        if constexpr (!DOWN && std::is_same_v<T, double>) {
            if (rz) {
                // fixed-order butterfly: every lane ends with the same sum
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) rzacc += __shfl_xor(rzacc, off, 64);
                if (l == 0) d.part[lt] = rzacc;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Fused 3D sweeps.  One launch runs one whole red-black sweep (colour c0, then
// 1-c0) over blocks of FX x FY interior columns and fz planes.  A block of
// PX x PY threads owns a window of as many xy positions (the interior plus a
// halo of H positions), one position per thread, and marches along z.  Each thread
// keeps its own position's iterate and operator (b and the three lower faces) for
// the planes in flight in registers; only the iterate and the x / y lower faces go
// through LDS, in a ring of plane slots, for the in-plane neighbours.  At step zt:
//   A  store plane zt (loaded two steps earlier) to its slot, load plane zt + 2
//   -- barrier --
//   C  colour c0 on plane zt - 1 (on HC rings around the interior): the in-plane
//      neighbours from the slot, the z-neighbours are the thread's own registers
//      (zt - 2 not yet updated, zt as loaded)
//   D  colour 1 - c0 on plane zt - 2 (HC - 1 rings): the z-neighbours zt - 3 and
//      zt - 1 are again the thread's own registers, both updated by C; the position
//      that updates in D is the one that updated in C (the colour flips with z)
//   plane zt - 2 is final on the interior and is written out.
// The halo recomputes exactly what the neighbouring blocks compute.  Restricting
// sweeps (H = 3, HC = 2) also store D's results to the slot and form the residual of
// the final iterate on plane zt - 3 into an LDS plane; after a second barrier one
// thread per coarse cell adds its eight children, two planes in turn, and writes the
// coarse right-hand side (and a zero coarse iterate).  Modes:
//   SW_LOAD      start from the stored iterate
//   SW_ZERO      start from zero (nothing loaded)
//   SW_*_RESTR   also restrict the final residual onto the coarse level
//   SW_PROLONG   add the piecewise-constant prolongation of the coarse correction to
//                the iterate as it is loaded
// Each cell update and residual uses the operand order of the per-colour kernels
// (k_smooth, residual_at, k_restrict), so both paths give bitwise equal results.
// A sweep never writes the array it reads.  Cells outside the level hold x = b = 0
// and zero faces, which leaves every sum exact.
// ---------------------------------------------------------------------------
enum SweepMode : int { SW_LOAD = 0, SW_ZERO = 1, SW_LOAD_RESTR = 2, SW_ZERO_RESTR = 3, SW_PROLONG = 4 };

template <int MODE>
struct Sweep3Mode {
    static constexpr bool RESTR = MODE == SW_LOAD_RESTR || MODE == SW_ZERO_RESTR;
    static constexpr bool LOADX = MODE == SW_LOAD || MODE == SW_LOAD_RESTR || MODE == SW_PROLONG;
    static constexpr bool PROL = MODE == SW_PROLONG;
    static constexpr int H = sweep3_halo(RESTR);    // halo positions of the window
    static constexpr int HC = RESTR ? 2 : 1;         // rings of the first colour around the interior
    static constexpr int HX = HC + 1;                // rings whose iterate is read
    static constexpr int FX = sweep3_fx(RESTR), FY = sweep3_fy(RESTR);
    static constexpr int PX = sweep3_px(RESTR), PY = sweep3_py(RESTR);
    static constexpr int R = RESTR ? 6 : 4;          // LDS plane slots
};

template <typename T, int R, int PX, int PY, bool RESTR>
struct Sweep3Lds {
    T x[R][PY][PX];
    T w0[R][PY][PX];
    T w1[R][PY][PX];
    T res[RESTR ? 2 : 1][RESTR ? PY : 1][PX];   // residual planes of two steps
};

template <typename T, int MODE>
__global__ void __launch_bounds__(1024)
k_sweep3(const LevelDesc* __restrict__ L, const GridState* __restrict__ S, JobList jl, int c0, int from_xs,
         int fz, int rz) {
    using M = Sweep3Mode<MODE>;
    constexpr int H = M::H, HC = M::HC, HX = M::HX, FX = M::FX, FY = M::FY, R = M::R;
    constexpr int PX = M::PX, PY = M::PY;
    // planes are loaded PF steps ahead; the registers hold planes zt - 3 .. zt + PF
    // (three steps ahead measured no faster than two)
    constexpr int PF = 2, NB = PF + 4;
    static_assert(HX == H, "every window position is read by a neighbour");
    __shared__ Sweep3Lds<T, R, PX, PY, M::RESTR> t;
    // the last up sweep of level 0 under FP64 CG (rz): each thread's b . x, summed in a
    // fixed order into one partial of r . z per window
    constexpr bool RZ = MODE == SW_LOAD && std::is_same_v<T, double>;
    __shared__ double shrz[RZ ? PX * PY : 1];
    const int lx = threadIdx.x % PX, ly = threadIdx.x / PX;
    // rings outside the interior: o >= H is interior; o >= H - HC takes the first colour,
    // o >= H - HC + 1 the second
    const int o = min(min(lx, PX - 1 - lx), min(ly, PY - 1 - ly));
    const bool in_c = o >= H - HC, in_d = o >= H - HC + 1, in_r = o >= H;
    const XcdOrder order(jl.total);
    for (int k = order.first(); order.more(k); k += order.per) {
        const int tt = order.tile(k);
        const int jb = find_job(jl.prefix, jl.njobs, tt);
        const LevelDesc& d = L[job_level(jl, jb)];
        if (!S[d.sidx].active) continue;
        const int lt = tt - job_start(jl, jb);
        const int n0 = d.n[0], n1 = d.n[1], n2 = d.n[2];
        const int tx_n = (n0 + FX - 1) / FX, ty_n = (n1 + FY - 1) / FY;
        const int tx = lt % tx_n, rest = lt / tx_n;
        const int gx0 = tx * FX - H, gy0 = (rest % ty_n) * FY - H;
        const int z0 = (rest / ty_n) * fz, z1 = min(z0 + fz, n2);
        // planes stored, and steps: [zs, ze); a restricting sweep takes one step more, in
        // which the owners add the last residual plane
        const int zs = z0 - HX, ze = z1 + HX + (M::RESTR ? 1 : 0);
        const int gx = gx0 + lx, gy = gy0 + ly;
        const bool in_xy = gx >= 0 && gx < n0 && gy >= 0 && gy < n1;
        const long sy = n0, sz = (long)n0 * n1;
        const long cxy = min(max(gx, 0), n0 - 1) + (long)min(max(gy, 0), n1 - 1) * sy;   // clamped column
        const gptr<T> xin = as_global(M::LOADX ? (from_xs ? Arr<T>::xs(d) : Arr<T>::x(d)) : Arr<T>::x(d));
        const gptr<T> xout = as_global(from_xs ? Arr<T>::x(d) : Arr<T>::xs(d));
        const gptr<T> bg = as_global(Arr<T>::b(d));
        const gptr<T> w0g = as_global(Arr<T>::w(d, 0));
        const gptr<T> w1g = as_global(Arr<T>::w(d, 1));
        const gptr<T> w2g = as_global(Arr<T>::w(d, 2));
        gptr<T> cx = nullptr, cb = nullptr;
        int cn0 = 0, cn1 = 0;
        long ccol = 0;
        if (M::PROL || M::RESTR) {
            const LevelDesc& cL = L[d.coarse];
            cx = as_global(Arr<T>::x(cL));
            cb = as_global(Arr<T>::b(cL));
            cn0 = cL.n[0];
            cn1 = cL.n[1];
            ccol = (min(max(gx, 0), n0 - 1) >> 1) + (long)cn0 * (min(max(gy, 0), n1 - 1) >> 1);
        }
        // the thread's planes in flight: iterate, b, lower faces (and the coarse correction)
        T X[NB], B[NB], W0[NB], W1[NB], W2[NB], CC[NB];
        // branch-free loads of plane gk at the clamped column (masked when stored)
        auto load = [&](auto Sl, int gk) {
            constexpr int q = decltype(Sl)::value;
            const int kc = min(max(min(gk, z1 + HX - 1), 0), n2 - 1);   // planes past the window: its last (cached)
            const long idx = cxy + kc * sz;
            if (M::LOADX) X[q] = xin[idx];
            B[q] = bg[idx];
            W0[q] = w0g[idx];
            W1[q] = w1g[idx];
            W2[q] = w2g[idx];
            if (M::PROL) CC[q] = cx[ccol + (long)cn0 * cn1 * (kc >> 1)];
        };
        T racc = T(0);
        double rzacc = 0.0;
        // coarse cell of the restriction owners: thread e < (FX/2)(FY/2)
        const int rci = threadIdx.x % (FX / 2), rcj = threadIdx.x / (FX / 2);
        const bool rown = M::RESTR && threadIdx.x < (FX / 2) * (FY / 2) && (gx0 + H) / 2 + rci < cn0 &&
                          (gy0 + H) / 2 + rcj < cn1;
        auto step = [&](auto Sc, int zt) {
            constexpr int q = decltype(Sc)::value;               // register slot of plane zt
            constexpr int q1 = (q + NB - 1) % NB, q2 = (q + NB - 2) % NB, q3 = (q + NB - 3) % NB;
            const int s0 = (zt - zs) % R;
            // A: plane zt enters the window (zero outside the level)
            {
                const bool in = in_xy && zt >= 0 && zt < n2;
                T xv = M::LOADX ? X[q] : T(0);
                if (M::PROL) xv += CC[q];
                X[q] = in ? xv : T(0);
                B[q] = in ? B[q] : T(0);
                W0[q] = in ? W0[q] : T(0);
                W1[q] = in ? W1[q] : T(0);
                W2[q] = in ? W2[q] : T(0);
                t.x[s0][ly][lx] = X[q];
                t.w0[s0][ly][lx] = W0[q];
                t.w1[s0][ly][lx] = W1[q];
            }
            // issued on every step (the plane is clamped): a conditional load makes the
            // compiler's wait before a plane's first use cover the next plane's loads too
            load(std::integral_constant<int, (q + PF) % NB>{}, zt + PF);
            __syncthreads();
            // C: colour c0 on plane zt - 1
            const int p1 = zt - 1;
            const bool act = ((gx + gy + p1) & 1) == c0;          // this position's colour on p1
            if (p1 >= z0 - HC && p1 < z1 + HC && p1 >= 0 && p1 < n2 && in_c && in_xy && act) {
                const int s1 = (p1 - zs) % R;
                T sm = B[q1], dg = T(1);
                T w = W0[q1];
                sm += w * t.x[s1][ly][lx - 1]; dg += w;
                w = t.w0[s1][ly][lx + 1];
                sm += w * t.x[s1][ly][lx + 1]; dg += w;
                w = W1[q1];
                sm += w * t.x[s1][ly - 1][lx]; dg += w;
                w = t.w1[s1][ly + 1][lx];
                sm += w * t.x[s1][ly + 1][lx]; dg += w;
                w = W2[q1];
                sm += w * X[q2]; dg += w;
                w = W2[q];
                sm += w * X[q]; dg += w;
                X[q1] = sm / dg;
                t.x[s1][ly][lx] = X[q1];
            }
            // D: colour 1 - c0 on plane zt - 2 (the same positions as C)
            const int p2 = zt - 2;
            if (p2 >= z0 - (HC - 1) && p2 < z1 + (HC - 1) && p2 >= 0 && p2 < n2 && in_d && in_xy && act) {
                const int s2 = (p2 - zs) % R;
                T sm = B[q2], dg = T(1);
                T w = W0[q2];
                sm += w * t.x[s2][ly][lx - 1]; dg += w;
                w = t.w0[s2][ly][lx + 1];
                sm += w * t.x[s2][ly][lx + 1]; dg += w;
                w = W1[q2];
                sm += w * t.x[s2][ly - 1][lx]; dg += w;
                w = t.w1[s2][ly + 1][lx];
                sm += w * t.x[s2][ly + 1][lx]; dg += w;
                w = W2[q2];
                sm += w * X[q3]; dg += w;
                w = W2[q1];
                sm += w * X[q1]; dg += w;
                X[q2] = sm / dg;
                if (M::RESTR) t.x[s2][ly][lx] = X[q2];
            }
            // plane zt - 2 is final on the interior
            if (p2 >= z0 && p2 < z1 && in_r && in_xy) {
                xout[cxy + p2 * sz] = X[q2];
                if constexpr (RZ) {
                    if (rz) rzacc += B[q2] * X[q2];
                }
            }
            if (M::RESTR) {
                // the owners add the residual plane formed one step earlier (this step's
                // barrier ordered its stores before these loads)
                const int pp = zt - 4;
                if (pp >= z0 && pp < z1 && rown) {
                    const int ax = H + 2 * rci, ay = H + 2 * rcj, sr = (pp - zs) & 1;
                    if (((pp - z0) & 1) == 0) racc = T(0);
                    racc += t.res[sr][ay][ax];
                    racc += t.res[sr][ay][ax + 1];
                    racc += t.res[sr][ay + 1][ax];
                    racc += t.res[sr][ay + 1][ax + 1];
                    if ((pp - z0) & 1) {
                        // the coarse level's sweeps start from zero (per-colour kernels read it)
                        const long cidx = (gx0 + H) / 2 + rci + (long)cn0 * ((gy0 + H) / 2 + rcj +
                                                                          (long)cn1 * (pp >> 1));
                        cb[cidx] = racc * T(0.125);
                        cx[cidx] = T(0);
                    }
                }
                // residual of the final iterate on plane zt - 3 (its in-plane neighbours and the
                // plane below from the slots, the plane above from the registers), into the
                // residual plane of this step's parity
                const int p3 = zt - 3;
                if (p3 >= z0 && p3 < z1) {                             // uniform
                    T r = T(0);
                    if (in_r && in_xy) {
                        const int s3 = (p3 - zs) % R, s4 = (p3 - 1 - zs) % R;
                        const T xc = X[q3];
                        r = B[q3] - xc;
                        r -= W0[q3] * (xc - t.x[s3][ly][lx - 1]);
                        r -= t.w0[s3][ly][lx + 1] * (xc - t.x[s3][ly][lx + 1]);
                        r -= W1[q3] * (xc - t.x[s3][ly - 1][lx]);
                        r -= t.w1[s3][ly + 1][lx] * (xc - t.x[s3][ly + 1][lx]);
                        r -= W2[q3] * (xc - t.x[s4][ly][lx]);
                        r -= W2[q2] * (xc - X[q2]);
                    }
                    t.res[M::RESTR ? (p3 - zs) & 1 : 0][M::RESTR ? ly : 0][lx] = r;
                }
            }
        };
        static_assert(PF == 2, "the prologue below loads two planes");
        load(std::integral_constant<int, 0>{}, zs);
        load(std::integral_constant<int, 1>{}, zs + 1);
        // whole rounds of NB steps without a branch between them, then the last steps
        int zb = zs;
        for (; zb + NB <= ze; zb += NB) unroll<NB>([&](auto Qc) { step(Qc, zb + decltype(Qc)::value); });
        unroll<NB - 1>([&](auto Qc) {
            if (zb + decltype(Qc)::value < ze) step(Qc, zb + decltype(Qc)::value);
        });
        __syncthreads();                                       // the slots are reused by the next tile
        if constexpr (RZ) {
            if (rz) {
                // thread order: lane l of wave 0 sums threads 16 l .. 16 l + 15, then the wave
                constexpr int NTH = PX * PY, PER = (NTH + 63) / 64;
                shrz[threadIdx.x] = rzacc;
                __syncthreads();
                if (threadIdx.x < 64) {
                    double v = 0.0;
                    for (int i = 0; i < PER; ++i) {
                        const int th = threadIdx.x * PER + i;
                        if (th < NTH) v += shrz[th];
                    }
                    v = wave_sum(v);
                    if (threadIdx.x == 0) d.part[lt] = v;
                }
                __syncthreads();                               // shrz is reused by the next tile
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Tail: one workgroup per grid runs the whole V-cycle below a level T out of
// LDS -- every tail level's x, b and face weights, plus the coarsest CG's
// search direction -- so the coarse levels cost one launch instead of a few
// per level.  The restriction from level T-1 left b_T in global memory and the
// prolongation to level T-1 reads the correction x_T back from global memory.
// ---------------------------------------------------------------------------
// Geometry of one tail level and the LDS offsets (in elements from the start of
// the tail's dynamic LDS) of its arrays.  The arrays are addressed as that base
// plus an offset in the kernel itself, so the compiler sees LDS pointers and
// emits ds_* instructions (pointers read back from memory would be generic and
// need flat instructions, which also wait on the vector memory counter).
struct TailGeom {
    int32_t n[3];
    int32_t ncell;
    int32_t hx;          // colour cells per row: ceil(nx / 2)
    float rhx;           // 1 / hx
    float rny;           // 1 / ny
    float rnx;           // 1 / nx
    int32_t ox, ob, ow[3];
    int32_t oa, has_a;   // Dirichlet ghost couplings (plans with Dirichlet faces)
    int32_t pm;          // neighbour mask (nb_mask): periodic axes, continuous faces
};

template <typename T>
struct TailLevel {
    int32_t n[3];
    int32_t ncell;
    int32_t hx;
    float rhx;
    float rny;
    float rnx;
    T* x;
    T* b;
    T* w[3];
    T* a;
    int32_t has_a;
    int32_t pm;
};

template <typename T>
__device__ __forceinline__ TailLevel<T> tl_at(const TailGeom& g, T* base) {
    TailLevel<T> t;
    t.n[0] = g.n[0]; t.n[1] = g.n[1]; t.n[2] = g.n[2];
    t.ncell = g.ncell;
    t.hx = g.hx;
    t.rhx = g.rhx;
    t.rny = g.rny;
    t.rnx = g.rnx;
    t.x = base + g.ox;
    t.b = base + g.ob;
    for (int a = 0; a < 3; ++a) t.w[a] = base + g.ow[a];
    t.a = base + g.oa;
    t.has_a = g.has_a;
    t.pm = g.pm;
    return t;
}
constexpr int kMaxTail = 16;

// q / d for 0 <= q < 2^20 and d <= 2^10 through a float reciprocal: (q + 1/2)/d
// lies at least 1/(2d) from an integer, far beyond the float rounding error.
__device__ __forceinline__ int fdiv(int q, float rd) { return (int)(((float)q + 0.5f) * rd); }

template <int DIM, typename T>
__device__ __forceinline__ void tl_coords(const TailLevel<T>& lv, int c, int& i, int& j, int& k) {
    const int r = fdiv(c, lv.rnx);
    i = c - r * lv.n[0];
    if (DIM == 3) {
        k = fdiv(r, lv.rny);
        j = r - k * lv.n[1];
    } else {
        j = r;
        k = 0;
    }
}

// Levels are passed by value: a copy in registers, since the LDS stores of a phase
// could otherwise alias the descriptor table in LDS and force its re-reading.
template <int DIM, typename T, bool BC, int NT>
__device__ __forceinline__ void tl_half_sweep(const TailLevel<T> lv, int color) {
    const int pmask = BC ? lv.pm : 0;
    const int sy = lv.n[0], sz = lv.n[0] * lv.n[1];
    const int rows = lv.n[1] * lv.n[2];
    for (int m = threadIdx.x; m < rows * lv.hx; m += NT) {
        const int r = fdiv(m, lv.rhx);
        int j = r, k = 0;
        if (DIM == 3) {
            k = fdiv(r, lv.rny);
            j = r - k * lv.n[1];
        }
        const int i = 2 * (m - r * lv.hx) + ((j + k + color) & 1);
        if (i >= lv.n[0]) continue;
        const long c = i + j * sy + k * sz;
        T s = lv.b[c], dg = T(1);
        T wl, xl, wr, xr, wd, xd, wu, xu;
        nb_lo(lv.w[0], lv.x, c, i, lv.n[0], 1, pmask, 0, wl, xl);
        nb_hi(lv.w[0], lv.x, c, i, lv.n[0], 1, pmask, 0, wr, xr);
        nb_lo(lv.w[1], lv.x, c, j, lv.n[1], sy, pmask, 1, wd, xd);
        nb_hi(lv.w[1], lv.x, c, j, lv.n[1], sy, pmask, 1, wu, xu);
        s += wl * xl; dg += wl;
        s += wr * xr; dg += wr;
        s += wd * xd; dg += wd;
        s += wu * xu; dg += wu;
        if (DIM == 3) {
            T wb, xb, wf, xf;
            nb_lo(lv.w[2], lv.x, c, k, lv.n[2], sz, pmask, 2, wb, xb);
            nb_hi(lv.w[2], lv.x, c, k, lv.n[2], sz, pmask, 2, wf, xf);
            s += wb * xb; dg += wb;
            s += wf * xf; dg += wf;
        }
        if (BC && lv.has_a) dg += lv.a[c];
        lv.x[c] = s / dg;
    }
    group_sync<NT>();
}

// The V-cycle of the tail levels from m0 down (level m0's b set, its x zero or warm),
// run by NT threads: the workgroup, or one wavefront for small levels.
template <int DIM, typename T, bool BC, int NT, int CPT>
__device__ __forceinline__ void tail_vcycle(const TailGeom* tl, T* sbase, int m0, int nl, int nu1, int nu2, T* p_sh,
                                            double* red) {
    // descend
    for (int m = m0; m + 1 < nl; ++m) {
        const TailLevel<T> f = tl_at(tl[m], sbase);
        const TailLevel<T> cT = tl_at(tl[m + 1], sbase);
        for (int it = 0; it < nu1; ++it) {
            tl_half_sweep<DIM, T, BC, NT>(f, 0);
            tl_half_sweep<DIM, T, BC, NT>(f, 1);
        }
        for (int c = threadIdx.x; c < cT.ncell; c += NT) {
            int I, J, K;
            tl_coords<DIM, T>(cT, c, I, J, K);
            T sum = T(0);
#pragma unroll
            for (int q = 0; q < (1 << DIM); ++q)
                sum += residual_at<DIM, T>(f.x, f.b, f.w[0], f.w[1], f.w[2], f.n, 2 * I + (q & 1),
                                           2 * J + ((q >> 1) & 1), DIM == 3 ? 2 * K + (q >> 2) : 0, f.a,
                                           BC && f.has_a != 0, BC ? f.pm : 0);
            cT.b[c] = sum * T(DIM == 3 ? 0.125 : 0.25);
            cT.x[c] = T(0);
        }
        group_sync<NT>();
    }
    // coarsest: CG from the current x (zero unless the grid has a single level)
    {
        const TailLevel<T> cT = tl_at(tl[nl - 1], sbase);
        block_cg<DIM, T, NT, CPT>(cT.n, cT.w[0], cT.w[1], cT.w[2], cT.b, cT.x, true, p_sh, red, cT.a,
                                  BC && cT.has_a != 0, BC ? cT.pm : 0);
    }
    // ascend
    for (int m = nl - 2; m >= m0; --m) {
        const TailLevel<T> f = tl_at(tl[m], sbase);
        const TailLevel<T> cT = tl_at(tl[m + 1], sbase);
        for (int c = threadIdx.x; c < f.ncell; c += NT) {
            int i, j, k;
            tl_coords<DIM, T>(f, c, i, j, k);
            f.x[c] += cT.x[(i >> 1) + cT.n[0] * ((j >> 1) + cT.n[1] * (k >> 1))];
        }
        group_sync<NT>();
        for (int it = 0; it < nu2; ++it) {
            tl_half_sweep<DIM, T, BC, NT>(f, 1);
            tl_half_sweep<DIM, T, BC, NT>(f, 0);
        }
    }
}

// BC: the plan has Dirichlet or periodic faces (extra diagonal, wrapped neighbours).
template <int DIM, typename T, bool BC>
__global__ void __launch_bounds__(kTailThreads)
k_tail(const LevelDesc* __restrict__ L, const GridState* __restrict__ S, JobList jl, int nu1, int nu2,
       int plain64) {
    extern __shared__ __align__(16) unsigned char tail_smem[];
    __shared__ TailGeom tl[kMaxTail];
    __shared__ int32_t off[kMaxTail + 1];
    __shared__ double red[2 * kTailThreads / 64];
    const int first = job_level(jl, blockIdx.x);
    const LevelDesc& d0 = L[first];
    if (!S[d0.sidx].active) return;
    const int hasa = (BC && Arr<T>::ad(d0) != nullptr) ? 1 : 0;
    // the grid's levels from `first` down are consecutive descriptors: thread m reads
    // level m's (no chain through the coarse links), then the LDS layout follows
    const int nl = min(d0.nlev - d0.level, kMaxTail);
    const int m_own = threadIdx.x;
    int32_t nown[3] = {0, 0, 0};
    if (m_own < nl) {
        const LevelDesc& d = L[first + m_own];
        nown[0] = d.n[0]; nown[1] = d.n[1]; nown[2] = d.n[2];
        off[m_own + 1] = (2 + DIM + hasa) * d.n[0] * d.n[1] * d.n[2];
    }
    if (threadIdx.x == 0) off[0] = 0;
    __syncthreads();
    if (m_own < nl) {
        int o = 0;
        for (int j = 0; j < m_own; ++j) o += off[j + 1];
        TailGeom& t = tl[m_own];
        t.n[0] = nown[0]; t.n[1] = nown[1]; t.n[2] = nown[2];
        t.ncell = nown[0] * nown[1] * nown[2];
        t.hx = (nown[0] + 1) / 2;
        t.rhx = 1.0f / (float)t.hx;
        t.rnx = 1.0f / (float)nown[0];
        t.rny = 1.0f / (float)nown[1];
        t.ox = o; o += t.ncell;
        t.ob = o; o += t.ncell;
        for (int a = 0; a < 3; ++a) {
            t.ow[a] = o;                                   // unused past DIM
            if (a < DIM) o += t.ncell;
        }
        t.oa = o;                                          // unused without Dirichlet faces
        t.has_a = hasa;
        t.pm = BC ? nb_mask(L[first + m_own]) : 0;          // continuous faces cut level 0 only
    }
    __syncthreads();
    T* const sbase = reinterpret_cast<T*>(tail_smem);
    T* p_sh = sbase + (tl[nl - 1].oa + hasa * tl[nl - 1].ncell);   // the coarsest CG's search direction
    // load every tail level's weights, and b and (warm) x of the first; loads of a
    // level are issued together, then stored
    for (int m = 0; m < nl; ++m) {
        const LevelDesc& d = L[first + m];
        const TailLevel<T> t = tl_at(tl[m], sbase);
        const gptr<T> s0 = as_global(Arr<T>::w(d, 0));
        const gptr<T> s1 = as_global(Arr<T>::w(d, 1));
        const gptr<T> s2 = as_global((DIM == 3) ? Arr<T>::w(d, 2) : Arr<T>::w(d, 0));
        const bool lead = (m == 0);
        const bool warm = lead && plain64 && d.level == 0;
        const gptr<T> bsrc = as_global(Arr<T>::b(d));
        const gptr<T> xsrc = as_global(Arr<T>::x(d));
        const gptr<T> asrc = as_global(hasa ? Arr<T>::ad(d) : Arr<T>::w(d, 0));
        for (int c = threadIdx.x; c < t.ncell; c += kTailThreads) {
            const T a0 = s0[c], a1 = s1[c];
            const T a2 = (DIM == 3) ? s2[c] : T(0);
            if (hasa) t.a[c] = asrc[c];
            const T bb = lead ? bsrc[c] : T(0);
            const T xx = warm ? xsrc[c] : T(0);
            t.w[0][c] = a0;
            t.w[1][c] = a1;
            if (DIM == 3) t.w[2][c] = a2;
            if (lead) {
                t.b[c] = bb;
                t.x[c] = xx;
            }
        }
    }
    __syncthreads();
    // Levels of at most kTailWaveCells cells run on one wavefront, without workgroup
    // barriers (they leave most of the block idle anyway): from the first such level
    // ws down, when the coarsest level has at most 64 cells (the wavefront's CG then
    // sums its products in the order the whole block would).
    int ws = nl;
    if (tl[nl - 1].ncell <= 64) {
        ws = nl - 1;
        while (ws > 0 && tl[ws - 1].ncell <= kTailWaveCells) --ws;
    }
    if (ws == nl) {
        tail_vcycle<DIM, T, BC, kTailThreads, kTailCPT>(tl, sbase, 0, nl, nu1, nu2, p_sh, red);
    } else {
        // the workgroup smooths and restricts the levels above ws, one wavefront runs
        // the V-cycle from ws, the workgroup prolongs and smooths back up
        for (int m = 0; m < ws; ++m) {
            const TailLevel<T> f = tl_at(tl[m], sbase);
            const TailLevel<T> cT = tl_at(tl[m + 1], sbase);
            for (int it = 0; it < nu1; ++it) {
                tl_half_sweep<DIM, T, BC, kTailThreads>(f, 0);
                tl_half_sweep<DIM, T, BC, kTailThreads>(f, 1);
            }
            for (int c = threadIdx.x; c < cT.ncell; c += kTailThreads) {
                int I, J, K;
                tl_coords<DIM, T>(cT, c, I, J, K);
                T sum = T(0);
#pragma unroll
                for (int q = 0; q < (1 << DIM); ++q)
                    sum += residual_at<DIM, T>(f.x, f.b, f.w[0], f.w[1], f.w[2], f.n, 2 * I + (q & 1),
                                               2 * J + ((q >> 1) & 1), DIM == 3 ? 2 * K + (q >> 2) : 0, f.a,
                                               BC && f.has_a != 0, BC ? f.pm : 0);
                cT.b[c] = sum * T(DIM == 3 ? 0.125 : 0.25);
                cT.x[c] = T(0);
            }
            __syncthreads();
        }
        if (threadIdx.x < 64) tail_vcycle<DIM, T, BC, 64, 1>(tl, sbase, ws, nl, nu1, nu2, p_sh, red);
        __syncthreads();
        for (int m = ws - 1; m >= 0; --m) {
            const TailLevel<T> f = tl_at(tl[m], sbase);
            const TailLevel<T> cT = tl_at(tl[m + 1], sbase);
            for (int c = threadIdx.x; c < f.ncell; c += kTailThreads) {
                int i, j, k;
                tl_coords<DIM, T>(f, c, i, j, k);
                f.x[c] += cT.x[(i >> 1) + cT.n[0] * ((j >> 1) + cT.n[1] * (k >> 1))];
            }
            __syncthreads();
            for (int it = 0; it < nu2; ++it) {
                tl_half_sweep<DIM, T, BC, kTailThreads>(f, 1);
                tl_half_sweep<DIM, T, BC, kTailThreads>(f, 0);
            }
        }
    }
    {
        const gptr<T> xdst = as_global(Arr<T>::x(L[first]));
        const TailLevel<T> t0 = tl_at(tl[0], sbase);
        for (int c = threadIdx.x; c < t0.ncell; c += kTailThreads) xdst[c] = t0.x[c];
    }
}

// ---------------------------------------------------------------------------
// Radiation moments of E per cell, after the step (Sec. 2.2 and 3.2): with the
// gradient and limiter of the coefficient pass, the flux F = -c lambda/(kappa
// rho) grad E (eq. fld_F), the force density f_r = rho kappa F / c (eq.
// rhd_force), the Eddington factor f = lambda + lambda^2 R^2 (eq. fld_Edd_fac)
// and the pressure tensor E (1/2 (1-f) I + 1/2 (3f-1) n n), n = grad E/|grad E|
// (eq. fld_Edd; n = 0 where the gradient vanishes).  With a velocity field, the
// photon-tiring work P : grad v = sum_ij P_ij dv_i/dx_j from 4th-order velocity
// gradients, and E - dt P : grad v (the explicit update of the energy equation,
// where the term sits on the left-hand side).  Stencil reads of E and v only:
// every output is written by its own cell.
// ---------------------------------------------------------------------------
template <int DIM>
__global__ void __launch_bounds__(kBlock)
k_moments(const LevelDesc* __restrict__ L, JobList jl, const MomentsIO* __restrict__ io, double c, int limiter) {
    const XcdOrder order(jl.total);
    for (int k_ = order.first(); order.more(k_); k_ += order.per) {
        const int t = order.tile(k_);
        const int jb = find_job(jl.prefix, jl.njobs, t);
        const LevelDesc& d = L[job_level(jl, jb)];
        const MomentsIO& m = io[d.grid];
#pragma unroll
        for (int m_ = 0; m_ < kCPT0; ++m_) {
            int i, j, k;
            cell_of_l0tile<DIM>(d.n, t - job_start(jl, jb), threadIdx.x + m_ * kBlock, i, j, k);
            if (i >= d.n[0] || j >= d.n[1] || k >= d.n[2]) continue;
            const long idx = i + (long)d.n[0] * (j + (long)d.n[1] * k);
            const double c12[3] = {d.hinv[0] / 12.0, d.hinv[1] / 12.0, d.hinv[2] / 12.0};
            const double e = m.E[idx], kk = m.kr[idx];
            double g[3];
            if (d.has_bc) grad4_bc_at<DIM>(m.E, i, j, k, d.n, c12, d, g);
            else grad4_at<DIM>(m.E, i, j, k, d.n, c12, g);
            double g2 = g[0] * g[0] + g[1] * g[1];
            if (DIM == 3) g2 += g[2] * g[2];
            const double gn = sqrt(g2);
            const double R = gn / (kk * e);
            const double lam = limiter_of(R, limiter);
    #pragma unroll
            for (int a = 0; a < DIM; ++a) {
                const double Fa = -c * lam / kk * g[a];
                if (m.F[a]) m.F[a][idx] = Fa;
                if (m.fr[a]) m.fr[a][idx] = kk * Fa / c;
            }
            const double f = R < 1e100 ? lam + lam * lam * R * R : lam + (lam * R) * (lam * R);
            if (m.edd) m.edd[idx] = f;
            double nv[3];
    #pragma unroll
            for (int a = 0; a < 3; ++a) nv[a] = (a < DIM && gn > 0.0) ? g[a] / gn : 0.0;
            const double iso = 0.5 * (1.0 - f), aniso = 0.5 * (3.0 * f - 1.0);
            double P[DIM][DIM];
            int q = 0;
    #pragma unroll
            for (int a = 0; a < DIM; ++a) {
    #pragma unroll
                for (int b = a; b < DIM; ++b, ++q) {
                    double tt = aniso * nv[a] * nv[b];
                    if (a == b) tt = tt + iso;
                    P[a][b] = e * tt;
                    P[b][a] = P[a][b];
                    if (m.P[q]) m.P[q][idx] = P[a][b];
                }
            }
            if (m.v[0]) {
                double tir = 0.0;
    #pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    double dv[3];
                    if (d.per_mask) grad4_per_at<DIM>(m.v[a], i, j, k, d.n, c12, d.per_mask, dv);
                    else grad4_at<DIM>(m.v[a], i, j, k, d.n, c12, dv);   // dv[b] = d v_a / d x_b
    #pragma unroll
                    for (int b = 0; b < DIM; ++b) tir = tir + P[a][b] * dv[b];
                }
                if (m.tiring) m.tiring[idx] = tir;
                if (m.E_out) m.E_out[idx] = e - m.dt * tir;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Level-0 FP64 residual r = b - A x and its per-tile partial ||r||^2.  In mixed
// precision the residual also becomes the FP32 right-hand side of the next
// correction V-cycle, whose correction starts from zero.
// ---------------------------------------------------------------------------
template <int DIM, bool MIXED>
__global__ void __launch_bounds__(kBlock)
k_residual(const LevelDesc* __restrict__ L, GridState* __restrict__ S, JobList jl, int select,
           int zero_x, int fin, double rtol, int max_cycles) {
    __shared__ double sh[2 * kBlock / 64];
    __shared__ int flag;
    const XcdOrder order(jl.total);
    for (int k_ = order.first(); order.more(k_); k_ += order.per) {
        const int t = order.tile(k_);
        const int jb = find_job(jl.prefix, jl.njobs, t);
        const LevelDesc& d = L[job_level(jl, jb)];
        const GridState& g = S[d.sidx];
        // select 0: grids still iterating; 1: grids that stopped with FLD_OK (their
        // recursive residual met the target), whose true residual is checked here
        if (select == 0 ? !g.active : (g.status != FLD_OK || g.active)) continue;   // uniform per tile
        const int lt = t - job_start(jl, jb);
        double r2 = 0.0, unused = 0.0;
        double rv[kCPT0];
        long ix[kCPT0];
        bool ok[kCPT0];
#pragma unroll
        for (int m_ = 0; m_ < kCPT0; ++m_) {
            int i, j, k;
            ix[m_] = l0_cell<DIM>(d, lt, m_, i, j, k, ok[m_]);
            rv[m_] = residual_at<DIM, double>(as_global(d.X), as_global(d.B0), as_global(d.w[0]),
                                              as_global(d.w[1]), as_global(DIM == 3 ? d.w[2] : d.w[0]),
                                              d.n, i, j, k, as_global(d.ad), d.ad != nullptr, nb_mask(d));
        }
#pragma unroll
        for (int m_ = 0; m_ < kCPT0; ++m_) {
            if (!ok[m_]) continue;
            const long idx = ix[m_];
            const double r = rv[m_];
            r2 += r * r;
            as_global(d.R)[idx] = r;
            if (MIXED) {
                as_global(d.b32)[idx] = (float)r;
                if (zero_x) as_global(d.x32)[idx] = 0.0f;
            } else if (zero_x) {
                as_global(d.x)[idx] = 0.0;
            }
        }
        tile_reduce_finish(d, S[d.sidx], lt, job_tiles(jl, jb), r2, unused, 1, fin, rtol,
                           max_cycles, sh, &flag);
    }
}

// ---------------------------------------------------------------------------
// Conjugate gradients on A with the V-cycle as preconditioner (FP64 scalars and
// vectors; in mixed precision the V-cycle itself is FP32).  One iteration:
//   z = V(r); rho = r.z; beta = rho/rho_old; p = z + beta p; q = A p;
//   alpha = rho/p.q; x += alpha p; r -= alpha q.
// The search direction is double-buffered by iteration parity so that q = A p
// can read neighbours' new p without a second pass.
// ---------------------------------------------------------------------------
// The preconditioned residual z: the V-cycle's level-0 iterate (FP32 in mixed
// precision), read through a global pointer.
template <bool MIXED>
struct ZArr {
    gptr<double> x64;
    gptr<float> x32;
    __device__ explicit ZArr(const LevelDesc& d) : x64(as_global(d.x)), x32(as_global(d.x32)) {}
    __device__ double operator[](long idx) const { return MIXED ? (double)x32[idx] : x64[idx]; }
};

template <int DIM, bool MIXED>
__global__ void __launch_bounds__(kBlock)
k_cg_rz(const LevelDesc* __restrict__ L, GridState* __restrict__ S, JobList jl, int fin, double rtol,
        int max_cycles) {
    __shared__ double sh[2 * kBlock / 64];
    __shared__ int flag;
    const XcdOrder order(jl.total);
    for (int k_ = order.first(); order.more(k_); k_ += order.per) {
        const int t = order.tile(k_);
        const int jb = find_job(jl.prefix, jl.njobs, t);
        const LevelDesc& d = L[job_level(jl, jb)];
        if (!S[d.sidx].active) continue;
        const int lt = t - job_start(jl, jb);
        double a = 0.0, unused = 0.0;
        const gptr<double> Rg = as_global(d.R);
        const ZArr<MIXED> z(d);
        double rv[kCPT0], zv[kCPT0];
        bool ok[kCPT0];
#pragma unroll
        for (int m_ = 0; m_ < kCPT0; ++m_) {
            int i, j, k;
            const long idx = l0_cell<DIM>(d, lt, m_, i, j, k, ok[m_]);
            rv[m_] = Rg[idx];
            zv[m_] = z[idx];
        }
#pragma unroll
        for (int m_ = 0; m_ < kCPT0; ++m_) a += ok[m_] ? rv[m_] * zv[m_] : 0.0;
        tile_reduce_finish(d, S[d.sidx], lt, job_tiles(jl, jb), a, unused, 1, fin, rtol,
                           max_cycles, sh, &flag);
    }
}

// Neighbour weight and search-direction value for k_cg_pq (see nb_pair).
template <typename F>
__device__ __forceinline__ void nb_p(gptr<double> w, long idx, int i, int n, long st, bool per, bool upper,
                                     const F& p_at, double& wn, double& pn) {
    const bool has = upper ? (i + 1 < n || per) : (i > 0 || per);
    const long nb = upper ? (i + 1 < n ? idx + st : (per ? idx - (long)(n - 1) * st : idx))
                          : (i > 0 ? idx - st : (per ? idx + (long)(n - 1) * st : idx));
    const double wv = w[upper ? nb : idx];
    wn = has ? wv : 0.0;
    pn = p_at(nb);
}

template <int DIM, bool MIXED>
__global__ void __launch_bounds__(kBlock)
k_cg_pq(const LevelDesc* __restrict__ L, GridState* __restrict__ S, JobList jl, int fin, double rtol,
        int max_cycles) {
    __shared__ double sh[2 * kBlock / 64];
    __shared__ int flag;
    const XcdOrder order(jl.total);
    for (int k_ = order.first(); order.more(k_); k_ += order.per) {
        const int t = order.tile(k_);
        const int jb = find_job(jl.prefix, jl.njobs, t);
        const LevelDesc& d = L[job_level(jl, jb)];
        GridState& g = S[d.sidx];
        if (!g.active) continue;
        const int lt = t - job_start(jl, jb);
        const int nt = job_tiles(jl, jb);
        const bool restart = g.iter == 0;            // p = z (the old direction is not read)
        double beta;
        if (fin == kFinFold) {
            // r.z from k_cg_rz's tile partials, summed here in k_finalize's order; the
            // grid's first tile records it (rho of this iteration's parity, beta)
            double rz, unused_;
            sum_parts(d.part, nt, 1, rz, unused_, sh);
            beta = cg_beta(g, rz);
            if (lt == 0 && threadIdx.x == 0) {
                g.rho[g.iter & 1] = rz;
                g.beta = beta;
            }
        } else {
            beta = g.beta;
        }
        const int par = g.iter & 1;
        const gptr<double> Pn = as_global(d.P[par]);
        const gptr<double> Po = as_global(d.P[par ^ 1]);
        const ZArr<MIXED> z(d);
        double pq = 0.0, unused = 0.0;
        // one cell at a time: the stencil loads of all four cells in flight at once need
        // more registers than the occupancy a large batch's bandwidth wants
#pragma unroll 1
        for (int m_ = 0; m_ < kCPT0; ++m_) {
            int i, j, k;
            bool ok;
            const long idx = l0_cell<DIM>(d, lt, m_, i, j, k, ok);     // loads of a clamped cell are
            {                                                             // issued unconditionally
                const long sy = d.n[0], sz = (long)d.n[0] * d.n[1];
                auto p_at = [&](long c) { return restart ? z[c] : z[c] + beta * Po[c]; };
                // every neighbour load is issued (from the cell itself across the boundary,
                // with weight 0: pc - pc adds exactly zero)
                const double pc = p_at(idx);
                const gptr<double> w0 = as_global(d.w[0]), w1 = as_global(d.w[1]);
                double wl, pl, wr, pr, wd, pd, wu, pu;
                const int pm = d.per_mask;
                nb_p(w0, idx, i, d.n[0], 1, pm & 1, false, p_at, wl, pl);
                nb_p(w0, idx, i, d.n[0], 1, pm & 1, true, p_at, wr, pr);
                nb_p(w1, idx, j, d.n[1], sy, (pm >> 1) & 1, false, p_at, wd, pd);
                nb_p(w1, idx, j, d.n[1], sy, (pm >> 1) & 1, true, p_at, wu, pu);
                double q = pc;
                q += wl * (pc - pl);
                q += wr * (pc - pr);
                q += wd * (pc - pd);
                q += wu * (pc - pu);
                if (DIM == 3) {
                    const gptr<double> w2 = as_global(d.w[2]);
                    double wb, pb, wf, pf;
                    nb_p(w2, idx, k, d.n[2], sz, (pm >> 2) & 1, false, p_at, wb, pb);
                    nb_p(w2, idx, k, d.n[2], sz, (pm >> 2) & 1, true, p_at, wf, pf);
                    q += wb * (pc - pb);
                    q += wf * (pc - pf);
                }
                if (d.ad) q += as_global(d.ad)[idx] * pc;
                if (ok) {
                    Pn[idx] = pc;
                    as_global(d.Q)[idx] = q;
                    pq += pc * q;
                }
            }
        }
        // folded: p.q partials after the r.z ones (k_cg_update sums them)
        tile_reduce_finish(d, g, lt, nt, pq, unused, 1, fin == kFinFold ? -1 : fin, rtol, max_cycles, sh, &flag,
                           fin == kFinFold ? d.part + g.ntiles0 : d.part);
    }
}

// The same direction update and product on 3D grids without Dirichlet or periodic
// faces as a z-march: a block owns a window of kPqPX x kPqPY xy positions (64 x 13
// interior columns and one halo position around them, one position per thread) and
// walks fz planes, forming p = z + beta p_old once per cell of the window; the in-plane
// neighbours' p and the x / y faces come from an LDS ring of three plane slots, the
// z-neighbours from the thread's own registers, so every plane of z, p_old and the
// faces is read once.  q follows k_cg_pq's operand order.  One partial of p . q per
// block tile, summed over the tile's cells in a fixed order (each thread's planes in
// turn, then a fixed-order block sum); a separate finalize sums the tile partials.
template <bool MIXED>
__global__ void __launch_bounds__(1024)
k_cg_pq3(const LevelDesc* __restrict__ L, GridState* __restrict__ S, JobList jl, int fz) {
    constexpr int PX = kPqPX, PY = kPqPY, FX = PX - 2, FY = PY - 2, R = 3, NB = 5;
    __shared__ double sp[R][PY][PX];
    __shared__ double sw0[R][PY][PX];
    __shared__ double sw1[R][PY][PX];
    __shared__ double sh[2 * 1024 / 64];
    const bool pos = threadIdx.x < PX * PY;                 // threads past the window only reduce
    const int lx = pos ? threadIdx.x % PX : 1, ly = pos ? threadIdx.x / PX : 1;
    const bool inner = pos && lx >= 1 && lx < PX - 1 && ly >= 1 && ly < PY - 1;
    const XcdOrder order(jl.total);
    for (int k = order.first(); order.more(k); k += order.per) {
        const int tt = order.tile(k);
        const int jb = find_job(jl.prefix, jl.njobs, tt);
        const LevelDesc& d = L[job_level(jl, jb)];
        GridState& g = S[d.sidx];
        if (!g.active) continue;
        const int lt = tt - job_start(jl, jb);
        const bool restart = g.iter == 0;                  // p = z (the old direction is not read)
        const double beta = g.beta;
        const int par = g.iter & 1;
        const gptr<double> Pn = as_global(d.P[par]);
        const gptr<double> Po = as_global(d.P[par ^ 1]);
        const gptr<double> Qg = as_global(d.Q);
        const ZArr<MIXED> zv(d);
        const gptr<double> w0g = as_global(d.w[0]), w1g = as_global(d.w[1]), w2g = as_global(d.w[2]);
        const int n0 = d.n[0], n1 = d.n[1], n2 = d.n[2];
        const int tx_n = (n0 + FX - 1) / FX, ty_n = (n1 + FY - 1) / FY;
        const int tx = lt % tx_n, rest = lt / tx_n;
        const int gx = tx * FX - 1 + lx, gy = (rest % ty_n) * FY - 1 + ly;
        const int z0 = (rest / ty_n) * fz, z1 = min(z0 + fz, n2);
        const int zs = z0 - 1, ze = z1 + 1;
        const bool in_xy = pos && gx >= 0 && gx < n0 && gy >= 0 && gy < n1;
        const long sz = (long)n0 * n1;
        const long cxy = min(max(gx, 0), n0 - 1) + (long)min(max(gy, 0), n1 - 1) * n0;
        double Z[NB], PO[NB], W0[NB], W1[NB], W2[NB], PV[NB];
        auto load = [&](auto Sl, int gk) {
            constexpr int q = decltype(Sl)::value;
            const long idx = cxy + min(max(min(gk, ze - 1), 0), n2 - 1) * sz;   // past the march: its last plane
            Z[q] = zv[idx];
            W0[q] = w0g[idx];
            W1[q] = w1g[idx];
            W2[q] = w2g[idx];
            if (!restart) PO[q] = Po[idx];        // last: the conditional load's wait stays exact
        };
        double acc = 0.0;
        auto step = [&](auto Sc, int zt) {
            constexpr int q = decltype(Sc)::value, q1 = (q + NB - 1) % NB, q2 = (q + NB - 2) % NB;
            const int s0 = (zt - zs) % R;
            {
                const bool in = in_xy && zt >= 0 && zt < n2;
                const double pnew = restart ? Z[q] : Z[q] + beta * PO[q];
                PV[q] = in ? pnew : 0.0;
                W0[q] = in ? W0[q] : 0.0;
                W1[q] = in ? W1[q] : 0.0;
                W2[q] = in ? W2[q] : 0.0;
                if (pos) {
                    sp[s0][ly][lx] = PV[q];
                    sw0[s0][ly][lx] = W0[q];
                    sw1[s0][ly][lx] = W1[q];
                }
            }
            load(std::integral_constant<int, (q + 2) % NB>{}, zt + 2);   // on every step (clamped plane)
            __syncthreads();
            const int p1 = zt - 1;
            if (p1 >= z0 && p1 < z1 && inner && in_xy) {
                const int s1 = (p1 - zs) % R;
                const double pc = PV[q1];
                double qv = pc;
                qv += W0[q1] * (pc - sp[s1][ly][lx - 1]);
                qv += sw0[s1][ly][lx + 1] * (pc - sp[s1][ly][lx + 1]);
                qv += W1[q1] * (pc - sp[s1][ly - 1][lx]);
                qv += sw1[s1][ly + 1][lx] * (pc - sp[s1][ly + 1][lx]);
                qv += W2[q1] * (pc - PV[q2]);
                qv += W2[q] * (pc - PV[q]);
                const long idx = cxy + p1 * sz;
                Pn[idx] = pc;
                Qg[idx] = qv;
                acc += pc * qv;
            }
        };
        load(std::integral_constant<int, 0>{}, zs);
        load(std::integral_constant<int, 1>{}, zs + 1);
        int zb = zs;
        for (; zb + NB <= ze; zb += NB) unroll<NB>([&](auto Qc) { step(Qc, zb + decltype(Qc)::value); });
        unroll<NB - 1>([&](auto Qc) {
            if (zb + decltype(Qc)::value < ze) step(Qc, zb + decltype(Qc)::value);
        });
        double unused = 0.0;
        block_sum2<1024>(acc, unused, sh);                 // its barriers also free the slots
        if (threadIdx.x == 0) d.part[lt] = acc;
    }
}

// The same direction update and product on 2D grids without Dirichlet or periodic
// faces as a row march: one wavefront owns a window of kMarchNP columns (two a lane:
// kMarchNP - 4 interior columns and a halo of two on each side, so that a lane's
// columns start at an even index and load as one vector) and walks fz rows, forming
// p = z + beta p_old once per cell; a cell's x-neighbours' p and its right face come
// from the lane's other column or, across the pair boundary, from the neighbouring
// lane by a DPP shift, its y-neighbours from the lane's own registers, so every row of
// z, p_old and the faces is read once.  q follows k_cg_pq's operand order (a boundary
// face's stored weight is 0 and the cell past it holds p = 0).  One partial of p . q
// per window, summed in a fixed order (each lane's rows in turn, even column first,
// then a butterfly over the wavefront); a separate finalize sums the partials.
template <bool MIXED>
__global__ void __launch_bounds__(64)
k_cg_pq2m(const LevelDesc* __restrict__ L, GridState* __restrict__ S, JobList jl, int fz) {
    constexpr int NP = kMarchNP, HX = 2, FX = NP - 2 * HX;
    constexpr int PF = 2, NB = PF + 3;                   // rows zt + 2 .. zt - 2
    using V2 = double __attribute__((ext_vector_type(2)));
    using ZT = std::conditional_t<MIXED, float, double>;
    using Z2 = ZT __attribute__((ext_vector_type(2)));
    const int l = threadIdx.x;
    const XcdOrder order(jl.total);
    for (int kk = order.first(); order.more(kk); kk += order.per) {
        const int tt = order.tile(kk);
        const int jb = find_job(jl.prefix, jl.njobs, tt);
        const LevelDesc& d = L[job_level(jl, jb)];
        GridState& g = S[d.sidx];
        if (!g.active) continue;                                      // uniform per window
        const int lt = tt - job_start(jl, jb);
        const bool restart = g.iter == 0;                             // p = z (the old direction is not read)
        const double beta = g.beta;
        const int par = g.iter & 1;
        const gptr<double> Pn = as_global(d.P[par]);
        const gptr<double> Po = as_global(d.P[par ^ 1]);
        const gptr<double> Qg = as_global(d.Q);
        const gptr<ZT> zg = as_global(MIXED ? (ZT*)d.x32 : (ZT*)d.x);
        const gptr<double> w0g = as_global(d.w[0]), w1g = as_global(d.w[1]);
        const int nx = d.n[0], ny = d.n[1];
        const int tx_n = (nx + FX - 1) / FX;
        const int gx0 = (lt % tx_n) * FX - HX;
        const int z0 = (lt / tx_n) * fz, z1 = min(z0 + fz, ny);
        const int zs = z0 - 1, ze = z1 + 1;
        const int ge = gx0 + 2 * l;
        const bool inx = ge >= 0 && ge < nx;                          // nx even: both columns or neither
        const int pc = min(max(ge, 0), nx - 2);
        const bool own = inx && l >= HX / 2 && l < (NP - HX) / 2;
        ZT Ze[NB], Zo[NB];
        double Oe[NB], Oo[NB], Pe[NB], Pq[NB], W0e[NB], W0o[NB], W1e[NB], W1o[NB];
        unroll<NB>([&](auto Qc) {
            constexpr int q = decltype(Qc)::value;
            Ze[q] = Zo[q] = ZT(0);
            Oe[q] = Oo[q] = Pe[q] = Pq[q] = W0e[q] = W0o[q] = W1e[q] = W1o[q] = 0.0;
        });
        auto load = [&](auto Sl, int gj) {
            constexpr int q = decltype(Sl)::value;
            const long idx = pc + (long)nx * min(max(min(gj, ze - 1), 0), ny - 1);   // past the march: its last row
            const Z2 z2 = *(const gptr<Z2>)(zg + idx);
            const V2 u2 = *(const gptr<V2>)(w0g + idx);
            const V2 v2 = *(const gptr<V2>)(w1g + idx);
            Ze[q] = z2.x;
            Zo[q] = z2.y;
            W0e[q] = u2.x;
            W0o[q] = u2.y;
            W1e[q] = v2.x;
            W1o[q] = v2.y;
            if (!restart) {
                const V2 o2 = *(const gptr<V2>)(Po + idx);
                Oe[q] = o2.x;
                Oo[q] = o2.y;
            }
        };
        double acc = 0.0;
        auto step = [&](auto Qc, int zt) {
            constexpr int q = decltype(Qc)::value, q1 = (q + NB - 1) % NB, q2 = (q + NB - 2) % NB;
            {
                // row zt enters: its p (zero outside the level)
                const bool in = inx && zt >= 0 && zt < ny;
                const double pe = restart ? (double)Ze[q] : (double)Ze[q] + beta * Oe[q];
                const double po = restart ? (double)Zo[q] : (double)Zo[q] + beta * Oo[q];
                Pe[q] = in ? pe : 0.0;
                Pq[q] = in ? po : 0.0;
                W0e[q] = in ? W0e[q] : 0.0;
                W0o[q] = in ? W0o[q] : 0.0;
                W1e[q] = in ? W1e[q] : 0.0;
                W1o[q] = in ? W1o[q] : 0.0;
            }
            load(std::integral_constant<int, (q + PF) % NB>{}, zt + PF);
            // q of row zt - 1
            const double pe = Pe[q1], po = Pq[q1];
            const double pl = lane_nb<true>(po), pr = lane_nb<false>(pe), wr = lane_nb<false>(W0e[q1]);
            double qe = pe;
            qe += W0e[q1] * (pe - pl);
            qe += W0o[q1] * (pe - po);
            qe += W1e[q1] * (pe - Pe[q2]);
            qe += W1e[q] * (pe - Pe[q]);
            double qo = po;
            qo += W0o[q1] * (po - pe);
            qo += wr * (po - pr);
            qo += W1o[q1] * (po - Pq[q2]);
            qo += W1o[q] * (po - Pq[q]);
            const int r = zt - 1;
            if (own && r >= z0 && r < z1) {
                const long idx = ge + (long)nx * r;
                V2 p2, q2v;
                p2.x = pe;
                p2.y = po;
                q2v.x = qe;
                q2v.y = qo;
                *(gptr<V2>)(Pn + idx) = p2;
                *(gptr<V2>)(Qg + idx) = q2v;
                acc += pe * qe;
                acc += po * qo;
            }
        };
        static_assert(PF == 2, "the prologue below loads two rows");
        load(std::integral_constant<int, 0>{}, zs);
        load(std::integral_constant<int, 1>{}, zs + 1);
        int zb = zs;
        for (; zb + NB <= ze; zb += NB) unroll<NB>([&](auto Qc) { step(Qc, zb + decltype(Qc)::value); });
        unroll<NB - 1>([&](auto Qc) {
            if (zb + decltype(Qc)::value < ze) step(Qc, zb + decltype(Qc)::value);
        });
        // fixed-order butterfly: every lane ends with the same sum (a + b = b + a exactly)
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if (l == 0) d.part[lt] = acc;
    }
}

template <int DIM, bool MIXED>
__global__ void __launch_bounds__(kBlock)
k_cg_update(const LevelDesc* __restrict__ L, GridState* __restrict__ S, JobList jl, int fin, double rtol,
        int max_cycles, int zero_z) {
    __shared__ double sh[2 * kBlock / 64];
    __shared__ int flag;
    const XcdOrder order(jl.total);
    for (int k_ = order.first(); order.more(k_); k_ += order.per) {
        const int t = order.tile(k_);
        const int jb = find_job(jl.prefix, jl.njobs, t);
        const LevelDesc& d = L[job_level(jl, jb)];
        GridState& g = S[d.sidx];
        if (!g.active) continue;
        const int lt = t - job_start(jl, jb);
        const gptr<double> P = as_global(d.P[g.iter & 1]);
        double r2 = 0.0, unused = 0.0;
        const gptr<double> X = as_global(d.X), R = as_global(d.R), Q = as_global(d.Q);
        double xv[kCPT0], pv[kCPT0], rv[kCPT0], qv[kCPT0];
        long ix[kCPT0];
        bool ok[kCPT0];
#pragma unroll
        for (int m_ = 0; m_ < kCPT0; ++m_) {
            int i, j, k;
            ix[m_] = l0_cell<DIM>(d, lt, m_, i, j, k, ok[m_]);
            xv[m_] = X[ix[m_]];
            pv[m_] = P[ix[m_]];
            rv[m_] = R[ix[m_]];
            qv[m_] = Q[ix[m_]];
        }
        double alpha;
        if (fin == kFinFold) {
            // p . q from k_cg_pq's partials (after the r.z ones), summed in k_finalize's
            // order; the grid's first tile records alpha (and a breakdown ends the grid)
            double pq, unused_;
            sum_parts(d.part + g.ntiles0, job_tiles(jl, jb), 1, pq, unused_, sh);
            alpha = cg_alpha(g, pq);
            if (lt == 0 && threadIdx.x == 0) {
                g.alpha = alpha;
                if (alpha == 0.0) {
                    g.active = 0;
                    g.status = (g.rnorm2 <= g.tol2) ? FLD_OK : FLD_ERR_NOT_CONVERGED;
                }
            }
            if (alpha == 0.0) continue;              // uniform per tile
        } else {
            alpha = g.alpha;
        }
#pragma unroll
        for (int m_ = 0; m_ < kCPT0; ++m_) {
            if (!ok[m_]) continue;
            const long idx = ix[m_];
            X[idx] = xv[m_] + alpha * pv[m_];
            const double r = rv[m_] - alpha * qv[m_];
            R[idx] = r;
            r2 += r * r;
            if (MIXED) {
                as_global(d.b32)[idx] = (float)r;
                if (zero_z) as_global(d.x32)[idx] = 0.0f;
            } else if (zero_z) {
                as_global(d.x)[idx] = 0.0;
            }
        }
        tile_reduce_finish(d, g, lt, job_tiles(jl, jb), r2, unused, 1, fin == kFinFold ? -1 : fin, rtol,
                           max_cycles, sh, &flag);
    }
}

template <int DIM, bool MIXED>
__global__ void __launch_bounds__(kBlock)
k_correct(const LevelDesc* __restrict__ L, const GridState* __restrict__ S, JobList jl) {
    const XcdOrder order(jl.total);
    for (int k_ = order.first(); order.more(k_); k_ += order.per) {
        const int t = order.tile(k_);
        const int jb = find_job(jl.prefix, jl.njobs, t);
        const LevelDesc& d = L[job_level(jl, jb)];
        if (!S[d.sidx].active) continue;
#pragma unroll
        for (int m_ = 0; m_ < kCPT0; ++m_) {
            int i, j, k;
            bool ok;
            const long idx = l0_cell<DIM>(d, t - job_start(jl, jb), m_, i, j, k, ok);
            const double z = MIXED ? (double)as_global(d.x32)[idx] : as_global(d.x)[idx];
            const double v = as_global(d.X)[idx] + z;
            if (ok) as_global(d.X)[idx] = v;
        }
    }
}

template <int DIM>
__global__ void __launch_bounds__(kBlock)
k_output(const LevelDesc* __restrict__ L, JobList jl, const StepIO* __restrict__ io) {
    const XcdOrder order(jl.total);
    for (int k_ = order.first(); order.more(k_); k_ += order.per) {
        const int t = order.tile(k_);
        const int jb = find_job(jl.prefix, jl.njobs, t);
        const LevelDesc& d = L[job_level(jl, jb)];
#pragma unroll
        for (int m_ = 0; m_ < kCPT0; ++m_) {
            int i, j, k;
            bool ok;
            const long idx = l0_cell<DIM>(d, t - job_start(jl, jb), m_, i, j, k, ok);
            const double v = as_global(d.X)[idx];
            if (ok) as_global(io[d.grid].E_out)[idx] = v;
        }
    }
}

__global__ void __launch_bounds__(kBlock)
k_count(const GridState* __restrict__ S, int ngrids, Control* ctrl) {
    __shared__ double sh[2 * kBlock / 64];
    double a = 0.0, b = 0.0;
    for (int g = threadIdx.x; g < ngrids; g += kBlock) a += S[g].active;
    block_sum2<kBlock>(a, b, sh);
    if (threadIdx.x == 0) ctrl->nactive = (int32_t)a;
}

__global__ void __launch_bounds__(kBlock)
k_set_active(GridState* __restrict__ S, int ngrids, int value) {
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < ngrids; g += gridDim.x * blockDim.x)
        S[g].active = value;
}

// ---------------------------------------------------------------------------
// Exchange.  With x = C y / (1+a2), C = (1+a2) eps + a2 E, the quartic
// a1 x^4 + (1+a2) x - C = 0 becomes g(y) = beta y^4 + y - 1 = 0 with
// beta = a1 C^3 / (1+a2)^4 >= 0: g is increasing and convex on y > 0,
// g(0) = -1 < 0 <= g(1), so the root is unique in (0, 1].  Halley's method
// starts from the upper bound min(1, beta^(-1/4)) inside a bracket that every
// iterate tightens; an iterate that leaves the bracket, or running out of
// Halley iterations, hands over to bisection of the bracket.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double quartic_root(double beta, int max_halley, double rtol, bool& bisected) {
    bisected = false;
    if (!(beta > 0.0)) return 1.0;
    double lo = 0.0, hi = 1.0;
    double y = fmin(1.0, 1.0 / sqrt(sqrt(beta)));
    for (int it = 0; it < max_halley; ++it) {
        const double y2 = y * y;
        const double g = beta * y2 * y2 + y - 1.0;
        if (g > 0.0) hi = y; else if (g < 0.0) lo = y; else return y;
        const double g1 = 4.0 * beta * y2 * y + 1.0;
        const double g2 = 12.0 * beta * y2;
        const double den = 2.0 * g1 * g1 - g * g2;
        const double step = 2.0 * g * g1 / den;
        const double yn = y - step;
        if (!(den > 0.0) || !(yn > lo) || !(yn < hi)) {
            // outside the bracket: bisect this once and go on with Halley
            y = 0.5 * (lo + hi);
            continue;
        }
        if (fabs(step) <= rtol * yn) return yn;
        y = yn;
    }
    bisected = true;
    for (int it = 0; it < 1100; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        const double m2 = mid * mid;
        if (beta * m2 * m2 + mid - 1.0 > 0.0) hi = mid; else lo = mid;
    }
    const double glo = fabs(beta * lo * lo * lo * lo + lo - 1.0);
    const double ghi = fabs(beta * hi * hi * hi * hi + hi - 1.0);
    return glo <= ghi ? lo : hi;
}

// Exchange of one cell over dt (Sec. 3.3), in place on (E, eps).  Returns false and
// leaves both untouched for an invalid cell (rho <= 0, kappa < 0, E < 0, eps < 0,
// a non-finite value); counts a bisection fallback in nbis.
struct ExConst {
    double c, a_rad, cv4;
    int max_halley;
    double root_rtol;
};

__device__ __forceinline__ bool exchange_cell(double& E, double& eps, double rho, double kap, double dt,
                                              const ExConst& k, long& nbis) {
    const bool ok = isfinite(E) && isfinite(eps) && isfinite(rho) && isfinite(kap) && rho > 0.0 &&
                    kap >= 0.0 && E >= 0.0 && eps >= 0.0;
    if (!ok) return false;
    const double a2 = k.c * kap * rho * dt;
    const double a1 = k.c * k.a_rad * kap * dt / (rho * rho * rho * k.cv4);
    const double opa = 1.0 + a2;
    const double C = opa * eps + a2 * E;
    if (!(C > 0.0)) return true;                    // no energy in gas or radiation
    const double s = C / opa;
    const double beta = a1 * s * s * s / opa;       // a1 C^3 / (1+a2)^4
    bool bis;
    const double y = quartic_root(beta, k.max_halley, k.root_rtol, bis);
    nbis += bis;
    const double eps_new = s * y;
    const double e2 = eps_new * eps_new;
    eps = eps_new;
    E = (a1 * e2 * e2 + E) / opa;
    return true;
}

__global__ void __launch_bounds__(kBlock)
k_exchange(const ExchangeIO* __restrict__ io, ExConst k, Control* ctrl) {
    const ExchangeIO p = io[blockIdx.y];
    int bad = 0;
    long nbis = 0;
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < p.n;
         idx += (long)gridDim.x * blockDim.x) {
        double E = p.E[idx], eps = p.eps[idx];
        if (!exchange_cell(E, eps, p.rho[idx], p.kappa[idx], p.dt, k, nbis)) { bad = 1; continue; }
        p.eps[idx] = eps;
        p.E[idx] = E;
    }
    if (bad) atomicOr(&ctrl->bad_exchange, 1);
    if (nbis) atomicAdd((unsigned long long*)&ctrl->bisected, (unsigned long long)nbis);
}

// One pointwise stage of the IMEX step (per grid, blockIdx.y): optionally
// kappa rho, then the explicit operator on the stage's energy
//     E_x = E [+ 2 (E_m - E_p)] [- dt_tir tir]
// (the midpoint stage adds dt times the implicit tendency (E_m - E_p)/(dt/2) of
// the half step, and the tiring source at the midpoint state), then the
// exchange of (E_x, eps) over tau, written to (E_out, eps_out).
__global__ void __launch_bounds__(kBlock)
k_imex_point(const ImexIO* __restrict__ io, ExConst k, Control* ctrl) {
    const ImexIO p = io[blockIdx.y];
    if (!p.kr && !p.E_out) return;                  // nothing for this grid in this stage
    int bad = 0;
    long nbis = 0;
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < p.n;
         idx += (long)gridDim.x * blockDim.x) {
        const double rho = p.rho[idx], kap = p.kappa[idx];
        if (p.kr) p.kr[idx] = kap * rho;
        if (!p.E_out) continue;
        double E = p.E[idx];
        if (p.Em) E += 2.0 * (p.Em[idx] - p.Ep[idx]);
        if (p.tir) E -= p.dt_tir * p.tir[idx];
        double eps = p.eps[idx];
        if (!exchange_cell(E, eps, rho, kap, p.tau, k, nbis)) bad = 1;
        p.E_out[idx] = E;
        p.eps_out[idx] = eps;
    }
    if (bad) atomicOr(&ctrl->bad_imex, 1);
    if (nbis) atomicAdd((unsigned long long*)&ctrl->bisected, (unsigned long long)nbis);
}

inline int blocks_for(int total, int nblk) { return total < nblk ? (total > 0 ? total : 1) : nblk; }
// block count for the XCD-ordered kernels: a multiple of kXcds
inline int blocks_for_xcd(int total, int nblk) {
    const int g = blocks_for(total, nblk);
    return (g + kXcds - 1) / kXcds * kXcds;
}

}  // namespace

// ---- launch wrappers ---------------------------------------------------------
// Each wrapper also states its kernel's algorithmic bytes for the accounting mode
// (acct_set): every array the kernel reads or writes counted once per cell it
// covers, w the word of the level arrays, d the dimension; a coarse level has
// 1/2^d of the fine cells.
namespace {
thread_local Acct* t_acct = nullptr;
// In accounting mode: add `bytes` and one launch, and tell the wrapper not to launch.
inline bool acct_add(double bytes) {
    if (!t_acct) return false;
    t_acct->bytes += bytes;
    t_acct->launches += 1;
    return true;
}
}  // namespace

void acct_set(Acct* a) { t_acct = a; }
Acct* acct_get() { return t_acct; }

#define FLD_DISPATCH_DIM(dim, ...) \
    do { if ((dim) == 3) { constexpr int D = 3; __VA_ARGS__; } else { constexpr int D = 2; __VA_ARGS__; } } while (0)

void launch_coeff(int dim, bool mixed, int bc, const LevelDesc* L, GridState* S, JobList jl,
                  const StepIO* io, double c, int limiter, int fin, double rtol, int max_cycles, int nblk,
                  hipStream_t s) {
    if (jl.total <= 0) return;
    // D pass: E, kappa rho read, D written; face pass: E, kappa rho, D read, faces, b, x written
    if (acct_add(jl.cells * (8.0 * 3 + 8.0 * (3 + dim + 2) + (mixed ? 4.0 * (dim + 2) : 0.0)))) return;
    const int g = blocks_for_xcd(jl.total, nblk);
#define FLD_COEFF(M, B) hipLaunchKernelGGL((k_coeff<D, M, B>), dim3(g), dim3(kBlock), 0, s, L, S, jl, io, c, limiter, fin, rtol, max_cycles)
    FLD_DISPATCH_DIM(dim, {
        if (bc) hipLaunchKernelGGL((k_cell_D<D, true>), dim3(g), dim3(kBlock), 0, s, L, jl, io, c, limiter);
        else hipLaunchKernelGGL((k_cell_D<D, false>), dim3(g), dim3(kBlock), 0, s, L, jl, io, c, limiter);
        if (bc) { if (mixed) FLD_COEFF(true, true); else FLD_COEFF(false, true); }
        else { if (mixed) FLD_COEFF(true, false); else FLD_COEFF(false, false); }
    });
#undef FLD_COEFF
}

void launch_finalize(const LevelDesc* L, GridState* S, JobList jl, int mode, double rtol,
                     int max_cycles, hipStream_t s) {
    if (jl.njobs <= 0) return;
    if (acct_add(0.0)) return;                           // a grid's tile partials: negligible
    hipLaunchKernelGGL(k_finalize, dim3(jl.njobs), dim3(kBlock), 0, s, L, S, jl, mode, rtol, max_cycles);
}

void launch_coarsen(int dim, bool mixed, const LevelDesc* L, JobList jl, int galerkin, int nblk, hipStream_t s) {
    if (jl.total <= 0) return;
    // fine faces read, coarse faces written (list: the fine levels)
    if (acct_add(jl.cells * (8.0 * dim + (mixed ? 4.0 * dim : 8.0 * dim) / (1 << dim)))) return;
    const int g = blocks_for_xcd(jl.total, nblk);
    FLD_DISPATCH_DIM(dim, {
        if (mixed) hipLaunchKernelGGL((k_coarsen<D, true>), dim3(g), dim3(kBlock), 0, s, L, jl, galerkin);
        else hipLaunchKernelGGL((k_coarsen<D, false>), dim3(g), dim3(kBlock), 0, s, L, jl, galerkin);
    });
}

void launch_smooth(int dim, bool fp32, const LevelDesc* L, const GridState* S, JobList jl,
                   int color, int nblk, hipStream_t s) {
    if (jl.total <= 0) return;
    // x of every cell, b of the updated half, every face array, x of the updated half written
    if (acct_add(jl.cells * (fp32 ? 4.0 : 8.0) * (2 + dim))) return;
    const int g = blocks_for_xcd(jl.total, nblk);
    FLD_DISPATCH_DIM(dim, {
        if (fp32) hipLaunchKernelGGL((k_smooth<D, float>), dim3(g), dim3(kBlock), 0, s, L, S, jl, color);
        else hipLaunchKernelGGL((k_smooth<D, double>), dim3(g), dim3(kBlock), 0, s, L, S, jl, color);
    });
}

void launch_restrict(int dim, bool fp32, const LevelDesc* L, const GridState* S, JobList jl,
                     int nblk, hipStream_t s) {
    if (jl.total <= 0) return;
    // list: coarse cells; the children's x, b and faces read, coarse b and x written
    if (acct_add(jl.cells * (fp32 ? 4.0 : 8.0) * ((1 << dim) * (2 + dim) + 2))) return;
    const int g = blocks_for_xcd(jl.total, nblk);
    FLD_DISPATCH_DIM(dim, {
        if (fp32) hipLaunchKernelGGL((k_restrict<D, float>), dim3(g), dim3(kBlock), 0, s, L, S, jl);
        else hipLaunchKernelGGL((k_restrict<D, double>), dim3(g), dim3(kBlock), 0, s, L, S, jl);
    });
}

void launch_prolong(int dim, bool fp32, const LevelDesc* L, const GridState* S, JobList jl,
                    int nblk, hipStream_t s) {
    if (jl.total <= 0) return;
    // list: fine cells; x read and written, the coarse correction read
    if (acct_add(jl.cells * (fp32 ? 4.0 : 8.0) * (2.0 + 1.0 / (1 << dim)))) return;
    const int g = blocks_for_xcd(jl.total, nblk);
    FLD_DISPATCH_DIM(dim, {
        if (fp32) hipLaunchKernelGGL((k_prolong<D, float>), dim3(g), dim3(kBlock), 0, s, L, S, jl);
        else hipLaunchKernelGGL((k_prolong<D, double>), dim3(g), dim3(kBlock), 0, s, L, S, jl);
    });
}

void launch_restrict_rhs(int dim, bool fp32, const LevelDesc* L, const GridState* S, JobList jl,
                         int nblk, hipStream_t s) {
    if (jl.total <= 0) return;
    // list: coarse cells; the children's b read, coarse b and x written
    if (acct_add(jl.cells * (fp32 ? 4.0 : 8.0) * ((1 << dim) + 2))) return;
    const int g = blocks_for_xcd(jl.total, nblk);
    FLD_DISPATCH_DIM(dim, {
        if (fp32) hipLaunchKernelGGL((k_restrict_rhs<D, float>), dim3(g), dim3(kBlock), 0, s, L, S, jl);
        else hipLaunchKernelGGL((k_restrict_rhs<D, double>), dim3(g), dim3(kBlock), 0, s, L, S, jl);
    });
}

void launch_fmg_interp(int dim, bool fp32, const LevelDesc* L, const GridState* S, JobList jl,
                       int nblk, hipStream_t s) {
    if (jl.total <= 0) return;
    // list: fine cells; the coarse solution read, x written
    if (acct_add(jl.cells * (fp32 ? 4.0 : 8.0) * (1.0 + 1.0 / (1 << dim)))) return;
    const int g = blocks_for_xcd(jl.total, nblk);
    FLD_DISPATCH_DIM(dim, {
        if (fp32) hipLaunchKernelGGL((k_fmg_interp<D, float>), dim3(g), dim3(kBlock), 0, s, L, S, jl);
        else hipLaunchKernelGGL((k_fmg_interp<D, double>), dim3(g), dim3(kBlock), 0, s, L, S, jl);
    });
}

bool fused3_supported(bool fp32) {
    (void)fp32;
    return true;
}

void launch_sweep3(bool fp32, const LevelDesc* L, const GridState* S, JobList jl, int mode, int c0,
                   int from_xs, int fz, int nblk, hipStream_t s, int rz) {
    if (jl.total <= 0) return;
    {   // b and three face arrays read, the iterate read (not from zero) and written; the
        // restricting sweep writes the coarse b and x, the prolonging one reads coarse x
        const double w = fp32 ? 4.0 : 8.0;
        const bool from_zero = mode == SW_ZERO || mode == SW_ZERO_RESTR;
        const bool restr = mode == SW_LOAD_RESTR || mode == SW_ZERO_RESTR;
        double words = 5.0 + (from_zero ? 0.0 : 1.0);
        if (restr) words += 2.0 / 8.0;
        if (mode == SW_PROLONG) words += 1.0 / 8.0;
        if (acct_add(jl.cells * w * words)) return;
    }
    const int g = blocks_for_xcd(jl.total, nblk);
#define FLD_SWEEP3(M)                                                                                   \
    do {                                                                                               \
        if (fp32) hipLaunchKernelGGL((k_sweep3<float, M>), dim3(g), dim3(Sweep3Mode<M>::PX * Sweep3Mode<M>::PY), \
                                     0, s, L, S, jl, c0, from_xs, fz, rz);                             \
        else hipLaunchKernelGGL((k_sweep3<double, M>), dim3(g), dim3(Sweep3Mode<M>::PX * Sweep3Mode<M>::PY), \
                                0, s, L, S, jl, c0, from_xs, fz, rz);                                  \
    } while (0)
    switch (mode) {
        case SW_LOAD: FLD_SWEEP3(SW_LOAD); break;
        case SW_ZERO: FLD_SWEEP3(SW_ZERO); break;
        case SW_LOAD_RESTR: FLD_SWEEP3(SW_LOAD_RESTR); break;
        case SW_ZERO_RESTR: FLD_SWEEP3(SW_ZERO_RESTR); break;
        default: FLD_SWEEP3(SW_PROLONG); break;
    }
#undef FLD_SWEEP3
}

bool fused2_supported(int nu) { return nu >= 1 && nu <= 3; }

bool fused2_shape_ok(bool fp32, int nu, int wide, int fy, bool down) {
    if (!fused2_supported(nu) || (wide != 0 && wide != 1) || (fy != 4 && fy != 8 && fy != 16 && fy != 32)) return false;
    return fused_lds(fp32 ? 4 : 8, down ? 2 * nu + 1 : 2 * nu, wide, fy) <= kFusedLdsMax;
}

#define FLD_NU_DISPATCH(nu, ...)                                          \
    do {                                                                  \
        if ((nu) == 1) { constexpr int NU = 1; __VA_ARGS__; }             \
        else if ((nu) == 2) { constexpr int NU = 2; __VA_ARGS__; }        \
        else { constexpr int NU = 3; __VA_ARGS__; }                       \
    } while (0)

#define FLD_SHAPE_DISPATCH(wide, fy, ...)                                 \
    do {                                                                  \
        if (wide) {                                                       \
            constexpr int WIDE = 1;                                       \
            if ((fy) == 4) { constexpr int FY = 4; __VA_ARGS__; }         \
            else if ((fy) == 8) { constexpr int FY = 8; __VA_ARGS__; }    \
            else if ((fy) == 16) { constexpr int FY = 16; __VA_ARGS__; }  \
            else { constexpr int FY = 32; __VA_ARGS__; }                  \
        } else {                                                          \
            constexpr int WIDE = 0;                                       \
            if ((fy) == 4) { constexpr int FY = 4; __VA_ARGS__; }         \
            else if ((fy) == 8) { constexpr int FY = 8; __VA_ARGS__; }    \
            else if ((fy) == 16) { constexpr int FY = 16; __VA_ARGS__; }  \
            else { constexpr int FY = 32; __VA_ARGS__; }                  \
        }                                                                 \
    } while (0)

namespace {
// Instantiates a fused kernel only for shapes whose tile fits the LDS; the host
// never selects the others (fused2_shape_ok).
template <typename T, int NU, int WIDE, int FY>
void down2_t(const LevelDesc* L, const GridState* S, JobList jl, int load_x, int threads, int g, hipStream_t s) {
    if constexpr (fused_lds(sizeof(T), 2 * NU + 1, WIDE, FY) <= kFusedLdsMax) {
        if (threads == 1024)
            hipLaunchKernelGGL((k_down2<T, NU, WIDE, FY, 1024>), dim3(g), dim3(1024), 0, s, L, S, jl, load_x);
        else
            hipLaunchKernelGGL((k_down2<T, NU, WIDE, FY, kBlock>), dim3(g), dim3(kBlock), 0, s, L, S, jl, load_x);
    }
}
template <typename T, int NU, int WIDE, int FY>
void up2_t(const LevelDesc* L, const GridState* S, JobList jl, int threads, int g, hipStream_t s) {
    if constexpr (fused_lds(sizeof(T), 2 * NU, WIDE, FY) <= kFusedLdsMax) {
        if (threads == 1024)
            hipLaunchKernelGGL((k_up2<T, NU, WIDE, FY, 1024>), dim3(g), dim3(1024), 0, s, L, S, jl);
        else
            hipLaunchKernelGGL((k_up2<T, NU, WIDE, FY, kBlock>), dim3(g), dim3(kBlock), 0, s, L, S, jl);
    }
}
}  // namespace

void launch_down2(bool fp32, const LevelDesc* L, const GridState* S, JobList jl, int nu, int load_x,
                  int wide, int fy, int threads, int nblk, hipStream_t s) {
    if (jl.total <= 0) return;
    // b and two face arrays read (+ x when it starts from the iterate), xs written,
    // coarse b and x written
    if (acct_add(jl.cells * (fp32 ? 4.0 : 8.0) * (4.0 + (load_x ? 1.0 : 0.0) + 2.0 / 4.0))) return;
    const int g = blocks_for_xcd(jl.total, nblk);
    FLD_NU_DISPATCH(nu, FLD_SHAPE_DISPATCH(wide, fy, {
        if (fp32) down2_t<float, NU, WIDE, FY>(L, S, jl, load_x, threads, g, s);
        else down2_t<double, NU, WIDE, FY>(L, S, jl, load_x, threads, g, s);
    }));
}

void launch_up2(bool fp32, const LevelDesc* L, const GridState* S, JobList jl, int nu, int wide, int fy,
                int threads, int nblk, hipStream_t s) {
    if (jl.total <= 0) return;
    // xs, b, two face arrays and the coarse correction read, x written
    if (acct_add(jl.cells * (fp32 ? 4.0 : 8.0) * (5.0 + 1.0 / 4.0))) return;
    const int g = blocks_for_xcd(jl.total, nblk);
    FLD_NU_DISPATCH(nu, FLD_SHAPE_DISPATCH(wide, fy, {
        if (fp32) up2_t<float, NU, WIDE, FY>(L, S, jl, threads, g, s);
        else up2_t<double, NU, WIDE, FY>(L, S, jl, threads, g, s);
    }));
}

void launch_march2(bool fp32, const LevelDesc* L, const GridState* S, JobList jl, int nu, int down, int load_x,
                   int fz, int nblk, hipStream_t s, int rz) {
    if (jl.total <= 0) return;
    // the same operands as the fused tile passes (k_down2 / k_up2)
    if (acct_add(jl.cells * (fp32 ? 4.0 : 8.0) *
                 (down ? 4.0 + (load_x ? 1.0 : 0.0) + 2.0 / 4.0 : 5.0 + 1.0 / 4.0)))
        return;
    // one block per window: a window's march is long, and a block that owns several runs
    // them back to back while other compute units may idle
    (void)nblk;
    const int g = blocks_for_xcd(jl.total, jl.total);
#define FLD_MARCH(T_, D_, X_) hipLaunchKernelGGL((k_march2<T_, NU, D_, X_>), dim3(g), dim3(64), 0, s, L, S, jl, fz, rz)
    FLD_NU_DISPATCH(nu, {
        if (down && load_x) { if (fp32) FLD_MARCH(float, true, true); else FLD_MARCH(double, true, true); }
        else if (down) { if (fp32) FLD_MARCH(float, true, false); else FLD_MARCH(double, true, false); }
        else { if (fp32) FLD_MARCH(float, false, true); else FLD_MARCH(double, false, true); }
    });
#undef FLD_MARCH
}

template <int DIM, typename T, bool BC>
static hipError_t tail_lds(size_t smem) {
    return hipFuncSetAttribute((const void*)k_tail<DIM, T, BC>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
}
int prepare_tail(int dim, bool fp32, size_t smem) {
    hipError_t e0, e1;
    if (dim == 3) {
        e0 = fp32 ? tail_lds<3, float, false>(smem) : tail_lds<3, double, false>(smem);
        e1 = fp32 ? tail_lds<3, float, true>(smem) : tail_lds<3, double, true>(smem);
    } else {
        e0 = fp32 ? tail_lds<2, float, false>(smem) : tail_lds<2, double, false>(smem);
        e1 = fp32 ? tail_lds<2, float, true>(smem) : tail_lds<2, double, true>(smem);
    }
    return (e0 == hipSuccess && e1 == hipSuccess) ? 0 : -1;
}

void launch_tail(int dim, bool fp32, int bc, const LevelDesc* L, const GridState* S, JobList jl, size_t smem,
                 int nu1, int nu2, int plain64, hipStream_t s) {
    if (jl.njobs <= 0) return;
    // list: each grid's first tail level; its b and the face arrays of every tail level
    // (2^d / (2^d - 1) times the first level's) read once, its x written
    if (acct_add(jl.cells * (fp32 ? 4.0 : 8.0) * (2.0 + dim * (double)(1 << dim) / ((1 << dim) - 1)))) return;
#define FLD_TAIL(T_, B) hipLaunchKernelGGL((k_tail<D, T_, B>), dim3(jl.njobs), dim3(kTailThreads), smem, s, L, S, jl, nu1, nu2, plain64)
    FLD_DISPATCH_DIM(dim, {
        if (bc) { if (fp32) FLD_TAIL(float, true); else FLD_TAIL(double, true); }
        else { if (fp32) FLD_TAIL(float, false); else FLD_TAIL(double, false); }
    });
#undef FLD_TAIL
}

void launch_coarse_solve(int dim, bool fp32, const LevelDesc* L, const GridState* S, JobList jl,
                         hipStream_t s) {
    if (jl.njobs <= 0) return;
    if (acct_add(jl.cells * (fp32 ? 4.0 : 8.0) * (2 + dim))) return;   // b, faces read, x written
    FLD_DISPATCH_DIM(dim, {
        if (fp32) hipLaunchKernelGGL((k_coarse_solve<D, float>), dim3(jl.njobs), dim3(kCoarseThreads), 0, s, L, S, jl);
        else hipLaunchKernelGGL((k_coarse_solve<D, double>), dim3(jl.njobs), dim3(kCoarseThreads), 0, s, L, S, jl);
    });
}

void launch_residual(int dim, bool mixed, const LevelDesc* L, GridState* S, JobList jl,
                     int select, int zero_x, int fin, double rtol, int max_cycles, int nblk, hipStream_t s) {
    if (jl.total <= 0) return;
    // X, B0 and the face arrays read, R written; mixed: the FP32 right-hand side (and a
    // zeroed FP32 iterate), else a zeroed FP64 iterate
    if (acct_add(jl.cells * (8.0 * (3 + dim) + (mixed ? 4.0 + (zero_x ? 4.0 : 0.0) : (zero_x ? 8.0 : 0.0)))))
        return;
    const int g = blocks_for_xcd(jl.total, nblk);
    FLD_DISPATCH_DIM(dim, {
        if (mixed) hipLaunchKernelGGL((k_residual<D, true>), dim3(g), dim3(kBlock), 0, s, L, S, jl, select, zero_x, fin, rtol, max_cycles);
        else hipLaunchKernelGGL((k_residual<D, false>), dim3(g), dim3(kBlock), 0, s, L, S, jl, select, zero_x, fin, rtol, max_cycles);
    });
}

#define FLD_CG_LAUNCH(kern, bytes_per_cell)                                                          \
    if (jl.total <= 0) return;                                                                       \
    if (acct_add(jl.cells * (bytes_per_cell))) return;                                               \
    const int g = blocks_for_xcd(jl.total, nblk);                                                        \
    FLD_DISPATCH_DIM(dim, {                                                                          \
        if (mixed) hipLaunchKernelGGL((kern<D, true>), dim3(g), dim3(kBlock), 0, s, L, S, jl, fin, rtol, max_cycles); \
        else hipLaunchKernelGGL((kern<D, false>), dim3(g), dim3(kBlock), 0, s, L, S, jl, fin, rtol, max_cycles);      \
    })

void launch_cg_rz(int dim, bool mixed, const LevelDesc* L, GridState* S, JobList jl, int fin, double rtol, int max_cycles, int nblk,
                  hipStream_t s) {
    FLD_CG_LAUNCH(k_cg_rz, 8.0 + (mixed ? 4.0 : 8.0));              // r, z read
}

void launch_cg_pq(int dim, bool mixed, const LevelDesc* L, GridState* S, JobList jl, int fin, double rtol, int max_cycles, int nblk,
                  hipStream_t s) {
    // z, the old direction and the face arrays read; p and q written
    FLD_CG_LAUNCH(k_cg_pq, (mixed ? 4.0 : 8.0) + 8.0 + 8.0 * dim + 16.0);
}

void launch_cg_pq3(bool mixed, const LevelDesc* L, GridState* S, JobList jl, int fz, int nblk, hipStream_t s) {
    if (jl.total <= 0) return;
    // z, the old direction and the three face arrays read once; p and q written
    if (acct_add(jl.cells * ((mixed ? 4.0 : 8.0) + 8.0 + 24.0 + 16.0))) return;
    const int g = blocks_for_xcd(jl.total, nblk);
    if (mixed) hipLaunchKernelGGL((k_cg_pq3<true>), dim3(g), dim3(1024), 0, s, L, S, jl, fz);
    else hipLaunchKernelGGL((k_cg_pq3<false>), dim3(g), dim3(1024), 0, s, L, S, jl, fz);
}

void launch_cg_pq2m(bool mixed, const LevelDesc* L, GridState* S, JobList jl, int fz, hipStream_t s) {
    if (jl.total <= 0) return;
    // z, the old direction and the two face arrays read once; p and q written
    if (acct_add(jl.cells * ((mixed ? 4.0 : 8.0) + 8.0 + 16.0 + 16.0))) return;
    const int g = blocks_for_xcd(jl.total, jl.total);           // one wavefront per window
    if (mixed) hipLaunchKernelGGL((k_cg_pq2m<true>), dim3(g), dim3(64), 0, s, L, S, jl, fz);
    else hipLaunchKernelGGL((k_cg_pq2m<false>), dim3(g), dim3(64), 0, s, L, S, jl, fz);
}

void launch_cg_update(int dim, bool mixed, const LevelDesc* L, GridState* S, JobList jl, int fin, double rtol, int max_cycles,
                      int zero_z, int nblk, hipStream_t s) {
    if (jl.total <= 0) return;
    // X, p, R, q read; X, R written; the next V-cycle's FP32 right-hand side and its
    // zeroed iterate written where they are separate arrays / read
    if (acct_add(jl.cells * (32.0 + 16.0 + (mixed ? 4.0 : 0.0) + (zero_z ? (mixed ? 4.0 : 8.0) : 0.0)))) return;
    const int g = blocks_for_xcd(jl.total, nblk);
    FLD_DISPATCH_DIM(dim, {
        if (mixed) hipLaunchKernelGGL((k_cg_update<D, true>), dim3(g), dim3(kBlock), 0, s, L, S, jl, fin, rtol, max_cycles, zero_z);
        else hipLaunchKernelGGL((k_cg_update<D, false>), dim3(g), dim3(kBlock), 0, s, L, S, jl, fin, rtol, max_cycles, zero_z);
    });
}

void launch_correct(int dim, bool mixed, const LevelDesc* L, const GridState* S, JobList jl, int nblk,
                    hipStream_t s) {
    if (jl.total <= 0) return;
    if (acct_add(jl.cells * (16.0 + (mixed ? 4.0 : 8.0)))) return;     // X and z read, X written
    const int g = blocks_for_xcd(jl.total, nblk);
    FLD_DISPATCH_DIM(dim, {
        if (mixed) hipLaunchKernelGGL((k_correct<D, true>), dim3(g), dim3(kBlock), 0, s, L, S, jl);
        else hipLaunchKernelGGL((k_correct<D, false>), dim3(g), dim3(kBlock), 0, s, L, S, jl);
    });
}

void launch_output(int dim, const LevelDesc* L, JobList jl, const StepIO* io, int nblk,
                   hipStream_t s) {
    if (jl.total <= 0) return;
    if (acct_add(jl.cells * 16.0)) return;                               // X read, E_out written
    const int g = blocks_for_xcd(jl.total, nblk);
    FLD_DISPATCH_DIM(dim, { hipLaunchKernelGGL((k_output<D>), dim3(g), dim3(kBlock), 0, s, L, jl, io); });
}

void launch_count(const GridState* S, int ngrids, Control* ctrl, hipStream_t s) {
    if (acct_add(0.0)) return;
    hipLaunchKernelGGL(k_count, dim3(1), dim3(kBlock), 0, s, S, ngrids, ctrl);
}

void launch_set_active(GridState* S, int ngrids, int value, hipStream_t s) {
    if (acct_add(0.0)) return;
    hipLaunchKernelGGL(k_set_active, dim3((ngrids + kBlock - 1) / kBlock), dim3(kBlock), 0, s, S, ngrids, value);
}

void launch_moments(int dim, const LevelDesc* L, JobList jl, const MomentsIO* io, double c, int limiter,
                    int nblk, hipStream_t s) {
    if (jl.total <= 0) return;
    const int g = blocks_for_xcd(jl.total, nblk);
    FLD_DISPATCH_DIM(dim, hipLaunchKernelGGL((k_moments<D>), dim3(g), dim3(kBlock), 0, s, L, jl, io, c, limiter));
}

static ExConst ex_const(double c, double a_rad, double c_v, int max_halley, double root_rtol) {
    const double cv2 = c_v * c_v;
    return ExConst{c, a_rad, cv2 * cv2, max_halley, root_rtol};
}

void launch_exchange(const ExchangeIO* io, int ngrids, int64_t max_n, double c, double a_rad,
                     double c_v, int max_halley, double root_rtol, Control* ctrl, int nblk,
                     hipStream_t s) {
    if (ngrids <= 0 || max_n <= 0) return;
    int64_t bx = (max_n + kBlock - 1) / kBlock;
    if (bx > nblk) bx = nblk;
    hipLaunchKernelGGL(k_exchange, dim3((unsigned)bx, (unsigned)ngrids), dim3(kBlock), 0, s, io,
                       ex_const(c, a_rad, c_v, max_halley, root_rtol), ctrl);
}

void launch_imex_point(const ImexIO* io, int ngrids, int64_t max_n, double c, double a_rad, double c_v,
                       int max_halley, double root_rtol, Control* ctrl, int nblk, hipStream_t s) {
    if (ngrids <= 0 || max_n <= 0) return;
    int64_t bx = (max_n + kBlock - 1) / kBlock;
    if (bx > nblk) bx = nblk;
    hipLaunchKernelGGL(k_imex_point, dim3((unsigned)bx, (unsigned)ngrids), dim3(kBlock), 0, s, io,
                       ex_const(c, a_rad, c_v, max_halley, root_rtol), ctrl);
}

}  // namespace fld
