// Host runtime of the FLD step: plans (multigrid hierarchies of one or many
// grids), the workspace layout inside caller-owned device memory, the launch
// work-lists, the V-cycle / defect-correction drivers with optional hipGraph
// replay, and the C ABI declared in include/fld.h.
//
// Nothing here allocates device memory: every device buffer lives in the
// workspace the caller binds (a torch tensor in the Python binding).  Host
// allocations are plain C++ containers plus a few pinned staging buffers.
#include "fld_internal.hpp"

#include <algorithm>
#include <cstddef>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <new>
#include <string>
#include <vector>

namespace fld {

thread_local std::string g_last_error;

void set_error(const char* where, hipError_t e) {
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s: %s", where, hipGetErrorString(e));
    g_last_error = buf;
}


namespace {

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess) { set_error("hipGetDevice", e); ok = false; prev = -1; return; }
        if (prev != dev && (e = hipSetDevice(dev)) != hipSuccess) { set_error("hipSetDevice", e); ok = false; }
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace

int validate_opts(const fld_opts& o) {
    if (!(o.c > 0.0) || !std::isfinite(o.c)) return FLD_ERR_INVALID_ARG;
    if (o.limiter < FLD_LIMITER_LP || o.limiter > FLD_LIMITER_LP_EXACT) return FLD_ERR_INVALID_ARG;
    for (int f = 0; f < 6; ++f) {
        if (o.bc[f] < 0) return FLD_ERR_INVALID_ARG;
        if (o.bc[f] != FLD_BC_ZERO_FLUX && o.bc[f] != FLD_BC_FIXED_GRADIENT && o.bc[f] != FLD_BC_DIRICHLET &&
            o.bc[f] != FLD_BC_PERIODIC && o.bc[f] != FLD_BC_CONTINUOUS)
            return FLD_ERR_UNSUPPORTED;
        // continuous faces make the operator unsymmetric: no conjugate gradients
        if (o.bc[f] == FLD_BC_CONTINUOUS && o.krylov) return FLD_ERR_INVALID_ARG;
        if (!std::isfinite(o.bc_grad[f])) return FLD_ERR_INVALID_ARG;
        if (o.bc[f] == FLD_BC_DIRICHLET && !(o.bc_value[f] >= 0.0 && std::isfinite(o.bc_value[f])))
            return FLD_ERR_INVALID_ARG;
    }
    for (int a = 0; a < 3; ++a)
        if ((o.bc[2 * a] == FLD_BC_PERIODIC) != (o.bc[2 * a + 1] == FLD_BC_PERIODIC)) return FLD_ERR_INVALID_ARG;
    if (o.precision != FLD_PREC_FP64 && o.precision != FLD_PREC_MIXED) return FLD_ERR_INVALID_ARG;
    if (!(o.rtol > 0.0) || !(o.rtol < 1.0)) return FLD_ERR_INVALID_ARG;
    if (o.max_cycles < 1 || o.max_cycles > 100000) return FLD_ERR_INVALID_ARG;
    if (o.nu1 < 0 || o.nu2 < 0 || o.nu1 + o.nu2 < 1 || o.nu1 > 16 || o.nu2 > 16) return FLD_ERR_INVALID_ARG;
    if (o.krylov && o.nu1 != o.nu2) return FLD_ERR_INVALID_ARG;   // CG needs a symmetric V-cycle
    if (o.krylov != 0 && o.krylov != 1) return FLD_ERR_INVALID_ARG;
    if (o.fused < 0 || o.fused > 3) return FLD_ERR_INVALID_ARG;
    if (o.autotune < 0 || o.autotune > 2) return FLD_ERR_INVALID_ARG;
    if (o.tile_rows != 0 && o.tile_rows != 4 && o.tile_rows != 8 && o.tile_rows != 16 && o.tile_rows != 32)
        return FLD_ERR_INVALID_ARG;
    if (o.tile_rows_coarse != 0 && o.tile_rows_coarse != 4 && o.tile_rows_coarse != 8 &&
        o.tile_rows_coarse != 16 && o.tile_rows_coarse != 32)
        return FLD_ERR_INVALID_ARG;
    if (o.tile_rows_up != 0 && o.tile_rows_up != 4 && o.tile_rows_up != 8 && o.tile_rows_up != 16 &&
        o.tile_rows_up != 32)
        return FLD_ERR_INVALID_ARG;
    if (o.tile_wide != 0 && o.tile_wide != 1) return FLD_ERR_INVALID_ARG;
    if (o.max_blocks < 0 || o.max_blocks > (1 << 20)) return FLD_ERR_INVALID_ARG;
    // the tuner picks the launch shape itself
    if (o.tile_depth != 0 && o.tile_depth != 16 && o.tile_depth != 32 && o.tile_depth != 64)
        return FLD_ERR_INVALID_ARG;
    if (o.fused3_levels < 0 || o.fused3_levels > 64) return FLD_ERR_INVALID_ARG;
    if (o.autotune && (o.tile_rows || o.tile_wide || o.max_blocks || o.tile_depth || o.fused3_levels ||
                       o.tile_rows_coarse || o.tile_rows_up))
        return FLD_ERR_INVALID_ARG;
    if (o.fmg != 0 && o.fmg != 1) return FLD_ERR_INVALID_ARG;
    if (o.fmg_depths < -1 || o.fmg_depths > 64) return FLD_ERR_INVALID_ARG;
    if (o.nu_coarse < 0 || o.nu_coarse > 16) return FLD_ERR_INVALID_ARG;
    if (o.coarse_op != FLD_COARSE_REDISCRETISED && o.coarse_op != FLD_COARSE_GALERKIN) return FLD_ERR_INVALID_ARG;
    return FLD_OK;
}

int validate_grid(const fld_grid& g) {
    if (g.ndim != 2 && g.ndim != 3) return FLD_ERR_INVALID_ARG;
    int64_t n = 1;
    for (int d = 0; d < g.ndim; ++d) {
        if (g.n[d] < 2 || g.n[d] > (1 << 20)) return FLD_ERR_INVALID_ARG;
        if (!(g.h[d] > 0.0) || !std::isfinite(g.h[d])) return FLD_ERR_INVALID_ARG;
        n *= g.n[d];
    }
    if (n > (int64_t(1) << 31) - 1) return FLD_ERR_INVALID_ARG;   // 32-bit tile/cell indices
    return FLD_OK;
}

namespace {

void finish_list(HostList& l, const std::vector<LevelDesc>& L, int (*tiles)(const LevelDesc&)) {
    l.prefix.assign(1, 0);
    for (int32_t li : l.levels) l.prefix.push_back(l.prefix.back() + tiles(L[li]));
}

int tiles_cell(const LevelDesc& d) { return cell_tiles(d.n); }
int tiles_l0(const LevelDesc& d) { return l0_tiles(d.n); }
int tiles_smooth(const LevelDesc& d) { return smooth_tiles(d.n); }
int tiles_one(const LevelDesc&) { return 1; }


// The level-0 cell kernels (coefficients, residual, CG vectors, output, moments) are
// streaming passes with a reduction per tile: they launch one workgroup per tile,
// whatever cap the stencil kernels are tuned to.  kCellBlocks bounds the plans whose
// CG scalars are formed inside the consuming kernels (every block then reads all of
// its grid's partials).
constexpr int kCellBlocks = 8192;
inline int cell_blocks(const Plan&) { return 1 << 30; }

// A fused 2D depth marches rows when its down pass has at least this many windows per
// compute unit (fld_opts.fused = 1).
constexpr int kMarchMinBlocks = 4;

// Fused-tile prefixes of the down / up lists (2D) and the sweep lists (3D) for the
// plan's launch shape.
void finish_fused(const Plan& p, DimLists& D) {
    D.fz_r.assign(D.sw3.size(), p.tile_depth);
    D.fz_s.assign(D.sw3.size(), p.tile_depth);
    // blocks run in rounds of one per compute unit, each round as long as a block's march
    // (fz planes plus its halo steps): the plane depth that needs the fewest block steps
    auto rounds = [&](const HostList& l, bool restr, int fz) {
        int64_t tiles = 0;
        for (int32_t li : l.levels) tiles += sweep3_tiles(p.levels[li].n, restr, fz);
        return ((tiles + p.ncu - 1) / p.ncu) * (fz + (restr ? 6 : 4));
    };
    for (size_t dpt = 0; dpt < D.sw3.size(); ++dpt) {
        HostList& a = D.sw3[dpt];
        HostList& r = D.sr3[dpt];
        // the finest depth's plain sweep marches the tuned depth; a coarser depth's, and
        // every restricting sweep (its narrower window makes more blocks), the depth of
        // fewest block steps among 8 .. 64 planes (the tuned depth on a tie)
        if (dpt > 0)
            for (int fz : {8, 16, 32, 64})
                if (rounds(a, false, fz) < rounds(a, false, D.fz_s[dpt])) D.fz_s[dpt] = fz;
        for (int fz : {8, 16, 32, 64})
            if (rounds(r, true, fz) < rounds(r, true, D.fz_r[dpt])) D.fz_r[dpt] = fz;
        a.prefix.assign(1, 0);
        r.prefix.assign(1, 0);
        for (int32_t li : a.levels)
            a.prefix.push_back(a.prefix.back() + sweep3_tiles(p.levels[li].n, false, D.fz_s[dpt]));
        for (int32_t li : r.levels)
            r.prefix.push_back(r.prefix.back() + sweep3_tiles(p.levels[li].n, true, D.fz_r[dpt]));
    }
    // a fused sweep marches through its planes in sequence, so a level needs many blocks
    // to fill the chip: by default only the leading depths whose plain sweep has at least
    // one block per two compute units run fused, the coarser ones per colour (at 256^3 the
    // two finest, as the autotuner also picks)
    // the last level-0 up sweep under FP64 CG also forms r . z; it marches a fixed plane
    // depth, so a grid's partials (one per window) do not depend on the tuned one
    D.rz3.levels = D.sw3.empty() ? std::vector<int32_t>{} : D.sw3[0].levels;
    D.rz3.prefix.assign(1, 0);
    for (int32_t li : D.rz3.levels)
        D.rz3.prefix.push_back(D.rz3.prefix.back() + sweep3_tiles(p.levels[li].n, false, kRz3Fz));
    const int nd = (int)D.sw3.size();
    if (p.sweep3_levels > 0) {
        D.levels3 = std::min(p.sweep3_levels, nd);
    } else {
        D.levels3 = 0;
        while (D.levels3 < nd && 2 * D.sw3[D.levels3].prefix.back() >= p.ncu) ++D.levels3;
    }
    D.thr_dn.assign(D.down2.size(), kBlock);
    D.thr_up.assign(D.up2.size(), kBlock);
    for (size_t dpt = 0; dpt < D.down2.size(); ++dpt) {
        const int n1 = dpt == 0 ? p.opts.nu1 : p.nuc1, n2 = dpt == 0 ? p.opts.nu2 : p.nuc2;
        const int fxd = fused_fx(2 * n1 + 1, p.tile_wide), fxu = fused_fx(2 * n2, p.tile_wide);
        HostList& dn = D.down2[dpt];
        HostList& up = D.up2[dpt];
        dn.prefix.assign(1, 0);
        up.prefix.assign(1, 0);
        const int rows = dpt == 0 ? p.tile_rows : p.tile_rows_c;
        const int rows_up = dpt == 0 ? p.tile_rows_u : p.tile_rows_c;
        for (int32_t li : dn.levels) dn.prefix.push_back(dn.prefix.back() + fused_tiles(p.levels[li].n, fxd, rows));
        for (int32_t li : up.levels) up.prefix.push_back(up.prefix.back() + fused_tiles(p.levels[li].n, fxu, rows_up));
        // a depth with no more tiles than compute units is bound by each tile's dependent
        // chain: 1024-thread tiles split it four ways; with more tiles, 256-thread tiles
        // keep more of them resident
        D.thr_dn[dpt] = dn.prefix.back() <= p.ncu ? 1024 : kBlock;
        D.thr_up[dpt] = up.prefix.back() <= p.ncu ? 1024 : kBlock;
    }
}

}  // namespace

// Coarsening rule: halve every axis while all are even and >= 4.
static void build_levels(Plan& p) {
    p.levels.clear();
    p.level0.clear();
    p.nlev.clear();
    p.ncell.clear();
    for (int g = 0; g < p.ngrids(); ++g) {
        const fld_grid& gr = p.grids[g];
        int32_t n[3] = {gr.n[0], gr.n[1], gr.ndim == 3 ? gr.n[2] : 1};
        double hinv[3] = {1.0 / gr.h[0], 1.0 / gr.h[1], gr.ndim == 3 ? 1.0 / gr.h[2] : 0.0};
        p.level0.push_back((int32_t)p.levels.size());
        p.ncell.push_back((int64_t)n[0] * n[1] * n[2]);
        int lev = 0;
        while (true) {
            LevelDesc d{};
            for (int a = 0; a < 3; ++a) { d.n[a] = n[a]; d.hinv[a] = hinv[a]; }
            d.ndim = gr.ndim;
            d.grid = g;
            d.sidx = g;
            d.level = lev;
            d.coarse = -1;
            d.fine = lev == 0 ? -1 : (int32_t)p.levels.size() - 1;
            for (int a = 0; a < gr.ndim; ++a)
                if (p.opts.bc[2 * a] == FLD_BC_PERIODIC) d.per_mask |= 1 << a;
            // continuous faces cut the finest operator only: the coarse levels keep the
            // zero-flux operator, which stays symmetric (the coarsest solve is CG); cutting
            // them too made the coarse corrections diverge on stiff grids
            for (int f = 0; f < 2 * gr.ndim; ++f)
                if (lev == 0 && p.opts.bc[f] == FLD_BC_CONTINUOUS) d.cont_mask |= 1 << f;
            if (lev == 0) {
                for (int f = 0; f < 2 * gr.ndim; ++f) {
                    const double G = p.opts.bc[f] == FLD_BC_FIXED_GRADIENT ? p.opts.bc_grad[f] : 0.0;
                    d.bcg[f] = G;
                    d.bcgh[f] = G * gr.h[f / 2];
                    if (G != 0.0) d.has_bc = 1;
                    if (p.opts.bc[f] == FLD_BC_DIRICHLET) {
                        d.dir_mask |= 1 << f;
                        d.bcv[f] = p.opts.bc_value[f];
                        d.has_bc = 1;
                    }
                    if (p.opts.bc[f] == FLD_BC_PERIODIC) d.has_bc = 1;   // wrapped gradient ghosts
                    if (p.opts.bc[f] == FLD_BC_CONTINUOUS) d.has_bc = 1; // extrapolated gradient ghosts
                }
            }
            if (lev > 0) p.levels.back().coarse = (int32_t)p.levels.size();
            p.levels.push_back(d);
            bool can = true;
            for (int a = 0; a < gr.ndim; ++a) can = can && (n[a] % 2 == 0) && (n[a] >= 4);
            if (!can) break;
            for (int a = 0; a < gr.ndim; ++a) { n[a] /= 2; hinv[a] *= 0.5; }
            ++lev;
        }
        p.nlev.push_back(lev + 1);
        for (int l = 0; l <= lev; ++l) p.levels[p.level0[g] + l].nlev = lev + 1;
    }
}

// First level of each grid's LDS tail: the finest level from which every coarser
// level (x, b, d face arrays) plus the coarsest CG's search direction fits the
// LDS budget, with a coarsest level small enough for the block CG.
static size_t tail_bytes(const Plan& p, int g, int t) {
    const int l0 = p.level0[g], L = p.nlev[g];
    const int dim = p.grids[g].ndim;
    const size_t word = p.mixed ? 4 : 8;
    size_t cells = 0;
    for (int l = t; l < L; ++l) {
        const LevelDesc& d = p.levels[l0 + l];
        cells += (size_t)(2 + dim + (p.has_dir ? 1 : 0)) * d.n[0] * d.n[1] * d.n[2];
    }
    const LevelDesc& c = p.levels[l0 + L - 1];
    cells += (size_t)c.n[0] * c.n[1] * c.n[2];
    return cells * word;
}

static void choose_tails(Plan& p) {
    p.tail_lev.assign(p.ngrids(), -1);
    for (int g = 0; g < p.ngrids(); ++g) {
        const int L = p.nlev[g];
        const LevelDesc& c = p.levels[p.level0[g] + L - 1];
        if ((int64_t)c.n[0] * c.n[1] * c.n[2] > kTailMaxCoarsest) continue;
        for (int t = 0; t < L; ++t) {
            if (tail_bytes(p, g, t) <= kTailLdsBudget) { p.tail_lev[g] = t; break; }
        }
    }
}

static void build_lists(Plan& p) {
    choose_tails(p);
    for (int di = 0; di < 2; ++di) {
        DimLists& D = p.dl[di];
        D = DimLists{};
        D.dim = di + 2;
        // wide (grid-parallel) depths of grid g: levels below its tail, or all but the coarsest
        auto wide = [&](int g) { return p.tail_lev[g] >= 0 ? p.tail_lev[g] : p.nlev[g] - 1; };
        int maxdepth = 0;
        for (int g = 0; g < p.ngrids(); ++g)
            if (p.grids[g].ndim == D.dim) maxdepth = std::max(maxdepth, wide(g));
        D.maxdepth = maxdepth;
        D.smooth.resize(maxdepth);
        D.restrict_.resize(maxdepth);
        D.prolong.resize(maxdepth);
        for (int g = 0; g < p.ngrids(); ++g) {
            if (p.grids[g].ndim != D.dim) continue;
            const int l0 = p.level0[g];
            D.l0_cell.levels.push_back(l0);
            for (int dpt = 0; dpt < wide(g); ++dpt) {
                D.smooth[dpt].levels.push_back(l0 + dpt);
                D.restrict_[dpt].levels.push_back(l0 + dpt);
                D.prolong[dpt].levels.push_back(l0 + dpt);
            }
            if (p.tail_lev[g] >= 0) {
                D.tail.levels.push_back(l0 + p.tail_lev[g]);
                D.tail_smem = std::max(D.tail_smem, tail_bytes(p, g, p.tail_lev[g]));
            } else {
                D.coarsest.levels.push_back(l0 + p.nlev[g] - 1);
            }
        }
        finish_list(D.l0_cell, p.levels, tiles_l0);
        finish_list(D.coarsest, p.levels, tiles_one);
        finish_list(D.tail, p.levels, tiles_one);
        // (built only for plans that start each step with full multigrid)
        const int nfrom = p.opts.fmg ? maxdepth : 0;
        D.tail_from.assign(nfrom, HostList{});
        D.coarsest_from.assign(nfrom, HostList{});
        for (int dpt = 0; dpt < nfrom; ++dpt) {
            for (int g = 0; g < p.ngrids(); ++g) {
                if (p.grids[g].ndim != D.dim || wide(g) <= dpt) continue;
                if (p.tail_lev[g] >= 0) D.tail_from[dpt].levels.push_back(p.level0[g] + p.tail_lev[g]);
                else D.coarsest_from[dpt].levels.push_back(p.level0[g] + p.nlev[g] - 1);
            }
            finish_list(D.tail_from[dpt], p.levels, tiles_one);
            finish_list(D.coarsest_from[dpt], p.levels, tiles_one);
        }
        // one same-address atomic per tile is cheaper than a finalize launch only for a few tiles
        int max_tiles = 0;
        for (size_t j = 0; j + 1 < D.l0_cell.prefix.size(); ++j)
            max_tiles = std::max(max_tiles, D.l0_cell.prefix[j + 1] - D.l0_cell.prefix[j]);
        D.fin_fused = max_tiles <= 32;
        // mid-sized plans: k_cg_pq and k_cg_update form beta and alpha from the partials
        // themselves (each block reads every partial of its grid: only for few tiles, and
        // only where launches are latency-bound: no more tiles in all than blocks launched)
        int64_t all_tiles = 0;
        for (size_t j = 0; j + 1 < D.l0_cell.prefix.size(); ++j) all_tiles += D.l0_cell.prefix[j + 1] - D.l0_cell.prefix[j];
        D.fold = !D.fin_fused && max_tiles <= kFoldMaxTiles && all_tiles <= kCellBlocks;
        // grids with zero-flux operators (no Dirichlet couplings, no wrapped neighbours) run
        // the CG direction update as a march when its reductions finish in a k_finalize
        // launch: 3D as a z-march, its plane depth balancing the blocks over the compute
        // units (rounds of one block per unit, fz + 2 steps each)
        D.pq3.prefix.assign(1, 0);
        bool even_rows = true;                       // 2D: rows of an even cell count load as pairs
        for (int32_t li : D.l0_cell.levels) even_rows = even_rows && p.levels[li].n[0] % 2 == 0;
        if (D.dim == 2 && even_rows && !p.nb_bc() && !D.fin_fused && !D.fold && !D.l0_cell.empty()) {
            // 2D: a row march, one wavefront per window of a fixed height, so that a grid's
            // p . q partials do not depend on what else the plan holds
            D.fz_pq = kPq2Rows;
            D.pq3.levels = D.l0_cell.levels;
            for (int32_t li : D.pq3.levels) D.pq3.prefix.push_back(D.pq3.prefix.back() + pq2_tiles(p.levels[li].n, D.fz_pq));
        }
        if (D.dim == 3 && !p.nb_bc() && !D.fin_fused && !D.fold && !D.l0_cell.empty()) {
            int64_t best = -1;
            for (int fz : {8, 16, 32, 64}) {
                int64_t tiles = 0;
                for (int32_t li : D.l0_cell.levels) tiles += pq3_tiles(p.levels[li].n, fz);
                const int64_t cost = ((tiles + p.ncu - 1) / p.ncu) * (fz + 2);
                if (best < 0 || cost < best) { best = cost; D.fz_pq = fz; }
            }
            D.pq3.levels = D.l0_cell.levels;
            D.pq3.prefix.assign(1, 0);
            for (int32_t li : D.pq3.levels) D.pq3.prefix.push_back(D.pq3.prefix.back() + pq3_tiles(p.levels[li].n, D.fz_pq));
        }
        // the fused level kernels know no Dirichlet couplings or wrapped neighbours: such plans
        // sweep per colour
        D.fused = D.dim == 2 && p.opts.fused && !p.nb_bc() && fused2_supported(p.opts.nu1) &&
                  fused2_supported(p.opts.nu2) && fused2_supported(p.nuc1) && fused2_supported(p.nuc2);
        D.down2.resize(D.fused ? maxdepth : 0);
        D.up2.resize(D.fused ? maxdepth : 0);
        D.mdn.resize(D.fused ? maxdepth : 0);
        D.mup.resize(D.fused ? maxdepth : 0);
        D.march.assign(D.fused ? maxdepth : 0, 0);
        D.mfz.assign(D.fused ? maxdepth : 0, kMarchFz);
        for (int dpt = 0; dpt < (int)D.down2.size(); ++dpt) {
            D.down2[dpt].levels = D.smooth[dpt].levels;
            D.up2[dpt].levels = D.smooth[dpt].levels;
            // row-marching windows: no rows recomputed, so they pay where a depth has many
            // windows to keep every compute unit busy (fused = 3 forces them, 2 forbids them)
            const int n1 = dpt == 0 ? p.opts.nu1 : p.nuc1, n2 = dpt == 0 ? p.opts.nu2 : p.nuc2;
            HostList& md = D.mdn[dpt];
            HostList& mu = D.mup[dpt];
            md.levels = mu.levels = D.smooth[dpt].levels;
            // windows of kMarchFz rows where they are many; of kMarchFzShort rows where that
            // doubles them to enough and the levels fill the windows (a single 1024^2 grid's
            // finest level: 576 windows of 16 rows, 12.5 us for its up pass against 15.0 us
            // with tiles; small levels in 128-column windows are mostly empty)
            int64_t w32 = 0, w16 = 0, cells = 0;
            for (int32_t li : md.levels) {
                w32 += march_tiles(p.levels[li].n, n1, true, kMarchFz);
                w16 += march_tiles(p.levels[li].n, n1, true, kMarchFzShort);
                cells += (int64_t)p.levels[li].n[0] * p.levels[li].n[1];
            }
            const bool many = w32 >= kMarchMinBlocks * p.ncu;
            const bool full = 4 * cells >= 3 * w16 * (int64_t)march_fx(n1, true) * kMarchFzShort;
            const bool enough = w16 >= kMarchMinBlocks / 2 * p.ncu && full;
            D.mfz[dpt] = (many || !enough) ? kMarchFz : kMarchFzShort;
            D.march[dpt] = p.opts.fused == 3 || (p.opts.fused == 1 && (many || enough));
            md.prefix.assign(1, 0);
            mu.prefix.assign(1, 0);
            for (int32_t li : md.levels)
                md.prefix.push_back(md.prefix.back() + march_tiles(p.levels[li].n, n1, true, D.mfz[dpt]));
            for (int32_t li : mu.levels)
                mu.prefix.push_back(mu.prefix.back() + march_tiles(p.levels[li].n, n2, false, D.mfz[dpt]));
        }
        // fused 3D sweeps alternate between x and xs, so the V-cycle's sweep count must be
        // even for its result to end in x
        D.fused3 = D.dim == 3 && p.opts.fused && !p.nb_bc() && fused3_supported(p.mixed) &&
                   p.opts.nu1 >= 1 &&
                   p.opts.nu2 >= 1 && (p.opts.nu1 + p.opts.nu2) % 2 == 0 && p.nuc1 >= 1 && p.nuc2 >= 1 &&
                   (p.nuc1 + p.nuc2) % 2 == 0;
        D.sw3.resize(D.fused3 ? maxdepth : 0);
        D.sr3.resize(D.fused3 ? maxdepth : 0);
        for (int dpt = 0; dpt < (int)D.sw3.size(); ++dpt) {
            D.sw3[dpt].levels = D.smooth[dpt].levels;
            D.sr3[dpt].levels = D.smooth[dpt].levels;
        }
        finish_fused(p, D);
        for (int dpt = 0; dpt < maxdepth; ++dpt) {
            finish_list(D.smooth[dpt], p.levels, tiles_smooth);
            finish_list(D.prolong[dpt], p.levels, tiles_cell);
            // restriction / coarsening tiles cover the coarse level
            HostList& r = D.restrict_[dpt];
            r.prefix.assign(1, 0);
            for (int32_t li : r.levels) r.prefix.push_back(r.prefix.back() + cell_tiles(p.levels[p.levels[li].coarse].n));
        }
        // coarse face weights are needed on every level, tails included
        D.coarsen.resize(0);
        int depth_all = 0;
        for (int g = 0; g < p.ngrids(); ++g)
            if (p.grids[g].ndim == D.dim) depth_all = std::max(depth_all, p.nlev[g] - 1);
        D.coarsen.resize(depth_all);
        for (int g = 0; g < p.ngrids(); ++g) {
            if (p.grids[g].ndim != D.dim) continue;
            for (int dpt = 0; dpt < p.nlev[g] - 1; ++dpt) D.coarsen[dpt].levels.push_back(p.level0[g] + dpt);
        }
        for (auto& c : D.coarsen) {
            c.prefix.assign(1, 0);
            for (int32_t li : c.levels) c.prefix.push_back(c.prefix.back() + cell_tiles(p.levels[p.levels[li].coarse].n));
        }
    }
}

static void layout(Plan& p);

int plan_init(Plan& p, const fld_grid* grids, int ngrids, const fld_opts& opts) {
    int rc = validate_opts(opts);
    if (rc != FLD_OK) return rc;
    for (int g = 0; g < ngrids; ++g)
        if ((rc = validate_grid(grids[g])) != FLD_OK) return rc;
    // host-only: a plan can be built without a usable device; bind reports HIP failures
    if (hipGetDevice(&p.device) != hipSuccess) p.device = 0;
    p.opts = opts;
    p.mixed = opts.precision == FLD_PREC_MIXED;
    p.krylov = opts.krylov != 0;
    p.nuc1 = opts.nu_coarse ? opts.nu_coarse : opts.nu1;
    p.nuc2 = opts.nu_coarse ? opts.nu_coarse : opts.nu2;
    p.has_dir = false;
    p.has_per = false;
    p.has_cont = false;
    p.any_bc = false;
    for (int f = 0; f < 6; ++f) {
        for (int g = 0; g < ngrids; ++g) {
            if (f >= 2 * grids[g].ndim) continue;
            if (opts.bc[f] == FLD_BC_DIRICHLET) p.has_dir = true;
            if (opts.bc[f] == FLD_BC_PERIODIC) p.has_per = true;
            if (opts.bc[f] == FLD_BC_CONTINUOUS) p.has_cont = true;
            if (opts.bc[f] != FLD_BC_ZERO_FLUX) p.any_bc = true;
        }
    }
    p.grids.assign(grids, grids + ngrids);
    for (auto& g : p.grids)
        if (g.ndim == 2) { g.n[2] = 1; g.h[2] = 1.0; }
    p.tile_wide = opts.tile_wide;
    p.tile_rows = opts.tile_rows ? opts.tile_rows : 8;
    p.tile_rows_c = opts.tile_rows_coarse ? opts.tile_rows_coarse : p.tile_rows;
    p.tile_rows_u = opts.tile_rows_up ? opts.tile_rows_up : p.tile_rows;
    p.nblk = opts.max_blocks ? opts.max_blocks : 2048;
    p.tile_depth = opts.tile_depth ? opts.tile_depth : 32;
    {   // compute units of the current device (the plan's), for balancing block counts
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            p.ncu = cus;
        else
            (void)hipGetLastError();
    }
    p.sweep3_levels = opts.fused3_levels;
    if (opts.fused && fused2_supported(opts.nu1) && fused2_supported(opts.nu2) && fused2_supported(p.nuc1) &&
        fused2_supported(p.nuc2) &&
        !(fused2_shape_ok(p.mixed, opts.nu1, p.tile_wide, p.tile_rows, true) &&
          fused2_shape_ok(p.mixed, opts.nu2, p.tile_wide, p.tile_rows, false) &&
          fused2_shape_ok(p.mixed, p.nuc1, p.tile_wide, p.tile_rows_c, true) &&
          fused2_shape_ok(p.mixed, p.nuc2, p.tile_wide, p.tile_rows_c, false) &&
          fused2_shape_ok(p.mixed, opts.nu2, p.tile_wide, p.tile_rows_u, false)))
        return FLD_ERR_INVALID_ARG;                            // the tile does not fit the LDS
    build_levels(p);
    build_lists(p);
    layout(p);
    p.io_host.assign(ngrids, StepIO{});
    p.st_host.assign(ngrids, GridState{});
    return FLD_OK;
}

static void layout(Plan& p) {
    const int G = p.ngrids();
    const size_t NL = p.levels.size();
    size_t off = 0;
    p.off_levels = off; off = align_up(off + NL * sizeof(LevelDesc));
    p.off_state = off;  off = align_up(off + G * sizeof(GridState));
    p.off_stepio = off; off = align_up(off + G * sizeof(StepIO));
    p.off_exio = off;   off = align_up(off + Plan::kExSlots * G * sizeof(ExchangeIO));
    p.off_moio = off;   off = align_up(off + Plan::kExSlots * G * sizeof(MomentsIO));
    p.off_imio = off;   off = align_up(off + Plan::kImStages * G * sizeof(ImexIO));
    p.off_ctrl = off;   off = align_up(off + sizeof(Control));
    auto place_list = [&](HostList& l) {
        l.off_levels = off; off = align_up(off + std::max<size_t>(1, l.levels.size()) * sizeof(int32_t));
        l.off_prefix = off; off = align_up(off + l.prefix.size() * sizeof(int32_t));
    };
    for (auto& D : p.dl) {
        place_list(D.l0_cell);
        place_list(D.pq3);
        place_list(D.rz3);
        place_list(D.coarsest);
        place_list(D.tail);
        for (auto& l : D.coarsen) place_list(l);
        for (auto& l : D.down2) place_list(l);
        for (auto& l : D.up2) place_list(l);
        for (auto& l : D.mdn) place_list(l);
        for (auto& l : D.mup) place_list(l);
        for (auto& l : D.sw3) place_list(l);
        for (auto& l : D.sr3) place_list(l);
        for (auto& l : D.smooth) place_list(l);
        for (auto& l : D.restrict_) place_list(l);
        for (auto& l : D.prolong) place_list(l);
        for (auto& l : D.tail_from) place_list(l);
        for (auto& l : D.coarsest_from) place_list(l);
    }
    p.table_bytes = off;
    p.foff.assign(NL, Plan::FieldOff{});
    p.field_off.assign(G, 0);
    p.field_bytes.assign(G, 0);
    // each grid's fields are laid out from its own origin (offset 0), so a grid can
    // live at any address (the server places requests in its arena)
    size_t goff = 0;
    auto take = [&](size_t bytes) { size_t o = goff; goff = align_up(goff + bytes); return o; };
    for (size_t li = 0; li < NL; ++li) {
        if (p.levels[li].level == 0) goff = 0;
        const int gcur = p.levels[li].grid;
        const LevelDesc& d = p.levels[li];
        Plan::FieldOff& f = p.foff[li];
        const size_t n = (size_t)d.n[0] * d.n[1] * d.n[2];
        const bool lev0 = d.level == 0;
        // FP64 weights at every level (coarse weights derive from them)
        for (int a = 0; a < d.ndim; ++a) f.w[a] = take(n * 8);
        if (p.has_dir) {
            f.ad = take(n * 8);
            if (p.mixed) f.ad32 = take(n * 4);
        }
        if (lev0) {
            // outer FP64 iteration: iterate, right-hand side, residual (+ CG vectors)
            f.lev0 = true;
            f.X = take(n * 8);
            f.B0 = take(n * 8);
            f.R = take(n * 8);
            if (p.krylov) {
                f.has_cg = true;
                f.P[0] = take(n * 8);
                f.P[1] = take(n * 8);
                f.Q = take(n * 8);
            }
            f.has_part = true;
            f.part = take(2 * (size_t)l0_tiles(d.n) * 8);
        }
        if (!p.mixed) {
            f.has_x = f.has_b = true;
            if (lev0) {
                // the V-cycle runs on (Z, R) under CG and on (X, B0) otherwise
                f.x = p.krylov ? take(n * 8) : f.X;
                f.b = p.krylov ? f.R : f.B0;
            } else {
                f.x = take(n * 8);
                f.b = take(n * 8);
            }
        } else {
            f.has_x32 = true;
            f.x32 = take(n * 4);
            f.b32 = take(n * 4);
            for (int a = 0; a < d.ndim; ++a) f.w32[a] = take(n * 4);
        }
        if (d.coarse < 0 && n > (size_t)kCoarseMaxLDS) {
            f.has_scratch = true;
            f.scratch = take(4 * n * 8);
        }
        // fused levels (every level with a coarser one) keep the down pass's output apart
        if (d.coarse >= 0 && ((d.ndim == 2 && p.dl[0].fused) || (d.ndim == 3 && p.dl[1].fused3))) {
            f.has_xs = true;
            f.xs = take(n * (p.mixed ? 4 : 8));
        }
        p.field_bytes[gcur] = goff;
    }
    for (int g = 0; g < G; ++g) {
        p.field_off[g] = off;
        if (p.field_base.empty()) off = align_up(off + p.field_bytes[g]);
    }
    p.ws_bytes = off;
}

// The multigrid part of one V-cycle of one dimension's grids (FP64 mode: on the
// solution, or on the CG preconditioner's iterate; mixed: the FP32 correction
// solve of the current residual).  Reads the solver state, never writes it.
// d0 > 0 runs the V-cycle of the levels from depth d0 down (a full-multigrid
// stage) over the grids with a level there, with the given tail / coarsest lists;
// load0: the level at d0 starts from its stored iterate instead of zero.
static void enqueue_mg_from(Plan& p, DimLists& D, hipStream_t s, int d0, int load0, const JobList& tail,
                            const JobList& coarsest, bool rz0 = false) {
    const bool f32 = p.mixed;
    const int plain64 = (!p.krylov && !p.mixed) ? 1 : 0;   // level-0 V-cycle starts from the iterate
    const int dim = D.dim;
    // fused 3D sweeps on the leading depths: sweep k of a level's V-cycle (1-based)
    // reads x and writes xs when k is odd, the reverse when k is even; nu1 + nu2 is
    // even, so the level's result ends in x
    const int L3 = (D.fused3 && p.sweep3) ? D.levels3 : 0;

    for (int d = d0; d < D.maxdepth; ++d) {
        const int nu1 = d == 0 ? p.opts.nu1 : p.nuc1;
        if (d < L3) {
            for (int k = 1; k <= nu1; ++k) {
                const bool load = k > 1 || (d == d0 && load0);
                const bool restr = k == nu1;
                const int mode = restr ? (load ? 2 : 3) : (load ? 0 : 1);
                launch_sweep3(f32, p.dL, p.dS, restr ? D.sr3[d].dev : D.sw3[d].dev, mode, 0, k % 2 == 0,
                              restr ? D.fz_r[d] : D.fz_s[d], p.nblk, s);
            }
            continue;
        }
        if (D.fused && D.march[d]) {
            launch_march2(f32, p.dL, p.dS, D.mdn[d].dev, nu1, 1, d == d0 ? load0 : 0, D.mfz[d], p.nblk, s);
            continue;
        }
        if (D.fused) {
            launch_down2(f32, p.dL, p.dS, D.down2[d].dev, nu1, d == d0 ? load0 : 0, p.tile_wide,
                         d == 0 ? p.tile_rows : p.tile_rows_c, D.thr_dn[d], p.nblk, s);
            continue;
        }
        for (int it = 0; it < nu1; ++it) {
            launch_smooth(dim, f32, p.dL, p.dS, D.smooth[d].dev, 0, p.nblk, s);
            launch_smooth(dim, f32, p.dL, p.dS, D.smooth[d].dev, 1, p.nblk, s);
        }
        launch_restrict(dim, f32, p.dL, p.dS, D.restrict_[d].dev, p.nblk, s);
    }
    // the tail's levels are below the finest unless the whole grid lives in it
    launch_tail(dim, f32, p.nb_bc(), p.dL, p.dS, tail, D.tail_smem, p.nuc1, p.nuc2, plain64, s);
    launch_coarse_solve(dim, f32, p.dL, p.dS, coarsest, s);
    for (int d = D.maxdepth - 1; d >= d0; --d) {
        const int nu1 = d == 0 ? p.opts.nu1 : p.nuc1, nu2 = d == 0 ? p.opts.nu2 : p.nuc2;
        if (d < L3) {
            for (int k = nu1 + 1; k <= nu1 + nu2; ++k) {
                const int mode = k == nu1 + 1 ? 4 : 0;
                const bool rz = rz0 && d == 0 && k == nu1 + nu2 && mode == 0;
                launch_sweep3(f32, p.dL, p.dS, rz ? D.rz3.dev : D.sw3[d].dev, mode, 1, k % 2 == 0,
                              rz ? kRz3Fz : D.fz_s[d], p.nblk, s, rz ? 1 : 0);
            }
            continue;
        }
        if (D.fused && D.march[d]) {
            launch_march2(f32, p.dL, p.dS, D.mup[d].dev, nu2, 0, 0, D.mfz[d], p.nblk, s, rz0 && d == 0 ? 1 : 0);
            continue;
        }
        if (D.fused) {
            launch_up2(f32, p.dL, p.dS, D.up2[d].dev, nu2, p.tile_wide, d == 0 ? p.tile_rows_u : p.tile_rows_c,
                       D.thr_up[d], p.nblk, s);
            continue;
        }
        launch_prolong(dim, f32, p.dL, p.dS, D.prolong[d].dev, p.nblk, s);
        for (int it = 0; it < nu2; ++it) {
            launch_smooth(dim, f32, p.dL, p.dS, D.smooth[d].dev, 1, p.nblk, s);
            launch_smooth(dim, f32, p.dL, p.dS, D.smooth[d].dev, 0, p.nblk, s);
        }
    }
}

// Whether the first smoothing kernel of level 0 in a V-cycle reads the iterate (the
// per-colour kernels do; fused sweeps from zero and the fused 2D down pass do not).
static bool level0_reads_iterate(const Plan& p, const DimLists& D) {
    if (D.dim == 3) return !(D.fused3 && p.sweep3 && D.levels3 >= 1);
    return !D.fused;
}

static void enqueue_mg(Plan& p, DimLists& D, hipStream_t s, bool rz0 = false) {
    const int plain64 = (!p.krylov && !p.mixed) ? 1 : 0;
    enqueue_mg_from(p, D, s, 0, plain64, D.tail.dev, D.coarsest.dev, rz0);
}

// Whether the level-0 up pass of the CG preconditioner also forms the r . z partials
// (one per window, summed by a k_finalize over the pass's list): FP64 (b is r), reductions
// that finish in a k_finalize launch anyway, and every grid's level 0 in the pass (a grid
// without a coarse level has none): in 2D a row march, in 3D a fused last sweep (a plain
// one: nu2 >= 2).
static bool rz_in_march(const Plan& p, const DimLists& D) {
    if (!p.krylov || p.mixed || D.fin_fused || D.fold) return false;
    if (D.dim == 3)
        return D.fused3 && p.sweep3 && D.levels3 >= 1 && p.opts.nu2 >= 2 &&
               D.sw3[0].levels.size() == D.l0_cell.levels.size();
    return D.fused && !D.march.empty() && D.march[0] && D.mfz[0] == kMarchFz &&
           D.mup[0].levels.size() == D.l0_cell.levels.size();
}
static const JobList& rz_list(const DimLists& D) { return D.dim == 3 ? D.rz3.dev : D.mup[0].dev; }

// Full-multigrid cycle on the V-cycle's level-0 arrays (Sec. 3.4 starts each solve
// with one): the right-hand side averaged down to every grid's deepest wide level,
// the tail V-cycle / coarsest solve there from zero, then per depth, coarse to
// fine, the interpolated coarser solution as the start of one V-cycle of that
// depth's levels.
static void enqueue_fmg(Plan& p, DimLists& D, hipStream_t s) {
    const bool f32 = p.mixed;
    for (int d = 0; d < D.maxdepth; ++d) launch_restrict_rhs(D.dim, f32, p.dL, p.dS, D.restrict_[d].dev, p.nblk, s);
    const int plain64 = (!p.krylov && !p.mixed) ? 1 : 0;
    launch_tail(D.dim, f32, p.nb_bc(), p.dL, p.dS, D.tail.dev, D.tail_smem, p.nuc1, p.nuc2, plain64, s);
    launch_coarse_solve(D.dim, f32, p.dL, p.dS, D.coarsest.dev, s);
    // by dimension: the 3D stages below the two finest still pay for their V-cycles
    const int fd = p.opts.fmg_depths >= 0 ? p.opts.fmg_depths : (D.dim == 3 ? 3 : 2);
    const int nv = fd > 0 ? fd : D.maxdepth;
    for (int d = D.maxdepth - 1; d >= 0; --d) {
        launch_fmg_interp(D.dim, f32, p.dL, p.dS, D.prolong[d].dev, p.nblk, s);
        if (d < nv) enqueue_mg_from(p, D, s, d, 1, D.tail_from[d].dev, D.coarsest_from[d].dev);
    }
}

// The first outer iteration of a step with the full-multigrid start: the FMG cycle
// in place of the V-cycle, then the FP64 update and residual.  Under CG the result
// corrects the iterate and CG restarts from its true residual.
static void enqueue_fmg_cycle(Plan& p, hipStream_t s) {
    for (auto& D : p.dl) {
        if (D.l0_cell.empty()) continue;
        enqueue_fmg(p, D, s);
        const JobList& l0 = D.l0_cell.dev;
        const bool corr = p.krylov || p.mixed;
        if (corr) launch_correct(D.dim, p.mixed, p.dL, p.dS, l0, cell_blocks(p), s);
        const int fin = p.krylov ? FIN_R_FMG : FIN_R_CYCLE;
        launch_residual(D.dim, p.mixed, p.dL, p.dS, l0, 0, corr ? 1 : 0, D.fin_fused ? fin : -1, p.opts.rtol,
                        p.opts.max_cycles, cell_blocks(p), s);
        if (!D.fin_fused) launch_finalize(p.dL, p.dS, l0, fin, p.opts.rtol, p.opts.max_cycles, s);
    }
}

void plan_vcycle_mg(Plan& p, hipStream_t s) {
    for (auto& D : p.dl)
        if (!D.l0_cell.empty()) enqueue_mg(p, D, s);
}

// Enqueue one outer iteration: the V-cycle followed by the CG update (or the
// defect correction) with the FP64 residual and stop test.
static void enqueue_cycle(Plan& p, hipStream_t s) {
    for (auto& D : p.dl) {
        if (D.l0_cell.empty()) continue;
        const int dim = D.dim;
        const bool rzm = rz_in_march(p, D);
        enqueue_mg(p, D, s, rzm);
        const JobList& l0 = D.l0_cell.dev;
        if (p.krylov) {
            const double rt = p.opts.rtol;
            const int mc = p.opts.max_cycles;
            const bool ff = D.fin_fused;
            // the r.z and p.q reductions finish in the last tile's block (few tiles), in the
            // next kernel's blocks (D.fold), or in a k_finalize launch
            const bool fin_launch = !ff && !D.fold;
            if (rzm) {
                launch_finalize(p.dL, p.dS, rz_list(D), FIN_RZ, rt, mc, s);
            } else {
                launch_cg_rz(dim, p.mixed, p.dL, p.dS, l0, ff ? FIN_RZ : -1, rt, mc, cell_blocks(p), s);
                if (fin_launch) launch_finalize(p.dL, p.dS, l0, FIN_RZ, rt, mc, s);
            }
            if (!D.pq3.empty()) {
                if (dim == 3) launch_cg_pq3(p.mixed, p.dL, p.dS, D.pq3.dev, D.fz_pq, cell_blocks(p), s);
                else launch_cg_pq2m(p.mixed, p.dL, p.dS, D.pq3.dev, D.fz_pq, s);
                launch_finalize(p.dL, p.dS, D.pq3.dev, FIN_PQ, rt, mc, s);
            } else {
                launch_cg_pq(dim, p.mixed, p.dL, p.dS, l0, ff ? FIN_PQ : (D.fold ? kFinFold : -1), rt, mc,
                             cell_blocks(p), s);
                if (fin_launch) launch_finalize(p.dL, p.dS, l0, FIN_PQ, rt, mc, s);
            }
            launch_cg_update(dim, p.mixed, p.dL, p.dS, l0, ff ? FIN_CG : (D.fold ? kFinFold : -1), rt, mc,
                             level0_reads_iterate(p, D) ? 1 : 0, cell_blocks(p), s);
            if (!ff) launch_finalize(p.dL, p.dS, l0, FIN_CG, rt, mc, s);
        } else {
            if (p.mixed) launch_correct(dim, true, p.dL, p.dS, l0, cell_blocks(p), s);
            launch_residual(dim, p.mixed, p.dL, p.dS, l0, 0, p.mixed ? 1 : 0, D.fin_fused ? FIN_R_CYCLE : -1,
                            p.opts.rtol, p.opts.max_cycles, cell_blocks(p), s);
            if (!D.fin_fused) launch_finalize(p.dL, p.dS, l0, FIN_R_CYCLE, p.opts.rtol, p.opts.max_cycles, s);
        }
    }
}

static int capture_graph(Plan& p) {
    if (p.graph_exec) { (void)hipGraphExecDestroy(p.graph_exec); p.graph_exec = nullptr; }
    if (p.graph) { (void)hipGraphDestroy(p.graph); p.graph = nullptr; }
    if (p.fmg_graph_exec) { (void)hipGraphExecDestroy(p.fmg_graph_exec); p.fmg_graph_exec = nullptr; }
    if (p.fmg_graph) { (void)hipGraphDestroy(p.fmg_graph); p.fmg_graph = nullptr; }
    if (!p.cap_stream) FLD_HIP(hipStreamCreateWithFlags(&p.cap_stream, hipStreamNonBlocking));
    FLD_HIP(hipStreamBeginCapture(p.cap_stream, hipStreamCaptureModeThreadLocal));
    enqueue_cycle(p, p.cap_stream);
    hipGraph_t g = nullptr;
    FLD_HIP(hipStreamEndCapture(p.cap_stream, &g));
    p.graph = g;
    FLD_HIP(hipGraphInstantiate(&p.graph_exec, p.graph, nullptr, nullptr, 0));
    if (p.opts.fmg) {
        FLD_HIP(hipStreamBeginCapture(p.cap_stream, hipStreamCaptureModeThreadLocal));
        enqueue_fmg_cycle(p, p.cap_stream);
        hipGraph_t f = nullptr;
        FLD_HIP(hipStreamEndCapture(p.cap_stream, &f));
        p.fmg_graph = f;
        FLD_HIP(hipGraphInstantiate(&p.fmg_graph_exec, p.fmg_graph, nullptr, nullptr, 0));
    }
    return FLD_OK;
}

static int upload_list(Plan& p, HostList& l) {
    int32_t* lv = reinterpret_cast<int32_t*>(p.ws + l.off_levels);
    int32_t* pf = reinterpret_cast<int32_t*>(p.ws + l.off_prefix);
    if (!l.levels.empty())
        FLD_HIP(hipMemcpy(lv, l.levels.data(), l.levels.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    FLD_HIP(hipMemcpy(pf, l.prefix.data(), l.prefix.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    int64_t cells = 0;
    for (int32_t li : l.levels) cells += (int64_t)p.levels[li].n[0] * p.levels[li].n[1] * p.levels[li].n[2];
    l.dev = JobList{lv, pf, (int32_t)l.levels.size(), l.prefix.back(), cells, l.levels.empty() ? -1 : l.levels[0], 0};
    return FLD_OK;
}

LaunchShape plan_shape(const Plan& p) {
    return LaunchShape{p.tile_wide, p.tile_rows, p.nblk, p.tile_depth, p.sweep3, p.sweep3_levels, p.tile_rows_c,
                       p.tile_rows_u};
}

int plan_set_shape(Plan& p, const LaunchShape& sh) {
    if (!p.ws) return FLD_ERR_NO_WORKSPACE;
    for (auto& D : p.dl)
        if (D.fused && !(fused2_shape_ok(p.mixed, p.opts.nu1, sh.wide, sh.rows, true) &&
                         fused2_shape_ok(p.mixed, p.opts.nu2, sh.wide, sh.rows, false) &&
                         fused2_shape_ok(p.mixed, p.nuc1, sh.wide, sh.rows_c, true) &&
                         fused2_shape_ok(p.mixed, p.nuc2, sh.wide, sh.rows_c, false) &&
                         fused2_shape_ok(p.mixed, p.opts.nu2, sh.wide, sh.rows_u, false)))
            return FLD_ERR_INVALID_ARG;
    if (sh.nblk < 1 || (sh.depth != 16 && sh.depth != 32 && sh.depth != 64) || (sh.sweep3 != 0 && sh.sweep3 != 1) ||
        sh.levels3 < 0)
        return FLD_ERR_INVALID_ARG;
    p.tile_wide = sh.wide;
    p.tile_rows = sh.rows;
    p.tile_rows_c = sh.rows_c;
    p.tile_rows_u = sh.rows_u;
    p.nblk = sh.nblk;
    p.tile_depth = sh.depth;
    p.sweep3 = sh.sweep3;
    p.sweep3_levels = sh.levels3;
    for (auto& D : p.dl) {
        finish_fused(p, D);
        int rc;
        for (auto& l : D.down2) if ((rc = upload_list(p, l)) != FLD_OK) return rc;
        for (auto& l : D.up2) if ((rc = upload_list(p, l)) != FLD_OK) return rc;
        for (auto& l : D.sw3) if ((rc = upload_list(p, l)) != FLD_OK) return rc;
        for (auto& l : D.sr3) if ((rc = upload_list(p, l)) != FLD_OK) return rc;
    }
    return FLD_OK;
}

// Copy a list into the table image and point its JobList at the device copy.
static void stage_list(Plan& p, HostList& l, char* img) {
    if (!l.levels.empty())
        std::memcpy(img + l.off_levels, l.levels.data(), l.levels.size() * sizeof(int32_t));
    std::memcpy(img + l.off_prefix, l.prefix.data(), l.prefix.size() * sizeof(int32_t));
    int64_t cells = 0;
    for (int32_t li : l.levels) cells += (int64_t)p.levels[li].n[0] * p.levels[li].n[1] * p.levels[li].n[2];
    l.dev = JobList{reinterpret_cast<int32_t*>(p.ws + l.off_levels), reinterpret_cast<int32_t*>(p.ws + l.off_prefix),
                    (int32_t)l.levels.size(), l.prefix.back(), cells, l.levels.empty() ? -1 : l.levels[0], 0};
}

int plan_bind(Plan& p, void* dev, size_t bytes, const GridState* init) {
    if (!dev) return FLD_ERR_INVALID_ARG;
    if (bytes < p.ws_bytes) return FLD_ERR_NO_WORKSPACE;
    if ((reinterpret_cast<uintptr_t>(dev) % kAlign) != 0) return FLD_ERR_INVALID_ARG;
    p.ws = static_cast<char*>(dev);
    char* const tab = p.ws;
    p.dL = reinterpret_cast<LevelDesc*>(tab + p.off_levels);
    p.dS = p.ext_state ? p.ext_state : reinterpret_cast<GridState*>(tab + p.off_state);
    p.dIO = reinterpret_cast<StepIO*>(tab + p.off_stepio);
    p.dEx = reinterpret_cast<ExchangeIO*>(tab + p.off_exio);
    p.dMo = reinterpret_cast<MomentsIO*>(tab + p.off_moio);
    p.dIm = reinterpret_cast<ImexIO*>(tab + p.off_imio);
    p.dCtrl = reinterpret_cast<Control*>(tab + p.off_ctrl);
    for (size_t li = 0; li < p.levels.size(); ++li) {
        LevelDesc& d = p.levels[li];
        const Plan::FieldOff& f = p.foff[li];
        char* const ws = p.field_base.empty() ? p.ws + p.field_off[d.grid] : p.field_base[d.grid];
        for (int a = 0; a < 3; ++a) {
            d.w[a] = a < d.ndim ? reinterpret_cast<double*>(ws + f.w[a]) : nullptr;
            d.w32[a] = (p.mixed && a < d.ndim) ? reinterpret_cast<float*>(ws + f.w32[a]) : nullptr;
        }
        d.x = f.has_x ? reinterpret_cast<double*>(ws + f.x) : nullptr;
        d.b = f.has_b ? reinterpret_cast<double*>(ws + f.b) : nullptr;
        d.x32 = f.has_x32 ? reinterpret_cast<float*>(ws + f.x32) : nullptr;
        d.b32 = f.has_x32 ? reinterpret_cast<float*>(ws + f.b32) : nullptr;
        d.part = f.has_part ? reinterpret_cast<double*>(ws + f.part) : nullptr;
        d.scratch = f.has_scratch ? reinterpret_cast<double*>(ws + f.scratch) : nullptr;
        auto dp = [&](size_t o, bool has) { return has ? reinterpret_cast<double*>(ws + o) : nullptr; };
        d.X = dp(f.X, f.lev0);
        d.B0 = dp(f.B0, f.lev0);
        d.R = dp(f.R, f.lev0);
        d.P[0] = dp(f.P[0], f.has_cg);
        d.P[1] = dp(f.P[1], f.has_cg);
        d.Q = dp(f.Q, f.has_cg);
        d.xs = (f.has_xs && !p.mixed) ? reinterpret_cast<double*>(ws + f.xs) : nullptr;
        d.xs32 = (f.has_xs && p.mixed) ? reinterpret_cast<float*>(ws + f.xs) : nullptr;
        d.ad = p.has_dir ? reinterpret_cast<double*>(ws + f.ad) : nullptr;
        d.ad32 = (p.has_dir && p.mixed) ? reinterpret_cast<float*>(ws + f.ad32) : nullptr;
        d.sidx = p.ext_state ? p.grid_slot[d.grid] : d.grid;
    }
    // every table of the workspace's table region, built on the host and uploaded at once
    const int G = p.ngrids();
    const size_t state_bytes = (p.ext_state && p.ext_state_init) ? G * sizeof(GridState) : 0;
    std::vector<char> host_img;
    char* img = nullptr;
    const bool async = p.bind_staging && p.bind_staging_bytes >= p.table_bytes + state_bytes;
    if (async) {
        img = p.bind_staging;
    } else {
        host_img.assign(p.table_bytes + state_bytes, 0);
        img = host_img.data();
    }
    std::memset(img, 0, p.table_bytes);
    std::memcpy(img + p.off_levels, p.levels.data(), p.levels.size() * sizeof(LevelDesc));
    GridState* st = p.ext_state ? reinterpret_cast<GridState*>(img + p.table_bytes)
                                : reinterpret_cast<GridState*>(img + p.off_state);
    if (!p.ext_state || p.ext_state_init) {
        for (int g = 0; g < G; ++g) {
            st[g] = init ? init[g] : GridState{};
            st[g].ntiles0 = l0_tiles(p.levels[p.level0[g]].n);
            st[g].done = 0;
        }
    }
    for (auto& D : p.dl) {
        stage_list(p, D.l0_cell, img);
        stage_list(p, D.pq3, img);
        stage_list(p, D.rz3, img);
        stage_list(p, D.coarsest, img);
        stage_list(p, D.tail, img);
        for (auto* v : {&D.coarsen, &D.down2, &D.up2, &D.mdn, &D.mup, &D.sw3, &D.sr3, &D.smooth, &D.restrict_,
                        &D.prolong, &D.tail_from, &D.coarsest_from})
            for (auto& l : *v) stage_list(p, l, img);
        if (!D.tail.empty() && prepare_tail(D.dim, p.mixed, D.tail_smem) != 0) {
            g_last_error = "hipFuncSetAttribute(max dynamic LDS) failed for the tail kernel";
            return FLD_ERR_HIP;
        }
    }
    if (async) {
        FLD_HIP(hipMemcpyAsync(p.ws, img, p.table_bytes, hipMemcpyHostToDevice, p.bind_stream));
        for (int g = 0; g < G && state_bytes; ++g)
            FLD_HIP(hipMemcpyAsync(p.ext_state + p.grid_slot[g], st + g, sizeof(GridState), hipMemcpyHostToDevice,
                                   p.bind_stream));
    } else {
        FLD_HIP(hipMemcpy(p.ws, img, p.table_bytes, hipMemcpyHostToDevice));
        for (int g = 0; g < G && state_bytes; ++g)
            FLD_HIP(hipMemcpy(p.ext_state + p.grid_slot[g], st + g, sizeof(GridState), hipMemcpyHostToDevice));
    }
    if (!p.hIO) FLD_HIP(hipHostMalloc((void**)&p.hIO, p.ngrids() * sizeof(StepIO), hipHostMallocDefault));
    if (!p.hCtrl) FLD_HIP(hipHostMalloc((void**)&p.hCtrl, sizeof(Control), hipHostMallocDefault));
    if (!p.hS) FLD_HIP(hipHostMalloc((void**)&p.hS, p.ngrids() * sizeof(GridState), hipHostMallocDefault));
    p.max_n = 0;
    for (auto n : p.ncell) p.max_n = std::max<int64_t>(p.max_n, n);
    // the tuner runs kernels over the fields: only on a plan that owns its workspace
    if (p.opts.autotune && !p.tune_done && !init && p.field_base.empty() && !p.noalloc && !p.ext_state) {
        std::vector<GridState> fresh(st, st + G);                // the tuner leaves its own states
        int rc = plan_autotune(p);
        if (rc != FLD_OK) return rc;
        FLD_HIP(hipMemcpy(p.dS, fresh.data(), fresh.size() * sizeof(GridState), hipMemcpyHostToDevice));
    }
    if (p.opts.use_graph && !p.noalloc) {
        int rc = capture_graph(p);
        if (rc != FLD_OK) return rc;
    }
    return FLD_OK;
}


int plan_upload_io(Plan& p, const StepIO* io, hipStream_t s) {
    if (p.hIO != io)
        for (int g = 0; g < p.ngrids(); ++g) p.hIO[g] = io[g];
    FLD_HIP(hipMemcpyAsync(p.dIO, p.hIO, p.ngrids() * sizeof(StepIO), hipMemcpyHostToDevice, s));
    return FLD_OK;
}

int plan_prologue(Plan& p, hipStream_t s) {
    const int zero_x = (p.krylov || p.mixed) ? 1 : 0;
    for (auto& D : p.dl) {
        if (D.l0_cell.empty()) continue;
        const JobList& l0 = D.l0_cell.dev;
        launch_coeff(D.dim, p.mixed, p.any_bc, p.dL, p.dS, l0, p.dIO, p.opts.c, p.opts.limiter, D.fin_fused ? FIN_B : -1,
                     p.opts.rtol, p.opts.max_cycles, cell_blocks(p), s);
        if (!D.fin_fused) launch_finalize(p.dL, p.dS, l0, FIN_B, p.opts.rtol, p.opts.max_cycles, s);
        for (auto& c : D.coarsen)
            launch_coarsen(D.dim, p.mixed, p.dL, c.dev, p.opts.coarse_op == FLD_COARSE_GALERKIN, p.nblk, s);
        launch_residual(D.dim, p.mixed, p.dL, p.dS, l0, 0, zero_x, D.fin_fused ? FIN_R_INIT : -1, p.opts.rtol,
                        p.opts.max_cycles, cell_blocks(p), s);
        if (!D.fin_fused) launch_finalize(p.dL, p.dS, l0, FIN_R_INIT, p.opts.rtol, p.opts.max_cycles, s);
    }
    FLD_HIP(hipGetLastError());
    return FLD_OK;
}

void plan_cycle(Plan& p, hipStream_t s) { enqueue_cycle(p, s); }

void plan_verify(Plan& p, hipStream_t s) {
    // CG stopped on its recursive residual: confirm on the true FP64 residual and
    // restart the grids whose true residual is still above the target
    for (auto& D : p.dl) {
        if (D.l0_cell.empty()) continue;
        launch_residual(D.dim, p.mixed, p.dL, p.dS, D.l0_cell.dev, 1, 1, D.fin_fused ? FIN_R_VERIFY : -1,
                        p.opts.rtol, p.opts.max_cycles, cell_blocks(p), s);
        if (!D.fin_fused)
            launch_finalize(p.dL, p.dS, D.l0_cell.dev, FIN_R_VERIFY, p.opts.rtol, p.opts.max_cycles, s);
    }
}

void plan_output(Plan& p, hipStream_t s) {
    for (auto& D : p.dl) {
        if (D.l0_cell.empty()) continue;
        launch_output(D.dim, p.dL, D.l0_cell.dev, p.dIO, cell_blocks(p), s);
    }
}

void plan_stats(const Plan& p, const GridState& st, int g, fld_stats* o) {
    // a grid still active after its iteration budget did not converge
    o->cycles = st.cycles;
    o->status = st.active ? FLD_ERR_NOT_CONVERGED : st.status;
    o->rel_residual = st.bnorm2 > 0 ? std::sqrt(st.rnorm2 / st.bnorm2) : 0.0;
    o->b_norm = std::sqrt(st.bnorm2);
    o->b_sum = st.bsum;
    const double N = (double)p.ncell[g];
    o->q_b = (st.bsum != 0.0) ? std::sqrt(st.bnorm2) / (std::sqrt(N) * std::fabs(st.bsum / N)) : INFINITY;
}

// krd: NULL, or 3 * ngrids per-direction kappa rho pointers (diagonal-tensor D; kr unused).
static int step(Plan& p, const double* const* E_in, const double* const* kr, double* const* E_out,
                const double* dt, hipStream_t s, fld_stats* stats, const double* const* krd = nullptr) {
    const int G = p.ngrids();
    std::vector<StepIO>& io = p.io_host;                 // sized when the plan was built
    for (int g = 0; g < G; ++g) {
        if (!E_in[g] || !E_out[g] || (!krd && !kr[g])) return FLD_ERR_INVALID_ARG;
        if (!(dt[g] > 0.0) || !std::isfinite(dt[g])) return FLD_ERR_INVALID_ARG;
        io[g] = StepIO{E_in[g], krd ? krd[3 * g] : kr[g], E_out[g], dt[g]};
        if (krd) {
            for (int a = 0; a < p.grids[g].ndim; ++a) {
                if (!krd[3 * g + a]) return FLD_ERR_INVALID_ARG;
                io[g].krd[a] = krd[3 * g + a];
            }
        }
    }
    int rc = plan_upload_io(p, io.data(), s);
    if (rc != FLD_OK) return rc;
    if ((rc = plan_prologue(p, s)) != FLD_OK) return rc;
    // V-cycles in rounds: each round replays `burst` cycles, then reads back how
    // many grids are still active.  The first burst is sized from the previous
    // step's cycle count so a typical step needs one or two host round trips.
    int done = 0;
    if (p.opts.fmg) {
        if (p.fmg_graph_exec) FLD_HIP(hipGraphLaunch(p.fmg_graph_exec, s));
        else enqueue_fmg_cycle(p, s);
        FLD_HIP(hipGetLastError());
        done = 1;
    }
    int burst = std::max(1, std::min(p.last_cycles > 0 ? p.last_cycles - done : 4, p.opts.max_cycles - done));
    while (done < p.opts.max_cycles) {
        const int nrun = std::min(burst, p.opts.max_cycles - done);
        for (int r = 0; r < nrun; ++r) {
            if (p.graph_exec) FLD_HIP(hipGraphLaunch(p.graph_exec, s));
            else enqueue_cycle(p, s);
        }
        FLD_HIP(hipGetLastError());
        done += nrun;
        // CG stops on its recursive residual: the grids that stopped are confirmed on the
        // true FP64 residual in the same round trip (a grid that misses the target
        // restarts; grids still iterating are not touched)
        if (p.krylov) plan_verify(p, s);
        launch_count(p.dS, G, p.dCtrl, s);
        FLD_HIP(hipMemcpyAsync(p.hCtrl, p.dCtrl, sizeof(Control), hipMemcpyDeviceToHost, s));
        FLD_HIP(hipStreamSynchronize(s));
        if (p.hCtrl->nactive == 0) break;
        burst = std::max(1, burst / 2);
    }
    plan_output(p, s);
    FLD_HIP(hipMemcpyAsync(p.hS, p.dS, G * sizeof(GridState), hipMemcpyDeviceToHost, s));
    FLD_HIP(hipStreamSynchronize(s));
    rc = FLD_OK;
    int maxc = 0;
    for (int g = 0; g < G; ++g) {
        fld_stats o;
        plan_stats(p, p.hS[g], g, &o);
        maxc = std::max(maxc, (int)o.cycles);
        if (stats) stats[g] = o;
        if (rc == FLD_OK && o.status != FLD_OK) rc = o.status;
    }
    p.last_cycles = maxc;
    return rc;
}

int plan_step_noalloc(Plan& p, void* dev, size_t bytes, const double* const* E_in, const double* const* kr,
                      double* const* E_out, const double* dt, hipStream_t s, fld_stats* stats) {
    if (p.ws) return FLD_ERR_INVALID_ARG;                 // bound to a caller workspace
    if (p.ws_bytes > bytes) return FLD_ERR_TOO_LARGE;
    p.noalloc = true;
    p.own_pinned = false;
    p.hIO = p.io_host.data();
    p.hS = p.st_host.data();
    p.hCtrl = &p.ctrl_host;
    int rc = plan_bind(p, dev, bytes, nullptr);
    if (rc == FLD_OK) rc = step(p, E_in, kr, E_out, dt, s, stats);
    // leave the plan unbound: the memory is shared by every call on this device
    p.ws = nullptr;
    p.dL = nullptr;
    p.dS = nullptr;
    p.dIO = nullptr;
    p.dEx = nullptr;
    p.dMo = nullptr;
    p.dIm = nullptr;
    p.dCtrl = nullptr;
    p.hIO = nullptr;
    p.hS = nullptr;
    p.hCtrl = nullptr;
    p.own_pinned = true;
    p.noalloc = false;
    return rc;
}

static int exchange(Plan& p, double* const* E, double* const* eps, const double* const* rho,
                    const double* const* kappa, const double* dt, const fld_gas& gas, hipStream_t s) {
    const int G = p.ngrids();
    if (!p.hEx)
        FLD_HIP(hipHostMalloc((void**)&p.hEx, Plan::kExSlots * G * sizeof(ExchangeIO), hipHostMallocDefault));
    for (auto& e : p.ex_done)
        if (!e) FLD_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    p.last_gas = gas;
    const int slot = p.ex_slot;
    p.ex_slot = (p.ex_slot + 1) % Plan::kExSlots;
    FLD_HIP(hipEventSynchronize(p.ex_done[slot]));     // staging slot free again
    ExchangeIO* h = p.hEx + (size_t)slot * G;
    for (int g = 0; g < G; ++g) {
        if (!E[g] || !eps[g] || !rho[g] || !kappa[g]) return FLD_ERR_INVALID_ARG;
        if (!(dt[g] >= 0.0) || !std::isfinite(dt[g])) return FLD_ERR_INVALID_ARG;
        h[g] = ExchangeIO{E[g], eps[g], rho[g], kappa[g], dt[g], p.ncell[g]};
    }
    ExchangeIO* d = p.dEx + (size_t)slot * G;
    FLD_HIP(hipMemcpyAsync(d, h, G * sizeof(ExchangeIO), hipMemcpyHostToDevice, s));
    launch_exchange(d, G, p.max_n, gas.c, gas.a_rad, gas.c_v, gas.max_halley, gas.root_rtol, p.dCtrl,
                    p.nblk, s);
    FLD_HIP(hipGetLastError());
    FLD_HIP(hipEventRecord(p.ex_done[slot], s));
    p.ex_last = slot;
    return FLD_OK;
}

static int moments(Plan& p, const double* const* E, const double* const* kr, const double* const* v,
                   const double* dt, const fld_moments_out* out, hipStream_t s) {
    const int G = p.ngrids();
    if (!p.hMo)
        FLD_HIP(hipHostMalloc((void**)&p.hMo, Plan::kExSlots * G * sizeof(MomentsIO), hipHostMallocDefault));
    for (auto& e : p.mo_done)
        if (!e) FLD_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    std::vector<MomentsIO> io(G);
    for (int g = 0; g < G; ++g) {
        const int nd = p.grids[g].ndim;
        const fld_moments_out& o = out[g];
        MomentsIO m{};
        if (!E[g] || !kr[g]) return FLD_ERR_INVALID_ARG;
        m.E = E[g];
        m.kr = kr[g];
        int nv = 0;
        for (int a = 0; a < nd; ++a) {
            m.v[a] = v ? v[3 * g + a] : nullptr;
            nv += m.v[a] != nullptr;
        }
        if (nv != 0 && nv != nd) return FLD_ERR_INVALID_ARG;          // all components or none
        if ((o.tiring || o.E_out) && nv == 0) return FLD_ERR_INVALID_ARG;
        if (o.E_out) {
            if (!dt || !std::isfinite(dt[g])) return FLD_ERR_INVALID_ARG;
            if (o.E_out == E[g]) return FLD_ERR_INVALID_ARG;            // neighbours still read E
            m.dt = dt[g];
        }
        for (int a = 0; a < nd; ++a) {
            m.F[a] = o.F[a];
            m.fr[a] = o.f_r[a];
        }
        m.edd = o.edd;
        for (int q = 0; q < nd * (nd + 1) / 2; ++q) m.P[q] = o.P[q];
        m.tiring = o.tiring;
        m.E_out = o.E_out;
        io[g] = m;
    }
    const int slot = p.mo_slot;
    p.mo_slot = (p.mo_slot + 1) % Plan::kExSlots;
    FLD_HIP(hipEventSynchronize(p.mo_done[slot]));     // staging slot free again
    MomentsIO* h = p.hMo + (size_t)slot * G;
    std::copy(io.begin(), io.end(), h);
    MomentsIO* d = p.dMo + (size_t)slot * G;
    FLD_HIP(hipMemcpyAsync(d, h, G * sizeof(MomentsIO), hipMemcpyHostToDevice, s));
    for (auto& D : p.dl)
        if (!D.l0_cell.empty()) launch_moments(D.dim, p.dL, D.l0_cell.dev, d, p.opts.c, p.opts.limiter, cell_blocks(p), s);
    FLD_HIP(hipGetLastError());
    FLD_HIP(hipEventRecord(p.mo_done[slot], s));
    return FLD_OK;
}

// Scratch of fld_imex_step per grid: kappa rho and E_* (Euler); kappa rho, E_+,
// E^{n+1/2} and the half-step gas energy / the midpoint tiring (midpoint).
static int imex_arrays(int scheme) { return scheme == FLD_IMEX_EULER ? 2 : 4; }

static size_t imex_scratch(const Plan& p, int scheme) {
    size_t b = 0;
    for (int g = 0; g < p.ngrids(); ++g) b += imex_arrays(scheme) * align_up((size_t)p.ncell[g] * 8);
    return b;
}

static int imex(Plan& p, double* const* E, double* const* eps, const double* const* rho,
                const double* const* kappa, const double* const* v, const double* dt, const fld_gas& gas,
                int scheme, char* scr, size_t scr_bytes, hipStream_t s, fld_stats* stats) {
    const int G = p.ngrids();
    if (scheme != FLD_IMEX_EULER && scheme != FLD_IMEX_MIDPOINT) return FLD_ERR_INVALID_ARG;
    if (!scr || scr_bytes < imex_scratch(p, scheme) || reinterpret_cast<uintptr_t>(scr) % kAlign)
        return FLD_ERR_INVALID_ARG;
    bool any_v = false;
    for (int g = 0; g < G; ++g) {
        if (!E[g] || !eps[g] || !rho[g] || !kappa[g] || E[g] == eps[g]) return FLD_ERR_INVALID_ARG;
        if (!(dt[g] > 0.0) || !std::isfinite(dt[g])) return FLD_ERR_INVALID_ARG;
        int nv = 0;
        for (int a = 0; a < p.grids[g].ndim; ++a) nv += (v && v[3 * g + a]) ? 1 : 0;
        if (nv != 0 && nv != p.grids[g].ndim) return FLD_ERR_INVALID_ARG;
        any_v = any_v || nv > 0;
    }
    if (!p.hIm)
        FLD_HIP(hipHostMalloc((void**)&p.hIm, Plan::kImStages * G * sizeof(ImexIO), hipHostMallocDefault));
    FLD_HIP(hipStreamSynchronize(s));                  // earlier work may still read the staging buffers
    const bool mid = scheme == FLD_IMEX_MIDPOINT;
    std::vector<double*> kr(G), T1(G), T2(G), T3(G);
    std::vector<double> tau1(G);
    {
        size_t off = 0;
        for (int g = 0; g < G; ++g) {
            const size_t a = align_up((size_t)p.ncell[g] * 8);
            double** dst[4] = {&kr[g], &T1[g], &T2[g], &T3[g]};
            for (int k = 0; k < imex_arrays(scheme); ++k, off += a) *dst[k] = reinterpret_cast<double*>(scr + off);
            tau1[g] = mid ? 0.5 * dt[g] : dt[g];
        }
    }
    // Stage tables: [0] kappa rho (+ the first explicit stage when there is no
    // velocity), [1] the first explicit stage after the tiring source, [2] the
    // midpoint's closing stage.
    ImexIO* h = p.hIm;
    for (int g = 0; g < G; ++g) {
        const bool gv = v && v[3 * g];
        const int64_t n = p.ncell[g];
        double* Es = mid ? T1[g] : (gv ? T1[g] : E[g]);          // E_* / E_+ after the explicit stage
        double* es = mid ? T3[g] : eps[g];
        ImexIO a{};
        a.rho = rho[g]; a.kappa = kappa[g]; a.kr = kr[g]; a.n = n;
        if (!gv) { a.E = E[g]; a.eps = eps[g]; a.E_out = Es; a.eps_out = es; a.tau = tau1[g]; }
        h[g] = a;
        ImexIO b{};
        b.rho = rho[g]; b.kappa = kappa[g]; b.n = n;
        if (gv) { b.E = T1[g]; b.eps = eps[g]; b.E_out = Es; b.eps_out = es; b.tau = tau1[g]; }
        h[G + g] = b;
        ImexIO c{};
        c.rho = rho[g]; c.kappa = kappa[g]; c.n = n;
        if (mid) {
            c.E = E[g]; c.eps = eps[g]; c.Em = T2[g]; c.Ep = T1[g];
            c.tir = gv ? T3[g] : nullptr; c.dt_tir = dt[g];
            c.E_out = E[g]; c.eps_out = eps[g]; c.tau = dt[g];
        }
        h[2 * G + g] = c;
    }
    FLD_HIP(hipMemcpyAsync(p.dIm, h, Plan::kImStages * G * sizeof(ImexIO), hipMemcpyHostToDevice, s));
    FLD_HIP(hipMemsetAsync(&p.dCtrl->bad_imex, 0, sizeof(int32_t), s));
    auto point = [&](int stage) {
        launch_imex_point(p.dIm + (size_t)stage * G, G, p.max_n, gas.c, gas.a_rad, gas.c_v, gas.max_halley,
                          gas.root_rtol, p.dCtrl, p.nblk, s);
    };
    // explicit operator over dt (Euler) or dt/2 (midpoint): tiring, then the exchange
    point(0);
    int rc;
    if (any_v) {
        std::vector<fld_moments_out> mo(G);
        std::vector<const double*> vv(3 * G, nullptr);
        for (int g = 0; g < G; ++g) {
            mo[g] = fld_moments_out{};
            if (v && v[3 * g]) {
                mo[g].E_out = T1[g];
                for (int a = 0; a < p.grids[g].ndim; ++a) vv[3 * g + a] = v[3 * g + a];
            }
        }
        std::vector<const double*> Ec(E, E + G), krc(kr.begin(), kr.end());
        if ((rc = moments(p, Ec.data(), krc.data(), vv.data(), tau1.data(), mo.data(), s)) != FLD_OK) return rc;
        point(1);
    }
    FLD_HIP(hipGetLastError());
    // implicit diffusion over the same time
    std::vector<const double*> Ein(G), krc(kr.begin(), kr.end());
    std::vector<double*> Eout(G);
    for (int g = 0; g < G; ++g) {
        const bool gv = v && v[3 * g];
        Ein[g] = mid ? T1[g] : (gv ? T1[g] : E[g]);
        Eout[g] = mid ? T2[g] : E[g];
    }
    const int rs = step(p, Ein.data(), krc.data(), Eout.data(), tau1.data(), s, stats);
    if (rs != FLD_OK && rs != FLD_ERR_NOT_CONVERGED && rs != FLD_ERR_BAD_INPUT) return rs;
    if (mid) {
        if (any_v) {
            // tiring at the midpoint state E^{n+1/2}
            std::vector<fld_moments_out> mo(G);
            std::vector<const double*> vv(3 * G, nullptr), Em(G);
            for (int g = 0; g < G; ++g) {
                mo[g] = fld_moments_out{};
                Em[g] = T2[g];
                if (v && v[3 * g]) {
                    mo[g].tiring = T3[g];
                    for (int a = 0; a < p.grids[g].ndim; ++a) vv[3 * g + a] = v[3 * g + a];
                }
            }
            if ((rc = moments(p, Em.data(), krc.data(), vv.data(), nullptr, mo.data(), s)) != FLD_OK) return rc;
        }
        point(2);
        FLD_HIP(hipGetLastError());
    }
    FLD_HIP(hipMemcpyAsync(p.hCtrl, p.dCtrl, sizeof(Control), hipMemcpyDeviceToHost, s));
    FLD_HIP(hipStreamSynchronize(s));
    if (rs != FLD_OK) return rs;
    return p.hCtrl->bad_imex ? FLD_ERR_BAD_INPUT : FLD_OK;
}

static int profile_kernel(Plan& p, int kernel, int level, int reps, hipStream_t s, double* avg_ms,
                          int64_t* cells) {
    const int G = p.ngrids();
    int64_t nc = 0;
    // collect the lists the kernel runs over (2D and 3D grids launch separately)
    for (auto& D : p.dl) {
        if (D.l0_cell.empty()) continue;
        const bool has_level = level >= 0 && level < D.maxdepth;
        const HostList* l = nullptr;
        switch (kernel) {
            case FLD_KERNEL_SMOOTH: if (has_level) l = &D.smooth[level]; break;
            case FLD_KERNEL_RESTRICT: if (has_level) l = &D.restrict_[level]; break;
            case FLD_KERNEL_PROLONG: if (has_level) l = &D.prolong[level]; break;
            case FLD_KERNEL_DOWN: if (has_level && D.fused) l = &D.down2[level]; break;
            case FLD_KERNEL_UP: if (has_level && D.fused) l = &D.up2[level]; break;
            case FLD_KERNEL_TAIL: l = D.tail.empty() ? nullptr : &D.tail; break;
            case FLD_KERNEL_SWEEP3: if (has_level && D.fused3) l = &D.sw3[level]; break;
            default: l = &D.l0_cell; break;
        }
        if (!l) continue;
        for (int32_t li : l->levels) nc += (int64_t)p.levels[li].n[0] * p.levels[li].n[1] * p.levels[li].n[2];
    }
    if (kernel == FLD_KERNEL_EXCHANGE) {
        if (p.ex_last < 0) return FLD_ERR_INVALID_ARG;
        nc = 0;
        for (auto n : p.ncell) nc += n;
    }
    if (nc == 0) return FLD_ERR_INVALID_ARG;
    hipEvent_t e0, e1;
    FLD_HIP(hipEventCreate(&e0));
    FLD_HIP(hipEventCreate(&e1));
    launch_set_active(p.dS, G, 1, s);
    auto once = [&]() {
        for (auto& D : p.dl) {
            if (D.l0_cell.empty()) continue;
            const bool has_level = level >= 0 && level < D.maxdepth;
            switch (kernel) {
                case FLD_KERNEL_SMOOTH:
                    if (has_level) launch_smooth(D.dim, p.mixed, p.dL, p.dS, D.smooth[level].dev, 0, p.nblk, s);
                    break;
                case FLD_KERNEL_RESIDUAL:
                    launch_residual(D.dim, p.mixed, p.dL, p.dS, D.l0_cell.dev, 0, 0, -1, p.opts.rtol,
                                    p.opts.max_cycles, cell_blocks(p), s);
                    break;
                case FLD_KERNEL_RESTRICT:
                    if (has_level) launch_restrict(D.dim, p.mixed, p.dL, p.dS, D.restrict_[level].dev, p.nblk, s);
                    break;
                case FLD_KERNEL_PROLONG:
                    if (has_level) launch_prolong(D.dim, p.mixed, p.dL, p.dS, D.prolong[level].dev, p.nblk, s);
                    break;
                case FLD_KERNEL_COEFF:
                    launch_coeff(D.dim, p.mixed, p.any_bc, p.dL, p.dS, D.l0_cell.dev, p.dIO, p.opts.c, p.opts.limiter,
                                 -1, p.opts.rtol, p.opts.max_cycles, cell_blocks(p), s);
                    break;
                case FLD_KERNEL_DOWN:
                    if (has_level && D.fused && D.march[level])
                        launch_march2(p.mixed, p.dL, p.dS, D.mdn[level].dev, level == 0 ? p.opts.nu1 : p.nuc1, 1, 0,
                                      D.mfz[level], p.nblk, s);
                    else if (has_level && D.fused) launch_down2(p.mixed, p.dL, p.dS, D.down2[level].dev,
                                                             level == 0 ? p.opts.nu1 : p.nuc1, 0,
                                                             p.tile_wide, level == 0 ? p.tile_rows : p.tile_rows_c,
                                                             D.thr_dn[level], p.nblk, s);
                    break;
                case FLD_KERNEL_UP:
                    if (has_level && D.fused && D.march[level])
                        launch_march2(p.mixed, p.dL, p.dS, D.mup[level].dev, level == 0 ? p.opts.nu2 : p.nuc2, 0, 0,
                                      D.mfz[level], p.nblk, s);
                    else if (has_level && D.fused) launch_up2(p.mixed, p.dL, p.dS, D.up2[level].dev,
                                                         level == 0 ? p.opts.nu2 : p.nuc2,
                                                         p.tile_wide, level == 0 ? p.tile_rows_u : p.tile_rows_c,
                                                         D.thr_up[level], p.nblk, s);
                    break;
                case FLD_KERNEL_SWEEP3:
                    if (has_level && D.fused3)
                        launch_sweep3(p.mixed, p.dL, p.dS, D.sw3[level].dev, 0, 0, 0, D.fz_s[level], p.nblk, s);
                    break;
                case FLD_KERNEL_TAIL:
                    launch_tail(D.dim, p.mixed, p.nb_bc(), p.dL, p.dS, D.tail.dev, D.tail_smem, p.nuc1, p.nuc2, 0, s);
                    break;
                default: break;
            }
        }
        if (kernel == FLD_KERNEL_VCYCLE) {
            if (p.graph_exec) (void)hipGraphLaunch(p.graph_exec, s);
            else enqueue_cycle(p, s);
            launch_set_active(p.dS, G, 1, s);
        }
        if (kernel == FLD_KERNEL_MG) plan_vcycle_mg(p, s);
        if (kernel == FLD_KERNEL_EXCHANGE) {
            const fld_gas* g = &p.last_gas;
            launch_exchange(p.dEx + (size_t)p.ex_last * G, G, p.max_n, g->c, g->a_rad, g->c_v, g->max_halley,
                            g->root_rtol, p.dCtrl, p.nblk, s);
        }
    };
    once();                                    // warm-up
    FLD_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) once();
    FLD_HIP(hipEventRecord(e1, s));
    FLD_HIP(hipGetLastError());
    FLD_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    FLD_HIP(hipEventElapsedTime(&ms, e0, e1));
    launch_set_active(p.dS, G, 0, s);
    FLD_HIP(hipStreamSynchronize(s));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_ms = (double)ms / reps;
    *cells = nc;
    return FLD_OK;
}

// Algorithmic bytes (and launches) of one pass of a driver, counted by replaying it
// with the launch wrappers in accounting mode: what = FLD_CYCLE_ITERATION one outer
// iteration (V-cycle, CG update or defect correction, stop test), FLD_CYCLE_MG the
// multigrid part of a V-cycle, FLD_CYCLE_FMG the first outer iteration of a step with
// the full-multigrid start.
int plan_cycle_bytes(Plan& p, int what, double* bytes, int64_t* launches) {
    Acct a;
    acct_set(&a);
    switch (what) {
        case FLD_CYCLE_ITERATION: enqueue_cycle(p, nullptr); break;
        case FLD_CYCLE_MG: plan_vcycle_mg(p, nullptr); break;
        case FLD_CYCLE_FMG: enqueue_fmg_cycle(p, nullptr); break;
        default: acct_set(nullptr); return FLD_ERR_INVALID_ARG;
    }
    acct_set(nullptr);
    *bytes = a.bytes;
    if (launches) *launches = a.launches;
    return FLD_OK;
}

}  // namespace fld

// ============================================================================
// C ABI
// ============================================================================
using fld::Plan;

struct fld_plan_s {
    Plan p;
};

namespace fld {
Plan* plan_of(fld_plan_t h) { return h ? &h->p : nullptr; }
}  // namespace fld

extern "C" {

int32_t fld_version(void) { return 100; }

const char* fld_strerror(int32_t code) {
    switch (code) {
        case FLD_OK: return "ok";
        case FLD_PENDING: return "pending";
        case FLD_ERR_INVALID_ARG: return "invalid argument";
        case FLD_ERR_BAD_INPUT: return "bad input (non-positive or non-finite field value)";
        case FLD_ERR_NOT_CONVERGED: return "not converged";
        case FLD_ERR_TOO_LARGE: return "request larger than the arena";
        case FLD_ERR_UNKNOWN_TICKET: return "unknown ticket";
        case FLD_ERR_HIP: return "HIP runtime error";
        case FLD_ERR_NO_WORKSPACE: return "no or too small workspace bound";
        case FLD_ERR_UNSUPPORTED: return "unsupported option";
        case FLD_ERR_SHUTDOWN: return "server shutting down";
        default: return "unknown status";
    }
}

const char* fld_last_error(void) { return fld::g_last_error.c_str(); }

void fld_opts_default(fld_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->c = 1.0;
    o->limiter = FLD_LIMITER_LP;
    for (int f = 0; f < 6; ++f) {
        o->bc[f] = FLD_BC_ZERO_FLUX;
        o->bc_grad[f] = 0.0;
    }
    o->precision = FLD_PREC_FP64;
    o->rtol = 1e-10;
    o->max_cycles = 50;
    o->nu1 = 2;
    o->nu2 = 2;
    // three sweeps on the coarse levels: about one outer iteration fewer per step, which
    // pays for the extra sweeps on every benchmark workload
    o->nu_coarse = 3;
    o->use_graph = 1;
    o->autotune = 0;
    o->krylov = 1;
    o->fused = 1;
    o->fmg = 1;
    o->fmg_depths = -1;
    o->coarse_op = FLD_COARSE_REDISCRETISED;
}

void fld_gas_default(fld_gas* g) {
    if (!g) return;
    g->c = 1.0;
    g->a_rad = 1.0;
    g->c_v = 1.0;
    g->max_halley = 100;
    g->root_rtol = 4.0 * 2.220446049250313e-16;
}

int32_t fld_plan_create(const fld_grid* grids, int32_t ngrids, const fld_opts* opts, fld_plan_t* out) {
    try {
        if (!grids || ngrids < 1 || !opts || !out) return FLD_ERR_INVALID_ARG;
        *out = nullptr;
        int rc = fld::validate_opts(*opts);
        if (rc != FLD_OK) return rc;
        for (int g = 0; g < ngrids; ++g)
            if ((rc = fld::validate_grid(grids[g])) != FLD_OK) return rc;
        auto* h = new fld_plan_s();
        rc = fld::plan_init(h->p, grids, ngrids, *opts);
        if (rc != FLD_OK) {
            delete h;
            return rc;
        }
        *out = h;
        return FLD_OK;
    } catch (const std::bad_alloc&) {
        return FLD_ERR_INVALID_ARG;
    } catch (...) {
        return FLD_ERR_INVALID_ARG;
    }
}

int32_t fld_plan_destroy(fld_plan_t plan) {
    if (!plan) return FLD_ERR_INVALID_ARG;
    fld::DeviceGuard dg(plan->p.device);
    delete plan;
    return FLD_OK;
}

int32_t fld_plan_workspace_bytes(fld_plan_t plan, size_t* bytes) {
    if (!plan || !bytes) return FLD_ERR_INVALID_ARG;
    *bytes = plan->p.ws_bytes;
    return FLD_OK;
}

int32_t fld_plan_bind_workspace(fld_plan_t plan, void* dev, size_t bytes) {
    if (!plan || !dev) return FLD_ERR_INVALID_ARG;
    if (bytes < plan->p.ws_bytes) return FLD_ERR_NO_WORKSPACE;
    try {
        fld::DeviceGuard dg(plan->p.device);
        if (!dg.ok) return FLD_ERR_HIP;
        int rc = fld::plan_bind(plan->p, dev, bytes, nullptr);
        if (rc != FLD_OK) plan->p.ws = nullptr;
        return rc;
    } catch (...) {
        plan->p.ws = nullptr;
        return FLD_ERR_INVALID_ARG;
    }
}

int32_t fld_plan_levels(fld_plan_t plan, int32_t g, int32_t* nlevels) {
    if (!plan || !nlevels || g < 0 || g >= plan->p.ngrids()) return FLD_ERR_INVALID_ARG;
    *nlevels = plan->p.nlev[g];
    return FLD_OK;
}

int32_t fld_plan_level_view(fld_plan_t plan, int32_t g, int32_t level, fld_level_view* out) {
    if (!plan || !out || g < 0 || g >= plan->p.ngrids()) return FLD_ERR_INVALID_ARG;
    Plan& p = plan->p;
    if (level < 0 || level >= p.nlev[g]) return FLD_ERR_INVALID_ARG;
    if (!p.ws) return FLD_ERR_NO_WORKSPACE;
    const fld::LevelDesc& d = p.levels[p.level0[g] + level];
    out->ndim = d.ndim;
    for (int a = 0; a < 3; ++a) {
        out->n[a] = d.n[a];
        out->w[a] = d.w[a];
        out->w32[a] = d.w32[a];
    }
    // level 0: the step's iterate and right-hand side; coarser: the V-cycle arrays
    out->x = level == 0 ? d.X : d.x;
    out->b = level == 0 ? d.B0 : d.b;
    out->x32 = d.x32;
    out->b32 = d.b32;
    out->ad = d.ad;
    return FLD_OK;
}

int32_t fld_coefficients(fld_plan_t plan, const double* const* E_in, const double* const* kappa_rho,
                         const double* dt, void* stream) {
    if (!plan || !E_in || !kappa_rho || !dt) return FLD_ERR_INVALID_ARG;
    Plan& p = plan->p;
    if (!p.ws) return FLD_ERR_NO_WORKSPACE;
    try {
        fld::DeviceGuard dg(p.device);
        if (!dg.ok) return FLD_ERR_HIP;
        hipStream_t s = static_cast<hipStream_t>(stream);
        const int G = p.ngrids();
        FLD_HIP(hipStreamSynchronize(s));            // the staging buffer is reused below
        for (int g = 0; g < G; ++g) {
            if (!E_in[g] || !kappa_rho[g]) return FLD_ERR_INVALID_ARG;
            if (!(dt[g] > 0.0) || !std::isfinite(dt[g])) return FLD_ERR_INVALID_ARG;
            p.hIO[g] = fld::StepIO{E_in[g], kappa_rho[g], nullptr, dt[g]};
        }
        FLD_HIP(hipMemcpyAsync(p.dIO, p.hIO, G * sizeof(fld::StepIO), hipMemcpyHostToDevice, s));
        for (auto& D : p.dl) {
            if (D.l0_cell.empty()) continue;
            fld::launch_coeff(D.dim, p.mixed, p.any_bc, p.dL, p.dS, D.l0_cell.dev, p.dIO, p.opts.c, p.opts.limiter,
                              D.fin_fused ? fld::FIN_B : -1, p.opts.rtol, p.opts.max_cycles, fld::cell_blocks(p), s);
            if (!D.fin_fused)
                fld::launch_finalize(p.dL, p.dS, D.l0_cell.dev, fld::FIN_B, p.opts.rtol, p.opts.max_cycles, s);
            for (auto& c : D.coarsen)
                fld::launch_coarsen(D.dim, p.mixed, p.dL, c.dev, p.opts.coarse_op == FLD_COARSE_GALERKIN, p.nblk, s);
        }
        FLD_HIP(hipGetLastError());
        FLD_HIP(hipStreamSynchronize(s));            // staging buffer free on return
        return FLD_OK;
    } catch (...) {
        return FLD_ERR_INVALID_ARG;
    }
}

int32_t fld_step(fld_plan_t plan, const double* const* E_in, const double* const* kappa_rho,
                 double* const* E_out, const double* dt, void* stream, fld_stats* stats) {
    if (!plan || !E_in || !kappa_rho || !E_out || !dt) return FLD_ERR_INVALID_ARG;
    Plan& p = plan->p;
    if (!p.ws) return FLD_ERR_NO_WORKSPACE;
    try {
        fld::DeviceGuard dg(p.device);
        if (!dg.ok) return FLD_ERR_HIP;
        hipStream_t s = static_cast<hipStream_t>(stream);
        FLD_HIP(hipStreamSynchronize(s));            // earlier work may still read the staging buffer
        return fld::step(p, E_in, kappa_rho, E_out, dt, s, stats);
    } catch (...) {
        return FLD_ERR_INVALID_ARG;
    }
}

int32_t fld_step_aniso(fld_plan_t plan, const double* const* E_in, const double* const* kappa_rho_dir,
                       double* const* E_out, const double* dt, void* stream, fld_stats* stats) {
    if (!plan || !E_in || !kappa_rho_dir || !E_out || !dt) return FLD_ERR_INVALID_ARG;
    Plan& p = plan->p;
    if (!p.ws) return FLD_ERR_NO_WORKSPACE;
    try {
        fld::DeviceGuard dg(p.device);
        if (!dg.ok) return FLD_ERR_HIP;
        hipStream_t s = static_cast<hipStream_t>(stream);
        FLD_HIP(hipStreamSynchronize(s));
        return fld::step(p, E_in, nullptr, E_out, dt, s, stats, kappa_rho_dir);
    } catch (...) {
        return FLD_ERR_INVALID_ARG;
    }
}

int32_t fld_exchange(fld_plan_t plan, double* const* E, double* const* eps, const double* const* rho,
                     const double* const* kappa, const double* dt, const fld_gas* gas, void* stream) {
    if (!plan || !E || !eps || !rho || !kappa || !dt || !gas) return FLD_ERR_INVALID_ARG;
    Plan& p = plan->p;
    if (!p.ws) return FLD_ERR_NO_WORKSPACE;
    if (!(gas->c > 0.0) || !(gas->a_rad >= 0.0) || !(gas->c_v > 0.0) || gas->max_halley < 0 ||
        !(gas->root_rtol > 0.0))
        return FLD_ERR_INVALID_ARG;
    try {
        fld::DeviceGuard dg(p.device);
        if (!dg.ok) return FLD_ERR_HIP;
        return fld::exchange(p, E, eps, rho, kappa, dt, *gas, static_cast<hipStream_t>(stream));
    } catch (...) {
        return FLD_ERR_INVALID_ARG;
    }
}

int32_t fld_exchange_status(fld_plan_t plan, void* stream, int64_t* bisected) {
    if (!plan) return FLD_ERR_INVALID_ARG;
    Plan& p = plan->p;
    if (!p.ws) return FLD_ERR_NO_WORKSPACE;
    fld::DeviceGuard dg(p.device);
    if (!dg.ok) return FLD_ERR_HIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    FLD_HIP(hipMemcpyAsync(p.hCtrl, p.dCtrl, sizeof(fld::Control), hipMemcpyDeviceToHost, s));
    FLD_HIP(hipStreamSynchronize(s));
    const int bad = p.hCtrl->bad_exchange;
    if (bisected) *bisected = p.hCtrl->bisected;
    // clear bad_exchange (offset 4) and bisected (offset 8): 12 contiguous bytes
    static_assert(offsetof(fld::Control, bisected) == offsetof(fld::Control, bad_exchange) + 4,
                  "Control layout");
    p.hCtrl->bad_exchange = 0;
    p.hCtrl->bisected = 0;
    FLD_HIP(hipMemcpyAsync(&p.dCtrl->bad_exchange, &p.hCtrl->bad_exchange, sizeof(int32_t) + sizeof(int64_t),
                           hipMemcpyHostToDevice, s));
    FLD_HIP(hipStreamSynchronize(s));
    return bad ? FLD_ERR_BAD_INPUT : FLD_OK;
}

int32_t fld_radiation_moments(fld_plan_t plan, const double* const* E, const double* const* kappa_rho,
                              const double* const* v, const double* dt, const fld_moments_out* out,
                              void* stream) {
    if (!plan || !E || !kappa_rho || !out) return FLD_ERR_INVALID_ARG;
    Plan& p = plan->p;
    if (!p.ws) return FLD_ERR_NO_WORKSPACE;
    try {
        fld::DeviceGuard dg(p.device);
        if (!dg.ok) return FLD_ERR_HIP;
        return fld::moments(p, E, kappa_rho, v, dt, out, static_cast<hipStream_t>(stream));
    } catch (...) {
        return FLD_ERR_INVALID_ARG;
    }
}

int32_t fld_imex_scratch_bytes(fld_plan_t plan, int32_t scheme, size_t* bytes) {
    if (!plan || !bytes) return FLD_ERR_INVALID_ARG;
    if (scheme != FLD_IMEX_EULER && scheme != FLD_IMEX_MIDPOINT) return FLD_ERR_INVALID_ARG;
    *bytes = fld::imex_scratch(plan->p, scheme);
    return FLD_OK;
}

int32_t fld_imex_step(fld_plan_t plan, double* const* E, double* const* eps, const double* const* rho,
                      const double* const* kappa, const double* const* v, const double* dt,
                      const fld_gas* gas, int32_t scheme, void* scratch, size_t scratch_bytes, void* stream,
                      fld_stats* stats) {
    if (!plan || !E || !eps || !rho || !kappa || !dt || !gas) return FLD_ERR_INVALID_ARG;
    Plan& p = plan->p;
    if (!p.ws) return FLD_ERR_NO_WORKSPACE;
    if (!(gas->c > 0.0) || gas->c != p.opts.c || !(gas->a_rad >= 0.0) || !(gas->c_v > 0.0) ||
        gas->max_halley < 0 || !(gas->root_rtol > 0.0))
        return FLD_ERR_INVALID_ARG;
    try {
        fld::DeviceGuard dg(p.device);
        if (!dg.ok) return FLD_ERR_HIP;
        return fld::imex(p, E, eps, rho, kappa, v, dt, *gas, scheme, static_cast<char*>(scratch), scratch_bytes,
                         static_cast<hipStream_t>(stream), stats);
    } catch (...) {
        return FLD_ERR_INVALID_ARG;
    }
}

int32_t fld_plan_tuning(fld_plan_t plan, fld_tuning* out) {
    if (!plan || !out) return FLD_ERR_INVALID_ARG;
    const Plan& p = plan->p;
    if (!p.ws) return FLD_ERR_NO_WORKSPACE;
    out->tile_rows = p.tile_rows;
    out->tile_wide = p.tile_wide;
    out->max_blocks = p.nblk;
    out->source = p.tune_source;
    out->candidates = p.tune_candidates;
    out->vcycle_us = p.tune_us;
    out->tile_depth = p.tile_depth;
    int l3 = 0;
    for (const auto& D : p.dl)
        if (D.fused3 && !D.l0_cell.empty() && p.sweep3) l3 = std::max(l3, D.levels3);
    out->fused3 = l3 > 0 ? 1 : 0;
    out->fused3_levels = l3;
    out->tile_rows_coarse = p.tile_rows_c;
    out->tile_rows_up = p.tile_rows_u;
    int m2 = 0;
    for (const auto& D : p.dl)
        for (size_t d = 0; d < D.march.size(); ++d) m2 += D.march[d] ? 1 : 0;
    out->march_levels = m2;
    out->march_rows = 0;
    for (const auto& D : p.dl)
        for (size_t d = 0; d < D.march.size(); ++d)
            if (D.march[d]) {
                out->march_rows = D.mfz[d];
                break;
            }
    out->pq_rows = 0;
    for (const auto& D : p.dl)
        if (!D.pq3.empty()) out->pq_rows = D.fz_pq;
    return FLD_OK;
}

int32_t fld_plan_cycle_bytes(fld_plan_t plan, int32_t what, double* bytes, int64_t* launches) {
    if (!plan || !bytes) return FLD_ERR_INVALID_ARG;
    if (!plan->p.ws) return FLD_ERR_NO_WORKSPACE;
    return fld::plan_cycle_bytes(plan->p, what, bytes, launches);
}

int32_t fld_profile_kernel(fld_plan_t plan, int32_t kernel, int32_t level, int32_t reps, void* stream,
                           double* avg_ms, int64_t* cells) {
    if (!plan || !avg_ms || !cells || reps < 1 || kernel < 0 || kernel > FLD_KERNEL_MG)
        return FLD_ERR_INVALID_ARG;
    Plan& p = plan->p;
    if (!p.ws) return FLD_ERR_NO_WORKSPACE;
    try {
        fld::DeviceGuard dg(p.device);
        if (!dg.ok) return FLD_ERR_HIP;
        return fld::profile_kernel(p, kernel, level, reps, static_cast<hipStream_t>(stream), avg_ms, cells);
    } catch (...) {
        return FLD_ERR_INVALID_ARG;
    }
}

}  // extern "C"
