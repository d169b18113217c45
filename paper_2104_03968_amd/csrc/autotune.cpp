// Launch-shape autotuner.  A bound plan's multigrid V-cycle (smoothing,
// transfers, tails; the solver state is only read) is timed for each
// candidate launch shape and the fastest is kept.  The candidates are, one
// dimension after the other: the fused 2D tile (64-wide or full-wave-wide,
// 4/8/16/32 rows), then the rows of the levels below the finest, then the
// finest level's rows again beside them, for its down and its up pass apart;
// for 3D grids
// the fused sweep's planes per block (16/32/64), then how many leading levels
// run fused (or none: per-colour kernels); and the cap on persistent workgroups.
// Choices are cached in a text file, one line per plan class:
//     <key> TAB <wide> <rows> <max_blocks> <depth> <sweep3> <levels3> <microseconds> <coarse rows> <up rows>
// keyed by the device architecture, precision, sweep counts and the size
// class of the plan's grids, so later plans of the same class skip the timing.
// The cache file is $FLD_AUTOTUNE_CACHE, else $HOME/.cache/fld_autotune.txt;
// failing to read or write it only costs a re-tune.
#include "fld_internal.hpp"

#include <sys/stat.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

namespace fld {

namespace {

using Shape = LaunchShape;

std::string cache_path() {
    if (const char* e = std::getenv("FLD_AUTOTUNE_CACHE")) return e;
    const char* home = std::getenv("HOME");
    if (!home || !*home) return "";
    std::string dir = std::string(home) + "/.cache";
    (void)mkdir(dir.c_str(), 0755);                  // may already exist
    return dir + "/fld_autotune.txt";
}

int log2_class(double v) { return v > 0 ? (int)std::lround(std::log2(v)) : 0; }

// Plans in one class share the same kernels, work-list depths and roughly the
// same tile counts: the grids' count and total/largest cells per dimension,
// each rounded to a power of two.
std::string plan_key(const Plan& p) {
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    int cus = 0;
    if (hipGetDeviceProperties(&prop, p.device) == hipSuccess) {
        arch = prop.gcnArchName;
        cus = prop.multiProcessorCount;
    }
    char buf[512];
    int n = std::snprintf(buf, sizeof(buf), "v7|%s|cu%d|%s|nu%d,%d,%d,%d|k%d|f%d", arch.c_str(), cus,
                          p.mixed ? "mixed" : "fp64", p.opts.nu1, p.opts.nu2, p.nuc1, p.nuc2, p.krylov ? 1 : 0,
                          p.opts.fused);
    for (int dim = 2; dim <= 3; ++dim) {
        int count = 0;
        double total = 0, largest = 0;
        for (int g = 0; g < p.ngrids(); ++g) {
            if (p.grids[g].ndim != dim) continue;
            ++count;
            total += (double)p.ncell[g];
            largest = std::max(largest, (double)p.ncell[g]);
        }
        n += std::snprintf(buf + n, sizeof(buf) - n, "|%dd:%d,%d,%d", dim, log2_class(count),
                           log2_class(total), log2_class(largest));
    }
    return buf;
}

bool cache_lookup(const std::string& key, Shape& out) {
    const std::string path = cache_path();
    if (path.empty()) return false;
    FILE* f = std::fopen(path.c_str(), "r");
    if (!f) return false;
    bool found = false;
    char line[1024];
    while (std::fgets(line, sizeof(line), f)) {
        char* tab = std::strchr(line, '\t');
        if (!tab) continue;
        *tab = 0;
        if (key != line) continue;
        Shape s{};
        double us = 0;
        if (std::sscanf(tab + 1, "%d %d %d %d %d %d %lf %d %d", &s.wide, &s.rows, &s.nblk, &s.depth, &s.sweep3,
                        &s.levels3, &us, &s.rows_c, &s.rows_u) == 9) {
            out = s;                                   // the last record of a key wins
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const std::string& key, const Shape& s, double us) {
    const std::string path = cache_path();
    if (path.empty()) return;
    FILE* f = std::fopen(path.c_str(), "a");
    if (!f) return;
    std::fprintf(f, "%s\t%d %d %d %d %d %d %.3f %d %d\n", key.c_str(), s.wide, s.rows, s.nblk, s.depth, s.sweep3,
                 s.levels3, us, s.rows_c, s.rows_u);
    std::fclose(f);
}

int max_list_tiles(const Plan& p) {
    int m = 0;
    auto see = [&](const HostList& l) { if (!l.prefix.empty()) m = std::max(m, l.prefix.back()); };
    for (const auto& D : p.dl) {
        for (const auto& l : D.smooth) see(l);
        for (const auto& l : D.restrict_) see(l);
        for (const auto& l : D.prolong) see(l);
        for (const auto& l : D.down2) see(l);
        for (const auto& l : D.up2) see(l);
        for (const auto& l : D.sw3) see(l);
        for (const auto& l : D.sr3) see(l);
        see(D.l0_cell);
    }
    return m;
}

// Microseconds of one multigrid V-cycle with shape s (median of five timed pairs).
int time_shape(Plan& p, const Shape& s, hipEvent_t e0, hipEvent_t e1, double& us) {
    int rc = plan_set_shape(p, s);
    if (rc != FLD_OK) return rc;
    plan_vcycle_mg(p, nullptr);                       // warm-up (instruction cache, lists)
    std::vector<double> t;
    for (int r = 0; r < 5; ++r) {
        FLD_HIP(hipEventRecord(e0, nullptr));
        for (int k = 0; k < 2; ++k) plan_vcycle_mg(p, nullptr);
        FLD_HIP(hipEventRecord(e1, nullptr));
        FLD_HIP(hipGetLastError());
        FLD_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        FLD_HIP(hipEventElapsedTime(&ms, e0, e1));
        t.push_back(500.0 * ms);                      // per V-cycle, microseconds
    }
    std::sort(t.begin(), t.end());
    us = t[2];
    return FLD_OK;
}

}  // namespace

int plan_autotune(Plan& p) {
    p.tune_done = true;
    const std::string key = plan_key(p);
    const Shape start = plan_shape(p);
    Shape best = start;
    if (p.opts.autotune == 1 && cache_lookup(key, best)) {
        if (plan_set_shape(p, best) == FLD_OK) {
            p.tune_source = 2;
            return FLD_OK;
        }
        best = start;                                     // stale record: time afresh
        (void)plan_set_shape(p, best);
    }
    // the timed kernels read the plan's fields: give them finite values, and let
    // every grid take part
    FLD_HIP(hipDeviceSynchronize());
    FLD_HIP(hipMemsetAsync(p.ws + p.table_bytes, 0, p.ws_bytes - p.table_bytes, nullptr));
    launch_set_active(p.dS, p.ngrids(), 1, nullptr);
    hipEvent_t e0, e1;
    FLD_HIP(hipEventCreate(&e0));
    FLD_HIP(hipEventCreate(&e1));
    struct EventGuard {
        hipEvent_t a, b;
        ~EventGuard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
    } guard{e0, e1};

    bool any2 = false, any3 = false;
    for (const auto& D : p.dl) {
        any2 = any2 || (D.fused && !D.down2.empty());
        any3 = any3 || (D.fused3 && !D.sw3.empty());
    }
    double best_us = 0;
    int timed = 0;
    // time the candidates of one dimension; the incumbent goes first and a challenger
    // must beat it by 2 % (timing noise)
    auto stage = [&](const std::vector<Shape>& cands) -> int {
        for (const Shape& c : cands) {
            double us = 0;
            int rc = time_shape(p, c, e0, e1, us);
            if (rc != FLD_OK) return rc;
            if (timed++ == 0 || us < 0.98 * best_us) { best = c; best_us = us; }
        }
        return FLD_OK;
    };
    int rc = stage({best});
    if (rc != FLD_OK) return rc;
    if (any2) {
        std::vector<Shape> c;
        for (int wide = 0; wide <= 1; ++wide)
            for (int rows : {4, 8, 16, 32}) {
                if (wide == best.wide && rows == best.rows) continue;
                if (!fused2_shape_ok(p.mixed, p.opts.nu1, wide, rows, true) ||
                    !fused2_shape_ok(p.mixed, p.opts.nu2, wide, rows, false) ||
                    !fused2_shape_ok(p.mixed, p.nuc1, wide, rows, true) ||
                    !fused2_shape_ok(p.mixed, p.nuc2, wide, rows, false))
                    continue;
                Shape s = best;
                s.wide = wide;
                s.rows = rows;
                s.rows_c = rows;
                s.rows_u = rows;
                c.push_back(s);
            }
        if ((rc = stage(c)) != FLD_OK) return rc;
        // then the rows of the coarser levels alone (fewer tiles there: shorter ones
        // can fill the chip where the finest level prefers taller ones)
        c.clear();
        for (int rows : {4, 8, 16, 32}) {
            if (rows == best.rows_c || !fused2_shape_ok(p.mixed, p.nuc1, best.wide, rows, true) ||
                !fused2_shape_ok(p.mixed, p.nuc2, best.wide, rows, false))
                continue;
            Shape s = best;
            s.rows_c = rows;
            c.push_back(s);
        }
        if ((rc = stage(c)) != FLD_OK) return rc;
        // and the finest level's rows once more, now beside the chosen coarse rows (the
        // first stage moved all levels together), for its down pass and then its up pass
        // apart (the down pass's wider halo favours taller tiles)
        c.clear();
        for (int rows : {4, 8, 16, 32}) {
            if (rows == best.rows || !fused2_shape_ok(p.mixed, p.opts.nu1, best.wide, rows, true)) continue;
            Shape s = best;
            s.rows = rows;
            c.push_back(s);
        }
        if ((rc = stage(c)) != FLD_OK) return rc;
        c.clear();
        for (int rows : {4, 8, 16, 32}) {
            if (rows == best.rows_u || !fused2_shape_ok(p.mixed, p.opts.nu2, best.wide, rows, false)) continue;
            Shape s = best;
            s.rows_u = rows;
            c.push_back(s);
        }
        if ((rc = stage(c)) != FLD_OK) return rc;
    }
    if (any3) {
        std::vector<Shape> c;
        for (int depth : {16, 32, 64}) {
            if (best.sweep3 == 1 && depth == best.depth) continue;
            Shape s = best;
            s.sweep3 = 1;
            s.depth = depth;
            c.push_back(s);
        }
        if ((rc = stage(c)) != FLD_OK) return rc;
        int depth3 = 0;
        for (const auto& D : p.dl) depth3 = std::max(depth3, (int)D.sw3.size());
        c.clear();
        for (int l = 1; l <= depth3; ++l) {
            if (l == best.levels3) continue;
            Shape s = best;
            s.sweep3 = 1;
            s.levels3 = l;
            c.push_back(s);
        }
        if (best.sweep3 == 1) {
            Shape s = best;
            s.sweep3 = 0;
            c.push_back(s);
        }
        if ((rc = stage(c)) != FLD_OK) return rc;
    }
    // block caps only matter where a launch has more tiles than the smallest cap
    if ((rc = plan_set_shape(p, best)) != FLD_OK) return rc;
    const int tiles = max_list_tiles(p);
    {
        std::vector<Shape> c;
        for (int nblk : {1024, 4096, 8192, 16384}) {
            if (nblk == best.nblk || (nblk > tiles && best.nblk >= tiles)) continue;
            Shape s = best;
            s.nblk = nblk;
            c.push_back(s);
        }
        if ((rc = stage(c)) != FLD_OK) return rc;
    }
    if ((rc = plan_set_shape(p, best)) != FLD_OK) return rc;
    FLD_HIP(hipDeviceSynchronize());
    p.tune_source = 1;
    p.tune_candidates = timed;
    p.tune_us = best_us;
    cache_store(key, best, best_us);
    return FLD_OK;
}

}  // namespace fld
