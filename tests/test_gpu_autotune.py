"""Launch shapes and the autotuner.

Every fused tile shape and every cap on persistent workgroups computes the same
red-black V-cycle (a tile recomputes its halo exactly as the neighbouring tiles
compute it, and the reductions sum per-cell-tile partials in a fixed order), so
results must be bitwise identical across shapes.  The autotuner's choice is one
of those shapes; its cache file round-trips."""

import numpy as np
import pytest
import torch

import oracle as O
import paper_2104_03968_amd as fld
import workloads as W
from tests.gpu_common import dev, rel_l2, run_step

pytestmark = pytest.mark.gpu

SHAPES = [(wide, rows) for wide in (0, 1) for rows in (4, 8, 16, 32)]


def fits(precision, wide, rows, nu=2):
    word = 4 if precision else 8
    for halo in (2 * nu + 1, 2 * nu):
        fx = 128 - 2 * halo if wide else 64
        if 4 * word * (fx + 2 * halo) * (rows + 2 * halo) > 160 * 1024:
            return False
    return True


def batch():
    shapes = [(196, 300), (128, 128), (200, 64), (36, 52)]
    return [W.random_grid(s, 91000 + i, dt=2e-3 * (i + 1)) for i, s in enumerate(shapes)]


@pytest.mark.parametrize("precision", [0, 1])
def test_every_tile_shape_gives_identical_results(precision):
    grids = batch()
    ref, sref, rc = run_step(grids, precision=precision)
    assert rc == 0
    ran = 0
    for wide, rows in SHAPES:
        if not fits(precision, wide, rows):
            with pytest.raises(fld.FLDError) as e:
                run_step(grids, precision=precision, tile_wide=wide, tile_rows=rows)
            assert e.value.code == fld.FLD_ERR_INVALID_ARG
            continue
        xs, st, rc = run_step(grids, precision=precision, tile_wide=wide, tile_rows=rows)
        assert rc == 0
        for i in range(len(grids)):
            assert np.array_equal(xs[i], ref[i]), (wide, rows, i)
            assert st[i]["cycles"] == sref[i]["cycles"]
        ran += 1
    assert ran >= 7 if precision else ran >= 6
    for i, g in enumerate(grids):
        x_or, _ = O.diffusion_step(g.E, g.kappa_rho, g.dt, g.h)
        # the FP64 residual reaches 1e-10 in both precisions; A is SPD with lambda_min >= 1
        assert rel_l2(ref[i], x_or) <= 1e-10 * O.q_b(g.E) * 1.01


@pytest.mark.parametrize("rows,rows_c,rows_u", [(8, 4, 0), (16, 4, 8), (4, 32, 16), (32, 8, 4)])
def test_coarse_tile_rows_give_identical_results(rows, rows_c, rows_u):
    grids = batch()
    ref, sref, _ = run_step(grids)
    xs, st, rc = run_step(grids, tile_rows=rows, tile_rows_coarse=rows_c, tile_rows_up=rows_u)
    assert rc == 0
    for i in range(len(grids)):
        assert np.array_equal(xs[i], ref[i]), (rows, rows_c, rows_u, i)
        assert st[i]["cycles"] == sref[i]["cycles"]


@pytest.mark.parametrize("max_blocks", [1, 7, 300, 1 << 16])
def test_block_cap_gives_identical_results(max_blocks):
    grids = batch() + [W.random_grid((24, 40, 32), 91100, dt=3e-3)]
    ref, sref, _ = run_step(grids)
    xs, st, rc = run_step(grids, max_blocks=max_blocks)
    assert rc == 0
    for i in range(len(grids)):
        assert np.array_equal(xs[i], ref[i]), (max_blocks, i)
        assert st[i]["cycles"] == sref[i]["cycles"]


def _solve(plan, grids):
    E = [dev(g.E) for g in grids]
    K = [dev(g.kappa_rho) for g in grids]
    out = [torch.empty_like(e) for e in E]
    rc, st = plan.step(E, K, out, [g.dt for g in grids])
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in out], st, rc


@pytest.mark.parametrize("precision", [0, 1])
def test_autotuned_plan_matches_default_and_caches(precision, tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("FLD_AUTOTUNE_CACHE", str(cache))
    grids = batch()
    shapes, hs = [g.E.shape for g in grids], [g.h for g in grids]
    ref, sref, _ = run_step(grids, precision=precision)

    tuned = fld.Plan(shapes, h=hs, precision=precision, autotune=1)
    t = tuned.tuning()
    assert t["source"] == 1 and t["candidates"] >= 2 and t["vcycle_us"] > 0, t
    assert t["tile_rows"] in (4, 8, 16, 32) and t["tile_wide"] in (0, 1) and t["max_blocks"] >= 1
    assert fits(precision, t["tile_wide"], t["tile_rows"])
    xs, st, rc = _solve(tuned, grids)
    assert rc == 0
    for i in range(len(grids)):
        assert np.array_equal(xs[i], ref[i]), i
        assert st[i]["cycles"] == sref[i]["cycles"]
    tuned.close()

    lines = cache.read_text().splitlines()
    assert len(lines) == 1
    key, rec = lines[0].split("\t")
    assert ("mixed" if precision else "fp64") in key
    wide, rows, nblk, depth, sweep3, levels3, us, rows_c, rows_u = rec.split()
    assert int(rows_c) == t["tile_rows_coarse"] and int(rows_u) == t["tile_rows_up"]
    assert (int(wide), int(rows), int(nblk)) == (t["tile_wide"], t["tile_rows"], t["max_blocks"])
    assert int(depth) == t["tile_depth"]

    # same class: taken from the cache, no timing
    again = fld.Plan(shapes, h=hs, precision=precision, autotune=1)
    t2 = again.tuning()
    assert t2["source"] == 2 and t2["candidates"] == 0
    assert (t2["tile_wide"], t2["tile_rows"], t2["max_blocks"]) == (t["tile_wide"], t["tile_rows"], t["max_blocks"])
    again.close()
    # autotune=2 always re-times and appends a record
    fresh = fld.Plan(shapes, h=hs, precision=precision, autotune=2)
    assert fresh.tuning()["source"] == 1
    fresh.close()
    assert len(cache.read_text().splitlines()) == 2


def test_stale_cache_record_is_retimed(tmp_path, monkeypatch):
    """A record naming a shape the plan cannot use (here: one whose tile does not fit
    the LDS) is ignored and the plan is timed afresh."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("FLD_AUTOTUNE_CACHE", str(cache))
    g = W.random_grid((256, 256), 91200, dt=4e-3)
    p = fld.Plan([g.E.shape], h=[g.h], autotune=1)
    key = cache.read_text().split("\t")[0]
    p.close()
    cache.write_text(f"{key}\t1 32 2048 32 1 0 1.0 32\n")
    q = fld.Plan([g.E.shape], h=[g.h], autotune=1)
    t = q.tuning()
    assert t["source"] == 1 and fits(0, t["tile_wide"], t["tile_rows"])
    (x,), (st,), rc = _solve(q, [g])
    (xr,), (sr,), _ = run_step([g])
    assert rc == 0 and np.array_equal(x, xr)
    q.close()


def test_untuned_plan_reports_its_options():
    g = W.random_grid((64, 64), 91300, dt=1e-3)
    p = fld.Plan([g.E.shape], h=[g.h], tile_rows=8, tile_wide=1, max_blocks=333)
    t = p.tuning()
    assert (t["tile_rows"], t["tile_wide"], t["max_blocks"], t["source"]) == (8, 1, 333, 0)
    assert t["fused3"] == 0                     # no 3D grid
    p.close()


def test_autotuner_times_the_3d_sweep_depths(tmp_path, monkeypatch):
    monkeypatch.setenv("FLD_AUTOTUNE_CACHE", str(tmp_path / "tune.txt"))
    g = W.random_grid((48, 64, 80), 91400, dt=3e-3)
    for precision in (0, 1):
        p = fld.Plan([g.E.shape], h=[g.h], precision=precision, autotune=2)
        t = p.tuning()
        # the incumbent, two other depths and the per-colour kernels (+ block caps)
        assert t["source"] == 1 and t["candidates"] >= 4, t
        assert t["tile_depth"] in (16, 32, 64) and t["fused3"] in (0, 1)
        (x,), (st,), rc = _solve(p, [g])
        (xr,), (sr,), _ = run_step([g], precision=precision)
        assert rc == 0 and np.array_equal(x, xr) and st["cycles"] == sr["cycles"]
        p.close()


def test_coarse_sweep_count_has_its_own_cache_record(tmp_path, monkeypatch):
    """The coarse tile carries the halo of nu_coarse sweeps, so a plan with another count is
    timed afresh under its own key rather than handed a shape tuned for the default; the
    tuned plan reproduces the untuned one bit for bit."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("FLD_AUTOTUNE_CACHE", str(cache))
    g = W.random_grid((256, 256), 91300, dt=4e-3)
    fld.Plan([g.E.shape], h=[g.h], autotune=1).close()
    p = fld.Plan([g.E.shape], h=[g.h], autotune=1, nu_coarse=2)
    t = p.tuning()
    assert t["source"] == 1 and t["candidates"] >= 2
    (x,), (st,), rc = _solve(p, [g])
    p.close()
    keys = [line.split("\t")[0] for line in cache.read_text().splitlines()]
    assert len(keys) == 2 and keys[0] != keys[1]
    (xr,), (sr,), rcr = run_step([g], nu_coarse=2)
    assert rc == 0 and rcr == 0 and np.array_equal(x, xr) and st["cycles"] == sr["cycles"]
