"""The row-marching 2D kernels.  The fused level kernels (k_march2) against the LDS-tile ones: the
same operand order on every cell update and residual, so a step through either gives
bitwise equal results, at every sweep count, in both precisions and under CG, plain
V-cycles and the full-multigrid start; and the default rule picks the march only on
depths with many windows."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import oracle as O                     # noqa: E402
import workloads as W                  # noqa: E402
import paper_2104_03968_amd as fld     # noqa: E402
from tests.gpu_common import run_step, rel_l2   # noqa: E402

# widths across and off the window widths (118 / 120 interior columns at nu = 2), odd
# coarsest levels, a grid narrower than one window, one taller than one march block
SHAPES = [(256, 256), (130, 372), (96, 64), (200, 120), (48, 40), (320, 236)]


def _grids(seed):
    return [W.random_grid(s, seed + 7 * i, dt=3e-3 * (1 + i % 3)) for i, s in enumerate(SHAPES)]


def _pair(grids, **kw):
    xa, sa, ra = run_step(grids, fused=3, **kw)
    xb, sb, rb = run_step(grids, fused=2, **kw)
    assert ra == 0 and rb == 0, (sa, sb)
    for i in range(len(grids)):
        assert sa[i]["cycles"] == sb[i]["cycles"], (i, sa[i], sb[i])
        assert np.array_equal(xa[i], xb[i]), (i, np.abs(xa[i] - xb[i]).max())
    return xa, sa


@pytest.mark.parametrize("nu", [1, 2, 3])
@pytest.mark.parametrize("precision", [0, 1])
def test_march_equals_tiles_bitwise(nu, precision):
    grids = _grids(640000 + 10 * nu)
    _pair(grids, precision=precision, nu1=nu, nu2=nu, nu_coarse=nu)


@pytest.mark.parametrize("krylov,fmg", [(0, 0), (0, 1), (1, 0)])
def test_march_equals_tiles_other_iterations(krylov, fmg):
    grids = _grids(641000)
    _pair(grids, precision=0, krylov=krylov, fmg=fmg)


def test_march_meets_the_oracle():
    grids = _grids(642000)[:3]
    rtol = min(1e-10 / O.q_b(g.E) for g in grids)
    xs, st = _pair(grids, precision=0, rtol=rtol)
    for g, x in zip(grids, xs):
        x_or, _ = O.diffusion_step(g.E, g.kappa_rho, g.dt, g.h)
        assert rel_l2(x, x_or) <= 1e-10 * 1.01


def test_default_rule_marches_only_where_windows_are_many():
    """32-row windows where there are at least four per compute unit; 16-row ones where
    those are at least two per unit and the levels fill them (one 1024^2 grid's finest
    level); tiles otherwise (one 512^2 grid)."""
    big = fld.Plan([(512, 512)] * 40, h=[(1 / 512, 1 / 512)] * 40)
    one = fld.Plan([(1024, 1024)], h=[(1 / 1024, 1 / 1024)])
    half = fld.Plan([(512, 512)], h=[(1 / 512, 1 / 512)])
    forced = fld.Plan([(64, 64)], h=[(1 / 64, 1 / 64)], fused=3)
    tiles = fld.Plan([(512, 512)] * 40, h=[(1 / 512, 1 / 512)] * 40, fused=2)
    assert big.tuning()["march_levels"] >= 1 and big.tuning()["march_rows"] == 32
    assert one.tuning()["march_levels"] == 1 and one.tuning()["march_rows"] == 16
    assert half.tuning()["march_levels"] == 0 and half.tuning()["march_rows"] == 0
    assert forced.tuning()["march_levels"] >= 1
    assert tiles.tuning()["march_levels"] == 0
    for p in (big, one, half, forced, tiles):
        p.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_short_windows_equal_tiles_and_meet_the_oracle(precision):
    """A single 1024^2 grid marches its finest level in 16-row windows (CG with the tile
    kernels' reductions): bitwise equal to the LDS tiles, and at the oracle."""
    g = W.random_grid((1024, 1024), 643000, dt=2e-3)
    rtol = 1e-10 / O.q_b(g.E)
    (xa,), (sa,), ra = run_step([g], precision=precision, rtol=rtol)
    (xb,), (sb,), rb = run_step([g], precision=precision, rtol=rtol, fused=2)
    assert ra == 0 and rb == 0 and sa["cycles"] == sb["cycles"]
    assert np.array_equal(xa, xb)
    x_or, _ = O.diffusion_step(g.E, g.kappa_rho, g.dt, g.h)
    assert rel_l2(xa, x_or) <= 1e-10 * 1.01


# The row-march CG direction update (k_cg_pq2m) runs on 2D plans whose reductions finish
# in a k_finalize launch (too many level-0 tiles to fold), zero-flux faces and even row
# lengths.  Its p . q partials are per window, so its sums round differently from the
# cell-tile kernel's: parity is against the oracle (1e-10 relative L2, the step target)
# and against each grid solved alone (cell-tile kernel), not bitwise.
def _big_batch(seed, odd=False):
    shapes = [(512, 512)] * 33 + [(384, 640), (256, 1024)]      # 8944 level-0 tiles: no folding
    if odd:
        shapes[5] = (512, 511)
    return [W.random_grid(s, seed + i, dt=2e-3 * (1 + i % 4)) for i, s in enumerate(shapes)]


@pytest.mark.parametrize("precision", [0, 1])
def test_pq_march_meets_the_oracle(precision):
    grids = _big_batch(650000)
    plan = fld.Plan([g.E.shape for g in grids], h=[g.h for g in grids], precision=precision)
    assert plan.tuning()["pq_rows"] > 0
    plan.close()
    pick = (0, 17, 33, 34)
    rtol = min(1e-10 / O.q_b(grids[i].E) for i in pick)
    xs, st, rc = run_step(grids, precision=precision, rtol=rtol)
    assert rc == 0, [s for s in st if s["status"] != 0][:2]
    for i in pick:
        x_or, _ = O.diffusion_step(grids[i].E, grids[i].kappa_rho, grids[i].dt, grids[i].h)
        assert rel_l2(xs[i], x_or) <= 1e-10, (i, rel_l2(xs[i], x_or))
        (x1,), _, rc1 = run_step([grids[i]], precision=precision, rtol=rtol)
        assert rc1 == 0 and rel_l2(xs[i], x1) <= 2e-10


def test_pq_march_skips_odd_rows():
    """An odd row length keeps the cell-tile CG kernels; that grid has no coarse level
    (no up pass), so r . z is not formed in the march either."""
    grids = _big_batch(651000, odd=True)
    plan = fld.Plan([g.E.shape for g in grids], h=[g.h for g in grids])
    assert plan.tuning()["pq_rows"] == 0
    plan.close()
    rtol = 1e-10 / O.q_b(grids[5].E)
    xs, st, rc = run_step(grids, rtol=rtol)
    assert rc == 0
    x_or, _ = O.diffusion_step(grids[5].E, grids[5].kappa_rho, grids[5].dt, grids[5].h)
    assert rel_l2(xs[5], x_or) <= 1e-10


@pytest.mark.parametrize("nu", [1, 3])
def test_short_windows_other_sweep_counts_bitwise(nu):
    """16-row windows with one and three sweeps per side (halos of 4 and 8 rows on the down
    pass): bitwise equal to the LDS tiles in both precisions."""
    g = W.random_grid((1024, 1024), 644000 + nu, dt=3e-3)
    for precision in (0, 1):
        kw = dict(precision=precision, nu1=nu, nu2=nu)
        plan = fld.Plan([g.E.shape], h=[g.h], **kw)
        assert plan.tuning()["march_rows"] == 16
        plan.close()
        (xa,), (sa,), ra = run_step([g], **kw)
        (xb,), (sb,), rb = run_step([g], fused=2, **kw)
        assert ra == 0 and rb == 0 and sa["cycles"] == sb["cycles"]
        assert np.array_equal(xa, xb), (nu, precision)
