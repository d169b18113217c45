"""Fused 3D sweeps.

A fused sweep launch performs one whole red-black sweep (and, as the first or last
sweep of a level, the prolongation or the restriction) with the same per-cell
arithmetic, in the same operand order, as the per-colour kernels.  The two paths
must therefore agree bitwise on every 3D grid, and both must meet the oracle."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2104_03968_amd as fld
import workloads as W
from tests.gpu_common import dev, rel_l2, run_step

pytestmark = pytest.mark.gpu

SHAPES = [(16, 16, 16), (40, 24, 48), (64, 96, 32), (30, 44, 36), (12, 20, 200), (130, 66, 34), (24, 24, 24)]


def grids3():
    return [W.random_grid(s, 93000 + i, dt=4e-3 * (1 + i % 3)) for i, s in enumerate(SHAPES)]


def run_fused(grids, levels, **kw):
    """One step with the fused sweeps forced onto the first `levels` depths (the default
    rule fuses only depths with at least one sweep block per two compute units, which
    these test grids do not reach); checks that the plan really runs them and returns
    (xs, stats, rc)."""
    plan = fld.Plan([g.E.shape for g in grids], h=[g.h for g in grids], fused3_levels=levels,
                    **{k: v for k, v in kw.items() if k != "max_cycles"},
                    max_cycles=kw.get("max_cycles", 50))
    tun = plan.tuning()
    assert tun["fused3"] == 1 and tun["fused3_levels"] >= 1, tun
    E = [dev(g.E) for g in grids]
    K = [dev(g.kappa_rho) for g in grids]
    out = [torch.empty_like(e) for e in E]
    rc, stats = plan.step(E, K, out, [g.dt for g in grids], check=False)
    torch.cuda.synchronize()
    xs = [o.cpu().numpy() for o in out]
    plan.close()
    return xs, stats, rc


_ORACLE = {}


def oracle_step(g):
    """The FP64 oracle's step of a seeded grid (cached: several tests reuse a grid)."""
    key = (g.E.shape, float(g.E.sum()), g.dt)
    if key not in _ORACLE:
        _ORACLE[key] = O.diffusion_step(g.E, g.kappa_rho, g.dt, g.h)[0]
    return _ORACLE[key]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("krylov", [1, 0])
def test_fused_sweeps_equal_per_colour_bitwise(precision, krylov):
    gs = grids3()
    # plain V-cycles may use up the 50-cycle budget on the stiffer grids: the two paths
    # must still agree on the status, the count and every bit of the output
    xa, sa, ra = run_fused(gs, 9, precision=precision, krylov=krylov, max_cycles=80)
    xb, sb, rb = run_step(gs, precision=precision, krylov=krylov, fused=0, max_cycles=80)
    assert ra == rb
    if krylov:
        assert ra == 0
    for i, g in enumerate(gs):
        assert sa[i]["cycles"] == sb[i]["cycles"] and sa[i]["status"] == sb[i]["status"], (i, sa[i], sb[i])
        assert np.array_equal(xa[i], xb[i]), (i, SHAPES[i], rel_l2(xa[i], xb[i]))
        if sa[i]["status"] == 0:
            assert rel_l2(xa[i], oracle_step(g)) <= 1e-10 * O.q_b(g.E) * 1.01, i


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("nu", [1, 2, 3])
@pytest.mark.parametrize("depth", [16, 32, 64])
def test_fused_sweeps_any_depth_and_sweep_count(nu, depth, precision):
    """Every plane depth and sweep count in both precisions: the fused sweeps (on every
    wide level) equal the per-colour path bitwise and meet the oracle."""
    gs = grids3()[1:4]
    xa, sa, ra = run_fused(gs, 9, nu1=nu, nu2=nu, tile_depth=depth, precision=precision)
    xb, sb, rb = run_step(gs, nu1=nu, nu2=nu, fused=0, precision=precision)
    assert ra == 0 and rb == 0
    for i, g in enumerate(gs):
        assert np.array_equal(xa[i], xb[i]) and sa[i]["cycles"] == sb[i]["cycles"], (nu, depth, i)
        assert rel_l2(xa[i], oracle_step(g)) <= 1e-10 * O.q_b(g.E) * 1.01, (nu, depth, precision, i)


@pytest.mark.parametrize("depth", [16, 32, 64])
def test_fp64_fused_finest_level_default_rule(depth):
    """A grid wide enough for the default rule to fuse its finest level in FP64 (at
    least one sweep block per two compute units at depth 16) at every plane depth,
    against the oracle."""
    g = W.random_grid((96, 192, 192), 93400, dt=2e-3)
    for lv in (0, 1):
        kw = {} if lv == 0 else {"fused3_levels": 1}
        plan = fld.Plan([g.E.shape], h=[g.h], tile_depth=depth, **kw)
        if lv == 0 and depth == 16:
            assert plan.tuning()["fused3_levels"] >= 1
        plan.close()
    xa, sa, ra = run_fused([g], 1, tile_depth=depth)
    assert ra == 0
    assert rel_l2(xa[0], oracle_step(g)) <= 1e-10 * O.q_b(g.E) * 1.01, (depth, sa[0])


@pytest.mark.parametrize("levels", [1, 2, 3, 9])
def test_any_number_of_fused_levels(levels):
    """Fused sweeps on the first k levels and per-colour kernels below them (the
    restricting sweep zeroes the coarse iterate the per-colour kernels start from)."""
    gs = [W.random_grid((64, 96, 32), 93300, dt=6e-3), W.random_grid((48, 32, 80), 93301, dt=3e-3)]
    for precision in (0, 1):
        xa, sa, ra = run_step(gs, precision=precision, fused3_levels=levels, tile_depth=16)
        xb, sb, rb = run_step(gs, precision=precision, fused=0)
        assert ra == 0 and rb == 0
        for i in range(len(gs)):
            assert np.array_equal(xa[i], xb[i]) and sa[i]["cycles"] == sb[i]["cycles"], (levels, precision, i)


@pytest.mark.parametrize("precision", [0, 1])
def test_plain_vcycles_fused_meet_the_oracle(precision):
    gs = [W.random_grid((32, 40, 48), 93050, dt=1e-3), W.random_grid((64, 64, 64), 93051, dt=5e-4)]
    xa, sa, ra = run_fused(gs, 9, krylov=0, precision=precision)
    assert ra == 0
    for i, g in enumerate(gs):
        assert rel_l2(xa[i], oracle_step(g)) <= 1e-10 * O.q_b(g.E) * 1.01, (i, sa[i])


def test_odd_sweep_total_uses_per_colour_kernels():
    """nu1 + nu2 odd (plain V-cycles only) keeps the per-colour kernels, same results."""
    gs = grids3()[:2]
    xa, sa, ra = run_step(gs, krylov=0, nu1=2, nu2=1)
    xb, sb, rb = run_step(gs, krylov=0, nu1=2, nu2=1, fused=0)
    assert ra == rb
    for i in range(len(gs)):
        assert np.array_equal(xa[i], xb[i])


def test_mixed_2d_3d_batch():
    gs = [W.random_grid((96, 80), 93100, dt=2e-3), W.random_grid((32, 48, 40), 93101, dt=2e-3),
          W.random_grid((200, 60), 93102, dt=5e-3)]
    xb, sb, rc = run_step(gs, precision=1)
    assert rc == 0
    for i, g in enumerate(gs):
        (xa,), (sa,), _ = run_step([g], precision=1)
        assert np.array_equal(xa, xb[i]) and sa["cycles"] == sb[i]["cycles"]


def test_profile_sweep_kernel():
    g = W.random_grid((64, 64, 64), 93200, dt=1e-3)
    p = fld.Plan([g.E.shape], h=[g.h], precision=1)
    ms, cells = p.profile(fld.FLD_KERNEL_SWEEP3, 0, 5)
    assert ms > 0 and cells == 64 ** 3
    with pytest.raises(fld.FLDError):
        p.profile(fld.FLD_KERNEL_SWEEP3, 9, 5)          # no such fused level
    p.close()
