"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: face weights <= 1e-14 relative per face plus the rounding bound of the
4th-order gradient where its terms cancel (see face_tolerance); one diffusion step <= 1e-10
relative L2 (the run stops at rtol = 1e-10 / q_b, so ||x - x*|| / ||x*|| <= 1e-10 is
guaranteed by the residual bound; the oracle itself is within 1e-13 q_b of x*);
exchange <= 1e-12 (eps + E) per cell.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import oracle as O                     # noqa: E402
import workloads as W                  # noqa: E402
import paper_2104_03968_amd as fld     # noqa: E402
from tests.gpu_common import dev, rel_l2, run_step   # noqa: E402


def _rtol_for(g):
    return 1e-10 / O.q_b(g.E)


EPS = np.finfo(np.float64).eps


def face_tolerance(g, limiter="lp"):
    """Per-face relative tolerance from the conditioning of the 4th-order gradient.

    The computed g_d carries an absolute rounding error of a few eps times
    S_d = (|E_-2| + 8|E_-1| + 8|E_+1| + |E_+2|) / (12 h_d) whatever the order of the
    sum, so |grad E| is uncertain by ~4 eps sum_d |g_d| S_d / |grad E|.  D depends on R
    with relative sensitivity s(R) = |d ln lambda / d ln R| <= 1 (0 for lambda = 1/3),
    and a harmonic face mean passes on at most the sum of its two cells' relative errors.
    """
    nd = g.E.ndim
    P = O.pad_mirror(g.E, 2)
    core = tuple(slice(2, 2 + s) for s in g.E.shape)
    grads = O.gradient4(g.E, g.h)
    gn = np.sqrt(sum(x * x for x in grads))
    acc = np.zeros_like(g.E)
    for d in range(nd):
        a = nd - 1 - d

        def sh(k):
            sl = list(core)
            sl[a] = slice(2 + k, 2 + k + g.E.shape[a])
            return np.abs(P[tuple(sl)])
        S = (sh(-2) + 8 * sh(-1) + 8 * sh(1) + sh(2)) / (12 * g.h[d])
        acc += np.abs(grads[d]) * S
    R = gn / (g.kappa_rho * g.E)
    if limiter == "lp":
        sens = R * np.abs(1 / (2 + R) - (3 + 2 * R) / (6 + 3 * R + R * R))
    elif limiter == "diffusion":
        sens = np.zeros_like(R)
    else:
        sens = np.ones_like(R)             # lambda falls no faster than 1/R
    # the exact form's coth R - 1/R loses up to ~300 ulp to cancellation just above
    # its series threshold, on both sides independently
    extra = 1000 * EPS if limiter == "lp_exact" else 0.0
    with np.errstate(invalid="ignore", divide="ignore"):
        rel_R = np.where(gn > 0, 4 * EPS * acc / (gn * gn), 0.0)
    cell = 8 * EPS + sens * rel_R + extra
    tol = []
    for d in range(nd):
        a = nd - 1 - d
        lo = [slice(None)] * nd
        hi = [slice(None)] * nd
        lo[a] = slice(0, g.E.shape[a] - 1)
        hi[a] = slice(1, g.E.shape[a])
        t = np.full_like(g.E, 1e-14)
        t[tuple(hi)] = 1e-14 + cell[tuple(lo)] + cell[tuple(hi)]
        tol.append(t)
    return tol


# ------------------------------------------------------------------ K1 coefficients
@pytest.mark.parametrize("shape,limiter", [((64, 64), "lp"), ((37, 100), "lp"), ((64, 64), "diffusion"),
                                           ((9, 13, 20), "lp"), ((2, 2), "lp"), ((3, 2, 5), "lp"),
                                           ((64, 64), "minerbo"), ((33, 47), "minerbo"), ((9, 13, 20), "minerbo"),
                                           ((64, 64), "lp_exact"), ((33, 47), "lp_exact"),
                                           ((9, 13, 20), "lp_exact")])
def test_face_weights_match_oracle(shape, limiter):
    g = W.pulse_2d() if shape == (64, 64) else W.random_grid(shape, 123000 + sum(shape), dt=3e-3)
    g.limiter = limiter
    plan = fld.Plan([g.E.shape], h=[g.h], limiter=fld.LIMITER_CODES[limiter], c=g.c)
    plan.coefficients([dev(g.E)], [dev(g.kappa_rho)], [g.dt])
    torch.cuda.synchronize()
    lv = plan.level_tensors(0, 0)
    D = O.diffusion_coefficient(g.E, g.kappa_rho, g.h, g.c, limiter)
    w_or = O.face_weights(D, g.dt, g.h)
    tol = face_tolerance(g, limiter)
    for d in range(g.E.ndim):
        wg = lv["w"][d].cpu().numpy()
        wo = w_or[d]
        assert np.all((wg == 0) == (wo == 0))
        err = np.abs(wg - wo) / np.where(wo == 0, 1.0, np.abs(wo))
        assert np.all(err <= tol[d]), (d, err.max(), (err / tol[d]).max())
    # the right-hand side copy and initial guess are E^n, bitwise
    assert np.array_equal(lv["b"].cpu().numpy(), g.E)
    plan.close()


def test_face_weights_full_size_1024_squared():
    g = W.c2_inputs(1024)
    plan = fld.Plan([g.E.shape], h=[g.h])
    plan.coefficients([dev(g.E)], [dev(g.kappa_rho)], [g.dt])
    torch.cuda.synchronize()
    lv = plan.level_tensors(0, 0)
    w_or = O.face_weights(O.diffusion_coefficient(g.E, g.kappa_rho, g.h), g.dt, g.h)
    tol = face_tolerance(g)
    for d in range(2):
        wg = lv["w"][d].cpu().numpy()
        err = np.abs(wg - w_or[d]) / np.where(w_or[d] == 0, 1.0, np.abs(w_or[d]))
        assert np.all(err <= tol[d]), (err.max(), (err / tol[d]).max())
        # most faces are well conditioned: the flat 1e-14 bound holds for > 99 % of them
        assert np.mean(err <= 1e-14) > 0.99
    plan.close()


# ------------------------------------------------------------------ one diffusion step
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("krylov", [1, 0])
@pytest.mark.parametrize("nu", [1, 2, 3, 4])
@pytest.mark.parametrize("fmg", [1, 0])
def test_pulse_64_squared_step_matches_lu(precision, krylov, nu, fmg):
    g = W.pulse_2d()
    x_or, info = O.diffusion_step(g.E, g.kappa_rho, g.dt, g.h, g.c, method="lu")
    (x,), (st,), rc = run_step([g], precision=precision, rtol=_rtol_for(g), krylov=krylov, nu1=nu, nu2=nu,
                               fmg=fmg)
    assert rc == 0 and st["status"] == 0, st
    assert rel_l2(x, x_or) <= 1e-10, (rel_l2(x, x_or), st)
    assert st["q_b"] == pytest.approx(O.q_b(g.E), rel=1e-12)
    # zero flux: 1^T A = 1^T, so sum x - sum b = -sum r, and |sum r| <= ||r||_1 <= sqrt(N) ||r||_2
    dsum = abs(x.sum() - g.E.sum())
    assert dsum <= np.sqrt(g.E.size) * st["rel_residual"] * np.linalg.norm(g.E) + 1e-13 * g.E.sum()
    if not fmg:
        # from the start E^n (sum b exactly) the V-cycles keep the mean far tighter
        assert dsum / g.E.sum() < 1e-12


@pytest.mark.parametrize("shape,dt", [((37, 100), 5e-3), ((96, 96), 1e-2), ((3, 5), 1e-2), ((2, 2), 1e-1),
                                      ((130, 66), 2e-3), ((20, 12, 8), 5e-3), ((24, 24, 24), 1e-2),
                                      ((9, 7, 5), 1e-2)])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("krylov", [1, 0])
@pytest.mark.parametrize("fused", [1, 0])
def test_ragged_and_odd_grids_match_oracle(shape, dt, precision, krylov, fused):
    g = W.random_grid(shape, 555000 + 7 * sum(shape), dt=dt)
    x_or, info = O.diffusion_step(g.E, g.kappa_rho, g.dt, g.h, method="auto")
    (x,), (st,), rc = run_step([g], precision=precision, rtol=_rtol_for(g), krylov=krylov, fused=fused)
    assert rc == 0 and st["status"] == 0, st
    assert rel_l2(x, x_or) <= 1e-10, (rel_l2(x, x_or), st, info)


@pytest.mark.parametrize("limiter", ["minerbo", "lp_exact"])
@pytest.mark.parametrize("precision", [0, 1])
def test_step_with_limiter_variants(limiter, precision):
    for shape in ((48, 40), (12, 16, 20)):
        g = W.random_grid(shape, 124000 + sum(shape), dt=3e-3)
        g.limiter = limiter
        (x,), (st,), rc = run_step([g], precision=precision, limiter=limiter, rtol=_rtol_for(g))
        x_or, _ = O.diffusion_step(g.E, g.kappa_rho, g.dt, g.h, g.c, limiter)
        assert rc == 0 and rel_l2(x, x_or) <= 1e-10, (shape, st)


def test_diffusion_limiter_matches_dct():
    """Constant coefficients, lambda = 1/3: the GPU step equals the spectral solution."""
    import scipy.fft
    n = 256
    E = W.random_grid((n, n), 99100, 1e-3).E
    kr = np.full_like(E, 10.0)
    g = W.GridInput(E=E, kappa_rho=kr, dt=1e-2, h=(1 / n, 1 / n), limiter="diffusion")
    k = np.arange(n)
    ev = 4 * n * n * np.sin(np.pi * k / (2 * n)) ** 2
    lam = ev[None, :] + ev[:, None]
    ref = scipy.fft.idctn(scipy.fft.dctn(E, type=2, norm="ortho") / (1 + g.dt / 30.0 * lam),
                          type=2, norm="ortho")
    (x,), (st,), rc = run_step([g], limiter="diffusion", rtol=_rtol_for(g))
    assert rc == 0 and rel_l2(x, ref) <= 1e-10


def test_in_place_output():
    g = W.random_grid((64, 80), 321000, dt=5e-3)
    x_or, _ = O.diffusion_step(g.E, g.kappa_rho, g.dt, g.h)
    (x,), (st,), rc = run_step([g], rtol=_rtol_for(g), in_place=True)
    assert rc == 0 and rel_l2(x, x_or) <= 1e-10


@pytest.mark.parametrize("krylov", [1, 0])
def test_graph_and_direct_launches_agree_bitwise(krylov):
    g = W.random_grid((128, 96), 77000, dt=5e-3)
    (xa,), (sa,), _ = run_step([g], use_graph=1, krylov=krylov)
    (xb,), (sb,), _ = run_step([g], use_graph=0, krylov=krylov)
    assert np.array_equal(xa, xb) and sa["cycles"] == sb["cycles"]


@pytest.mark.parametrize("precision", [0, 1])
def test_fused_and_per_colour_kernels_agree(precision):
    """The fused LDS level kernels run the same red-black V-cycle as the one-kernel-per-
    colour path: same iteration count, results equal to rounding."""
    g = W.random_grid((512, 384), 4242, dt=5e-3)
    (xa,), (sa,), ra = run_step([g], precision=precision, fused=1)
    (xb,), (sb,), rb = run_step([g], precision=precision, fused=0)
    assert ra == 0 and rb == 0
    assert sa["cycles"] == sb["cycles"], (sa, sb)
    assert rel_l2(xa, xb) <= 1e-12


@pytest.mark.parametrize("precision", [0, 1])
def test_stiff_trajectory_converges_quickly(precision):
    """A grid of the 512-grid batch (288^2, dt = 9.2e-3, coarsest 9^2) whose third step sharpens D
    enough that plain V-cycles need ~30 iterations; CG with the V-cycle stays <= 16."""
    n, dt = W.c4_layout()[118]
    g = W.c4_grid(118, n, dt)
    E = dev(g.E)
    K = dev(g.kappa_rho)
    plan = fld.Plan([g.E.shape], h=[g.h], precision=precision)
    for step in range(3):
        E_in = E.cpu().numpy()
        rc, (st,) = plan.step([E], [K], [E], [g.dt])
        assert rc == 0 and st["cycles"] <= 16, (step, st)
    x = E.cpu().numpy()
    x_or, _ = O.diffusion_step(E_in, g.kappa_rho, g.dt, g.h)
    assert rel_l2(x, x_or) <= 1e-10 * O.q_b(E_in) * 1.01
    plan.close()


def test_reported_residual_is_the_oracle_residual():
    g = W.random_grid((200, 120), 88000, dt=1e-2)
    (x,), (st,), rc = run_step([g])
    D = O.diffusion_coefficient(g.E, g.kappa_rho, g.h)
    A = O.assemble_operator(O.face_weights(D, g.dt, g.h))
    rr = O.relative_residual(A, x, g.E)
    assert rr <= 1e-10 * 1.01
    assert st["rel_residual"] == pytest.approx(rr, rel=1e-3, abs=1e-16)
    assert 1 <= st["cycles"] <= 20


@pytest.mark.parametrize("precision", [0, 1])
def test_vanishing_time_step(precision):
    """dt -> 0: A -> I + O(dt), so the step stays within O(dt |L|) of E^n and one or two
    cycles reach the stop rule; against the oracle's step."""
    g = W.random_grid((96, 80), 620000, dt=1e-12)
    (x,), (st,), rc = run_step([g], precision=precision)
    assert rc == 0 and st["cycles"] <= 2, st
    assert rel_l2(x, g.E) <= 1e-6
    x_or, _ = O.diffusion_step(g.E, g.kappa_rho, g.dt, g.h)
    assert rel_l2(x, x_or) <= 1e-10 * O.q_b(g.E) * 1.01


# ------------------------------------------------------------------ batching
def test_batched_equals_alone_bitwise():
    shapes = [(64, 64), (96, 96), (37, 100), (160, 160), (24, 24, 24)]
    grids = [W.random_grid(s, 600000 + 13 * i, dt=2e-3 * (i + 1)) for i, s in enumerate(shapes)]
    xb, sb, rc = run_step(grids)
    assert rc == 0
    for i, g in enumerate(grids):
        (xa,), (sa,), _ = run_step([g])
        assert np.array_equal(xa, xb[i]), i
        assert sa["cycles"] == sb[i]["cycles"]
        x_or, _ = O.diffusion_step(g.E, g.kappa_rho, g.dt, g.h)
        assert rel_l2(xb[i], x_or) <= 1e-10 * O.q_b(g.E) * 1.01


@pytest.mark.parametrize("precision", [0, 1])
def test_reduction_placement_does_not_change_a_result(precision):
    """Where a grid's r.z and p.q sums are finished depends on the plan, not on the grid.
    Alone, a 600^2 grid (380 level-0 tiles) has its CG scalars formed by the blocks of the
    kernels that use them; with a 64 x 96 grid (6 tiles) too; the small grid alone, by the
    last tile's block.  These sum the same per-tile partials in the same order: bitwise equal.
    Batched with a 2944^2 grid (more tiles than any block count) the plan finishes in
    k_finalize launches and takes the row-march CG update and r.z inside the level-0 up
    march (FP64), whose partials are per window: a grid's result is then bitwise the same in
    every such plan (with or without the small grid), and within rounding of the tile-partial
    result (both meet the oracle)."""
    a = W.random_grid((600, 600), 610000, dt=4e-3)
    big = W.random_grid((2944, 2944), 610001, dt=1e-3)
    small = W.random_grid((64, 96), 610002, dt=4e-3)
    (xa,), (sa,), ra = run_step([a], precision=precision)
    xp, sp, rp = run_step([a, small], precision=precision)
    (xs,), (ss,), rs = run_step([small], precision=precision)
    xb, sb, rb = run_step([a, big, small], precision=precision)
    xc, sc, rc = run_step([a, big], precision=precision)
    assert ra == 0 and rp == 0 and rs == 0 and rb == 0 and rc == 0
    assert np.array_equal(xa, xp[0]) and sa["cycles"] == sp[0]["cycles"]
    assert np.array_equal(xs, xp[1]) and ss["cycles"] == sp[1]["cycles"]
    assert np.array_equal(xb[0], xc[0]) and sb[0]["cycles"] == sc[0]["cycles"]
    assert np.array_equal(xb[1], xc[1])
    tol = 1e-10 * O.q_b(a.E) * 1.01
    x_or, _ = O.diffusion_step(a.E, a.kappa_rho, a.dt, a.h)
    assert rel_l2(xa, x_or) <= tol
    assert rel_l2(xb[0], x_or) <= tol
    assert rel_l2(xb[0], xa) <= 2 * tol


# ------------------------------------------------------------------ failure paths
def test_bad_input_reported():
    g = W.random_grid((32, 32), 1000, dt=1e-3)
    g.E[5, 5] = -1.0
    (x,), (st,), rc = run_step([g])
    assert rc == fld.FLD_ERR_BAD_INPUT and st["status"] == fld.FLD_ERR_BAD_INPUT
    g2 = W.random_grid((32, 32), 1001, dt=1e-3)
    g2.kappa_rho[0, 0] = np.nan
    _, (st2,), rc2 = run_step([g2])
    assert rc2 == fld.FLD_ERR_BAD_INPUT
    # a good grid in the same batch is still solved
    g3 = W.random_grid((32, 32), 1002, dt=1e-3)
    xs, sts, rc3 = run_step([g, g3])
    assert rc3 == fld.FLD_ERR_BAD_INPUT and sts[1]["status"] == 0
    x_or, _ = O.diffusion_step(g3.E, g3.kappa_rho, g3.dt, g3.h)
    assert rel_l2(xs[1], x_or) <= 1e-10 * O.q_b(g3.E)


def test_not_converged_reported_with_stats():
    g = W.random_grid((128, 128), 1003, dt=1e-2)
    (x,), (st,), rc = run_step([g], rtol=1e-15, max_cycles=2)
    assert rc == fld.FLD_ERR_NOT_CONVERGED and st["status"] == fld.FLD_ERR_NOT_CONVERGED
    assert st["cycles"] == 2 and 0 < st["rel_residual"] < 1e-1
    assert np.all(np.isfinite(x))


# ------------------------------------------------------------------ exchange
def _exchange_gpu(g, max_halley=100):
    plan = fld.Plan([g.E.shape], h=[g.h])
    E, eps, rho, kap = dev(g.E), dev(g.eps), dev(g.rho), dev(g.kappa)
    plan.exchange([E], [eps], [rho], [kap], [g.dt], fld.fld_gas_default(max_halley=max_halley))
    rc, nbis = plan.exchange_status()
    out = E.cpu().numpy(), eps.cpu().numpy(), rc, nbis
    plan.close()
    return out


@pytest.mark.parametrize("n", [64, 1024])
def test_exchange_matches_oracle(n):
    g = W.c2_inputs(n)
    E2, eps2, rc, nbis = _exchange_gpu(g)
    Eo, epso = O.exchange(g.E, g.eps, g.rho, g.kappa, g.dt)
    tot = g.E + g.eps
    assert rc == 0 and nbis == 0
    assert np.all(np.abs(eps2 - epso) <= 1e-12 * tot)
    assert np.all(np.abs(E2 - Eo) <= 1e-12 * tot)
    assert np.all(np.abs(E2 + eps2 - tot) <= 1e-14 * tot)


def test_exchange_bisection_fallback_gives_same_root():
    g = W.c2_inputs(64)
    E_h, eps_h, _, nb_h = _exchange_gpu(g, 100)
    E_b, eps_b, rc, nb_b = _exchange_gpu(g, 0)
    assert rc == 0 and nb_h == 0 and nb_b == g.E.size
    tot = g.E + g.eps
    assert np.all(np.abs(eps_b - eps_h) <= 4e-16 * tot)


def test_exchange_wide_dynamic_range():
    """Roots across many decades of beta (cgs-like and stiff cases)."""
    rng = np.random.default_rng(9)
    n = 50000
    shape = (250, 200)
    g = W.GridInput(E=10.0 ** rng.uniform(-3, 3, n).reshape(shape), kappa_rho=np.ones(shape), dt=1.0,
                    h=(1 / 200, 1 / 250))
    g.eps = 10.0 ** rng.uniform(-3, 3, n).reshape(shape)
    g.rho = 10.0 ** rng.uniform(-2, 2, n).reshape(shape)
    g.kappa = 10.0 ** rng.uniform(-3, 3, n).reshape(shape)
    g.dt = 0.37
    E2, eps2, rc, _ = _exchange_gpu(g)
    Eo, epso = O.exchange(g.E, g.eps, g.rho, g.kappa, g.dt)
    tot = g.E + g.eps
    assert rc == 0
    assert np.all(np.abs(eps2 - epso) <= 1e-12 * tot)


def test_exchange_rejects_bad_cells():
    g = W.c2_inputs(32)
    g.rho[3, 3] = -1.0
    E2, eps2, rc, _ = _exchange_gpu(g)
    assert rc == fld.FLD_ERR_BAD_INPUT
    assert E2[3, 3] == g.E[3, 3] and eps2[3, 3] == g.eps[3, 3]
