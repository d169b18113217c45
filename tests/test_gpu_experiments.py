"""The paper's two hot-path experiments run through the device path (Sec. 4.1
heating and cooling; Sec. 4.4 optically thin limit), with the parameters the
paper states (tests/golden) and CGS constants, checked against the FP64 oracle
step by step and against the behaviour the paper reports."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import oracle as O                     # noqa: E402
import workloads as W                  # noqa: E402
import paper_2104_03968_amd as fld     # noqa: E402
from tests.gpu_common import dev       # noqa: E402


def equilibrium(g0):
    """e_eq with a_r (e / (rho c_v))^4 = E_eq and E_eq + e_eq = E0 + e0 (bisection)."""
    rho, E0, e0 = g0.rho[0, 0], g0.E[0, 0], g0.eps[0, 0]
    lo, hi = 0.0, E0 + e0
    for _ in range(300):
        mid = 0.5 * (lo + hi)
        f = g0.a_r * (mid / (rho * g0.c_v)) ** 4 - (E0 + e0 - mid)
        lo, hi = (mid, hi) if f < 0 else (lo, mid)
    e_eq = 0.5 * (lo + hi)
    return e_eq, E0 + e0 - e_eq


def e_equil_for(fac):
    """e_eq for an initial gas energy fac * e_eq: fixed point of the map above."""
    g = W.e1_grid(1.0)
    e_eq = 1.0
    for _ in range(60):
        g.eps[:] = fac * e_eq
        e_new, _ = equilibrium(g)
        if abs(e_new - e_eq) <= 1e-15 * e_new:
            break
        e_eq = e_new
    return e_eq


@pytest.mark.parametrize("dt", W.E1_HEATCOOL["dts"])
@pytest.mark.parametrize("fac", W.E1_HEATCOOL["e_factors"])
def test_heating_cooling_relaxation_on_device(fac, dt):
    e_eq = e_equil_for(fac)
    g = W.e1_grid(fac * e_eq)
    E_eq = g.E[0, 0] + g.eps[0, 0] - e_eq
    plan = fld.Plan([g.E.shape], h=[g.h], c=g.c)
    E, eps, rho, kap = dev(g.E), dev(g.eps), dev(g.rho), dev(g.kappa)
    gas = fld.fld_gas_default(c=g.c, a_rad=g.a_r, c_v=g.c_v)
    # the oracle on one cell of the uniform box: no faces, so its implicit stage is the
    # identity exactly (on a larger copy its sparse LU of I + dt L, with face weights
    # ~1e8 here, would add cond(A) eps to E at every step)
    Eo, eo = g.E[:1, :1].copy(), g.eps[:1, :1].copy()
    hist = [g.eps[0, 0]]
    steps = int(round(5e-9 / dt))
    for s in range(steps):
        rc, _ = plan.imex_step([E], [eps], [rho], [kap], [dt], gas=gas, scheme="euler")
        assert rc == fld.FLD_OK
        Eo, eo = O.imex_step(Eo, eo, g.rho[:1, :1], g.kappa[:1, :1], dt, g.h, c=g.c, a_r=g.a_r, c_v=g.c_v,
                             scheme="euler")
        if s % 50 == 0 or s == steps - 1:
            e_gpu, E_gpu = eps.cpu().numpy(), E.cpu().numpy()
            assert np.all(e_gpu == e_gpu[0, 0]) and np.all(E_gpu == E_gpu[0, 0])      # stays uniform
            # the exchange roots agree to a few ulp of E + eps per step
            assert abs(e_gpu[0, 0] - eo[0, 0]) <= 1e-9 * e_eq, (s, e_gpu[0, 0], eo[0, 0])
            assert abs(E_gpu[0, 0] - Eo[0, 0]) <= 1e-12 * E_eq, (s, E_gpu[0, 0], Eo[0, 0])
            # the total carries one rounding of E per step
            assert E_gpu[0, 0] + e_gpu[0, 0] == pytest.approx(g.E[0, 0] + g.eps[0, 0], rel=1e-12)
            hist.append(e_gpu[0, 0])
    hist = np.array(hist)
    d = np.diff(hist)
    if fac < 1:
        assert np.all(d >= 0) and hist[-1] < e_eq * (1 + 1e-9)          # heats from below
        assert hist[-1] > 0.02 * e_eq
    else:
        assert np.all(d <= 0) and hist[-1] > e_eq * (1 - 1e-9)          # cools from above
        assert hist[-1] < 2 * e_eq
    E_gpu = E.cpu().numpy()[0, 0]
    assert abs(E_gpu - g.E[0, 0]) / g.E[0, 0] < 1e-2                    # E stays essentially constant
    # longer steps: the box settles on the equilibrium
    for _ in range(200):
        plan.imex_step([E], [eps], [rho], [kap], [1e-8], gas=gas, scheme="euler")
    assert eps.cpu().numpy()[0, 0] == pytest.approx(e_eq, rel=1e-6)
    assert E.cpu().numpy()[0, 0] == pytest.approx(E_eq, rel=1e-9)
    plan.close()


@pytest.mark.parametrize("limiter", ["lp", "diffusion"])
def test_optically_thin_front_on_device(limiter):
    """Each step starts from the oracle's previous state (the 22 decades between E1 and
    E0 put the far field below any residual-based stop rule), is compared with the
    oracle's step, and the front of the device's steps is checked: with the limiter it
    moves no faster than c; with lambda = 1/3 it runs ahead."""
    g = W.e4_grid(4)
    p = W.E4_THIN
    hx = g.h[0]
    xc = p["x_lo"] + (np.arange(p["n"]) + 0.5) * hx
    plan = fld.Plan([g.E.shape], h=[g.h], c=g.c, limiter=fld.LIMITER_CODES[limiter])
    K = dev(g.kappa_rho)
    x_or = g.E.copy()
    steps = 60
    for s in range(steps):
        E_in = dev(x_or)
        out = torch.empty_like(E_in)
        rc, (st,) = plan.step([E_in], [K], [out], [g.dt])
        assert rc == fld.FLD_OK
        x_gpu = out.cpu().numpy()
        x_next, _ = O.diffusion_step(x_or, g.kappa_rho, g.dt, g.h, c=g.c, limiter=limiter, method="direct")
        bound = 8 * (st["rel_residual"] + 1e-13) * st["b_norm"] + 1e-12 * np.abs(x_next)
        assert np.all(np.abs(x_gpu - x_next) <= bound), (s, np.max(np.abs(x_gpu - x_next) / bound))
        x_or = x_next
    t = steps * g.dt
    row = x_gpu[0]
    half = 0.5 * p["E1"]
    front = xc[np.nonzero(row < half)[0][0]]
    ahead = xc > g.c * t + 8 * hx
    frac = (np.clip(row[ahead], 0, None)).sum() / row.sum()
    if limiter == "lp":
        assert 0.5 * g.c * t <= front <= g.c * t + 3 * hx
        assert frac < 1e-2
    else:
        assert frac > 0.2
    plan.close()
