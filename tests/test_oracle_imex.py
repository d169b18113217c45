"""Pins of the radiation-only IMEX oracle (Sec. 3.1 splitting, Sec. 3.3 exchange,
Sec. 3.4 diffusion): total-energy conservation, radiative equilibrium as a fixed
point, the temporal order of the Euler (1) and midpoint (2) schemes measured by
step halving, and the work done by an expanding flow."""
import numpy as np
import pytest

import oracle as O
import workloads as W


def _state(shape, seed, span=(-1.0, 1.0)):
    g = W.random_grid(shape, seed, dt=1e-3)
    kappa = 10.0 ** W.span(W.smooth_field(shape, seed + 5), *span)
    rho = np.full(shape, 1.0)
    eps = g.E ** 0.25 * (1.0 + 0.3 * W.smooth_field(shape, seed + 6))
    eps = np.abs(eps) + 0.1
    return g.E, eps, rho, kappa, g.h


@pytest.mark.parametrize("scheme", ["euler", "midpoint"])
def test_total_energy_is_conserved(scheme):
    E, eps, rho, kappa, h = _state((24, 20), 901)
    E1, eps1 = O.imex_step(E, eps, rho, kappa, 5e-3, h, scheme=scheme)
    assert (E1 + eps1).sum() == pytest.approx((E + eps).sum(), rel=1e-12)
    assert np.all(E1 > 0) and np.all(eps1 > 0)


@pytest.mark.parametrize("scheme", ["euler", "midpoint"])
def test_radiative_equilibrium_is_a_fixed_point(scheme):
    """Uniform T with E = a_r T^4 and eps = rho c_v T: no gradient, no net exchange."""
    shape = (12, 10)
    T = 1.7
    a_r, c_v = 0.8, 1.3
    rho = np.full(shape, 2.0)
    E = np.full(shape, a_r * T ** 4)
    eps = rho * c_v * T
    kappa = np.full(shape, 3.0)
    E1, eps1 = O.imex_step(E, eps, rho, kappa, 0.1, (1 / 10, 1 / 12), a_r=a_r, c_v=c_v, scheme=scheme)
    assert np.allclose(E1, E, rtol=1e-12) and np.allclose(eps1, eps, rtol=1e-12)


def _rate(scheme, state, T, **kw):
    """Observed order from errors against a fine midpoint run at dt = T/8 and T/16.

    The midpoint step amplifies a stiff mode by (1 + z/2)/(1 - z/2), z = dt mu (the
    reused implicit tendency makes it the trapezoidal rule there): stable, but the
    asymptotic rate only shows once dt |mu| is moderate, hence the finer steps."""
    E, eps, rho, kappa, h = state
    Er, er = E, eps
    for _ in range(256):
        Er, er = O.imex_step(Er, er, rho, kappa, T / 256, h, scheme="midpoint", **kw)

    def err(n):
        Ex, ex = E, eps
        for _ in range(n):
            Ex, ex = O.imex_step(Ex, ex, rho, kappa, T / n, h, scheme=scheme, **kw)
        return np.linalg.norm(Ex - Er) + np.linalg.norm(ex - er)
    return np.log2(err(8) / err(16))


@pytest.mark.parametrize("with_v", [False, True])
def test_temporal_order_without_the_exchange(with_v):
    """Linear diffusion (lambda = 1/3) and the tiring source: Euler is first order, the
    midpoint scheme (eqs. G_expl - G_implexpl) second order."""
    shape = (16, 16)
    state = _state(shape, 911, span=(-0.5, 0.5))
    kw = dict(limiter="diffusion", exchange=False)
    if with_v:
        coords = np.meshgrid(*[(np.arange(s) + 0.5) for s in shape], indexing="ij")
        h = state[4]
        kw["v"] = [np.sin(3 * coords[0] * h[1]) * 0.4, np.cos(2 * coords[1] * h[0]) * 0.3]
    T = 2e-3 if with_v else 2e-2                       # the tiring term reaches its rate later
    assert abs(_rate("euler", state, T, **kw) - 1) < 0.25
    assert abs(_rate("midpoint", state, T, **kw) - 2) < 0.25


def test_exchange_stage_converges_first_order():
    """The local implicit exchange is a backward-Euler stage in both schemes."""
    state = _state((16, 16), 912, span=(-0.5, 0.5))
    for scheme in ("euler", "midpoint"):
        assert abs(_rate(scheme, state, 4e-3) - 1) < 0.3


def test_expansion_removes_radiation_energy():
    shape = (16, 16)
    E, eps, rho, kappa, h = _state(shape, 921)
    coords = np.meshgrid(*[(np.arange(s) + 0.5) for s in shape], indexing="ij")
    v = [coords[1] * h[0] * 0.5, coords[0] * h[1] * 0.5]
    for scheme in ("euler", "midpoint"):
        E1, eps1 = O.imex_step(E, eps, rho, kappa, 1e-3, h, scheme=scheme, v=v)
        E0, eps0 = O.imex_step(E, eps, rho, kappa, 1e-3, h, scheme=scheme)
        assert (E1 + eps1).sum() < (E0 + eps0).sum()
