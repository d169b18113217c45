"""Pins of the fixed-gradient boundary oracle (Sec. 3.4 Neumann conditions): zero
gradients give the zero-flux step, the ghost rule is exact for linear profiles, a
linear profile with matching face gradients is a steady state, the energy budget
equals the boundary fluxes exactly, and a planted sign error fails."""
import numpy as np
import pytest

import oracle as O
import workloads as W


@pytest.mark.parametrize("shape", [(30, 26), (8, 10, 12)])
def test_zero_gradients_give_the_zero_flux_step(shape):
    g = W.random_grid(shape, 63000 + len(shape), dt=3e-3)
    xa, _ = O.diffusion_step_bc(g.E, g.kappa_rho, g.dt, g.h, grad_bc=[0.0] * 6, method="direct")
    xb, _ = O.diffusion_step(g.E, g.kappa_rho, g.dt, g.h, method="direct")
    assert np.array_equal(xa, xb) or np.allclose(xa, xb, rtol=1e-14, atol=0)
    ga = O.gradient4_bc(g.E, g.h, None)
    gb = O.gradient4(g.E, g.h)
    for a, b in zip(ga, gb):
        assert np.allclose(a, b, rtol=1e-14, atol=1e-14 * np.abs(b).max())


def test_ghost_rule_exact_for_linear_profiles():
    nx, ny, nz = 9, 7, 6
    h = (0.3, 0.2, 0.5)
    G = (1.5, -0.7, 2.25)
    X = (np.arange(nx) + 0.5) * h[0]
    Y = (np.arange(ny) + 0.5) * h[1]
    Z = (np.arange(nz) + 0.5) * h[2]
    E = 10.0 + G[0] * X[None, None, :] + G[1] * Y[None, :, None] + G[2] * Z[:, None, None]
    gr = O.gradient4_bc(E, h, [G[0], G[0], G[1], G[1], G[2], G[2]])
    for d in range(3):
        assert np.allclose(gr[d], G[d], rtol=1e-12, atol=1e-12)


def test_linear_profile_with_matching_gradients_is_steady():
    """lambda = 1/3 and constant kappa rho: interior fluxes and the two boundary fluxes
    are all D G, so every cell's content is unchanged."""
    nx, ny = 64, 12
    h = (1.0 / nx, 0.5 / ny)
    G = 3.0
    X = (np.arange(nx) + 0.5) * h[0]
    E = np.tile(5.0 + G * X, (ny, 1))
    x, info = O.diffusion_step_bc(E, np.full(E.shape, 2.0), 0.05, h, grad_bc=[G, G, 0, 0], limiter="diffusion",
                                  method="direct")
    assert np.allclose(x, E, rtol=1e-12, atol=0)
    # the same profile under zero flux relaxes (the walls block the flux)
    x0, _ = O.diffusion_step(E, np.full(E.shape, 2.0), 0.05, h, limiter="diffusion", method="direct")
    assert np.abs(x0 - E).max() > 1e-3


@pytest.mark.parametrize("shape", [(40, 36), (10, 12, 14)])
def test_energy_budget_is_the_boundary_flux(shape):
    """A = I + dt L has unit column sums, so sum(E^{n+1}) - sum(E^n) equals the summed
    boundary source (dt / h) (-D G_lo) and (dt / h) (D G_hi), for any limiter."""
    g = W.random_grid(shape, 63100 + len(shape), dt=4e-3)
    gb = [0.3, -1.1, 2.0, 0.5, -0.4, 0.8][:2 * len(shape)]
    x, info = O.diffusion_step_bc(g.E, g.kappa_rho, g.dt, g.h, grad_bc=gb, method="direct")
    src = info.extra["b"] - g.E
    assert (x.sum() - g.E.sum()) == pytest.approx(src.sum(), rel=1e-10, abs=1e-12 * g.E.sum())
    # and that source sits on the boundary cells only: a positive gradient at the lower x
    # face drains the cells there (flux -D G < 0), a negative one at the upper x face too
    nd = len(shape)
    inner = tuple(slice(1, s - 1) for s in shape)
    assert np.all(src[inner] == 0.0)
    edge_lo = tuple([slice(1, s - 1) for s in shape[:-1]] + [0])
    edge_hi = tuple([slice(1, s - 1) for s in shape[:-1]] + [shape[-1] - 1])
    assert np.all(src[edge_lo] < 0) and np.all(src[edge_hi] < 0)


def test_planted_sign_error_fails_the_steady_state():
    nx, ny = 32, 4
    h = (1.0 / nx, 1.0 / ny)
    G = 2.0
    X = (np.arange(nx) + 0.5) * h[0]
    E = np.tile(5.0 + G * X, (ny, 1))
    kr = np.full(E.shape, 1.0)
    # an implementation with the lower source sign flipped is the oracle with -G below
    x_bad, _ = O.diffusion_step_bc(E, kr, 0.05, h, grad_bc=[-G, G, 0, 0], limiter="diffusion",
                                   method="direct")
    assert np.abs(x_bad - E).max() > 1e-3
