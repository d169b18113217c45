"""Pins of the Dirichlet-boundary oracle (Sec. 3.4, ghost cells holding E^{n+1}):
the discrete sine transform solves the constant-coefficient step exactly, a field
equal to the ghost value is steady, the energy budget is the flow through the
Dirichlet faces, the operator is symmetric positive definite, the general ghost
rule reproduces the zero-flux and fixed-gradient oracles, and a planted error in
the ghost distance fails the closed form."""
import numpy as np
import pytest
import scipy.fft as F
import scipy.sparse as sp

import oracle as O
import workloads as W

D3 = 1.0 / 3.0


def _closed_form(E, kr, dt, h, kinds, EB=0.0):
    """lambda = 1/3, constant kappa rho, ghost value 0: per axis DST-I (Dirichlet at both
    ends, ghosts at one cell width) or DCT-II (zero flux at both ends)."""
    nd = E.ndim
    D = D3 / kr
    X = E.copy()
    denom = np.ones(E.shape)
    for d in range(nd):
        a = nd - 1 - d
        n = E.shape[a]
        k = np.arange(n)
        if kinds[2 * d] == "dirichlet":
            X = F.dst(X, type=1, axis=a, norm="ortho")
            lam = 4.0 * np.sin(np.pi * (k + 1) / (2.0 * (n + 1))) ** 2
        else:
            X = F.dct(X, type=2, axis=a, norm="ortho")
            lam = 4.0 * np.sin(np.pi * k / (2.0 * n)) ** 2
        shp = [1] * nd
        shp[a] = n
        denom = denom + dt * D / h[d] ** 2 * lam.reshape(shp)
    X = X / denom
    for d in range(nd):
        a = nd - 1 - d
        if kinds[2 * d] == "dirichlet":
            X = F.idst(X, type=1, axis=a, norm="ortho")
        else:
            X = F.idct(X, type=2, axis=a, norm="ortho")
    return X


@pytest.mark.parametrize("shape,kinds", [
    ((24, 30), ["dirichlet", "dirichlet", "zero_flux", "zero_flux"]),
    ((16, 20), ["zero_flux", "zero_flux", "dirichlet", "dirichlet"]),
    ((10, 12, 14), ["dirichlet"] * 6),
    ((8, 10, 12), ["dirichlet", "dirichlet", "zero_flux", "zero_flux", "dirichlet", "dirichlet"])])
def test_sine_transform_closed_form(shape, kinds):
    rng = np.random.default_rng(7 + len(shape))
    E = 1.0 + rng.random(shape)
    kr = 2.5
    h = [0.05, 0.04, 0.03][:len(shape)]
    dt = 4e-3
    x, info = O.diffusion_step_general(E, np.full(shape, kr), dt, h, kinds, [0.0] * 6, limiter="diffusion",
                                       method="direct")
    want = _closed_form(E, kr, dt, h, kinds)
    assert np.abs(x - want).max() <= 1e-12 * np.abs(want).max()


def test_planted_ghost_distance_error_fails_the_closed_form():
    """A ghost at half a cell width (twice the coupling) is a plausible mistake."""
    shape, kinds = (20, 24), ["dirichlet", "dirichlet", "zero_flux", "zero_flux"]
    rng = np.random.default_rng(3)
    E = 1.0 + rng.random(shape)
    h, dt, kr = [0.05, 0.05], 4e-3, 2.5
    _, info = O.diffusion_step_general(E, np.full(shape, kr), dt, h, kinds, [0.0] * 6, limiter="diffusion",
                                       method="direct")
    A_bad = info.extra["A"] + sp.diags(info.extra["alpha"].ravel())
    x_bad = sp.linalg.spsolve(A_bad.tocsc(), E.ravel()).reshape(shape)
    want = _closed_form(E, kr, dt, h, kinds)
    assert np.abs(x_bad - want).max() > 1e-6 * np.abs(want).max()


@pytest.mark.parametrize("limiter", ["lp", "minerbo"])
@pytest.mark.parametrize("shape", [(20, 16), (6, 8, 10)])
def test_field_at_the_ghost_value_is_steady(shape, limiter):
    g = W.random_grid(shape, 71500 + len(shape), dt=5e-3)
    EB = 2.75
    E = np.full(shape, EB)
    kinds = ["dirichlet", "zero_flux", "dirichlet", "dirichlet", "zero_flux", "dirichlet"]
    x, info = O.diffusion_step_general(E, g.kappa_rho, g.dt, g.h, kinds, [EB] * 6, limiter=limiter,
                                       method="direct")
    assert np.abs(x - EB).max() <= 1e-13 * EB
    for gd in O.gradient4_general(E, g.h, kinds, [EB] * 6):
        assert np.abs(gd).max() == 0.0


@pytest.mark.parametrize("shape", [(24, 20), (8, 10, 6)])
def test_energy_budget_is_the_flow_through_dirichlet_faces(shape):
    g = W.random_grid(shape, 71600 + len(shape), dt=4e-3)
    kinds = ["dirichlet", "gradient", "zero_flux", "dirichlet", "dirichlet", "zero_flux"]
    vals = [0.5, 0.3, 0.0, 3.0, 1.5, 0.0]
    x, info = O.diffusion_step_general(g.E, g.kappa_rho, g.dt, g.h, kinds, vals, method="direct")
    A, b, alpha = info.extra["A"], info.extra["b"], info.extra["alpha"]
    r = b.ravel() - A @ x.ravel()
    # 1^T A = 1^T + alpha^T: sum x - sum E^n = sum of the face sources minus sum alpha x - sum r
    src = (b - g.E).sum()
    lhs = x.sum() - g.E.sum()
    assert abs(lhs - (src - (alpha * x).sum())) <= np.abs(r).sum() + 1e-13 * abs(g.E.sum())
    assert (alpha > 0).sum() > 0


@pytest.mark.parametrize("shape", [(12, 10), (6, 5, 4)])
def test_operator_is_spd_with_lambda_min_at_least_one(shape):
    g = W.random_grid(shape, 71700 + len(shape), dt=1e-2)
    kinds = ["dirichlet"] * 6
    _, info = O.diffusion_step_general(g.E, g.kappa_rho, g.dt, g.h, kinds, [1.0] * 6, method="lu")
    A = info.extra["A"].toarray()
    assert np.abs(A - A.T).max() == 0.0
    ev = np.linalg.eigvalsh(A)
    assert ev.min() >= 1.0 - 1e-12
    # each boundary cell's diagonal exceeds its off-diagonal row sum by 1 + alpha
    off = np.abs(A - np.diag(np.diag(A))).sum(axis=1)
    assert np.allclose(np.diag(A) - off, 1.0 + info.extra["alpha"].ravel(), rtol=0, atol=1e-12)


@pytest.mark.parametrize("shape", [(18, 14), (7, 9, 8)])
def test_general_rule_reduces_to_the_other_boundary_oracles(shape):
    g = W.random_grid(shape, 71800 + len(shape), dt=3e-3)
    G = [0.4, -0.2, 0.1, 0.0, -0.3, 0.25]
    kinds = ["gradient"] * 6
    for a, b in zip(O.gradient4_general(g.E, g.h, kinds, G), O.gradient4_bc(g.E, g.h, G)):
        assert np.allclose(a, b, rtol=1e-14, atol=1e-14 * np.abs(b).max())
    for a, b in zip(O.gradient4_general(g.E, g.h, None, None), O.gradient4(g.E, g.h)):
        assert np.allclose(a, b, rtol=1e-14, atol=1e-14 * np.abs(b).max())
    xa, _ = O.diffusion_step_general(g.E, g.kappa_rho, g.dt, g.h, kinds, G, method="direct")
    xb, _ = O.diffusion_step_bc(g.E, g.kappa_rho, g.dt, g.h, grad_bc=G, method="direct")
    assert np.allclose(xa, xb, rtol=1e-12, atol=0)


def test_unknown_kind_is_rejected():
    with pytest.raises(ValueError):
        O.gradient4_general(np.ones((4, 4)), (0.25, 0.25), ["open"] * 4, None)
