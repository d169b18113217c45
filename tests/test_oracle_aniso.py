"""Pins of the diagonal-tensor (anisotropic) diffusion oracle: the isotropic case,
the spectral (DCT-II) solution for constant per-direction coefficients, the
per-axis growth of a pulse's variance, the free-streaming bound per direction, and
planted mistakes (swapped directions, one opacity for all faces) that must fail."""
import numpy as np
import pytest
import scipy.fft

import oracle as O
import workloads as W


def _dct_solve_aniso(E, Dd, dt, h):
    """(I + dt sum_d D_d L_d)^{-1} E for constant D_d under zero flux: the orthonormal
    DCT-II diagonalises each 1D Neumann Laplacian with eigenvalues (4/h^2) sin^2(pi k/(2n))."""
    nd = E.ndim
    Ehat = scipy.fft.dctn(E, type=2, norm="ortho")
    lam = np.zeros_like(E)
    for d in range(nd):
        n = E.shape[nd - 1 - d]
        k = np.arange(n)
        ev = Dd[d] * 4.0 / h[d] ** 2 * np.sin(np.pi * k / (2 * n)) ** 2
        sh = [1] * nd
        sh[nd - 1 - d] = n
        lam = lam + ev.reshape(sh)
    return scipy.fft.idctn(Ehat / (1.0 + dt * lam), type=2, norm="ortho")


@pytest.mark.parametrize("shape", [(40, 36), (10, 12, 14)])
def test_equal_opacities_give_the_isotropic_step(shape):
    g = W.random_grid(shape, 61000 + len(shape), dt=3e-3)
    for lim in ("lp", "minerbo"):
        xa, _ = O.diffusion_step_aniso(g.E, [g.kappa_rho] * len(shape), g.dt, g.h, c=1.7, limiter=lim,
                                       method="direct")
        xi, _ = O.diffusion_step(g.E, g.kappa_rho, g.dt, g.h, c=1.7, limiter=lim, method="direct")
        assert np.allclose(xa, xi, rtol=1e-13, atol=0)


@pytest.mark.parametrize("shape,h", [((24, 30), (1 / 30, 1 / 24)), ((6, 8, 10), (0.1, 0.125, 0.2))])
def test_dct_closed_form_per_direction(shape, h):
    """lambda = 1/3 and a constant, different kappa rho per direction."""
    rng = np.random.default_rng(8)
    E = 1.0 + rng.random(shape)
    krs = [0.4, 3.0, 11.0][:len(shape)]
    c, dt = 1.3, 2e-3
    Dd = [c / (3 * k) for k in krs]
    ref = _dct_solve_aniso(E, Dd, dt, h)
    x, _ = O.diffusion_step_aniso(E, [np.full(shape, k) for k in krs], dt, h, c=c, limiter="diffusion",
                                  method="direct")
    assert np.abs(x - ref).max() / np.abs(ref).max() < 1e-12
    # the same with the directions swapped is a different solution
    swapped = _dct_solve_aniso(E, Dd[::-1], dt, h)
    assert np.abs(x - swapped).max() / np.abs(ref).max() > 1e-4


def test_pulse_variance_grows_per_axis():
    """Backward Euler with constant D_d: the variance along axis d grows by exactly
    2 D_d dt per step (the discrete Laplacian of a quadratic is exact)."""
    nx, ny = 96, 64
    h = (1.0 / nx, 1.5 / ny)
    xc = (np.arange(nx) + 0.5) * h[0]
    yc = (np.arange(ny) + 0.5) * h[1]
    X, Y = np.meshgrid(xc, yc, indexing="xy")
    u0 = 1e3 * np.exp(-((X - 0.5) ** 2 + (Y - 0.75) ** 2) / (2 * 0.05 ** 2))
    E = 1.0 + u0
    krx, kry, c, dt = 5.0, 1.25, 2.0, 2e-4
    Dx, Dy = c / (3 * krx), c / (3 * kry)
    x = E.copy()
    mass = u0.sum()
    vx = [((X - 0.5) ** 2 * u0).sum() / mass]
    vy = [((Y - 0.75) ** 2 * u0).sum() / mass]
    for _ in range(3):
        x, _ = O.diffusion_step_aniso(x, [np.full_like(E, krx), np.full_like(E, kry)], dt, h, c=c,
                                      limiter="diffusion", method="direct")
        u = x - 1.0
        vx.append(((X - 0.5) ** 2 * u).sum() / mass)
        vy.append(((Y - 0.75) ** 2 * u).sum() / mass)
    assert np.allclose(np.diff(vx), 2 * Dx * dt, rtol=1e-6)
    assert np.allclose(np.diff(vy), 2 * Dy * dt, rtol=1e-6)


def test_free_streaming_bound_per_direction():
    """|F_d| = D_d |dE/dx_d| <= c E whatever the opacity of direction d (Sec. 2.2)."""
    g = W.random_grid((48, 40), 61100, dt=1e-3)
    krs = [g.kappa_rho * 1e-6, g.kappa_rho * 1e4]
    Ds = O.diffusion_tensor(g.E, krs, g.h, c=2.0)
    grads = O.gradient4(g.E, g.h)
    gnorm = np.sqrt(sum(x * x for x in grads))
    for d in range(2):
        assert np.all(Ds[d] * gnorm <= 2.0 * g.E * (1 + 1e-12))
    # thin along x: D_x approaches c E / |grad E|; thick along y: D_y -> c / (3 kappa rho)_y
    assert np.allclose(Ds[0] * gnorm, 2.0 * g.E, rtol=1e-3)
    thick = gnorm / (krs[1] * g.E) < 0.01
    assert thick.sum() > 100 and np.all(np.abs(Ds[1] * 3 * krs[1] / 2.0 - 1)[thick] < 0.01)


def test_planted_mistakes_fail():
    """A kernel that swapped the directions or used the x opacity for every face would
    differ from the oracle by far more than rounding."""
    g = W.random_grid((32, 28), 61200, dt=5e-3)
    krs = [g.kappa_rho, g.kappa_rho * 7.0]
    x, _ = O.diffusion_step_aniso(g.E, krs, g.dt, g.h, method="direct")
    xs, _ = O.diffusion_step_aniso(g.E, krs[::-1], g.dt, g.h, method="direct")
    x1, _ = O.diffusion_step(g.E, krs[0], g.dt, g.h, method="direct")
    scale = np.abs(x).max()
    assert np.abs(x - xs).max() > 1e-6 * scale and np.abs(x - x1).max() > 1e-6 * scale
