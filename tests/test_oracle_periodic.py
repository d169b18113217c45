"""Pins of the periodic-boundary oracle: the discrete Fourier transform solves the
constant-coefficient step exactly (alone and mixed with DCT-II axes), shifting the
inputs along a periodic axis shifts the result (wrapped gradient, wrap face and
operator together), the mean is conserved, and unpaired periodic faces are rejected."""
import numpy as np
import pytest
import scipy.fft as F

import oracle as O
import workloads as W


def _closed_form(E, kr, dt, h, periodic_axes):
    """lambda = 1/3 and constant kappa rho: per axis the DFT (periodic, eigenvalues
    4 sin^2(pi k / n)) or the DCT-II (zero flux, 4 sin^2(pi k / (2 n)))."""
    nd = E.ndim
    D = 1.0 / (3.0 * kr)
    X = E.astype(complex)
    denom = np.ones(E.shape)
    for d in range(nd):
        a = nd - 1 - d
        n = E.shape[a]
        k = np.arange(n)
        if d in periodic_axes:
            X = F.fft(X, axis=a)
            lam = 4.0 * np.sin(np.pi * k / n) ** 2
        else:
            X = F.dct(X.real, type=2, axis=a, norm="ortho") + 1j * F.dct(X.imag, type=2, axis=a, norm="ortho")
            lam = 4.0 * np.sin(np.pi * k / (2.0 * n)) ** 2
        shp = [1] * nd
        shp[a] = n
        denom = denom + dt * D / h[d] ** 2 * lam.reshape(shp)
    X = X / denom
    for d in range(nd):
        a = nd - 1 - d
        if d in periodic_axes:
            X = F.ifft(X, axis=a)
        else:
            X = F.idct(X.real, type=2, axis=a, norm="ortho") + 1j * F.idct(X.imag, type=2, axis=a, norm="ortho")
    return X.real


@pytest.mark.parametrize("shape,axes", [((24, 30), (0,)), ((16, 20), (0, 1)), ((10, 12, 14), (0, 1, 2)),
                                        ((8, 10, 12), (1,))])
def test_fourier_closed_form(shape, axes):
    nd = len(shape)
    kinds = []
    for d in range(nd):
        kinds += ["periodic", "periodic"] if d in axes else ["zero_flux", "zero_flux"]
    rng = np.random.default_rng(17 + nd)
    E = 1.0 + rng.random(shape)
    h = [0.05, 0.04, 0.03][:nd]
    x, _ = O.diffusion_step_general(E, np.full(shape, 2.0), 5e-3, h, kinds, None, limiter="diffusion",
                                    method="direct")
    want = _closed_form(E, 2.0, 5e-3, h, axes)
    assert np.abs(x - want).max() <= 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("limiter", ["lp", "minerbo"])
@pytest.mark.parametrize("shape", [(20, 28), (8, 10, 12)])
def test_shift_along_a_periodic_axis_shifts_the_result(shape, limiter):
    g = W.random_grid(shape, 72000 + len(shape), dt=5e-3)
    nd = len(shape)
    kinds = ["periodic", "periodic"] + ["zero_flux"] * (2 * nd - 2)
    x0, _ = O.diffusion_step_general(g.E, g.kappa_rho, g.dt, g.h, kinds, None, limiter=limiter, method="direct")
    for s in (1, 5):
        Es = np.roll(g.E, s, axis=nd - 1)
        Ks = np.roll(g.kappa_rho, s, axis=nd - 1)
        xs, _ = O.diffusion_step_general(Es, Ks, g.dt, g.h, kinds, None, limiter=limiter, method="direct")
        assert np.allclose(xs, np.roll(x0, s, axis=nd - 1), rtol=1e-11, atol=0)
    # the zero-flux step is not shift invariant: the check has teeth
    z, _ = O.diffusion_step_general(np.roll(g.E, 5, axis=nd - 1), np.roll(g.kappa_rho, 5, axis=nd - 1), g.dt,
                                    g.h, None, None, limiter=limiter, method="direct")
    assert not np.allclose(z, np.roll(x0, 5, axis=nd - 1), rtol=1e-6, atol=0)


@pytest.mark.parametrize("shape", [(24, 20), (8, 10, 6)])
def test_mean_is_conserved(shape):
    g = W.random_grid(shape, 72100 + len(shape), dt=4e-3)
    kinds = ["periodic"] * (2 * len(shape))
    x, info = O.diffusion_step_general(g.E, g.kappa_rho, g.dt, g.h, kinds, None, method="direct")
    A = info.extra["A"]
    assert np.allclose(np.asarray(A.sum(axis=0)).ravel(), 1.0, rtol=0, atol=1e-12)
    r = info.extra["b"].ravel() - A @ x.ravel()
    assert abs(x.sum() - g.E.sum()) <= np.abs(r).sum() + 1e-13 * g.E.sum()


def test_unpaired_periodic_face_is_rejected():
    with pytest.raises(ValueError):
        O.gradient4_general(np.ones((4, 4)), (0.25, 0.25), ["periodic", "zero_flux", "zero_flux", "zero_flux"])
