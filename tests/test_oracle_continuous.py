"""Pins of the continuous-boundary oracle (Sec. 3.4: E^{n+1} extrapolated linearly
into the ghost cells).

* The 4th-order gradient over the extrapolated ghosts is exact for linear fields at
  every cell, the boundary cells included.
* A linear profile is a steady state of the step (constant D): no divergence at the
  boundary cells, where a zero-flux face would bend it.
* Closed form (constant D, continuous x faces, zero-flux y faces): a DCT-II along y
  decouples the y-modes; in each mode the boundary cells' x-rows lose their coupling,
  so they keep b / (1 + w_y lambda_y), and the interior is the Dirichlet problem with
  those end values, solved by a DST-I.
* LU == SuperLU == Gauss-Seidel on tiny grids (the operator is an M-matrix but not
  symmetric).
* Planted mistakes (mirror ghosts, a flipped coupling sign, constant-extrapolated
  gradient ghosts) fail a pin."""
import numpy as np
import pytest
import scipy.fft as F
import scipy.sparse as sp

import oracle as O
from oracle import dirichlet as OD

D3 = 1.0 / 3.0
CONT_X = ["continuous", "continuous", "zero_flux", "zero_flux"]


@pytest.mark.parametrize("shape", [(12, 16), (6, 8, 10)])
def test_gradient_exact_for_linear_fields(shape):
    nd = len(shape)
    h = [0.05, 0.04, 0.03][:nd]
    coef = [0.7, -1.3, 0.4][:nd]
    E = np.full(shape, 2.0)
    for d in range(nd):
        a = nd - 1 - d
        xc = (np.arange(shape[a]) + 0.5) * h[d]
        sh = [1] * nd
        sh[a] = shape[a]
        E = E + coef[d] * xc.reshape(sh)
    g = OD.gradient4_general(E, h, ["continuous"] * (2 * nd))
    for d in range(nd):
        assert np.allclose(g[d], coef[d], rtol=0, atol=1e-12), d
    # the mirror ghosts of zero flux bend the gradient at the boundary cells
    g0 = OD.gradient4_general(E, h, ["zero_flux"] * (2 * nd))
    assert not np.allclose(g0[0], coef[0], atol=1e-6)


def test_linear_profile_is_steady():
    shape = (10, 24)
    h = [1.0 / 24, 1.0 / 10]
    x = (np.arange(24) + 0.5) / 24
    E = np.broadcast_to(1.0 + 0.8 * x, shape).copy()
    kr = np.full(shape, 3.0)
    xs, info = OD.diffusion_step_general(E, kr, 2e-2, h, CONT_X, limiter="diffusion", method="direct")
    assert np.abs(xs - E).max() <= 1e-13 * E.max()
    xz, _ = OD.diffusion_step_general(E, kr, 2e-2, h, ["zero_flux"] * 4, limiter="diffusion", method="direct")
    assert np.abs(xz - E).max() > 1e-3            # zero flux bends the profile at the faces


def closed_form_cont_x(b, w_x, w_y):
    """(I + dt L) x = b for constant weights, continuous x faces and zero-flux y faces."""
    ny, nx = b.shape
    B = F.dct(b, type=2, axis=0, norm="ortho")
    lam_y = 4.0 * np.sin(np.pi * np.arange(ny) / (2.0 * ny)) ** 2
    X = np.empty_like(B)
    m = nx - 2
    k = np.arange(1, m + 1)
    lam_x = 4.0 * np.sin(np.pi * k / (2.0 * (m + 1))) ** 2
    for ky in range(ny):
        dgy = 1.0 + w_y * lam_y[ky]
        u0 = B[ky, 0] / dgy
        un = B[ky, -1] / dgy
        rhs = B[ky, 1:-1].copy()
        rhs[0] += w_x * u0
        rhs[-1] += w_x * un
        R = F.dst(rhs, type=1, norm="ortho")
        U = F.idst(R / (dgy + w_x * lam_x), type=1, norm="ortho")
        X[ky, 0], X[ky, -1], X[ky, 1:-1] = u0, un, U
    return F.idct(X, type=2, axis=0, norm="ortho")


@pytest.mark.parametrize("shape", [(9, 14), (16, 31)])
def test_closed_form_constant_coefficients(shape):
    rng = np.random.default_rng(11)
    E = 1.0 + rng.random(shape)
    kr = 2.0
    h = [0.03, 0.05]
    dt = 5e-3
    x, info = OD.diffusion_step_general(E, np.full(shape, kr), dt, h, CONT_X, limiter="diffusion",
                                        method="direct")
    D = D3 / kr
    ref = closed_form_cont_x(E, dt * D / h[0] ** 2, dt * D / h[1] ** 2)
    assert np.abs(x - ref).max() <= 1e-12 * np.abs(ref).max()


def test_direct_lu_and_gauss_seidel_agree():
    rng = np.random.default_rng(5)
    for shape in [(6, 7), (4, 5, 6)]:
        nd = len(shape)
        E = 1.0 + rng.random(shape)
        kr = 10.0 ** rng.uniform(-1, 1, shape)
        h = [1.0 / s for s in reversed(shape)]
        kinds = ["continuous", "zero_flux", "continuous", "continuous", "zero_flux", "continuous"][:2 * nd]
        xl, info = OD.diffusion_step_general(E, kr, 3e-3, h, kinds, method="lu")
        A, b = info.extra["A"], info.extra["b"]
        xd = sp.linalg.spsolve(A.tocsc(), b.ravel()).reshape(shape)
        xg, _ = O.solve(A, b, method="gs", tol=1e-14)
        assert np.abs(xl - xd).max() <= 1e-12 * np.abs(xd).max()
        assert np.abs(xg - xd).max() <= 1e-11 * np.abs(xd).max()


def test_operator_is_an_m_matrix_and_not_symmetric():
    rng = np.random.default_rng(9)
    shape = (8, 9)
    E = 1.0 + rng.random(shape)
    kr = 10.0 ** rng.uniform(-1, 1, shape)
    _, info = OD.diffusion_step_general(E, kr, 1e-2, [1 / 9, 1 / 8], CONT_X, method="lu")
    A = info.extra["A"].toarray()
    off = A - np.diag(np.diag(A))
    assert (off <= 0).all() and (np.diag(A) >= 1.0 - 1e-15).all()
    assert np.abs(A - A.T).max() > 1e-6


# ---- planted mistakes -------------------------------------------------------------
def _mutated_step(E, kr, dt, h, mistake):
    """The oracle's continuous-face step with one plausible mistake planted."""
    gr = OD.gradient4_general(E, h, CONT_X)
    if mistake == "const_ghost_gradient":
        gr = OD.gradient4_general(E, h, ["zero_flux"] * 4)
    R = np.sqrt(sum(g * g for g in gr)) / (kr * E)
    D = O.flux_limiter(R, "diffusion") / kr
    w = O.face_weights(D, dt, h)
    A = O.assemble_operator(w)
    C = OD.continuous_coupling(w, CONT_X)
    if mistake == "mirror_ghost":
        C = C * 0.0
    elif mistake == "sign":
        C = -C
    A = (A + C).tocsr()
    return sp.linalg.spsolve(A.tocsc(), E.ravel()).reshape(E.shape), gr


@pytest.mark.parametrize("mistake", ["mirror_ghost", "sign", "const_ghost_gradient"])
def test_planted_mistakes_fail_a_pin(mistake):
    shape = (9, 14)
    h = [0.03, 0.05]
    dt = 5e-3
    rng = np.random.default_rng(11)
    E = 1.0 + rng.random(shape)
    kr = np.full(shape, 2.0)
    x, gr = _mutated_step(E, kr, dt, h, mistake)
    D = D3 / 2.0
    ref = closed_form_cont_x(E, dt * D / h[0] ** 2, dt * D / h[1] ** 2)
    xl = (np.arange(14) + 0.5) * h[0]
    lin = np.broadcast_to(2.0 + 0.7 * xl, shape)
    _, gl = _mutated_step(lin.copy(), kr, dt, h, mistake)
    closed_ok = np.abs(x - ref).max() <= 1e-12 * np.abs(ref).max()
    grad_ok = np.allclose(gl[0], 0.7, atol=1e-12)
    assert not (closed_ok and grad_ok), mistake
