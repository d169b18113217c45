"""Pins of the radiation-moment oracle (flux, force, Eddington factor and tensor,
photon tiring) against limits and identities the paper and the mathematics fix
(Sec. 2.2: the thick and free-streaming limits, causality, the Eddington
tensor's form; Sec. 3.2: the 4th-order gradient, exact on low-degree
polynomials away from the walls)."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _field(shape, seed, span=(-2.0, 2.0)):
    g = W.random_grid(shape, seed, dt=1e-3)
    kr = 10.0 ** W.span(W.smooth_field(shape, seed + 7), *span)
    return g.E, kr, g.h


def _full_tensor(P, nd):
    comps = O.tensor_components(nd)
    T = np.zeros(P[0].shape + (nd, nd))
    for k, (i, j) in enumerate(comps):
        T[..., i, j] = P[k]
        T[..., j, i] = P[k]
    return T


def test_uniform_field_is_the_isotropic_equilibrium():
    E = np.full((12, 16), 3.7)
    kr = 10.0 ** W.span(W.smooth_field((12, 16), 3), -2, 2)
    m = O.radiation_moments(E, kr, (1 / 16, 1 / 12))
    for Fi in m["F"] + m["f_r"]:
        assert np.max(np.abs(Fi)) <= 1e-12 * 3.7 * 16 / kr.min()
    assert np.allclose(m["f"], 1 / 3, rtol=0, atol=1e-12)
    P = m["P"]                                          # xx, xy, yy
    assert np.allclose(P[0], 3.7 / 3, rtol=1e-12) and np.allclose(P[2], 3.7 / 3, rtol=1e-12)
    assert np.max(np.abs(P[1])) <= 1e-12


@pytest.mark.parametrize("shape,span", [((40, 48), (-2, 2)), ((20, 24, 28), (-6, 6)), ((64, 64), (-10, -4))])
def test_flux_is_causal_and_down_the_gradient(shape, span):
    E, kr, h = _field(shape, 11 + len(shape), span)
    m = O.radiation_moments(E, kr, h, c=2.5)
    Fmag = np.sqrt(sum(Fi * Fi for Fi in m["F"]))
    assert np.all(Fmag <= 2.5 * E * (1 + 1e-12))           # |F| <= c E (Sec. 2.2)
    g = O.gradient4(E, h)
    assert np.all(sum(Fi * gi for Fi, gi in zip(m["F"], g)) <= 0.0)
    f = m["f"]
    assert np.all(f >= 1 / 3 - 1e-15) and np.all(f <= 1 + 1e-12)


def test_free_streaming_limit():
    """kappa rho -> 0: lambda -> 1/R, |F| -> c E and f -> 1 (Sec. 2.2)."""
    n = 64
    x = (np.arange(n) + 0.5) / n
    E = np.tile(1.0 + 1e3 * np.exp(-((x - 0.5) / 0.1) ** 2), (8, 1))
    kr = np.full_like(E, 1e-10)
    m = O.radiation_moments(E, kr, (1 / n, 1 / 8), c=3.0)
    Fmag = np.sqrt(sum(Fi * Fi for Fi in m["F"]))
    steep = np.abs(O.gradient4(E, (1 / n, 1 / 8))[0]) > 1.0
    assert np.all(Fmag[steep] / (3.0 * E[steep]) > 0.999)
    assert np.all(m["f"][steep] > 0.999)


def test_thick_limit_is_fickian_diffusion():
    """kappa rho -> inf: F -> -c/(3 kappa rho) grad E, f -> 1/3 (Sec. 2.2)."""
    E, _, h = _field((32, 40), 21)
    kr = np.full_like(E, 1e9)
    m = O.radiation_moments(E, kr, h, c=2.0)
    g = O.gradient4(E, h)
    for Fi, fi, gi in zip(m["F"], m["f_r"], g):
        assert np.allclose(Fi, -2.0 * gi / (3 * kr), rtol=1e-6, atol=0)
        # the force balances the gradient of the isotropic pressure E/3 (Eq. 1st_cmf, static)
        assert np.allclose(fi, -gi / 3, rtol=1e-6, atol=0)
    assert np.max(np.abs(m["f"] - 1 / 3)) < 1e-6


def test_pressure_tensor_eigenstructure_3d():
    """P has eigenvalue f E along grad E and (1-f)/2 E twice across it; tr P = E."""
    E, kr, h = _field((10, 12, 14), 31, (-3, 1))
    m = O.radiation_moments(E, kr, h)
    T = _full_tensor(m["P"], 3)
    lam, vec = np.linalg.eigh(T)
    f = m["f"]
    assert np.allclose(lam[..., 2], f * E, rtol=1e-12)
    assert np.allclose(lam[..., 0], 0.5 * (1 - f) * E, rtol=1e-10)
    assert np.allclose(lam[..., 1], 0.5 * (1 - f) * E, rtol=1e-10)
    assert np.allclose(np.trace(T, axis1=-2, axis2=-1), E, rtol=1e-12)
    g = np.stack(O.gradient4(E, h), axis=-1)
    gn = g / np.linalg.norm(g, axis=-1, keepdims=True)
    aligned = np.abs(np.sum(gn * vec[..., :, 2], axis=-1))
    strong = (f - 1 / 3) > 1e-6                        # a distinct top eigenvalue
    assert np.all(aligned[strong] > 1 - 1e-8)


def test_pressure_tensor_in_plane_trace_2d():
    """In 2D the out-of-plane eigenvalue (1-f)/2 E is not stored: Pxx + Pyy = (1+f)/2 E."""
    E, kr, h = _field((30, 26), 41)
    m = O.radiation_moments(E, kr, h)
    P = m["P"]
    assert np.allclose(P[0] + P[2], 0.5 * (1 + m["f"]) * E, rtol=1e-12)


@pytest.mark.parametrize("nd", [2, 3])
def test_tiring_exact_for_quadratic_velocity(nd):
    """The 4th-order gradient is exact for polynomials of degree <= 4: away from the
    walls P : grad v equals sum_ij P_ij dv_i/dx_j of the analytic velocity."""
    shape = (14, 16) if nd == 2 else (12, 14, 10)
    E, kr, h = _field(shape, 51 + nd, (-2, 1))
    rng = np.random.default_rng(5)
    A = rng.normal(size=(nd, nd))                       # non-symmetric linear part
    B = rng.normal(size=(nd, nd))                       # quadratic part: v_i += B_ij x_j^2
    coords = np.meshgrid(*[(np.arange(s) + 0.5) for s in shape], indexing="ij")
    xs = [coords[nd - 1 - d] * h[d] for d in range(nd)]  # x first
    v = [sum(A[i, j] * xs[j] + B[i, j] * xs[j] ** 2 for j in range(nd)) for i in range(nd)]
    m = O.radiation_moments(E, kr, h, v=v, dt=0.0)
    T = _full_tensor(m["P"], nd)
    exact = sum(T[..., i, j] * (A[i, j] + 2 * B[i, j] * xs[j]) for i in range(nd) for j in range(nd))
    core = tuple(slice(2, s - 2) for s in shape)
    assert np.allclose(m["tiring"][core], exact[core], rtol=1e-9, atol=1e-9 * np.abs(exact).max())


def test_tiring_removes_energy_under_expansion():
    """A uniformly expanding flow does work against the radiation: E decreases."""
    shape = (16, 20)
    E, kr, h = _field(shape, 61)
    coords = np.meshgrid(*[(np.arange(s) + 0.5) for s in shape], indexing="ij")
    v = [coords[1] * h[0] * 0.3, coords[0] * h[1] * 0.3]
    m = O.radiation_moments(E, kr, h, v=v, dt=1e-2)
    core = (slice(2, -2), slice(2, -2))
    assert np.all(m["tiring"][core] > 0) and np.all(m["E_new"][core] < E[core])
    # trace identity: dv_i/dx_j = 0.3 delta_ij, so P : grad v = 0.3 (Pxx + Pyy)
    assert np.allclose(m["tiring"][core], 0.3 * (m["P"][0] + m["P"][2])[core], rtol=1e-10)


def test_rotation_swaps_components_2d():
    E, kr, h = _field((24, 24), 71)
    a = O.radiation_moments(E, kr, (1 / 24, 1 / 24))
    b = O.radiation_moments(E.T.copy(), kr.T.copy(), (1 / 24, 1 / 24))
    assert np.allclose(b["F"][0], a["F"][1].T, rtol=1e-13, atol=0)
    assert np.allclose(b["F"][1], a["F"][0].T, rtol=1e-13, atol=0)
    assert np.allclose(b["P"][0], a["P"][2].T, rtol=1e-13) and np.allclose(b["P"][2], a["P"][0].T, rtol=1e-13)
    assert np.allclose(b["P"][1], a["P"][1].T, rtol=1e-12, atol=1e-300)
