"""Pins of the coarse-operator oracle (Sec. 3.4 multigrid): the Galerkin product
R A P against its entry-by-entry definition, the energy identity it implies,
unit row sums and symmetry, and closed forms for constant and linearly varying
face weights (which also pin the rediscretised coarse operator)."""
import itertools

import numpy as np
import pytest

import oracle as O
import workloads as W


def _random_weights(shape, seed):
    rng = np.random.default_rng(seed)
    nd = len(shape)
    w = []
    for d in range(nd):
        a = nd - 1 - d
        wd = rng.uniform(0.1, 5.0, size=shape) * (10.0 ** d)     # axes at different scales
        lo = [slice(None)] * nd
        lo[a] = 0
        wd[tuple(lo)] = 0.0
        w.append(wd)
    return w


@pytest.mark.parametrize("shape", [(4, 6), (6, 4), (4, 4, 6)])
def test_galerkin_equals_its_entrywise_definition(shape):
    """(A_c)_{IJ} = 2^-d sum over children i of I and j of J of A_ij, by plain loops."""
    w = _random_weights(shape, 71 + len(shape))
    A = O.assemble_operator(w).toarray()
    nd = len(shape)
    cs = tuple(n // 2 for n in shape)
    Nc = int(np.prod(cs))
    fine_cells = list(np.ndindex(*shape))
    parent = [np.ravel_multi_index(tuple(c // 2 for c in cell), cs) for cell in fine_cells]
    Ac = np.zeros((Nc, Nc))
    for i, I in enumerate(parent):
        for j, J in enumerate(parent):
            Ac[I, J] += A[i, j]
    Ac /= 2 ** nd
    G = O.galerkin_operator(O.assemble_operator(w), shape).toarray()
    assert np.allclose(G, Ac, rtol=0, atol=1e-13 * np.abs(Ac).max())
    # the coarse matrix has the operator's form: rebuilding it from its face weights
    wc = O.coarse_weights_galerkin(w)
    assert np.allclose(O.assemble_operator(wc).toarray(), Ac, rtol=0, atol=1e-13 * np.abs(Ac).max())


@pytest.mark.parametrize("shape", [(8, 12), (6, 8, 4)])
def test_galerkin_energy_identity_rows_and_symmetry(shape):
    """v^T A_c v = (P v)^T A (P v) / 2^d, through the matrix-free fine operator;
    A_c is symmetric with unit row sums (zero flux conserves the mean)."""
    w = _random_weights(shape, 5 + len(shape))
    cs = tuple(n // 2 for n in shape)
    Ac = O.galerkin_operator(O.assemble_operator(w), shape)
    rng = np.random.default_rng(9)
    for _ in range(3):
        v = rng.standard_normal(cs)
        Pv = v
        for a in range(len(shape)):
            Pv = np.repeat(Pv, 2, axis=a)
        lhs = v.ravel() @ (Ac @ v.ravel())
        rhs = Pv.ravel() @ O.apply_operator(w, Pv).ravel() / 2 ** len(shape)
        assert abs(lhs - rhs) <= 1e-12 * abs(rhs)
    assert abs(Ac - Ac.T).max() == 0.0
    assert np.allclose(Ac @ np.ones(Ac.shape[0]), 1.0, rtol=0, atol=1e-13)


@pytest.mark.parametrize("shape", [(16, 8), (8, 4, 6)])
def test_constant_coefficients_closed_forms(shape):
    """Constant D: fine weights dt D / h^2; the rediscretised coarse operator is the
    same formula at spacing 2h (a quarter), the Galerkin one is twice that."""
    nd = len(shape)
    h = [0.1, 0.07, 0.2][:nd]
    D = np.full(shape, 0.37)
    dt = 3e-3
    w = O.face_weights(D, dt, h)
    cs = tuple(n // 2 for n in shape)
    w2h = O.face_weights(np.full(cs, 0.37), dt, [2 * x for x in h])
    red = O.coarse_weights_rediscretised(w)
    gal = O.coarse_weights_galerkin(w)
    for d in range(nd):
        assert np.allclose(red[d], w2h[d], rtol=1e-15, atol=0)
        assert np.allclose(gal[d], 2.0 * w2h[d], rtol=1e-15, atol=0)


def test_linearly_varying_weights():
    """Face weights linear across the face direction: the mean of the sub-faces is the
    value at the coarse face's centre (rediscretised, /4), the Galerkin sum twice it."""
    ny, nx = 12, 10
    yc = np.arange(ny) + 0.5
    wx = np.tile((2.0 + 0.25 * yc)[:, None], (1, nx))
    wx[:, 0] = 0.0
    wy = np.zeros((ny, nx))
    w = [wx, wy]
    red = O.coarse_weights_rediscretised(w)
    gal = O.coarse_weights_galerkin(w)
    Yc = 2.0 * (np.arange(ny // 2) + 0.5)                    # coarse centres in fine units
    want = np.tile((2.0 + 0.25 * Yc)[:, None] / 4.0, (1, nx // 2))
    want[:, 0] = 0.0
    assert np.allclose(red[0], want, rtol=1e-15, atol=0)
    assert np.allclose(gal[0], 2.0 * want, rtol=1e-15, atol=0)
    assert np.abs(red[1]).max() == 0.0 and np.abs(gal[1]).max() == 0.0


def test_coarse_weights_of_a_seeded_field_are_positive_and_bounded():
    g = W.random_grid((24, 20), 88001, dt=2e-3)
    D = O.diffusion_coefficient(g.E, g.kappa_rho, g.h)
    w = O.face_weights(D, g.dt, g.h)
    for rule in (O.coarse_weights_rediscretised, O.coarse_weights_galerkin):
        wc = rule(w)
        for d, a in enumerate((1, 0)):
            inner = np.take(wc[d], np.arange(1, wc[d].shape[a]), axis=a)
            assert (inner > 0).all()
            assert inner.max() <= w[d].max()


def test_odd_axes_are_rejected():
    with pytest.raises(ValueError):
        O.prolongation_constant((5, 4))
    with pytest.raises(ValueError):
        O.coarse_weights_galerkin([np.ones((4, 3)), np.ones((4, 3))])


@pytest.mark.parametrize("shape", [(4, 4), (4, 4, 4)])
def test_planted_axis_swap_is_caught(shape):
    """A plausible mistake (x and y weights exchanged) breaks the entrywise check."""
    w = _random_weights(shape, 300)
    wc = O.coarse_weights_galerkin(w)
    swapped = [wc[1], wc[0]] + list(wc[2:])
    Ac = O.galerkin_operator(O.assemble_operator(w), shape).toarray()
    assert not np.allclose(O.assemble_operator(swapped).toarray(), Ac, rtol=0,
                           atol=1e-9 * np.abs(Ac).max())
    assert list(itertools.chain(*[x.shape for x in wc]))  # shapes are the coarse grid's


def test_weights_varying_along_their_own_axis():
    """A coarse face sits on the fine faces of its lower children (fine index 2I), not on
    the faces inside a coarse cell: weights linear in the face index pin which ones."""
    ny, nx = 6, 12
    i = np.arange(nx)
    wx = np.tile((2.0 + 0.3 * i)[None, :], (ny, 1))
    wx[:, 0] = 0.0
    w = [wx, np.zeros((ny, nx))]
    I = np.arange(nx // 2)
    want = np.tile(((2.0 + 0.3 * 2 * I) / 4.0)[None, :], (ny // 2, 1))
    want[:, 0] = 0.0
    assert np.allclose(O.coarse_weights_rediscretised(w)[0], want, rtol=1e-15, atol=0)
    assert np.allclose(O.coarse_weights_galerkin(w)[0], 2.0 * want, rtol=1e-15, atol=0)
