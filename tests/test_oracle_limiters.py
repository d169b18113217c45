"""Pins of the flux-limiter variants (Sec. 2.2): the rational Levermore-Pomraning
law of eq. fld_lambda, Levermore and Pomraning's exact (coth R - 1/R)/R form and
Minerbo's two-branch limiter, which the paper names as the user's alternative.
Each is pinned to its thick and free-streaming limits, causality, closed-form
values, and (for the exact form) a 50-digit reference."""
from decimal import Decimal, getcontext

import numpy as np
import pytest

import oracle as O

PHYSICAL = ("lp", "minerbo", "lp_exact")


def _coth_ref(r: float) -> float:
    """(coth r - 1/r)/r at 50 significant digits (decimal exp)."""
    getcontext().prec = 60
    x = Decimal(r)
    e2 = (2 * x).exp()
    coth = (e2 + 1) / (e2 - 1)
    return float((coth - 1 / x) / x)


@pytest.mark.parametrize("kind", PHYSICAL)
def test_limits_and_causality(kind):
    R = np.concatenate([[0.0], np.logspace(-8, 8, 4001)])
    lam = O.flux_limiter(R, kind)
    assert lam[0] == pytest.approx(1 / 3, rel=1e-15)           # optically thick
    assert np.all(lam <= 1 / 3 + 1e-15)
    assert np.all(np.diff(lam) <= 4e-16 * lam[1:])              # decreasing in R (to rounding)
    assert np.all(lam * R < 1.0)                                # |F| = c lambda R E < c E
    assert lam[-1] * R[-1] > 0.9998                             # free streaming: lambda -> 1/R


def test_minerbo_branches_meet_smoothly():
    lo = lambda r: 2.0 / (3.0 + np.sqrt(9.0 + 12.0 * r * r))
    hi = lambda r: 1.0 / (1.0 + r + np.sqrt(1.0 + 2.0 * r))
    assert lo(1.5) == pytest.approx(2 / 9, rel=1e-15) and hi(1.5) == pytest.approx(2 / 9, rel=1e-15)
    h = 1e-6
    assert (lo(1.5) - lo(1.5 - h)) / h == pytest.approx(-2 / 27, rel=1e-5)
    assert (hi(1.5 + h) - hi(1.5)) / h == pytest.approx(-2 / 27, rel=1e-5)
    R = np.array([0.0, 0.5, 1.5, 1.5 + 1e-9, 3.0, 40.0])
    lam = O.flux_limiter(R, "minerbo")
    assert np.allclose(lam[:3], lo(R[:3]), rtol=1e-15) and np.allclose(lam[3:], hi(R[3:]), rtol=1e-15)


@pytest.mark.parametrize("r", [1e-7, 1e-3, 0.05, 0.0999, 0.1, 0.1001, 0.5, 1.0, 2.0, 10.0, 100.0, 1e5])
def test_exact_lp_against_high_precision(r):
    assert O.flux_limiter(np.array([r]), "lp_exact")[0] == pytest.approx(_coth_ref(r), rel=2e-13)


def test_exact_lp_known_value_and_rational_approximation():
    # lambda(1) = coth(1) - 1
    assert O.flux_limiter(np.array([1.0]), "lp_exact")[0] == pytest.approx(0.3130352854993313, rel=1e-15)
    R = np.logspace(-4, 4, 2001)
    rel = np.abs(O.flux_limiter(R, "lp") / O.flux_limiter(R, "lp_exact") - 1)
    assert rel.max() < 0.075                                    # the rational law is a ~7 % fit
    assert rel[0] < 1e-8 and rel[-1] < 1e-3                     # exact at both ends


@pytest.mark.parametrize("kind", PHYSICAL)
def test_moments_causal_for_every_limiter(kind):
    import workloads as W
    g = W.random_grid((40, 36), 81, dt=1e-3)
    kr = 10.0 ** W.span(W.smooth_field((40, 36), 82), -8, 2)
    m = O.radiation_moments(g.E, kr, g.h, c=1.5, limiter=kind)
    Fmag = np.sqrt(sum(Fi * Fi for Fi in m["F"]))
    assert np.all(Fmag <= 1.5 * g.E * (1 + 1e-12))
    assert np.all(m["f"] >= 1 / 3 - 1e-15) and np.all(m["f"] <= 1 + 1e-12)
