"""Plant plausible mistakes in the radiation-moment oracle (on the CPU) and check
that one of its pins fails for each."""
import numpy as np
import pytest

import oracle
import oracle.moments as M
import oracle.fld as FLD
import tests.test_oracle_limiters as PL
import tests.test_oracle_moments as P

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _patch(monkeypatch, name, fn):
    monkeypatch.setattr(M, name, fn)
    monkeypatch.setattr(oracle, name, fn)


def _factor_wrong_power(lam, R):
    return lam + lam * R * R


def _tensor_wrong_iso(E, f, g):
    nd = len(g)
    gnorm = np.sqrt(sum(gi * gi for gi in g))
    n = [np.where(gnorm > 0, gi / np.where(gnorm > 0, gnorm, 1), 0) for gi in g]
    res = []
    for i, j in M.tensor_components(nd):
        t = 0.5 * (3 * f - 1) * n[i] * n[j]
        if i == j:
            t = t + 0.5 * (1 + f)
        res.append(E * t)
    return res


def _tiring_diagonal_only(Pt, v, h):
    nd = len(v)
    comp = {ij: k for k, ij in enumerate(M.tensor_components(nd))}
    out = np.zeros_like(v[0])
    for i in range(nd):
        out = out + Pt[comp[(i, i)]] * oracle.gradient4(v[i], h)[i]
    return out


_orig_limiter = FLD.flux_limiter


def _minerbo_branches_swapped(R, kind="lp"):
    if kind != "minerbo":
        return _orig_limiter(R, kind)
    R = np.asarray(R, dtype=np.float64)
    lo = 2.0 / (3.0 + np.sqrt(9.0 + 12.0 * R * R))
    hi = 1.0 / (1.0 + R + np.sqrt(1.0 + 2.0 * R))
    return np.where(R <= 1.5, hi, lo)


def _exact_lp_missing_over_r(R, kind="lp"):
    if kind != "lp_exact":
        return _orig_limiter(R, kind)
    return _orig_limiter(R, kind) * np.where(np.asarray(R) > 0, np.asarray(R), 1.0)


_orig_moments = M.radiation_moments


def _moments_flux_sign(*a, **k):
    m = _orig_moments(*a, **k)
    m["F"] = [-Fi for Fi in m["F"]]
    return m


def _moments_no_c(E, kr, h, c=1.0, **k):
    m = _orig_moments(E, kr, h, c=c, **k)
    m["F"] = [Fi / c for Fi in m["F"]]
    return m


def _moments_force_no_c(E, kr, h, c=1.0, **k):
    m = _orig_moments(E, kr, h, c=c, **k)
    m["f_r"] = [kr * Fi for Fi in m["F"]]
    return m


CASES = [
    ("eddington_factor", _factor_wrong_power,
     lambda: P.test_flux_is_causal_and_down_the_gradient((40, 48), (-2, 2))),
    ("pressure_tensor", _tensor_wrong_iso, P.test_pressure_tensor_in_plane_trace_2d),
    ("photon_tiring", _tiring_diagonal_only, lambda: P.test_tiring_exact_for_quadratic_velocity(2)),
    ("radiation_moments", _moments_flux_sign,
     lambda: P.test_flux_is_causal_and_down_the_gradient((40, 48), (-2, 2))),
    ("radiation_moments", _moments_no_c, P.test_free_streaming_limit),
    ("radiation_moments", _moments_force_no_c, P.test_thick_limit_is_fickian_diffusion),
]


LIMITER_CASES = [
    (_minerbo_branches_swapped, lambda: PL.test_limits_and_causality("minerbo")),
    (_exact_lp_missing_over_r, lambda: PL.test_exact_lp_against_high_precision(2.0)),
]


@pytest.mark.parametrize("fn,pin", LIMITER_CASES, ids=[c[0].__name__ for c in LIMITER_CASES])
def test_limiter_pin_catches_mutation(monkeypatch, fn, pin):
    monkeypatch.setattr(FLD, "flux_limiter", fn)
    monkeypatch.setattr(oracle, "flux_limiter", fn)
    with pytest.raises(AssertionError):
        pin()


@pytest.mark.parametrize("name,fn,pin", CASES, ids=[f"{c[0]}:{c[1].__name__}" for c in CASES])
def test_pin_catches_mutation(monkeypatch, name, fn, pin):
    _patch(monkeypatch, name, fn)
    with pytest.raises(AssertionError):
        pin()


def test_pins_pass_unmutated():
    P.test_flux_is_causal_and_down_the_gradient((40, 48), (-2, 2))
    P.test_pressure_tensor_in_plane_trace_2d()
    P.test_tiring_exact_for_quadratic_velocity(2)
    P.test_free_streaming_limit()
    P.test_thick_limit_is_fickian_diffusion()
