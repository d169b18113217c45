"""Plant plausible mistakes in the oracle (on the CPU) and check that a pin catches each.

Every mutation replaces one oracle function by a wrong variant (a dropped term, a
wrong sign, a swapped axis, a transposed operand) and runs the pin that should
fail.  This shows the pins constrain every step the oracle takes.
"""
import numpy as np
import pytest

import oracle
import oracle.fld as F
import tests.test_oracle_pins as P


def _patch(monkeypatch, name, fn):
    monkeypatch.setattr(F, name, fn)
    monkeypatch.setattr(oracle, name, fn)


def _lim_sign(R, kind="lp"):
    return (2.0 - R) / (6.0 + 3.0 * R + R * R) if kind == "lp" else np.full_like(R, 1 / 3)


def _lim_dropped(R, kind="lp"):
    return 2.0 / (6.0 + 3.0 * R + R * R) if kind == "lp" else np.full_like(R, 1 / 3)


def _grad2(E, h):
    nd = E.ndim
    Pd = np.pad(E, 1, mode="symmetric")
    out = []
    for d in range(nd):
        a = nd - 1 - d
        sl_p = [slice(1, 1 + s) for s in E.shape]
        sl_m = [slice(1, 1 + s) for s in E.shape]
        sl_p[a] = slice(2, 2 + E.shape[a])
        sl_m[a] = slice(0, E.shape[a])
        out.append((Pd[tuple(sl_p)] - Pd[tuple(sl_m)]) / (2 * h[d]))
    return out


_orig_faces = F.face_weights


def _faces_arith(D, dt, h):
    nd = D.ndim
    out = []
    for d in range(nd):
        a = nd - 1 - d
        w = np.zeros_like(D)
        lo = [slice(None)] * nd
        hi = [slice(None)] * nd
        lo[a] = slice(0, D.shape[a] - 1)
        hi[a] = slice(1, D.shape[a])
        w[tuple(hi)] = dt * 0.5 * (D[tuple(lo)] + D[tuple(hi)]) / h[d] ** 2
        out.append(w)
    return out


def _faces_no_dt(D, dt, h):
    return _orig_faces(D, 1.0, h)


def _faces_swapped_h(D, dt, h):
    return _orig_faces(D, dt, tuple(reversed(h)))


def _faces_h_not_squared(D, dt, h):
    return [w * hd for w, hd in zip(_orig_faces(D, dt, h), h)]


_orig_grad = F.gradient4


def _grad_swapped_h(E, h):
    return _orig_grad(E, tuple(reversed(h)))


def _dcoef_transposed(E, kappa_rho, h, c=1.0, limiter="lp"):
    R = F.radiation_parameter(E, kappa_rho, h)
    return c * F.flux_limiter(R, limiter) * kappa_rho


def _coef_no_dt(rho, kappa, dt, c, a_r, c_v):
    return c * a_r * kappa / (rho ** 3 * c_v ** 4), c * kappa * rho * dt


def _coef_rho_power(rho, kappa, dt, c, a_r, c_v):
    return c * a_r * kappa * dt / (rho ** 4 * c_v ** 4), c * kappa * rho * dt


def _pad_edge(E, width=2):
    return np.pad(E, width, mode="edge")


MUTATIONS = [
    ("flux_limiter", _lim_sign, lambda gd: P.test_limiter_limits_and_monotonicity()),
    ("flux_limiter", _lim_dropped, lambda gd: P.test_limiter_limits_and_monotonicity()),
    ("gradient4", _grad2, lambda gd: P.test_gradient_exact_for_quartics(2)),
    ("gradient4", _grad_swapped_h, lambda gd: P.test_gradient_exact_for_quartics(2)),
    ("face_weights", _faces_arith, lambda gd: P.test_harmonic_face_is_series_conductance()),
    ("face_weights", _faces_no_dt, lambda gd: P.test_dct_closed_form_constant_coefficients(
        (12, 7), (0.03, 0.05))),
    ("face_weights", _faces_swapped_h, lambda gd: P.test_dct_closed_form_constant_coefficients(
        (12, 7), (0.03, 0.05))),
    ("face_weights", _faces_h_not_squared, lambda gd: P.test_thick_pulse_variance_grows_exactly()),
    ("diffusion_coefficient", _dcoef_transposed, lambda gd: P.test_constant_energy_gives_thick_limit()),
    ("exchange_coefficients", _coef_no_dt, lambda gd: P.test_exchange_conserves_and_satisfies_implicit_pair()),
    ("exchange_coefficients", _coef_rho_power, lambda gd: P.test_exchange_root_closed_form_and_roots()),
    ("pad_mirror", _pad_edge, lambda gd: P.test_mirror_ghosts_are_even_reflection()),
]


@pytest.mark.parametrize("name,fn,pin", MUTATIONS, ids=[f"{m[0]}:{m[1].__name__}" for m in MUTATIONS])
def test_pin_catches_planted_mistake(monkeypatch, golden_dir, name, fn, pin):
    _patch(monkeypatch, name, fn)
    with pytest.raises(AssertionError):
        pin(golden_dir)


def test_unmutated_pins_pass(golden_dir):
    """Control: the same pins pass on the unmodified oracle."""
    for _, _, pin in MUTATIONS:
        pin(golden_dir)
