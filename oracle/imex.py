"""Plain FP64 oracle of the radiation-only IMEX time step (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
leg may use this module.  It shares no code with the HIP path.

The paper splits the update into an explicit operator G_ex (explicit sources,
then the local implicit heating/cooling, then advection) and the implicit
diffusion G_im (Sec. 3.1, eqs. G_expl_1 - G_expl_3 and G_expl - G_implexpl).
For the radiation subsystem alone (no advection; kappa, rho fixed) the state is
(E, eps) and, per grid:

* G_ex over a time tau: the photon-tiring source E <- E - tau P:grad v (when a
  velocity is given; eq. G_expl_1), then the point-implicit exchange over tau
  (Sec. 3.3; eq. G_expl_2);
* G_im over a time tau: one backward-Euler diffusion solve with D lagged at its
  input (Sec. 3.4).

``euler``: u* = G_ex(u^n, dt), then u^{n+1} = G_im(u*, dt).
``midpoint`` (eqs. G_expl - G_implexpl): u_+ = G_ex(u^n, dt/2);
u^{n+1/2} = G_im(u_+, dt/2), whose tendency G_im = (E^{n+1/2} - E_+)/(dt/2) is
reused; the full step starts from u^n, adds dt G_im and the explicit tiring
source at the midpoint state E^{n+1/2}, and applies the exchange over dt (the
G_ex sub-scheme for a full step, as the paper states for the last operation).
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

from . import fld as _fld
from . import moments as _mom

__all__ = ["imex_step"]


def _tiring(E, kr, h, c, limiter, v):
    return _mom.radiation_moments(E, kr, h, c=c, limiter=limiter, v=v)["tiring"]


def imex_step(E: np.ndarray, eps: np.ndarray, rho: np.ndarray, kappa: np.ndarray, dt: float,
              h: Sequence[float], c: float = 1.0, a_r: float = 1.0, c_v: float = 1.0,
              limiter: str = "lp", scheme: str = "midpoint",
              v: Optional[Sequence[np.ndarray]] = None, exchange: bool = True):
    """One radiation-only IMEX step; returns (E^{n+1}, eps^{n+1}).

    exchange=False leaves the gas out (G_ex is the tiring source alone): with a
    linear diffusion operator the midpoint scheme is then second order.  The
    exchange stage is a backward-Euler step over the stage's time in both schemes
    (eq. G_expl_2), so with it, and with D lagged at the stage input, the step is
    first order in dt.
    """
    E = np.asarray(E, dtype=np.float64)
    eps = np.asarray(eps, dtype=np.float64)
    kr = kappa * rho                                   # one opacity serves D and the exchange

    def explicit(Ein, epsin, tau, E_tir=None):
        Ex = Ein if v is None else Ein - tau * _tiring(E_tir if E_tir is not None else Ein, kr, h, c, limiter, v)
        if not exchange:
            return Ex, epsin
        return _fld.exchange(Ex, epsin, rho, kappa, tau, c, a_r, c_v)

    def implicit(Ein, tau):
        x, _ = _fld.diffusion_step(Ein, kr, tau, h, c, limiter)
        return x

    if scheme == "euler":
        Es, epss = explicit(E, eps, dt)
        return implicit(Es, dt), epss
    if scheme == "midpoint":
        Ep, epsp = explicit(E, eps, 0.5 * dt)
        Em = implicit(Ep, 0.5 * dt)
        G_im = (Em - Ep) / (0.5 * dt)
        base = E + dt * G_im
        return explicit(base, eps, dt, E_tir=Em)
    raise ValueError(f"unknown scheme {scheme!r}")
