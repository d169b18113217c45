"""Plain FP64 oracle of the FLD step with fixed-gradient (Neumann) boundaries
(TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
leg may use this module.  It shares no code with the HIP path.

Sec. 3.4 lets a boundary fix the gradient of E^{n+1} at the interface between
the ghost cells and the domain (Neumann conditions; zero flux is the case of a
zero gradient).  Readings, per boundary face with prescribed gradient G (the
derivative along +x_d):

* ghost cells continue the mirror image with the linear part that has slope G
  at the face: E_{-k} = E_{k-1} - (2k - 1) h G below, E_{n-1+k} = E_{n-k} +
  (2k - 1) h G above (k = 1, 2), which is exact for linear profiles; the 4th-order
  gradient of Sec. 3.2 (and so R, lambda and D) uses them;
* the flux through the face is F = -D G with D the boundary cell's own (lagged)
  value (the ghost has no D of its own); it enters the right-hand side,
  b = E^n + (dt / h) (-D G) below and b = E^n + (dt / h) (D G) above, and the
  operator keeps zero weight on the domain faces.

``grad_bc`` lists the six faces x-, x+, y-, y+, z-, z+ (None or 0 = zero flux).
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np

from . import fld as _fld

__all__ = ["pad_fixed_gradient", "gradient4_bc", "boundary_source", "diffusion_step_bc"]


def _face_values(grad_bc, nd):
    g = [0.0] * 6
    for f, v in enumerate(grad_bc or []):
        if f < 2 * nd and v is not None:
            g[f] = float(v)
    return g


def pad_fixed_gradient(E: np.ndarray, axis_d: int, h: float, g_lo: float, g_hi: float) -> np.ndarray:
    """E with two ghost layers along dimension d (x = 0) following the rule above."""
    nd = E.ndim
    a = _fld._axis(nd, axis_d)
    E = np.moveaxis(E, a, 0)
    lo = [E[1] - 3.0 * h * g_lo, E[0] - 1.0 * h * g_lo]
    hi = [E[-1] + 1.0 * h * g_hi, E[-2] + 3.0 * h * g_hi]
    P = np.concatenate([np.stack(lo), E, np.stack(hi)], axis=0)
    return np.moveaxis(P, 0, a)


def gradient4_bc(E: np.ndarray, h: Sequence[float], grad_bc=None) -> List[np.ndarray]:
    """The 4th-order central gradient (Sec. 3.2) with the ghost rule above."""
    nd = E.ndim
    g = _face_values(grad_bc, nd)
    out = []
    for d in range(nd):
        a = _fld._axis(nd, d)
        P = pad_fixed_gradient(E, d, h[d], g[2 * d], g[2 * d + 1])
        n = E.shape[a]

        def sh(k):
            sl = [slice(None)] * nd
            sl[a] = slice(2 + k, 2 + k + n)
            return P[tuple(sl)]
        out.append((sh(-2) / 12.0 - 2.0 * sh(-1) / 3.0 + 2.0 * sh(1) / 3.0 - sh(2) / 12.0) / h[d])
    return out


def boundary_source(D: np.ndarray, dt: float, h: Sequence[float], grad_bc=None) -> np.ndarray:
    """dt times the boundary fluxes entering each boundary cell, divided by its width."""
    nd = D.ndim
    g = _face_values(grad_bc, nd)
    s = np.zeros_like(D)
    for d in range(nd):
        a = _fld._axis(nd, d)
        lo = [slice(None)] * nd
        hi = [slice(None)] * nd
        lo[a] = 0
        hi[a] = D.shape[a] - 1
        s[tuple(lo)] += dt / h[d] * (-D[tuple(lo)] * g[2 * d])
        s[tuple(hi)] += dt / h[d] * (D[tuple(hi)] * g[2 * d + 1])
    return s


def diffusion_step_bc(E: np.ndarray, kappa_rho: np.ndarray, dt: float, h: Sequence[float],
                      grad_bc: Optional[Sequence] = None, c: float = 1.0, limiter: str = "lp",
                      method: str = "auto", tol=None):
    """One backward-Euler FLD step (Sec. 3.4) with the fixed-gradient faces of grad_bc."""
    E = np.asarray(E, dtype=np.float64)
    kr = np.asarray(kappa_rho, dtype=np.float64)
    gr = gradient4_bc(E, h, grad_bc)
    R = np.sqrt(sum(x * x for x in gr)) / (kr * E)
    D = c * _fld.flux_limiter(R, limiter) / kr
    w = _fld.face_weights(D, dt, h)
    A = _fld.assemble_operator(w)
    b = E + boundary_source(D, dt, h, grad_bc)
    x, info = _fld.solve(A, b, method=method, tol=tol, w=w)
    info.extra["b"] = b
    return x, info
