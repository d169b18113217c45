"""Plain FP64 oracle of the FLD step with a diagonal-tensor diffusion coefficient
(TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
leg may use this module.  It shares no code with the HIP path.

The paper reports testing an anisotropic D, a diagonal tensor whose element d is
the diffusion coefficient along grid direction d, and leaves the notation of
Sec. 3 to be carried over (Sec. 5).  Reading: the caller supplies one kappa rho
per direction (line-of-sight opacities), and every quantity of Sec. 2.2 / 3.4 is
formed per direction with it,

    R_d = |grad E| / ((kappa rho)_d E),   D_d = c lambda(R_d) / (kappa rho)_d,

with the 4th-order gradient of Sec. 3.2, and the faces normal to d take the
harmonic mean of D_d of their two cells (eq. discdiff with D -> D_d).  Equal
opacities give back the isotropic step.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np

from . import fld as _fld

__all__ = ["diffusion_tensor", "face_weights_aniso", "diffusion_step_aniso"]


def diffusion_tensor(E: np.ndarray, kappa_rho_dirs: Sequence[np.ndarray], h: Sequence[float],
                     c: float = 1.0, limiter: str = "lp") -> List[np.ndarray]:
    """Diagonal elements D_d, x first (one array per dimension)."""
    E = np.asarray(E, dtype=np.float64)
    g = _fld.gradient4(E, h)
    gnorm = np.sqrt(sum(gi * gi for gi in g))
    out = []
    for d in range(E.ndim):
        kr = np.asarray(kappa_rho_dirs[d], dtype=np.float64)
        R = gnorm / (kr * E)
        out.append(c * _fld.flux_limiter(R, limiter) / kr)
    return out


def face_weights_aniso(Ds: Sequence[np.ndarray], dt: float, h: Sequence[float]) -> List[np.ndarray]:
    """Lower-face weights along d from the harmonic mean of D_d (zero at the domain faces)."""
    return [_fld.face_weights(Ds[d], dt, h)[d] for d in range(len(Ds))]


def diffusion_step_aniso(E: np.ndarray, kappa_rho_dirs: Sequence[np.ndarray], dt: float,
                         h: Sequence[float], c: float = 1.0, limiter: str = "lp",
                         method: str = "auto", tol=None):
    """One backward-Euler step ``(I + dt L(D^n)) E^{n+1} = E^n`` with the diagonal D."""
    E = np.asarray(E, dtype=np.float64)
    w = face_weights_aniso(diffusion_tensor(E, kappa_rho_dirs, h, c, limiter), dt, h)
    A = _fld.assemble_operator(w)
    x, info = _fld.solve(A, E, method=method, tol=tol, w=w)
    info.extra["q_b"] = _fld.q_b(E)
    return x, info
