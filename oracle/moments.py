"""Plain FP64 oracle of the radiation moments derived from E (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
leg may use this module.  It shares no code with the HIP path.

Given E, kappa rho and the cell widths, per cell (Moens et al., "Radiation-
hydrodynamics with MPI-AMRVAC: flux-limited diffusion"):

1. the 4th-order gradient of E with mirrored ghosts (Sec. 3.2, eq. ileyk_flux),
   R and the flux limiter lambda(R) (Sec. 2.2), exactly as for the diffusion
   coefficient;
2. the co-moving flux ``F = -c lambda / (kappa rho) grad E`` (Sec. 2.2, eq. fld_F);
3. the radiation force density ``f_r = rho kappa F / c`` (Sec. 2.1,
   eq. rhd_force; one opacity serves every mean, as for D);
4. the scalar Eddington factor ``f = lambda + lambda^2 R^2`` (Sec. 2.2,
   eq. fld_Edd_fac);
5. the pressure tensor ``P = E (1/2 (1 - f) I + 1/2 (3 f - 1) n n)`` with
   ``n = grad E / |grad E|`` (Sec. 2.2, eq. fld_Edd; n is taken as 0 where the
   gradient vanishes, where f = 1/3 and the n n term has weight 0);
6. given a velocity field, the photon-tiring work ``P : grad v =
   sum_ij P_ij d v_i / d x_j`` with the same 4th-order gradient and mirrored
   ghosts for v (Sec. 3.2, "Radiation force and photon tiring"), and the
   explicit update ``E' = E - dt P : grad v``: the sign of the energy equation
   (Sec. 2.1, eq. 0th_cmf, where the term sits on the left-hand side).

Arrays are C-ordered ``(ny, nx)`` / ``(nz, ny, nx)``; vectors are lists with the
x component first; the symmetric tensor is returned as its upper triangle in
row-major order: (xx, xy, yy) in 2D, (xx, xy, xz, yy, yz, zz) in 3D.
"""
from __future__ import annotations

from typing import Dict, List, Optional, Sequence

import numpy as np

from . import fld as _fld

__all__ = ["tensor_components", "eddington_factor", "pressure_tensor", "photon_tiring", "radiation_moments"]


def tensor_components(ndim: int) -> List[tuple]:
    """Index pairs (i, j), i <= j, of the stored upper triangle, row-major."""
    return [(i, j) for i in range(ndim) for j in range(i, ndim)]


def eddington_factor(lam: np.ndarray, R: np.ndarray) -> np.ndarray:
    """``f = lambda + lambda^2 R^2`` (Sec. 2.2, eq. fld_Edd_fac)."""
    return lam + lam * lam * R * R


def pressure_tensor(E: np.ndarray, f: np.ndarray, g: Sequence[np.ndarray]) -> List[np.ndarray]:
    """Upper triangle of ``P = E (1/2 (1-f) I + 1/2 (3f-1) n n)``, n = g/|g| (eq. fld_Edd)."""
    nd = len(g)
    gnorm = np.sqrt(sum(gi * gi for gi in g))
    safe = np.where(gnorm > 0.0, gnorm, 1.0)
    n = [np.where(gnorm > 0.0, gi / safe, 0.0) for gi in g]
    iso = 0.5 * (1.0 - f)
    aniso = 0.5 * (3.0 * f - 1.0)
    out = []
    for i, j in tensor_components(nd):
        t = aniso * n[i] * n[j]
        if i == j:
            t = t + iso
        out.append(E * t)
    return out


def photon_tiring(P: Sequence[np.ndarray], v: Sequence[np.ndarray], h: Sequence[float]) -> np.ndarray:
    """``P : grad v = sum_ij P_ij dv_i/dx_j`` with 4th-order gradients of each component."""
    nd = len(v)
    dv = [_fld.gradient4(v[i], h) for i in range(nd)]    # dv[i][j] = d v_i / d x_j
    comp = {ij: k for k, ij in enumerate(tensor_components(nd))}
    out = np.zeros_like(v[0])
    for i in range(nd):
        for j in range(nd):
            out = out + P[comp[(min(i, j), max(i, j))]] * dv[i][j]
    return out


def radiation_moments(E: np.ndarray, kappa_rho: np.ndarray, h: Sequence[float], c: float = 1.0,
                      limiter: str = "lp", v: Optional[Sequence[np.ndarray]] = None,
                      dt: float = 0.0) -> Dict[str, object]:
    """Flux, force, Eddington factor, pressure tensor (and tiring, updated E) per cell.

    Returns a dict with ``F`` and ``f_r`` (lists, x first), ``f``, ``P`` (upper
    triangle), ``lam`` and ``R``; with ``v`` also ``tiring`` and ``E_new``.
    """
    E = np.asarray(E, dtype=np.float64)
    kappa_rho = np.asarray(kappa_rho, dtype=np.float64)
    g = _fld.gradient4(E, h)                                    # eq. ileyk_flux
    gnorm = np.sqrt(sum(gi * gi for gi in g))
    R = gnorm / (kappa_rho * E)                                 # Sec. 2.2
    lam = _fld.flux_limiter(R, limiter)                         # eq. fld_lambda
    F = [-c * lam / kappa_rho * gi for gi in g]                 # eq. fld_F
    f_r = [kappa_rho * Fi / c for Fi in F]                      # eq. rhd_force
    f = eddington_factor(lam, R)                                # eq. fld_Edd_fac
    P = pressure_tensor(E, f, g)                                # eq. fld_Edd
    out: Dict[str, object] = {"F": F, "f_r": f_r, "f": f, "P": P, "lam": lam, "R": R}
    if v is not None:
        vv = [np.asarray(vi, dtype=np.float64) for vi in v]
        tiring = photon_tiring(P, vv, h)
        out["tiring"] = tiring
        out["E_new"] = E - dt * tiring                          # eq. 0th_cmf
    return out
