"""Plain FP64 oracle of the FLD step with Dirichlet and periodic boundaries
(TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
leg may use this module.  It shares no code with the HIP path.

Sec. 3.4 lets a boundary define E^{n+1} in the ghost cells (Dirichlet conditions)
beside the Neumann (fixed-gradient) ones.  Readings, per face with ghost value E_B:

* both ghost layers hold E_B; the 4th-order gradient of Sec. 3.2 (and so R,
  lambda and D of the cells next to the face) uses them;
* the ghost couples to the boundary cell like an interior neighbour over the
  centre distance h, with the boundary cell's own lagged D (the ghost carries no
  opacity, so there is no harmonic mean to take): the cell's row of eq. discdiff
  (times dt) gains alpha = dt D / h^2 on the diagonal and alpha E_B on the
  right-hand side.  The operator stays symmetric positive definite with
  lambda_min >= 1; energy now leaves or enters through the face.

Periodic axes (both faces "periodic") wrap: the ghosts are the cells at the other
end, and the face between the last and the first cell is an interior face like any
other (harmonic mean of the two D, stored in the first cell's lower-face slot).

Continuous faces (Sec. 3.4 lists a linear extrapolation of E^{n+1} into the ghost
cells as the third kind of boundary).  Readings:

* the ghosts continue the line through the two cells next to the face:
  E_{-k} = E_0 + k (E_0 - E_1) below, E_{n-1+k} = E_{n-1} + k (E_{n-1} - E_{n-2})
  above (k = 1, 2); the 4th-order gradient of R uses them, which keeps it exact for
  linear profiles;
* in eq. discdiff the ghost of the implicit solve is the same extrapolation of the
  unknown E^{n+1}, coupled to the boundary cell through the boundary face.  The paper
  gives no opacity for the ghost, so the boundary face takes the flux coefficient of
  the first interior face (the coefficient, like E, is continued across the face): the
  boundary cell's row gains w_B (x_0 - x_ghost) = w_B (x_1 - x_0) with w_B the weight
  of the face between cells 0 and 1.  A stays an M-matrix (that row loses its coupling
  along the axis) but is no longer symmetric, and energy crosses the face.

Faces are listed x-, x+, y-, y+, z-, z+.  ``kind`` per face is "zero_flux",
"gradient" (the fixed-gradient faces of ``oracle.bc``), "dirichlet", "periodic" or
"continuous"; ``value`` per face is the prescribed gradient or ghost value.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np
import scipy.sparse as sp

from . import fld as _fld

__all__ = ["pad_general", "gradient4_general", "dirichlet_diagonal", "boundary_rhs",
           "face_weights_general", "assemble_general", "continuous_coupling", "diffusion_step_general"]

KINDS = ("zero_flux", "gradient", "dirichlet", "periodic", "continuous")


def _faces(kind, value, nd):
    k = ["zero_flux"] * 6
    v = [0.0] * 6
    for f in range(2 * nd):
        if kind is not None and kind[f] is not None:
            if kind[f] not in KINDS:
                raise ValueError(f"unknown boundary kind {kind[f]!r}")
            k[f] = kind[f]
        if value is not None and value[f] is not None:
            v[f] = float(value[f])
    for d in range(nd):
        if (k[2 * d] == "periodic") != (k[2 * d + 1] == "periodic"):
            raise ValueError("a periodic axis needs both of its faces periodic")
    return k, v


def pad_general(E: np.ndarray, d: int, h: float, kind_lo: str, val_lo: float, kind_hi: str,
                val_hi: float) -> np.ndarray:
    """E with two ghost layers along dimension d (x = 0): mirror image for zero flux, mirror
    plus the linear part of slope G for a fixed gradient, E_B in both layers for Dirichlet."""
    nd = E.ndim
    a = _fld._axis(nd, d)
    M = np.moveaxis(E, a, 0)

    def ghosts(edge0, edge1, kind, val, sign):
        if kind == "dirichlet":
            return [np.full_like(edge0, val), np.full_like(edge0, val)]
        if kind == "continuous":
            # the line through the boundary cell and its inner neighbour, one and two
            # cell widths beyond the face
            return [edge0 + (edge0 - edge1), edge0 + 2.0 * (edge0 - edge1)]
        g = val if kind == "gradient" else 0.0
        # [inner ghost, outer ghost]: E_{-1} = E_0 -/+ h G, E_{-2} = E_1 -/+ 3 h G
        return [edge0 + sign * h * g, edge1 + sign * 3.0 * h * g]

    if kind_lo == "periodic":
        lo, hi = [M[-1], M[-2]], [M[0], M[1]]
    else:
        lo = ghosts(M[0], M[1], kind_lo, val_lo, -1.0)
        hi = ghosts(M[-1], M[-2], kind_hi, val_hi, 1.0)
    P = np.concatenate([np.stack([lo[1], lo[0]]), M, np.stack([hi[0], hi[1]])], axis=0)
    return np.moveaxis(P, 0, a)


def gradient4_general(E: np.ndarray, h: Sequence[float], kind=None, value=None) -> List[np.ndarray]:
    """The 4th-order central gradient (Sec. 3.2) over the ghosts of ``pad_general``."""
    nd = E.ndim
    k, v = _faces(kind, value, nd)
    out = []
    for d in range(nd):
        a = _fld._axis(nd, d)
        P = pad_general(E, d, h[d], k[2 * d], v[2 * d], k[2 * d + 1], v[2 * d + 1])
        n = E.shape[a]

        def sh(q):
            sl = [slice(None)] * nd
            sl[a] = slice(2 + q, 2 + q + n)
            return P[tuple(sl)]
        out.append(((sh(-2) - sh(2)) + 8.0 * (sh(1) - sh(-1))) / (12.0 * h[d]))
    return out


def _boundary_slices(shape, d):
    nd = len(shape)
    a = _fld._axis(nd, d)
    lo = [slice(None)] * nd
    hi = [slice(None)] * nd
    lo[a] = 0
    hi[a] = shape[a] - 1
    return tuple(lo), tuple(hi)


def dirichlet_diagonal(D: np.ndarray, dt: float, h: Sequence[float], kind=None) -> np.ndarray:
    """alpha per cell: dt D / h_d^2 for each Dirichlet face of the cell."""
    nd = D.ndim
    k, _ = _faces(kind, None, nd)
    alpha = np.zeros_like(D)
    for d in range(nd):
        lo, hi = _boundary_slices(D.shape, d)
        if k[2 * d] == "dirichlet":
            alpha[lo] += dt * D[lo] / (h[d] * h[d])
        if k[2 * d + 1] == "dirichlet":
            alpha[hi] += dt * D[hi] / (h[d] * h[d])
    return alpha


def boundary_rhs(D: np.ndarray, dt: float, h: Sequence[float], kind=None, value=None) -> np.ndarray:
    """What the faces add to b = E^n: alpha E_B on Dirichlet faces, dt/h times the flux
    -D G (below) or D G (above) through fixed-gradient faces."""
    nd = D.ndim
    k, v = _faces(kind, value, nd)
    s = np.zeros_like(D)
    for d in range(nd):
        for side, sl in enumerate(_boundary_slices(D.shape, d)):
            f = 2 * d + side
            if k[f] == "dirichlet":
                s[sl] += dt * D[sl] / (h[d] * h[d]) * v[f]
            elif k[f] == "gradient":
                s[sl] += dt / h[d] * (D[sl] * v[f] if side else -D[sl] * v[f])
    return s


def face_weights_general(D: np.ndarray, dt: float, h: Sequence[float], kind=None) -> List[np.ndarray]:
    """Lower-face weights (``oracle.fld.face_weights``) plus, on periodic axes, the face
    between the last and the first cell in the first cell's slot."""
    nd = D.ndim
    k, _ = _faces(kind, None, nd)
    w = _fld.face_weights(D, dt, h)
    for d in range(nd):
        if k[2 * d] != "periodic":
            continue
        lo, hi = _boundary_slices(D.shape, d)
        DL, DR = D[hi], D[lo]
        w[d][lo] = dt * (2.0 * DL * DR / (DL + DR)) / (h[d] * h[d])
    return w


def assemble_general(w: Sequence[np.ndarray], kind=None) -> sp.csr_matrix:
    """``oracle.fld.assemble_operator`` plus the wrap-around faces of periodic axes."""
    shape = w[0].shape
    nd = len(shape)
    k, _ = _faces(kind, None, nd)
    A = _fld.assemble_operator(w).tolil()
    idx = np.arange(int(np.prod(shape))).reshape(shape)
    for d in range(nd):
        if k[2 * d] != "periodic":
            continue
        lo, hi = _boundary_slices(shape, d)
        first, last, wf = idx[lo].ravel(), idx[hi].ravel(), w[d][lo].ravel()
        for a, b, x in zip(first, last, wf):
            A[a, a] += x
            A[b, b] += x
            A[a, b] -= x
            A[b, a] -= x
    return A.tocsr()


def continuous_coupling(w: Sequence[np.ndarray], kind=None) -> sp.csr_matrix:
    """What the continuous faces add to A: for a boundary cell c with inner neighbour c1,
    the ghost x_g = 2 x_c - x_c1 couples through the boundary face with the weight w_B of
    the face between c and c1, so row c gains w_B (x_c - x_g) = w_B (x_c1 - x_c)."""
    shape = w[0].shape
    nd = len(shape)
    k, _ = _faces(kind, None, nd)
    N = int(np.prod(shape))
    idx = np.arange(N).reshape(shape)
    rows, cols, vals = [], [], []
    for d in range(nd):
        a = _fld._axis(nd, d)
        n = shape[a]
        if n < 2:
            continue
        for side in (0, 1):
            if k[2 * d + side] != "continuous":
                continue
            sl_c = [slice(None)] * nd
            sl_1 = [slice(None)] * nd
            sl_w = [slice(None)] * nd
            sl_c[a] = 0 if side == 0 else n - 1
            sl_1[a] = 1 if side == 0 else n - 2
            sl_w[a] = 1 if side == 0 else n - 1      # lower-face slot of the face between c and c1
            c = idx[tuple(sl_c)].ravel()
            c1 = idx[tuple(sl_1)].ravel()
            wB = w[d][tuple(sl_w)].ravel()
            rows += [c, c]
            cols += [c, c1]
            vals += [-wB, wB]
    if not rows:
        return sp.csr_matrix((N, N))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))


def diffusion_step_general(E: np.ndarray, kappa_rho: np.ndarray, dt: float, h: Sequence[float],
                           kind: Optional[Sequence] = None, value: Optional[Sequence] = None,
                           c: float = 1.0, limiter: str = "lp", method: str = "auto", tol=None):
    """One backward-Euler FLD step (Sec. 3.4) with per-face zero-flux, fixed-gradient,
    Dirichlet, periodic or continuous boundaries.  ``info.extra`` holds b, alpha and A.
    With continuous faces A is not symmetric: ``method="auto"`` then takes the sparse
    direct solve (SuperLU) instead of CG."""
    E = np.asarray(E, dtype=np.float64)
    kr = np.asarray(kappa_rho, dtype=np.float64)
    gr = gradient4_general(E, h, kind, value)
    R = np.sqrt(sum(x * x for x in gr)) / (kr * E)
    D = c * _fld.flux_limiter(R, limiter) / kr
    w = face_weights_general(D, dt, h, kind)
    alpha = dirichlet_diagonal(D, dt, h, kind)
    A = (assemble_general(w, kind) + sp.diags(alpha.ravel()) + continuous_coupling(w, kind)).tocsr()
    b = E + boundary_rhs(D, dt, h, kind, value)
    k, _ = _faces(kind, None, E.ndim)
    if method == "auto" and "continuous" in k and E.size > 4096:
        method = "direct"
    x, info = _fld.solve(A, b, method=method, tol=tol, w=w)
    info.extra["b"] = b
    info.extra["alpha"] = alpha
    info.extra["A"] = A
    return x, info
