"""Plain, slow FP64 oracle of the FLD radiation-energy step (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
leg may use this module.  It shares no code with the HIP path.

What it computes, in the paper's order (Moens et al., "Radiation-hydrodynamics
with MPI-AMRVAC: flux-limited diffusion"):

1. Ghost cells by even reflection across zero-flux domain faces (Sec. 3.4,
   Neumann "fixed gradient" boundaries with zero gradient).
2. The 4th-order, 5-point central gradient of E (Sec. 3.2, eq. ileyk_flux).
3. The radiation parameter ``R = |grad E| / (kappa rho E)`` (Sec. 2.2, the
   definition of R as mean free path over the energy scale height).
4. The flux limiter: the rational Levermore-Pomraning bridging law
   ``lambda = (2+R)/(6+3R+R^2)`` (Sec. 2.2, eq. fld_lambda) or the diffusion
   limit ``lambda = 1/3`` (Sec. 2.2).
5. ``D = c lambda / (kappa rho)`` at cell centres (Sec. 2.2, eq. fld_F;
   Sec. 3.4).
6. Face coefficients by the harmonic mean of the two cell values (Sec. 3.4).
7. The backward-Euler operator with lagged ``D^n``: the 5-point (2D) or
   7-point (3D) finite-volume stencil of Sec. 3.4, eq. discdiff, multiplied by
   dt: ``(A x)_i = x_i + sum_faces w_f (x_i - x_nb)`` with
   ``w_f = dt D_f / h_d^2``; ``A x = E^n``.
8. A (near-)exact solve of that linear system: dense LU on tiny grids,
   Gauss-Seidel or Jacobi-preconditioned CG otherwise, to a relative residual
   of 1e-13 or 10x the FP64 residual floor, whichever is larger.
9. The point-implicit gas-radiation energy exchange (Sec. 3.3): the quartic
   for the new gas internal energy, its unique root in ``]0, eps + E[``, and
   the back-substitution for E.  The root is found by bisection to adjacent
   doubles, not by the paper's Halley iteration, so the oracle does not mirror
   the GPU's root finder; the root is unique, so both give the same number.

Arrays are C-ordered ``(ny, nx)`` / ``(nz, ny, nx)``: x is the LAST array
axis.  ``h`` is given in x, y[, z] order.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

__all__ = [
    "LIMITERS", "pad_mirror", "gradient4", "radiation_parameter", "flux_limiter",
    "diffusion_coefficient", "face_weights", "assemble_operator", "apply_operator",
    "relative_residual", "q_b", "solve", "SolveInfo", "OracleNotConverged", "diffusion_step", "exchange",
    "exchange_coefficients", "fld_step", "residual_floor_tol",
]

LIMITERS = ("lp", "diffusion", "minerbo", "lp_exact")


# --------------------------------------------------------------------------------------
# 1-6: coefficients
# --------------------------------------------------------------------------------------
def _axis(ndim: int, d: int) -> int:
    """Array axis of spatial dimension d (d = 0 is x, the last axis)."""
    return ndim - 1 - d


def pad_mirror(E: np.ndarray, width: int = 2) -> np.ndarray:
    """Ghost layers by even reflection: ``E_{-1} = E_0, E_{-2} = E_1`` (and at the top end).

    Zero-flux (zero-gradient Neumann) boundaries of Sec. 3.4; corners are never
    read because every stencil here is axis-aligned.
    """
    return np.pad(E, width, mode="symmetric")


def gradient4(E: np.ndarray, h: Sequence[float]) -> List[np.ndarray]:
    """4th-order central gradient, one array per dimension (x first).

    Sec. 3.2, eq. ileyk_flux: ``(grad E)_x = (E_{i-2}/12 - 2E_{i-1}/3 + 2E_{i+1}/3
    - E_{i+2}/12) / dx``, applied along every axis with mirrored ghosts.
    """
    nd = E.ndim
    P = pad_mirror(E, 2)
    core = tuple(slice(2, 2 + s) for s in E.shape)
    out = []
    for d in range(nd):
        a = _axis(nd, d)

        def sh(k):
            sl = list(core)
            sl[a] = slice(2 + k, 2 + k + E.shape[a])
            return P[tuple(sl)]

        g = (sh(-2) / 12.0 - 2.0 * sh(-1) / 3.0 + 2.0 * sh(1) / 3.0 - sh(2) / 12.0) / h[d]
        out.append(g)
    return out


def radiation_parameter(E: np.ndarray, kappa_rho: np.ndarray, h: Sequence[float]) -> np.ndarray:
    """``R = |grad E| / (kappa rho E)``: Euclidean norm of the gradient (Sec. 2.2)."""
    g = gradient4(E, h)
    gnorm = np.sqrt(sum(gi * gi for gi in g))
    return gnorm / (kappa_rho * E)


def flux_limiter(R: np.ndarray, kind: str = "lp") -> np.ndarray:
    """Flux limiter lambda(R) (Sec. 2.2).

    ``"lp"``: the rational bridging law ``(2+R)/(6+3R+R^2)`` (eq. fld_lambda);
    ``"diffusion"``: the optically thick value 1/3;
    ``"minerbo"``: Minerbo (1978), the alternative Sec. 2.2 names without giving
    its form: ``2/(3 + sqrt(9 + 12 R^2))`` for R <= 3/2, ``1/(1 + R + sqrt(1 + 2R))``
    above (the two branches meet with equal value and slope at 3/2);
    ``"lp_exact"``: Levermore and Pomraning's own form ``(coth R - 1/R)/R``, which
    the rational law of eq. fld_lambda approximates; below R = 0.1 its series
    ``1/3 - R^2/45 + 2R^4/945 - R^6/4725 + 2R^8/93555`` (truncation < 1e-16)
    replaces the cancelling difference.
    """
    R = np.asarray(R, dtype=np.float64)
    if kind == "lp":
        return (2.0 + R) / (6.0 + 3.0 * R + R * R)
    if kind == "diffusion":
        return np.full_like(R, 1.0 / 3.0)
    if kind == "minerbo":
        lo = 2.0 / (3.0 + np.sqrt(9.0 + 12.0 * R * R))
        hi = 1.0 / (1.0 + R + np.sqrt(1.0 + 2.0 * R))
        return np.where(R <= 1.5, lo, hi)
    if kind == "lp_exact":
        R2 = R * R
        series = 1.0 / 3.0 + R2 * (-1.0 / 45.0 + R2 * (2.0 / 945.0 + R2 * (-1.0 / 4725.0 + R2 * 2.0 / 93555.0)))
        Rs = np.where(R < 0.1, 1.0, R)
        direct = (1.0 / np.tanh(Rs) - 1.0 / Rs) / Rs
        return np.where(R < 0.1, series, direct)
    raise ValueError(f"unknown limiter {kind!r}")


def diffusion_coefficient(E, kappa_rho, h, c: float = 1.0, limiter: str = "lp") -> np.ndarray:
    """Cell-centred ``D = c lambda(R) / (kappa rho)`` (Sec. 2.2 eq. fld_F; Sec. 3.4)."""
    R = radiation_parameter(E, kappa_rho, h)
    return c * flux_limiter(R, limiter) / kappa_rho


def face_weights(D: np.ndarray, dt: float, h: Sequence[float]) -> List[np.ndarray]:
    """Lower-face weights ``w_d[i] = dt * D_{i-1/2} / h_d^2`` per dimension (x first).

    ``D_{i-1/2} = 2 D_i D_{i-1} / (D_i + D_{i-1})`` (harmonic mean, Sec. 3.4).
    Entry i of ``w_d`` belongs to the face between cells i-1 and i along d; the
    entry at i = 0 is the domain face and carries no flux (zero-flux BC), so it is 0.
    """
    nd = D.ndim
    out = []
    for d in range(nd):
        a = _axis(nd, d)
        w = np.zeros_like(D)
        lo = [slice(None)] * nd
        hi = [slice(None)] * nd
        lo[a] = slice(0, D.shape[a] - 1)
        hi[a] = slice(1, D.shape[a])
        DL, DR = D[tuple(lo)], D[tuple(hi)]
        w[tuple(hi)] = dt * (2.0 * DL * DR / (DL + DR)) / (h[d] * h[d])
        out.append(w)
    return out


# --------------------------------------------------------------------------------------
# 7: operator
# --------------------------------------------------------------------------------------
def assemble_operator(w: Sequence[np.ndarray]) -> sp.csr_matrix:
    """Sparse ``A = I + dt L`` from lower-face weights (eq. discdiff times dt).

    Row i: diagonal ``1 + sum_f w_f``, off-diagonal ``-w_f`` to each neighbour.
    Symmetric, strictly diagonally dominant, ``lambda_min(A) >= 1``.
    """
    shape = w[0].shape
    nd = len(shape)
    N = int(np.prod(shape))
    idx = np.arange(N).reshape(shape)
    diag = np.ones(N)
    rows, cols, vals = [], [], []
    for d in range(nd):
        a = _axis(nd, d)
        hi = [slice(None)] * nd
        lo = [slice(None)] * nd
        hi[a] = slice(1, shape[a])
        lo[a] = slice(0, shape[a] - 1)
        wf = w[d][tuple(hi)].ravel()
        i_hi = idx[tuple(hi)].ravel()
        i_lo = idx[tuple(lo)].ravel()
        np.add.at(diag, i_hi, wf)
        np.add.at(diag, i_lo, wf)
        rows += [i_hi, i_lo]
        cols += [i_lo, i_hi]
        vals += [-wf, -wf]
    rows.append(np.arange(N))
    cols.append(np.arange(N))
    vals.append(diag)
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    return A


def apply_operator(w: Sequence[np.ndarray], x: np.ndarray) -> np.ndarray:
    """Matrix-free ``A x`` with the same stencil as ``assemble_operator``."""
    nd = x.ndim
    y = x.copy()
    for d in range(nd):
        a = _axis(nd, d)
        hi = [slice(None)] * nd
        lo = [slice(None)] * nd
        hi[a] = slice(1, x.shape[a])
        lo[a] = slice(0, x.shape[a] - 1)
        flux = w[d][tuple(hi)] * (x[tuple(hi)] - x[tuple(lo)])
        y[tuple(hi)] += flux
        y[tuple(lo)] -= flux
    return y


def relative_residual(A, x: np.ndarray, b: np.ndarray) -> float:
    """``||b - A x||_2 / ||b||_2`` in FP64 (the residual norm read of Sec. 3.4's "requested residual")."""
    r = b.ravel() - A @ x.ravel()
    return float(np.linalg.norm(r) / np.linalg.norm(b.ravel()))


def q_b(b: np.ndarray) -> float:
    """``||b||_2 / (sqrt(N) |mean b|)``: relative error <= q_b * relative residual.

    A is SPD with lambda_min >= 1 and conserves the sum under zero flux, so
    ``||x - x*|| <= ||b - A x||`` and ``||x*|| >= |sum b| / sqrt(N)``.
    """
    b = b.ravel()
    return float(np.linalg.norm(b) / (math.sqrt(b.size) * abs(b.mean())))


def residual_floor_tol(w: Sequence[np.ndarray], target: float = 1e-13) -> Tuple[float, str]:
    """Stop tolerance ``max(target, 10 x FP64 residual floor)`` and which limit applied.

    The floor of a computed FP64 residual grows with the stencil weight; it is
    estimated as ``1.5e-15 * max_i sum_f w_f(i)`` (10x a measured floor of
    ~1.5e-16 per unit weight for an iterative solve).
    """
    s = np.zeros_like(w[0])
    nd = s.ndim
    for d in range(nd):
        a = _axis(nd, d)
        s += w[d]
        hi = [slice(None)] * nd
        lo = [slice(None)] * nd
        hi[a] = slice(1, s.shape[a])
        lo[a] = slice(0, s.shape[a] - 1)
        s[tuple(lo)] += w[d][tuple(hi)]
    floor = 1.5e-15 * float(s.max())
    return (target, "target") if target >= floor else (floor, "fp64-floor")


# --------------------------------------------------------------------------------------
# 8: solve
# --------------------------------------------------------------------------------------
@dataclass
class SolveInfo:
    method: str
    iterations: int
    rel_residual: float
    tol: float
    tol_kind: str
    seconds: float
    extra: Dict = field(default_factory=dict)


class OracleNotConverged(RuntimeError):
    """The solve ended above its tolerance; ``info`` holds where it stopped."""

    def __init__(self, msg: str, info: "SolveInfo"):
        super().__init__(msg)
        self.info = info


def _pcg(A, b, x0, tol, maxiter):
    """Jacobi-preconditioned conjugate gradients on SPD A (plain textbook loop)."""
    dinv = 1.0 / A.diagonal()
    x = x0.copy()
    bnorm = np.linalg.norm(b)
    r = b - A @ x
    z = dinv * r
    p = z.copy()
    rz = r @ z
    it = 0
    best = (np.linalg.norm(r) / bnorm, x.copy())
    stall = 0
    while it < maxiter:
        Ap = A @ p
        alpha = rz / (p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        it += 1
        if it % 50 == 0 or np.linalg.norm(r) <= tol * bnorm:
            r = b - A @ x                      # replace the recursive residual by the true one
            rel = np.linalg.norm(r) / bnorm
            if rel < best[0] * 0.999:
                best = (rel, x.copy())
                stall = 0
            else:
                stall += 1
            if rel <= tol or stall >= 6:
                break
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    rel = np.linalg.norm(b - A @ x) / bnorm
    if best[0] < rel:
        x, rel = best[1], best[0]
    return x, it, float(rel)


def _gauss_seidel(A, b, x0, tol, maxiter):
    """Lexicographic Gauss-Seidel: ``x <- (D + L)^{-1} (b - U x)`` until the residual target."""
    L = sp.tril(A, k=0, format="csr")
    U = sp.triu(A, k=1, format="csr")
    x = x0.copy()
    bnorm = np.linalg.norm(b)
    it = 0
    rel = np.linalg.norm(b - A @ x) / bnorm
    while it < maxiter and rel > tol:
        x = spla.spsolve_triangular(L, b - U @ x, lower=True)
        it += 1
        rel = np.linalg.norm(b - A @ x) / bnorm
    return x, it, float(rel)


def solve(A, b: np.ndarray, method: str = "auto", tol: Optional[float] = None,
          w: Optional[Sequence[np.ndarray]] = None, x0: Optional[np.ndarray] = None,
          maxiter: int = 200000) -> Tuple[np.ndarray, SolveInfo]:
    """Solve ``A x = b`` (near-)exactly in FP64.

    ``method``: ``"lu"`` (dense LU, N <= 4096), ``"gs"``, ``"cg"`` (Jacobi-PCG),
    ``"direct"`` (sparse LU, SuperLU) or ``"auto"`` (LU for N <= 4096, else CG).
    """
    shape = b.shape
    bb = b.ravel().astype(np.float64)
    N = bb.size
    if tol is None:
        tol, kind = residual_floor_tol(w) if w is not None else (1e-13, "target")
    else:
        kind = "given"
    if method == "auto":
        method = "lu" if N <= 4096 else "cg"
    t0 = time.perf_counter()
    xs = bb.copy() if x0 is None else x0.ravel().astype(np.float64).copy()
    if method == "lu":
        if N > 4096:
            raise ValueError("dense LU is for N <= 4096")
        x = np.linalg.solve(A.toarray(), bb)
        it = 1
    elif method == "direct":
        x = spla.spsolve(A.tocsc(), bb)
        it = 1
    elif method == "gs":
        x, it, _ = _gauss_seidel(A, bb, xs, tol, maxiter)
    elif method == "cg":
        x, it, _ = _pcg(A, bb, xs, tol, maxiter)
    else:
        raise ValueError(f"unknown method {method!r}")
    rel = float(np.linalg.norm(bb - A @ x) / np.linalg.norm(bb))
    info = SolveInfo(method=method, iterations=it, rel_residual=rel, tol=tol, tol_kind=kind,
                     seconds=time.perf_counter() - t0)
    if not rel <= tol:
        # an answer that misses its own stop rule is no reference: refuse it
        raise OracleNotConverged(f"{method} stopped at relative residual {rel:.3e} > tol {tol:.3e} "
                                 f"after {it} iterations (N = {N})", info)
    return x.reshape(shape), info


def diffusion_step(E: np.ndarray, kappa_rho: np.ndarray, dt: float, h: Sequence[float],
                   c: float = 1.0, limiter: str = "lp", method: str = "auto",
                   tol: Optional[float] = None, return_operator: bool = False):
    """One backward-Euler FLD step with lagged D (Sec. 3.4).

    Solves ``E^{n+1}/dt - div(D^n grad E^{n+1}) = E^n/dt`` in the dt-multiplied
    form ``A E^{n+1} = E^n``.  Returns ``(E_new, info)`` (plus ``(A, w)`` if asked).
    """
    E = np.asarray(E, dtype=np.float64)
    D = diffusion_coefficient(E, kappa_rho, h, c, limiter)
    w = face_weights(D, dt, h)
    A = assemble_operator(w)
    x, info = solve(A, E, method=method, tol=tol, w=w)
    info.extra["q_b"] = q_b(E)
    if return_operator:
        return x, info, A, w
    return x, info


# --------------------------------------------------------------------------------------
# 9: energy exchange
# --------------------------------------------------------------------------------------
def exchange_coefficients(rho, kappa, dt, c, a_r, c_v):
    """``a1, a2`` of the exchange quartic (Sec. 3.3).

    From the point-implicit pair of Sec. 3.3 with ``T_g = eps / (rho c_v)``,
    ``c_v = k_b / ((gamma - 1) mu m_p)`` and ``4 sigma = c a_r``:
    ``a1 = c a_r kappa dt / (rho^3 c_v^4)`` and ``a2 = c kappa rho dt``.
    (The printed a1 omits the ``(mu m_p / k_b)^4`` factor and places dt
    ambiguously; this is the value for which the quartic and the
    back-substitution of Sec. 3.3 both hold.)
    """
    a1 = c * a_r * kappa * dt / (rho ** 3 * c_v ** 4)
    a2 = c * kappa * rho * dt
    return a1, a2


def exchange(E: np.ndarray, eps: np.ndarray, rho: np.ndarray, kappa: np.ndarray, dt: float,
             c: float = 1.0, a_r: float = 1.0, c_v: float = 1.0):
    """Implicit gas-radiation energy exchange per cell (Sec. 3.3).

    New gas energy: the root of ``a1 x^4 + (1+a2) x - ((1+a2) eps + a2 E) = 0``
    in ``]0, eps + E[``; new radiation energy: ``(a1 x^4 + E)/(1 + a2)``.
    Scaling ``x = C y / (1 + a2)`` with ``C = (1+a2) eps + a2 E`` turns the
    quartic into ``beta y^4 + y - 1 = 0`` (``beta = a1 C^3/(1+a2)^4``), whose
    root lies in ``(0, 1]``; it is bracketed and halved until the bracket is two
    adjacent doubles.  Returns ``(E_new, eps_new)``.
    """
    E = np.asarray(E, dtype=np.float64)
    eps = np.asarray(eps, dtype=np.float64)
    a1, a2 = exchange_coefficients(rho, kappa, dt, c, a_r, c_v)
    a1 = np.broadcast_to(a1, E.shape)
    a2 = np.broadcast_to(a2, E.shape)
    C = (1.0 + a2) * eps + a2 * E
    beta = a1 * C ** 3 / (1.0 + a2) ** 4

    def f(y):
        return beta * y ** 4 + y - 1.0

    lo = np.zeros_like(E)
    hi = np.ones_like(E)
    for _ in range(1200):
        mid = 0.5 * (lo + hi)
        active = (mid > lo) & (mid < hi)
        if not active.any():
            break
        fm = f(mid)
        up = active & (fm > 0.0)
        dn = active & ~(fm > 0.0)
        hi = np.where(up, mid, hi)
        lo = np.where(dn, mid, lo)
    y = np.where(np.abs(f(lo)) <= np.abs(f(hi)), lo, hi)
    eps_new = C * y / (1.0 + a2)
    E_new = (a1 * eps_new ** 4 + E) / (1.0 + a2)
    return E_new, eps_new


# --------------------------------------------------------------------------------------
# full step
# --------------------------------------------------------------------------------------
def fld_step(E, kappa_rho, dt, h, c=1.0, limiter="lp", gas: Optional[dict] = None,
             method="auto", tol=None):
    """Diffusion then (optionally) exchange: one step of the radiation-only split.

    The paper's explicit operator applies the local implicit exchange before the
    implicit diffusion; this step applies diffusion first and then exchange.
    ``gas`` holds ``eps, rho, kappa, a_r, c_v`` (``c`` is shared).  Returns
    ``(E_new, eps_new_or_None, info)``.
    """
    x, info = diffusion_step(E, kappa_rho, dt, h, c, limiter, method, tol)
    if gas is None:
        return x, None, info
    E2, eps2 = exchange(x, gas["eps"], gas["rho"], gas["kappa"], dt, c, gas["a_r"], gas["c_v"])
    return E2, eps2, info

