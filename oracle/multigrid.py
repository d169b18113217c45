"""Plain FP64 oracle of the multigrid coarse operators (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
leg may use this module.  It shares no code with the HIP path.

Sec. 3.4 solves the backward-Euler system with a multigrid solver whose coarse
levels the paper does not spell out.  Two coarse operators of the cell-centred
hierarchy (every axis halved, a coarse cell owning its 2^d children) are written
out here:

* rediscretised: the coarse face between two coarse cells carries the mean of
  the fine face weights dt D_f / h^2 of its 2^(d-1) sub-faces, times 1/4 for the
  doubled cell width, i.e. the operator of eq. discdiff rebuilt on the coarse
  grid from the averaged face coefficients;
* Galerkin: ``A_c = R A P`` with P the piecewise-constant prolongation (every
  child takes its parent's value) and ``R = P^T / 2^d`` (the mean of the
  children), the coarse operator that the restriction and prolongation of the
  V-cycle imply.

Both keep the form ``(A_c x)_I = x_I + sum_faces w_c (x_I - x_nb)``, so each is
returned as lower-face weights in the layout of ``oracle.fld.face_weights``.
Arrays are C-ordered with x the last axis.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np
import scipy.sparse as sp

from . import fld as _fld

__all__ = [
    "prolongation_constant", "restriction_mean", "galerkin_operator",
    "coarse_weights_galerkin", "coarse_weights_rediscretised", "weights_from_operator",
]


def _coarse_shape(shape: Sequence[int]) -> tuple:
    if any(n % 2 for n in shape):
        raise ValueError("every axis must be even to coarsen")
    return tuple(n // 2 for n in shape)


def prolongation_constant(shape: Sequence[int]) -> sp.csr_matrix:
    """P: fine x coarse, 1 where the fine cell lies in the coarse cell."""
    shape = tuple(shape)
    cs = _coarse_shape(shape)
    fine = np.indices(shape).reshape(len(shape), -1)
    parent = np.ravel_multi_index(tuple(fine // 2), cs)
    N, Nc = int(np.prod(shape)), int(np.prod(cs))
    return sp.csr_matrix((np.ones(N), (np.arange(N), parent)), shape=(N, Nc))


def restriction_mean(shape: Sequence[int]) -> sp.csr_matrix:
    """R = P^T / 2^d: the mean over the 2^d children."""
    return (prolongation_constant(shape).T / float(2 ** len(shape))).tocsr()


def galerkin_operator(A: sp.spmatrix, shape: Sequence[int]) -> sp.csr_matrix:
    """``A_c = R A P`` on the coarse grid of ``shape``."""
    P = prolongation_constant(shape)
    return (restriction_mean(shape) @ A @ P).tocsr()


def weights_from_operator(A: sp.spmatrix, shape: Sequence[int]) -> List[np.ndarray]:
    """Lower-face weights of a matrix of the form I + sum w (x_i - x_nb): w is minus the
    off-diagonal entry between a cell and its lower neighbour along each axis."""
    shape = tuple(shape)
    nd = len(shape)
    A = A.tocsr()
    idx = np.arange(int(np.prod(shape))).reshape(shape)
    out = []
    for d in range(nd):
        a = nd - 1 - d                                    # x is the last axis
        w = np.zeros(shape)
        hi = [slice(None)] * nd
        lo = [slice(None)] * nd
        hi[a] = slice(1, shape[a])
        lo[a] = slice(0, shape[a] - 1)
        rows = idx[tuple(hi)].ravel()
        cols = idx[tuple(lo)].ravel()
        w[tuple(hi)] = -np.asarray(A[rows, cols]).ravel().reshape(w[tuple(hi)].shape)
        out.append(w)
    return out


def coarse_weights_galerkin(w: Sequence[np.ndarray]) -> List[np.ndarray]:
    """Coarse lower-face weights of ``R A P`` for the fine weights ``w``."""
    shape = w[0].shape
    return weights_from_operator(galerkin_operator(_fld.assemble_operator(w), shape), _coarse_shape(shape))


def coarse_weights_rediscretised(w: Sequence[np.ndarray]) -> List[np.ndarray]:
    """Coarse lower-face weights by averaging the sub-face weights, times 1/4."""
    shape = w[0].shape
    nd = len(shape)
    cs = _coarse_shape(shape)
    out = []
    for d in range(nd):
        a = nd - 1 - d
        wc = np.zeros(cs)
        # the fine faces on coarse face I (lower face of coarse cell I along d) are the
        # lower faces of the children with even index along d
        sel = [slice(None)] * nd
        sel[a] = slice(0, shape[a], 2)
        sub = w[d][tuple(sel)]                               # shape cs along a, fine elsewhere
        acc = np.zeros(cs)
        for off in np.ndindex(*([2] * nd)):
            if off[a]:
                continue
            pick = tuple(slice(o, None, 2) if ax != a else slice(None) for ax, o in enumerate(off))
            acc += sub[pick]
        wc[...] = acc / float(2 ** (nd - 1)) / 4.0
        lo = [slice(None)] * nd
        lo[a] = 0
        wc[tuple(lo)] = 0.0                                   # domain face
        out.append(wc)
    return out
