"""Seeded synthetic inputs for the FLD radiation-energy step.

This module defines INPUTS only: smooth random fields, the five workload
recipes (sizes, opacity / energy / gas-temperature fields, time steps, the
request stream), and nothing of the method itself (no gradient, limiter,
operator, solver or energy exchange).  Both the FP64 oracle and the GPU
harness draw their inputs from here, so the two sides see identical arrays.

Array layout: a 2D grid is a C-ordered ``(ny, nx)`` array and a 3D grid a
``(nz, ny, nx)`` array, so x is the fastest index
(``idx = i + nx*(j + ny*k)``).  Cell centres of the unit square / cube are
``x_i = (i + 1/2) h`` with ``h = 1/n``.

Smooth random field (a definition of the inputs):
  * ``numpy.random.default_rng(seed)`` (PCG64);
  * 32 integer wave vectors ``k_m`` drawn uniformly from ``{-8..8}^d``,
    redrawn while zero;
  * amplitudes ``a_m ~ N(0,1)/(1+|k_m|)``, phases ``phi_m ~ U[0, 2 pi)``;
  * ``f(x) = sum_m a_m cos(2 pi k_m . x + phi_m)`` at the cell centres.
"Spanning lo..hi" is the affine rescale of ``f`` onto ``[lo, hi]`` by its grid
min / max; "log-normal sigma" is ``exp(sigma (f - mean f) / std f)``.

Seeds: single-grid workloads use ``1000*config + field``; per-grid and
per-request fields use ``10**6*config + 10*index + field``
(field 1 = kappa*rho, 2 = E, 3 = gas-temperature factor).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "smooth_field", "span", "lognormal", "cell_centres",
    "GridInput", "pulse_2d", "random_grid", "gas_for", "c2_inputs",
    "c3_inputs", "c4_layout", "c4_grid", "c4_inputs", "c5_stream", "Request",
    "E1_HEATCOOL", "E4_THIN", "CGS", "e1_grid", "e4_grid",
]

N_MODES = 32
K_MAX = 8


def cell_centres(n: int) -> np.ndarray:
    """Cell-centre coordinates of ``n`` uniform cells on [0, 1]."""
    return (np.arange(n, dtype=np.float64) + 0.5) / n


def _modes(ndim: int, seed: int, n_modes: int = N_MODES, kmax: int = K_MAX):
    rng = np.random.default_rng(seed)
    ks = np.zeros((n_modes, ndim), dtype=np.int64)
    for m in range(n_modes):
        while True:
            k = rng.integers(-kmax, kmax + 1, size=ndim)
            if np.any(k != 0):
                break
        ks[m] = k
    amp = rng.standard_normal(n_modes) / (1.0 + np.linalg.norm(ks, axis=1))
    phase = rng.uniform(0.0, 2.0 * math.pi, size=n_modes)
    return ks, amp, phase


def smooth_field(shape: Sequence[int], seed: int, backend: str = "numpy",
                 device=None):
    """Sum of 32 random Fourier modes at the cell centres of ``shape``.

    ``shape`` is the array shape (``(ny, nx)`` or ``(nz, ny, nx)``).  The mode
    draw always comes from numpy's PCG64; ``backend="torch"`` evaluates the
    same sum with torch (float64) on ``device`` for bulk generation.
    """
    shape = tuple(int(s) for s in shape)
    ndim = len(shape)
    ks, amp, phase = _modes(ndim, seed)
    # axis a of the array is spatial dimension ndim-1-a (x is the last axis)
    if backend == "numpy":
        xs = [cell_centres(shape[ndim - 1 - d]) for d in range(ndim)]
        out = np.zeros(shape, dtype=np.float64)
        for m in range(len(amp)):
            # separable evaluation: exp(i(2pi k.x + phi)) = e^{i phi} prod_d e^{2 pi i k_d x_d}
            acc = np.exp(1j * phase[m]) * amp[m]
            term = None
            for d in range(ndim):
                e = np.exp(2j * math.pi * ks[m, d] * xs[d])
                sh = [1] * ndim
                sh[ndim - 1 - d] = shape[ndim - 1 - d]
                e = e.reshape(sh)
                term = e if term is None else term * e
            out += (acc * term).real
        return out
    if backend == "torch":
        import torch
        dev = torch.device(device if device is not None else "cpu")
        xs = [(torch.arange(shape[ndim - 1 - d], dtype=torch.float64, device=dev) + 0.5)
              / shape[ndim - 1 - d] for d in range(ndim)]
        out = torch.zeros(shape, dtype=torch.float64, device=dev)
        for m in range(len(amp)):
            acc = complex(np.exp(1j * phase[m]) * amp[m])
            term = None
            for d in range(ndim):
                e = torch.exp(2j * math.pi * float(ks[m, d]) * xs[d].to(torch.complex128))
                sh = [1] * ndim
                sh[ndim - 1 - d] = shape[ndim - 1 - d]
                e = e.reshape(sh)
                term = e if term is None else term * e
            out += (acc * term).real
        return out
    raise ValueError(f"unknown backend {backend!r}")


def span(f, lo: float, hi: float):
    """Affine rescale of ``f`` onto [lo, hi] using its min / max."""
    fmin, fmax = f.min(), f.max()
    return lo + (hi - lo) * (f - fmin) / (fmax - fmin)


def lognormal(f, sigma: float):
    """``exp(sigma * (f - mean f) / std f)`` (population standard deviation)."""
    if isinstance(f, np.ndarray):
        return np.exp(sigma * (f - f.mean()) / f.std())
    return (sigma * (f - f.mean()) / f.std(correction=0)).exp()


@dataclass
class GridInput:
    """One grid's inputs for the diffusion step (and the gas, if any)."""
    E: np.ndarray                  # radiation energy density E^n, shape (ny,nx) or (nz,ny,nx)
    kappa_rho: np.ndarray          # kappa*rho at cell centres
    dt: float
    h: tuple                       # (hx, hy[, hz]) cell widths, x first
    c: float = 1.0
    limiter: str = "lp"            # "lp" (rational Levermore-Pomraning) or "diffusion" (lambda = 1/3)
    rho: Optional[np.ndarray] = None
    kappa: Optional[np.ndarray] = None
    eps: Optional[np.ndarray] = None   # gas internal energy density
    a_r: float = 1.0
    c_v: float = 1.0

    @property
    def ndim(self) -> int:
        return self.E.ndim

    @property
    def n(self) -> tuple:
        """Cell counts in x, y[, z] order."""
        return tuple(reversed(self.E.shape))


def pulse_2d(n: int = 64, kappa_rho: float = 10.0, amp: float = 1e3, sigma: float = 0.05,
             dt: float = 1e-3, c: float = 1.0, limiter: str = "lp") -> GridInput:
    """The 64^2 pulse workload: a Gaussian pulse on the unit square, constant kappa*rho.

    ``E = 1 + amp*exp(-r^2/(2 sigma^2))`` with r measured from (1/2, 1/2).
    """
    x = cell_centres(n)
    X, Y = np.meshgrid(x, x, indexing="xy")     # X varies along the last axis
    r2 = (X - 0.5) ** 2 + (Y - 0.5) ** 2
    E = 1.0 + amp * np.exp(-r2 / (2.0 * sigma ** 2))
    kr = np.full((n, n), kappa_rho, dtype=np.float64)
    return GridInput(E=E, kappa_rho=kr, dt=dt, h=(1.0 / n, 1.0 / n), c=c, limiter=limiter)


def random_grid(shape: Sequence[int], seed_base: int, dt: float,
                logkr_span=(-2.0, 2.0), e_sigma: float = 1.0, backend: str = "numpy",
                device=None) -> GridInput:
    """Random smooth opacity / log-normal energy fields on the unit square/cube.

    ``log10(kappa*rho)`` spans ``logkr_span`` (field seed ``seed_base+1``) and
    ``E`` is log-normal (field seed ``seed_base+2``).
    """
    shape = tuple(int(s) for s in shape)
    f1 = smooth_field(shape, seed_base + 1, backend=backend, device=device)
    f2 = smooth_field(shape, seed_base + 2, backend=backend, device=device)
    kr = 10.0 ** span(f1, *logkr_span)
    E = lognormal(f2, e_sigma)
    h = tuple(1.0 / s for s in reversed(shape))
    return GridInput(E=E, kappa_rho=kr, dt=dt, h=h)


def gas_for(g: GridInput, seed: int, u_span=(-0.5, 0.5)) -> GridInput:
    """Attach a gas to ``g``: rho = 1 (so kappa = kappa*rho), c = a_r = c_v = 1.

    ``T_g = (E/a_r)^(1/4) * 10^u`` with u a smooth field spanning ``u_span``
    (field seed ``seed``), so cells both heat and cool; ``eps = rho c_v T_g``.
    """
    u = span(smooth_field(g.E.shape, seed), *u_span)
    rho = np.ones_like(g.E)
    T = (g.E / g.a_r) ** 0.25 * 10.0 ** u
    g.rho = rho
    g.kappa = g.kappa_rho / rho
    g.eps = rho * g.c_v * T
    return g


def c2_inputs(n: int = 1024) -> GridInput:
    """The 2D workload with gas: n x n, log10(kappa rho) in [-2, 2], log-normal E, dt = 1e-3."""
    g = random_grid((n, n), 2000, dt=1e-3)
    return gas_for(g, 2003)


def c3_inputs(n: int = 256, backend: str = "numpy", device=None) -> GridInput:
    """The 3D workload: n^3 with the 2D workload's field recipe in 3D (seeds 3001, 3002), dt = 1e-3."""
    return random_grid((n, n, n), 3000, dt=1e-3, backend=backend, device=device)


C4_SIDES = tuple(range(64, 513, 32))           # {64, 96, ..., 512}: 15 values


def c4_layout(n_grids: int = 512, sides: Sequence[int] = C4_SIDES, seed: int = 4000,
              dt_range=(1e-4, 1e-2)):
    """Sizes and time steps of the 512-grid batch: side ``n_j ~ U(sides)``, ``dt_j ~ U[dt_range]``."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.asarray(sides), size=n_grids)
    dts = rng.uniform(dt_range[0], dt_range[1], size=n_grids)
    return [(int(n), float(d)) for n, d in zip(ns, dts)]


def c4_grid(j: int, n: int, dt: float, backend: str = "numpy", device=None) -> GridInput:
    """Grid ``j`` of the 512-grid batch (its own opacity / energy fields)."""
    return random_grid((n, n), 4 * 10 ** 6 + 10 * j, dt=dt, backend=backend, device=device)


def c4_inputs(n_grids: int = 512, **kw) -> List[GridInput]:
    """The 512-grid batch: independent 2D grids with seeded sides, dt and fields."""
    return [c4_grid(j, n, dt) for j, (n, dt) in enumerate(c4_layout(n_grids, **kw))]


@dataclass
class Request:
    """One request of the served stream."""
    index: int
    t_arrival: float          # seconds from stream start
    shape: tuple              # array shape
    dt: float
    seed_base: int

    @property
    def cells(self) -> int:
        return int(np.prod(self.shape))

    def inputs(self, backend: str = "numpy", device=None) -> GridInput:
        return random_grid(self.shape, self.seed_base, dt=self.dt, backend=backend, device=device)


C5_SIDES_2D = tuple(range(128, 1025, 32))      # {128, 160, ..., 1024}
C5_SIDES_3D = tuple(range(32, 193, 16))        # {32, 48, ..., 192}


def c5_stream(n_requests: int = 4096, rate: float = 2000.0, seed: int = 5000,
              sides_2d: Sequence[int] = C5_SIDES_2D, sides_3d: Sequence[int] = C5_SIDES_3D,
              dt_range=(1e-4, 1e-2)) -> List[Request]:
    """The served stream: Poisson arrivals of mixed 2D / 3D solves (exponential gaps)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    is3d = rng.random(n_requests) < 0.5
    s2 = rng.choice(np.asarray(sides_2d), size=n_requests)
    s3 = rng.choice(np.asarray(sides_3d), size=n_requests)
    dts = rng.uniform(dt_range[0], dt_range[1], size=n_requests)
    reqs = []
    for i in range(n_requests):
        shape = (int(s3[i]),) * 3 if is3d[i] else (int(s2[i]),) * 2
        reqs.append(Request(index=i, t_arrival=float(t[i]), shape=shape, dt=float(dts[i]),
                            seed_base=5 * 10 ** 6 + 10 * i))
    return reqs


# --- physical set-ups of the paper's two hot-path experiments (cgs units) ----------------
CGS = dict(
    c=2.99792458e10,           # speed of light [cm/s]
    sigma=5.670374419e-5,      # Stefan-Boltzmann [erg cm^-2 s^-1 K^-4]
    k_b=1.380649e-16,          # Boltzmann [erg/K]
    m_p=1.67262192369e-24,     # proton mass [g]
)
CGS["a_r"] = 4.0 * CGS["sigma"] / CGS["c"]

# Heating/cooling relaxation test (section "Heating and Cooling"): zero velocity,
# constant density; parameters as the paper states them.
E1_HEATCOOL = dict(rho=1e-7, kappa=0.4, gamma=5.0 / 3.0, mu=0.6, E=1e12,
                   e_factors=(1e-6, 1e2), dts=(1e-12, 1e-11))

# Optically thin front test (section "Optically thin limit"): diffusion only.
E4_THIN = dict(x_lo=-0.5, x_hi=1.5, n=256, rho=0.025, kappa=0.4, d=0.05,
               E1=1.4e11, E0=1.4e-11, dt=1e-13)


def e1_grid(e0: float, n: int = 8) -> GridInput:
    """The heating/cooling box as an n x n grid of uniform cells (the periodic
    boundaries of the test play no part: every field is uniform), with initial gas
    energy density ``e0``; CGS constants, c_v = k_b / ((gamma - 1) mu m_p)."""
    p = E1_HEATCOOL
    shape = (n, n)
    c_v = CGS["k_b"] / ((p["gamma"] - 1.0) * p["mu"] * CGS["m_p"])
    g = GridInput(E=np.full(shape, p["E"]), kappa_rho=np.full(shape, p["kappa"] * p["rho"]),
                  dt=p["dts"][0], h=(1.0 / n, 1.0 / n), c=CGS["c"], a_r=CGS["a_r"], c_v=c_v)
    g.rho = np.full(shape, p["rho"])
    g.kappa = np.full(shape, p["kappa"])
    g.eps = np.full(shape, float(e0))
    return g


def e4_grid(ny: int = 4) -> GridInput:
    """The optically thin slab as an n x ny grid (x across the front, ny copies):
    E = E0 + (1 - erf(x / d)) E1 / 2 at the cell centres, kappa rho uniform, CGS c."""
    from math import erf
    p = E4_THIN
    hx = (p["x_hi"] - p["x_lo"]) / p["n"]
    xc = p["x_lo"] + (np.arange(p["n"]) + 0.5) * hx
    row = p["E0"] + 0.5 * (1.0 - np.array([erf(x / p["d"]) for x in xc])) * p["E1"]
    E = np.tile(row, (ny, 1))
    return GridInput(E=E, kappa_rho=np.full(E.shape, p["rho"] * p["kappa"]), dt=p["dt"], h=(hx, hx),
                     c=CGS["c"])

