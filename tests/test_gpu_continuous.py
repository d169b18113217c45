"""Continuous boundaries (Sec. 3.4: E^{n+1} extrapolated linearly into the ghost cells)
on the device against the FP64 oracle, alone and mixed with the other face kinds.

The operator is an M-matrix whose rows all sum to one, but it is not symmetric, so the
plans iterate plain V-cycles (defect correction) and the residual bounds the error
only in the max norm (||x - x*||_inf <= ||b - A x||_inf); the runs solve to a relative
residual of 1e-12 and are compared with the oracle's sparse direct solve at 1e-10
relative L2."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import oracle as O                     # noqa: E402
from oracle import dirichlet as OD     # noqa: E402
import workloads as W                  # noqa: E402
import paper_2104_03968_amd as fld     # noqa: E402
from tests.gpu_common import dev, rel_l2   # noqa: E402

CODES = {"zero_flux": fld.FLD_BC_ZERO_FLUX, "gradient": fld.FLD_BC_FIXED_GRADIENT,
         "dirichlet": fld.FLD_BC_DIRICHLET, "continuous": fld.FLD_BC_CONTINUOUS}
KINDS = ["continuous", "continuous", "zero_flux", "continuous", "continuous", "zero_flux"]
MIXED_KINDS = ["continuous", "dirichlet", "gradient", "continuous", "zero_flux", "continuous"]
VALUES = [0.0, 1.5, -0.6, 0.0, 0.0, 0.0]


def _opts(kinds, values):
    return dict(bc=[CODES[k] for k in kinds],
                bc_grad=[v if k == "gradient" else 0.0 for k, v in zip(kinds, values)],
                bc_value=[v if k == "dirichlet" else 0.0 for k, v in zip(kinds, values)])


def _run(grids, kinds, values, **kw):
    plan = fld.Plan([g.E.shape for g in grids], h=[g.h for g in grids], krylov=0, **_opts(kinds, values), **kw)
    E = [dev(g.E) for g in grids]
    K = [dev(g.kappa_rho) for g in grids]
    out = [torch.empty_like(e) for e in E]
    rc, st = plan.step(E, K, out, [g.dt for g in grids], check=False)
    torch.cuda.synchronize()
    return plan, rc, st, [o.cpu().numpy() for o in out]


@pytest.mark.parametrize("kinds", [KINDS, MIXED_KINDS], ids=["continuous", "mixed-kinds"])
@pytest.mark.parametrize("fmg", [1, 0])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("limiter", ["lp", "diffusion"])
def test_continuous_step_matches_oracle(limiter, precision, fmg, kinds):
    gs = [W.random_grid((70, 96), 66000, dt=4e-3), W.random_grid((16, 18, 20), 66100, dt=4e-3),
          W.random_grid((33, 40), 66200, dt=1e-2)]
    refs = [OD.diffusion_step_general(g.E, g.kappa_rho, g.dt, g.h, kinds[:2 * g.E.ndim], VALUES[:2 * g.E.ndim],
                                      c=1.2, limiter=limiter, method="direct") for g in gs]
    plan, rc, st, xs = _run(gs, kinds, VALUES, rtol=1e-12, precision=precision, fmg=fmg,
                            limiter=fld.LIMITER_CODES[limiter], c=1.2, max_cycles=200)
    assert rc == fld.FLD_OK, st
    for (x_or, info), x, s in zip(refs, xs, st):
        assert rel_l2(x, x_or) <= 1e-10, (x.shape, rel_l2(x, x_or), s)
        assert s["b_sum"] == pytest.approx(info.extra["b"].sum(), rel=1e-12)
    plan.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_linear_profile_is_steady(precision):
    """A profile linear in x with continuous x faces (constant D) does not change; zero
    flux at the same faces bends it."""
    for shape in ((40, 96), (10, 12, 48)):
        g = W.random_grid(shape, 66300 + len(shape), dt=2e-2)
        xc = (np.arange(shape[-1]) + 0.5) / shape[-1]
        g.E = np.broadcast_to(1.0 + 0.9 * xc, shape).copy()
        g.kappa_rho = np.full(shape, 2.0)
        kinds = ["continuous", "continuous", "zero_flux", "zero_flux", "zero_flux", "zero_flux"]
        plan, rc, (st,), (x,) = _run([g], kinds, [0.0] * 6, rtol=1e-13, precision=precision,
                                     limiter=fld.FLD_LIMITER_DIFFUSION)
        assert rc == fld.FLD_OK, st
        assert np.abs(x - g.E).max() <= 1e-11 * g.E.max()
        plan.close()


def test_moments_use_the_continuous_ghosts():
    g = W.random_grid((40, 52), 66400, dt=1e-3)
    kinds, vals = ["continuous", "zero_flux", "continuous", "continuous"], [0.0] * 4
    plan, rc, _, _ = _run([g], kinds, vals)
    (out,) = plan.radiation_moments([dev(g.E)], [dev(g.kappa_rho)], want=("F",))
    torch.cuda.synchronize()
    gr = OD.gradient4_general(g.E, g.h, kinds, vals)
    gn = np.sqrt(sum(x * x for x in gr))
    lam = O.flux_limiter(gn / (g.kappa_rho * g.E))
    for a in range(2):
        Fo = -lam / g.kappa_rho * gr[a]
        Fg = out["F"][a].cpu().numpy()
        scale = np.abs(g.E).max() / (g.kappa_rho * min(g.h)) * 1e-12
        assert np.all(np.abs(Fg - Fo) <= 1e-9 * np.abs(Fo) + scale), a
    plan.close()
