"""Fixed-gradient (Neumann) boundaries on the device against the FP64 oracle.

With the face fluxes in b, A = I + dt L is unchanged (symmetric, unit column
sums, lambda_min >= 1), so a solve to relative residual r <= 1e-10 / q_b(b) is
within 1e-10 of x* in relative 2-norm, as for zero flux."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import oracle as O                     # noqa: E402
import workloads as W                  # noqa: E402
import paper_2104_03968_amd as fld     # noqa: E402
from tests.gpu_common import dev, rel_l2   # noqa: E402

EPS = np.finfo(np.float64).eps


def run(grids, grad, precision=0, limiter="lp", c=1.0, rtol=None):
    nd = max(g.E.ndim for g in grids)
    bc = [fld.FLD_BC_FIXED_GRADIENT if (v is not None) else fld.FLD_BC_ZERO_FLUX for v in grad]
    bg = [0.0 if v is None else v for v in grad]
    plan = fld.Plan([g.E.shape for g in grids], h=[g.h for g in grids], precision=precision,
                    rtol=rtol or 1e-10, limiter=fld.LIMITER_CODES[limiter], c=c, bc=bc, bc_grad=bg)
    E = [dev(g.E) for g in grids]
    K = [dev(g.kappa_rho) for g in grids]
    out = [torch.empty_like(e) for e in E]
    rc, st = plan.step(E, K, out, [g.dt for g in grids], check=False)
    torch.cuda.synchronize()
    res = [o.cpu().numpy() for o in out]
    return plan, rc, st, res


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("limiter", ["lp", "diffusion"])
def test_fixed_gradient_step_matches_oracle(limiter, precision):
    """Every face of a ragged 2D grid and a 3D grid prescribes a gradient (one face left
    at zero flux)."""
    grad = [0.8, -1.3, None, 2.1, -0.6, 0.4]
    gs = [W.random_grid((70, 93), 64000, dt=4e-3), W.random_grid((14, 18, 22), 64100, dt=4e-3)]
    refs = [O.diffusion_step_bc(g.E, g.kappa_rho, g.dt, g.h, grad_bc=grad[:2 * g.E.ndim], c=1.2, limiter=limiter)
            for g in gs]
    rt = min(1e-10 / O.q_b(info.extra["b"]) for _, info in refs)
    plan, rc, st, xs = run(gs, grad, precision=precision, limiter=limiter, c=1.2, rtol=rt)
    assert rc == fld.FLD_OK
    for (x_or, info), x, s in zip(refs, xs, st):
        assert rel_l2(x, x_or) <= 1e-10 * 1.01
        b = info.extra["b"]
        assert s["b_sum"] == pytest.approx(b.sum(), rel=1e-12)        # the boundary source is in b
    plan.close()


def test_linear_profile_is_steady_on_device():
    nx, ny = 128, 24
    h = (1.0 / nx, 0.5 / ny)
    G = 3.0
    X = (np.arange(nx) + 0.5) * h[0]
    E = np.tile(5.0 + G * X, (ny, 1))
    g = W.GridInput(E=E, kappa_rho=np.full(E.shape, 2.0), dt=0.05, h=h)
    plan, rc, (st,), (x,) = run([g], [G, G, None, None, None, None], limiter="diffusion", rtol=1e-12)
    assert rc == fld.FLD_OK
    assert np.abs(x - E).max() <= 8 * (st["rel_residual"] + 1e-14) * st["b_norm"]
    plan.close()


def test_energy_budget_on_device():
    g = W.random_grid((96, 80), 64200, dt=5e-3)
    grad = [0.4, 0.9, -0.2, 1.5, None, None]
    x_or, info = O.diffusion_step_bc(g.E, g.kappa_rho, g.dt, g.h, grad_bc=grad[:4])
    plan, rc, (st,), (x,) = run([g], grad, rtol=1e-12)
    assert rc == fld.FLD_OK
    src = info.extra["b"] - g.E
    slack = np.sqrt(g.E.size) * (st["rel_residual"] + 1e-14) * st["b_norm"]
    assert abs((x.sum() - g.E.sum()) - src.sum()) <= slack + 1e-12 * g.E.sum()
    plan.close()


def test_moments_use_the_boundary_ghosts():
    """The flux of fld_radiation_moments takes the same ghosts: F = -c lambda / (kappa rho)
    grad E with the fixed-gradient ghost rule at the walls."""
    g = W.random_grid((40, 52), 64300, dt=1e-3)
    grad = [1.5, -0.5, 0.7, 2.0, None, None]
    plan, rc, _, _ = run([g], grad)
    (out,) = plan.radiation_moments([dev(g.E)], [dev(g.kappa_rho)], want=("F",))
    torch.cuda.synchronize()
    gr = O.gradient4_bc(g.E, g.h, grad[:4])
    gn = np.sqrt(sum(x * x for x in gr))
    lam = O.flux_limiter(gn / (g.kappa_rho * g.E))
    for a in range(2):
        Fo = -lam / g.kappa_rho * gr[a]
        Fg = out["F"][a].cpu().numpy()
        scale = np.abs(g.E).max() / (g.kappa_rho * min(g.h)) * 1e-12
        assert np.all(np.abs(Fg - Fo) <= 1e-9 * np.abs(Fo) + scale), a
    plan.close()
