"""fld_step_aniso (diagonal-tensor D, one kappa rho per grid direction) against the
FP64 oracle.  The solve stops at the FP64 relative residual rtol = 1e-10 / q_b, so
||x - x*|| / ||x*|| <= 1e-10 (A is SPD with lambda_min >= 1); the face weights
carry only the rounding of D (exact to a few ulp with lambda = 1/3; the limiter's
sensitivity to R with the rational law)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import oracle as O                     # noqa: E402
import workloads as W                  # noqa: E402
import paper_2104_03968_amd as fld     # noqa: E402
from tests.gpu_common import dev, rel_l2   # noqa: E402
from tests.test_gpu_parity import face_tolerance   # noqa: E402


def opacities(g, seed):
    """Per-direction kappa rho: the grid's own along x, scaled by smooth factors of
    up to 10^{+-2} along the others."""
    out = [g.kappa_rho]
    for a in range(1, g.E.ndim):
        out.append(g.kappa_rho * 10.0 ** W.span(W.smooth_field(g.E.shape, seed + a), -2.0, 2.0))
    return out


def run(grids, krs, precision=0, limiter="lp", c=1.0, aniso=True):
    rt = min(1e-10 / O.q_b(g.E) for g in grids)
    plan = fld.Plan([g.E.shape for g in grids], h=[g.h for g in grids], precision=precision, rtol=rt,
                    limiter=fld.LIMITER_CODES[limiter], c=c)
    E = [dev(g.E) for g in grids]
    out = [torch.empty_like(e) for e in E]
    if aniso:
        K = [[dev(k) for k in kk] for kk in krs]
        rc, st = plan.step_aniso(E, K, out, [g.dt for g in grids], check=False)
    else:
        rc, st = plan.step(E, [dev(kk[0]) for kk in krs], out, [g.dt for g in grids], check=False)
    torch.cuda.synchronize()
    w = [[t.cpu().numpy() for t in plan.level_tensors(i, 0)["w"]] for i in range(len(grids))]
    res = [o.cpu().numpy() for o in out]
    plan.close()
    return rc, st, res, w


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("limiter", ["lp", "minerbo", "diffusion"])
def test_aniso_step_matches_oracle(limiter, precision):
    """A ragged 2D grid and a 3D grid in one batch."""
    gs = [W.random_grid((90, 131), 62000, dt=4e-3), W.random_grid((18, 21, 26), 62100, dt=4e-3)]
    krs = [opacities(g, 62200 + 10 * i) for i, g in enumerate(gs)]
    rc, st, xs, ws = run(gs, krs, precision=precision, limiter=limiter, c=1.5)
    assert rc == fld.FLD_OK
    for g, kr, x, w in zip(gs, krs, xs, ws):
        x_or, _ = O.diffusion_step_aniso(g.E, kr, g.dt, g.h, c=1.5, limiter=limiter)
        assert rel_l2(x, x_or) <= 1e-10 * 1.01
        w_or = O.face_weights_aniso(O.diffusion_tensor(g.E, kr, g.h, c=1.5, limiter=limiter), g.dt, g.h)
        for a in range(g.E.ndim):
            ga = W.GridInput(E=g.E, kappa_rho=kr[a], dt=g.dt, h=g.h)      # direction a's opacity
            tol = face_tolerance(ga, limiter)[a]
            assert np.all((w[a] == 0) == (w_or[a] == 0))
            err = np.abs(w[a] - w_or[a]) / np.where(w_or[a] == 0, 1.0, np.abs(w_or[a]))
            assert np.all(err <= tol), (a, limiter, (err / tol).max())


def test_equal_opacities_reproduce_the_isotropic_step_bitwise():
    gs = [W.random_grid((64, 80), 62300, dt=3e-3), W.random_grid((16, 20, 12), 62301, dt=3e-3)]
    krs = [[g.kappa_rho] * g.E.ndim for g in gs]
    ra, sa, xa, wa = run(gs, krs)
    rb, sb, xb, wb = run(gs, krs, aniso=False)
    assert ra == rb == fld.FLD_OK
    for i in range(len(gs)):
        assert np.array_equal(xa[i], xb[i]) and sa[i]["cycles"] == sb[i]["cycles"]
        for a in range(gs[i].E.ndim):
            assert np.array_equal(wa[i][a], wb[i][a])


def test_swapped_opacities_differ():
    g = W.random_grid((48, 64), 62400, dt=5e-3)
    kr = opacities(g, 62410)
    _, _, (xa,), _ = run([g], [kr])
    _, _, (xb,), _ = run([g], [kr[::-1]])
    assert rel_l2(xa, xb) > 1e-6


def test_aniso_errors():
    g = W.random_grid((32, 32), 62500, dt=1e-3)
    plan = fld.Plan([g.E.shape], h=[g.h])
    E = dev(g.E)
    out = torch.empty_like(E)
    kx = dev(g.kappa_rho)
    rc, _ = plan.step_aniso([E], [[kx, None]], [out], [1e-3], check=False)
    assert rc == fld.FLD_ERR_INVALID_ARG
    ky = dev(np.where(np.arange(32)[None, :] == 5, 0.0, g.kappa_rho))
    rc, _ = plan.step_aniso([E], [[kx, ky]], [out], [1e-3], check=False)
    assert rc == fld.FLD_ERR_BAD_INPUT
    plan.close()
