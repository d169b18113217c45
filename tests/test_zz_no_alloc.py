"""fld_step_noalloc (the step for callers that cannot allocate) through the C ABI: two
calls in a row, the second on a smaller grid, each bitwise equal to fld_step of the
same options on a bound workspace, and within 1e-10 of the oracle; the plan is left
unbound; too large a plan and a bound plan are refused."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import oracle as O                     # noqa: E402
import workloads as W                  # noqa: E402
import paper_2104_03968_amd as fld     # noqa: E402
from tests.gpu_common import dev, rel_l2   # noqa: E402


def _bound_step(g, opts):
    plan = fld.Plan([g.E.shape], h=[g.h], **opts)
    E, K = dev(g.E), dev(g.kappa_rho)
    out = torch.empty_like(E)
    rc, st = plan.step([E], [K], [out], [g.dt], check=False)
    torch.cuda.synchronize()
    plan.close()
    return rc, st, out.cpu().numpy()


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_step_equals_the_bound_step(precision):
    grids = [W.random_grid((20, 48, 40), 77000, dt=3e-3), W.random_grid((96, 130), 77100, dt=2e-3)]
    opts = dict(precision=precision, rtol=1e-10 / 1.7)
    for g in grids:                                    # the second call is on a smaller grid
        h = fld.fld_plan_create([fld.make_grid(tuple(reversed(g.E.shape)), g.h)], fld.fld_opts_default(**opts))
        assert fld.fld_plan_workspace_bytes(h) <= fld.FLD_NOALLOC_MAX_BYTES
        E, K = dev(g.E), dev(g.kappa_rho)
        out = torch.full_like(E, float("nan"))
        torch.cuda.synchronize()
        rc, st = fld.fld_step_noalloc(h, [E], [K], [out], [g.dt], stream=torch.cuda.current_stream(), check=False)
        torch.cuda.synchronize()
        assert rc == fld.FLD_OK, st
        x = out.cpu().numpy()
        rc2, st2, x2 = _bound_step(g, opts)
        assert rc2 == fld.FLD_OK
        assert np.array_equal(x, x2) and st[0]["cycles"] == st2[0]["cycles"], g.E.shape
        x_or, _ = O.diffusion_step(g.E, g.kappa_rho, g.dt, g.h)
        assert rel_l2(x, x_or) <= 1e-10, (g.E.shape, rel_l2(x, x_or))
        # the plan is left unbound
        with pytest.raises(fld.FLDError) as e:
            fld.fld_plan_tuning(h)
        assert e.value.code == fld.FLD_ERR_NO_WORKSPACE
        fld.fld_plan_destroy(h)


def test_noalloc_refuses_large_and_bound_plans():
    big = fld.fld_plan_create([fld.make_grid((128, 128, 128))], fld.fld_opts_default())
    assert fld.fld_plan_workspace_bytes(big) > fld.FLD_NOALLOC_MAX_BYTES
    E = torch.ones((128, 128, 128), dtype=torch.float64, device="cuda")
    rc, _ = fld.fld_step_noalloc(big, [E], [E], [E], [1e-3], check=False)
    assert rc == fld.FLD_ERR_TOO_LARGE
    fld.fld_plan_destroy(big)
    g = W.random_grid((32, 32), 77200, dt=1e-3)
    p = fld.Plan([g.E.shape], h=[g.h])
    E, K = dev(g.E), dev(g.kappa_rho)
    rc, _ = fld.fld_step_noalloc(p.handle, [E], [K], [E], [g.dt], check=False)
    assert rc == fld.FLD_ERR_INVALID_ARG
    p.close()
