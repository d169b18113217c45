"""Parity at the benchmark's full sizes, in the launch configuration the benchmark
times (autotuned launch shapes, full-multigrid start):

* 1024^2 FP64 with the gas exchange, three steps, each step's oracle fed the
  device's previous state (the per-step contract): E and eps within 1e-10 relative
  L2.  The device stops at rtol = 1e-10 / (2 q_b), so its solve is within 1e-10 / 2
  of x* (A is SPD with lambda_min >= 1 and zero flux conserves the mean); the
  oracle's CG is at the FP64 floor; the exchange maps both through the same
  per-cell root (1e-12 per cell).
* 256^3 with FP32 V-cycles in FP64 defect correction: the oracle's own FP64
  operator, built from E^n with its own face weights, applied to the device's
  result leaves a relative residual below 1e-10 (a property at any size, which
  bounds the error by q_b times it), and the energy is conserved to that residual.
* the 512-grid batch (FP64): sampled grids of the one batched step against the
  oracle's solve of each grid alone.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import oracle as O                     # noqa: E402
import workloads as W                  # noqa: E402
import paper_2104_03968_amd as fld     # noqa: E402
from tests.gpu_common import dev, rel_l2   # noqa: E402


def test_1024_squared_steps_with_exchange_per_step():
    g = W.c2_inputs(1024)
    rtol = 1e-10 / (2.0 * O.q_b(g.E))
    plan = fld.Plan([g.E.shape], h=[g.h], rtol=rtol, autotune=1, c=g.c)
    gas = fld.fld_gas_default(c=g.c, a_rad=g.a_r, c_v=g.c_v)
    E, eps, rho, kap, K = dev(g.E), dev(g.eps), dev(g.rho), dev(g.kappa), dev(g.kappa_rho)
    out = torch.empty_like(E)
    for step in range(3):
        E_n, eps_n = E.cpu().numpy(), eps.cpu().numpy()
        rc, (st,) = plan.step([E], [K], [out], [g.dt], check=False)
        assert rc == fld.FLD_OK, (step, st)
        E.copy_(out)
        plan.exchange([E], [eps], [rho], [kap], [g.dt], gas)
        torch.cuda.synchronize()
        assert O.q_b(E_n) < 2.0 * O.q_b(g.E)      # the stop rule above still bounds the error
        Eo, epso, info = O.fld_step(E_n, g.kappa_rho, g.dt, g.h, g.c,
                                    gas=dict(eps=eps_n, rho=g.rho, kappa=g.kappa, a_r=g.a_r, c_v=g.c_v))
        assert rel_l2(E.cpu().numpy(), Eo) <= 1e-10, (step, rel_l2(E.cpu().numpy(), Eo), st)
        assert rel_l2(eps.cpu().numpy(), epso) <= 1e-10, step
    plan.close()


def test_256_cubed_mixed_step_residual_certificate():
    g = W.c3_inputs(256)
    plan = fld.Plan([g.E.shape], h=[g.h], precision=fld.FLD_PREC_MIXED, rtol=1e-10, autotune=1, c=g.c)
    E, K = dev(g.E), dev(g.kappa_rho)
    out = torch.empty_like(E)
    rc, (st,) = plan.step([E], [K], [out], [g.dt], check=False)
    torch.cuda.synchronize()
    assert rc == fld.FLD_OK, st
    x = out.cpu().numpy()
    plan.close()
    D = O.diffusion_coefficient(g.E, g.kappa_rho, g.h, g.c)
    w = O.face_weights(D, g.dt, g.h)
    r = g.E - O.apply_operator(w, x)
    rel = np.linalg.norm(r) / np.linalg.norm(g.E)
    assert rel <= 1e-10 * (1 + 1e-3), (rel, st)
    assert abs(rel - st["rel_residual"]) <= 1e-3 * 1e-10 + 1e-3 * st["rel_residual"]
    assert abs(x.sum() - g.E.sum()) <= np.sqrt(g.E.size) * np.linalg.norm(r) + 1e-13 * g.E.sum()


def test_512_grid_batch_sampled_grids():
    """The 512-grid batch in one plan (FP64, autotuned): the smallest, the largest and two
    seeded grids of the batch against the oracle's solve of each alone."""
    grids = [W.c4_grid(j, n, dt) for j, (n, dt) in enumerate(W.c4_layout())]
    rtol = 1e-10 / max(O.q_b(g.E) for g in grids)
    plan = fld.Plan([g.E.shape for g in grids], h=[g.h for g in grids], rtol=rtol, autotune=1)
    E = [dev(g.E) for g in grids]
    K = [dev(g.kappa_rho) for g in grids]
    out = [torch.empty_like(e) for e in E]
    rc, st = plan.step(E, K, out, [g.dt for g in grids], check=False)
    torch.cuda.synchronize()
    assert rc == fld.FLD_OK
    sides = [g.E.shape[0] for g in grids]
    rng = np.random.default_rng(404)
    pick = {int(np.argmin(sides)), int(np.argmax(sides))} | set(int(i) for i in rng.choice(len(grids), 2, replace=False))
    for i in sorted(pick):
        g = grids[i]
        x_or, _ = O.diffusion_step(g.E, g.kappa_rho, g.dt, g.h)
        assert rel_l2(out[i].cpu().numpy(), x_or) <= 1e-10, (i, g.E.shape, st[i])
    plan.close()
