"""Parity at the benchmark's full sizes, in the launch configuration the benchmark
times (autotuned launch shapes, full-multigrid start):

* 1024^2 FP64 with the gas exchange, three steps, each step's oracle fed the
  device's previous state (the per-step contract): E and eps within 1e-10 relative
  L2.  The device stops at rtol = 1e-10 / (2 q_b), so its solve is within 1e-10 / 2
  of x* (A is SPD with lambda_min >= 1 and zero flux conserves the mean); the
  oracle's CG is at the FP64 floor; the exchange maps both through the same
  per-cell root (1e-12 per cell).
* 256^3 in FP64 and with FP32 V-cycles in FP64 defect correction, all five steps,
  each from the device's previous output: the oracle's own FP64 operator, built
  from E^n with its own face weights, applied to the device's result leaves a
  relative residual below tau = 1e-10 / (q_b n_steps) (a property at any size,
  which bounds the error against the oracle's step by q_b times it), and the
  energy is conserved to that residual.
* the 512-grid batch (FP64 and mixed): every grid certified the same way, sampled
  grids against the oracle's solve of each grid alone.
* the request server with requests at the served stream's largest sizes.
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


def certified_error(E_n, kappa_rho, dt, h, c, x):
    """Bound on the relative L2 error of x against the oracle's exact step from E_n.

    The oracle's own FP64 operator A (its face weights, from E_n) applied to x leaves
    r = E_n - A x.  A is SPD with lambda_min >= 1 and conserves the mean under zero
    flux, so ||x - x*|| <= ||r|| and ||x*|| >= |sum E_n| / sqrt(N): the relative error is
    at most q_b ||r|| / ||E_n||.  Returns (relative residual, error bound, |sum x - sum E_n|,
    ||r||)."""
    D = O.diffusion_coefficient(E_n, kappa_rho, h, c)
    w = O.face_weights(D, dt, h)
    r = E_n - O.apply_operator(w, x)
    rn = float(np.linalg.norm(r))
    rel = rn / float(np.linalg.norm(E_n))
    return rel, O.q_b(E_n) * rel, abs(float(x.sum()) - float(E_n.sum())), rn


@pytest.mark.parametrize("precision", [fld.FLD_PREC_FP64, fld.FLD_PREC_MIXED])
def test_256_cubed_five_steps_certified_against_the_oracle(precision):
    """The 256^3 workload over its five steps, each step's input the device's previous
    output, in the benchmark's launch configuration.  Each step stops at
    tau = 1e-10 / (q_b n_steps) and is certified under the oracle's own operator, so each
    step is within 1e-10 / n_steps of the oracle's step from the same input (the
    per-step contract) and the five-step trajectory within 1e-10 of the oracle's
    steps chained on the device's states."""
    nsteps = 5
    g = W.c3_inputs(256)
    qb0 = O.q_b(g.E)
    tau = 1e-10 / (1.05 * qb0 * nsteps)          # 5 % margin for q_b drifting over the steps
    plan = fld.Plan([g.E.shape], h=[g.h], precision=precision, rtol=tau, autotune=1, c=g.c)
    E, K = dev(g.E), dev(g.kappa_rho)
    out = torch.empty_like(E)
    total = 0.0
    for step in range(nsteps):
        E_n = E.cpu().numpy()
        rc, (st,) = plan.step([E], [K], [out], [g.dt], check=False)
        torch.cuda.synchronize()
        assert rc == fld.FLD_OK, (step, st)
        x = out.cpu().numpy()
        rel, bound, dsum, rn = certified_error(E_n, g.kappa_rho, g.dt, g.h, g.c, x)
        print(f"256^3 precision={precision} step {step}: cycles {st['cycles']} device rel_res "
              f"{st['rel_residual']:.3e} oracle-operator rel_res {rel:.3e} error vs oracle <= {bound:.3e}",
              flush=True)
        assert O.q_b(E_n) <= 1.05 * qb0
        assert rel <= tau * (1 + 1e-3), (step, rel, tau)
        assert bound <= 1e-10 / nsteps, (step, bound)
        # the device's residual is the oracle's residual of the same iterate
        assert abs(rel - st["rel_residual"]) <= 1e-3 * tau + 1e-3 * st["rel_residual"], (step, rel, st)
        assert dsum <= np.sqrt(x.size) * rn + 1e-13 * abs(float(E_n.sum())), step
        total += bound
        E.copy_(out)
    assert total <= 1e-10
    plan.close()


@pytest.mark.parametrize("precision", [fld.FLD_PREC_FP64, fld.FLD_PREC_MIXED])
def test_512_grid_batch_sampled_grids(precision):
    """The 512-grid batch in one plan (autotuned, FP64 and mixed): the smallest, the
    largest and four seeded grids of the batch against the oracle's solve of each
    alone, and every grid of the batch certified under the oracle's operator."""
    grids = [W.c4_grid(j, n, dt) for j, (n, dt) in enumerate(W.c4_layout())]
    rtol = 1e-10 / max(O.q_b(g.E) for g in grids)
    plan = fld.Plan([g.E.shape for g in grids], h=[g.h for g in grids], rtol=rtol, autotune=1,
                    precision=precision)
    E = [dev(g.E) for g in grids]
    K = [dev(g.kappa_rho) for g in grids]
    out = [torch.empty_like(e) for e in E]
    rc, st = plan.step(E, K, out, [g.dt for g in grids], check=False)
    torch.cuda.synchronize()
    assert rc == fld.FLD_OK
    xs = [o.cpu().numpy() for o in out]
    plan.close()
    for i, g in enumerate(grids):
        rel, bound, _, _ = certified_error(g.E, g.kappa_rho, g.dt, g.h, g.c, xs[i])
        assert bound <= 1e-10 * (1 + 1e-3), (i, g.E.shape, rel, st[i])
    sides = [g.E.shape[0] for g in grids]
    rng = np.random.default_rng(404)
    pick = {int(np.argmin(sides)), int(np.argmax(sides))} | set(int(i) for i in rng.choice(len(grids), 4, replace=False))
    for i in sorted(pick):
        g = grids[i]
        x_or, _ = O.diffusion_step(g.E, g.kappa_rho, g.dt, g.h)
        assert rel_l2(xs[i], x_or) <= 1e-10, (i, g.E.shape, st[i])


def test_server_takes_requests_at_the_streams_largest_sizes():
    """One 1024^2 and one 192^3 request (the largest sides of the served stream) through
    the server together with two small ones, mixed precision: each result certified under
    the oracle's operator, the 1024^2 one also against the oracle's solve."""
    shapes = [((1024, 1024), 6e-3), ((192, 192, 192), 4e-3), ((128, 128), 1e-3), ((32, 32, 32), 1e-2)]
    items = [W.random_grid(s, 5_100_000 + 10 * i, dt=dt) for i, (s, dt) in enumerate(shapes)]
    rtol = 1e-10 / max(O.q_b(g.E) for g in items)
    srv = fld.Server(8 << 30, precision=fld.FLD_PREC_MIXED, rtol=rtol)
    keep = [(dev(g.E), dev(g.kappa_rho)) for g in items]
    torch.cuda.synchronize()
    tickets = [srv.submit(E_, K_, g.dt, h=g.h) for (E_, K_), g in zip(keep, items)]
    xs = []
    for t, g in zip(tickets, items):
        rc, res = srv.wait(t, 300.0)
        assert rc == 0 and res.stats.status == 0, (g.E.shape, rc)
        xs.append(srv.result_tensor(res, g.E.shape).cpu().numpy().copy())
        assert srv.release(t) == 0
    srv.close()
    for g, x in zip(items, xs):
        rel, bound, _, _ = certified_error(g.E, g.kappa_rho, g.dt, g.h, g.c, x)
        assert bound <= 1e-10 * (1 + 1e-3), (g.E.shape, rel)
    x_or, _ = O.diffusion_step(items[0].E, items[0].kappa_rho, items[0].dt, items[0].h)
    assert rel_l2(xs[0], x_or) <= 1e-10
