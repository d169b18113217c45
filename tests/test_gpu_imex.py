"""The radiation-only IMEX step on the GPU (fld_imex_step) against the FP64 oracle.

Bound per cell: the implicit stage is solved to a relative residual r (FP64
residual in both precisions); A = I + dt L is symmetric with rows summing to 1 and
a non-positive off-diagonal, so ||A^-1||_2 <= 1 and ||A^-1||_inf <= 1, and the
solve's error in every cell is at most r ||b||_2 (b the stage input).  The
midpoint scheme doubles it (E_x = E + 2 (E_m - E_+)); the exchange maps an error
in E to errors in E and eps no larger (the map is monotone in E with E + eps
fixed); the pointwise stages add rounding (the exchange root is within a few ulp
of (E + eps)).  The bound below takes 8 r ||b||_2 + 1e-11 (E + eps)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import oracle as O                     # noqa: E402
import workloads as W                  # noqa: E402
import paper_2104_03968_amd as fld     # noqa: E402
from tests.gpu_common import dev       # noqa: E402

A_R, C_V = 0.9, 1.3


def gas_grid(shape, seed, with_v):
    """Seeded E, kappa rho as for the diffusion tests; rho log-uniform in [10^-0.5,
    10^0.5], kappa = (kappa rho)/rho; a gas temperature within half a decade of
    the radiation temperature; a smooth velocity of order 1."""
    g = W.random_grid(shape, seed, dt=1e-3)
    rho = 10.0 ** W.span(W.smooth_field(shape, seed + 11), -0.5, 0.5)
    kappa = g.kappa_rho / rho
    T = (g.E / A_R) ** 0.25 * 10.0 ** W.span(W.smooth_field(shape, seed + 12), -0.5, 0.5)
    eps = rho * C_V * T
    v = [W.smooth_field(shape, seed + 20 + a) * (1.0 + 0.5 * a) for a in range(len(shape))] if with_v else None
    return dict(E=g.E, eps=eps, rho=rho, kappa=kappa, h=g.h, dt=g.dt, v=v)


def run_gpu(gs, scheme, precision=0, rtol=1e-12, c=1.0, limiter="lp"):
    plan = fld.Plan([g["E"].shape for g in gs], h=[g["h"] for g in gs], precision=precision, rtol=rtol,
                    c=c, limiter=fld.LIMITER_CODES[limiter])
    E = [dev(g["E"]) for g in gs]
    eps = [dev(g["eps"]) for g in gs]
    rho = [dev(g["rho"]) for g in gs]
    kap = [dev(g["kappa"]) for g in gs]
    v = [[dev(a) for a in g["v"]] if g["v"] is not None else None for g in gs]
    gas = fld.fld_gas_default(c=c, a_rad=A_R, c_v=C_V)
    rc, stats = plan.imex_step(E, eps, rho, kap, [g["dt"] for g in gs], gas=gas, scheme=scheme,
                               v=v if any(x is not None for x in v) else None, check=False)
    torch.cuda.synchronize()
    out = [(e.cpu().numpy(), s.cpu().numpy()) for e, s in zip(E, eps)]
    plan.close()
    return rc, stats, out


def oracle(g, scheme, c=1.0, limiter="lp"):
    return O.imex_step(g["E"], g["eps"], g["rho"], g["kappa"], g["dt"], g["h"], c=c, a_r=A_R, c_v=C_V,
                       limiter=limiter, scheme=scheme, v=g["v"])


def check(g, st, got, want):
    Eg, eg = got
    Eo, eo = want
    bound = 8 * (st["rel_residual"] + 1e-13) * st["b_norm"] + 1e-11 * (g["E"] + g["eps"])
    assert st["status"] == 0
    assert np.all(np.abs(Eg - Eo) <= bound), np.max(np.abs(Eg - Eo) / bound)
    assert np.all(np.abs(eg - eo) <= bound), np.max(np.abs(eg - eo) / bound)
    assert np.linalg.norm(Eg - Eo) <= 1e-10 * np.linalg.norm(Eo)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("with_v", [False, True])
@pytest.mark.parametrize("scheme", ["euler", "midpoint"])
def test_imex_matches_oracle(scheme, with_v, precision):
    """A 2D grid with a ragged tail and a 3D grid in one batch."""
    gs = [gas_grid((96, 130), 98000, with_v), gas_grid((17, 20, 23), 98100, with_v)]
    rc, stats, out = run_gpu(gs, scheme, precision=precision)
    assert rc == fld.FLD_OK
    for g, st, got in zip(gs, stats, out):
        check(g, st, got, oracle(g, scheme))


@pytest.mark.parametrize("limiter", ["minerbo", "lp_exact"])
def test_imex_limiters_and_c(limiter):
    """The other physical limiters with c != 1.  (lambda = 1/3 is left out: in thin
    cells it gives f = 1/3 + R^2/9 > 1 and an unbounded tiring source.)"""
    g = gas_grid((64, 80), 98200, True)
    rc, stats, out = run_gpu([g], "midpoint", c=2.5, limiter=limiter)
    assert rc == fld.FLD_OK
    check(g, stats[0], out[0], oracle(g, "midpoint", c=2.5, limiter=limiter))


@pytest.mark.parametrize("scheme", ["euler", "midpoint"])
def test_imex_conserves_total_energy(scheme):
    """Without a velocity, zero flux and the exchange keep sum(E + eps): the solve's
    residual r changes sum(E) by at most sqrt(N) r ||b||_2."""
    g = gas_grid((200, 168), 98300, False)
    rc, stats, out = run_gpu([g], scheme)
    assert rc == fld.FLD_OK
    E1, e1 = out[0]
    tot0 = (g["E"] + g["eps"]).sum()
    slack = 2 * np.sqrt(g["E"].size) * (stats[0]["rel_residual"] + 1e-13) * stats[0]["b_norm"]
    assert abs((E1 + e1).sum() - tot0) <= slack + 1e-12 * tot0
    assert np.all(E1 > 0) and np.all(e1 > 0)


def test_imex_equilibrium_is_a_fixed_point():
    shape = (40, 48)
    T = 1.7
    rho = np.full(shape, 2.0)
    g = dict(E=np.full(shape, A_R * T ** 4), eps=rho * C_V * T, rho=rho, kappa=np.full(shape, 3.0),
             h=(1 / 48, 1 / 40), dt=0.1, v=None)
    for scheme in ("euler", "midpoint"):
        rc, _, out = run_gpu([g], scheme)
        assert rc == fld.FLD_OK
        assert np.allclose(out[0][0], g["E"], rtol=1e-12) and np.allclose(out[0][1], g["eps"], rtol=1e-12)


def test_imex_full_size_2d_conservation():
    """1024^2 cells (the 2D benchmark grid): total energy kept, outputs positive."""
    g = W.c2_inputs(1024)
    d = dict(E=g.E, eps=g.eps, rho=g.rho, kappa=g.kappa, h=g.h, dt=g.dt, v=None)
    rc, stats, out = run_gpu([d], "midpoint", precision=1, rtol=1e-10)
    assert rc == fld.FLD_OK
    E1, e1 = out[0]
    tot0 = (g.E + g.eps).sum()
    slack = 2 * np.sqrt(g.E.size) * (stats[0]["rel_residual"] + 1e-13) * stats[0]["b_norm"]
    assert abs((E1 + e1).sum() - tot0) <= slack + 1e-12 * tot0
    assert np.all(E1 > 0) and np.all(e1 > 0)
    # sampled cells: away from steep gradients the step changes E by little
    assert np.all(np.isfinite(E1)) and np.all(np.isfinite(e1))


def test_imex_argument_errors():
    g = gas_grid((32, 32), 98400, True)
    plan = fld.Plan([g["E"].shape], h=[g["h"]])
    E, eps, rho, kap = dev(g["E"]), dev(g["eps"]), dev(g["rho"]), dev(g["kappa"])
    vx, vy = dev(g["v"][0]), dev(g["v"][1])
    gas = fld.fld_gas_default(c=1.0)
    need = fld.fld_imex_scratch_bytes(plan.handle, fld.FLD_IMEX_MIDPOINT)
    buf = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    base = buf.data_ptr()
    base += (-base) % 256

    def call(**kw):
        a = dict(E=[E], eps=[eps], v=None, scheme=fld.FLD_IMEX_MIDPOINT, scratch=base, nbytes=need, gas=gas)
        a.update(kw)
        rc, _ = fld.fld_imex_step(plan.handle, a["E"], a["eps"], [rho], [kap], [1e-3], a["gas"], a["scheme"],
                                  a["scratch"], a["nbytes"], v=a["v"], check=False)
        return rc

    assert call(nbytes=need - 8) == fld.FLD_ERR_INVALID_ARG            # scratch too small
    assert call(scratch=base + 8) == fld.FLD_ERR_INVALID_ARG           # misaligned
    assert call(eps=[E]) == fld.FLD_ERR_INVALID_ARG                    # E aliasing eps
    assert call(v=[[vx, None]]) == fld.FLD_ERR_INVALID_ARG             # partial velocity
    assert call(scheme=5) == fld.FLD_ERR_INVALID_ARG
    assert call(gas=fld.fld_gas_default(c=3.0)) == fld.FLD_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert np.array_equal(E.cpu().numpy(), g["E"]) and np.array_equal(eps.cpu().numpy(), g["eps"])
    assert call(v=[[vx, vy]]) == fld.FLD_OK
    plan.close()


def test_imex_flags_invalid_cells():
    g = gas_grid((32, 40), 98500, False)
    g["rho"][5, 7] = -1.0
    rc, _, out = run_gpu([g], "euler")
    assert rc == fld.FLD_ERR_BAD_INPUT
