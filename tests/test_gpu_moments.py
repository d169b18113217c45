"""Radiation moments on the GPU (fld_radiation_moments) against the FP64 oracle.

Both sides evaluate the same formulas in FP64 with a different operation order,
so the bound per cell comes from the magnitudes that enter each result: the
gradient's stencil sum S_d = (|E_-2| + 8 |E_-1| + 8 |E_+1| + |E_+2|) / (12 h_d)
(cancellation in the 4th-order difference), |P_ij| <= E, and f in [1/3, 1]."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2104_03968_amd as fld
import workloads as W
from tests.gpu_common import dev

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def stencil_scale(A, h):
    """Per axis (x first): sum of |terms| of the 4th-order gradient of A, over 12 h."""
    nd = A.ndim
    P = np.pad(np.abs(A), 2, mode="symmetric")
    out = []
    for d in range(nd):
        ax = nd - 1 - d

        def sh(k):
            sl = [slice(2, 2 + s) for s in A.shape]
            sl[ax] = slice(2 + k, 2 + k + A.shape[ax])
            return P[tuple(sl)]
        out.append((sh(-2) + 8 * sh(-1) + 8 * sh(1) + sh(2)) / (12 * h[d]))
    return out


def velocity(shape, seed):
    return [W.smooth_field(shape, seed + a) * (1.0 + a) for a in range(len(shape))]


def run(grids, c=1.0, limiter="lp", with_v=True, dt=1e-3):
    plan = fld.Plan([g.E.shape for g in grids], h=[g.h for g in grids], c=c, limiter=fld.LIMITER_CODES[limiter])
    E = [dev(g.E) for g in grids]
    K = [dev(g.kappa_rho) for g in grids]
    vs = [[dev(a) for a in velocity(g.E.shape, 777 + i)] for i, g in enumerate(grids)] if with_v else None
    want = ("F", "f_r", "edd", "P") + (("tiring", "E_out") if with_v else ())
    outs = plan.radiation_moments(E, K, v=vs, dt=[dt] * len(grids) if with_v else None, want=want)
    torch.cuda.synchronize()
    res = [{k: ([t.cpu().numpy() for t in v] if isinstance(v, list) else v.cpu().numpy()) for k, v in o.items()}
           for o in outs]
    plan.close()
    return res


def check(g, got, c, lim, with_v, dt=1e-3):
    v = velocity(g.E.shape, 777 + check.index) if with_v else None
    m = O.radiation_moments(g.E, g.kappa_rho, g.h, c=c, limiter=lim, v=v, dt=dt)
    S = stencil_scale(g.E, g.h)
    gnorm = np.sqrt(sum(gi * gi for gi in O.gradient4(g.E, g.h)))
    Ssum = sum(S) + gnorm
    lam_max = 1.0 / 3.0
    extra = 1000 * EPS if lim == "lp_exact" else 0.0      # cancellation in coth R - 1/R
    for a in range(g.E.ndim):
        tolF = 64 * EPS * (c * lam_max / g.kappa_rho * Ssum + np.abs(m["F"][a])) + extra * np.abs(m["F"][a])
        assert np.all(np.abs(got["F"][a] - m["F"][a]) <= tolF), a
        tolr = 64 * EPS * (lam_max * Ssum + np.abs(m["f_r"][a])) + extra * np.abs(m["f_r"][a])
        assert np.all(np.abs(got["f_r"][a] - m["f_r"][a]) <= tolr), a
    # f and P: R carries the gradient's absolute error; f is flat in R at R = 0
    relR = 64 * EPS * (Ssum / np.maximum(gnorm, 1e-300)) + extra
    tolf = 64 * EPS + extra + np.minimum(relR, 1.0) * np.abs(m["f"] - 1.0 / 3.0) * 2
    assert np.all(np.abs(got["edd"] - m["f"]) <= tolf)
    for q in range(len(m["P"])):
        assert np.all(np.abs(got["P"][q] - m["P"][q]) <= 64 * EPS * g.E + tolf * g.E), q
    if with_v:
        Sv = [stencil_scale(vi, g.h) for vi in v]
        bound = g.E * sum(sum(s) for s in Sv)
        assert np.all(np.abs(got["tiring"] - m["tiring"]) <= 256 * EPS * bound + np.max(tolf) * bound)
        assert np.all(np.abs(got["E_out"] - m["E_new"]) <= 64 * EPS * np.abs(g.E) + dt * (256 * EPS + np.max(tolf)) * bound)


@pytest.mark.parametrize("limiter", ["lp", "diffusion", "minerbo", "lp_exact"])
@pytest.mark.parametrize("shape", [(96, 130), (37, 50), (24, 40, 32), (17, 20, 23)])
def test_moments_match_oracle(shape, limiter):
    g = W.random_grid(shape, 97000 + sum(shape), dt=1e-3)
    c = 2.0
    (got,) = run([g], c=c, limiter=limiter)
    check.index = 0
    check(g, got, c, limiter, True)


def test_batched_2d_3d_equals_alone():
    gs = [W.random_grid((64, 48), 97100, dt=1e-3), W.random_grid((20, 16, 24), 97101, dt=1e-3)]
    both = run(gs)
    for i, g in enumerate(gs):
        (alone,) = run([g])
        # velocity seeds follow the batch index: compare the v-free outputs bitwise
        for k in ("F", "f_r", "P"):
            for x, y in zip(both[i][k], alone[k]):
                assert np.array_equal(x, y), (i, k)
        assert np.array_equal(both[i]["edd"], alone["edd"])


def test_free_streaming_flux_is_causal():
    n = 128
    x = (np.arange(n) + 0.5) / n
    E = np.tile(1.0 + 1e6 * np.exp(-((x - 0.5) / 0.05) ** 2), (16, 1))
    g = W.GridInput(E=E, kappa_rho=np.full_like(E, 1e-9), dt=1e-3, h=(1 / n, 1 / 16))
    (got,) = run([g], c=3.0, with_v=False)
    Fmag = np.sqrt(got["F"][0] ** 2 + got["F"][1] ** 2)
    assert np.all(Fmag <= 3.0 * E * (1 + 1e-12))
    assert Fmag.max() / (3.0 * E[np.unravel_index(np.argmax(Fmag), E.shape)]) > 0.999
    assert np.all(got["edd"] <= 1 + 1e-12) and np.all(got["edd"] >= 1 / 3 - 1e-15)


def test_argument_errors():
    g = W.random_grid((32, 32), 97200, dt=1e-3)
    plan = fld.Plan([g.E.shape], h=[g.h])
    E, K = [dev(g.E)], [dev(g.kappa_rho)]
    vx = dev(g.E)
    out = torch.empty_like(E[0])
    # tiring without a velocity; E_out aliasing E; a partial velocity
    with pytest.raises(fld.FLDError) as e:
        fld.fld_radiation_moments(plan.handle, E, K, [{"tiring": out}])
    assert e.value.code == fld.FLD_ERR_INVALID_ARG
    with pytest.raises(fld.FLDError) as e:
        fld.fld_radiation_moments(plan.handle, E, K, [{"E_out": E[0]}], v=[[vx, vx]], dt=[1e-3])
    assert e.value.code == fld.FLD_ERR_INVALID_ARG
    with pytest.raises(fld.FLDError) as e:
        fld.fld_radiation_moments(plan.handle, E, K, [{"tiring": out}], v=[[vx, None]])
    assert e.value.code == fld.FLD_ERR_INVALID_ARG
    plan.close()
