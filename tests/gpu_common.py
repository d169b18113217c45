"""Shared helpers for the GPU tests: move seeded inputs to the device, run the
library through the C ABI, and bring results back as numpy arrays."""
import numpy as np
import torch

import paper_2104_03968_amd as fld


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def run_step(grids, precision=0, rtol=1e-10, limiter="lp", c=1.0, max_cycles=50, use_graph=1,
             in_place=False, **kw):
    """One fld_step over a list of GridInput (same limiter and c); returns (xs, stats, rc)."""
    plan = fld.Plan([g.E.shape for g in grids], h=[g.h for g in grids], precision=precision,
                    rtol=rtol, limiter=fld.LIMITER_CODES[limiter], c=c, max_cycles=max_cycles,
                    use_graph=use_graph, **kw)
    E = [dev(g.E) for g in grids]
    K = [dev(g.kappa_rho) for g in grids]
    out = E if in_place else [torch.empty_like(e) for e in E]
    rc, stats = plan.step(E, K, out, [g.dt for g in grids], check=False)
    torch.cuda.synchronize()
    xs = [o.cpu().numpy() for o in out]
    plan.close()
    return xs, stats, rc


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))
