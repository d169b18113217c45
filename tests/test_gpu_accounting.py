"""The algorithmic-byte accounting of a driver pass (fld_plan_cycle_bytes), which the
benchmark divides by the pass's measured time: it launches nothing, scales with the
word size of the multigrid arrays, and the outer iteration adds exactly the FP64
Krylov vectors to the multigrid V-cycle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_2104_03968_amd as fld     # noqa: E402


@pytest.mark.parametrize("shape", [(48, 64, 40), (96, 160)])
def test_cycle_bytes_word_size_and_krylov_part(shape):
    N = int(np.prod(shape))
    d = len(shape)
    res = {}
    for prec in (fld.FLD_PREC_FP64, fld.FLD_PREC_MIXED):
        p = fld.Plan([shape], precision=prec, fused=0)
        mg, n_mg = p.cycle_bytes(fld.FLD_CYCLE_MG)
        it, n_it = p.cycle_bytes(fld.FLD_CYCLE_ITERATION)
        fm, _ = p.cycle_bytes(fld.FLD_CYCLE_FMG)
        res[prec] = (mg, it, fm)
        assert n_it > n_mg > 0 and mg > 0 and fm > mg
        p.close()
    # every multigrid kernel moves words of the plan's multigrid precision; FP32 levels may
    # also start the LDS tail (which moves less than a swept level) one level higher
    mg64, mg32 = res[fld.FLD_PREC_FP64][0], res[fld.FLD_PREC_MIXED][0]
    if d == 3:
        assert mg32 == pytest.approx(0.5 * mg64, rel=1e-12)
    else:
        assert 0.3 * mg64 < mg32 <= 0.5 * mg64 * (1 + 1e-12)
    # CG part per level-0 cell: r.z (r, z), p/q (z, p_old, d faces; p, q), update (X, p, R, q; X, R, next rhs)
    z64, z32 = 8.0, 4.0
    for prec, z in ((fld.FLD_PREC_FP64, z64), (fld.FLD_PREC_MIXED, z32)):
        mg, it, _ = res[prec]
        cg = (8 + z) + (z + 8 + 8 * d + 16) + (32 + 16 + 8)
        assert it - mg == pytest.approx(cg * N, rel=1e-12), prec


def test_fused_levels_move_fewer_bytes_than_per_colour_sweeps():
    shape = (64, 64, 64)
    a = fld.Plan([shape], fused3_levels=9)
    b = fld.Plan([shape], fused=0)
    assert a.tuning()["fused3_levels"] >= 1
    assert a.cycle_bytes(fld.FLD_CYCLE_MG)[0] < b.cycle_bytes(fld.FLD_CYCLE_MG)[0]
    a.close()
    b.close()
