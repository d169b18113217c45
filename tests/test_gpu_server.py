"""GPU tests of the request server: results against the oracle, the same result
alone and in a mix (bitwise), admission under a small arena, and rejections."""
import threading
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import oracle as O                     # noqa: E402
import workloads as W                  # noqa: E402
import paper_2104_03968_amd as fld     # noqa: E402
from tests.gpu_common import dev, rel_l2   # noqa: E402

MIX = [((64, 64), 4e-3), ((96, 160), 1e-2), ((24, 24, 24), 5e-3), ((128, 128), 1e-4), ((40, 32, 48), 8e-3),
       ((288, 288), 9e-3), ((37, 100), 2e-3), ((32, 32, 32), 1e-2)]


def _inputs(i, shape, dt):
    return W.random_grid(shape, 7_000_000 + 10 * i, dt=dt)


def _run(server, items, on_device=True):
    tickets = []
    for g in items:
        if on_device:
            # device inputs are read at admission: keep them alive until the request is done
            keep = (dev(g.E), dev(g.kappa_rho))
            tickets.append((server.submit(keep[0], keep[1], g.dt, h=g.h, on_device=True), keep))
        else:
            E = np.ascontiguousarray(g.E)
            K = np.ascontiguousarray(g.kappa_rho)
            tickets.append((server.submit(E, K, g.dt, h=g.h, on_device=False), None))
    out = []
    for (t, _), g in zip(tickets, items):
        rc, res = server.wait(t, 120.0)
        assert rc == 0, (rc, res.stats.status)
        x = server.result_tensor(res, g.E.shape).cpu().numpy().copy()
        out.append((x, res))
        assert server.release(t) == 0
    return out


@pytest.mark.parametrize("precision", [1, 0])
def test_server_results_match_oracle(precision):
    items = [_inputs(i, s, dt) for i, (s, dt) in enumerate(MIX)]
    srv = fld.Server(1 << 30, precision=precision, rtol=2e-11)
    res = _run(srv, items)
    for g, (x, r) in zip(items, res):
        x_or, _ = O.diffusion_step(g.E, g.kappa_rho, g.dt, g.h)
        assert rel_l2(x, x_or) <= 2e-11 * O.q_b(g.E) * 1.01, g.E.shape
        assert r.t_submit <= r.t_admit <= r.t_start <= r.t_done
        assert r.stats.status == 0 and r.stats.rel_residual <= 2e-11
    info = srv.info()
    assert info["completed"] == len(items) and info["failed"] == 0 and info["error"] == 0
    assert info["arena_free"] == info["arena_bytes"] - (info["arena_bytes"] - info["arena_free"])
    srv.close()


def test_result_is_the_same_alone_and_in_a_mix():
    items = [_inputs(i, s, dt) for i, (s, dt) in enumerate(MIX)]
    srv = fld.Server(1 << 30)
    alone = []
    for g in items:                                   # one at a time
        alone.append(_run(srv, [g])[0][0])
    mixed = _run(srv, items)                          # all at once
    for a, (m, _) in zip(alone, mixed):
        assert np.array_equal(a, m)
    # and the same as one fld_step of the grid alone with the same options
    for g, a in zip(items[:3], alone[:3]):
        plan = fld.Plan([g.E.shape], h=[g.h], precision=1, use_graph=0, fmg=0)   # servers run V-cycles only
        E = dev(g.E)
        out = torch.empty_like(E)
        plan.step([E], [dev(g.kappa_rho)], [out], [g.dt])
        assert np.array_equal(out.cpu().numpy(), a)
        plan.close()
    srv.close()


def test_host_and_device_inputs_agree():
    items = [_inputs(i, s, dt) for i, (s, dt) in enumerate(MIX[:4])]
    srv = fld.Server(1 << 29)
    a = _run(srv, items, on_device=True)
    b = _run(srv, items, on_device=False)
    for (x, _), (y, _) in zip(a, b):
        assert np.array_equal(x, y)
    srv.close()


def test_admission_waits_for_arena_space():
    """An arena that holds about two of these requests at a time still completes all of
    them, in arrival order of admission, and never holds more than fits."""
    items = [_inputs(100 + i, (256, 256), 5e-3) for i in range(6)]
    srv = fld.Server(24 << 20, max_slots=8)           # ~2 x (plan + inputs + result) of 256^2
    peak = [0]
    stop = [False]

    def watch():
        while not stop[0]:
            peak[0] = max(peak[0], srv.info()["resident"])
            time.sleep(0.0005)

    th = threading.Thread(target=watch)
    th.start()
    keep = [(dev(g.E), dev(g.kappa_rho)) for g in items]
    tickets = [srv.submit(E, K, g.dt, h=g.h) for (E, K), g in zip(keep, items)]
    results = []
    for t, g in zip(tickets, items):
        rc, res = srv.wait(t, 120.0)
        assert rc == 0
        results.append(res)
        srv.release(t)
    stop[0] = True
    th.join()
    admits = [r.t_admit for r in results]
    assert admits == sorted(admits)                   # FIFO admission
    assert 1 <= peak[0] <= 3
    for g, r in zip(items, results):
        assert r.stats.status == 0
    srv.close()


def test_rejections_and_tickets():
    srv = fld.Server(8 << 20)
    big = W.random_grid((512, 512), 1, dt=1e-3)
    with pytest.raises(fld.FLDError) as e:
        srv.submit(dev(big.E), dev(big.kappa_rho), big.dt)
    assert e.value.code == fld.FLD_ERR_TOO_LARGE
    rc, _ = srv.poll(123456)
    assert rc == fld.FLD_ERR_UNKNOWN_TICKET
    g = _inputs(5, (64, 64), 1e-3)
    g.E[3, 3] = -1.0                                  # rejected by the device checks
    E, K = dev(g.E), dev(g.kappa_rho)
    t = srv.submit(E, K, g.dt, h=g.h)
    rc, res = srv.wait(t, 60.0)
    assert rc == fld.FLD_ERR_BAD_INPUT
    assert srv.release(t) == 0 and srv.release(t) == fld.FLD_ERR_UNKNOWN_TICKET
    srv.close()


def test_device_inputs_are_read_after_their_producer_stream():
    """Inputs still being written on another stream when they are submitted: the server's
    copy waits for the work enqueued on that stream before fld_submit, so the request sees
    the final values (zeros would be rejected as bad input)."""
    g = _inputs(31, (96, 128), 3e-3)
    ref = _run(fld.Server(1 << 28), [g])[0][0]
    side = torch.cuda.Stream()
    E = torch.zeros(g.E.shape, dtype=torch.float64, device="cuda")
    K = torch.zeros(g.E.shape, dtype=torch.float64, device="cuda")
    src_E, src_K = dev(g.E), dev(g.kappa_rho)
    torch.cuda.synchronize()
    big = torch.ones((4096, 4096), dtype=torch.float32, device="cuda")
    srv = fld.Server(1 << 28)
    with torch.cuda.stream(side):
        for _ in range(8):                      # keep the producer stream busy for a while
            big = torch.mm(big, big) * 1e-4
        E.copy_(src_E)
        K.copy_(src_K)
        t = srv.submit(E, K, g.dt, h=g.h, stream=side)
    rc, res = srv.wait(t, 120.0)
    assert rc == 0, rc
    x = srv.result_tensor(res, g.E.shape).cpu().numpy()
    assert np.array_equal(x, ref)
    assert srv.release(t) == 0
    srv.close()


@pytest.mark.parametrize("cycles_per_round", [1, 2])
@pytest.mark.parametrize("order", [(3, 1), (0, 1), (3, 0, 1)])
def test_a_grid_keeps_converging_when_earlier_grids_leave(order, cycles_per_round):
    """The grids admitted first finish first; the rebuilt composite then holds the
    remaining grid at a lower index while its solver state stays in the same slot.
    Every kernel must find that state (and the per-grid work of the fused tiles)
    through the slot, so the result is bitwise the one the grid gets alone."""
    items = [_inputs(i, MIX[i][0], MIX[i][1]) for i in order]
    srv = fld.Server(1 << 30, precision=1, rtol=2e-11, cycles_per_round=cycles_per_round)
    alone = _run(srv, [items[-1]])[0][0]
    mixed = _run(srv, items)
    assert srv.info()["failed"] == 0
    assert np.array_equal(mixed[-1][0], alone)
    assert mixed[-1][1].stats.cycles > max(r.stats.cycles for _, r in mixed[:-1])
    srv.close()
