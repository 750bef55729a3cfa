"""GPU tests of the serving runtime (continuous batching on one GPU).

* every result is the same alone (one slot, one request at a time) and in a
  mix of concurrent requests with uneven channel counts, lags, orders and
  precisions (bit for bit: kernels are deterministic and a request's work
  stays on its slot), and equal to a plain context's identification;
* admission keeps the device memory the slots hold within the budget, so a
  budget for two requests caps the requests running at once at two;
* a request queued behind others reports busy until it has run;
* invalid requests and requests larger than the budget are refused at submit.
"""
import dataclasses

import numpy as np
import pytest

from paper_2411_05510_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _mix():
    """Six windows of different structures."""
    from paper_2411_05510_amd import ssicov
    out = []
    specs = [(24, 6, (12,), ssicov.PREC_FP32), (60, 10, (12, 20), ssicov.PREC_FP32),
             (120, 8, (10,), ssicov.PREC_BF16), (36, 12, (16, 24), ssicov.PREC_BF16X3),
             (60, 8, (20,), ssicov.PREC_FP32), (90, 14, (12,), ssicov.PREC_BF16)]
    for i, (l, modes, lags, prec) in enumerate(specs):
        rank = 2 * modes + 20
        wl = synth.Workload(name=f"req{i}", l=l, n=20000, fs=100.0, n_modes=modes,
                            f_range=(0.5, 20.0), zeta_range=(0.005, 0.03), noise=0.05,
                            lags=lags, svd="randomized", rank=rank, oversample=20,
                            power_iters=2, order_min=2, order_max=rank, order_step=2,
                            struct_seed=500 + i, noise_seed=600 + i, sketch_seed=700 + i)
        _, y = synth.make_record(wl)
        p = ssicov.Params(fs=wl.fs, lags=list(lags), order_min=2, order_max=rank, order_step=2,
                          svd=ssicov.SVD_RANDOMIZED, rank=rank, oversample=20, power_iters=2,
                          seed=wl.sketch_seed, prec=prec)
        out.append((y, p))
    return out


KEYS = ("sigma", "count", "f", "xi", "mu", "phi", "flags")


def _equal(a, b):
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), f"{k} differs"


def test_results_same_alone_and_in_mix():
    _need_gpu()
    from paper_2411_05510_amd import ssicov
    reqs = _mix()
    alone = []
    srv = ssicov.Server(0, max_inflight=1)
    for y, p in reqs:
        t = srv.submit(y, p)
        info = srv.wait(t)
        assert info["status"] == ssicov.SSI_OK
        alone.append(srv.result(t))
        srv.release(t)
    srv.close()

    srv = ssicov.Server(0, max_inflight=4)
    tickets = [srv.submit(y, p) for y, p in reqs]
    infos = [srv.wait(t) for t in tickets]
    for t, ref in zip(tickets, alone):
        _equal(srv.result(t), ref)
        srv.release(t)
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["peak_inflight"] >= 2, "requests never overlapped"
    # overlapping execution windows on different slots
    spans = sorted((i["t_start_us"], i["t_done_us"]) for i in infos)
    assert any(spans[k + 1][0] < spans[k][1] for k in range(len(spans) - 1))

    # the same as a plain context
    ctx = ssicov.Context(0)
    y, p = reqs[1]
    o = ctx.identify(torch.from_numpy(y).cuda(), p)
    ctx.synchronize()
    _equal({k: getattr(o, k).cpu().numpy() for k in KEYS}, alone[1])
    ctx.close()


def test_admission_by_footprint():
    _need_gpu()
    from paper_2411_05510_amd import ssicov
    reqs = _mix()
    fps = [ssicov.footprint(p, y.shape[0], y.shape[1]) for y, p in reqs]
    budget = int(2.2 * max(fps))
    srv = ssicov.Server(0, max_inflight=6, hbm_budget=budget)
    tickets = [srv.submit(y, p) for y, p in reqs]
    for t in tickets:
        assert srv.wait(t)["status"] == ssicov.SSI_OK
    st = srv.stats()
    srv.close()
    assert st["budget"] == budget
    assert st["peak_bytes"] <= budget
    assert st["completed"] == len(reqs)


def test_queued_request_reports_busy():
    _need_gpu()
    from paper_2411_05510_amd import ssicov
    reqs = _mix()
    srv = ssicov.Server(0, max_inflight=1)
    tickets = [srv.submit(y, p) for y, p in reqs[:4]]
    assert srv.poll(tickets[-1]) is None          # still queued behind three others
    with pytest.raises(ssicov.SSIError) as e:
        srv.result(tickets[-1])
    assert e.value.status in (ssicov.SSI_EBUSY,)
    info = srv.wait(tickets[-1])
    assert info["status"] == ssicov.SSI_OK
    assert info["t_submit_us"] <= info["t_start_us"] <= info["t_done_us"]
    assert srv.poll(tickets[-1]) is not None
    srv.close()


def test_submit_rejects_invalid_and_oversized():
    _need_gpu()
    from paper_2411_05510_amd import ssicov
    y, p = _mix()[0]
    srv = ssicov.Server(0, max_inflight=2, hbm_budget=1 << 20)
    with pytest.raises(ssicov.SSIError) as e:
        srv.submit(y, p)                           # needs far more than 1 MiB
    assert e.value.status == ssicov.SSI_ENOMEM
    bad = dataclasses.replace(p, order_max=p.rank + 2)
    with pytest.raises(ssicov.SSIError) as e:
        srv.submit(y, bad)
    assert e.value.status == ssicov.SSI_EINVAL
    srv.close()
