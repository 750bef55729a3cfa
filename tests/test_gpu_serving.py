"""GPU tests of the serving runtime (continuous batching on one GPU).

* every result is the same alone (one slot, one request at a time) and in a
  mix of concurrent requests with uneven channel counts, lags, orders and
  precisions (bit for bit: kernels are deterministic and a request's work
  stays on its slot), and equal to a plain context's identification;
* every result of the mix matches the FP64 checker's identification of the
  same window with the same sketch on its physical poles: at the FP32 gates
  (f rel 1e-5, xi abs 1e-4, MAC 0.9999) for FP32 products, at the
  reduced-precision gates (f rel 1e-3, xi abs 2e-3, MAC 0.99) for the
  split-BF16 range finders, and within f rel 1e-2 for plain BF16 (a
  lower-accuracy mode);
* admission keeps the device memory the slots hold within the budget, so a
  budget for two requests caps the requests running at once at two;
* a request queued behind others reports busy until it has run;
* invalid requests and requests larger than the budget are refused at submit.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2411_05510_amd import synth
from modelref import mac

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _mix(with_models=False):
    """Six windows of different structures."""
    from paper_2411_05510_amd import ssicov
    out = []
    specs = [(24, 6, (12,), ssicov.PREC_FP32), (60, 10, (12, 20), ssicov.PREC_FP32),
             (120, 8, (10,), ssicov.PREC_BF16), (36, 12, (16, 24), ssicov.PREC_BF16X3),
             (60, 8, (20,), ssicov.PREC_BF16X6), (90, 14, (12,), ssicov.PREC_BF16)]
    for i, (l, modes, lags, prec) in enumerate(specs):
        rank = 2 * modes + 20
        wl = synth.Workload(name=f"req{i}", l=l, n=20000, fs=100.0, n_modes=modes,
                            f_range=(0.5, 20.0), zeta_range=(0.005, 0.03), noise=0.05,
                            lags=lags, svd="randomized", rank=rank, oversample=20,
                            power_iters=2, order_min=2, order_max=rank, order_step=2,
                            struct_seed=500 + i, noise_seed=600 + i, sketch_seed=700 + i)
        sysm, y = synth.make_record(wl)
        p = ssicov.Params(fs=wl.fs, lags=list(lags), order_min=2, order_max=rank, order_step=2,
                          svd=ssicov.SVD_RANDOMIZED, rank=rank, oversample=20, power_iters=2,
                          seed=wl.sketch_seed, prec=prec,
                          refine=1 if prec == ssicov.PREC_BF16X3 else 0)
        out.append((y, p, sysm) if with_models else (y, p))
    return out


def _check_against_oracle(y, p, sysm, res):
    """Physical poles of a served result (host arrays in the ssi_output
    layout) against the FP64 checker with the same sketch."""
    from paper_2411_05510_amd import ssicov
    gates = {ssicov.PREC_FP32: (1e-5, 1e-4, 0.9999), ssicov.PREC_BF16X6: (1e-3, 2e-3, 0.99),
             ssicov.PREC_BF16X3: (1e-3, 2e-3, 0.99), ssicov.PREC_BF16: (1e-2, None, None)}[p.prec]
    ref = oracle.identify(y, p.fs, p.lags, p.orders, svd="randomized", rank=p.rank,
                          oversample=p.oversample, power_iters=p.power_iters, seed=p.seed)
    worst, n = [0.0, 0.0, 1.0], 0
    for li, lag in enumerate(ref):
        for oi, r in enumerate(lag.poles):
            off = ssicov.pole_offset(p, oi)
            cnt = int(res["count"][li, oi])
            assert res["flags"][li, oi] == 0
            gf = res["f"][li, off:off + cnt]
            gx = res["xi"][li, off:off + cnt]
            gphi = res["phi"][li, off:off + cnt].astype(np.float64)
            gphi = gphi[..., 0] + 1j * gphi[..., 1]
            for k, fr in enumerate(sysm.freqs):
                if len(r) == 0 or cnt == 0:
                    continue
                i = int(np.argmin(np.abs(r.f - fr)))
                if abs(r.f[i] - fr) / fr >= 0.01 or mac(r.phi[i], sysm.shapes[:, k]) < 0.9:
                    continue
                j = int(np.argmin(np.abs(gf - r.f[i])))
                worst[0] = max(worst[0], abs(gf[j] - r.f[i]) / r.f[i])
                worst[1] = max(worst[1], abs(gx[j] - r.xi[i]))
                worst[2] = min(worst[2], mac(gphi[j], r.phi[i]))
                n += 1
    assert n > 0
    assert worst[0] <= gates[0], worst
    if gates[1] is not None:
        assert worst[1] <= gates[1] and worst[2] >= gates[2], worst
    return worst, n


KEYS = ("sigma", "count", "f", "xi", "mu", "phi", "flags")


def _equal(a, b):
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), f"{k} differs"


def test_results_same_alone_and_in_mix():
    _need_gpu()
    from paper_2411_05510_amd import ssicov
    models = _mix(with_models=True)
    reqs = [(y, p) for y, p, _ in models]
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
    for t, ref, (y, p, sysm) in zip(tickets, alone, models):
        got = srv.result(t)
        _equal(got, ref)
        worst, n = _check_against_oracle(y, p, sysm, got)
        print(f"served l={y.shape[0]} lags={list(p.lags)} prec={p.prec}: {n} physical poles, "
              f"max f rel {worst[0]:.2e}, max xi abs {worst[1]:.2e}, min MAC {worst[2]:.6f}",
              flush=True)
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


def _light_mix():
    """Four windows with few channels (small records, quick to submit) and
    several lags each (a long chain of device work per request)."""
    from paper_2411_05510_amd import ssicov
    out = []
    specs = [(24, 6, (12, 20, 28), ssicov.PREC_FP32), (36, 12, (16, 24, 32), ssicov.PREC_BF16X3),
             (24, 8, (10, 18, 26), ssicov.PREC_BF16), (36, 10, (12, 20, 28), ssicov.PREC_BF16X6)]
    for i, (l, modes, lags, prec) in enumerate(specs):
        rank = 2 * modes + 20
        wl = synth.Workload(name=f"light{i}", l=l, n=20000, fs=100.0, n_modes=modes,
                            f_range=(0.5, 20.0), zeta_range=(0.005, 0.03), noise=0.05,
                            lags=lags, svd="randomized", rank=rank, oversample=20,
                            power_iters=2, order_min=2, order_max=rank, order_step=2,
                            struct_seed=800 + i, noise_seed=900 + i, sketch_seed=1000 + i)
        _, y = synth.make_record(wl)
        p = ssicov.Params(fs=wl.fs, lags=list(lags), order_min=2, order_max=rank, order_step=2,
                          svd=ssicov.SVD_RANDOMIZED, rank=rank, oversample=20, power_iters=2,
                          seed=wl.sketch_seed, prec=prec,
                          refine=1 if prec == ssicov.PREC_BF16X3 else 0)
        out.append((y, p))
    return out


def test_sixty_four_in_flight():
    """64 slots: 96 requests over four windows, submitted at once; every
    result equals the same window served alone, and more than 16 requests ran
    at once at some point.  The windows are light to submit and long to
    serve (three lags each), so the submission loop outruns completion and
    the peak reflects the slot count rather than the host's copy rate."""
    _need_gpu()
    from paper_2411_05510_amd import ssicov
    reqs = _light_mix()
    srv = ssicov.Server(0, max_inflight=1)
    alone = []
    for y, p in reqs:
        t = srv.submit(y, p)
        srv.wait(t)
        alone.append(srv.result(t))
        srv.release(t)
    srv.close()
    print("64 slots: submitting 96 requests", flush=True)
    srv = ssicov.Server(0, max_inflight=64)
    tickets = [srv.submit(*reqs[i % len(reqs)]) for i in range(96)]
    for i, t in enumerate(tickets):
        assert srv.wait(t)["status"] == ssicov.SSI_OK
        _equal(srv.result(t), alone[i % len(reqs)])
        srv.release(t)
    st = srv.stats()
    srv.close()
    print(f"64 slots: peak in flight {st['peak_inflight']}, peak bytes {st['peak_bytes']}")
    assert st["completed"] == 96 and st["failed"] == 0
    assert st["peak_inflight"] > 16
