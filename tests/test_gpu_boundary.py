"""The C-ABI boundary beyond the stage calls: host-record ingest, a caller
sketch, non-finite input, the eigen-analysis sweep limit, host results with
their accessors, a caller allocator and the bounded graph cache.

Results that run the same kernels on the same inputs are compared bit for
bit; the caller sketch is compared with the FP64 checker given the same
sketch, at the FP32 gates (frequencies rel 1e-5, damping abs 1e-4, MAC
0.9999 on physical poles; singular values rel 1e-4 above 1e-3 sigma_1)."""
import numpy as np
import pytest

import oracle
from paper_2411_05510_amd import synth
from modelref import mac

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

REC = synth.Workload(name="abi", l=24, n=12000, fs=50.0, n_modes=4, f_range=(0.5, 10.0),
                     zeta_range=(0.01, 0.03), noise=0.05, lags=(8, 12), svd="randomized",
                     rank=24, oversample=8, power_iters=1, order_min=2, order_max=24,
                     order_step=2, struct_seed=81, noise_seed=82, sketch_seed=83)


@pytest.fixture(scope="module")
def ctx():
    from paper_2411_05510_amd import ssicov
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ssicov.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def record():
    return synth.make_record(REC)


def _params(**kw):
    from paper_2411_05510_amd import ssicov
    d = dict(fs=REC.fs, lags=list(REC.lags), order_min=REC.order_min, order_max=REC.order_max,
             order_step=REC.order_step, svd=ssicov.SVD_RANDOMIZED, rank=REC.rank,
             oversample=REC.oversample, power_iters=REC.power_iters, seed=REC.sketch_seed)
    d.update(kw)
    return ssicov.Params(**d)


def _host(out):
    return {k: getattr(out, k).cpu().numpy() for k in ("sigma", "count", "f", "xi", "mu", "phi",
                                                       "flags")}


def _same(a, b):
    for k in a:
        assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), k


def test_host_record_equals_device_record(ctx, record):
    _, y = record
    p = _params()
    ref = _host(ctx.identify(torch.from_numpy(y).cuda(), p))
    ctx.synchronize()
    pageable = torch.from_numpy(y.copy())
    pinned = torch.from_numpy(y.copy()).pin_memory()
    for host in (pageable, pinned):
        out = ctx.identify(host, p)
        ctx.synchronize()
        _same(ref, _host(out))
    # a host record with a leading dimension beyond n
    wide = np.zeros((REC.l, REC.n + 5), dtype=np.float32)
    wide[:, :REC.n] = y
    out = ctx.identify(torch.from_numpy(wide)[:, :REC.n], p)
    ctx.synchronize()
    _same(ref, _host(out))


def test_caller_sketch_matches_checker(ctx, record):
    """A caller sketch (plain numpy Gaussian, not Philox), one m_max x ell
    array for both lags: lag i uses its leading j_b,i l rows on both sides."""
    sysm, y = record
    ell = REC.rank + REC.oversample
    m_max = max(REC.lags) * REC.l
    om = np.random.default_rng(84).standard_normal((m_max, ell + 3)).astype(np.float32)
    omd = torch.from_numpy(om).cuda()[:, :ell]            # leading dimension ell + 3
    p = _params(omega=omd)
    out = ctx.identify(torch.from_numpy(y).cuda(), p)
    ctx.synchronize()
    res = oracle.identify(y, REC.fs, REC.lags, REC.orders, svd="randomized", rank=REC.rank,
                          oversample=REC.oversample, power_iters=REC.power_iters,
                          omegas=[om[:jb * REC.l, :ell].astype(np.float64) for jb in REC.lags])
    n_phys = 0
    for li, lag_res in enumerate(res):
        sig = out.sigma[li].cpu().numpy()
        keep = lag_res.sigma >= 1e-3 * lag_res.sigma[0]
        assert np.max(np.abs(sig[keep] - lag_res.sigma[keep]) / lag_res.sigma[keep]) <= 1e-4
        for oi in range(len(REC.orders)):
            g, r = out.poles(li, oi), lag_res.poles[oi]
            assert g["flag"] == 0
            for k, fr in enumerate(sysm.freqs):
                if len(r) == 0:
                    continue
                i = int(np.argmin(np.abs(r.f - fr)))
                if abs(r.f[i] - fr) / fr >= 0.01 or mac(r.phi[i], sysm.shapes[:, k]) < 0.9:
                    continue
                j = int(np.argmin(np.abs(g["f"] - r.f[i])))
                assert abs(g["f"][j] - r.f[i]) / r.f[i] <= 1e-5
                assert abs(g["xi"][j] - r.xi[i]) <= 1e-4
                assert mac(g["phi"][j], r.phi[i]) >= 0.9999
                n_phys += 1
    assert n_phys > 20
    # a different sketch changes the result: the caller's array was used
    other = ctx.identify(torch.from_numpy(y).cuda(), _params())
    ctx.synchronize()
    assert not np.array_equal(other.sigma.cpu().numpy(), out.sigma.cpu().numpy())


@pytest.mark.parametrize("corr", [0, 1, 2], ids=["fp32", "bf16x6", "f16x3"])
@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_non_finite_record_is_rejected(ctx, record, bad, corr):
    from paper_2411_05510_amd import ssicov
    _, y = record
    yb = y.copy()
    yb[3, 777] = bad
    print(f"non-finite record: sample (3, 777) = {bad}, correlation mode {corr}", flush=True)
    ctx.set_corr_mode(corr)
    try:
        ctx.identify(torch.from_numpy(yb).cuda(), _params())
        with pytest.raises(ssicov.SSIError) as ei:
            ctx.synchronize()
        assert ei.value.status == ssicov.SSI_EINVAL
        assert "non-finite" in str(ei.value)
        # the context stays usable and the status word was cleared
        out = ctx.identify(torch.from_numpy(y).cuda(), _params())
        ctx.synchronize()
        assert int(out.flags.sum().item()) == 0
    finally:
        ctx.set_corr_mode(2)


def test_sweep_limit_gives_enoconv(ctx, record):
    from paper_2411_05510_amd import ssicov
    _, y = record
    yd = torch.from_numpy(y).cuda()
    p = _params()
    try:
        ctx.set_eig_max_sweeps(0)
        out = ctx.identify(yd, p)
        with pytest.raises(ssicov.SSIError) as ei:
            ctx.synchronize()
        assert ei.value.status == ssicov.SSI_ENOCONV
        assert "sweep limit" in str(ei.value)
        flags = out.flags.cpu().numpy()
        orders = np.array(p.orders)
        # orders of size 2 need no sweep; every larger order hit the limit
        assert (flags[:, orders > 2] == 1).all() and (flags[:, orders == 2] == 0).all()
        assert (out.count.cpu().numpy()[:, orders > 2] == 0).all()
    finally:
        ctx.set_eig_max_sweeps(30)
    out = ctx.identify(yd, p)
    ctx.synchronize()
    assert int(out.flags.sum().item()) == 0


def test_host_result_accessors(ctx, record):
    _, y = record
    p = _params()
    dev = ctx.identify(torch.from_numpy(y).cuda(), p)
    ctx.synchronize()
    for src in (y, torch.from_numpy(y).cuda()):
        res = ctx.identify_result(src, p)
        d = res.dims()
        assert d == {"n_lags": 2, "n_orders": len(p.orders), "l": REC.l}
        for li in range(2):
            assert np.array_equal(res.singular_values(li), dev.sigma[li].cpu().numpy())
            for oi, n in enumerate(p.orders):
                a, b = res.poles(li, oi), dev.poles(li, oi)
                assert a["order"] == n and a["flag"] == b["flag"] == 0
                for k in ("f", "xi", "mu", "phi"):
                    assert np.array_equal(a[k], b[k]), (li, n, k)
        res.close()
    fetched = ctx.fetch(dev, REC.l)
    assert np.array_equal(fetched.poles(1, 5)["f"], dev.poles(1, 5)["f"])


def test_torch_allocator(record):
    """Workspace from torch's caching allocator: same results bit for bit, and
    the workspace shows up in torch's allocated bytes."""
    from paper_2411_05510_amd import ssicov
    _, y = record
    yd = torch.from_numpy(y).cuda()
    p = _params()
    plain = ssicov.Context(0)
    ref = _host(plain.identify(yd, p))
    plain.synchronize()
    plain.close()
    c = ssicov.Context(0)
    try:
        c.use_torch_allocator()
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        out = c.identify(yd, p)
        c.synchronize()
        assert torch.cuda.memory_allocated() - before >= c.workspace_bytes > 0
        _same(ref, _host(out))
        res = c.identify_result(yd, p)
        assert np.array_equal(res.singular_values(0), ref["sigma"][0])
        res.close()
    finally:
        c.close()


def test_graph_cache_stays_correct_past_its_bound(ctx, record):
    """Ten distinct output-buffer sets (more than the eight graphs kept),
    each used twice in a scrambled order: every launch gives the eager result."""
    _, y = record
    yd = torch.from_numpy(y).cuda()
    p = _params()
    ref = _host(ctx.identify(yd, p))
    ctx.synchronize()
    outs = [ctx.alloc_output(p, REC.l, REC.n) for _ in range(10)]
    try:
        ctx.set_graphs(True)
        for i in [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 0, 9, 5, 1, 8, 2, 7, 3, 6, 4]:
            for t in (outs[i].f, outs[i].phi):
                t.zero_()
            ctx.identify(yd, p, outs[i])
            ctx.synchronize()
            _same(ref, _host(outs[i]))
    finally:
        ctx.set_graphs(False)
