"""GPU parity of the modal stage and of the whole identification against the
FP64 checker.

Gates (FP32 path): singular values rel <= 1e-4 for sigma_i >= 1e-3 sigma_1;
frequencies rel <= 1e-5 on physical poles.  A physical pole is a checker pole
within 1 % in frequency and with MAC >= 0.9 to a generated mode; each must
have a GPU pole at the same (lag, order), matched by nearest frequency.
Damping and MAC of those poles are gated at abs 1e-4 and 0.9999.
"""
import types

import numpy as np
import pytest

import oracle
from paper_2411_05510_amd import synth
from modelref import mac, modal_correlations

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

F_RTOL = 1e-5
XI_ATOL = 1e-4
MAC_MIN = 0.9999
SIGMA_RTOL, SIGMA_FLOOR = 1e-4, 1e-3


@pytest.fixture(scope="module")
def ctx():
    from paper_2411_05510_amd import ssicov
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ssicov.Context(0)
    yield c
    c.close()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _params(wl, lags=None, **kw):
    from paper_2411_05510_amd import ssicov
    d = dict(fs=wl.fs, lags=list(lags or wl.lags), order_min=wl.order_min,
             order_max=wl.order_max, order_step=wl.order_step,
             svd=ssicov.SVD_FULL if wl.svd == "full" else ssicov.SVD_RANDOMIZED,
             rank=wl.rank, oversample=wl.oversample, power_iters=wl.power_iters,
             seed=wl.sketch_seed)
    d.update(kw)
    return ssicov.Params(**d)


def _physical(poles, sysm, f_tol=0.01, mac_min=0.9):
    """Indices of checker poles that are physical, with their mode index."""
    out = []
    for r, fr in enumerate(sysm.freqs):
        if len(poles) == 0:
            continue
        i = int(np.argmin(np.abs(poles.f - fr)))
        if abs(poles.f[i] - fr) / fr < f_tol and mac(poles.phi[i], sysm.shapes[:, r]) >= mac_min:
            out.append(i)
    return out


def _compare_order(gpu, ref, phys, stats):
    assert gpu["flag"] == 0
    gf = gpu["f"]
    for i in phys:
        j = int(np.argmin(np.abs(gf - ref.f[i])))
        ef = abs(gf[j] - ref.f[i]) / ref.f[i]
        ex = abs(gpu["xi"][j] - ref.xi[i])
        em = mac(gpu["phi"][j], ref.phi[i])
        stats["f"].append(ef)
        stats["xi"].append(ex)
        stats["mac"].append(em)


def _check_lag(out, lag_i, res, sysm, orders, stats):
    for oi, order in enumerate(orders):
        ref = res.poles[oi]
        gpu = out.poles(lag_i, oi)
        _compare_order(gpu, ref, _physical(ref, sysm), stats)
        # every order: counts agree up to pole pairs at the real axis
        assert abs(len(gpu["f"]) - len(ref)) <= 1 + len(ref) // 20


def _assert_stats(stats):
    assert stats["f"], "no physical poles compared"
    f = np.array(stats["f"]); x = np.array(stats["xi"]); m = np.array(stats["mac"])
    assert f.max() <= F_RTOL, f"max f rel err {f.max():.3e}"
    assert x.max() <= XI_ATOL, f"max xi abs err {x.max():.3e}"
    assert m.min() >= MAC_MIN, f"min MAC {m.min():.6f}"


def _check_sigma(got, ref):
    keep = ref >= SIGMA_FLOOR * ref[0]
    rel = np.abs(got[: len(ref)][keep] - ref[keep]) / ref[keep]
    assert rel.max() <= SIGMA_RTOL, f"max sigma rel err {rel.max():.3e}"


# ------------------------------------------------------------ modal stage
def test_modal_stage_same_inputs(ctx):
    """Checker U and sigma of the small record's Toeplitz matrix into both
    modal stages: every physical pole agrees to near FP64 precision."""
    from paper_2411_05510_amd import ssicov
    wl = synth.WORKLOADS["small-full-svd"]
    sysm, y = synth.make_record(wl)
    jb = wl.lags[0]
    t = oracle.toeplitz(oracle.correlations(y, 2 * jb - 1), jb)
    u, s = oracle.full_svd(t, wl.order_max)
    p = _params(wl)
    out = ctx.alloc_output(p, wl.l, wl.n)
    ctx.modal(_dev(u), _dev(s), wl.l, p, 0, out)
    ctx.synchronize()
    ref = oracle.modal(u, s, wl.l, wl.orders, wl.fs)
    stats = {"f": [], "xi": [], "mac": []}
    for oi in range(len(wl.orders)):
        gpu = out.poles(0, oi)
        _compare_order(gpu, ref[oi], _physical(ref[oi], sysm), stats)
        # all poles, not only physical ones: same count and near-equal values
        assert len(gpu["f"]) == len(ref[oi])
        if len(ref[oi]):
            np.testing.assert_allclose(gpu["f"], ref[oi].f, rtol=1e-8)
            np.testing.assert_allclose(gpu["xi"], ref[oi].xi, rtol=1e-6, atol=1e-10)
    f = np.array(stats["f"])
    assert f.max() <= 1e-10
    # mode shapes are returned as FP32 complex: MAC resolution about 1e-7
    assert np.array(stats["mac"]).min() >= 1 - 1e-6


def test_modal_exact_model(ctx):
    """Exact correlations of the generator's model: the order-2n poles are the
    generated modes."""
    wl = synth.WORKLOADS["small-full-svd"]
    sysm = synth.draw_system(wl.l, wl.n_modes, wl.f_range, wl.zeta_range, wl.fs,
                             wl.struct_seed)
    jb = 6
    t = oracle.toeplitz(modal_correlations(sysm, 2 * jb - 1), jb)
    u, s = oracle.full_svd(t, 2 * wl.n_modes)
    p = _params(wl, lags=[jb], order_min=2 * wl.n_modes, order_max=2 * wl.n_modes)
    out = ctx.alloc_output(p, wl.l, 1000)
    ctx.modal(_dev(u), _dev(s), wl.l, p, 0, out)
    ctx.synchronize()
    g = out.poles(0, 0)
    np.testing.assert_allclose(g["f"], sysm.freqs, rtol=1e-10)
    np.testing.assert_allclose(g["xi"], sysm.zetas, rtol=1e-8)
    for r in range(wl.n_modes):
        assert mac(g["phi"][r], sysm.shapes[:, r]) > 1 - 1e-6   # phi stored FP32


# ------------------------------------------------------------ identification
def test_identify_small_full_svd(ctx):
    wl = synth.WORKLOADS["small-full-svd"]
    sysm, y = synth.make_record(wl)
    p = _params(wl)
    out = ctx.identify(_dev(y), p)
    ctx.synchronize()
    res = oracle.identify(y, wl.fs, wl.lags, wl.orders, svd="full")
    _check_sigma(out.sigma[0].cpu().numpy(), res[0].sigma)
    stats = {"f": [], "xi": [], "mac": []}
    _check_lag(out, 0, res[0], sysm, wl.orders, stats)
    _assert_stats(stats)


def test_identify_two_lags_odd_orders(ctx):
    wl = synth.WORKLOADS["small-full-svd"]
    sysm, y = synth.make_record(wl, n=12000)
    lags, orders = [9, 14], list(range(3, 26, 1))
    p = _params(wl, lags=lags, order_min=3, order_max=25, order_step=1)
    out = ctx.identify(_dev(y), p)
    ctx.synchronize()
    res = oracle.identify(y, wl.fs, lags, orders, svd="full")
    stats = {"f": [], "xi": [], "mac": []}
    for i in range(len(lags)):
        _check_sigma(out.sigma[i].cpu().numpy(), res[i].sigma)
        _check_lag(out, i, res[i], sysm, orders, stats)
    _assert_stats(stats)


def test_identify_randomized_two_lags(ctx):
    """Randomized SVD per lag (Philox stream = lag index), 60 channels."""
    wl = synth.Workload(name="mid", l=60, n=30000, fs=100.0, n_modes=8,
                        f_range=(0.5, 20.0), zeta_range=(0.005, 0.03), noise=0.05,
                        lags=(12, 20), svd="randomized", rank=60, oversample=10,
                        power_iters=2, order_min=2, order_max=60, order_step=2,
                        struct_seed=77, noise_seed=78, sketch_seed=79)
    sysm, y = synth.make_record(wl)
    p = _params(wl)
    out = ctx.identify(_dev(y), p)
    ctx.synchronize()
    res = oracle.identify(y, wl.fs, wl.lags, wl.orders, svd="randomized", rank=wl.rank,
                          oversample=wl.oversample, power_iters=wl.power_iters,
                          seed=wl.sketch_seed)
    stats = {"f": [], "xi": [], "mac": []}
    for i in range(len(wl.lags)):
        _check_sigma(out.sigma[i].cpu().numpy(), res[i].sigma)
        _check_lag(out, i, res[i], sysm, wl.orders, stats)
    _assert_stats(stats)


def test_modal_orders_above_200_same_inputs(ctx):
    """Orders 196..224 (above 200 the Hessenberg matrix is kept in global
    memory) fed the checker's U and sigma of a 40-channel record's 320 x 320
    Toeplitz matrix: both modal stages see identical FP64 inputs.  The noise
    part of the spectrum is flat here (sigma_200 / sigma_1 ~ 5e-6), so the
    identification itself is ill-conditioned at these orders (rounding R to
    FP32 moves the checker's own physical poles by ~1e-4); with identical
    inputs the two eigen-analyses must still agree to FP64 precision."""
    wl = synth.Workload(name="wide", l=40, n=20000, fs=100.0, n_modes=6,
                        f_range=(1.0, 20.0), zeta_range=(0.01, 0.03), noise=0.05,
                        lags=(8,), svd="randomized", rank=224, oversample=16,
                        power_iters=1, order_min=196, order_max=224, order_step=4,
                        struct_seed=5, noise_seed=6, sketch_seed=7)
    sysm, y = synth.make_record(wl)
    jb = wl.lags[0]
    t = oracle.toeplitz(oracle.correlations(y, 2 * jb - 1), jb)
    u, s = oracle.rsvd(t, wl.rank, wl.oversample, wl.power_iters,
                       oracle.sketch(wl.sketch_seed, t.shape[0], wl.rank + wl.oversample, 0))
    p = _params(wl)
    out = ctx.alloc_output(p, wl.l, wl.n)
    ctx.modal(_dev(u), _dev(s), wl.l, p, 0, out)
    ctx.synchronize()
    ref = oracle.modal(u, s, wl.l, wl.orders, wl.fs)
    stats = {"f": [], "xi": [], "mac": []}
    for oi in range(len(wl.orders)):
        gpu = out.poles(0, oi)
        assert gpu["flag"] == 0
        _compare_order(gpu, ref[oi], _physical(ref[oi], sysm), stats)
        # every pole: same count up to a pair at the real axis, and each
        # checker pole has a GPU pole at nearly the same discrete eigenvalue
        assert abs(len(gpu["f"]) - len(ref[oi])) <= 1
        mu_gpu = gpu["mu"]
        dmu = np.array([np.min(np.abs(mu_gpu - m)) for m in ref[oi].mu])
        assert np.sum(dmu > 1e-8) <= 1, f"order {wl.orders[oi]}: max |d mu| {dmu.max():.2e}"
    assert np.array(stats["f"]).max() <= 1e-10
    assert np.array(stats["xi"]).max() <= 1e-9
    assert np.array(stats["mac"]).min() >= 1 - 1e-6


def test_modal_orders_to_448_same_inputs(ctx):
    """Orders 196..448 step 12 (448 is the largest the modal kernels take),
    fed the checker's U and sigma of a 60-channel record's 540 x 540 Toeplitz
    matrix (k = 456): the QR iteration in LDS (196) and in global memory, the
    Hessenberg reduction in registers (up to 224) and in global memory
    (above), and pole vectors with seven rows per lane.  Physical poles: f rel <= 1e-10, xi abs <= 1e-9, MAC >= 1 - 1e-6.
    Every checker eigenvalue has a GPU eigenvalue within what a backward
    stable eigen-solver may move it: 1e3 eps ||X_n||_F kappa_i, kappa_i the
    eigenvalue's condition number (1 / |y_i^H x_i| for unit left and right
    eigenvectors) of X_n = S^1/2 A_n S^-1/2, the matrix the GPU reduces."""
    import scipy.linalg
    wl = synth.Workload(name="wide400", l=60, n=20000, fs=100.0, n_modes=8,
                        f_range=(1.0, 20.0), zeta_range=(0.01, 0.03), noise=0.05,
                        lags=(9,), svd="randomized", rank=456, oversample=16,
                        power_iters=1, order_min=196, order_max=448, order_step=12,
                        struct_seed=15, noise_seed=16, sketch_seed=17)
    sysm, y = synth.make_record(wl)
    jb = wl.lags[0]
    t = oracle.toeplitz(oracle.correlations(y, 2 * jb - 1), jb)
    u, s = oracle.rsvd(t, wl.rank, wl.oversample, wl.power_iters,
                       oracle.sketch(wl.sketch_seed, t.shape[0], wl.rank + wl.oversample, 0))
    p = _params(wl)
    out = ctx.alloc_output(p, wl.l, wl.n)
    ctx.modal(_dev(u), _dev(s), wl.l, p, 0, out)
    ctx.synchronize()
    ref = oracle.modal(u, s, wl.l, wl.orders, wl.fs)
    stats = {"f": [], "xi": [], "mac": []}
    eps = np.finfo(np.float64).eps
    worst = 0.0
    for oi, n in enumerate(wl.orders):
        gpu = out.poles(0, oi)
        assert gpu["flag"] == 0, f"order {n}"
        _compare_order(gpu, ref[oi], _physical(ref[oi], sysm), stats)
        assert abs(len(gpu["f"]) - len(ref[oi])) <= 1, f"order {n}"
        a, _ = oracle.shift_ls(u, s, wl.l, n)
        sq = np.sqrt(s[:n])
        x = sq[:, None] * a / sq[None, :]
        ev, vl, vr = scipy.linalg.eig(x, left=True, right=True)
        kappa = 1.0 / np.maximum(np.abs(np.sum(vl.conj() * vr, axis=0)), 1e-300)
        bound = 1e3 * eps * np.linalg.norm(x) * kappa
        mu_gpu = gpu["mu"]
        for m in ref[oi].mu:
            i = int(np.argmin(np.abs(ev - m)))
            d = np.min(np.abs(mu_gpu - m))
            worst = max(worst, d / bound[i])
            assert d <= bound[i], (f"order {n}: |d mu| {d:.2e} > bound {bound[i]:.2e} "
                                   f"(kappa {kappa[i]:.1e})")
    print(f"orders 196..448: {len(stats['f'])} physical poles, max f rel "
          f"{max(stats['f']):.2e}, max |d mu| / bound {worst:.2e}")
    assert np.array(stats["f"]).max() <= 1e-10
    assert np.array(stats["xi"]).max() <= 1e-9
    assert np.array(stats["mac"]).min() >= 1 - 1e-6


def test_identify_deterministic(ctx):
    wl = synth.WORKLOADS["small-full-svd"]
    _, y = synth.make_record(wl, n=8000)
    p = _params(wl)
    yd = _dev(y)
    a = ctx.identify(yd, p)
    ctx.synchronize()
    fa = a.f.clone(); pa = a.phi.clone()
    b = ctx.identify(yd, p)
    ctx.synchronize()
    assert torch.equal(fa, b.f) and torch.equal(pa, b.phi)


def test_identify_eig_workgroups_same_results(ctx):
    """A smaller eigen-analysis grid (raised to one workgroup per order)
    changes which workgroup computes each order and pole, not the arithmetic:
    the poles equal those of the default grid."""
    wl = synth.WORKLOADS["small-full-svd"]
    _, y = synth.make_record(wl, n=8000)
    p = _params(wl)
    yd = _dev(y)
    a = ctx.identify(yd, p)
    ctx.synchronize()
    fa, pa, ca = a.f.clone(), a.phi.clone(), a.count.clone()
    ctx.set_eig_workgroups(3)
    try:
        b = ctx.identify(yd, p)
        ctx.synchronize()
    finally:
        ctx.set_eig_workgroups(0)
    assert torch.equal(ca, b.count)
    assert torch.allclose(fa, b.f, rtol=1e-12, atol=0)
    assert torch.allclose(pa, b.phi, rtol=1e-10, atol=1e-12)


_BRIDGE_REF = {}


def _bridge_reference():
    """The bridge record and the checker's steps on it, with its correlation
    stack kept for the comparison; computed once per module."""
    if not _BRIDGE_REF:
        wl = synth.WORKLOADS["bridge-180ch"]
        sysm, y = synth.make_record(wl)
        L = 2 * wl.lags[0] - 1
        r_ref = oracle.correlations(y, L)
        t = oracle.toeplitz(r_ref, wl.lags[0])
        u, s = oracle.rsvd(t, wl.rank, wl.oversample, wl.power_iters,
                           oracle.sketch(wl.sketch_seed, t.shape[0], wl.rank + wl.oversample, 0))
        del t
        res = types.SimpleNamespace(sigma=s, poles=oracle.modal(u, s, wl.l, wl.orders, wl.fs))
        _BRIDGE_REF.update(wl=wl, sysm=sysm, y=y, L=L, r_ref=r_ref, res=res)
    return _BRIDGE_REF


@pytest.mark.parametrize("corr_mode", [1, 2], ids=["corr_bf16x6", "corr_f16x3"])
def test_identify_bridge_record(ctx, corr_mode):
    """The 180-channel, 30-minute record at j_b = 60 (10800 x 10800 Toeplitz),
    randomized SVD k = 200, p = 20, q = 2, orders 2..200: the configuration
    the benchmark times, with each split correlation path.  The whole
    correlation stack (119 x 180 x 180) is compared element by element, the
    singular values and physical poles at the FP32 gates, and the error
    distribution of every pole (spurious ones included) is reported."""
    ref = _bridge_reference()
    wl, sysm, y, L, r_ref, res = (ref[k] for k in ("wl", "sysm", "y", "L", "r_ref", "res"))
    p = _params(wl)
    yd = _dev(y)
    ctx.set_corr_mode(corr_mode)
    try:
        out = ctx.identify(yd, p)
        r_gpu = ctx.correlate(yd, L)
        ctx.synchronize()
    finally:
        ctx.set_corr_mode(2)
    rms = np.sqrt(np.mean(y.astype(np.float64) ** 2, axis=1))
    err = np.abs(r_gpu.cpu().numpy().astype(np.float64) - r_ref) / np.outer(rms, rms)[None]
    rel = np.abs(r_gpu.cpu().numpy().astype(np.float64) - r_ref) / np.maximum(np.abs(r_ref), 1e-300)
    big = np.abs(r_ref) >= 1e-2 * np.outer(rms, rms)[None]
    print(f"bridge R stack ({corr_mode}): {r_ref.size} entries, max |dR| / (rms_a rms_b) "
          f"{err.max():.2e}, max rel where |R| >= 1e-2 rms_a rms_b {rel[big].max():.2e}")
    assert err.max() <= 1e-6
    _check_sigma(out.sigma[0].cpu().numpy(), res.sigma)
    stats = {"f": [], "xi": [], "mac": []}
    _check_lag(out, 0, res, sysm, wl.orders, stats)
    _assert_stats(stats)
    print(f"bridge ({corr_mode}): {len(stats['f'])} physical poles, max f rel {max(stats['f']):.2e}, "
          f"max xi abs {max(stats['xi']):.2e}, min MAC {min(stats['mac']):.8f}")
    # every GPU pole against the nearest checker pole of the same order
    allf, unmatched, n_gpu, n_ref = [], 0, 0, 0
    for oi in range(len(wl.orders)):
        g, r = out.poles(0, oi), res.poles[oi]
        n_gpu += len(g["f"])
        n_ref += len(r)
        for fg in g["f"]:
            if len(r) == 0:
                unmatched += 1
                continue
            allf.append(np.min(np.abs(r.f - fg)) / fg)
    allf = np.array(allf)
    print(f"bridge, all poles: {n_gpu} GPU / {n_ref} checker; nearest-pole f rel p50 "
          f"{np.percentile(allf, 50):.1e} p90 {np.percentile(allf, 90):.1e} p99 "
          f"{np.percentile(allf, 99):.1e} max {allf.max():.1e}; share above 1e-5 "
          f"{np.mean(allf > 1e-5):.4f}")
    assert abs(n_gpu - n_ref) <= 2 + 0.05 * n_ref
