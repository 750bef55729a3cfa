"""The randomized SVD's approximation error against the exact SVD, reported
(not gated) as the paper's Table 2 reports it for its own data: physical
poles identified through the randomized SVD against those identified through
the exact SVD of the same Toeplitz matrix, as relative frequency and absolute
damping differences and the MAC of the mode shapes.

* CPU: the FP64 checker's randomized SVD against its one-sided Jacobi SVD on
  the 12-channel record (240 x 240 Toeplitz), k = 40, p = 8, q = 0 and 2;
* GPU: the library's randomized SVD against its exact SVD on 30 channels of
  the 180-channel record at j_b = 30 (900 x 900 Toeplitz), k = 200, p = 20,
  q = 2 (the bench's settings), orders 2..200.

The assertions only catch gross failures (a physical pole missing or moved
by more than 1 %); the printed figures are the report."""
import types

import numpy as np
import pytest

import oracle
from paper_2411_05510_amd import synth
from modelref import mac


def _physical(poles_f, poles_phi, sysm):
    out = []
    for r, fr in enumerate(sysm.freqs):
        if len(poles_f) == 0:
            continue
        i = int(np.argmin(np.abs(poles_f - fr)))
        if abs(poles_f[i] - fr) / fr < 0.01 and mac(poles_phi[i], sysm.shapes[:, r]) >= 0.9:
            out.append(i)
    return out


def _compare(exact, approx, sysm):
    """exact, approx: per order (f, xi, phi).  Deltas of the exact SVD's
    physical poles against the nearest randomized-SVD pole."""
    df, dx, mm = [], [], []
    for (fe, xe, pe), (fa, xa, pa) in zip(exact, approx):
        for i in _physical(fe, pe, sysm):
            j = int(np.argmin(np.abs(fa - fe[i])))
            df.append(abs(fa[j] - fe[i]) / fe[i])
            dx.append(abs(xa[j] - xe[i]))
            mm.append(mac(pa[j], pe[i]))
    return np.array(df), np.array(dx), np.array(mm)


def _report(name, df, dx, mm):
    print(f"{name}: {len(df)} physical poles; f rel max {df.max():.2e} mean {df.mean():.2e} "
          f"(max {100 * df.max():.4f} %); xi abs max {dx.max():.2e} mean {dx.mean():.2e}; "
          f"MAC min {mm.min():.6f} mean {mm.mean():.6f}")


def test_report_oracle_rsvd_vs_jacobi_small_record():
    wl = synth.WORKLOADS["small-full-svd"]
    sysm, y = synth.make_record(wl)
    jb = wl.lags[0]
    t = oracle.toeplitz(oracle.correlations(y, 2 * jb - 1), jb)
    ue, se = oracle.full_svd(t, 40)
    exact = [(p.f, p.xi, p.phi) for p in oracle.modal(ue, se, wl.l, wl.orders, wl.fs)]
    for q in (0, 2):
        om = oracle.sketch(wl.sketch_seed, t.shape[0], 48, 0)
        ua, sa = oracle.rsvd(t, 40, 8, q, om)
        srel = np.abs(sa - se) / se
        approx = [(p.f, p.xi, p.phi) for p in oracle.modal(ua, sa, wl.l, wl.orders, wl.fs)]
        df, dx, mm = _compare(exact, approx, sysm)
        print(f"12-channel record, 240 x 240, k = 40, p = 8, q = {q}: sigma rel max "
              f"{srel.max():.2e} (sigma_1 {srel[0]:.1e})")
        _report(f"  randomized vs Jacobi SVD (q = {q})", df, dx, mm)
        assert len(df) > 0 and df.max() < 0.01


@pytest.mark.gpu
def test_report_gpu_rsvd_vs_exact_svd():
    torch = pytest.importorskip("torch")
    from paper_2411_05510_amd import ssicov
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    wl = synth.WORKLOADS["bridge-180ch"]
    sysm, y = synth.make_record(wl)
    l = 30
    ys = np.ascontiguousarray(y[:l])
    # the generated modes as the first l channels see them
    sub = types.SimpleNamespace(freqs=sysm.freqs, shapes=sysm.shapes[:l])
    jb = 30
    ctx = ssicov.Context(0)
    try:
        yd = torch.from_numpy(ys).cuda()
        base = dict(fs=wl.fs, lags=[jb], order_min=2, order_max=200, order_step=2,
                    rank=200, oversample=20, power_iters=2, seed=wl.sketch_seed)
        outs = {}
        for name, svd in (("exact", ssicov.SVD_FULL), ("rsvd", ssicov.SVD_RANDOMIZED)):
            out = ctx.identify(yd, ssicov.Params(svd=svd, **base))
            ctx.synchronize()
            outs[name] = out
        orders = list(range(2, 201, 2))

        def per_order(out):
            return [(g["f"], g["xi"], g["phi"]) for g in (out.poles(0, i) for i in range(len(orders)))]

        se = outs["exact"].sigma[0].cpu().numpy()
        sa = outs["rsvd"].sigma[0].cpu().numpy()
        srel = np.abs(sa - se) / se
        df, dx, mm = _compare(per_order(outs["exact"]), per_order(outs["rsvd"]), sub)
        print(f"30 channels of the 180-channel record, j_b = 30 (900 x 900), k = 200, p = 20, "
              f"q = 2: sigma rel max {srel.max():.2e}, sigma_200 rel {srel[-1]:.2e}")
        _report("  randomized vs exact SVD (GPU)", df, dx, mm)
        assert len(df) > 0 and df.max() < 0.01
    finally:
        ctx.close()
