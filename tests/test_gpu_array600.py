"""The 600-channel configuration against the FP64 checker, at its full shape
on a shortened record: 600 channels, N = 20000 samples, lag j_b = 100 (a
60000 x 60000 Toeplitz matrix), randomized SVD k = 400, p = 40, q = 3, orders
2..400 step 4.  The checker's values come from tests/golden/make_array600.py
(checker only; T passed to its randomized SVD as a block-row operator), once
from the FP64 correlations and once from the same correlations rounded to
FP32.  The library's R stack is FP32, so the difference between the two
checker runs is how far rounding the input alone moves each result; the
gates below are the FP32-path tolerances (singular values rel 1e-4,
frequencies rel 1e-5), widened for a pole only where that rounding alone
moves the checker's own pole by more (four times its shift)."""
import os

import numpy as np
import pytest

from paper_2411_05510_amd import synth
from modelref import mac

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

REF = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "array600_n20000.npz")


@pytest.fixture(scope="module")
def ctx():
    from paper_2411_05510_amd import ssicov
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ssicov.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ref():
    return dict(np.load(REF))


def _split(ref, tag):
    cnt = ref[f"{tag}_count"]
    edges = np.concatenate([[0], np.cumsum(cnt)])
    return [{k: ref[f"{tag}_{k}"][edges[i]:edges[i + 1]] for k in ("f", "xi", "mu")}
            for i in range(len(cnt))]


def _physical(p, sysm):
    """Indices of checker poles within 1 % in frequency and 0.02 in damping of
    a mode of the generating system (nearest in frequency)."""
    out = []
    for r, fr in enumerate(sysm.freqs):
        if len(p["f"]) == 0:
            continue
        i = int(np.argmin(np.abs(p["f"] - fr)))
        if abs(p["f"][i] - fr) / fr < 0.01 and abs(p["xi"][i] - sysm.zetas[r]) < 0.02:
            out.append((i, r))
    return out


def _identify(ctx, prec, refine, n):
    from paper_2411_05510_amd import ssicov
    wl = synth.WORKLOADS["array-600ch"]
    sysm, y = synth.make_record(wl, n=n)
    p = ssicov.Params(fs=wl.fs, lags=list(wl.lags), order_min=wl.order_min,
                      order_max=wl.order_max, order_step=wl.order_step,
                      svd=ssicov.SVD_RANDOMIZED, rank=wl.rank, oversample=wl.oversample,
                      power_iters=wl.power_iters, seed=wl.sketch_seed, prec=prec, refine=refine)
    out = ctx.identify(torch.from_numpy(y).cuda(), p)
    ctx.synchronize()
    return wl, sysm, out


def test_array600_fp32_path_against_checker(ctx, ref):
    from paper_2411_05510_amd import ssicov
    wl, sysm, out = _identify(ctx, ssicov.PREC_FP32, 0, int(ref["n"]))
    s64, s32 = ref["r64_sigma"], ref["r32_sigma"]
    sig = out.sigma[0].cpu().numpy()
    keep = s64 >= 1e-3 * s64[0]
    srel = np.abs(sig[keep] - s64[keep]) / s64[keep]
    print(f"sigma rel max {srel.max():.2e} (input rounding alone "
          f"{(np.abs(s32[keep] - s64[keep]) / s64[keep]).max():.2e}) over {keep.sum()} values")
    assert srel.max() <= 1e-4
    p64, p32 = _split(ref, "r64"), _split(ref, "r32")
    n_phys = n_tight = 0
    worst = 0.0
    for oi, n in enumerate(wl.orders):
        g = out.poles(0, oi)
        assert g["flag"] == 0, f"order {n}"
        for i, r in _physical(p64[oi], sysm):
            mu = p64[oi]["mu"][i]
            j = int(np.argmin(np.abs(g["mu"] - mu)))
            j32 = int(np.argmin(np.abs(p32[oi]["mu"] - mu)))
            f = p64[oi]["f"][i]
            ef = abs(g["f"][j] - f) / f
            spread = abs(p32[oi]["f"][j32] - f) / f
            tol = max(1e-5, 4.0 * spread)
            worst = max(worst, ef / tol)
            assert ef <= tol, f"order {n}, mode {r}: f rel {ef:.2e} > {tol:.2e}"
            n_phys += 1
            n_tight += tol == 1e-5
    print(f"{n_phys} physical poles, {n_tight} at the 1e-5 gate, worst error / tolerance "
          f"{worst:.2f}")
    assert n_phys > 2000
    for n in (118, 238, 398):
        oi = list(wl.orders).index(n)
        g = out.poles(0, oi)
        idx, phi64, spread = ref[f"phi_idx_{n}"], ref[f"phi_{n}"], ref[f"phi_spread_{n}"]
        for q, i in enumerate(idx):
            mu = p64[oi]["mu"][i]
            j = int(np.argmin(np.abs(g["mu"] - mu)))
            m_gpu = mac(g["phi"][j], phi64[q])
            assert m_gpu >= 1.0 - max(1e-6, 4.0 * spread[q]), f"order {n}: MAC {m_gpu:.8f}"


def test_array600_fp8_against_checker(ctx, ref):
    """FP8 range finder with one full-precision refinement step, against the
    FP64 checker: the reduced-precision gates (f rel 1e-3, damping abs 2e-3,
    MAC 0.99) at every order up to 198 (MAC at order 118), and the leading
    2 x 60 singular values (the modes' subspace) within 1e-4.  The smaller
    singular values and the orders above 198, whose extra columns come from
    the noise part of the basis that the FP8 sketch and power steps resolve
    less well, are reported."""
    from paper_2411_05510_amd import ssicov
    wl, sysm, out = _identify(ctx, ssicov.PREC_FP8, 1, int(ref["n"]))
    s64 = ref["r64_sigma"]
    sig = out.sigma[0].cpu().numpy()
    keep = s64 >= 1e-3 * s64[0]
    srel = (np.abs(sig[keep] - s64[keep]) / s64[keep]).max()
    lead = 2 * wl.n_modes
    srel_lead = (np.abs(sig[:lead] - s64[:lead]) / s64[:lead]).max()
    p64 = _split(ref, "r64")
    lo, hi = [0.0, 0.0], [0.0, 0.0]
    for oi, n in enumerate(wl.orders):
        g = out.poles(0, oi)
        assert g["flag"] == 0, f"order {n}"
        for i, r in _physical(p64[oi], sysm):
            j = int(np.argmin(np.abs(g["mu"] - p64[oi]["mu"][i])))
            ef = abs(g["f"][j] - p64[oi]["f"][i]) / p64[oi]["f"][i]
            ex = abs(g["xi"][j] - p64[oi]["xi"][i])
            acc = lo if n <= 198 else hi
            acc[0], acc[1] = max(acc[0], ef), max(acc[1], ex)
    macs = {}
    for n in (118, 238, 398):
        oi = list(wl.orders).index(n)
        g = out.poles(0, oi)
        macs[n] = 1.0
        for q, i in enumerate(ref[f"phi_idx_{n}"]):
            j = int(np.argmin(np.abs(g["mu"] - p64[oi]["mu"][i])))
            macs[n] = min(macs[n], mac(g["phi"][j], ref[f"phi_{n}"][q]))
    print(f"fp8: sigma rel max {srel_lead:.2e} (leading {lead}), {srel:.2e} (all above 1e-3 "
          f"sigma_1); orders <= 198: f rel {lo[0]:.2e}, xi abs {lo[1]:.2e}, MAC at 118 "
          f"{macs[118]:.6f}; orders 202..398: f rel {hi[0]:.2e}, xi abs {hi[1]:.2e}, MAC at "
          f"238 / 398 {macs[238]:.6f} / {macs[398]:.6f}")
    assert srel_lead <= 1e-4
    assert lo[0] <= 1e-3 and lo[1] <= 2e-3 and macs[118] >= 0.99
