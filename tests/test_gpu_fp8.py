"""GPU parity of the FP8 (block-scaled E4M3) range finder.

The sketch and power-iteration products quantize T and X to FP8 E4M3 along
the contraction index (32 elements per power-of-two scale) and accumulate in
FP32; the projection, every orthonormalization and everything after stay
FP64.  Gates:

* operands that the block-scaled FP8 format represents exactly and sums
  that FP32 holds exactly (small integers): the products are exact, so with
  q = 0 the whole randomized SVD equals the FP64 checker's to FP64 rounding
  (ragged shapes, unaligned leading dimensions and tails);
* general inputs: with q = 0 the singular values equal those of the
  checker's randomized SVD run on the checker's own FP8 quantization of T and
  of the sketch (oracle/fp8.py), to the FP32 accumulation's effect (2e-6
  sigma_1 / sigma_i relative);
* the identification of the 180-channel record with one full-precision
  refinement step (the form the mode is meant to run in) is held to the
  accuracy documented for the mode: singular values within 1e-6, the
  reduced-precision gates (f rel 1e-3, damping abs 2e-3, MAC 0.99) at every
  order up to 100, and physical poles within 1e-2 relative in frequency at
  every order.  A CPU model with the checker's quantizer gives the same
  picture: the gates hold up to order 104, and above it the poles move by up
  to 7e-3, as the checker's own poles do there when only the sketch seed
  changes.
"""
import numpy as np
import pytest

import oracle
from oracle import fp8
from oracle.ssicov_ref import qr_pos, jacobi_svd
from paper_2411_05510_amd import synth
from modelref import mac

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


def _rsvd_fp8(ctx, t32, k, p, q, omega=None, seed=7, pad=0):
    from paper_2411_05510_amd import ssicov
    m = t32.shape[0]
    tt = np.zeros((m, m + pad), dtype=np.float32)
    tt[:, :m] = t32
    om = _dev(omega) if omega is not None else None
    u, s = ctx.rsvd(_dev(tt), k, p, q, omega=om, seed=seed, prec=ssicov.PREC_FP8)
    ctx.synchronize()
    return u.cpu().numpy(), s.cpu().numpy()


@pytest.mark.parametrize("m,k,p,pad", [(701, 30, 7, 3), (640, 48, 16, 0), (97, 20, 5, 1),
                                       (1500, 200, 20, 2), (130, 17, 0, 0)])
def test_rsvd_fp8_exact_operands(ctx, m, k, p, pad):
    """Integer T (|t| <= 16) and integer Omega (|w| <= 4) are exact in E4M3
    under their block scales, and every sum is an integer below 2^24, so
    Y = T Omega is exact and with q = 0 the result equals the checker's."""
    rng = np.random.Generator(np.random.PCG64(m + 31 * k))
    t32 = rng.integers(-16, 17, size=(m, m)).astype(np.float32)
    om = rng.integers(-4, 5, size=(m, k + p)).astype(np.float32)
    u, s = _rsvd_fp8(ctx, t32, k, p, 0, omega=om, pad=pad)
    ur, sr = oracle.rsvd(t32.astype(np.float64), k, p, 0, om.astype(np.float64))
    np.testing.assert_allclose(s, sr, rtol=1e-10)
    gaps = np.abs(np.diff(sr)) / sr[0]
    for i in range(k - 1):
        if gaps[i] > 1e-3 and (i == 0 or gaps[i - 1] > 1e-3):
            assert abs(abs(u[:, i] @ ur[:, i]) - 1.0) < 1e-8


@pytest.mark.parametrize("m,k,p,pad,decay", [(701, 30, 7, 3, 0.8), (1200, 60, 12, 0, 0.9),
                                             (333, 40, 9, 1, 0.85)])
def test_rsvd_fp8_matches_checker_quantization(ctx, m, k, p, pad, decay):
    """General inputs, q = 0: the checker forms Y from its own FP8
    quantization of T and of a Gaussian sketch, then follows the randomized
    SVD (QR, P = Q^T T, Jacobi SVD of P).  Singular values above 1e-3
    sigma_1 agree to 2e-6 sigma_1 / sigma_i relative: the FP32 accumulation of
    Y, a few 1e-7 of sigma_1, turns the basis in direction i by that over
    sigma_i, and sigma_i of P = Q^T T moves with it (with q = 0 the basis is
    not an exact singular subspace).  One element quantized to a neighbouring
    E4M3 value would move Y by 2^-4 of its term, far more.  Against the FP64
    randomized SVD the difference is the FP8 rounding itself (reported; the
    leading singular value within 2^-4)."""
    t32 = synth.random_lowrank(m, m, k, seed=2 * m + k, decay=decay, noise=1e-4)
    # the sketch is handed over as FP32 values, so that both sides quantize
    # the same numbers (a difference of one FP32 rounding in an element next
    # to an E4M3 rounding boundary would move it by a whole FP8 step)
    om = oracle.sketch(23, m, k + p, 0).astype(np.float32).astype(np.float64)
    u, s = _rsvd_fp8(ctx, t32, k, p, 0, omega=om.astype(np.float32), pad=pad)
    t64 = t32.astype(np.float64)
    y = fp8.product(t32, om)
    qm = qr_pos(y)
    pm = qm.T @ t64
    r_p = np.linalg.qr(pm.T, mode="r")
    _, s_model, _ = jacobi_svd(r_p.T)
    s_model = s_model[:k]
    keep = s_model >= 1e-3 * s_model[0]
    rel = np.abs(s[keep] - s_model[keep]) / s_model[keep]
    bound = 2e-6 * s_model[0] / s_model[keep]
    worst = int(np.argmax(rel / bound))
    print(f"fp8 vs checker quantization: sigma rel err max {rel.max():.2e}; at sigma_{worst} "
          f"{rel[worst]:.2e} against bound {bound[worst]:.2e}")
    assert np.all(rel <= bound), "singular values off the checker's FP8 model"
    _, s64 = oracle.rsvd(t64, k, p, 0, om)
    rel64 = np.abs(s - s64) / s64
    print(f"  against the FP64 randomized SVD (report): sigma_1 {rel64[0]:.2e}, "
          f"max above 1e-2 sigma_1 {rel64[s64 >= 1e-2 * s64[0]].max():.2e}")
    assert rel64[0] <= 2.0 ** -4
    assert np.abs(u.T @ u - np.eye(k)).max() < 1e-8


def test_identify_bridge_fp8_refined(ctx):
    """The 180-channel record (lag 60, k = 200, q = 2) with FP8 products and
    one full-precision refinement step, against the FP64 checker with the
    same sketch."""
    from paper_2411_05510_amd import ssicov
    wl = synth.WORKLOADS["bridge-180ch"]
    sysm, y = synth.make_record(wl)
    res = oracle.identify(y, wl.fs, wl.lags, wl.orders, svd="randomized", rank=wl.rank,
                          oversample=wl.oversample, power_iters=wl.power_iters,
                          seed=wl.sketch_seed)[0]
    p = ssicov.Params(fs=wl.fs, lags=list(wl.lags), order_min=wl.order_min,
                      order_max=wl.order_max, order_step=wl.order_step,
                      svd=ssicov.SVD_RANDOMIZED, rank=wl.rank, oversample=wl.oversample,
                      power_iters=wl.power_iters, seed=wl.sketch_seed, prec=ssicov.PREC_FP8,
                      refine=1)
    out = ctx.identify(_dev(y), p)
    ctx.synchronize()
    sig = out.sigma[0].cpu().numpy()
    keep = res.sigma >= 1e-2 * res.sigma[0]
    srel = float((np.abs(sig[keep] - res.sigma[keep]) / res.sigma[keep]).max())
    worst_f, n_phys = 0.0, 0
    low = [0.0, 0.0, 1.0]                       # orders <= 100: f, xi, MAC
    for oi, n in enumerate(wl.orders):
        g = out.poles(0, oi)
        assert g["flag"] == 0
        ref = res.poles[oi]
        for r, fr in enumerate(sysm.freqs):
            if len(ref) == 0:
                continue
            i = int(np.argmin(np.abs(ref.f - fr)))
            if abs(ref.f[i] - fr) / fr >= 0.01 or mac(ref.phi[i], sysm.shapes[:, r]) < 0.9:
                continue
            j = int(np.argmin(np.abs(g["f"] - ref.f[i])))
            ef = abs(g["f"][j] - ref.f[i]) / ref.f[i]
            worst_f = max(worst_f, ef)
            if n <= 100:
                low[0] = max(low[0], ef)
                low[1] = max(low[1], abs(g["xi"][j] - ref.xi[i]))
                low[2] = min(low[2], mac(g["phi"][j], ref.phi[i]))
            n_phys += 1
    print(f"bridge fp8 refine 1: sigma rel max {srel:.2e}; {n_phys} physical poles; orders "
          f"<= 100: max f rel {low[0]:.2e}, max xi abs {low[1]:.2e}, min MAC {low[2]:.6f}; "
          f"all orders: max f rel {worst_f:.2e}")
    assert n_phys > 1000
    assert srel <= 1e-6
    assert low[0] <= 1e-3 and low[1] <= 2e-3 and low[2] >= 0.99
    assert worst_f <= 1e-2
