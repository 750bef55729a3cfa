"""GPU parity of the reduced-precision (BF16) range finder.

The sketch and power-iteration products round T and X to BF16 (nearest
even) and accumulate in FP32; the projection, every orthonormalization and
everything after stay FP64.  Gates:

* operands that BF16 represents exactly and sums that FP32 holds exactly
  (small integers): the BF16 products are exact, so with q = 0 the whole
  randomized SVD equals the FP64 checker's to FP64 rounding;
* general inputs: singular values within 1e-3 relative of the checker for
  sigma_i >= 1e-2 sigma_1 (BF16 keeps 8 significant bits, a relative
  rounding of 2^-9 per operand; the exact projection turns that into a
  perturbation of the basis only), and the leading subspace within the
  same error scaled by the inverse relative gap;
* the whole identification of the 180-channel record with the split-BF16
  range finder: physical poles within f rel 1e-3, damping abs 2e-3 and MAC
  0.99 of the FP64 checker at every order; plain BF16 is held to the
  accuracy it is documented to have (it is not offered at equal accuracy).
"""
import numpy as np
import pytest

import oracle
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


def _rsvd_bf16(ctx, t32, k, p, q, omega=None, seed=7, pad=0, prec=None):
    from paper_2411_05510_amd import ssicov
    m = t32.shape[0]
    tt = np.zeros((m, m + pad), dtype=np.float32)
    tt[:, :m] = t32
    om = _dev(omega) if omega is not None else None
    u, s = ctx.rsvd(_dev(tt), k, p, q, omega=om, seed=seed,
                    prec=ssicov.PREC_BF16 if prec is None else prec)
    ctx.synchronize()
    return u.cpu().numpy(), s.cpu().numpy()


@pytest.mark.parametrize("mode", ["bf16", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("m,k,p,pad", [(701, 30, 7, 3), (640, 48, 16, 0), (97, 20, 5, 1),
                                       (1500, 200, 20, 2)])
def test_rsvd_bf16_exact_operands(ctx, m, k, p, pad, mode):
    """Integer T (|t| <= 128) and integer Omega (|w| <= 4): BF16 holds every
    operand and FP32 every partial sum, so Y = T Omega is exact and with q = 0
    the result equals the checker's randomized SVD to FP64 rounding.  Ragged
    m, ell and leading dimensions cover the unaligned loads and the tails."""
    rng = np.random.Generator(np.random.PCG64(m + 17 * k))
    t32 = rng.integers(-128, 129, size=(m, m)).astype(np.float32)
    om = rng.integers(-4, 5, size=(m, k + p)).astype(np.float32)
    from paper_2411_05510_amd import ssicov
    prec = {"bf16": ssicov.PREC_BF16, "bf16x3": ssicov.PREC_BF16X3,
            "bf16x6": ssicov.PREC_BF16X6}[mode]
    u, s = _rsvd_bf16(ctx, t32, k, p, 0, omega=om, pad=pad, prec=prec)
    ur, sr = oracle.rsvd(t32.astype(np.float64), k, p, 0, om.astype(np.float64))
    np.testing.assert_allclose(s, sr, rtol=1e-10)
    # same left singular vectors up to sign where the spectrum is separated
    gaps = np.abs(np.diff(sr)) / sr[0]
    for i in range(k - 1):
        if gaps[i] > 1e-3 and (i == 0 or gaps[i - 1] > 1e-3):
            assert abs(abs(u[:, i] @ ur[:, i]) - 1.0) < 1e-8


@pytest.mark.parametrize("m,k,p,q,pad,decay", [(701, 30, 7, 2, 3, 0.8), (1200, 60, 12, 1, 0, 0.9),
                                               (330, 40, 9, 3, 1, 0.8)])
def test_rsvd_bf16_accuracy(ctx, m, k, p, q, pad, decay):
    """Low rank plus noise, Philox sketch, power iterations through both
    product orientations (T X and T^T X)."""
    t32 = synth.random_lowrank(m, m, k, seed=m + k, decay=decay, noise=1e-5)
    u, s = _rsvd_bf16(ctx, t32, k, p, q, seed=11, pad=pad)
    ur, sr = oracle.rsvd(t32.astype(np.float64), k, p, q, oracle.sketch(11, m, k + p, 0))
    keep = sr >= 1e-2 * sr[0]
    rel = np.abs(s[keep] - sr[keep]) / sr[keep]
    assert rel.max() <= 1e-3, f"max sigma rel err {rel.max():.3e}"
    assert np.abs(u.T @ u - np.eye(k)).max() < 1e-8
    c = k // 2
    rel_gap = (sr[c - 1] - sr[c]) / sr[0]
    gap = np.linalg.norm(u[:, :c] - ur[:, :c] @ (ur[:, :c].T @ u[:, :c]), 2)
    assert gap <= 1e-3 / min(1.0, rel_gap), f"subspace gap {gap:.3e}"


@pytest.fixture(scope="module")
def bridge():
    """The 180-channel record and the FP64 checker's identification of it."""
    wl = synth.WORKLOADS["bridge-180ch"]
    sysm, y = synth.make_record(wl)
    res = oracle.identify(y, wl.fs, wl.lags, wl.orders, svd="randomized", rank=wl.rank,
                          oversample=wl.oversample, power_iters=wl.power_iters,
                          seed=wl.sketch_seed)[0]
    return wl, sysm, y, res


def _bridge_errors(ctx, bridge, prec, refine=0):
    """Per-order worst errors of the physical poles of the 180-channel record
    identified with range-finder products `prec`, against the FP64 checker
    (same record, same Philox sketch)."""
    from paper_2411_05510_amd import ssicov
    wl, sysm, y, res = bridge
    p = ssicov.Params(fs=wl.fs, lags=list(wl.lags), order_min=wl.order_min,
                      order_max=wl.order_max, order_step=wl.order_step,
                      svd=ssicov.SVD_RANDOMIZED, rank=wl.rank, oversample=wl.oversample,
                      power_iters=wl.power_iters, seed=wl.sketch_seed, prec=prec, refine=refine)
    out = ctx.identify(_dev(y), p)
    ctx.synchronize()
    sig = out.sigma[0].cpu().numpy()
    keep = res.sigma >= 1e-2 * res.sigma[0]
    srel = float((np.abs(sig[keep] - res.sigma[keep]) / res.sigma[keep]).max())
    per_order = {}
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
            e = per_order.setdefault(n, [0.0, 0.0, 1.0, 0])
            e[0] = max(e[0], abs(g["f"][j] - ref.f[i]) / ref.f[i])
            e[1] = max(e[1], abs(g["xi"][j] - ref.xi[i]))
            e[2] = min(e[2], mac(g["phi"][j], ref.phi[i]))
            e[3] += 1
    return srel, per_order


@pytest.mark.parametrize("mode,refine", [("bf16x3", 0), ("bf16x3", 1), ("bf16x6", 0)])
def test_identify_bridge_split_bf16(ctx, bridge, mode, refine):
    """The split-BF16 range finders on the 180-channel record (lag 60), with
    and without the full-precision refinement step: physical poles at every
    one of the 100 orders within f rel 1e-3, damping abs 2e-3 and MAC 0.99 of
    the FP64 checker (the 3D sweep holds the refined forms to the same gates
    at lags 20 and 100)."""
    from paper_2411_05510_amd import ssicov
    prec = {"bf16x3": ssicov.PREC_BF16X3, "bf16x6": ssicov.PREC_BF16X6}[mode]
    srel, per_order = _bridge_errors(ctx, bridge, prec, refine)
    wl = bridge[0]
    f = max(e[0] for e in per_order.values())
    x = max(e[1] for e in per_order.values())
    m = min(e[2] for e in per_order.values())
    n = sum(e[3] for e in per_order.values())
    print(f"bridge {mode} refine {refine}: sigma rel max {srel:.2e}; {len(per_order)} orders, {n} physical "
          f"poles, max f rel {f:.2e}, max xi abs {x:.2e}, min MAC {m:.6f}")
    assert len(per_order) >= len(wl.orders) - 5     # the lowest orders hold no physical pole
    assert srel <= 1e-6
    assert f <= 1e-3 and x <= 2e-3 and m >= 0.99


def test_identify_bridge_plain_bf16_accuracy(ctx, bridge):
    """Plain BF16 operands (SSI_PREC_BF16) are a lower-accuracy mode, not an
    equal-accuracy one: BF16 keeps 8 significant bits, and the randomized
    SVD's singular vectors at orders near k depend on the products to far
    better than that (the FP64 checker's own poles at orders 160 and up move
    by up to 6e-3 when only the sketch seed changes), and a full-precision
    refinement step does not recover them (measured with refine = 1, as
    here: 3e-3 to 6e-3 at lags 20..100).  What the mode does
    meet, and what this test holds it to: singular values within 1e-6
    relative above 1e-2 sigma_1, the reduced-precision gates at every order
    up to 84 (sigma_n above 2^-9 sigma_1 on this record), and poles within
    1e-2 relative in frequency at every order."""
    from paper_2411_05510_amd import ssicov
    srel, per_order = _bridge_errors(ctx, bridge, ssicov.PREC_BF16, refine=1)
    low = [e for n, e in per_order.items() if n <= 84]
    f_all = max(e[0] for e in per_order.values())
    print(f"bridge bf16: sigma rel max {srel:.2e}; orders <= 84: max f rel "
          f"{max(e[0] for e in low):.2e}, max xi abs {max(e[1] for e in low):.2e}, min MAC "
          f"{min(e[2] for e in low):.6f}; all orders: max f rel {f_all:.2e}")
    assert srel <= 1e-6
    assert max(e[0] for e in low) <= 1e-3
    assert max(e[1] for e in low) <= 2e-3
    assert min(e[2] for e in low) >= 0.99
    assert f_all <= 1e-2
