"""GPU parity of the stage entry points against the FP64 checker."""
import numpy as np
import pytest

import oracle
from paper_2411_05510_amd import synth

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


def _corr_check(ctx, y, n_corr, tol=1e-5, fwd_tol=1e-6):
    """Correlated records: relative Frobenius error per lag <= tol.  Every
    entry: |error| <= fwd_tol * rms_a * rms_b, the scale of the forward error
    bound of a dot product (|sum x y| <= |x| |y|), which also covers
    uncorrelated inputs whose R_j are near-zero sums."""
    r = ctx.correlate(_dev(y), n_corr)
    ctx.synchronize()
    got = r.cpu().numpy().astype(np.float64)
    ref = oracle.correlations(y, n_corr)
    rms = np.sqrt(np.mean(y.astype(np.float64) ** 2, axis=1))
    scale = np.outer(rms, rms)
    bad = np.abs(got - ref) > fwd_tol * scale
    assert not bad.any(), f"{bad.sum()} entries beyond {fwd_tol} * rms_a rms_b"
    if tol is not None:
        for j in range(n_corr):
            den = max(np.linalg.norm(ref[j]), 1e-300)
            err = np.linalg.norm(got[j] - ref[j]) / den
            assert err <= tol, f"lag {j + 1}: rel Frobenius error {err:.3e}"
    return got, ref


# ------------------------------------------------------------ correlations
MODES = pytest.mark.parametrize("mode", [0, 1, 2], ids=["fp32", "bf16x6", "f16x3"])


@MODES
def test_correlate_small_record(ctx, mode):
    ctx.set_corr_mode(mode)
    wl = synth.WORKLOADS["small-full-svd"]
    _, y = synth.make_record(wl)
    _corr_check(ctx, y, 2 * wl.lags[0] - 1)


@pytest.mark.parametrize("l,n,L", [(37, 5003, 23), (5, 777, 60), (1, 2, 1), (1, 3000, 300),
                                   (70, 4099, 3), (3, 129, 128)])
@MODES
def test_correlate_ragged(ctx, l, n, L, mode):
    ctx.set_corr_mode(mode)
    y = synth.random_matrix(l, n, seed=l * 1000 + L)
    _corr_check(ctx, y, L, tol=None)


@MODES
def test_correlate_bridge_record_sampled(ctx, mode):
    """Full 180-channel, 30-minute record, 119 lags; sampled channel pairs."""
    ctx.set_corr_mode(mode)
    wl = synth.WORKLOADS["bridge-180ch"]
    _, y = synth.make_record(wl)
    L = 2 * wl.lags[0] - 1
    r = ctx.correlate(_dev(y), L)
    ctx.synchronize()
    got = r.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(0)
    rms = np.sqrt(np.mean(y.astype(np.float64) ** 2, axis=1))
    pairs = [(0, 0), (179, 179), (0, 179), (179, 0), (63, 64), (64, 63), (127, 128)]
    pairs += [tuple(int(v) for v in rng.integers(0, 180, 2)) for _ in range(9)]
    for a, b in pairs:
        ref = oracle.correlations(y[[a, b]], L)          # 2-channel checker run
        for (ia, ib), (ga, gb) in (((0, 1), (a, b)), ((1, 0), (b, a)), ((0, 0), (a, a))):
            err = np.max(np.abs(got[:, ga, gb] - ref[:, ia, ib]))
            assert err <= 1e-6 * rms[ga] * rms[gb], (a, b, err)
            rel = np.linalg.norm(got[:, ga, gb] - ref[:, ia, ib]) / np.linalg.norm(ref[:, ia, ib])
            assert rel <= 1e-5, (a, b, rel)


@MODES
def test_correlate_deterministic(ctx, mode):
    ctx.set_corr_mode(mode)
    y = synth.random_matrix(20, 9000, seed=3)
    yd = _dev(y)
    r1 = ctx.correlate(yd, 40).clone()
    r2 = ctx.correlate(yd, 40)
    ctx.synchronize()
    assert torch.equal(r1, r2)


def test_correlate_modes_agree_exact_inputs(ctx):
    """Samples with at most 8 significant bits (small integers times a power of
    two): the BF16 split is hi alone, the FP16 split of the scaled sample is hi
    alone, every product is exact in each path, and sums below 2^24 (after the
    power-of-two channel scale) are exact in FP32, so all paths return
    identical stacks."""
    rng = np.random.default_rng(5)
    y = (rng.integers(-15, 16, size=(19, 3000)) * 0.25).astype(np.float32)
    y[7] *= 2.0 ** -40            # channels of very different scale
    y[11] *= 2.0 ** 30
    out = []
    for mode in (0, 1, 2):
        ctx.set_corr_mode(mode)
        out.append(ctx.correlate(_dev(y), 25).cpu().numpy())
    ctx.set_corr_mode(2)
    ref = oracle.correlations(y, 25)
    assert np.array_equal(out[0], out[1])
    assert np.array_equal(out[0], out[2])
    # the exact sums are scaled by 1/N and rounded to FP32 once
    np.testing.assert_allclose(out[1].astype(np.float64), ref, rtol=2.0 ** -23, atol=0)


@MODES
def test_correlate_channel_scales(ctx, mode):
    """Channels far outside the FP16 range (1e15 and 1e-15 times a unit
    record), an all-zero channel and a ragged size: every mode matches the
    checker to 1e-6 rms_a rms_b per entry, and the zero channel's
    correlations are exactly zero.  Without the per-channel power-of-two
    scale the FP16 parts of the large channel would overflow and those of the
    small one underflow."""
    y = synth.random_matrix(9, 4001, seed=17).astype(np.float64)
    y[2] *= 1e15
    y[5] *= 1e-15
    y[7] = 0.0
    y = y.astype(np.float32)
    L = 13
    ctx.set_corr_mode(mode)
    try:
        got = ctx.correlate(_dev(y), L).cpu().numpy().astype(np.float64)
        ctx.synchronize()
    finally:
        ctx.set_corr_mode(2)
    ref = oracle.correlations(y, L)
    rms = np.sqrt(np.mean(y.astype(np.float64) ** 2, axis=1))
    scale = np.outer(rms, rms)[None]
    nz = scale > 0
    err = np.abs(got - ref)
    assert np.all(np.isfinite(got))
    assert (err[np.broadcast_to(nz, err.shape)] / np.broadcast_to(scale, err.shape)[
        np.broadcast_to(nz, err.shape)]).max() <= 1e-6
    assert np.all(got[:, 7, :] == 0.0) and np.all(got[:, :, 7] == 0.0)


# ---------------------------------------------------------------- Toeplitz
@pytest.mark.parametrize("l,jb,pad", [(12, 20, 0), (7, 9, 3), (180, 60, 16), (4, 2, 0),
                                      (1, 5, 1)])
def test_toeplitz_bit_exact(ctx, l, jb, pad):
    r = synth.random_stack(2 * jb - 1, l, seed=l + jb)
    m = jb * l
    t = ctx.toeplitz(_dev(r.reshape(2 * jb - 1, l, l)), jb, ldt=m + pad)
    ctx.synchronize()
    got = t.cpu().numpy()[:, :m].astype(np.float64)
    ref = oracle.toeplitz(r.astype(np.float64), jb)
    assert np.array_equal(got, ref)


def test_toeplitz_uses_leading_blocks_only(ctx):
    # more blocks than needed: only R_1..R_{2jb-1} are read
    l, jb = 8, 5
    r = synth.random_stack(3 * jb, l, seed=9)
    t = ctx.toeplitz(_dev(r), jb)
    ctx.synchronize()
    ref = oracle.toeplitz(r.astype(np.float64), jb)
    assert np.array_equal(t.cpu().numpy().astype(np.float64), ref)


# ------------------------------------------------------------------ sketch
@pytest.mark.parametrize("m,ell,stream,seed", [(101, 37, 0, 7), (10800, 220, 0, 3002),
                                               (64, 3, 5, 2 ** 40 + 3)])
def test_sketch_matches_checker(ctx, m, ell, stream, seed):
    om = ctx.sketch(seed, stream, m, ell)
    ctx.synchronize()
    got = om.cpu().numpy().astype(np.float64)
    ref = oracle.sketch(seed, m, ell, stream)
    # FP64 Box-Muller on both sides, rounded to FP32 on the device
    assert np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1.0)) < 2.0 ** -23
