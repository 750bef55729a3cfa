"""The allocation-free stability entry point (ssi_stability_noalloc) against
ssi_stability, called through the C ABI on the same poles: MPC, MPD and the
flags must be bit-identical (the same kernels run; only the scratch differs).
Two calls in a row, the second on a smaller diagram, so that the second call
runs on a scratch that still holds the first call's verdicts."""
import ctypes

import numpy as np
import pytest

from paper_2411_05510_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

REC = synth.Workload(name="noalloc", l=40, n=20000, fs=100.0, n_modes=6, f_range=(0.5, 20.0),
                     zeta_range=(0.005, 0.03), noise=0.05, lags=(10, 14, 18),
                     svd="randomized", rank=48, oversample=8, power_iters=1, order_min=2,
                     order_max=48, order_step=2, struct_seed=71, noise_seed=72, sketch_seed=73)


def _params(lags, order_max):
    from paper_2411_05510_amd import ssicov
    return ssicov.Params(fs=REC.fs, lags=list(lags), order_min=2, order_max=order_max,
                         order_step=2, svd=ssicov.SVD_RANDOMIZED, rank=48, oversample=8,
                         power_iters=1, seed=REC.sketch_seed)


def test_noalloc_matches_workspace_stability_twice():
    from paper_2411_05510_amd import ssicov
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("noalloc: identification l=40 n=20000 lags (10, 14, 18) / (10, 14)", flush=True)
    ctx = ssicov.Context(0)
    try:
        _, y = synth.make_record(REC)
        yd = torch.from_numpy(y).cuda()
        cases = [_params((10, 14, 18), 48), _params((10, 14), 30)]
        outs = [ctx.identify(yd, p) for p in cases]
        ctx.synchronize()
        for i, (p, out) in enumerate(zip(cases, outs)):
            ref = ctx.stability(out, REC.l)
            ctx.synchronize()
            # outputs pre-filled with a pattern so that unwritten slots show
            shape = ref[0].shape
            into = (torch.full(shape, -7.0, dtype=torch.float64, device="cuda"),
                    torch.full(shape, -7.0, dtype=torch.float64, device="cuda"),
                    torch.full(shape, 0xAB, dtype=torch.uint8, device="cuda"))
            got = ctx.stability(out, REC.l, noalloc=True, into=into)
            ctx.synchronize()
            for a, b, name in zip(ref, got, ("mpc", "mpd", "flags")):
                a, b = a.cpu().numpy(), b.cpu().numpy()
                assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), f"call {i}: {name}"
            n_stable = int(((got[2] & ssicov.POLE_STABLE) != 0).sum().item())
            print(f"noalloc call {i}: {shape[0]} lags x {shape[1]} slots, {n_stable} stable",
                  flush=True)
            assert int(out.count.sum().item()) > 0
    finally:
        ctx.close()


def test_noalloc_rejects_more_slots_than_the_scratch():
    from paper_2411_05510_amd import ssicov
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cap = int(ssicov.lib().ssi_stability_noalloc_max_slots())
    assert cap == 4 << 20
    ctx = ssicov.Context(0)
    try:
        # 2048 lags of orders 2..400: 2048 * 20000 slots > cap.  Only the
        # host-side size check runs; the buffers are never touched.
        lags = list(range(2, 2050))
        p = ssicov.Params(fs=100.0, lags=lags, order_min=2, order_max=400, order_step=2,
                          svd=ssicov.SVD_RANDOMIZED, rank=400, seed=1)
        dummy = torch.zeros(1, dtype=torch.float64, device="cuda")
        lay = {"n_lags": len(lags), "n_orders": 200, "pole_cap": ssicov.pole_offset(p, 200),
               "sigma_per_lag": 400, "l": 1, "n_corr": 1}
        assert lay["n_lags"] * lay["pole_cap"] > cap
        out = ssicov.Output(layout=lay, params=p, sigma=dummy, count=dummy, f=dummy, xi=dummy,
                            mu=dummy, phi=dummy, flags=dummy)
        with pytest.raises(ssicov.SSIError) as ei:
            ctx.stability(out, 1, noalloc=True, into=(dummy, dummy, dummy))
        assert ei.value.status == ssicov.SSI_EINVAL
        assert "exceed" in str(ei.value)
    finally:
        ctx.close()
