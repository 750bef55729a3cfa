"""GPU parity of the stability analysis (hard criteria, MPC, MPD and the
soft criteria along orders and lags of Eq. (19)) against the FP64 checker,
both evaluated on the same poles (the GPU identification's own output), so
the two take every decision on identical inputs in FP64.

Gates: MPC and MPD within 1e-12 absolute; flags bit-identical except where a
criterion value lies within 1e-9 of its threshold (summation order alone
can flip such a decision)."""
import numpy as np
import pytest

from oracle import stability as st
from paper_2411_05510_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MID = synth.Workload(name="mid3d", l=60, n=30000, fs=100.0, n_modes=8, f_range=(0.5, 20.0),
                     zeta_range=(0.005, 0.03), noise=0.05, lags=(12, 16, 20, 24),
                     svd="randomized", rank=60, oversample=10, power_iters=2, order_min=2,
                     order_max=60, order_step=2, struct_seed=91, noise_seed=92, sketch_seed=93)

TH = dict(xi_max=0.10, mpc_min=0.60, mpd_max=0.50, alpha_f=0.01, alpha_xi=0.03, alpha_mac=0.02)


def _near_threshold(p, q, i, j):
    """True if any soft criterion of pole pair (i of p, j of q) is within
    1e-9 of its threshold."""
    rel = lambda a, b: abs(a - b) / max(a, b)
    vals = [(rel(p["f"][i], q["f"][j]), TH["alpha_f"]),
            (rel(p["xi"][i], q["xi"][j]), TH["alpha_xi"]),
            (1 - st.mac(p["phi"][i], q["phi"][j]), TH["alpha_mac"])]
    return any(abs(v - t) < 1e-9 for v, t in vals)


def test_stability_matches_checker():
    from paper_2411_05510_amd import ssicov
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = ssicov.Context(0)
    _, y = synth.make_record(MID)
    p = ssicov.Params(fs=MID.fs, lags=list(MID.lags), order_min=2, order_max=60, order_step=2,
                      svd=ssicov.SVD_RANDOMIZED, rank=60, oversample=10, power_iters=2,
                      seed=MID.sketch_seed)
    out = ctx.identify(torch.from_numpy(y).cuda(), p)
    mpc, mpd, flags = ctx.stability(out, MID.l, **TH)
    ctx.synchronize()
    mpc, mpd, flags = mpc.cpu().numpy(), mpd.cpu().numpy(), flags.cpu().numpy()
    orders = p.orders
    diagram = [[out.poles(t, m) for m in range(len(orders))] for t in range(len(MID.lags))]
    ref = st.stability(diagram, **TH)
    n_stable = n_total = mism = 0
    for t in range(len(MID.lags)):
        for m in range(len(orders)):
            off = ssicov.pole_offset(p, m)
            cnt = len(diagram[t][m]["f"])
            sl = slice(off, off + cnt)
            np.testing.assert_allclose(mpc[t, sl], ref[t][m]["mpc"], atol=1e-12)
            np.testing.assert_allclose(mpd[t, sl], ref[t][m]["mpd"], atol=1e-12)
            g = flags[t, sl]
            r = ref[t][m]["flags"]
            for i in np.nonzero(g != r)[0]:
                # a flipped decision must sit on a threshold
                mism += 1
                near = False
                for (tt, mm) in ((t, m - 1), (t - 1, m)):
                    if tt < 0 or mm < 0:
                        continue
                    q = diagram[tt][mm]
                    near |= any(_near_threshold(diagram[t][m], q, i, j) for j in range(len(q["f"])))
                assert near, f"lag {t} order {orders[m]} pole {i}: gpu {g[i]} checker {r[i]}"
            # slots past the count are zero
            assert not flags[t, off + cnt: off + orders[m] // 2].any()
            n_stable += int((g & st.POLE_STABLE).astype(bool).sum())
            n_total += cnt
    print(f"stability: {n_total} poles, {n_stable} stable, {mism} threshold ties")
    assert n_stable > 0
    ctx.close()
