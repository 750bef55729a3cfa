"""C-ABI checks that need no GPU: exported symbols, host helpers, validation."""
import ctypes
import os
import re

import pytest

import oracle
from paper_2411_05510_amd import ssicov as S
from modelref import read_golden

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "include", "ssicov.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(ssi_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = S.lib()
    names = _declared()
    assert len(names) >= 20
    assert sorted(S.EXPORTED) == names
    for n in names:
        assert getattr(lib, n) is not None


def test_parameter_rules_match_worked_examples():
    g = {row[0]: row[1] for row in read_golden("parameter_rules.txt")}
    assert S.lag_rule(200.0, 5.319) == int(g["jb_10dof"])
    assert S.lag_rule(200.0, 5.319, 9.0) == int(g["jbmin_10dof"])
    assert S.lag_rule(40.0, 2.64) == int(g["jb_sf"])
    assert abs(S.tau(189, 200.0) - float(g["tau_10dof"])) < 1e-12
    assert abs(S.tau(76, 40.0) - float(g["tau_sf"])) < 1e-12
    assert S.default_rank(1890) == int(g["cols_10dof"])
    assert S.default_rank(8664) == oracle.default_rank(8664) == 2166
    for t in (100, 1000, 3420, 11400, 60000):
        assert S.default_rank(t) == oracle.default_rank(t)


def _p(**kw):
    base = dict(fs=100.0, lags=[60], order_min=2, order_max=200, order_step=2,
                svd=S.SVD_RANDOMIZED, rank=200, oversample=20, power_iters=2, seed=1)
    base.update(kw)
    return S.Params(**base)


def test_validate_accepts_the_bridge_workload():
    S.validate(_p(), 180, 180000)
    lay = S.output_layout(_p(), 180, 180000)
    assert lay["n_orders"] == 100 and lay["n_corr"] == 119
    assert lay["pole_cap"] == sum(n // 2 for n in range(2, 201, 2))
    assert S.pole_offset(_p(), 3) == 1 + 2 + 3
    assert S.workspace_estimate(_p(), 180, 180000) > 0


@pytest.mark.parametrize("kw,l,n", [
    (dict(rank=100), 180, 180000),                  # k < order_max
    (dict(lags=[1]), 180, 180000),                  # j_b < 2
    (dict(lags=[60, 50]), 180, 180000),             # not increasing
    (dict(lags=[60]), 180, 100),                    # 2 j_b - 1 >= N
    (dict(order_min=0), 180, 180000),
    (dict(order_step=0), 180, 180000),
    (dict(fs=0.0), 180, 180000),
    (dict(fs=float("nan")), 180, 180000),
    (dict(svd=7), 180, 180000),
    (dict(oversample=-1), 180, 180000),
    (dict(lags=[3], order_max=20, rank=20, oversample=0), 4, 1000),   # order > l (jb - 1)
    (dict(lags=[20], rank=20, oversample=0, order_max=20, svd=S.SVD_FULL), 300, 100000),
])
def test_validate_rejects(kw, l, n):
    with pytest.raises(S.SSIError) as ei:
        S.validate(_p(**kw), l, n)
    assert ei.value.status == S.SSI_EINVAL


def test_create_without_gpu_reports_device_error():
    torch = pytest.importorskip("torch")
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    st = S.lib().ssi_create(0, None, ctypes.byref(h))
    assert st == S.SSI_EDEVICE
    assert S.lib().ssi_last_error()


def test_validate_checks_the_caller_sketch():
    torch = pytest.importorskip("torch")
    om = torch.zeros((10800, 230), dtype=torch.float32)        # only its stride is read here
    S.validate(_p(omega=om), 180, 180000)
    with pytest.raises(S.SSIError) as ei:                      # ld < k + p
        S.validate(_p(omega=torch.zeros((10800, 200))), 180, 180000)
    assert ei.value.status == S.SSI_EINVAL
    with pytest.raises(S.SSIError) as ei:                      # full SVD takes no sketch
        S.validate(_p(omega=om, lags=[4], svd=S.SVD_FULL, order_max=20, rank=20), 180, 180000)
    assert ei.value.status == S.SSI_EINVAL


def test_result_accessors_reject_null():
    lib = S.lib()
    n = ctypes.c_int32()
    assert lib.ssi_result_dims(None, ctypes.byref(n), None, None) == S.SSI_EINVAL
    assert lib.ssi_result_poles(None, 0, 0, None, None, None, None, None, None,
                                None) == S.SSI_EINVAL
    assert lib.ssi_result_singular_values(None, 0, None, None) == S.SSI_EINVAL
    lib.ssi_result_free(None)
    assert lib.ssi_set_eig_max_sweeps(None, 3) == S.SSI_EINVAL
    assert lib.ssi_set_eig_workgroups(None, 0) == S.SSI_EINVAL
    assert lib.ssi_set_product_tile_rows(None, 64) == S.SSI_EINVAL
    assert b"NULL" in lib.ssi_last_error()
