"""Pins of the stability-analysis checker (oracle/stability.py) against
closed forms, invariants, an independent eigenvalue formula and hand-built
diagrams."""
import math

import numpy as np

from oracle import stability as st


def test_mpc_closed_forms():
    rng = np.random.default_rng(3)
    a = rng.standard_normal(25)
    assert st.mpc(a.astype(complex)) == 1.0                       # real mode
    assert abs(st.mpc((0.3 - 1.7j) * a) - 1.0) < 1e-14            # rotated real mode
    # orthogonal real and imaginary parts of equal norm: no collinearity
    b = rng.standard_normal(25)
    b -= (b @ a) / (a @ a) * a
    b *= np.linalg.norm(a) / np.linalg.norm(b)
    assert abs(st.mpc(a + 1j * b)) < 1e-14


def test_mpc_equals_eigenvalue_gap():
    """MPC is the squared relative gap of the eigenvalues of the Gram matrix
    of [Re phi, Im phi] (computed here by LAPACK)."""
    rng = np.random.default_rng(4)
    for _ in range(20):
        phi = rng.standard_normal(40) + 1j * rng.standard_normal(40) * rng.uniform(0, 2)
        x = np.stack([phi.real, phi.imag], axis=1)
        lam = np.linalg.eigvalsh(x.T @ x)
        want = ((lam[1] - lam[0]) / (lam[1] + lam[0])) ** 2
        assert abs(st.mpc(phi) - want) < 1e-12


def test_mpd_closed_forms():
    rng = np.random.default_rng(5)
    a = rng.standard_normal(30)
    assert st.mpd(a.astype(complex)) < 1e-7                        # real mode
    assert st.mpd((2.0 + 0.5j) * a) < 1e-7                         # rotation invariant
    # equal-magnitude components at +/- alpha around the real axis: the
    # principal line is the real axis and every component deviates by alpha
    for alpha in (0.1, 0.4, 0.7):
        phi = np.array([np.exp(1j * alpha), np.exp(-1j * alpha)] * 6)
        assert abs(st.mpd(phi) - alpha / (math.pi / 2)) < 1e-12
        assert abs(st.mpd(np.exp(0.9j) * phi) - alpha / (math.pi / 2)) < 1e-12
    # circular scatter of equal magnitudes: mean deviation pi/4 -> 0.5
    ang = np.linspace(0, 2 * np.pi, 64, endpoint=False)
    assert abs(st.mpd(np.exp(1j * ang)) - 0.5) < 1e-3


def _pole(f, xi, phi):
    return {"f": np.array(f, float), "xi": np.array(xi, float), "phi": np.array(phi, complex)}


def test_soft_criteria_hand_diagram():
    """Two lags x three orders built by hand; thresholds alpha_f = 1 %,
    alpha_xi = 3 %, alpha_MAC = 2 %."""
    e1 = np.array([1.0, 0.0, 0.0])
    e2 = np.array([0.0, 1.0, 0.0])
    mix = np.array([1.0, 0.3, 0.0])        # MAC with e1 = 1/1.09 ~ 0.917
    d = [
        [_pole([2.0], [0.02], [e1]),                       # t0 m0
         _pole([2.01, 5.0], [0.0203, 0.02], [e1, e2]),      # t0 m1: 0.5 %, 1.5 % -> stable(order)
         _pole([2.05, 5.0], [0.02, 0.05], [e1, e2])],       # t0 m2: f 2 % off; xi 150 % off
        [_pole([2.0], [0.02], [mix]),                       # t1 m0: MAC fails vs t0 m0
         _pole([2.01, 5.02], [0.0203, 0.02], [e1, e2]),     # t1 m1: lag match (same pole at t0)
         _pole([2.05, 5.0], [0.02, 0.2], [e1, e2])],        # t1 m2: xi 20 % fails hard criteria
    ]
    r = st.stability(d)
    HC, SO, SL, S = st.POLE_HC, st.POLE_STABLE_ORDER, st.POLE_STABLE_LAG, st.POLE_STABLE
    assert list(r[0][0]["flags"]) == [HC]
    assert list(r[0][1]["flags"]) == [HC | SO | S, HC]
    assert list(r[0][2]["flags"]) == [HC, HC]
    assert list(r[1][0]["flags"]) == [HC]
    # pole 2.01 of t1 m1: order neighbour is `mix` (MAC fails), lag neighbour 2.01 matches
    assert list(r[1][1]["flags"]) == [HC | SL | S, HC | SL | S]
    # 2.05 at t1 m2: lag neighbour 2.05 at t0 m2 matches; 5.0 with xi 0.2 fails HC
    assert list(r[1][2]["flags"]) == [HC | SL | S, 0]


def test_hard_criteria_thresholds():
    a = np.array([1.0, -2.0, 0.5], complex)
    assert st.hard_criteria(0.05, a, 0.10, 0.6, 0.5)
    assert not st.hard_criteria(0.11, a, 0.10, 0.6, 0.5)
    assert not st.hard_criteria(-0.01, a, 0.10, 0.6, 0.5)
    circ = np.exp(1j * np.linspace(0, 2 * np.pi, 16, endpoint=False))
    assert not st.hard_criteria(0.05, circ, 0.10, 0.6, 0.5)        # MPC ~ 0
