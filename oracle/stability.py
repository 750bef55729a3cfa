"""Plain FP64 checker of the stability analysis of a (3D) stabilization
diagram.

TEST INFRASTRUCTURE ONLY (see the package header).  Written from the paper:

  hard criteria   Section 2.1 end: a pole is discarded when its damping
                  ratio exceeds xi_max, its modal phase collinearity is at
                  most mpc_min, or its mean phase deviation is at least
                  mpd_max; both indicators are dimensionless in [0, 1]
  soft criteria   Section 2.1 end (consecutive orders) and Eq. (19) (3D:
                  consecutive orders or consecutive time lags): relative
                  differences |a - b| / max(a, b) of frequency and damping
                  and the MAC of the mode shapes against thresholds

Readings taken where the paper leaves details to its references:
  * MPC = ((Sxx - Syy)^2 + 4 Sxy^2) / (Sxx + Syy)^2 with Sxx = |Re phi|^2,
    Syy = |Im phi|^2, Sxy = Re phi . Im phi: the squared relative gap of the
    two eigenvalues of the 2 x 2 Gram matrix of [Re phi, Im phi]
    (1 for collinear components, 0 for circular scatter);
  * MPD = the |phi_a|-weighted mean angle between each component phi_a
    (a point of the complex plane) and the principal line through the origin
    (the dominant right singular vector of [Re phi, Im phi]), divided by
    pi/2 so that it lies in [0, 1];
  * damping must also be positive (a pole with xi <= 0 is not a structural
    mode);
  * "1 - MAC <= alpha_MAC" for the MAC criterion, and the order axis
    compares order m with the previous order of the sweep, the lag axis lag t
    with the previous lag of the sweep;
  * a neighbour counts only if it passes the hard criteria itself, and one
    neighbour must meet all three soft thresholds.
"""
from __future__ import annotations

import math
from typing import List, Sequence

import numpy as np

__all__ = ["mpc", "mpd", "mac", "hard_criteria", "stability"]

POLE_HC, POLE_STABLE_ORDER, POLE_STABLE_LAG, POLE_STABLE = 1, 2, 4, 8


def mpc(phi: np.ndarray) -> float:
    """Modal phase collinearity of one complex mode shape."""
    re = np.real(phi).astype(np.float64)
    im = np.imag(phi).astype(np.float64)
    sxx, syy, sxy = re @ re, im @ im, re @ im
    tr = sxx + syy
    if tr == 0.0:
        return 0.0
    return ((sxx - syy) ** 2 + 4.0 * sxy * sxy) / (tr * tr)


def mpd(phi: np.ndarray) -> float:
    """Mean phase deviation of one complex mode shape, in [0, 1]."""
    pts = np.stack([np.real(phi), np.imag(phi)], axis=1).astype(np.float64)
    r = np.hypot(pts[:, 0], pts[:, 1])
    if not np.any(r > 0):
        return 1.0
    # principal line: dominant right singular vector of the l x 2 matrix
    _, _, vt = np.linalg.svd(pts, full_matrices=False)
    d = vt[0]
    total, acc = 0.0, 0.0
    for a in range(pts.shape[0]):
        if r[a] > 0:
            c = min(1.0, abs(pts[a] @ d) / r[a])
            total += r[a]
            acc += r[a] * math.acos(c)
    return acc / total / (math.pi / 2.0)


def mac(a: np.ndarray, b: np.ndarray) -> float:
    """Modal assurance criterion |a^H b|^2 / ((a^H a)(b^H b))."""
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real))


def hard_criteria(xi: float, phi: np.ndarray, xi_max: float, mpc_min: float,
                  mpd_max: float) -> bool:
    return bool(0.0 < xi <= xi_max and mpc(phi) > mpc_min and mpd(phi) < mpd_max)


def _rel(a: float, b: float) -> float:
    return abs(a - b) / max(a, b)


def _matches(fi, xii, phii, fj, xij, phij, alpha_f, alpha_xi, alpha_mac) -> bool:
    return (_rel(fi, fj) <= alpha_f and _rel(xii, xij) <= alpha_xi
            and 1.0 - mac(phii, phij) <= alpha_mac)


def stability(diagram: Sequence[Sequence[dict]], xi_max: float = 0.10, mpc_min: float = 0.60,
              mpd_max: float = 0.50, alpha_f: float = 0.01, alpha_xi: float = 0.03,
              alpha_mac: float = 0.02) -> List[List[dict]]:
    """diagram[t][m] holds the poles of lag t, order m as a dict with arrays
    f, xi and phi (n_poles x l).  Returns per (t, m) a dict with mpc, mpd and
    flags (POLE_* bits) per pole."""
    T = len(diagram)
    out = []
    hc = []
    for t in range(T):
        row, hrow = [], []
        for m in range(len(diagram[t])):
            p = diagram[t][m]
            n = len(p["f"])
            c = np.array([mpc(p["phi"][i]) for i in range(n)])
            d = np.array([mpd(p["phi"][i]) for i in range(n)])
            h = np.array([0.0 < p["xi"][i] <= xi_max and c[i] > mpc_min and d[i] < mpd_max
                          for i in range(n)], dtype=bool)
            row.append({"mpc": c, "mpd": d, "flags": h.astype(np.uint8) * POLE_HC})
            hrow.append(h)
        out.append(row)
        hc.append(hrow)
    for t in range(T):
        for m in range(len(diagram[t])):
            p = diagram[t][m]
            for i in range(len(p["f"])):
                if not hc[t][m][i]:
                    continue
                axes = []
                for (tt, mm) in ((t, m - 1), (t - 1, m)):
                    ok = False
                    if tt >= 0 and mm >= 0:
                        q = diagram[tt][mm]
                        for j in range(len(q["f"])):
                            if hc[tt][mm][j] and _matches(p["f"][i], p["xi"][i], p["phi"][i],
                                                           q["f"][j], q["xi"][j], q["phi"][j],
                                                           alpha_f, alpha_xi, alpha_mac):
                                ok = True
                                break
                    axes.append(ok)
                fl = POLE_HC
                if axes[0]:
                    fl |= POLE_STABLE_ORDER
                if axes[1]:
                    fl |= POLE_STABLE_LAG
                if axes[0] or axes[1]:
                    fl |= POLE_STABLE
                out[t][m]["flags"][i] = fl
    return out
