"""Closed-form model quantities used to pin the checker (tests only).

These are properties of the state-space models that generate the inputs, not
steps of the identification: exact output correlations of a model
(R_j = C A^{j-1} G with G = A Sigma C^T, Section 2.1, Eq. (7)) and the
10-storey shear frame of Section 3.1.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.linalg as sla

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def modal_correlations(system, count: int) -> np.ndarray:
    """Exact R_1..R_count of the generator's modal model with unit stationary
    variance per mode: R_j = sum_r Re(mu_r^j) phi_r phi_r^T."""
    return np.stack([(system.shapes * np.real(system.mu ** j)) @ system.shapes.T
                     for j in range(1, count + 1)])


def shear_frame(floors: int = 10, mass: float = 100.0, k: float = 5.0e6,
                xi: float = 0.01, modes=(0, 3)):
    """Mass, stiffness and Rayleigh damping of the shear frame of Section 3.1."""
    m = np.eye(floors) * mass
    kk = np.zeros((floors, floors))
    for i in range(floors):
        kk[i, i] = k + (k if i < floors - 1 else 0.0)
        if i < floors - 1:
            kk[i, i + 1] = kk[i + 1, i] = -k
    w = np.sqrt(sla.eigh(kk, m, eigvals_only=True))
    i, j = modes
    a0, a1 = np.linalg.solve([[1 / (2 * w[i]), w[i] / 2], [1 / (2 * w[j]), w[j] / 2]],
                             [xi, xi])
    return m, kk, a0 * m + a1 * kk


def frame_state_space(fs: float = 200.0):
    """Discrete state-space (A, C, G) of the frame with acceleration outputs and
    white floor forces; G = A Sigma C^T with Sigma the stationary covariance."""
    m, kk, cd = shear_frame()
    n = m.shape[0]
    minv = np.linalg.inv(m)
    ac = np.block([[np.zeros((n, n)), np.eye(n)], [-minv @ kk, -minv @ cd]])
    cc = np.hstack([-minv @ kk, -minv @ cd])
    a = sla.expm(ac / fs)
    bq = np.vstack([np.zeros((n, n)), minv])
    q = bq @ bq.T * 1.0e6 / fs + 1e-12 * np.eye(2 * n)
    sigma = sla.solve_discrete_lyapunov(a, q)
    return a, cc, a @ sigma @ cc.T


def state_space_correlations(a, c, g, count: int) -> np.ndarray:
    """Exact R_j = C A^{j-1} G, j = 1..count."""
    out = []
    p = np.eye(a.shape[0])
    for _ in range(count):
        out.append(c @ p @ g)
        p = p @ a
    return np.stack(out)


def read_golden(name: str):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def mac(a: np.ndarray, b: np.ndarray) -> float:
    """Modal assurance criterion |a^H b|^2 / (|a|^2 |b|^2)."""
    num = abs(np.vdot(a, b)) ** 2
    return float(num / (np.vdot(a, a).real * np.vdot(b, b).real))
