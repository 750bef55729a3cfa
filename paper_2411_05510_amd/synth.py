"""Seeded synthetic monitoring records (inputs only).

This module produces the inputs that both the identification library and its
independent checker consume: multichannel output records drawn from the
discrete stochastic state-space model of Eq. (5) (state recursion driven by
white process noise, outputs observed through C with additive white
measurement noise), plus seeded test matrices and Gaussian sketch matrices for
stage-level checks.  It performs no step of the identification itself
(no correlation, Toeplitz assembly, decomposition, least squares or
eigen-analysis); the only modal arithmetic here is the forward map from drawn
(f, zeta) to the discrete poles that drive the simulation (Eq. (3) and
mu = exp(lambda * dt)).

Model used for every workload
-----------------------------
* n modes, each a 2-state block of A that acts as multiplication by the complex
  pole mu_r on z_r = x_{2r} + i x_{2r+1}  (so A is block-diagonal with
  [[Re mu, -Im mu], [Im mu, Re mu]] blocks, a real-valued form of Eq. (2)).
* C[:, 2r] = phi_r (i.i.d. N(0, 1) entries), C[:, 2r+1] = 0.
* Process noise w_r ~ N(0, (1 - |mu_r|^2) I_2) so that each mode has unit
  stationary variance per state component; x_0 is drawn from the stationary law.
* Measurement noise v_a ~ N(0, (eta * rms_a)^2), rms_a = RMS of the clean
  output of channel a.
* y is returned float32, channel-major (l x N).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np

__all__ = [
    "ModalSystem", "draw_system", "simulate", "Workload", "WORKLOADS",
    "make_record", "random_matrix", "random_lowrank", "random_stack",
]


@dataclasses.dataclass
class ModalSystem:
    """A drawn structure: sampling rate, modal parameters and mode shapes."""
    fs: float
    freqs: np.ndarray      # (n_modes,) Hz, ascending
    zetas: np.ndarray      # (n_modes,) damping ratios
    shapes: np.ndarray     # (l, n_modes) real mode shapes
    mu: np.ndarray         # (n_modes,) discrete poles, Im > 0

    @property
    def l(self) -> int:
        return int(self.shapes.shape[0])

    @property
    def n_modes(self) -> int:
        return int(self.freqs.shape[0])


def _poles(freqs: np.ndarray, zetas: np.ndarray, fs: float) -> np.ndarray:
    # Eq. (3): lambda = -zeta*omega + i*omega*sqrt(1 - zeta^2); discrete pole
    # of the sampled system is exp(lambda / fs).
    omega = 2.0 * math.pi * freqs
    lam = -zetas * omega + 1j * omega * np.sqrt(1.0 - zetas ** 2)
    return np.exp(lam / fs)


def draw_system(l: int, n_modes: int, f_range: Sequence[float],
                zeta_range: Sequence[float], fs: float, seed: int,
                min_rel_spacing: float = 0.01) -> ModalSystem:
    """Draw modal parameters: f ~ U[f_range], zeta ~ U[zeta_range], sorted by f,
    redrawn until adjacent frequencies differ by at least `min_rel_spacing`;
    mode shapes i.i.d. N(0, 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    for _ in range(10000):
        f = np.sort(rng.uniform(f_range[0], f_range[1], n_modes))
        if n_modes < 2 or np.all(np.diff(f) / f[1:] >= min_rel_spacing):
            break
    else:  # pragma: no cover - only for absurd spacing requests
        raise RuntimeError("could not draw well-separated frequencies")
    z = rng.uniform(zeta_range[0], zeta_range[1], n_modes)
    shapes = rng.standard_normal((l, n_modes))
    return ModalSystem(fs=float(fs), freqs=f, zetas=z, shapes=shapes,
                       mu=_poles(f, z, fs))


def simulate(system: ModalSystem, n: int, noise_frac: float, seed: int,
             dtype=np.float32) -> np.ndarray:
    """Simulate n samples of the model; returns y (l x n), channel-major."""
    from scipy.signal import lfilter

    rng = np.random.Generator(np.random.PCG64(seed))
    nm = system.n_modes
    rho2 = np.abs(system.mu) ** 2
    z = np.empty((nm, n), dtype=np.complex128)
    for r in range(nm):
        s = math.sqrt(max(1.0 - rho2[r], 0.0))
        w = s * (rng.standard_normal(n) + 1j * rng.standard_normal(n))
        z0 = rng.standard_normal() + 1j * rng.standard_normal()
        # z[h] = mu z[h-1] + w[h-1] for h >= 1 and z[0] = z0: filter the
        # shifted noise sequence with initial condition mu*z0.
        drive = np.concatenate(([0.0 + 0.0j], w[:-1]))
        zi = np.array([system.mu[r] * z0])
        out, _ = lfilter([1.0], [1.0, -system.mu[r]], drive, zi=zi)
        out[0] = z0
        z[r] = out
    y = system.shapes @ z.real
    if noise_frac > 0.0:
        rms = np.sqrt(np.mean(y * y, axis=1, keepdims=True))
        y = y + noise_frac * rms * rng.standard_normal(y.shape)
    return np.ascontiguousarray(y.astype(dtype))


@dataclasses.dataclass
class Workload:
    """One synthetic workload: generator settings plus identification settings."""
    name: str
    l: int
    n: int
    fs: float
    n_modes: int
    f_range: tuple
    zeta_range: tuple
    noise: float
    lags: tuple            # j_b values
    svd: str               # "full" or "randomized"
    rank: int = 0
    oversample: int = 0
    power_iters: int = 0
    order_min: int = 2
    order_max: int = 2
    order_step: int = 2
    struct_seed: int = 0
    noise_seed: int = 0
    sketch_seed: int = 0
    min_rel_spacing: float = 0.01   # adjacent generated frequencies differ by at least this

    @property
    def orders(self) -> List[int]:
        return list(range(self.order_min, self.order_max + 1, self.order_step))


def _wl(idx: int, **kw) -> Workload:
    kw.setdefault("struct_seed", 1000 + idx)
    kw.setdefault("noise_seed", 2000 + idx)
    kw.setdefault("sketch_seed", 3000 + idx)
    return Workload(**kw)


# The named workloads.  "small-full-svd" is the 12-channel record with a full
# SVD of the 240 x 240 Toeplitz matrix; "bridge-180ch" is the 180-channel,
# 30-minute record with the randomized SVD of the 10800 x 10800 Toeplitz
# matrix; "bridge-180ch-3d" sweeps nine lags on the same record;
# "array-600ch" is the 600-channel, one-hour record.
WORKLOADS: Dict[str, Workload] = {
    "small-full-svd": _wl(1, name="small-full-svd", l=12, n=20000, fs=50.0,
                          n_modes=4, f_range=(0.5, 10.0),
                          zeta_range=(0.01, 0.03), noise=0.05, lags=(20,),
                          svd="full", order_min=2, order_max=40, order_step=2),
    "bridge-180ch": _wl(2, name="bridge-180ch", l=180, n=180000, fs=100.0,
                        n_modes=20, f_range=(0.5, 20.0),
                        zeta_range=(0.005, 0.03), noise=0.05, lags=(60,),
                        svd="randomized", rank=200, oversample=20,
                        power_iters=2, order_min=2, order_max=200,
                        order_step=2),
    "bridge-180ch-3d": _wl(3, name="bridge-180ch-3d", l=180, n=180000,
                           fs=100.0, n_modes=20, f_range=(0.5, 20.0),
                           zeta_range=(0.005, 0.03), noise=0.05,
                           lags=tuple(range(20, 101, 10)), svd="randomized",
                           rank=200, oversample=20, power_iters=2,
                           order_min=2, order_max=200, order_step=2,
                           struct_seed=1002, noise_seed=2002),
    "array-600ch": _wl(5, name="array-600ch", l=600, n=360000, fs=100.0,
                       n_modes=60, f_range=(0.3, 30.0),
                       zeta_range=(0.005, 0.03), noise=0.03, lags=(100,),
                       svd="randomized", rank=400, oversample=40,
                       power_iters=3, order_min=2, order_max=400,
                       order_step=4, min_rel_spacing=0.002),
}


def make_record(wl: Workload, n: Optional[int] = None):
    """Draw the structure and simulate the record of workload `wl`.

    Returns (system, y) with y float32 of shape (l, n)."""
    sysm = draw_system(wl.l, wl.n_modes, wl.f_range, wl.zeta_range, wl.fs,
                       wl.struct_seed, wl.min_rel_spacing)
    y = simulate(sysm, wl.n if n is None else n, wl.noise, wl.noise_seed)
    return sysm, y


def random_matrix(rows: int, cols: int, seed: int, dtype=np.float32,
                  scale: float = 1.0) -> np.ndarray:
    """Dense i.i.d. N(0, scale^2) matrix."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.ascontiguousarray(
        (scale * rng.standard_normal((rows, cols))).astype(dtype))


def random_stack(count: int, l: int, seed: int, dtype=np.float32) -> np.ndarray:
    """`count` dense l x l blocks with i.i.d. N(0, 1) entries."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.ascontiguousarray(
        rng.standard_normal((count, l, l)).astype(dtype))


def random_lowrank(m: int, n: int, rank: int, seed: int, decay: float = 0.7,
                   noise: float = 0.0, dtype=np.float32) -> np.ndarray:
    """m x n matrix with geometrically decaying spectrum of the given rank
    (singular values decay**i), plus optional i.i.d. noise."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = np.linalg.qr(rng.standard_normal((m, rank)))[0]
    b = np.linalg.qr(rng.standard_normal((n, rank)))[0]
    s = decay ** np.arange(rank)
    mat = (a * s) @ b.T
    if noise > 0.0:
        mat = mat + noise * rng.standard_normal((m, n))
    return np.ascontiguousarray(mat.astype(dtype))
