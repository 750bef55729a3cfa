"""Plain FP64 CPU checker for the SSI-COV identification path.

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports this module; only
the tests, the smoke entry point and the CPU-baseline leg of the benchmark may
import or call it.  It shares no code with the GPU path: its only common
ground with the library is the seeded inputs both receive.

Every function follows the paper's equations in the paper's order, in float64,
with library primitives (matrix product, Householder QR, least squares,
nonsymmetric eigen-decomposition) standing in only for single steps:

  correlations    Section 2.1, the correlation matrices R_1..R_{2j_b-1}
                  (estimator written out as a definition, see below)
  toeplitz        Eq. (6), block (r, c) = R_{j_b + r - c}
  jacobi_svd      Eq. (8): one-sided (Hestenes) Jacobi SVD
  rsvd            Algorithm 1 with Eq. (13)-(18), plus oversampling and
                  subspace (power) iterations with a QR after every product
  shift_ls        Eq. (9)-(10): O = U S^1/2, C = first l rows,
                  A = pinv(O_top) O_bot (least squares)
  poles           Eq. (11)-(12) read through Eq. (3): eig(A), lambda = ln(mu)/dt,
                  f = |lambda| / 2 pi, xi = -Re(lambda) / |lambda|, phi = C psi
  identify        the whole path for every (lag, order): Section 2.3 step i

Readings taken where the paper is silent or garbled:
  * correlation estimator: R_j = (1/N) sum_{k=0}^{N-1-j} y_{k+j} y_k^T, no
    mean removal;
  * Eq. (10): O_top / O_bot are the first / last l (j_b - 1) rows;
  * Eq. (11): A = Psi M Psi^{-1} (the printed transpose is a typo);
  * Eq. (12): f and xi from Eq. (3): f = |lambda|/2pi, xi = -Re lambda/|lambda|;
  * one pole per conjugate pair (Im mu > 0), real mu dropped, principal log;
  * mode shapes: unit 2-norm, largest-modulus entry real and positive;
  * poles of one order sorted by (f, xi);
  * oversampling p and q power iterations (absent from Algorithm 1) follow the
    randomized range finder with re-orthonormalisation after every product;
    p = q = 0 is Algorithm 1 exactly;
  * Q of every QR has a positive diagonal in R.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from .philox import sketch as philox_sketch

__all__ = [
    "correlations", "toeplitz", "jacobi_svd", "qr_pos", "rsvd", "full_svd",
    "shift_ls", "eig_poles", "modal", "identify", "Poles", "sketch",
    "tau", "lag_rule", "lag_range_3d", "default_rank_percent", "default_rank",
]

sketch = philox_sketch


# ----------------------------------------------------------------- Section 2.1
def correlations(y: np.ndarray, n_lags: int) -> np.ndarray:
    """R[j-1] = (1/N) sum_{k=0}^{N-1-j} y[:, k+j] y[:, k]^T for j = 1..n_lags.

    y: (l, N) channel-major.  Returns (n_lags, l, l) float64."""
    yy = np.asarray(y, dtype=np.float64)
    l, n = yy.shape
    if not 1 <= n_lags < n:
        raise ValueError("need 1 <= n_lags < N")
    out = np.empty((n_lags, l, l))
    for j in range(1, n_lags + 1):
        out[j - 1] = yy[:, j:] @ yy[:, : n - j].T / n
    return out


def toeplitz(r_stack: np.ndarray, jb: int) -> np.ndarray:
    """Eq. (6): T[r l + a, c l + b] = R_{jb + r - c}[a, b], 0 <= r, c < jb.

    r_stack[j-1] holds R_j; it must hold at least 2 jb - 1 blocks."""
    cnt, l, _ = r_stack.shape
    if jb < 1 or cnt < 2 * jb - 1:
        raise ValueError("need 2*jb-1 correlation blocks")
    t = np.empty((jb * l, jb * l))
    for r in range(jb):
        for c in range(jb):
            t[r * l:(r + 1) * l, c * l:(c + 1) * l] = r_stack[jb + r - c - 1]
    return t


# ------------------------------------------------------------------- Eq. (8)
def jacobi_svd(m: np.ndarray, tol: float = 1e-15, max_sweeps: int = 60
               ) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """One-sided Jacobi SVD of a tall matrix (rows >= cols).

    Plane rotations are applied to column pairs (i, j), i < j, in cyclic order
    until every pair is orthogonal to `tol` relative to the column norms.
    Returns (U, s, V) with m = U diag(s) V^T, s descending."""
    x = np.array(m, dtype=np.float64, copy=True)
    rows, cols = x.shape
    if rows < cols:
        raise ValueError("jacobi_svd needs rows >= cols")
    v = np.eye(cols)
    for _ in range(max_sweeps):
        rotated = False
        for i in range(cols - 1):
            for j in range(i + 1, cols):
                xi = x[:, i]
                xj = x[:, j]
                alpha = xi @ xi
                beta = xj @ xj
                gamma = xi @ xj
                if abs(gamma) <= tol * math.sqrt(alpha * beta) or gamma == 0.0:
                    continue
                rotated = True
                zeta = (beta - alpha) / (2.0 * gamma)
                t = math.copysign(1.0, zeta) / (abs(zeta) + math.sqrt(1.0 + zeta * zeta))
                c = 1.0 / math.sqrt(1.0 + t * t)
                s = c * t
                x[:, i], x[:, j] = c * xi - s * xj, s * xi + c * xj
                vi = v[:, i].copy()
                vj = v[:, j]
                v[:, i], v[:, j] = c * vi - s * vj, s * vi + c * vj
        if not rotated:
            break
    else:
        raise RuntimeError("Jacobi SVD did not converge")
    sig = np.sqrt(np.einsum("ij,ij->j", x, x))
    order = np.argsort(-sig, kind="stable")
    sig = sig[order]
    x = x[:, order]
    v = v[:, order]
    u = np.zeros_like(x)
    nz = sig > 0
    u[:, nz] = x[:, nz] / sig[nz]
    return u, sig, v


def full_svd(t: np.ndarray, k: Optional[int] = None):
    """Left singular vectors and singular values of T (Eq. (8)), leading k."""
    u, s, _ = jacobi_svd(t)
    if k is None:
        k = s.shape[0]
    return u[:, :k], s[:k]


# ---------------------------------------------------- Eq. (13)-(18), Alg. 1
def qr_pos(y: np.ndarray) -> np.ndarray:
    """Economy Householder QR (LAPACK), columns signed so that diag(R) > 0."""
    q, r = np.linalg.qr(y, mode="reduced")
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d


def rsvd(t: np.ndarray, k: int, oversample: int, power_iters: int,
         omega: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Randomized SVD of T: returns (U[:, :k], sigma[:k]).

    Y = T Omega, Q = qr(Y) (Eq. (14), Alg. 1); q times Q = qr(T^T Q),
    Q = qr(T Q); P = Q^T T (Eq. (15)); P = U~ S V^T (Eq. (16)); U = Q U~
    (Eq. (18)).  The SVD of the short, wide P is the one-sided Jacobi SVD of
    R_P^T where P^T = Q_P R_P, which has the same left singular vectors and
    singular values as P."""
    m = t.shape[0]
    ell = k + oversample
    if omega.shape != (t.shape[1], ell):
        raise ValueError("omega must be n x (k + p)")
    q = qr_pos(t @ omega)
    for _ in range(power_iters):
        q = qr_pos(t.T @ q)
        q = qr_pos(t @ q)
    p = q.T @ t
    r_p = np.linalg.qr(p.T, mode="r")
    u_t, s, _ = jacobi_svd(r_p.T)
    u = q @ u_t
    assert u.shape == (m, ell)
    return u[:, :k], s[:k]


# ------------------------------------------------------------ Eq. (9)-(10)
def shift_ls(u: np.ndarray, s: np.ndarray, l: int, n: int):
    """For order n: O = U_n S_n^1/2, C = O[:l], A = pinv(O_top) O_bot."""
    o = u[:, :n] * np.sqrt(s[:n])
    m = o.shape[0]
    c = o[:l]
    a = np.linalg.lstsq(o[: m - l], o[l:], rcond=None)[0]
    return a, c


# ----------------------------------------------------------- Eq. (11)-(12)
@dataclasses.dataclass
class Poles:
    """Poles of one (lag, order): one entry per conjugate pair, sorted by f."""
    f: np.ndarray          # Hz
    xi: np.ndarray         # damping ratio
    mu: np.ndarray         # complex discrete eigenvalue
    phi: np.ndarray        # (n_poles, l) complex mode shapes

    def __len__(self) -> int:
        return int(self.f.shape[0])


def eig_poles(a: np.ndarray, c: np.ndarray, fs: float) -> Poles:
    """Eigen-decomposition of A (Eq. (11)) and the continuous poles (Eq. (12)),
    with f and xi taken from Eq. (3)."""
    mu, psi = np.linalg.eig(a)
    keep = mu.imag > 0.0
    mu = mu[keep]
    psi = psi[:, keep]
    lam = np.log(mu) * fs
    f = np.abs(lam) / (2.0 * np.pi)
    xi = -lam.real / np.abs(lam)
    phi = (c @ psi).T
    for i in range(phi.shape[0]):
        nrm = np.linalg.norm(phi[i])
        if nrm > 0:
            phi[i] /= nrm
            big = np.argmax(np.abs(phi[i]))
            phi[i] *= np.conj(phi[i, big]) / abs(phi[i, big])
    order = np.lexsort((xi, f))
    return Poles(f=f[order], xi=xi[order], mu=mu[order], phi=phi[order])


def modal(u: np.ndarray, s: np.ndarray, l: int, orders: Sequence[int],
          fs: float) -> List[Poles]:
    """Poles for every model order (the order sweep of Section 2.1)."""
    out = []
    for n in orders:
        a, c = shift_ls(u, s, l, n)
        out.append(eig_poles(a, c, fs))
    return out


# ------------------------------------------------------------- Section 2.3
@dataclasses.dataclass
class LagResult:
    jb: int
    sigma: np.ndarray
    poles: List[Poles]


def identify(y: np.ndarray, fs: float, lags: Sequence[int],
             orders: Sequence[int], svd: str = "randomized", rank: int = 0,
             oversample: int = 0, power_iters: int = 0, seed: int = 0,
             omegas: Optional[Sequence[np.ndarray]] = None) -> List[LagResult]:
    """Modal identification for every time lag j_b and every model order:
    correlations once for the largest lag, then per lag Toeplitz -> (R)SVD ->
    A, C -> eig -> poles.  The sketch of lag index i is the Philox stream i of
    `seed` unless `omegas` is given."""
    l = y.shape[0]
    r_stack = correlations(y, 2 * max(lags) - 1)
    res = []
    for i, jb in enumerate(lags):
        t = toeplitz(r_stack, jb)
        if svd == "full":
            u, s = full_svd(t, max(orders))
        else:
            ell = rank + oversample
            om = omegas[i] if omegas is not None else sketch(seed, t.shape[1], ell, i)
            u, s = rsvd(t, rank, oversample, power_iters, om)
        res.append(LagResult(jb=jb, sigma=s, poles=modal(u, s, l, orders, fs)))
    return res


# --------------------------------------------- parameter rules, Eq. (20)-(23)
def tau(jb: int, fs: float) -> float:
    """Eq. (20): time lag tau = (2 j_b - 1) / f_s."""
    return (2 * jb - 1) / fs


def lag_rule(fs: float, f0: float, factor: float = 10.0) -> int:
    """Eq. (22) (factor 10) and the lower end of Eq. (23) (factor 9), with
    'int' read as rounding up, the only reading that reproduces every worked
    example in Section 3."""
    return int(math.ceil(factor * fs / (2.0 * f0) - 1e-9))


def lag_range_3d(fs: float, f0: float, n_lags: int, beta: float = 1.5) -> List[int]:
    """Eq. (23): n_lags values from j_b,min to ceil(beta j_b,min), evenly
    spaced and rounded to the nearest integer."""
    lo = lag_rule(fs, f0, 9.0)
    hi = int(math.ceil(beta * lo - 1e-9))
    return [int(math.floor(v + 0.5)) for v in np.linspace(lo, hi, n_lags)]


def default_rank_percent(t_size: int) -> float:
    """Eq. (21): minimum rank in percent of the Toeplitz size T."""
    return max(30.0 - 0.00156 * t_size, 25.0)


def default_rank(t_size: int) -> int:
    """Number of retained columns: ceil(kbar(T) * T / 100)."""
    return int(math.ceil(default_rank_percent(t_size) * t_size / 100.0 - 1e-9))
