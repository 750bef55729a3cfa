"""Reference values for the 600-channel configuration at a shortened record,
computed by the FP64 checker alone (oracle/), for tests/test_gpu_array600.py.

The record is the 600-channel array workload (60 modes, 3 % noise) cut to
N = 20000 samples; the identification keeps the configuration's shape: lag
j_b = 100 (a 60000 x 60000 Toeplitz matrix, Eq. (6)), randomized SVD with
k = 400, p = 40, q = 3 (Algorithm 1), orders 2..400 step 4.  The checker's
randomized SVD takes T through its products only, so T is passed as an
operator that builds one block row of Eq. (6) at a time from the R stack
(the 28.8 GB FP64 matrix is never formed); every arithmetic step is the
checker's own.  Two references are written: from the FP64 correlations, and
from the same correlations rounded to FP32 (the precision of the library's
R stack), whose difference measures how far rounding the input to FP32
alone moves each result.

Run from the repository root:  python tests/golden/make_array600.py
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2411_05510_amd import synth  # noqa: E402

N = 20000
OUT = os.path.join(HERE, "array600_n20000.npz")
PHI_ORDERS = (118, 238, 398)


def physical(f, xi, sysm):
    """(pole index, mode index) of the poles within 1 % in frequency and 0.02
    in damping of a mode of the generating system (nearest in frequency)."""
    out = []
    for r, fr in enumerate(sysm.freqs):
        if len(f) == 0:
            continue
        i = int(np.argmin(np.abs(f - fr)))
        if abs(f[i] - fr) / fr < 0.01 and abs(xi[i] - sysm.zetas[r]) < 0.02:
            out.append((i, r))
    return out


class BlockToeplitz:
    """T of Eq. (6) (or its transpose) as an operator: T[r l + a, c l + b] =
    R_{jb + r - c}[a, b]; products are formed one block row of l rows at a
    time."""
    __array_ufunc__ = None           # ndarray @ op defers to op.__rmatmul__

    def __init__(self, r_stack: np.ndarray, jb: int, transposed: bool = False):
        self.r, self.jb, self.tr = r_stack, jb, transposed
        self.l = r_stack.shape[1]
        self.shape = (jb * self.l, jb * self.l)

    def _block_row(self, rr: int) -> np.ndarray:
        return np.hstack([self.r[self.jb + rr - c - 1] for c in range(self.jb)])

    @property
    def T(self) -> "BlockToeplitz":
        return BlockToeplitz(self.r, self.jb, not self.tr)

    def __matmul__(self, x: np.ndarray) -> np.ndarray:
        l = self.l
        out = np.zeros((self.shape[0], x.shape[1]))
        for rr in range(self.jb):
            row = self._block_row(rr)                     # l x m
            if self.tr:
                out += row.T @ x[rr * l:(rr + 1) * l]
            else:
                out[rr * l:(rr + 1) * l] = row @ x
        return out

    def __rmatmul__(self, q: np.ndarray) -> np.ndarray:   # q @ T = (T^T q^T)^T
        return (self.T @ q.T).T


def mac(a: np.ndarray, b: np.ndarray) -> float:
    """Modal assurance criterion |a^H b|^2 / (|a|^2 |b|^2)."""
    return float(abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real))


def check_operator() -> None:
    """The operator against the checker's explicit T on a small stack."""
    rng = np.random.Generator(np.random.PCG64(5))
    r = rng.standard_normal((9, 3, 3))
    t = oracle.toeplitz(r, 5)
    op = BlockToeplitz(r, 5)
    x = rng.standard_normal((15, 4))
    assert np.allclose(op @ x, t @ x, rtol=0, atol=1e-12)
    assert np.allclose(op.T @ x, t.T @ x, rtol=0, atol=1e-12)
    assert np.allclose(x.T @ op, x.T @ t, rtol=0, atol=1e-12)


def reference(r_stack, wl, om):
    t0 = time.time()
    u, s = oracle.rsvd(BlockToeplitz(r_stack, wl.lags[0]), wl.rank, wl.oversample,
                       wl.power_iters, om)
    print(f"  rsvd {time.time() - t0:.0f} s", flush=True)
    poles = oracle.modal(u, s, wl.l, wl.orders, wl.fs)
    print(f"  modal {time.time() - t0:.0f} s", flush=True)
    return s, poles


def main() -> None:
    check_operator()
    wl = synth.WORKLOADS["array-600ch"]
    sysm, y = synth.make_record(wl, n=N)
    jb = wl.lags[0]
    t0 = time.time()
    r64 = oracle.correlations(y, 2 * jb - 1)
    print(f"correlations {time.time() - t0:.0f} s", flush=True)
    om = oracle.sketch(wl.sketch_seed, jb * wl.l, wl.rank + wl.oversample, 0)
    out = {"n": np.array(N), "orders": np.array(wl.orders)}
    res = {}
    for tag, r in (("r64", r64), ("r32", r64.astype(np.float32).astype(np.float64))):
        print(tag, flush=True)
        s, poles = reference(r, wl, om)
        res[tag] = poles
        out[f"{tag}_sigma"] = s
        out[f"{tag}_count"] = np.array([len(p) for p in poles])
        out[f"{tag}_f"] = np.concatenate([p.f for p in poles])
        out[f"{tag}_xi"] = np.concatenate([p.xi for p in poles])
        out[f"{tag}_mu"] = np.concatenate([p.mu for p in poles])
    # mode shapes of the physical poles at two orders (FP64 input), and how far
    # rounding the input to FP32 moves each (1 - MAC against the FP32-input pole
    # nearest in discrete eigenvalue)
    for n in PHI_ORDERS:
        oi = list(wl.orders).index(n)
        p64, p32 = res["r64"][oi], res["r32"][oi]
        idx = [i for i, _ in physical(p64.f, p64.xi, sysm)]
        spread = [1.0 - mac(p32.phi[int(np.argmin(np.abs(p32.mu - p64.mu[i])))], p64.phi[i])
                  for i in idx]
        out[f"phi_idx_{n}"] = np.array(idx)
        out[f"phi_{n}"] = p64.phi[idx].astype(np.complex64)
        out[f"phi_spread_{n}"] = np.array(spread)
    np.savez_compressed(OUT, **out)
    print(f"wrote {OUT} ({os.path.getsize(OUT) / 1e6:.2f} MB)")


if __name__ == "__main__":
    main()
