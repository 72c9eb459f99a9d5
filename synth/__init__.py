"""Seeded synthetic inputs for the BLWS-SVT library, its tests and its bench.

This module only draws random data with ``numpy.random.Generator(PCG64(seed))``.
It holds none of the method's arithmetic (no SVD, no thresholding, no ALM step):
both the CPU oracle and the GPU library receive the arrays it returns.

Workload recipes follow the paper's experimental section (RPCA data in the manner of
the inexact-ALM experiments; MC data as two Gaussian factors and a uniformly sampled
set of observed entries), with the sizes of the target configurations:

* RPCA(m, n, r, frac, amp, seed): A0 = L R^T with L (m x r), R (n x r) iid N(0, 1);
  E0 has exactly round(frac * m * n) nonzeros at positions drawn uniformly without
  replacement, values iid U[-amp, amp]; D = A0 + E0.
* MC(m, n, r, frac, seed): M = L R^T as above; Omega is a uniform sample without
  replacement of round(frac * m * n) entries, sorted row-major and stored as CSR
  (int32 row_ptr / col_idx) with the values of M on Omega.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "rng",
    "rpca_instance",
    "mc_instance",
    "gaussian",
    "orthonormal",
    "prescribed_spectrum",
    "ill_conditioned_block",
    "sample_positions",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def rpca_instance(m: int, n: int, r: int, frac: float, amp: float, seed: int) -> dict:
    """Low-rank plus sparse data. Draw order: L, R, support, values."""
    g = rng(seed)
    L = g.standard_normal((m, r))
    R = g.standard_normal((n, r))
    A0 = L @ R.T
    k = int(round(frac * m * n))
    idx = g.choice(m * n, size=k, replace=False)
    vals = g.uniform(-amp, amp, size=k)
    E0 = np.zeros(m * n)
    E0[idx] = vals
    E0 = E0.reshape(m, n)
    D = A0 + E0
    return {"D": np.ascontiguousarray(D), "A0": A0, "E0": E0, "L": L, "R": R,
            "lam": 1.0 / np.sqrt(max(m, n)), "nnz": k}


def mc_instance(m: int, n: int, r: int, frac: float, seed: int) -> dict:
    """Matrix completion data: factors, then the sampled set Omega as CSR."""
    g = rng(seed)
    L = g.standard_normal((m, r))
    R = g.standard_normal((n, r))
    k = int(round(frac * m * n))
    idx = np.sort(g.choice(m * n, size=k, replace=False))
    rows = (idx // n).astype(np.int64)
    cols = (idx % n).astype(np.int32)
    # entries of M = L R^T on Omega, computed in float64 row block by row block
    vals = np.empty(k)
    step = 1 << 20
    for s in range(0, k, step):
        e = min(k, s + step)
        vals[s:e] = np.einsum("ij,ij->i", L[rows[s:e]], R[cols[s:e]])
    row_ptr = np.zeros(m + 1, dtype=np.int32)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    return {"row_ptr": row_ptr, "col_idx": cols, "values": vals, "L": L, "R": R,
            "nnz": k, "m": m, "n": n}


def gaussian(shape, seed: int) -> np.ndarray:
    return rng(seed).standard_normal(shape)


def orthonormal(rows: int, cols: int, seed: int) -> np.ndarray:
    """Random matrix with orthonormal columns (Q factor of a Gaussian)."""
    q, r = np.linalg.qr(gaussian((rows, cols), seed))
    return q * np.sign(np.where(np.diag(r) == 0, 1.0, np.diag(r)))


def prescribed_spectrum(m: int, n: int, sigma, seed: int):
    """W = Q1 diag(sigma) Q2^T with random orthonormal Q1 (m x p), Q2 (n x p)."""
    sigma = np.asarray(sigma, dtype=np.float64)
    p = sigma.size
    q1 = orthonormal(m, p, seed)
    q2 = orthonormal(n, p, seed + 7919)
    return (q1 * sigma) @ q2.T, q1, q2


def sample_positions(m: int, n: int, count: int, seed: int) -> np.ndarray:
    """Seeded distinct flat positions used for sampled parity checks."""
    count = min(count, m * n)
    return np.sort(rng(seed).choice(m * n, size=count, replace=False))


def ill_conditioned_block(m: int, n: int, b: int, kappa: float, side: str, seed: int) -> dict:
    """A matrix W and a warm block (U, V) whose new Krylov block is
    ill-conditioned without being singular.

    W = X diag(sigma) Y^T (random orthonormal X, Y) with sigma_1 = 100, ten
    values from 60 down to 40, a geometric tail from 20 and a last value
    100 / kappa. side "V": V = [(y_1 + y_p) / sqrt(2), (y_1 - y_p) / sqrt(2),
    y_2, .., y_{b-1}] and U random, so the first two columns of W V are
    (sigma_1 x_1 +- sigma_p x_p) / sqrt(2): after the columns are scaled to
    unit norm, the sine of the angle between them is about 2 / kappa (the
    left block's condition number is about kappa). side "U": the same with
    the roles of (U, x) and (V, y) exchanged. Every singular pair above 30 is
    spanned by both halves of the block, so one step reaches them exactly."""
    p = min(m, n)
    sigma = np.r_[100.0, np.linspace(60.0, 40.0, 10), np.geomspace(20.0, 1e-2, p - 12),
                  100.0 / kappa]
    W, X, Y = prescribed_spectrum(m, n, sigma, seed)
    pair = lambda Z: np.c_[(Z[:, 0] + Z[:, p - 1]) / np.sqrt(2.0),
                           (Z[:, 0] - Z[:, p - 1]) / np.sqrt(2.0), Z[:, 1:b - 1]]
    if side == "V":
        U, V = orthonormal(m, b, seed + 1), pair(Y)
    else:
        U, V = pair(X), orthonormal(n, b, seed + 1)
    return {"W": np.ascontiguousarray(W), "U": np.ascontiguousarray(U),
            "V": np.ascontiguousarray(V), "sigma": sigma}
