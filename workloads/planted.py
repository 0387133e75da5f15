"""Planted-spectrum test matrices and the served request stream.

Every matrix is A = U diag(sigma) V^H (+ optional i.i.d. noise) with U the
orthonormal factor of a seeded Gaussian m x n matrix and V the orthonormal
factor of a seeded Gaussian n x n matrix, the construction the paper uses for
its synthetic experiments (Sec. 1.1, "Easy"/"Hard"; Sec. 4.1; Sec. 4.2).
Spectra follow the five workload descriptions of the hot path:

* ``cfg1``  4000 x 50, k=1: sigma_1..sigma_49 log-spaced 1 -> 1e-3, sigma_50 = 1e-6.
* ``cfg2``  1e6 x 200, k=1: n-2 equal geometric steps from 1 plus one drop by 10
  between sigma_{n-1} and sigma_n, sigma_n = 1e-12.
* ``cfg3``  1e6 x 1000 complex, k=10: sigma_1..sigma_990 log-spaced 1 -> 1e-4,
  the last 10 zero, plus complex Gaussian noise with E|N_ij|^2 = (1e-14)^2.
* ``cfg4``  2e6 x 500, k=5: as cfg2 with sigma_min = 1e-10 and a drop of 100
  between sigma_{n-5} and sigma_{n-4}.
* ``e5``    1e6 x 2000, the block-size study (Sec. 5.2): clustered spectrum
  sigma_i = exp(-log(1e10) ((i-1)/(n-1))^(1/256)), k = 1, blocks 1, 3, 5, 10.
* ``cfg5``  the served stream: m ~ U[1e4, 5e5], n ~ U[20, 400], k ~ U{1..10},
  a drop of 10 at sigma_{n-k}, sigma_min = 10^U[-12,-4], Poisson arrivals.

Two backends draw the same recipe: numpy on the host (small and medium sizes,
bit-reproducible everywhere) and torch on a device (full sizes, where a host QR
of a 1e6-row matrix would dominate the run).  The two backends draw different
random numbers; a run uses one of them for both the GPU path and its checks.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class ConfigSpec:
    name: str
    m: int
    n: int
    k: int
    d: int
    zeta: int
    is_complex: bool
    data_seed: int
    sketch_seed: int
    noise_std: float = 0.0


# Sketch dimension d and sparsity zeta per workload: d = 4n (3n for the complex
# nullspace workload), 8 nonzeros per column of S.
CONFIGS = {
    "cfg1": ConfigSpec("cfg1", 4000, 50, 1, 200, 8, False, 1001, 2001),
    "cfg2": ConfigSpec("cfg2", 1_000_000, 200, 1, 800, 8, False, 1002, 2002),
    "cfg3": ConfigSpec("cfg3", 1_000_000, 1000, 10, 3000, 8, True, 1003, 2003, 1e-14),
    "cfg4": ConfigSpec("cfg4", 2_000_000, 500, 5, 2000, 8, False, 1004, 2004),
    "e5": ConfigSpec("e5", 1_000_000, 2000, 1, 8000, 8, False, 1005, 2005),
}


def config_spec(name: str) -> ConfigSpec:
    return CONFIGS[name]


def spectrum_gap(n: int, k: int, sigma_min: float, gamma: float) -> np.ndarray:
    """Descending spectrum: sigma_1 = 1, n-2 equal geometric steps plus one drop
    by ``gamma`` between sigma_{n-k} and sigma_{n-k+1}; sigma_n = sigma_min."""
    if n < 3 or not (1 <= k < n):
        raise ValueError("spectrum_gap needs n >= 3 and 1 <= k < n")
    total = -math.log10(sigma_min)
    step = (total - math.log10(gamma)) / (n - 2)
    i = np.arange(1, n + 1, dtype=np.float64)
    expo = np.where(i <= n - k, -step * (i - 1), -step * (i - 2) - math.log10(gamma))
    s = 10.0 ** expo
    s[0] = 1.0
    s[-1] = sigma_min
    return s


def spectrum_logspace_tail(n: int, top_lo: float, tail: float) -> np.ndarray:
    """sigma_1..sigma_{n-1} log-spaced from 1 to ``top_lo``; sigma_n = ``tail``."""
    s = np.empty(n)
    s[: n - 1] = np.logspace(0.0, math.log10(top_lo), n - 1)
    s[n - 1] = tail
    return s


def spectrum_nullspace(n: int, k: int, lo: float) -> np.ndarray:
    """sigma_1..sigma_{n-k} log-spaced from 1 to ``lo``; the last k are zero."""
    s = np.zeros(n)
    s[: n - k] = np.logspace(0.0, math.log10(lo), n - k)
    return s


def spectrum_clustered(n: int, a: float = 1.0 / 256.0, cond: float = 1e10) -> np.ndarray:
    """sigma_i = exp(-log(cond) ((i-1)/(n-1))^a), i = 1..n (Sec. 5.2): sigma_1 = 1,
    sigma_n = 1/cond, with the values crowded towards 1/cond for small a (at
    n = 2000 and a = 1/256, (sigma_{n-1}^2 - sigma_n^2)/sigma_n^2 = 9e-5)."""
    if n < 2:
        raise ValueError("spectrum_clustered needs n >= 2")
    x = np.arange(n, dtype=np.float64) / (n - 1)
    return np.exp(-math.log(cond) * x ** a)


def config_spectrum(name: str) -> np.ndarray:
    c = CONFIGS[name]
    if name == "cfg1":
        return spectrum_logspace_tail(c.n, 1e-3, 1e-6)
    if name == "cfg2":
        return spectrum_gap(c.n, c.k, 1e-12, 10.0)
    if name == "cfg3":
        return spectrum_nullspace(c.n, c.k, 1e-4)
    if name == "cfg4":
        return spectrum_gap(c.n, c.k, 1e-10, 100.0)
    if name == "e5":
        return spectrum_clustered(c.n)
    raise KeyError(name)


def _gaussian_np(rng: np.random.Generator, shape, is_complex: bool) -> np.ndarray:
    if not is_complex:
        return rng.standard_normal(shape)
    # Re and Im each N(0, 1/2), so E|g|^2 = 1.
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) * math.sqrt(0.5)


def planted_numpy(m: int, n: int, sigma: np.ndarray, seed: int, *,
                  is_complex: bool = False, noise_std: float = 0.0):
    """Return (A, V, sigma): A = U diag(sigma) V^H (+ noise), C-ordered.

    Draw order: the m x n Gaussian for U, then the n x n Gaussian for V, then
    the noise.  U and V are the Q factors of numpy's Householder QR.
    """
    rng = np.random.default_rng(seed)
    G = _gaussian_np(rng, (m, n), is_complex)
    U, _ = np.linalg.qr(G)
    del G
    H = _gaussian_np(rng, (n, n), is_complex)
    V, _ = np.linalg.qr(H)
    A = (U * np.asarray(sigma)[None, :]) @ V.conj().T
    del U
    if noise_std:
        A += noise_std * _gaussian_np(rng, (m, n), is_complex)
    return np.ascontiguousarray(A), V, np.asarray(sigma, dtype=np.float64)


def planted_torch(m: int, n: int, sigma, seed: int, *, device="cuda",
                  is_complex: bool = False, noise_std: float = 0.0,
                  row_chunk: int = 1 << 17):
    """Device-side draw of the same recipe (torch RNG, CholeskyQR2 for U).

    Returns (A, V, sigma) as torch tensors on ``device``.  U's orthonormal
    factor comes from two rounds of Cholesky QR over the Gaussian, which has
    condition number close to 1 when m >> n, so two rounds reach orthogonality
    to working precision.
    """
    import torch

    dt = torch.complex128 if is_complex else torch.float64
    g = torch.Generator(device=device)
    g.manual_seed(seed)

    def gauss(shape):
        if not is_complex:
            return torch.randn(shape, generator=g, device=device, dtype=torch.float64)
        re = torch.randn(shape, generator=g, device=device, dtype=torch.float64)
        im = torch.randn(shape, generator=g, device=device, dtype=torch.float64)
        return torch.complex(re, im) * math.sqrt(0.5)

    X = gauss((m, n))
    for _ in range(2):
        Gm = torch.zeros((n, n), device=device, dtype=dt)
        for r0 in range(0, m, row_chunk):
            blk = X[r0:r0 + row_chunk]
            Gm += blk.conj().T.contiguous() @ blk
        L = torch.linalg.cholesky(Gm)
        # X <- X L^{-H}, with the small n x n inverse formed once
        eye = torch.eye(n, device=device, dtype=dt)
        Linv_h = torch.linalg.solve_triangular(L, eye, upper=False).conj().T.contiguous()
        for r0 in range(0, m, row_chunk):
            X[r0:r0 + row_chunk] = X[r0:r0 + row_chunk] @ Linv_h
    H = gauss((n, n))
    V, _ = torch.linalg.qr(H)
    s = torch.as_tensor(np.asarray(sigma, dtype=np.float64), device=device)
    Vh = (V.conj().T * 1.0).contiguous()
    for r0 in range(0, m, row_chunk):
        blk = X[r0:r0 + row_chunk] * s.to(dt)[None, :]
        X[r0:r0 + row_chunk] = blk @ Vh
    if noise_std:
        for r0 in range(0, m, row_chunk):
            nr = min(row_chunk, m - r0)
            X[r0:r0 + nr] += noise_std * gauss((nr, n))
    return X.contiguous(), V, s


def integer_matrix(m: int, n: int, seed: int, lo: int = -8, hi: int = 8, *,
                   is_complex: bool = False) -> np.ndarray:
    """Small-integer-valued matrix: sums of its rows are exact in FP64."""
    rng = np.random.default_rng(seed)
    A = rng.integers(lo, hi + 1, size=(m, n)).astype(np.float64)
    if is_complex:
        A = A + 1j * rng.integers(lo, hi + 1, size=(m, n)).astype(np.float64)
    return A


@dataclass(frozen=True)
class Request:
    rid: int
    arrival_s: float
    m: int
    n: int
    k: int
    log10_sigma_min: float
    data_seed: int
    sketch_seed: int


def served_requests(count: int = 256, rate_per_s: float = 100.0, seed: int = 5000,
                    m_range=(10_000, 500_000), n_range=(20, 400), k_range=(1, 10),
                    log_smin_range=(-12.0, -4.0)):
    """The served stream: Poisson arrivals at ``rate_per_s`` and per-request
    shapes drawn uniformly.  Request r uses data seed 6000+r and sketch seed
    7000+r; each request keeps 3k <= n."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(count):
        t += rng.exponential(1.0 / rate_per_s)
        m = int(rng.integers(m_range[0], m_range[1] + 1))
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        k = int(rng.integers(k_range[0], k_range[1] + 1))
        k = max(1, min(k, n // 3))
        ls = float(rng.uniform(*log_smin_range))
        out.append(Request(r, t, m, n, k, ls, 6000 + r, 7000 + r))
    return out


def request_spectrum(req: Request) -> np.ndarray:
    return spectrum_gap(req.n, req.k, 10.0 ** req.log10_sigma_min, 10.0)
