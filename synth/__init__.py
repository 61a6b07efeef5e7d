"""Seeded synthetic inputs for the randomized block-CG workloads.

This module only draws random numbers and assembles problem data (matrices,
right-hand sides, Gaussian blocks, shift grids).  It holds none of the
solver's arithmetic, and both the CPU oracle and the GPU library consume the
exact same bits it produces.

Seeds follow ``numpy.random.SeedSequence([2501, 18717, config_id, stream])``
with streams 0 = matrix factors, 1 = right-hand side / true solution,
2 = Gaussian block Omega, 3 = noise, 4 = per-system parameters of a batch.

The paper's own test problems (its ``fastdecay`` family and the spectra of
its test-problem figure) are defined only in code that is not available, so
these generators stand in for them with spectra of the same kinds: algebraic
eigenvalue decay for dense SPD systems (Sec. 1, regularized system),
exponentially decaying singular values for ridge regression (Sec. 1, ridge
regression), and a kernel covariance for Gaussian sampling (Sec. 1, sampling
Gaussians).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng", "orthogonal", "spd_from_spectrum", "power_spectrum", "gaussian_block",
    "dense_problem", "ridge_problem", "rbf_problem", "batch_params", "mu_grid",
]

_ROOT = (2501, 18717)


def rng(config_id: int, stream: int) -> np.random.Generator:
    """Generator for (config, stream); independent streams per purpose."""
    return np.random.default_rng(np.random.SeedSequence([*_ROOT, int(config_id), int(stream)]))


def orthogonal(d: int, g: np.random.Generator) -> np.ndarray:
    """Haar-like orthogonal d x d matrix: Q factor of a Gaussian matrix with
    column signs fixed by sign(diag R)."""
    G = g.standard_normal((d, d))
    Q, R = np.linalg.qr(G)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s


def power_spectrum(d: int, p: float) -> np.ndarray:
    """lambda_i = i^(-p), i = 1..d (1-indexed, decreasing)."""
    return np.arange(1, d + 1, dtype=np.float64) ** (-float(p))


def spd_from_spectrum(lam: np.ndarray, g: np.random.Generator) -> np.ndarray:
    """A = Q diag(lam) Q^T, symmetrised in FP64 so that A == A.T bitwise."""
    d = lam.shape[0]
    Q = orthogonal(d, g)
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    return np.ascontiguousarray(A)


def gaussian_block(d: int, k: int, g: np.random.Generator) -> np.ndarray:
    """Omega stored as k vectors of length d (shape (k, d), row-major)."""
    return np.ascontiguousarray(g.standard_normal((k, d)))


def mu_grid(L: int = 64, lo: float = -6.0, hi: float = 0.0) -> np.ndarray:
    """Log-spaced shifts, inclusive of both ends."""
    return np.logspace(lo, hi, L)


def dense_problem(config_id: int, d: int, p: float, k: int, mu: float) -> dict:
    """Dense SPD system A_mu x = b with lambda_i = i^-p, b ~ N(0, I),
    Omega ~ N(0, 1)^(k x d)."""
    lam = power_spectrum(d, p)
    A = spd_from_spectrum(lam, rng(config_id, 0))
    b = rng(config_id, 1).standard_normal(d)
    Om = gaussian_block(d, k, rng(config_id, 2))
    return {"A": A, "lam": lam, "b": b, "omega": Om, "mu": float(mu), "d": d, "k": k}


def ridge_problem(config_id: int, n: int, d: int, k: int, decay: float = 400.0,
                  noise: float = 0.01, L: int = 64) -> dict:
    """Ridge regression data: Z = G diag(s) stored in FP32 with s_j = exp(-j/decay)
    (1-indexed), x* ~ N(0, I), f = Z x* + noise * N(0, I) (in FP64 from the
    FP32 Z values), right-hand side b = Z^T f (FP64).  ``mus`` is the
    regularization path."""
    g0 = rng(config_id, 0)
    s = np.exp(-np.arange(1, d + 1, dtype=np.float64) / decay)
    Z = np.empty((n, d), dtype=np.float32)
    rows = 8192
    for r0 in range(0, n, rows):
        r1 = min(n, r0 + rows)
        Z[r0:r1] = (g0.standard_normal((r1 - r0, d)) * s).astype(np.float32)
    xs = rng(config_id, 1).standard_normal(d)
    e = rng(config_id, 3).standard_normal(n)
    f = np.empty(n)
    b = np.zeros(d)
    for r0 in range(0, n, rows):
        r1 = min(n, r0 + rows)
        Zc = Z[r0:r1].astype(np.float64)
        f[r0:r1] = Zc @ xs + noise * e[r0:r1]
        b += Zc.T @ f[r0:r1]
    Om = gaussian_block(d, k, rng(config_id, 2))
    return {"Z": Z, "s": s, "xstar": xs, "f": f, "b": b, "omega": Om,
            "mus": mu_grid(L), "n": n, "d": d, "k": k}


def rbf_problem(config_id: int, npts: int, nsamples: int, ell: float = 0.1,
                nugget: float = 1e-6) -> dict:
    """Gaussian-process covariance A_ij = exp(-|x_i - x_j|^2 / (2 ell^2)) + nugget
    delta_ij on points uniform in [0,1]^3, and nsamples standard normal
    vectors stored as rows (shape (nsamples, npts))."""
    X = rng(config_id, 0).random((npts, 3))
    sq = np.einsum("ij,ij->i", X, X)
    A = np.empty((npts, npts))
    rows = 2048
    for r0 in range(0, npts, rows):
        r1 = min(npts, r0 + rows)
        D2 = sq[r0:r1, None] + sq[None, :] - 2.0 * (X[r0:r1] @ X.T)
        np.maximum(D2, 0.0, out=D2)
        A[r0:r1] = np.exp(-D2 / (2.0 * ell * ell))
    A = 0.5 * (A + A.T)
    A[np.diag_indices(npts)] += nugget
    B = rng(config_id, 1).standard_normal((nsamples, npts))
    return {"A": np.ascontiguousarray(A), "points": X, "B": np.ascontiguousarray(B),
            "d": npts, "ell": ell, "nugget": nugget}


def batch_params(config_id: int, nsys: int, d_lo: int, d_hi: int,
                 ks=(8, 16, 32, 64, 128), p_lo: float = 1.0, p_hi: float = 3.0,
                 logmu_lo: float = -6.0, logmu_hi: float = -2.0) -> list[dict]:
    """Per-system sizes and parameters of a batch of independent systems:
    d ~ U{d_lo..d_hi}, p ~ U[p_lo, p_hi], mu = 10^U[logmu_lo, logmu_hi],
    k ~ U(ks)."""
    g = rng(config_id, 4)
    out = []
    for i in range(nsys):
        d = int(g.integers(d_lo, d_hi + 1))
        p = float(g.uniform(p_lo, p_hi))
        mu = float(10.0 ** g.uniform(logmu_lo, logmu_hi))
        k = int(ks[int(g.integers(0, len(ks)))])
        k = min(k, d - 1)
        out.append({"sys": i, "d": d, "p": p, "mu": mu, "k": k})
    return out


def batch_system(config_id: int, params: dict) -> dict:
    """Materialise one system of a batch from its parameters (seeded by the
    system index so systems can be streamed one at a time)."""
    i = params["sys"]
    sub = 1000 + i
    lam = power_spectrum(params["d"], params["p"])
    A = spd_from_spectrum(lam, rng(config_id * 100000 + sub, 0))
    b = rng(config_id * 100000 + sub, 1).standard_normal(params["d"])
    Om = gaussian_block(params["d"], params["k"], rng(config_id * 100000 + sub, 2))
    return {"A": A, "lam": lam, "b": b, "omega": Om, "mu": params["mu"],
            "d": params["d"], "k": params["k"]}


# ---- batches at full size: spectra exact, eigenvectors from a few Householder reflectors, so a
#      d = 16000 system is formed in O(d^2) (on the GPU for the benchmark, in numpy for oracle checks)

def reflector_vectors(d: int, r: int, g: np.random.Generator) -> np.ndarray:
    """r unit vectors of length d (shape (r, d)), Gaussian directions."""
    V = g.standard_normal((r, d))
    return V / np.linalg.norm(V, axis=1, keepdims=True)


def spd_from_reflectors(lam: np.ndarray, V: np.ndarray) -> np.ndarray:
    """A = H_r ... H_1 diag(lam) H_1 ... H_r with H_i = I - 2 v_i v_i^T (numpy, FP64)."""
    A = np.diag(np.asarray(lam, dtype=np.float64))
    for v in V:
        w = A @ v
        A = A - 2.0 * np.outer(v, w) - 2.0 * np.outer(w, v) + 4.0 * float(v @ w) * np.outer(v, v)
    return np.ascontiguousarray(0.5 * (A + A.T))


def spd_from_reflectors_torch(lam: np.ndarray, V: np.ndarray, device):
    """The same matrix formed with torch on `device` (FP64), for sizes the host cannot hold."""
    import torch
    lam_t = torch.as_tensor(np.asarray(lam, dtype=np.float64), device=device)
    A = torch.diag(lam_t)
    for v in V:
        vt = torch.as_tensor(v, device=device)
        w = A @ vt
        A.addr_(vt, w, alpha=-2.0)
        A.addr_(w, vt, alpha=-2.0)
        A.addr_(vt, vt, alpha=4.0 * float(vt @ w))
    A = 0.5 * (A + A.T)
    return A.contiguous()


def batch_system_fast(config_id: int, params: dict, reflectors: int = 4) -> dict:
    """One system of a batch with a reflector-built eigenbasis: the spectrum, right-hand side,
    Gaussian block and reflector vectors (A itself is formed by the caller, on the device or in
    numpy)."""
    i = params["sys"]
    sub = 1000 + i
    d = params["d"]
    lam = power_spectrum(d, params["p"])
    V = reflector_vectors(d, reflectors, rng(config_id * 100000 + sub, 3))
    b = rng(config_id * 100000 + sub, 1).standard_normal(d)
    Om = gaussian_block(d, params["k"], rng(config_id * 100000 + sub, 2))
    return {"lam": lam, "V": V, "b": b, "omega": Om, "mu": params["mu"], "d": d, "k": params["k"]}
