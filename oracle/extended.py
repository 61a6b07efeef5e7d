"""Block-CG in extended precision (x87 80-bit ``numpy.longdouble``, unit
roundoff 5.4e-20).  Test infrastructure only.

Purpose: certify which side of a GPU-vs-oracle difference carries the error
on ill-conditioned systems.  Two correct FP64 implementations of block-CG
agree only to about kappa(A_mu) u64; this module computes the same iterate
with a unit roundoff 2000 times smaller, so the FP64 results can each be
measured against it.

Passages followed:
  * block-CG iterate by optimality over K_t(A, [b Omega])   Sec. 3, def. BCG
  * block Krylov space                                      Sec. 1.1, eq. block_krylov_def

The inputs (FP64 arrays) are exact in extended precision.  The basis is built
by block Gram-Schmidt on the products A Q_j (every new block projected against
all previous ones twice, then orthonormalised column by column twice), the
Galerkin system V^T A_mu V y = V^T b is solved by a Cholesky factorization
written out here, and x = V y.  All of it is plain loops over numpy longdouble
arrays (no LAPACK, which has no extended-precision routines).
"""
from __future__ import annotations

import numpy as np

LD = np.longdouble


def _orthonormalise(W, Qprev, drop_rel):
    """Columns of W made orthonormal to Qprev and to each other (two passes of
    block projection against Qprev, then two passes of modified Gram-Schmidt
    inside the block).  A column whose norm after projection falls below
    drop_rel times its norm before is dropped (it lies in the space already)."""
    W = np.array(W, dtype=LD, copy=True)
    pre = np.sqrt(np.sum(W * W, axis=0))
    for _ in range(2):
        if Qprev is not None and Qprev.shape[1]:
            W = W - Qprev @ (Qprev.T @ W)
    cols = []
    for c in range(W.shape[1]):
        w = W[:, c].copy()
        for _ in range(2):
            for q in cols:
                w = w - q * (q @ w)
        nw = np.sqrt(w @ w)
        if nw <= drop_rel * max(pre[c], LD(1e-300)):
            continue
        cols.append(w / nw)
    if not cols:
        return np.zeros((W.shape[0], 0), dtype=LD)
    return np.column_stack(cols)


def _cholesky_solve(H, r):
    """Solve H y = r for symmetric positive definite H by H = L L^T."""
    n = H.shape[0]
    L = np.zeros_like(H)
    for j in range(n):
        s = H[j, j] - L[j, :j] @ L[j, :j]
        if not s > 0:
            raise np.linalg.LinAlgError("extended Cholesky: non-positive pivot")
        L[j, j] = np.sqrt(s)
        if j + 1 < n:
            L[j + 1:, j] = (H[j + 1:, j] - L[j + 1:, :j] @ L[j, :j]) / L[j, j]
    z = np.zeros(n, dtype=LD)
    for i in range(n):
        z[i] = (r[i] - L[i, :i] @ z[:i]) / L[i, i]
    y = np.zeros(n, dtype=LD)
    for i in range(n - 1, -1, -1):
        y[i] = (z[i] - L[i + 1:, i] @ y[i + 1:]) / L[i, i]
    return y


def krylov_basis(A, B, t, drop_rel=1e-14):
    """Orthonormal basis (d x n, longdouble) of K_t(A, B) = span{B, AB, ...,
    A^(t-1) B} with b = B[:, 0] as the first direction (t - 1 products)."""
    A = np.asarray(A, dtype=LD)
    blocks = [_orthonormalise(np.asarray(B, dtype=LD), None, drop_rel)]
    for _ in range(t - 1):
        Qall = np.hstack(blocks)
        U = _orthonormalise(A @ blocks[-1], Qall, drop_rel)
        if U.shape[1] == 0:
            break
        blocks.append(U)
    return np.hstack(blocks)


def bcg_extended(A, mu, b, Omega, t):
    """bcg_t(mu) of def. BCG with B = [b Omega] in extended precision; returns
    the iterate as longdouble (length d)."""
    b = np.asarray(b, dtype=np.float64)
    B = np.column_stack([b, np.asarray(Omega, dtype=np.float64).T]) if Omega is not None and len(Omega) else b[:, None]
    V = krylov_basis(A, B, t)
    AV = np.asarray(A, dtype=LD) @ V
    H = V.T @ AV + LD(mu) * (V.T @ V)
    H = (H + H.T) / 2
    y = _cholesky_solve(H, V.T @ b.astype(LD))
    return V @ y


def rel_a_err_ext(A, mu, x, xref):
    """||x - xref||_{A_mu} / ||xref||_{A_mu} evaluated in extended precision."""
    A = np.asarray(A, dtype=LD)
    e = np.asarray(x, dtype=LD) - np.asarray(xref, dtype=LD)
    xr = np.asarray(xref, dtype=LD)
    num = e @ (A @ e) + LD(mu) * (e @ e)
    den = xr @ (A @ xr) + LD(mu) * (xr @ xr)
    return float(np.sqrt(max(num, LD(0)) / den))


def galerkin_residual(A, mu, V, x, b):
    """||V^T (b - A_mu x)|| / ||b|| in extended precision: zero for the Galerkin
    solution over range(V) (the optimality condition of def. BCG)."""
    A = np.asarray(A, dtype=LD)
    x = np.asarray(x, dtype=LD)
    bl = np.asarray(b, dtype=LD)
    r = bl - (A @ x + LD(mu) * x)
    return float(np.sqrt(np.sum((V.T @ r) ** 2)) / np.sqrt(bl @ bl))
