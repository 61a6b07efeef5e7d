"""Block-CG oracle (float64, CPU).  Test infrastructure only.

Paper passages followed:
  * block Krylov space and its shift invariance        Sec. 1.1, eq. block_krylov_def
  * block-CG iterate by optimality                      Sec. 3, def. BCG
  * block-Lanczos: orthonormal Q_t with range K_t(A,B)
    and T_t = Q_t^T A Q_t (block tridiagonal)           Sec. 3.2
  * block-CG for many shifts from one (Q_t, T_t)        Sec. 3.2, eq. bcg_alg
  * block-Lanczos square root                           Sec. 5, def. blansq
  * inverse square root                                 Sec. 5.1, def. blanisq

Counting convention: ``t`` is the number of block products with A that are
performed.  After t products the basis spans K_t(A, B) = span{B, AB, ...,
A^(t-1) B} and T_t = Q_t^T A Q_t is available, so the iterate lies in K_t.

Rank deficiency (Sec. 3.2, finite-precision remarks): after projecting a new
block against the whole basis, directions whose singular value falls below
``eta`` times the norm of the block before projection are dropped, so block
widths may shrink.  When nothing is left, the Krylov space is invariant and
the iteration stops early (the iterate is then exact).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

ETA = 1e-10


def as_operator(A):
    """Return a callable X -> A X for a dense array or a callable."""
    if callable(A):
        return A
    A = np.asarray(A, dtype=np.float64)
    return lambda X: A @ X


def gram_operator(Z):
    """A = Z^T Z applied as Z^T (Z X) (Sec. 1, ridge regression), in float64
    from the stored values of Z."""
    Z64 = np.asarray(Z, dtype=np.float64)
    return lambda X: Z64.T @ (Z64 @ X)


# ---------------------------------------------------------------- definition tier
def krylov_basis_explicit(apply_A, B, t, rtol=1e-12):
    """Orthonormal basis of K_t(A, B) = span{B, AB, ..., A^(t-1) B}
    (eq. block_krylov_def), from the explicit blocks.  Each power block is
    rescaled (span unchanged); singular values below rtol * sigma_1 are
    dropped.  Only for tiny, well-conditioned inputs."""
    blocks = []
    Y = np.array(B, dtype=np.float64, copy=True)
    for _ in range(t):
        blocks.append(Y / np.linalg.norm(Y))
        Y = apply_A(blocks[-1])
    K = np.hstack(blocks)
    U, s, _ = np.linalg.svd(K, full_matrices=False)
    r = int(np.sum(s > rtol * s[0]))
    return U[:, :r]


def galerkin(apply_A, mu, V, b):
    """argmin over x in range(V) of ||A_mu^-1 b - x||_{A_mu} for orthonormal V:
    x = V (V^T A_mu V)^-1 V^T b (the optimality condition of def. BCG)."""
    AV = apply_A(V)
    H = V.T @ AV + mu * (V.T @ V)
    H = 0.5 * (H + H.T)
    y = np.linalg.solve(H, V.T @ b)
    return V @ y


def bcg_definition(A, mu, b, Omega, t):
    """Block-CG iterate bcg_t^(1)(mu) straight from def. BCG with
    B = [b Omega] (Thm. main), via an explicit basis of K_t(A, B)."""
    apply_A = as_operator(A)
    B = np.column_stack([b, np.asarray(Omega).T]) if Omega is not None and len(Omega) else b[:, None]
    V = krylov_basis_explicit(apply_A, B, t)
    return galerkin(apply_A, mu, V, b)


# ----------------------------------------------------------------- algorithm tier
def _orthonormal_directions(W, scale, eta):
    """Orthonormal basis of range(W) keeping singular directions with
    sigma > eta * scale; also returns the coefficient block C with W ~ U C."""
    if W.shape[1] == 0:
        return W[:, :0], np.zeros((0, 0))
    U, s, Vt = np.linalg.svd(W, full_matrices=False)
    keep = s > eta * max(scale, np.finfo(float).tiny)
    U = U[:, keep]
    return U, U.T @ W


def _project_out(W, Q):
    """W <- W - Q (Q^T W), applied twice (full reorthogonalisation)."""
    for _ in range(2):
        if Q.shape[1]:
            W = W - Q @ (Q.T @ W)
    return W


def block_lanczos(A, B, t, eta=ETA, first_fixed=True):
    """Block-Lanczos with full reorthogonalisation for t block products
    (Sec. 3.2).

    The start block B (d x m) is orthonormalised with its first column kept
    as b / ||b|| when ``first_fixed`` (needed for the ||b|| e_1 right-hand
    side of eq. bcg_alg).  Then for j = 1..t: W = A Q_j; project W against
    all basis vectors so far (twice); the surviving directions form
    Q_{j+1}.  T_t is formed as Q_t^T (A Q_t), its definition in Sec. 3.2.

    Returns a dict with
      Q      d x n orthonormal basis of K_t(A, B)   (n = sum of block widths)
      AQ     d x n, A applied to Q (the t products)
      T      n x n symmetric, Q^T A Q
      widths list of block widths [m_1, ..., m_t]
      Qnext  d x m_{t+1} next basis block (from the t-th product)
      Bnext  m_{t+1} x m_t with Q_{t+1} Bnext = (I - Q Q^T) A Q_t
      loads  number of block products actually performed
      exact  True if the space became invariant (iteration stopped early)
    """
    apply_A = as_operator(A)
    B = np.asarray(B, dtype=np.float64)
    d, m = B.shape
    if first_fixed:
        b = B[:, :1]
        nb = np.linalg.norm(b)
        if nb == 0.0:
            raise ValueError("b must be nonzero")
        q0 = b / nb
        rest = _project_out(B[:, 1:], q0)
        scale = np.max(np.linalg.norm(B[:, 1:], axis=0)) if m > 1 else 0.0
        U, _ = _orthonormal_directions(rest, scale, eta)
        Q1 = np.hstack([q0, U])
    else:
        scale = np.max(np.linalg.norm(B, axis=0))
        Q1, _ = _orthonormal_directions(B, scale, eta)
    blocks = [Q1]
    products = []
    Qnext = np.zeros((d, 0))
    Bnext = np.zeros((0, Q1.shape[1]))
    exact = False
    for j in range(t):
        Qj = blocks[-1]
        W = apply_A(Qj)
        products.append(W)
        Qall = np.hstack(blocks)
        P = _project_out(W, Qall)
        scale = np.max(np.linalg.norm(W, axis=0)) if W.shape[1] else 0.0
        U, C = _orthonormal_directions(P, scale, eta)
        Qnext, Bnext = U, U.T @ W
        if j == t - 1:
            break
        if U.shape[1] == 0:
            exact = True
            break
        blocks.append(U)
    Q = np.hstack(blocks)
    AQ = np.hstack(products)
    T = Q.T @ AQ
    T = 0.5 * (T + T.T)
    return {"Q": Q, "AQ": AQ, "T": T, "widths": [blk.shape[1] for blk in blocks],
            "Qnext": Qnext, "Bnext": Bnext, "loads": len(products), "exact": exact}


def shifted_solve(T, mu, rhs):
    """(T + mu I)^-1 rhs by Cholesky (T + mu I is SPD for mu >= 0 when A is)."""
    n = T.shape[0]
    c = sla.cho_factor(T + mu * np.eye(n), lower=False)
    return sla.cho_solve(c, rhs)


def bcg(A, mus, b, Omega, t, eta=ETA):
    """Block-CG iterates bcg_t^(1)(mu) for every mu in ``mus`` from one
    block-Lanczos run on B = [b Omega] (eq. bcg_alg):
        x(mu) = ||b|| Q_t (T_t + mu I)^-1 e_1.
    Returns (X, lanczos) with X of shape (len(mus), d)."""
    b = np.asarray(b, dtype=np.float64)
    Om = np.zeros((0, b.shape[0])) if Omega is None else np.asarray(Omega, dtype=np.float64)
    B = np.column_stack([b, Om.T]) if Om.shape[0] else b[:, None]
    lz = block_lanczos(A, B, t, eta=eta, first_fixed=True)
    n = lz["T"].shape[0]
    e1 = np.zeros(n)
    e1[0] = np.linalg.norm(b)
    X = np.empty((len(np.atleast_1d(mus)), b.shape[0]))
    for i, mu in enumerate(np.atleast_1d(mus)):
        X[i] = lz["Q"] @ shifted_solve(lz["T"], float(mu), e1)
    return X, lz


def bcg_residual_estimate(lz, mu, bnorm):
    """Norm of the residual b - A_mu x_t of the iterate, from the Lanczos
    relation A Q_t = Q_t T_t + Q_{t+1} B_t E_t^T:  || B_t y_last ||, where
    y = (T_t + mu I)^-1 ||b|| e_1 and y_last is its last block (Sec. 4
    remark on a-posteriori residuals)."""
    n = lz["T"].shape[0]
    e1 = np.zeros(n)
    e1[0] = bnorm
    y = shifted_solve(lz["T"], mu, e1)
    mt = lz["widths"][-1]
    return float(np.linalg.norm(lz["Bnext"] @ y[n - mt:]))


def bcg_refined(A, mu, b, Omega, t, sweeps, eta=ETA):
    """Iterative refinement on top of block-CG: x <- x + bcg_t(r) with
    r = b - A_mu x in float64, each sweep a fresh block Krylov space
    [r Omega].  Not in the paper (used to check mixed-precision runs only
    through their converged answers)."""
    apply_A = as_operator(A)
    x = np.zeros_like(np.asarray(b, dtype=np.float64))
    for _ in range(sweeps):
        r = b - (apply_A(x[:, None])[:, 0] + mu * x)
        if np.linalg.norm(r) == 0.0:
            break
        X, _ = bcg(A, [mu], r, Omega, t, eta=eta)
        x = x + X[0]
    return x


# -------------------------------------------------------------------- sampling
def sqrt_apply_exact(A, Bs, t, eta=ETA):
    """Block-Lanczos square root iterates bsq_t^(i) (def. blansq) for the
    samples in the rows of Bs (shape (m, d)), using the block of samples as
    the start block (each sample's augmentation is the other samples).

    (2/pi) int_0^inf (T + z^2 I)^-1 dz = T^-1/2 for SPD T (the scalar identity
    behind eq. sqrt_rational applied eigenvalue-wise), so
        bsq = (A Q_t) T_t^-1/2 Q_t^T B.
    Returns (Y, lanczos) with Y of shape (m, d)."""
    Bs = np.atleast_2d(np.asarray(Bs, dtype=np.float64))
    lz = block_lanczos(A, Bs.T, t, eta=eta, first_fixed=False)
    w, V = np.linalg.eigh(lz["T"])
    Tmh = (V / np.sqrt(w)) @ V.T
    Y = lz["AQ"] @ (Tmh @ (lz["Q"].T @ Bs.T))
    return Y.T, lz


def sqrt_apply_quadrature(A, Bs, t, shifts, weights, eta=ETA, lz=None):
    """Same iterate with the z-integral replaced by a quadrature rule:
        bsq ~ sum_j w_j (A Q_t) (T_t + s_j I)^-1 Q_t^T B,  s_j = z_j^2."""
    Bs = np.atleast_2d(np.asarray(Bs, dtype=np.float64))
    if lz is None:
        lz = block_lanczos(A, Bs.T, t, eta=eta, first_fixed=False)
    R = lz["Q"].T @ Bs.T
    acc = np.zeros_like(R)
    for s, w in zip(shifts, weights):
        acc += w * shifted_solve(lz["T"], float(s), R)
    return (lz["AQ"] @ acc).T, lz


def inv_sqrt_apply_exact(A, Bs, t, eta=ETA):
    """Block-Lanczos inverse square root iterates (def. blanisq):
    (2/pi) int bcg(z^2) dz = Q_t T_t^-1/2 Q_t^T B."""
    Bs = np.atleast_2d(np.asarray(Bs, dtype=np.float64))
    lz = block_lanczos(A, Bs.T, t, eta=eta, first_fixed=False)
    w, V = np.linalg.eigh(lz["T"])
    Tmh = (V / np.sqrt(w)) @ V.T
    return (lz["Q"] @ (Tmh @ (lz["Q"].T @ Bs.T))).T, lz


# ---------------------------------------------------------------------- metrics
def a_norm(apply_A, mu, v):
    """||v||_{A_mu} = sqrt(v^T (A + mu I) v) (Sec. 1.3 notation)."""
    v = np.asarray(v, dtype=np.float64)
    return float(np.sqrt(max(v @ apply_A(v[:, None])[:, 0] + mu * (v @ v), 0.0)))


def rel_a_err(A, mu, x, xref):
    """Relative A_mu-norm error ||x - xref||_{A_mu} / ||xref||_{A_mu}
    (the error measure of the paper's convergence figures)."""
    apply_A = as_operator(A)
    return a_norm(apply_A, mu, np.asarray(x) - np.asarray(xref)) / a_norm(apply_A, mu, xref)
