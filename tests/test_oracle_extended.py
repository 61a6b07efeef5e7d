"""CPU pins of the extended-precision block-CG reference (oracle/extended.py),
which certifies GPU and oracle errors on ill-conditioned systems."""
import numpy as np
import pytest

from oracle import block_cg as ob
from oracle import extended as ox
from oracle import truth as ot

from pins import small_spd


def _problem(d, p, k, seed):
    A, lam = small_spd(d, p=p, seed=seed)
    g = np.random.default_rng(seed + 100)
    return A, lam, g.standard_normal(d), g.standard_normal((k, d))


def test_extended_matches_fp64_oracle_when_well_conditioned():
    """kappa(A_mu) ~ 100: the FP64 block-Lanczos oracle and the extended
    iterate agree to FP64 rounding at every t (and the FP64 definition tier,
    whose monomial basis loses digits as t grows, at small t)."""
    A, _, b, Om = _problem(80, 1.0, 3, 51)
    for t in (1, 2, 4, 6):
        xe = ox.bcg_extended(A, 1e-2, b, Om, t)
        assert ox.rel_a_err_ext(A, 1e-2, ob.bcg(A, [1e-2], b, Om, t)[0][0], xe) < 1e-14
        if t <= 4:
            assert ox.rel_a_err_ext(A, 1e-2, ob.bcg_definition(A, 1e-2, b, Om, t), xe) < 1e-13


def test_extended_galerkin_condition_ill_conditioned():
    """kappa(A) = 1.6e6: the residual of the extended iterate is orthogonal to
    the Krylov basis (the optimality condition of def. BCG) to extended
    rounding times ||A|| ||x|| / ||b|| (about 1e6 here; FP64 would leave
    about 1e-10), and the basis is orthonormal to extended rounding."""
    A, _, b, Om = _problem(300, 2.5, 8, 52)
    B = np.column_stack([b, Om.T])
    V = ox.krylov_basis(A, B, 6)
    assert float(np.max(np.abs(V.T @ V - np.eye(V.shape[1], dtype=ox.LD)))) < 1e-16
    x = ox.bcg_extended(A, 0.0, b, Om, 6)
    assert ox.galerkin_residual(A, 0.0, V, x, b) < 1e-13


def test_extended_exact_termination_residual():
    """(k+1) t >= d: the extended iterate solves A_mu x = b; its residual,
    evaluated in extended precision, is far below what FP64 can reach at
    kappa = 1e6, and the FP64 dense Cholesky solve agrees to kappa u64."""
    A, lam, b, Om = _problem(120, 2.9, 11, 53)      # kappa = 120^2.9 = 1.1e6
    x = ox.bcg_extended(A, 0.0, b, Om, 10)
    r = np.asarray(b, dtype=ox.LD) - np.asarray(A, dtype=ox.LD) @ x
    assert float(np.sqrt(r @ r) / np.sqrt(np.asarray(b, dtype=ox.LD) @ np.asarray(b, dtype=ox.LD))) < 1e-13
    xd = np.linalg.solve(A, b)
    kappa = lam[0] / lam[-1]
    assert ox.rel_a_err_ext(A, 0.0, xd, x) < 10 * kappa * 2.0 ** -53


def test_extended_shift_enters_galerkin_system(monkeypatch):
    """Planted mistake: the shift dropped from the Galerkin system moves the
    iterate, and the exact-termination check above rejects it."""
    A, _, b, Om = _problem(60, 1.0, 5, 54)
    mu = 1e-1
    x = ox.bcg_extended(A, mu, b, Om, 10)
    xt = ot.solve_dense(A, mu, b)
    assert ox.rel_a_err_ext(A, mu, xt, x) < 1e-13
    orig = ox._cholesky_solve
    monkeypatch.setattr(ox, "_cholesky_solve", lambda H, r: orig(H - ox.LD(mu) * np.eye(H.shape[0], dtype=ox.LD), r))
    xb = ox.bcg_extended(A, mu, b, Om, 10)
    assert ox.rel_a_err_ext(A, mu, xt, xb) > 1e-6


def test_extended_basis_one_block_short_is_caught(monkeypatch):
    """Planted mistake: a basis one block short (t - 2 products) breaks the
    agreement with the FP64 definition tier."""
    A, _, b, Om = _problem(80, 1.0, 3, 51)
    orig = ox.krylov_basis
    monkeypatch.setattr(ox, "krylov_basis", lambda A_, B_, t, drop_rel=1e-14: orig(A_, B_, max(1, t - 1), drop_rel))
    xe = ox.bcg_extended(A, 1e-2, b, Om, 4)
    xd = ob.bcg_definition(A, 1e-2, b, Om, 4)
    assert ox.rel_a_err_ext(A, 1e-2, xd, xe) > 1e-6
