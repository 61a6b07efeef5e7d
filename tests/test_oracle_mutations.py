"""Planted mistakes, on the CPU only: each test swaps one step of the oracle
for a plausible wrong variant and checks that at least one pin rejects it.
This shows the pins are sharp enough to catch a dropped term, a wrong sign,
a wrong index or a transposed operand."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import block_cg as ob
from oracle import quadrature as oq

import pins


def _wrong_sign_shift(T, mu, rhs):
    n = T.shape[0]
    return np.linalg.solve(T - mu * np.eye(n) + 2 * abs(mu) * 0, rhs)


def _dropped_shift(T, mu, rhs):
    return np.linalg.solve(T, rhs)


def _transposed_lower(T, mu, rhs):
    # a non-symmetric T (only the lower triangle kept) as if one operand were transposed
    n = T.shape[0]
    return np.linalg.solve(np.tril(T) + mu * np.eye(n), rhs)


@pytest.mark.parametrize("bad", [_wrong_sign_shift, _dropped_shift, _transposed_lower])
def test_pins_reject_bad_shifted_solve(monkeypatch, bad):
    monkeypatch.setattr(ob, "shifted_solve", bad)
    assert max(pins.path_gap(), pins.exact_termination_gap()) > 1e-6


def test_pins_reject_wrong_rhs_index(monkeypatch):
    orig = ob.shifted_solve

    def e2(T, mu, rhs):
        r = np.roll(rhs, 1)
        return orig(T, mu, r)
    monkeypatch.setattr(ob, "shifted_solve", e2)
    assert pins.definition_gap() > 1e-6


def test_pins_reject_missing_reorthogonalisation(monkeypatch):
    # dropping the projection altogether breaks orthogonality of the basis
    monkeypatch.setattr(ob, "_project_out", lambda W, Q: W)
    assert max(pins.definition_gap(), pins.exact_termination_gap()) > 1e-6


def test_pins_reject_missing_operator_in_T(monkeypatch):
    orig = ob.block_lanczos

    def no_A(A, B, t, eta=ob.ETA, first_fixed=True):
        lz = orig(A, B, t, eta=eta, first_fixed=first_fixed)
        lz["T"] = lz["Q"].T @ lz["Q"]
        return lz
    monkeypatch.setattr(ob, "block_lanczos", no_A)
    assert pins.definition_gap() > 1e-6


def test_pins_reject_dropped_b_column(monkeypatch):
    orig = ob.block_lanczos

    def no_b(A, B, t, eta=ob.ETA, first_fixed=True):
        B = np.array(B, copy=True)
        if B.shape[1] > 1:
            B[:, 0] = B[:, 1] + 1e-3 * B[:, 0]
        return orig(A, B, t, eta=eta, first_fixed=first_fixed)
    monkeypatch.setattr(ob, "block_lanczos", no_b)
    assert pins.definition_gap() > 1e-6


def test_pins_reject_sqrt_without_leading_A(monkeypatch):
    orig = ob.block_lanczos

    def wrong(A, B, t, eta=ob.ETA, first_fixed=True):
        lz = orig(A, B, t, eta=eta, first_fixed=first_fixed)
        lz["AQ"] = lz["Q"]          # drops the leading A of def. blansq
        return lz
    monkeypatch.setattr(ob, "block_lanczos", wrong)
    assert pins.sqrt_full_space_gap() > 1e-6


def test_pins_reject_quadrature_missing_factor(monkeypatch):
    orig = oq.sqrt_rule

    def wrong(m, M, N, dps=40):
        s, w = orig(m, M, N, dps)
        return s, w / np.sqrt(m)     # the sqrt(m) Jacobian factor dropped
    monkeypatch.setattr(oq, "sqrt_rule", wrong)
    assert pins.quadrature_gap() > 1e-6


def test_pins_reject_quadrature_off_by_half_node(monkeypatch):
    import mpmath as mp

    def wrong(m, M, N, dps=40):
        with mp.workdps(dps):
            kp2 = 1 - mp.mpf(m) / mp.mpf(M)
            Kp = mp.ellipk(kp2)
            s = np.empty(N)
            w = np.empty(N)
            for j in range(N):
                v = (j + 1) * Kp / (N + 1)       # trapezoid-like nodes with midpoint weights
                sn, cn, dn = (mp.ellipfun(f, v, m=kp2) for f in ("sn", "cn", "dn"))
                s[j] = float(m * (sn / cn) ** 2)
                w[j] = float(2 / mp.pi * Kp / N * mp.sqrt(m) * dn / cn ** 2)
        return s, w
    monkeypatch.setattr(oq, "sqrt_rule", wrong)
    assert pins.quadrature_gap() > 1e-6


def _inv_sqrt_keeps_leading_A(A, Bs, t, eta=ob.ETA):
    return ob.sqrt_apply_exact(A, Bs, t, eta=eta)


def _inv_sqrt_positive_power(A, Bs, t, eta=ob.ETA):
    Bs = np.atleast_2d(np.asarray(Bs, dtype=np.float64))
    lz = ob.block_lanczos(A, Bs.T, t, eta=eta, first_fixed=False)
    w, V = np.linalg.eigh(lz["T"])
    return (lz["Q"] @ ((V * np.sqrt(w)) @ V.T) @ (lz["Q"].T @ Bs.T)).T, lz


@pytest.mark.parametrize("bad", [_inv_sqrt_keeps_leading_A, _inv_sqrt_positive_power])
def test_pins_reject_bad_inverse_square_root(monkeypatch, bad):
    monkeypatch.setattr(ob, "inv_sqrt_apply_exact", bad)
    gap, ratio = pins.inv_sqrt_identity_gaps()
    assert gap > 1e-6 or ratio > 1.0 + 1e-10


def test_pins_reject_sampling_start_basis_not_spanning_B(monkeypatch):
    """A start basis that does not span the samples (one sample replaced by a
    random vector) changes the sampling iterates outside the full space; the
    definition pin over an explicit Krylov basis must catch it."""
    orig = ob.block_lanczos

    def wrong(A, B, t, eta=ob.ETA, first_fixed=True):
        B = np.array(B, copy=True)
        if not first_fixed and B.shape[1] > 1:
            B[:, -1] = np.random.default_rng(0).standard_normal(B.shape[0])
        return orig(A, B, t, eta=eta, first_fixed=first_fixed)
    monkeypatch.setattr(ob, "block_lanczos", wrong)
    gs, gi = pins.sampling_definition_gaps()
    assert gs > 1e-6 and gi > 1e-6


def test_pins_reject_sampling_basis_one_block_short(monkeypatch):
    """Dropping the last Krylov block (t - 1 products) is an index mistake
    that the full-space pin cannot see once m (t - 1) >= d; the definition
    pin at m t < d must."""
    orig = ob.block_lanczos

    def short(A, B, t, eta=ob.ETA, first_fixed=True):
        return orig(A, B, max(1, t - 1), eta=eta, first_fixed=first_fixed)
    monkeypatch.setattr(ob, "block_lanczos", short)
    gs, gi = pins.sampling_definition_gaps(ts=(2, 3, 5))
    assert gs > 1e-6 and gi > 1e-6


def _pcg_unpreconditioned(A, mu, b, Pinv, t):
    # the preconditioner forgotten: the Krylov space of A_mu itself
    from oracle import krylov as ok
    return ok.cg_definition(A, mu, b, t)


def _pcg_wrong_start(A, mu, b, Pinv, t):
    # K_t(P^-1 A_mu, b) instead of K_t(P^-1 A_mu, P^-1 b)
    from oracle import krylov as ok
    apply_A = ob.as_operator(A)
    M = lambda v: Pinv @ (apply_A(v[:, None])[:, 0] + mu * v)
    V = ok.krylov_basis_reorth(M, b, t)
    return ob.galerkin(apply_A, mu, V, b)


def _pcg_preconditioner_not_inverted(A, mu, b, Pinv, t):
    # P applied where P^-1 belongs
    from oracle import krylov as ok
    apply_A = ob.as_operator(A)
    P = np.linalg.inv(Pinv)
    M = lambda v: P @ (apply_A(v[:, None])[:, 0] + mu * v)
    V = ok.krylov_basis_reorth(M, P @ b, t)
    return ob.galerkin(apply_A, mu, V, b)


@pytest.mark.parametrize("bad", [_pcg_unpreconditioned, _pcg_wrong_start, _pcg_preconditioner_not_inverted])
def test_pins_reject_bad_pcg_definition(monkeypatch, bad):
    from oracle import krylov as ok
    monkeypatch.setattr(ok, "pcg_definition", bad)
    assert pins.pcg_gap() > 1e-6
