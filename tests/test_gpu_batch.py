"""Batched independent systems of uneven size and block width in one rbcg_solve
call (the batching extension): every system against the oracle's block-CG
iterate at the same t, and a batched refinement run to a residual target.

Systems follow the batch recipe (lambda_i = i^-p, p ~ U[1, 3],
mu = 10^U[-6, -2], k ~ U{8, 16, 32, 64}) at sizes the oracle finishes in
seconds, with eigenbases from four Householder reflectors (the construction
the full-size benchmark forms on the GPU).
"""
import numpy as np
import pytest

import synth
from oracle import block_cg as ob

from gpu_util import a_err, fp64_bound, note, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_18717_amd import rbcg
    return rbcg, rbcg.Context()


def _systems(n):
    params = synth.batch_params(11, n, 300, 1400, ks=(8, 16, 32, 64))
    out = []
    for p in params:
        S = synth.batch_system_fast(11, p)
        S["A"] = synth.spd_from_reflectors(S["lam"], S["V"])
        out.append(S)
    return out


def test_batched_iterates_match_oracle(R):
    import torch
    rbcg, ctx = R
    systems = _systems(10)
    t = 9
    note("batch of 10 uneven systems, t = 9")
    ops = [rbcg.DenseOperator(ctx, to_dev(S["A"])) for S in systems]
    bs = [to_dev(S["b"]) for S in systems]
    oms = [to_dev(S["omega"]) for S in systems]
    xs = [torch.zeros_like(b) for b in bs]
    rc, info = rbcg.solve(ctx, ops, [S["mu"] for S in systems], bs, oms, xs, [rbcg.opts(t) for _ in systems])
    assert rc == 0
    for S, x, inf in zip(systems, xs, info):
        X, _ = ob.bcg(S["A"], [S["mu"]], S["b"], S["omega"], t)
        kappa = (S["lam"][0] + S["mu"]) / (S["lam"][-1] + S["mu"])
        e = a_err(S["A"], S["mu"], x.cpu().numpy(), X[0])
        # two FP64 implementations of the recurrence, each with d-term dot products rounded to
        # about sqrt(d) u, differ by up to that times kappa(A_mu) on each side
        bound = fp64_bound(kappa)
        note(f"d={S['d']} k={S['k']} mu={S['mu']:.1e} err {e:.1e} bound {bound:.1e}")
        assert e < bound


def test_batched_refinement_reaches_target(R):
    import torch
    rbcg, ctx = R
    systems = _systems(10)
    ops = [rbcg.DenseOperator(ctx, to_dev(S["A"])) for S in systems]
    bs = [to_dev(S["b"]) for S in systems]
    oms = [to_dev(S["omega"]) for S in systems]
    xs = [torch.zeros_like(b) for b in bs]
    opts = [rbcg.opts(64, rtol=1e-10, refine_max=3) for _ in systems]
    rc, info = rbcg.solve(ctx, ops, [S["mu"] for S in systems], bs, oms, xs, opts)
    assert rc == 0
    for S, x, inf in zip(systems, xs, info):
        A, mu, b = S["A"], S["mu"], S["b"]
        xc = x.cpu().numpy()
        rel = np.linalg.norm(b - (A @ xc + mu * xc)) / np.linalg.norm(b)
        note(f"d={S['d']} k={S['k']} loads {inf['matrix_loads']} relres {inf['relres']:.1e} (host {rel:.1e})")
        assert rel <= 1.5e-10
        # two FP64 evaluations of b - A_mu x (different summation orders) differ by up to about
        # sqrt(d) u (||A_mu|| ||x|| + ||b||)
        lam_max = float(S["lam"][0])
        floor = 4.0 * np.sqrt(S["d"]) * 2.0 ** -53 * ((lam_max + mu) * np.linalg.norm(xc) + np.linalg.norm(b))
        assert abs(rel - inf["relres"]) <= 1e-2 * rel + floor / np.linalg.norm(b)


def _systems_all_widths():
    """One system of every block width of the batch recipe (k = 8, 16, 32, 64,
    128) plus five more drawn from it, at oracle-friendly sizes."""
    params = synth.batch_params(12, 10, 300, 1400)
    widths = (8, 16, 32, 64, 128)
    for i, k in enumerate(widths):
        params[i]["k"] = min(k, params[i]["d"] - 1)
    out = []
    for p in params:
        S = synth.batch_system_fast(12, p)
        S["A"] = synth.spd_from_reflectors(S["lam"], S["V"])
        out.append(S)
    assert {S["k"] for S in out} >= set(widths)
    return out


def test_batched_mixed_refinement_all_widths(R):
    """FP32-MFMA block products with FP64 refinement for a batch that holds
    every block width (9 ... 129), one rbcg_solve call: every system within
    1e-8 relative A_mu-norm error of the dense Cholesky solution."""
    import torch
    from oracle import truth as ot
    rbcg, ctx = R
    systems = _systems_all_widths()
    note("batch of 10 uneven systems, all five widths, FP32 products + FP64 refinement")
    ops = [rbcg.DenseOperator(ctx, to_dev(S["A"]), lo="f32") for S in systems]
    bs = [to_dev(S["b"]) for S in systems]
    oms = [to_dev(S["omega"]) for S in systems]
    xs = [torch.zeros_like(b) for b in bs]
    opts = [rbcg.opts(64, rtol=1e-10, matvec="f32", refine_max=24) for _ in systems]
    rc, info = rbcg.solve(ctx, ops, [S["mu"] for S in systems], bs, oms, xs, opts)
    worst = 0.0
    for S, x, inf in zip(systems, xs, info):
        xt = ot.solve_dense(S["A"], S["mu"], S["b"])
        e = a_err(S["A"], S["mu"], x.cpu().numpy(), xt)
        worst = max(worst, e)
        note(f"d={S['d']} k={S['k']} mu={S['mu']:.1e} sweeps {inf['refine_sweeps']} loads {inf['matrix_loads']} "
             f"relres {inf['relres']:.1e} err vs Cholesky {e:.1e}")
        assert inf["precision_used"] == 1
    assert rc == 0, info
    assert worst < 1e-8


def test_batched_fp64_errors_attributed_extended_precision(R):
    """Which side carries the kappa-sized FP64 differences: the GPU iterate and
    the oracle's iterate, each against block-CG at the same t in extended
    precision (oracle/extended.py).  No direction deflates in these spaces
    (checked on both sides), so all three compute the same iterate.  FP64
    block-CG leaves a relative A_mu-norm error of up to about kappa(A_mu) u;
    the GPU is held to max(1e-12, 0.1 kappa u) (1e-12 below kappa ~ 1e5), the
    oracle to 1e-12."""
    import torch
    from oracle import extended as ox
    rbcg, ctx = R
    systems = _systems(10)
    t = 9
    note("batch of 10 uneven systems, t = 9, extended-precision attribution")
    ops = [rbcg.DenseOperator(ctx, to_dev(S["A"])) for S in systems]
    bs = [to_dev(S["b"]) for S in systems]
    oms = [to_dev(S["omega"]) for S in systems]
    xs = [torch.zeros_like(b) for b in bs]
    rc, info = rbcg.solve(ctx, ops, [S["mu"] for S in systems], bs, oms, xs, [rbcg.opts(t) for _ in systems])
    assert rc == 0
    for S, x, inf in zip(systems, xs, info):
        xe = ox.bcg_extended(S["A"], S["mu"], S["b"], S["omega"], t)
        X, lz = ob.bcg(S["A"], [S["mu"]], S["b"], S["omega"], t)
        eg = ox.rel_a_err_ext(S["A"], S["mu"], x.cpu().numpy(), xe)
        eo = ox.rel_a_err_ext(S["A"], S["mu"], X[0], xe)
        kappa = (S["lam"][0] + S["mu"]) / (S["lam"][-1] + S["mu"])
        note(f"d={S['d']} k={S['k']} kappa {kappa:.1e} deflated {inf['deflated']}: GPU vs extended {eg:.2e}, "
             f"oracle vs extended {eo:.2e}")
        assert inf["deflated"] == 0 and sum(lz["widths"]) == t * (S["k"] + 1)
        assert eo < 1e-12
        assert eg < fp64_bound(kappa)
