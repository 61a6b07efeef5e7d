"""The reflector-built batch generator: exact spectrum, bitwise symmetry, and the torch build equal
to the numpy build (the GPU benchmark forms the matrices with torch, oracle checks with numpy)."""
import numpy as np

import synth


def test_reflector_spd_has_the_prescribed_spectrum():
    lam = synth.power_spectrum(257, 2.3)
    V = synth.reflector_vectors(257, 4, synth.rng(3, 3))
    A = synth.spd_from_reflectors(lam, V)
    assert np.array_equal(A, A.T)
    w = np.sort(np.linalg.eigvalsh(A))[::-1]
    assert np.abs(w - lam).max() <= 1e-14 * lam[0]
    # the eigenbasis is not the identity: off-diagonal mass is substantial
    assert np.abs(A - np.diag(np.diag(A))).max() > 1e-3


def test_reflector_spd_torch_matches_numpy():
    lam = synth.power_spectrum(300, 1.2)
    V = synth.reflector_vectors(300, 4, synth.rng(4, 3))
    A = synth.spd_from_reflectors(lam, V)
    At = synth.spd_from_reflectors_torch(lam, V, "cpu").numpy()
    assert np.abs(At - A).max() <= 1e-15


def test_batch_system_fast_is_seeded_per_system():
    p = synth.batch_params(7, 3, 200, 400)
    a = synth.batch_system_fast(7, p[1])
    b = synth.batch_system_fast(7, p[1])
    c = synth.batch_system_fast(7, p[2])
    assert np.array_equal(a["V"], b["V"]) and np.array_equal(a["b"], b["b"])
    assert a["d"] != c["d"] or not np.array_equal(a["b"][:10], c["b"][:10])
