"""Pins of the oracle's seeded Gaussian generator (oracle/philox.py), on the CPU.

* Known-answer vectors of Philox4x32-10 as published with the generator
  (Salmon et al., SC 2011; the Random123 distribution's test vectors): zero
  counter and key, all-ones counter and key, and the counter/key taken from the
  hexadecimal digits of pi.
* The block layout: element e = r cols + c of a rows x cols block depends on e
  only (so a 3 x 5 block is the first 15 numbers of a 1 x 15 block), and
  distinct seeds or streams give distinct blocks.
* The Box-Muller output is standard normal: moments and a Kolmogorov-Smirnov
  test on 2^20 numbers, and the pair (g0, g1) of one call uncorrelated.
A planted mistake (one Weyl constant off by one) must fail the known answers.
"""
import numpy as np
import pytest
from scipy import stats

from oracle import philox as ph

KAT = [
    ((0x00000000, 0x00000000, 0x00000000, 0x00000000), (0x00000000, 0x00000000),
     (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF), (0xFFFFFFFF, 0xFFFFFFFF),
     (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,want", KAT)
def test_philox_known_answers(ctr, key, want):
    got = ph.philox4x32_10(np.array(ctr, dtype=np.uint32), np.array(key, dtype=np.uint32))
    assert [int(v) for v in got] == list(want)


def test_philox_vectorised_matches_single_calls():
    ctr = np.array([k[0] for k in KAT], dtype=np.uint32)
    # one key for the batch: the zero key row reproduces the first vector only
    got = ph.philox4x32_10(ctr[:1], np.zeros(2, dtype=np.uint32))
    assert [int(v) for v in got[0]] == list(KAT[0][2])


def test_block_layout_and_streams():
    a = ph.gaussian_block(7, 0, 3, 5)
    b = ph.gaussian_block(7, 0, 1, 15)
    assert np.array_equal(a.ravel(), b.ravel())
    c = ph.gaussian_block(7, 1, 3, 5)
    d = ph.gaussian_block(8, 0, 3, 5)
    assert not np.allclose(a, c) and not np.allclose(a, d)
    odd = ph.gaussian_block(7, 0, 1, 7)             # odd count: last call's second number dropped
    assert np.array_equal(odd.ravel(), ph.gaussian_block(7, 0, 1, 8).ravel()[:7])


def test_gaussian_statistics():
    g = ph.gaussian_block(2501, 3, 1024, 1024).ravel()
    n = g.size
    assert abs(g.mean()) < 5.0 / np.sqrt(n)
    assert abs(g.var() - 1.0) < 5.0 * np.sqrt(2.0 / n)
    assert abs(stats.skew(g)) < 5.0 * np.sqrt(6.0 / n)
    assert abs(stats.kurtosis(g)) < 5.0 * np.sqrt(24.0 / n)
    assert stats.kstest(g, "norm").pvalue > 1e-4
    pair = np.corrcoef(g[0::2], g[1::2])[0, 1]
    assert abs(pair) < 5.0 / np.sqrt(n / 2)


def test_planted_weyl_constant_fails_known_answer(monkeypatch):
    monkeypatch.setattr(ph, "_W0", np.uint32(0x9E3779BA))
    got = ph.philox4x32_10(np.array(KAT[2][0], dtype=np.uint32), np.array(KAT[2][1], dtype=np.uint32))
    assert [int(v) for v in got] != list(KAT[2][2])
