"""Counter-based Gaussian generator for the seeded start block Omega.  Test
infrastructure only (the oracle side's own implementation; the GPU library has
its own, and the two share no code).

When a caller passes no Omega, the library draws the k x d block on the device
from a 64-bit seed.  The oracle reproduces the same numbers from the published
definition of the generator, so a seeded solve can be checked against the
oracle run on an explicit Omega.

Generator: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC 2011).  A 128-bit counter (c0, c1, c2, c3)
and a 64-bit key (k0, k1) go through ten rounds; one round multiplies c0 and
c2 by the constants 0xD2511F53 and 0xCD9E8D57 (full 64-bit products split into
high and low words) and mixes:
    (c0, c1, c2, c3) <- (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
and the key is bumped by the Weyl constants (0x9E3779B9, 0xBB67AE85) between
rounds.

Layout of the block (this library's convention): element e = r d + c of the
row-major k x d block Omega (row r = Gaussian vector r) is Gaussian number
e mod 2 of Philox call p = e div 2 with counter (lo32 p, hi32 p, stream, 0) and
key (lo32 seed, hi32 seed).  A call's outputs x0..x3 give two uniforms in
(0, 1) with 53 random bits each,
    u1 = ((x0 * 2^32 + x1) >> 11 + 1/2) 2^-53,   u2 = ((x2 * 2^32 + x3) >> 11 + 1/2) 2^-53,
and the Box-Muller transform gives the pair
    g0 = sqrt(-2 ln u1) cos(2 pi u2),   g1 = sqrt(-2 ln u1) sin(2 pi u2).
`stream` separates independent blocks drawn from one seed (system s of a
batched solve uses stream s; a path uses stream 0).
"""
from __future__ import annotations

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint32(0x9E3779B9)
_W1 = np.uint32(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Philox4x32-10 on arrays of counters.  ctr: (..., 4) uint32, key: (2,)
    uint32.  Returns (..., 4) uint32."""
    c = np.array(ctr, dtype=np.uint32, copy=True)
    k0, k1 = np.uint32(key[0]), np.uint32(key[1])
    c0, c1, c2, c3 = (c[..., i].astype(np.uint64) for i in range(4))
    for rnd in range(10):
        if rnd:
            k0 = np.uint32((int(k0) + int(_W0)) & 0xFFFFFFFF)
            k1 = np.uint32((int(k1) + int(_W1)) & 0xFFFFFFFF)
        p0 = _M0 * c0                       # < 2^64: exact in uint64
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1, hi0 ^ c3 ^ np.uint64(k1), lo0)
    out = np.stack([c0, c1, c2, c3], axis=-1)
    return out.astype(np.uint32)


def gaussian_block(seed: int, stream: int, rows: int, cols: int) -> np.ndarray:
    """The rows x cols row-major block of standard normals described in the
    module docstring (float64)."""
    n = rows * cols
    ncall = (n + 1) // 2
    p = np.arange(ncall, dtype=np.uint64)
    ctr = np.zeros((ncall, 4), dtype=np.uint32)
    ctr[:, 0] = (p & _MASK).astype(np.uint32)
    ctr[:, 1] = (p >> np.uint64(32)).astype(np.uint32)
    ctr[:, 2] = np.uint32(stream & 0xFFFFFFFF)
    key = (np.uint32(seed & 0xFFFFFFFF), np.uint32((seed >> 32) & 0xFFFFFFFF))
    x = philox4x32_10(ctr, key).astype(np.uint64)
    a = ((x[:, 0] << np.uint64(32)) | x[:, 1]) >> np.uint64(11)
    b = ((x[:, 2] << np.uint64(32)) | x[:, 3]) >> np.uint64(11)
    u1 = (a.astype(np.float64) + 0.5) * 2.0 ** -53
    u2 = (b.astype(np.float64) + 0.5) * 2.0 ** -53
    r = np.sqrt(-2.0 * np.log(u1))
    g = np.empty(2 * ncall)
    g[0::2] = r * np.cos(2.0 * np.pi * u2)
    g[1::2] = r * np.sin(2.0 * np.pi * u2)
    return g[:n].reshape(rows, cols)
