"""O2 -- counter-based normals for the bisection construction.

Test infrastructure only (see ``oracle/__init__``).

The paper draws each bisection offset with the Box-Muller formula from two uniforms produced by the
SPRNG library (Sec. 4.1). A counter-based generator replaces SPRNG so that any sample of any path
can be regenerated independently: Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11): a 4x32-bit counter, a 2x32-bit key, ten
rounds, each round two 32x32->64 multiplications by the published multipliers, xor of the high
halves with the other counter words and the round key, the key bumped by the published Weyl
increments between rounds.

Stream layout (a reading: the paper's SPRNG stream has no counter structure):
* one generator call per *pair* of heap nodes (2j, 2j+1) of one path; heap node h in 1..N-1 is
  the bisection point of level n = floor(log2 h)+1 with offset i = h - 2^(n-1);
* counter = (j, path_lo32, path_hi32, stream), key = (seed_lo32, seed_hi32);
* u1 = odd53(out0 | out1<<32), u2 = odd53(out2 | out3<<32) with odd53(b) = ((b>>11) | 1) * 2^-53,
  an odd multiple of 2^-53, so 0 < u < 1 exactly (the paper's interval [0,1] would allow ln 0);
* Box-Muller: r = sqrt(-2 ln u1), theta = 2 pi u2; node 2j takes r cos(theta), node 2j+1 takes
  r sin(theta) (the paper uses only the cosine branch; both are independent standard normals).
  Node 1 pairs with the non-existent node 0, whose cosine output is unused.

Pins (tests/test_oracle_rng.py): published known-answer vectors of Philox4x32-10; bit-for-bit
agreement with an independent implementation (rocRAND's open-source header, called from a host
program); moments and a Kolmogorov-Smirnov test of the normals.
"""
from __future__ import annotations

import numpy as np

PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
_MASK32 = 0xFFFFFFFF


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Ten Philox4x32 rounds on uint32 arrays c0..c3 with scalar key (k0, k1). Returns 4 uint32 arrays."""
    c0 = np.asarray(c0, dtype=np.uint64) & _MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & _MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & _MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & _MASK32
    k0 = int(k0) & _MASK32
    k1 = int(k1) & _MASK32
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    s32 = np.uint64(32)
    msk = np.uint64(_MASK32)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + PHILOX_W0) & _MASK32
            k1 = (k1 + PHILOX_W1) & _MASK32
        p0 = m0 * c0                      # < 2^64: exact in uint64
        p1 = m1 * c2
        hi0, lo0 = p0 >> s32, p0 & msk
        hi1, lo1 = p1 >> s32, p1 & msk
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0)), lo1, (hi0 ^ c3 ^ np.uint64(k1)), lo0
    return (c0.astype(np.uint32), c1.astype(np.uint32), c2.astype(np.uint32), c3.astype(np.uint32))


def odd53(lo32, hi32):
    """Uniform in (0,1): ((b >> 11) | 1) * 2^-53 for the 64-bit word b = lo32 | hi32 << 32."""
    b = (np.asarray(hi32, dtype=np.uint64) << np.uint64(32)) | np.asarray(lo32, dtype=np.uint64)
    k = (b >> np.uint64(11)) | np.uint64(1)
    return k.astype(np.float64) * 2.0 ** -53


def uniforms(seed: int, stream: int, path, pair):
    """(u1, u2) of generator call ``pair`` (= heap node >> 1) for path indices ``path``."""
    path = np.asarray(path, dtype=np.uint64)
    pair = np.asarray(pair, dtype=np.uint64)
    path, pair = np.broadcast_arrays(path, pair)
    o0, o1, o2, o3 = philox4x32_10(pair & np.uint64(_MASK32), path & np.uint64(_MASK32),
                                   path >> np.uint64(32), np.full(path.shape, stream & _MASK32, np.uint64),
                                   seed & _MASK32, (seed >> 32) & _MASK32)
    return odd53(o0, o1), odd53(o2, o3)


def node_normals(seed: int, stream: int, path, node, pair_offset: int = 0):
    """Standard normal z_h for heap node(s) ``node`` (h >= 1) of path(s) ``path``.

    Box-Muller on the call's uniform pair; even h takes the cosine output, odd h the sine output.
    ``pair_offset`` is added to the generator call index (h >> 1): coordinate c of a path in several
    dimensions draws with offset c * 2^20, above every call index of a one-dimensional path
    (N <= 2^20), so coordinate 0 is the one-dimensional draw.
    """
    node = np.asarray(node, dtype=np.uint64)
    u1, u2 = uniforms(seed, stream, path, (node >> np.uint64(1)) + np.uint64(pair_offset))
    r = np.sqrt(-2.0 * np.log(u1))
    theta = 2.0 * np.pi * u2
    node_b = np.broadcast_to(node, r.shape)
    return np.where((node_b & np.uint64(1)) == 0, r * np.cos(theta), r * np.sin(theta))
