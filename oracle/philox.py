"""Philox4x64-10 counter-based random number generator, written from its published definition.

J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11.  Philox4x64 keeps a 4-word counter and a 2-word key; each of the 10 rounds
multiplies words 0 and 2 by fixed odd constants, splits the 128-bit products into high and
low halves, mixes the high halves with words 1 and 3 and the key, and permutes; the key is
advanced by two Weyl constants between rounds.

The paper does not fix a generator (random draws appear in the sampling step of Sec. II B and in
the Metropolis filter, Eq. (3)); Philox is used here so that every draw is a pure function of
(key, counter) and the HIP path can reproduce the oracle's stream exactly.

Uniform convention (shared by both sides, defined here in prose): draw number ``i`` of a stream
with key ``(k0, k1)`` and counter words ``(c1, c2, c3)`` is word ``i & 3`` of the Philox block at
counter ``(i >> 2, c1, c2, c3)``; the 64-bit word ``w`` becomes ``u = (w >> 11) * 2**-53`` in
[0, 1) with 53 random bits.

This is test infrastructure (see the package docstring).
"""
import numpy as np

_MASK = (1 << 64) - 1
_M0 = 0xD2E7470EE14C6C93
_M1 = 0xCA5A826395121157
_W0 = 0x9E3779B97F4A7C15   # golden ratio
_W1 = 0xBB67AE8584CAA73B   # sqrt(3) - 1


def philox4x64_10(counter, key):
    """One Philox4x64-10 block: 4 uint64 words from a 4-word counter and a 2-word key.

    Plain Python integers; this is the scalar reference that the vectorised version is checked
    against and that is checked against ``numpy.random.Philox``.
    """
    x0, x1, x2, x3 = (int(c) & _MASK for c in counter)
    k0, k1 = (int(k) & _MASK for k in key)
    for _ in range(10):
        p0 = _M0 * x0
        p1 = _M1 * x2
        hi0, lo0 = p0 >> 64, p0 & _MASK
        hi1, lo1 = p1 >> 64, p1 & _MASK
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
        k0 = (k0 + _W0) & _MASK
        k1 = (k1 + _W1) & _MASK
    return [x0, x1, x2, x3]


def _mulhilo64(a, m):
    """128-bit product of uint64 array ``a`` with the constant ``m``, as (hi, lo) uint64 arrays."""
    a = a.astype(np.uint64)
    m_lo, m_hi = np.uint64(m & 0xFFFFFFFF), np.uint64(m >> 32)
    a_lo = a & np.uint64(0xFFFFFFFF)
    a_hi = a >> np.uint64(32)
    ll = a_lo * m_lo
    lh = a_lo * m_hi
    hl = a_hi * m_lo
    hh = a_hi * m_hi
    mid = (ll >> np.uint64(32)) + (lh & np.uint64(0xFFFFFFFF)) + (hl & np.uint64(0xFFFFFFFF))
    lo = (ll & np.uint64(0xFFFFFFFF)) | (mid << np.uint64(32))
    hi = hh + (lh >> np.uint64(32)) + (hl >> np.uint64(32)) + (mid >> np.uint64(32))
    return hi, lo


def philox4x64_10_vec(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x64-10 over broadcastable uint64 arrays; returns 4 uint64 arrays."""
    with np.errstate(over="ignore"):
        shape = np.broadcast(c0, c1, c2, c3, k0, k1).shape
        x0, x1, x2, x3 = (np.broadcast_to(np.asarray(c, dtype=np.uint64), shape).copy()
                          for c in (c0, c1, c2, c3))
        k0 = np.broadcast_to(np.asarray(k0, dtype=np.uint64), shape).copy()
        k1 = np.broadcast_to(np.asarray(k1, dtype=np.uint64), shape).copy()
        for _ in range(10):
            hi0, lo0 = _mulhilo64(x0, _M0)
            hi1, lo1 = _mulhilo64(x2, _M1)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
            k0 = k0 + np.uint64(_W0)
            k1 = k1 + np.uint64(_W1)
    return x0, x1, x2, x3


def uniforms(key, index, c1=0, c2=0, c3=0):
    """53-bit uniforms in [0, 1) for draw numbers ``index`` (array) of the stream described above.

    ``key`` is a pair (k0, k1); ``index``, ``c1``, ``c2``, ``c3`` broadcast against each other.
    """
    index = np.asarray(index, dtype=np.uint64)
    words = philox4x64_10_vec(index >> np.uint64(2), c1, c2, c3, key[0], key[1])
    sel = (index & np.uint64(3)).astype(np.int64)
    w = np.choose(sel, words)
    return (w >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


# Stream identifiers (second key word) for the three places the method draws random numbers.
STREAM_COUPLINGS = 0
STREAM_PROPOSAL = 1
STREAM_ACCEPT = 2
