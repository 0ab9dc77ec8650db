"""Pins of oracle.philox and oracle.instance against numpy's Philox4x64-10 and printed values.

numpy.random.Philox implements the same published generator; it advances its 256-bit counter by
one before producing each block, so a generator started at counter C - 1 yields block C first.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import instance, philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_points.json")
M64 = (1 << 64) - 1


def numpy_block(counter_words, key):
    """Philox block at counter (c0..c3) from numpy, using its pre-increment."""
    c = sum(int(w) << (64 * i) for i, w in enumerate(counter_words))
    c = (c - 1) % (1 << 256)
    bg = np.random.Philox(key=np.array([int(key[0]), int(key[1])], dtype=np.uint64), counter=c)
    return [int(x) for x in bg.random_raw(4)]


@pytest.mark.parametrize("ctr,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((M64, M64, M64, M64), (M64, M64)),
    ((1, 2, 3, 4), (5, 6)),
    ((0x243F6A8885A308D3, 0x13198A2E03707344, 0xA4093822299F31D0, 0x082EFA98EC4E6C89),
     (0x452821E638D01377, 0xBE5466CF34E90C6C)),
])
def test_block_matches_numpy(ctr, key):
    assert philox.philox4x64_10(ctr, key) == numpy_block(ctr, key)


def test_vectorised_matches_scalar():
    rng = np.random.default_rng(7)
    c = rng.integers(0, 2 ** 63, size=(4, 50), dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    k = rng.integers(0, 2 ** 63, size=(2, 50), dtype=np.uint64)
    out = philox.philox4x64_10_vec(c[0], c[1], c[2], c[3], k[0], k[1])
    for j in range(50):
        ref = philox.philox4x64_10([c[i, j] for i in range(4)], [k[0, j], k[1, j]])
        assert [int(o[j]) for o in out] == ref


def test_uniform_stream_layout_matches_numpy_sequence():
    # draws 0..4n-1 with counter words (c1, c2, c3) = (0, 0, 0) are numpy's raw stream from
    # counter 0, since only word 0 of the counter advances
    n = 64
    bg = np.random.Philox(key=np.array([11, 2], dtype=np.uint64), counter=np.array([M64] * 4, dtype=np.uint64))
    raw = bg.random_raw(4 * n)
    u = philox.uniforms((11, 2), np.arange(4 * n))
    ref = (raw >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    np.testing.assert_array_equal(u, ref)
    assert np.all(u >= 0) and np.all(u < 1)


def test_uniform_counter_words():
    u = philox.uniforms((3, 1), np.arange(8), c1=5, c2=7, c3=9)
    blocks = [numpy_block((j, 5, 7, 9), (3, 1)) for j in range(2)]
    ref = [(w >> 11) * 2.0 ** -53 for b in blocks for w in b]
    np.testing.assert_array_equal(u, ref)


def test_couplings_threshold_numpy_stream():
    L, p, seed = 9, 0.3, 4
    Jh, Jv = instance.couplings(seed, L, p)
    n = L * (L - 1) * 2
    bg = np.random.Philox(key=np.array([seed, philox.STREAM_COUPLINGS], dtype=np.uint64),
                         counter=np.array([M64] * 4, dtype=np.uint64))
    u = (bg.random_raw(n) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    J = np.where(u < p, -1, 1)
    np.testing.assert_array_equal(Jh.ravel(), J[:L * (L - 1)])
    np.testing.assert_array_equal(Jv.ravel(), J[L * (L - 1):])
    assert Jh.shape == (L, L - 1) and Jv.shape == (L - 1, L)


def test_couplings_fraction_binomial():
    # i.i.d. law of Sec. III A: fraction of antiferromagnetic bonds ~ Binomial(N_B, p) / N_B
    L, p = 128, 0.109
    Jh, Jv = instance.couplings(0, L, p)
    nb = Jh.size + Jv.size
    assert nb == instance.bond_count(L) == 2 * L * (L - 1)
    frac = (np.count_nonzero(Jh < 0) + np.count_nonzero(Jv < 0)) / nb
    assert abs(frac - p) < 5 * math.sqrt(p * (1 - p) / nb)


def test_nishimori_beta_mnp_printed():
    g = json.load(open(GOLDEN))["mnp"]
    T = 1.0 / instance.nishimori_beta(g["p"])
    assert round(T, g["digits_T"]) == g["T"]


@pytest.mark.parametrize("p", [0.01, 0.10, 0.109, 0.12, 0.3])
def test_nishimori_line_definition(p):
    b = instance.nishimori_beta(p)
    assert math.isclose(math.exp(-2.0 * b), p / (1.0 - p), rel_tol=1e-14)
