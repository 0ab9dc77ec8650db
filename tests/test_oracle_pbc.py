"""Pins of the site fields (oracle.energy / envbuild / sampler with field=h) and of oracle.pbc,
the periodic lattice by a frozen line pair and its open block (Sec. IV; Sec. I).

* torus energy: invariance under translating spins and couplings together (a wrong wrap index
  breaks it) and the open-lattice energy plus the explicit wrap bonds;
* block decomposition: E_torus(merge(s, s_b)) - E_block(s_b) does not depend on the block
  configuration s_b and equals minus the bonds between frozen spins (a wrong field sign, index or
  neighbour breaks it);
* field build and sampling in the exact regime: ln Z_TN equals brute-force enumeration of the
  open lattice in its fields, and q(s) = P(s | fields) for every configuration;
* the whole step: at exact chi every proposal is accepted; with chi = 1 (biased proposals) the
  chain of steps over random lines reproduces the exact torus energy histogram.
"""
import math

import numpy as np
import pytest
from scipy import stats

import synth
from oracle import energy, envbuild, exact, instance, pbc, sampler


def _torus_case(seed, L, p=0.3):
    Jh_t, Jv_t = synth.torus_couplings(seed, L, p)
    s_t = synth.random_spins(seed + 100, 1, L)[0]
    return Jh_t, Jv_t, s_t


@pytest.mark.parametrize("L", [3, 4, 6])
def test_torus_energy_translation_and_wrap(L):
    Jh_t, Jv_t, _ = _torus_case(L, L)
    s = synth.random_spins(7, 20, L)
    E = pbc.torus_energy(s, Jh_t, Jv_t)
    for dr, dc in [(1, 0), (0, 1), (2, 3)]:
        Er = pbc.torus_energy(np.roll(s, (dr, dc), axis=(1, 2)), np.roll(Jh_t, (dr, dc), axis=(0, 1)),
                              np.roll(Jv_t, (dr, dc), axis=(0, 1)))
        np.testing.assert_array_equal(Er, E)
    s64 = s.astype(np.int64)
    wrap = -(Jh_t[:, L - 1][None, :] * s64[:, :, L - 1] * s64[:, :, 0]).sum(axis=1) \
        - (Jv_t[L - 1, :][None, :] * s64[:, L - 1, :] * s64[:, 0, :]).sum(axis=1)
    np.testing.assert_array_equal(E, energy.energy(s, Jh_t[:, :L - 1], Jv_t[:L - 1, :]) + wrap)
    up = np.ones((1, L, L), dtype=np.int8)
    assert pbc.torus_energy(up, Jh_t, Jv_t)[0] == -(int(Jh_t.sum()) + int(Jv_t.sum()))


def _frozen_bond_energy(Jh_t, Jv_t, s_t, r0, c0):
    """-sum of J s s over torus bonds with both ends on the frozen row or column."""
    L = s_t.shape[0]
    on = lambda r, c: r == r0 or c == c0
    E = 0
    for r in range(L):
        for c in range(L):
            if on(r, c) and on(r, (c + 1) % L):
                E -= int(Jh_t[r, c]) * int(s_t[r, c]) * int(s_t[r, (c + 1) % L])
            if on(r, c) and on((r + 1) % L, c):
                E -= int(Jv_t[r, c]) * int(s_t[r, c]) * int(s_t[(r + 1) % L, c])
    return E


@pytest.mark.parametrize("L,r0,c0", [(3, 0, 0), (3, 2, 1), (4, 1, 3), (5, 4, 2), (6, 0, 5)])
def test_block_decomposition_constant_offset(L, r0, c0):
    Jh_t, Jv_t, s_t = _torus_case(10 * L + r0, L)
    Jh, Jv, h, s_b = pbc.block(Jh_t, Jv_t, s_t, r0, c0)
    assert Jh.shape == (L - 1, L - 2) and Jv.shape == (L - 2, L - 1) and h.shape == (L - 1, L - 1)
    # the block's own part, and the torus state rebuilt from it, unchanged
    np.testing.assert_array_equal(pbc.merge(s_t, s_b, r0, c0), s_t)
    off = _frozen_bond_energy(Jh_t, Jv_t, s_t, r0, c0)
    blocks = synth.random_spins(L + 3, 25, L - 1)
    Eb = energy.energy(blocks, Jh, Jv, field=h)
    Et = np.array([pbc.torus_energy(pbc.merge(s_t, b, r0, c0)[None], Jh_t, Jv_t)[0] for b in blocks])
    np.testing.assert_array_equal(Et - Eb, np.full(len(blocks), off))
    # only the block's boundary carries fields, and at most two frozen neighbours each
    inner = h[1:-1, 1:-1]
    assert not inner.any() and np.abs(h).max() <= 2


@pytest.mark.parametrize("shape,seed", [((3, 3), 0), ((3, 4), 1), ((4, 4), 2), ((2, 5), 3)])
def test_field_build_and_sampler_exact(shape, seed):
    """Arbitrary integer fields on an open lattice (a partial block), exact chi."""
    Lr, Lc = shape
    Jh, Jv = instance.couplings(seed, Lr, 0.3, Lc=Lc)
    rng = np.random.default_rng(seed)
    h = rng.integers(-2, 3, size=(Lr, Lc)).astype(np.int8)
    beta = 0.8
    chi = 2 ** (min(Lr, Lc) // 2 + 1)
    env = envbuild.build_env(Jh, Jv, beta, chi, field=h)
    bf = exact.brute_force(Jh, Jv, beta, field=h)
    assert abs(env["lnZ"] - bf["lnZ"]) < 1e-11 * abs(bf["lnZ"]) + 1e-12
    # differs from the field-free lattice (the field is used)
    assert abs(exact.brute_force(Jh, Jv, beta)["lnZ"] - bf["lnZ"]) > 1e-3
    q = sampler.run(env, Jh, Jv, beta, teacher=bf["configs"], field=h)
    np.testing.assert_allclose(q["logq"], bf["logP"], rtol=0, atol=1e-10)
    # zero fields: the same environments as no fields, bit for bit
    z = envbuild.build_env(Jh, Jv, beta, chi, field=np.zeros_like(h))
    o = envbuild.build_env(Jh, Jv, beta, chi)
    np.testing.assert_array_equal(z["lognorm"], o["lognorm"])


def test_step_exact_chi_accepts_everything():
    L, beta = 5, 0.9
    Jh_t, Jv_t, s_t = _torus_case(3, L)
    lines = synth.frozen_lines(4, 6, L)
    acc = 0
    for t, (r0, c0) in enumerate(lines):
        s_t, info = pbc.step(Jh_t, Jv_t, s_t, beta, 8, int(r0), int(c0), K=10, seed=1,
                             first_proposal=10 * t, first_step=10 * t)
        acc += int(info["chain"]["accepted"].sum())
        # exact chi: log w = -beta E - log q is the same for every block configuration
        lw = -beta * info["E_prop"] - info["proposals"]["logq"]
        lw0 = -beta * info["E_cur"] - info["logq_cur"]
        assert np.max(np.abs(lw - lw0)) < 1e-10
    assert acc == 6 * 10


def test_step_init_takes_first_proposal():
    """A fresh start: the step's first proposal becomes the state unconditionally (not counted
    as accepted), and the rest of the step is the chain from there."""
    L, beta = 5, 0.9
    Jh_t, Jv_t, s_t = _torus_case(8, L)
    s_new, info = pbc.step(Jh_t, Jv_t, s_t, beta, 2, 1, 3, K=6, seed=3, init=True)
    ch = info["chain"]
    assert ch["init"][0] and not ch["accepted"][0] and ch["current"][0] == 0
    assert info["logq_cur"] is None
    final = int(ch["current"][-1])
    np.testing.assert_array_equal(s_new, pbc.merge(s_t, info["proposals"]["spins"][final], 1, 3))


def test_pbc_chain_reproduces_torus_histogram():
    """chi = 1 on the 3 x 3 blocks of a 4 x 4 torus: biased proposals, exact chain."""
    L, beta, K, steps = 4, 0.7, 4, 3000
    Jh_t, Jv_t, s_t = _torus_case(5, L, p=0.25)
    lines = synth.frozen_lines(6, steps, L)
    Es, acc = [], 0
    for t, (r0, c0) in enumerate(lines):
        s_t, info = pbc.step(Jh_t, Jv_t, s_t, beta, 1, int(r0), int(c0), K=K, seed=2,
                             first_proposal=K * t, first_step=K * t)
        acc += int(info["chain"]["accepted"].sum())
        Es.append(int(pbc.torus_energy(s_t[None], Jh_t, Jv_t)[0]))
    pa = acc / (K * steps)
    assert 0.05 < pa < 0.99
    allc = exact.all_configs(L, L)
    Eall = pbc.torus_energy(allc, Jh_t, Jv_t)
    lw = -beta * Eall.astype(np.float64)
    P = np.exp(lw - lw.max())
    P /= P.sum()
    levels = np.unique(Eall)
    Pl = np.array([P[Eall == e].sum() for e in levels])
    Es = np.array(Es)
    counts = np.array([np.count_nonzero(Es == e) for e in levels], dtype=np.float64)
    expected = len(Es) * Pl
    keep = expected > 10
    # successive steps share the frozen lines' spins: inflate by an integrated time of ~4
    chi2 = float(np.sum((counts[keep] - expected[keep]) ** 2 / expected[keep])) / 4.0
    assert stats.chi2.sf(chi2, df=int(keep.sum()) - 1) > 1e-4
    mean_exact = float((P * Eall).sum())
    assert abs(Es.mean() - mean_exact) < 0.6
