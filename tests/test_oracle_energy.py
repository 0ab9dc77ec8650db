"""Pins of oracle.energy (Sec. III A, Eq. (10)) and oracle.exact (Eqs. (1)-(2)).

A hand-worked example, symmetries of E, and Nishimori's exact disorder-averaged energy on the
Nishimori line, [<E>] = -N_B (1 - 2p), evaluated exhaustively over all disorder configurations
of a 3 x 3 lattice (the identity pins energy + enumeration together: a wrong sign, a dropped
bond or a wrong Boltzmann weight would break it).
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import energy, exact, instance


def test_hand_example_2x2():
    # spins   +1 -1      Jh = [[+1], [-1]]   Jv = [[-1, +1]]
    #         +1 +1
    # bonds: (0,0)-(0,1): J=+1, s s = -1 -> +1 to E;  (1,0)-(1,1): J=-1, s s = +1 -> +1
    #        (0,0)-(1,0): J=-1, s s = +1 -> +1;       (0,1)-(1,1): J=+1, s s = -1 -> +1
    s = np.array([[[1, -1], [1, 1]]], dtype=np.int8)
    Jh = np.array([[1], [-1]], dtype=np.int8)
    Jv = np.array([[-1, 1]], dtype=np.int8)
    assert energy.energy(s, Jh, Jv)[0] == 4


def test_symmetries():
    L = 7
    Jh, Jv = instance.couplings(2, L, 0.3)
    s = synth.random_spins(1, 40, L)
    E = energy.energy(s, Jh, Jv)
    nb = instance.bond_count(L)
    np.testing.assert_array_equal(E, energy.energy(-s, Jh, Jv))            # global flip
    assert np.all((E - nb) % 2 == 0) and np.all(np.abs(E) <= nb)             # parity, bound
    up = np.ones((1, L, L), dtype=np.int8)
    assert energy.energy(up, Jh, Jv)[0] == -(int(Jh.sum()) + int(Jv.sum()))
    # gauge covariance: J'_ij = e_i J_ij e_j, s' = e s  =>  E'(s') = E(s)
    e = synth.random_pm1(3, (L, L))
    Jh2 = (e[:, :-1] * Jh * e[:, 1:]).astype(np.int8)
    Jv2 = (e[:-1, :] * Jv * e[1:, :]).astype(np.int8)
    np.testing.assert_array_equal(energy.energy(s * e, Jh2, Jv2), E)


def test_single_flip_local_field():
    L = 6
    Jh, Jv = instance.couplings(5, L, 0.2)
    s = synth.random_spins(9, 1, L)[0]
    E0 = energy.energy(s[None], Jh, Jv)[0]
    for r, c in itertools.product(range(L), range(L)):
        h = 0
        if c > 0:
            h += Jh[r, c - 1] * s[r, c - 1]
        if c < L - 1:
            h += Jh[r, c] * s[r, c + 1]
        if r > 0:
            h += Jv[r - 1, c] * s[r - 1, c]
        if r < L - 1:
            h += Jv[r, c] * s[r + 1, c]
        t = s.copy()
        t[r, c] = -t[r, c]
        assert energy.energy(t[None], Jh, Jv)[0] - E0 == 2 * int(s[r, c]) * int(h)


@pytest.mark.parametrize("p", [0.109, 0.25])
def test_nishimori_exact_disorder_average_3x3(p):
    L = 3
    beta = instance.nishimori_beta(p)
    nb = instance.bond_count(L)
    configs = exact.all_configs(L, L)
    total = 0.0
    per_bond = 0.0
    for bits in range(2 ** nb):
        J = np.array([1 - 2 * ((bits >> j) & 1) for j in range(nb)], dtype=np.int8)
        Jh = J[:L * (L - 1)].reshape(L, L - 1)
        Jv = J[L * (L - 1):].reshape(L - 1, L)
        n_af = int(np.count_nonzero(J < 0))
        w = p ** n_af * (1 - p) ** (nb - n_af)
        bf = exact.brute_force(Jh, Jv, beta)
        P = np.exp(bf["logP"])
        total += w * float(np.sum(P * bf["E"]))
        # bond-by-bond form: [J_01 <s_0 s_1>] = 1 - 2p for the bond (0,0)-(0,1)
        per_bond += w * float(Jh[0, 0]) * float(np.sum(P * configs[:, 0, 0] * configs[:, 0, 1]))
    assert abs(total - (-nb * (1 - 2 * p))) < 1e-11
    assert abs(per_bond - (1 - 2 * p)) < 1e-12


def test_transfer_matrix_matches_brute_force():
    L = 4
    for seed in range(3):
        Jh, Jv = instance.couplings(seed, L, 0.3)
        beta = 0.8
        assert abs(exact.transfer_matrix(Jh, Jv, beta)["lnZ"]
                   - exact.brute_force(Jh, Jv, beta)["lnZ"]) < 1e-12
    # rectangular 3 x 5
    Jh, Jv = instance.couplings(1, 3, 0.4, Lc=5)
    assert abs(exact.transfer_matrix(Jh, Jv, 0.7)["lnZ"]
               - exact.brute_force(Jh, Jv, 0.7)["lnZ"]) < 1e-12


def test_bit_packing_round_trip():
    s = synth.random_spins(4, 5, 3, 130)
    w = synth.pack_rows(s)
    assert w.shape == (5, 3, 3) and w.dtype == np.uint64
    np.testing.assert_array_equal(synth.unpack_rows(w, 130), s)
    # bit j of word j // 64 is set iff the value is -1
    assert int(w[0, 0, 0]) & 1 == int(s[0, 0, 0] < 0)
