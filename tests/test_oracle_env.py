"""Pins of oracle.envbuild (Sec. II B contraction with SVD truncation).

* exact regime (chi >= 2^floor(Lc/2)): ln Z and every ln ||E_r|| equal the exact transfer matrix
  (independent code) and brute-force enumeration;
* strips: a single column / single row is a 1D chain, whose process vectors and partition function
  Appendix A gives in closed form, Z = 2 (2 cosh beta)^(L-1) for any +-1 couplings;
* p = 0, large chi: the second difference of ln Z over L tends to Onsager's bulk free energy;
* truncated regime: gauge covariance (J'_ij = e_i J_ij e_j leaves the truncated contraction
  invariant) and right-orthonormality of the stored sites.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

import synth
from oracle import envbuild, exact, instance

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_points.json")


@pytest.mark.parametrize("L,chi,seed,p", [(3, 2, 0, 0.3), (4, 4, 1, 0.109), (6, 8, 2, 0.109),
                                          (8, 16, 3, 0.2), (10, 32, 4, 0.109)])
def test_exact_regime_matches_transfer_matrix(L, chi, seed, p):
    Jh, Jv = instance.couplings(seed, L, p)
    beta = instance.nishimori_beta(p)
    env = envbuild.build_env(Jh, Jv, beta, chi)
    tm = exact.transfer_matrix(Jh, Jv, beta)
    assert abs(env["lnZ"] - tm["lnZ"]) < 1e-12 * abs(tm["lnZ"]) + 1e-12
    np.testing.assert_allclose(env["lognorm"], tm["lognorm"], rtol=1e-13, atol=1e-12)
    if L <= 4:
        assert abs(env["lnZ"] - exact.brute_force(Jh, Jv, beta)["lnZ"]) < 1e-12


def test_exact_regime_rectangular_and_functions():
    # 5 rows x 4 columns, chi = 4 is exact; compare the represented E_r(x) entry by entry
    Jh, Jv = instance.couplings(6, 5, 0.3, Lc=4)
    beta = 0.9
    env = envbuild.build_env(Jh, Jv, beta, 4)
    tm = exact.transfer_matrix(Jh, Jv, beta)
    ys = exact.all_configs(1, 4)[:, 0, :]
    for r in range(5):
        sites = env["sites"][r]
        vals = []
        for y in ys:
            m = np.ones((1, 1))
            for c in range(4):
                m = m @ sites[c][:, 0 if y[c] > 0 else 1, :]
            vals.append(m[0, 0])
        vals = np.exp(env["lognorm"][r]) * np.array(vals)
        sc, vec = tm["envs"][r]
        np.testing.assert_allclose(vals, np.exp(sc) * vec, rtol=1e-12)


@pytest.mark.parametrize("L", [2, 5, 9])
def test_strip_single_column_closed_form(L):
    # one column: E_r of the single site is (2 cosh b)^(L-1-r) for both spins (Appendix A's
    # process vectors z_i = (2 cosh b)^(L-i)), so ln ||E_r|| = ln sqrt(2) + (L-1-r) ln(2 cosh b)
    beta = 0.83
    Jh, Jv = instance.couplings(8, L, 0.4, Lc=1)
    env = envbuild.build_env(Jh, Jv, beta, 1)
    r = np.arange(L)
    ref = 0.5 * math.log(2) + (L - 1 - r) * math.log(2 * math.cosh(beta))
    np.testing.assert_allclose(env["lognorm"], ref, rtol=1e-14)
    assert abs(env["lnZ"] - (math.log(2) + (L - 1) * math.log(2 * math.cosh(beta)))) < 1e-12


@pytest.mark.parametrize("Lc", [2, 6, 17])
def test_strip_single_row_closed_form(Lc):
    beta = 1.1
    Jh = instance.couplings(9, 1, 0.5, Lc=Lc)[0]
    Jv = np.zeros((0, Lc), dtype=np.int8)
    env = envbuild.build_env(Jh, Jv, beta, 1)
    assert abs(env["lnZ"] - (math.log(2) + (Lc - 1) * math.log(2 * math.cosh(beta)))) < 1e-12


def onsager_minus_beta_f(beta):
    """Onsager's bulk -beta f of the square-lattice Ising model (textbook closed form)."""
    c2, s2 = math.cosh(2 * beta) ** 2, math.sinh(2 * beta)
    val, _ = integrate.dblquad(lambda t1, t2: math.log(c2 - s2 * (math.cos(t1) + math.cos(t2))),
                               0, math.pi, 0, math.pi, epsabs=1e-13, epsrel=1e-13)
    return math.log(2) + val / (2 * math.pi ** 2)


def test_onsager_formula_critical_point_printed():
    # the log argument reaches 0 exactly at the printed pure-Ising T_c = 2 / ln(1 + sqrt 2)
    g = json.load(open(GOLDEN))["pure_ising_tc"]
    Tc = 2.0 / math.log(1.0 + math.sqrt(2.0))
    assert g["T"] == "2/ln(1+sqrt(2))"
    b = 1.0 / Tc
    assert abs(math.cosh(2 * b) ** 2 - 2 * math.sinh(2 * b)) < 1e-14


def test_onsager_bulk_free_energy_p0():
    beta = 0.3
    Jz = lambda L: (np.ones((L, L - 1), np.int8), np.ones((L - 1, L), np.int8))
    lnz = {}
    for L in (10, 11, 12):
        Jh, Jv = Jz(L)
        lnz[L] = envbuild.build_env(Jh, Jv, beta, 64)["lnZ"]
    second = 0.5 * (lnz[12] - 2 * lnz[11] + lnz[10])
    assert abs(second - onsager_minus_beta_f(beta)) < 1e-7


@pytest.mark.parametrize("L,chi", [(8, 4), (12, 6)])
def test_gauge_covariance_truncated(L, chi):
    p = 0.109
    beta = instance.nishimori_beta(p)
    Jh, Jv = instance.couplings(11, L, p)
    e = synth.random_pm1(12, (L, L))
    Jh2 = (e[:, :-1] * Jh * e[:, 1:]).astype(np.int8)
    Jv2 = (e[:-1, :] * Jv * e[1:, :]).astype(np.int8)
    a = envbuild.build_env(Jh, Jv, beta, chi)
    b = envbuild.build_env(Jh2, Jv2, beta, chi)
    assert envbuild.sensitivity(a, 1e-15) < 1e-10
    np.testing.assert_allclose(a["lognorm"], b["lognorm"], rtol=1e-12)
    assert abs(a["lnZ"] - b["lnZ"]) < 1e-11 * abs(a["lnZ"])
    # the truncation is real: the truncated lnZ differs from the exact one
    assert abs(a["lnZ"] - exact.transfer_matrix(Jh, Jv, beta)["lnZ"]) > 1e-8


def test_right_canonical_sites_and_unit_norm():
    Jh, Jv = instance.couplings(13, 9, 0.109)
    env = envbuild.build_env(Jh, Jv, instance.nishimori_beta(0.109), 5)
    for r in range(9):
        sites = env["sites"][r]
        for A in sites[1:]:
            M = A.reshape(A.shape[0], -1)
            np.testing.assert_allclose(M @ M.T, np.eye(A.shape[0]), atol=1e-12)
        assert abs(np.linalg.norm(sites[0]) - 1.0) < 1e-13
        assert max(A.shape[0] for A in sites) <= 5
