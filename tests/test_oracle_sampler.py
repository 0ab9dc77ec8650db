"""Pins of oracle.sampler (Eqs. (4)-(6), Sec. II B sampling in reverse contraction order).

* q is a normalised distribution for any chi: sum over all 2^N configurations of q(s) = 1;
* exact regime: q(s) = P(s) for every configuration (brute force) or for random configurations
  (exact transfer matrix), i.e. every conditional equals Eq. (5);
* strips: a single row reproduces Appendix A's exact 1D sampling, q(s) = exp(-beta E) / Z_1D;
* sampling draws from q: empirical frequencies of sampled configurations match q (chi^2), and
  the draw rule, u < p+ <=> s = +1, is checked against the Philox uniforms;
* sampled and teacher-forced log q agree; gauge covariance of q in the truncated regime.
"""
import math

import numpy as np
import pytest
from scipy import stats

import synth
from oracle import energy, envbuild, exact, instance, sampler


def _setup(L, chi, seed, p=0.109, Lc=None):
    Jh, Jv = instance.couplings(seed, L, p, Lc=Lc)
    beta = instance.nishimori_beta(p)
    return Jh, Jv, beta, envbuild.build_env(Jh, Jv, beta, chi)


@pytest.mark.parametrize("L,chi", [(3, 1), (3, 2), (4, 1), (4, 2), (4, 3)])
def test_q_normalised_any_chi(L, chi):
    Jh, Jv, beta, env = _setup(L, chi, seed=L + chi)
    allc = exact.all_configs(L, L)
    q = np.exp(sampler.run(env, Jh, Jv, beta, teacher=allc)["logq"])
    assert abs(q.sum() - 1.0) < 1e-12
    if chi < 2:
        # truncated: q differs from P somewhere (the Metropolis step has work to do)
        P = np.exp(exact.brute_force(Jh, Jv, beta)["logP"])
        assert np.max(np.abs(q - P)) > 1e-6


def test_exact_regime_all_configs_4x4():
    Jh, Jv, beta, env = _setup(4, 4, seed=1)
    bf = exact.brute_force(Jh, Jv, beta)
    res = sampler.run(env, Jh, Jv, beta, teacher=bf["configs"])
    np.testing.assert_allclose(res["logq"], bf["logP"], rtol=0, atol=1e-12)
    assert res["fallbacks"] == 0


@pytest.mark.parametrize("L,chi", [(6, 8), (8, 16)])
def test_exact_regime_random_configs(L, chi):
    Jh, Jv, beta, env = _setup(L, chi, seed=L)
    lnZ = exact.transfer_matrix(Jh, Jv, beta)["lnZ"]
    s = synth.random_spins(L, 64, L)
    res = sampler.run(env, Jh, Jv, beta, teacher=s)
    np.testing.assert_allclose(res["logq"], exact.log_prob(s, Jh, Jv, beta, lnZ), rtol=1e-13,
                               atol=1e-11)
    # and for configurations the sampler itself draws
    smp = sampler.run(env, Jh, Jv, beta, K=64, seed=3)
    np.testing.assert_allclose(smp["logq"], exact.log_prob(smp["spins"], Jh, Jv, beta, lnZ),
                               rtol=1e-13, atol=1e-11)


@pytest.mark.parametrize("Lc", [3, 11])
def test_single_row_is_exact_1d_sampling(Lc):
    beta = 0.95
    Jh = instance.couplings(2, 1, 0.5, Lc=Lc)[0]
    Jv = np.zeros((0, Lc), dtype=np.int8)
    env = envbuild.build_env(Jh, Jv, beta, 1)
    s = synth.random_spins(5, 30, 1, Lc)
    lnZ1d = math.log(2) + (Lc - 1) * math.log(2 * math.cosh(beta))
    res = sampler.run(env, Jh, Jv, beta, teacher=s)
    ref = -beta * energy.energy(s, Jh, Jv) - lnZ1d
    np.testing.assert_allclose(res["logq"], ref, atol=1e-12)


def test_sampled_frequencies_match_q():
    L, chi = 3, 1
    Jh, Jv, beta, env = _setup(L, chi, seed=21, p=0.25)
    K = 60000
    smp = sampler.run(env, Jh, Jv, beta, K=K, seed=5, realization=2)
    idx = ((smp["spins"].reshape(K, -1) < 0).astype(np.int64) << np.arange(L * L)).sum(1)
    counts = np.bincount(idx, minlength=2 ** (L * L))
    q = np.exp(sampler.run(env, Jh, Jv, beta, teacher=exact.all_configs(L, L))["logq"])
    expected = K * q
    keep = expected > 5
    chi2 = float(np.sum((counts[keep] - expected[keep]) ** 2 / expected[keep]))
    pval = stats.chi2.sf(chi2, df=int(keep.sum()) - 1)
    assert pval > 1e-4
    # the log q of each sample is the log of its own probability under q
    np.testing.assert_allclose(np.exp(smp["logq"]), q[idx], rtol=1e-12)


def test_draw_rule_uses_philox_uniforms():
    Jh, Jv, beta, env = _setup(5, 2, seed=4)
    smp = sampler.run(env, Jh, Jv, beta, K=20, seed=9, realization=3, first_proposal=100)
    for r in range(5):
        u = sampler.proposal_uniforms(9, 3, 100 + np.arange(20), r, 5)
        np.testing.assert_array_equal(smp["spins"][:, r, :] > 0, u < smp["pplus"][:, r, :])


def test_teacher_forcing_reproduces_sampled_logq():
    Jh, Jv, beta, env = _setup(10, 4, seed=3)
    smp = sampler.run(env, Jh, Jv, beta, K=40, seed=1)
    tf = sampler.run(env, Jh, Jv, beta, teacher=smp["spins"])
    np.testing.assert_array_equal(tf["logq"], smp["logq"])


def test_gauge_covariance_of_q_truncated():
    L, chi, p = 8, 3, 0.109
    beta = instance.nishimori_beta(p)
    Jh, Jv = instance.couplings(14, L, p)
    e = synth.random_pm1(15, (L, L))
    Jh2 = (e[:, :-1] * Jh * e[:, 1:]).astype(np.int8)
    Jv2 = (e[:-1, :] * Jv * e[1:, :]).astype(np.int8)
    a = envbuild.build_env(Jh, Jv, beta, chi)
    b = envbuild.build_env(Jh2, Jv2, beta, chi)
    s = synth.random_spins(16, 32, L)
    la = sampler.run(a, Jh, Jv, beta, teacher=s)["logq"]
    lb = sampler.run(b, Jh2, Jv2, beta, teacher=s * e)["logq"]
    np.testing.assert_allclose(la, lb, rtol=1e-11)
