"""Pins of oracle.accept and the whole oracle chain (Eq. (3); Appendix A), and oracle.observables.

* Appendix A's periodic 1D example: free-chain proposals for a periodic target are accepted with
  probability min{1, exp(beta s'_1 s'_L) / exp(beta s_1 s_L)}; the decisions of the chain must be
  exactly u < that probability;
* the chain over deliberately poor proposals (chi = 1) reproduces the exact Boltzmann energy
  histogram, while the raw proposals do not;
* Nishimori's [<E>] = -N_B (1 - 2p) through the full TNMC chain, disorder-averaged;
* observables: definitions on special configurations and Nishimori's [<q^2>] = [<m^2>] using
  exact samples.
"""
import math

import numpy as np
from scipy import stats

from oracle import accept, energy, envbuild, exact, instance, observables, sampler


def test_periodic_1d_acceptance_closed_form():
    L, beta, K = 12, 0.7, 400
    # proposals from the free chain (all J = +1): exact Bayes sampling of Appendix A
    Jh = np.ones((1, L - 1), dtype=np.int8)
    Jv = np.zeros((0, L), dtype=np.int8)
    env = envbuild.build_env(Jh, Jv, beta, 1)
    smp = sampler.run(env, Jh, Jv, beta, K=K, seed=2)
    s = smp["spins"][:, 0, :].astype(np.int64)
    # target: periodic chain, E_P = E_free - s_1 s_L
    E_P = energy.energy(smp["spins"], Jh, Jv) - s[:, 0] * s[:, -1]
    out = accept.chain(E_P, smp["logq"], beta, seed=4, realization=1, chain_index=0)
    u = accept.accept_uniforms(4, 1, 0, np.arange(K))
    cur = 0
    for k in range(1, K):
        pa = min(1.0, math.exp(beta * s[k, 0] * s[k, -1]) / math.exp(beta * s[cur, 0] * s[cur, -1]))
        acc = u[k] < pa
        assert out["accepted"][k] == acc or abs(u[k] - pa) < 1e-12
        if out["accepted"][k]:
            cur = k
        assert out["current"][k] == cur
    assert out["init"][0] and not out["accepted"][0]


def _energy_hist_pvalue(E_samples, E_levels, P_levels, inflation):
    counts = np.array([np.count_nonzero(E_samples == e) for e in E_levels], dtype=np.float64)
    n = len(E_samples)
    expected = n * P_levels
    keep = expected > 10
    chi2 = float(np.sum((counts[keep] - expected[keep]) ** 2 / expected[keep])) / inflation
    return stats.chi2.sf(chi2, df=int(keep.sum()) - 1)


def test_chain_reproduces_exact_energy_histogram():
    L, chi, p = 4, 1, 0.109
    beta = instance.nishimori_beta(p)
    Jh, Jv = instance.couplings(30, L, p)
    env = envbuild.build_env(Jh, Jv, beta, chi)
    K = 120000
    smp = sampler.run(env, Jh, Jv, beta, K=K, seed=6)
    E = energy.energy(smp["spins"], Jh, Jv)
    out = accept.chain(E, smp["logq"], beta, seed=6)
    pa = out["accepted"].sum() / (K - 1)
    assert 0.05 < pa < 0.999
    chainE = E[out["current"]]
    bf = exact.brute_force(Jh, Jv, beta)
    levels = np.unique(bf["E"])
    P = np.array([np.exp(bf["logP"][bf["E"] == e]).sum() for e in levels])
    tau = 2.0 / pa                                    # independence sampler: tau ~ 1/p_a
    assert _energy_hist_pvalue(chainE, levels, P, inflation=tau) > 1e-4
    # the uncorrected proposals are measurably biased
    assert _energy_hist_pvalue(E, levels, P, inflation=1.0) < 1e-6


def test_nishimori_identity_through_tnmc_chain():
    L, chi, p = 5, 2, 0.109
    beta = instance.nishimori_beta(p)
    nb = instance.bond_count(L)
    means = []
    for seed in range(60):
        Jh, Jv = instance.couplings(seed, L, p)
        env = envbuild.build_env(Jh, Jv, beta, chi)
        smp = sampler.run(env, Jh, Jv, beta, K=1500, seed=0, realization=seed)
        E = energy.energy(smp["spins"], Jh, Jv)
        out = accept.chain(E, smp["logq"], beta, seed=0, realization=seed)
        means.append(E[out["current"]].mean())
    means = np.array(means)
    target = -nb * (1 - 2 * p)
    err = means.std(ddof=1) / math.sqrt(len(means))
    assert abs(means.mean() - target) < 5 * err + 0.05


def test_observables_definitions():
    L = 8
    up = np.ones((1, 1, L, L), dtype=np.int8)
    acc = observables.accumulate(np.concatenate([up, -up]), np.array([[3], [5]]))
    assert acc[0] == 2 and acc[1] == 8 and acc[2] == 34
    assert acc[3] == 2 and acc[4] == 2 and acc[5] == 2          # m^2, m^4, m_edge^2 of +-uniform
    assert acc[6] == -1 and acc[7] == 1 and acc[8] == 1          # q of opposite uniform states
    s = np.ones((L, L), dtype=np.int8)
    s[L // 4:(3 * L) // 4, 0] = -1                                # flip the left segment
    assert observables.edge_magnetization(s) == (2 * L - 2 * (L // 2)) / (2 * L)
    s2 = np.ones((L, L), dtype=np.int8)
    s2[L // 4 - 1, 0] = -1                                        # outside the segment
    assert observables.edge_magnetization(s2) == 1.0


def test_nishimori_overlap_equals_magnetisation_exact_samples():
    # [<q^2>] = [<m^2>] on the Nishimori line (gauge identity), with exact samples per realization
    L, p = 3, 0.109
    beta = instance.nishimori_beta(p)
    rng = np.random.default_rng(0)
    q2, m2 = [], []
    for seed in range(400):
        Jh, Jv = instance.couplings(seed, L, p)
        bf = exact.brute_force(Jh, Jv, beta)
        P = np.exp(bf["logP"])
        idx = rng.choice(len(P), size=(2, 400), p=P / P.sum())
        acc = observables.accumulate(bf["configs"][idx], bf["E"][idx])
        q2.append(acc[7] / 400)
        m2.append(acc[3] / 800)
    q2, m2 = np.array(q2), np.array(m2)
    d = q2 - m2
    assert abs(d.mean()) < 5 * d.std(ddof=1) / math.sqrt(len(d)) + 1e-3
