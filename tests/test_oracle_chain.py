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
import pytest
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


def test_observables_checkerboard_and_random_configurations():
    L = 8
    r, c = np.indices((L, L))
    cb = np.where((r + c) % 2 == 0, 1, -1).astype(np.int8)
    up = np.ones((L, L), dtype=np.int8)
    assert observables.magnetization(cb) == 0.0
    assert observables.edge_magnetization(cb) == 0.0      # each segment alternates, L/2 even
    assert observables.overlap(cb, up) == 0.0 and observables.overlap(cb, cb) == 1.0
    # random configurations against plain loops over the sites and the four edge segments
    rng = np.random.default_rng(4)
    for L in (4, 8, 12):
        s = rng.choice(np.array([-1, 1], dtype=np.int8), size=(3, L, L))
        for k in range(3):
            m = sum(int(s[k, i, j]) for i in range(L) for j in range(L)) / (L * L)
            assert observables.magnetization(s[k]) == pytest.approx(m, abs=1e-15)
            seg = range(L // 4, (3 * L) // 4)
            me = sum(int(s[k, 0, i]) + int(s[k, L - 1, i]) + int(s[k, i, 0]) + int(s[k, i, L - 1])
                     for i in seg) / (2 * L)
            assert observables.edge_magnetization(s[k]) == pytest.approx(me, abs=1e-15)
            q = sum(int(s[k, i, j]) * int(s[(k + 1) % 3, i, j])
                    for i in range(L) for j in range(L)) / (L * L)
            assert observables.overlap(s[k], s[(k + 1) % 3]) == pytest.approx(q, abs=1e-15)


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


def test_disorder_averages_closed_form():
    """Eqs. (15)-(16) and chi_edge on hand-built chains: two realizations, two chains, two steps.
    Realization A: (up, up) then (up, down): <q> = 0, <q^2> = <q^4> = 1.  Realization B:
    (checkerboard, up) then (up, up): <q> = <q^2> = <q^4> = 1/2.  So [<q>] = 1/4, [<q^2>] =
    [<q^4>] = 3/4, [<q^2>^2] = 5/8, Q_q = 6/5, chi_q = L^2 beta (3/4 - 1/16)."""
    L, beta = 8, 0.7
    r, c = np.indices((L, L))
    up = np.ones((L, L), dtype=np.int8)
    cb = np.where((r + c) % 2 == 0, 1, -1).astype(np.int8)
    A = np.array([[up, up], [up, -up]])               # (chain, step, L, L)
    B = np.array([[cb, up], [up, up]])
    rows = []
    for sp in (A, B):
        E = np.array([[-10, -12], [-14, -16]])
        rows.append(observables.accumulate(sp, E))
    out = dict(zip(observables.AVG_NAMES, observables.disorder_averages(np.array(rows), L, beta, 2)))
    assert out["q"] == pytest.approx(0.25) and out["q2"] == pytest.approx(0.75)
    assert out["q4"] == pytest.approx(0.75) and out["q2sq"] == pytest.approx(5 / 8)
    assert out["Q_q"] == pytest.approx(6 / 5)
    assert out["chi_q"] == pytest.approx(L * L * beta * (0.75 - 0.0625))
    assert out["E"] == pytest.approx(-13.0) and out["E2"] == pytest.approx((100 + 144 + 196 + 256) / 4)
    # m^2: A all 1; B: checkerboard 0, three uniform -> 3/4; [<m^2>] = 7/8
    assert out["m2"] == pytest.approx(7 / 8) and out["m4"] == pytest.approx(7 / 8)
    # m_edge^2: uniform 1, checkerboard 0 -> same as m^2 here; chi_edge = L [<m_edge^2>]
    assert out["medge2"] == pytest.approx(7 / 8) and out["chi_edge"] == pytest.approx(L * 7 / 8)
