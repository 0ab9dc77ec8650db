"""Sampled quantities of Sec. III C, accumulated over the steps of the chains.

* magnetisation m = (1/N) sum_i s_i;
* replica overlap q = (1/L^2) sum_i s_i^(1) s_i^(2) (two chains of the same realization);
* edge magnetisation m_edge = (1/2L) sum over four segments of length L/2 centred on the four
  edges (reading: 0-based positions i = L/4 .. 3L/4 - 1 along each edge, i.e. L/2 sites per
  edge and 2L sites in total, so that m_edge = +-1 for a uniform configuration).

Accumulator layout (one row per realization), sums over steps and chains:
  0 count of (chain, step) samples      1 sum E        2 sum E^2
  3 sum m^2                             4 sum m^4      5 sum m_edge^2
  6 sum q   (chain pair 0,1)            7 sum q^2      8 sum q^4
``disorder_averages`` forms the disorder averages of Sec. III C from these per-realization sums:
the Binder ratio Q_q, Eq. (15), the overlap susceptibility chi_q, Eq. (16), and the edge
susceptibility chi_edge.

This is test infrastructure (see the package docstring).
"""
import numpy as np

N_OBS = 9


def magnetization(s):
    s = np.asarray(s, dtype=np.float64)
    return s.reshape(s.shape[:-2] + (-1,)).mean(axis=-1)


def edge_magnetization(s):
    s = np.asarray(s, dtype=np.float64)
    L = s.shape[-1]
    a, b = L // 4, (3 * L) // 4
    tot = (s[..., 0, a:b].sum(-1) + s[..., L - 1, a:b].sum(-1)
           + s[..., a:b, 0].sum(-1) + s[..., a:b, L - 1].sum(-1))
    return tot / (2.0 * L)


def overlap(s1, s2):
    s1 = np.asarray(s1, dtype=np.float64)
    s2 = np.asarray(s2, dtype=np.float64)
    return (s1 * s2).reshape(s1.shape[:-2] + (-1,)).mean(axis=-1)


def accumulate(spins, E):
    """Sums for one realization.

    spins : (n_chain, T, L, L) configurations of each chain after each step
    E     : (n_chain, T) their energies
    """
    spins = np.asarray(spins)
    E = np.asarray(E, dtype=np.float64)
    out = np.zeros(N_OBS)
    m = magnetization(spins)
    me = edge_magnetization(spins)
    out[0] = E.size
    out[1] = E.sum()
    out[2] = (E * E).sum()
    out[3] = (m ** 2).sum()
    out[4] = (m ** 4).sum()
    out[5] = (me ** 2).sum()
    if spins.shape[0] >= 2:
        q = overlap(spins[0], spins[1])
        out[6] = q.sum()
        out[7] = (q ** 2).sum()
        out[8] = (q ** 4).sum()
    return out


N_AVG = 12
AVG_NAMES = ("E", "E2", "m2", "m4", "medge2", "q", "q2", "q4", "q2sq", "Q_q", "chi_q", "chi_edge")


def disorder_averages(accum, L, beta, n_chain):
    """Disorder averages [ ] of the thermal averages < > of Sec. III C from per-realization sums.

    accum : (n, N_OBS) sums as laid out above, one row per realization of side L
    The thermal average of realization i is its sum divided by its sample count (count/n_chain
    for the overlap, which is formed once per step from chains 0 and 1).  Returns, in the order
    of AVG_NAMES: [<E>], [<E^2>], [<m^2>], [<m^4>], [<m_edge^2>], [<q>], [<q^2>], [<q^4>],
    [<q^2>^2], the Binder ratio Q_q = [<q^4>] / [<q^2>^2] (Eq. (15)), the overlap
    susceptibility chi_q = (L^2 / T) ([<q^2>] - [<q>]^2) (Eq. (16)) and the edge susceptibility
    chi_edge = L [<m_edge^2>].
    """
    a = np.asarray(accum, dtype=np.float64)
    cnt = a[:, 0]
    th = a[:, 1:6] / cnt[:, None]                     # <E>, <E^2>, <m^2>, <m^4>, <m_edge^2>
    tq = a[:, 6:9] / (cnt / n_chain)[:, None]         # <q>, <q^2>, <q^4>
    out = np.zeros(N_AVG)
    out[0:5] = th.mean(axis=0)
    out[5:8] = tq.mean(axis=0)
    out[8] = np.mean(tq[:, 1] ** 2)
    out[9] = out[7] / out[8]
    out[10] = L * L * beta * (out[6] - out[5] ** 2)
    out[11] = L * out[4]
    return out
