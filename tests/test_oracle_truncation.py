"""Pins of the truncation in oracle.envbuild.compress (Sec. II B: SVD truncation of the bond
dimension to D = chi).

The exact-regime, strip and Onsager pins never truncate, and gauge covariance and the
normalisation of q hold for any truncation, so they cannot tell which singular directions the
compression keeps.  These pins can, with dense vectors built by independent code (the exact
row transfer operator of oracle.exact and SVDs of the unfoldings):

* one cut (Eckart-Young): when exactly one bond of the row-operator-applied MPS exceeds chi, the
  canonical compression must return the best rank-chi approximation of that exact vector at the
  cut, entry by entry, its squared error must equal the sum of the discarded squared singular
  values, and its norm must fall below the exact norm by exactly that amount;
* several cuts (TT-SVD bound, Oseledets, SIAM J. Sci. Comput. 33 (2011), Thm. 2.2): a sweep of
  SVD truncations from one end of a vector whose other sites are isometries has squared error at
  most the sum over cuts of the exact unfoldings' discarded squared singular values, and at least
  the largest of them;
* bond dimension: ln Z_TN approaches the exact ln Z monotonically over chi = 1, 2, 4, 8, 16 at
  L = 8 (16 is exact), and is far off at chi = 1.

Keeping the smallest singular values, swapping U and V at a bond, or dropping the carried S all
fail the first pin.
"""
import math

import numpy as np
import pytest

from oracle import envbuild, exact, instance


def mps_vector(sites):
    """Dense vector of an MPS: index sum_c bit_c 2^c, bit_c = 1 iff the spin of column c is -1
    (the row-state convention of oracle.exact)."""
    Lc = len(sites)
    v = sites[0][0]                                   # (2, dr): physical index of column 0
    for c in range(1, Lc):
        A = sites[c]                                  # (dl, 2, dr)
        # v[(bits of columns < c), a] -> new[(bit c), (bits < c), b]
        v = np.einsum("ia,asb->sib", v, A).reshape(-1, A.shape[2])
    assert v.shape[1] == 1
    return v[:, 0]


def apply_row_dense(vec, Jh_row, Jv_row, beta, Lc):
    """(V H f)(x) for a dense f over row states: the exact row operator of oracle.exact."""
    ys = exact._row_spins(Lc)
    f = np.exp(exact._row_weight(Jh_row, beta, ys)) * vec
    return exact._apply_vertical(f, Jv_row, beta, Lc)


def unfolding(vec, Lc, cut):
    """Matrix of the vector with columns 0..cut-1 as the column index, cut..Lc-1 as the row index
    (C order of the row-state index: the high bits are the later columns)."""
    return vec.reshape(2 ** (Lc - cut), 2 ** cut)


def last_step(L, Lc, chi, seed, p=0.3, beta=0.9):
    """The compressed E_0 of an L x Lc lattice at bond chi, the exact row operator applied to the
    (possibly truncated) E_1 from which it was compressed, and the couplings."""
    Jh, Jv = instance.couplings(seed, L, p, Lc=Lc)
    env = envbuild.build_env(Jh, Jv, beta, chi)
    e1 = math.exp(env["lognorm"][1]) * mps_vector(env["sites"][1])
    exact_e0 = apply_row_dense(e1, Jh[1], Jv[0], beta, Lc)
    trunc_e0 = math.exp(env["lognorm"][0]) * mps_vector(env["sites"][0])
    return exact_e0, trunc_e0, env


@pytest.mark.parametrize("chi,seed", [(4, 0), (5, 1), (6, 2)])
def test_single_cut_is_best_rank_chi_approximation(chi, seed):
    # 4 rows x 6 columns: E_1 has rank <= 4 at every cut (exact at chi >= 4); applying row 1 gives
    # rank <= 8 at the middle cut (c = 3) and <= 4 elsewhere, so only that cut is truncated
    # (beta = 0.9, p = 0.3: the discarded singular values are 1e-7 .. 1e-4 of the largest).
    L, Lc, cut = 4, 6, 3
    exact_e0, trunc_e0, env = last_step(L, Lc, chi, seed)
    U, S, Vt = np.linalg.svd(unfolding(exact_e0, Lc, cut), full_matrices=False)
    assert S[chi] > 1e-8 * S[0] and S[chi - 1] - S[chi] > 1e-8 * S[0]   # a real, unique cut
    for c in range(1, Lc):
        if c != cut:
            s_c = np.linalg.svd(unfolding(exact_e0, Lc, c), compute_uv=False)
            assert np.sum(s_c > 1e-12 * s_c[0]) <= chi                  # no truncation there
    best = (U[:, :chi] * S[:chi]) @ Vt[:chi]
    got = unfolding(trunc_e0, Lc, cut)
    scale = np.linalg.norm(exact_e0)
    np.testing.assert_allclose(got, best, rtol=0, atol=1e-11 * scale)
    discarded = float(np.sum(S[chi:] ** 2))
    err2 = float(np.sum((exact_e0 - trunc_e0) ** 2))
    assert abs(err2 - discarded) < 1e-6 * discarded
    # the truncated norm is below the exact one by exactly the discarded weight (the difference
    # of two norms cancels: rounding of 1e-16 relative to the norm remains)
    n2_exact, n2_trunc = float(np.sum(exact_e0 ** 2)), math.exp(2 * env["lognorm"][0])
    assert abs((n2_exact - n2_trunc) - discarded) < 1e-3 * discarded + 1e-14 * scale ** 2
    assert env["lognorm"][0] < 0.5 * math.log(n2_exact)


@pytest.mark.parametrize("chi,seed", [(3, 3), (4, 4), (5, 5)])
def test_several_cuts_tt_svd_error_bound(chi, seed):
    # 5 rows x 8 columns: several cuts exceed chi in the last compression
    L, Lc = 5, 8
    exact_e0, trunc_e0, env = last_step(L, Lc, chi, seed)
    tails = []
    for c in range(1, Lc):
        s_c = np.linalg.svd(unfolding(exact_e0, Lc, c), compute_uv=False)
        tails.append(float(np.sum(s_c[chi:] ** 2)))
    assert sum(t > 0 for t in tails) >= 2
    err2 = float(np.sum((exact_e0 - trunc_e0) ** 2))
    scale2 = float(np.sum(exact_e0 ** 2))
    assert err2 <= sum(tails) * (1 + 1e-9) + 1e-13 * scale2
    # no rank-chi approximation at any single cut beats Eckart-Young there
    assert err2 >= max(tails) * (1 - 1e-9) - 1e-13 * scale2
    # and the kept state is not far from the exact one
    assert err2 < 0.5 * scale2


@pytest.mark.parametrize("seed", [7, 8, 9])
def test_lnz_error_monotone_in_chi(seed):
    L, p = 8, 0.109
    beta = instance.nishimori_beta(p)
    Jh, Jv = instance.couplings(seed, L, p)
    ref = exact.transfer_matrix(Jh, Jv, beta)["lnZ"]
    errs = [abs(envbuild.build_env(Jh, Jv, beta, chi)["lnZ"] - ref) for chi in (1, 2, 4, 8, 16)]
    assert errs[-1] < 1e-11 * abs(ref)                       # chi = 16 = 2^(L/2) is exact
    for a, b in zip(errs, errs[1:]):
        assert b <= a * (1 + 1e-9) + 1e-12 * abs(ref), errs
    assert errs[0] > 1e-3                                     # chi = 1 is a real truncation
