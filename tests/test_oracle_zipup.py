"""Pins of the zip-up mode of oracle.envbuild (the contraction variant of Sec. II B listed as a
next step: one sweep of SVD truncations, Stoudenmire and White 2010).

* exact regime: with chi >= 2^floor(Lc/2) nothing is truncated and every lambda_r and ln Z equal
  the exact transfer matrix;
* gauge: each sweep leaves the sites behind it orthonormal (right-orthonormal after a right-to-
  left sweep, left-orthonormal after a left-to-right one), the stored MPS has unit norm, and the
  directions alternate row by row;
* every truncated row against the same sweep done with dense projections (independent code on
  full configuration spaces): right to left, the block to the right of each cut is projected on
  its chi leading right singular vectors; left to right, the block to the left on its leading
  left singular vectors; no zip-up row beats the optimal truncation at its worst cut;
* gauge covariance in the truncated regime.
"""
import math

import numpy as np
import pytest

import synth
from oracle import envbuild, exact, instance

from test_oracle_truncation import apply_row_dense, mps_vector, unfolding


@pytest.mark.parametrize("L,chi,seed,p", [(4, 4, 1, 0.109), (6, 8, 2, 0.109), (8, 16, 3, 0.2),
                                          (9, 16, 5, 0.3)])
def test_zipup_exact_regime(L, chi, seed, p):
    Jh, Jv = instance.couplings(seed, L, p)
    beta = instance.nishimori_beta(p)
    env = envbuild.build_env(Jh, Jv, beta, chi, method="zipup")
    tm = exact.transfer_matrix(Jh, Jv, beta)
    assert abs(env["lnZ"] - tm["lnZ"]) < 1e-12 * abs(tm["lnZ"])
    np.testing.assert_allclose(env["lognorm"], tm["lognorm"], rtol=1e-13, atol=1e-12)


def test_zipup_gauge_and_alternation():
    L = 9
    Jh, Jv = instance.couplings(13, L, 0.109)
    env = envbuild.build_env(Jh, Jv, instance.nishimori_beta(0.109), 5, method="zipup")
    assert [envbuild.zipup_direction(L, r) for r in range(L - 1, 0, -1)][:4] == ["rl", "lr",
                                                                                "rl", "lr"]
    for r in range(L - 1):
        sites = env["sites"][r]
        assert abs(np.linalg.norm(mps_vector(sites)) - 1.0) < 1e-12
        if envbuild.zipup_direction(L, r + 1) == "rl":          # E_r came from a right-to-left sweep
            for A in sites[1:]:
                M = A.reshape(A.shape[0], -1)
                np.testing.assert_allclose(M @ M.T, np.eye(A.shape[0]), atol=1e-12)
        else:
            for A in sites[:-1]:
                M = A.reshape(-1, A.shape[2])
                np.testing.assert_allclose(M.T @ M, np.eye(A.shape[2]), atol=1e-12)
        assert max(A.shape[0] for A in sites) <= 5


def dense_zipup(big, chi, direction):
    """The zip-up as projections of dense blocks: sweeping right to left, the block of the
    operator-applied MPS to the right of each cut (bond index x every configuration of the
    swept columns) is replaced by its projection on its chi leading right singular vectors;
    left to right, the block to the left by the projection on its chi leading left singular
    vectors.  Returns the dense vector (bit c of the index = column c)."""
    Lc = len(big)
    if direction == "rl":
        R = np.ones((1, 1))                                   # (bond at the right end, configs)
        shape = ()
        for c in range(Lc - 1, 0, -1):
            R = np.einsum("asb,b...->as...", big[c], R.reshape((R.shape[0],) + shape))
            shape = (2,) + shape
            M = R.reshape(R.shape[0], -1)
            _, _, Vt = np.linalg.svd(M, full_matrices=False)
            k = min(chi, Vt.shape[0])
            R = M @ Vt[:k].T @ Vt[:k]
        full = np.einsum("asb,b...->as...", big[0], R.reshape((R.shape[0],) + shape))[0]
    else:
        Lb = np.ones((1, 1))                                  # (configs, bond at the left end)
        shape = ()
        for c in range(Lc - 1):
            Lb = np.einsum("...a,asb->...sb", Lb.reshape(shape + (Lb.shape[-1],)), big[c])
            shape = shape + (2,)
            M = Lb.reshape(-1, Lb.shape[-1])
            U, _, _ = np.linalg.svd(M, full_matrices=False)
            k = min(chi, U.shape[1])
            Lb = U[:, :k] @ U[:, :k].T @ M
        full = np.einsum("...a,asb->...sb", Lb.reshape(shape + (Lb.shape[-1],)), big[Lc - 1])[..., 0]
    # axes (s_0, ..., s_{Lc-1}) -> index with s_0 the lowest bit
    return full.transpose(tuple(range(Lc - 1, -1, -1))).reshape(-1)


@pytest.mark.parametrize("L,Lc,chi,seed", [(5, 6, 3, 0), (5, 6, 4, 1), (6, 7, 4, 2), (6, 8, 5, 3)])
def test_zipup_matches_dense_projections(L, Lc, chi, seed):
    """Every row of a truncated zip-up build against the same sweep done with dense
    projections (both directions occur: the rows alternate)."""
    beta = 0.9
    Jh, Jv = instance.couplings(seed, L, 0.3, Lc=Lc)
    env = envbuild.build_env(Jh, Jv, beta, chi, method="zipup")
    truncated = 0
    for r in range(L - 1, 0, -1):
        big = envbuild.apply_row_mpo(env["sites"][r], Jh[r], Jv[r - 1], beta)
        ref = math.exp(env["lognorm"][r]) * dense_zipup(big, chi, envbuild.zipup_direction(L, r))
        got = math.exp(env["lognorm"][r - 1]) * mps_vector(env["sites"][r - 1])
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-11 * np.linalg.norm(ref))
        exact_next = apply_row_dense(math.exp(env["lognorm"][r]) * mps_vector(env["sites"][r]),
                                     Jh[r], Jv[r - 1], beta, Lc)
        if np.linalg.norm(got - exact_next) > 1e-8 * np.linalg.norm(exact_next):
            truncated += 1
            # no truncation beats the optimal one at the worst cut (Eckart-Young)
            best = max(float(np.sum(np.linalg.svd(unfolding(exact_next, Lc, c),
                                                  compute_uv=False)[chi:] ** 2))
                       for c in range(1, Lc))
            assert float(np.sum((got - exact_next) ** 2)) >= best * (1 - 1e-9)
    assert truncated >= 2


@pytest.mark.parametrize("L,chi", [(8, 4), (11, 6)])
def test_zipup_gauge_covariance_truncated(L, chi):
    p = 0.109
    beta = instance.nishimori_beta(p)
    Jh, Jv = instance.couplings(11, L, p)
    e = synth.random_pm1(12, (L, L))
    Jh2 = (e[:, :-1] * Jh * e[:, 1:]).astype(np.int8)
    Jv2 = (e[:-1, :] * Jv * e[1:, :]).astype(np.int8)
    a = envbuild.build_env(Jh, Jv, beta, chi, method="zipup")
    b = envbuild.build_env(Jh2, Jv2, beta, chi, method="zipup")
    np.testing.assert_allclose(a["lognorm"], b["lognorm"], rtol=1e-12)
    assert abs(a["lnZ"] - b["lnZ"]) < 1e-11 * abs(a["lnZ"])
    assert abs(a["lnZ"] - exact.transfer_matrix(Jh, Jv, beta)["lnZ"]) > 1e-8
