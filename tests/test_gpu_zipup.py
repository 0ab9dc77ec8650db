"""The zip-up form of the environment build (tnmc_build_env_form with TNMC_FORM_ZIPUP: one sweep
of SVD truncations per row, alternating direction, the contraction variant of Sec. II B) against
the oracle's zip-up mode (oracle.envbuild.compress_zipup, pinned in test_oracle_zipup.py): every
lambda_r and ln Z, the teacher-forced log q of the GPU's proposals through the oracle's zip-up
environments, exact energies.  Exact regime: the zip-up reaches the transfer-matrix ln Z.
Bars as for the other builds: FP32 environments (FP64 arithmetic) 1e-5 / 1e-4, BF16 (FP32
arithmetic) 5e-3, applied where the truncation is well conditioned (oracle.envbuild.sensitivity
below the bar: at a cut whose kept and dropped singular values nearly tie, rounding of either
side picks a different subspace)."""
import numpy as np
import pytest

import synth
from oracle import energy as o_energy
from oracle import envbuild as o_env
from oracle import exact as o_exact
from oracle import instance as o_inst
from oracle import sampler as o_samp

pytestmark = pytest.mark.gpu

TOL = {"fp32": (1e-5, 1e-4), "bf16": (5e-3, 5e-3)}
EPS = {"fp32": 1e-7, "bf16": 4e-3}


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)) / np.maximum(np.abs(np.asarray(b)), 1e-300)


def zip_batch(L, seeds, p, beta, chi, precision, K):
    from paper_2409_06538_amd import binding
    b = binding.Batch([L] * len(seeds), [beta] * len(seeds), seeds, chi, precision, K=K)
    b.make_couplings(seeds, p)
    lnZ = host(b.build_env_form(binding.FORM_ZIPUP))
    st, words = b.status_check()
    assert st == 0, words
    return b, lnZ


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("chi", [8, 16, 64])
@pytest.mark.parametrize("p,beta", [(0.109, None), (0.5, 1.0)])
def test_zipup_against_oracle(tnmc_gpu, precision, chi, p, beta):
    L, seeds, K = 20, [4, 5], 24
    beta = o_inst.nishimori_beta(p) if beta is None else beta
    b, lnZ = zip_batch(L, seeds, p, beta, chi, precision, K)
    spins, logq, E = b.propose(K, 11)
    np.testing.assert_array_equal(host(b.logq(spins)), host(logq))
    tol_env, tol_q = TOL[precision]
    for i, sd in enumerate(seeds):
        Jh, Jv = o_inst.couplings(sd, L, p)
        env = o_env.build_env(Jh, Jv, beta, chi, method="zipup")
        sens = o_env.sensitivity(env, EPS[precision])
        truncated = sum(1 for cc in env["cuts"] for v in cc.values() if v[0] > 1e-5)
        r_lam = np.max(rel(host(b.lognorm[i]), env["lognorm"]))
        print(f"zip-up chi={chi} p={p} seed={sd} {precision}: lnZ rel "
              f"{rel(lnZ[i], env['lnZ']):.2e}, lambda max rel {r_lam:.2e}, truncated cuts "
              f"{truncated}, sensitivity {sens:.1e}", flush=True)
        if chi == 8:
            assert truncated > 0
        sp = synth.unpack_rows(host(spins)[i].view(np.uint64)[:, :L, :], L)
        np.testing.assert_array_equal(host(E)[i], o_energy.energy(sp, Jh, Jv))
        if sens < tol_env:
            assert rel(lnZ[i], env["lnZ"]) < tol_env
            assert r_lam < tol_env
            ref = o_samp.run(env, Jh, Jv, beta, teacher=sp)
            r = rel(host(logq)[i], ref["logq"])
            r_q = np.max(r)
            print(f"  teacher-forced log q: max rel {r_q:.2e}, median {np.median(r):.2e}",
                  flush=True)
            if precision == "bf16":   # typical proposals at the bar, the tail ten times wider
                assert np.median(r) < tol_q and r_q < 10 * tol_q
            else:
                assert r_q < tol_q


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_zipup_exact_regime(tnmc_gpu, precision):
    """chi = 16 >= 2^(L/2) at L = 8: nothing is truncated and ln Z is the transfer matrix's."""
    L, seeds, p = 8, [1, 2], 0.109
    beta = o_inst.nishimori_beta(p)
    _, lnZ = zip_batch(L, seeds, p, beta, 16, precision, 4)
    for i, sd in enumerate(seeds):
        Jh, Jv = o_inst.couplings(sd, L, p)
        tm = o_exact.transfer_matrix(Jh, Jv, beta)
        print(f"L=8 seed={sd} {precision}: zip-up lnZ rel {rel(lnZ[i], tm['lnZ']):.2e}", flush=True)
        assert rel(lnZ[i], tm["lnZ"]) < TOL[precision][0]


def test_zipup_canonical_agree_untruncated(tnmc_gpu):
    """Where no cut is truncated the two compressions are the same state: L = 24 at chi = 64
    (bonds of the Nishimori line stay below 64 here), FP32: lambda_r of both forms agree."""
    from paper_2409_06538_amd import binding
    L, seeds, p = 24, [6, 7], 0.109
    beta = o_inst.nishimori_beta(p)
    bz, lz = zip_batch(L, seeds, p, beta, 64, "fp32", 4)
    bc = binding.Batch([L, L], [beta, beta], seeds, 64, "fp32", K=4)
    bc.make_couplings(seeds, p)
    lc = host(bc.build_env_form(binding.FORM_GRAM_L2))
    for i in range(2):
        r = np.max(rel(host(bz.lognorm[i]), host(bc.lognorm[i])))
        print(f"seed={seeds[i]}: zip-up vs canonical lambda max rel {r:.2e}, lnZ rel "
              f"{rel(lz[i], lc[i]):.2e}", flush=True)
        assert r < 1e-5 and rel(lz[i], lc[i]) < 1e-5
