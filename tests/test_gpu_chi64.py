"""Bond dimension 64 (the Gram-form build with global scratch and the chi = 64 proposal tiles):
parity with the FP64 oracle on lattices where the bonds reach 64, including cuts whose numerical
rank exceeds 64 (the Jacobi path), for FP32 and BF16 environments."""
import numpy as np
import pytest

import synth
from oracle import energy as o_energy
from oracle import envbuild as o_env
from oracle import instance as o_inst
from oracle import sampler as o_samp

pytestmark = pytest.mark.gpu

TOL = {"fp32": (1e-5, 1e-4), "bf16": (5e-3, 5e-3)}


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)) / np.maximum(np.abs(np.asarray(b)), 1e-300)


def run_case(L, seed, p, beta, precision, K):
    from paper_2409_06538_amd import binding
    chi = 64
    b = binding.Batch([L, L], [beta, beta], [seed, seed + 1], chi, precision, K=K)
    b.make_couplings([seed, seed + 1], p)
    lnZ = host(b.build_env())
    st, words = b.status_check()
    assert st == 0, words
    spins, logq, E = b.propose(K, 9)
    tol_env, tol_q = TOL[precision]
    for i, sd in enumerate((seed, seed + 1)):
        Jh, Jv = o_inst.couplings(sd, L, p)
        env = o_env.build_env(Jh, Jv, beta, chi)
        r_lam = np.max(rel(host(b.lognorm[i]), env["lognorm"]))
        print(f"L={L} p={p} seed={sd} {precision}: lnZ rel {rel(lnZ[i], env['lnZ']):.2e}, "
              f"lambda max rel {r_lam:.2e}", flush=True)
        assert rel(lnZ[i], env["lnZ"]) < tol_env
        assert r_lam < tol_env
        words = host(spins)[i].view(np.uint64)
        sp = synth.unpack_rows(words[:, :L, :], L)
        np.testing.assert_array_equal(host(E)[i], o_energy.energy(sp, Jh, Jv))
        ref = o_samp.run(env, Jh, Jv, beta, teacher=sp)
        r = rel(host(logq)[i], ref["logq"])
        r_q = np.max(r)
        print(f"  teacher-forced log q of GPU proposals: max rel {r_q:.2e}, median "
              f"{np.median(r):.2e}", flush=True)
        if precision == "bf16":
            # GPU proposals follow the BF16 q: one that passes a site whose FP64 conditional is
            # much smaller than its BF16-rounded one carries that site's whole log ratio, so the
            # bar holds for typical proposals and the tail is bounded ten times wider
            assert np.median(r) < tol_q and r_q < 10 * tol_q
        else:
            assert r_q < tol_q
    np.testing.assert_array_equal(host(b.logq(spins)), host(logq))
    e = b.env_tensor(0).float().cpu().numpy()
    return (np.abs(e) > 0).any(axis=(2, 4)).sum(axis=-1)     # left bond of every site


@pytest.mark.parametrize("precision,L", [("fp32", 14), ("bf16", 48)])
def test_chi64_nishimori(tnmc_gpu, precision, L):
    """The Nishimori line at chi = 64 (no cut of these lattices needs more than 64: the
    truncation is the numerical-rank cut).  BF16 on L = 48: on smaller lattices a few sites
    whose small conditional weight the 8-bit mantissas change dominate the relative log q
    error (L = 14: 1e-2)."""
    p = 0.109
    run_case(L, 3, p, o_inst.nishimori_beta(p), precision, K=48)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_chi64_spin_glass(tnmc_gpu, precision):
    run_case(18, 5, 0.5, 1.0, precision, K=32)


@pytest.mark.parametrize("chi", [8, 16, 32])
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("p,beta", [(0.109, None), (0.5, 1.0)])
def test_gram_l2_form_truncated(tnmc_gpu, chi, precision, p, beta):
    """The same build form at chi = 8, 16, 32 where the truncation to chi is real (cuts of
    numerical rank above chi: the one-sided Jacobi step and the choice of the chi largest
    singular directions run): all log-norms and ln Z against the oracle, L = 20."""
    from paper_2409_06538_amd import binding
    L, seeds = 20, [7, 8]
    beta = o_inst.nishimori_beta(p) if beta is None else beta
    b = binding.Batch([L, L], [beta, beta], seeds, chi, precision, K=16)
    b.make_couplings(seeds, p)
    lnZ = host(b.build_env_form(binding.FORM_GRAM_L2))
    st, words = b.status_check()
    assert st == 0, words
    tol_env, tol_q = TOL[precision]
    for i, sd in enumerate(seeds):
        Jh, Jv = o_inst.couplings(sd, L, p)
        env = o_env.build_env(Jh, Jv, beta, chi)
        truncated = sum(1 for cc in env["cuts"] for v in cc.values() if v[0] > 1e-5)
        r_lam = np.max(rel(host(b.lognorm[i]), env["lognorm"]))
        print(f"chi={chi} p={p} seed={sd} {precision}: lnZ rel {rel(lnZ[i], env['lnZ']):.2e}, "
              f"lambda max rel {r_lam:.2e}, truncated cuts {truncated}, "
              f"sensitivity {o_env.sensitivity(env, 1e-7):.1e}", flush=True)
        if chi == 8:
            assert truncated > 0
        if o_env.sensitivity(env, 1e-7 if precision == "fp32" else 4e-3) < 0.1 * tol_env:
            assert rel(lnZ[i], env["lnZ"]) < tol_env
            assert r_lam < tol_env
    spins, logq, E = b.propose(16, 3)
    np.testing.assert_array_equal(host(b.logq(spins)), host(logq))
