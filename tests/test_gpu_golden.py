"""Full-size parity against stored oracle values (tests/golden/oracle_*.json, written by
tests/golden/make_oracle_goldens.py, which calls only the oracle; the oracle needs minutes per
realization at these sizes).

Each case builds the whole batch of its workload in one launch, as the benchmark does, and
compares for the stored realization: every environment log-norm lambda_r and ln Z_TN (Sec. II B),
and the GPU's teacher-forced log q of the oracle's own proposals (Eqs. (4)-(6)), whose exact
energies must also match bit for bit (Eq. (10)).  Bars: BF16 environments 5e-3 relative, FP32
1e-5 (log-norms) and 1e-4 (log q); absolute errors are printed beside them.
"""
import json
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    with open(os.path.join(GOLDEN, f"oracle_{name}.json")) as f:
        g = json.load(f)
    if "proposals" in g:
        pr = g["proposals"]
        g["spins_words"] = np.array([[[int(w, 16) for w in row.split()] for row in conf]
                                     for conf in pr["spins_hex"]], dtype=np.uint64)
    return g


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


def check_case(b, i, g, tol_env, tol_q, lnZ):
    """Realization i of batch b against golden g: all log-norms, ln Z, teacher-forced log q."""
    import torch
    L = g["L"]
    lam = host(b.lognorm[i])
    ref = np.array([np.nan if x is None else x for x in g["lognorm"]])
    built = ~np.isnan(ref)
    r_env = rel(lam[built], ref[built])
    print(f"L={L} chi={g['chi']} p={g['p']} seed={g['coupling_seed']} {b.precision}: "
          f"lambda max rel {r_env.max():.2e} (abs {np.abs(lam[built] - ref[built]).max():.3e}) "
          f"over {built.sum()} rows", flush=True)
    assert r_env.max() < tol_env
    if "lnZ" in g:
        print(f"  lnZ rel {rel(lnZ[i], g['lnZ']):.2e} (abs {abs(lnZ[i] - g['lnZ']):.3e})")
        assert rel(lnZ[i], g["lnZ"]) < tol_env
    if "proposals" in g:
        pr = g["proposals"]
        K = len(pr["logq"])
        W = synth.words_per_row(b.Lmax)
        words = np.zeros((b.n, K, b.Lmax, W), dtype=np.uint64)
        words[i, :, :L, :g["spins_words"].shape[2]] = g["spins_words"]
        d = torch.from_numpy(words.view(np.int64)).to(b.device)
        lq = host(b.logq(d))[i]
        r_q = rel(lq, pr["logq"])
        print(f"  teacher-forced log q max rel {r_q.max():.2e} "
              f"(abs {np.abs(lq - np.array(pr['logq'])).max():.3e}, log q ~ {pr['logq'][0]:.1f})",
              flush=True)
        assert r_q.max() < tol_q
        E = host(b.energy(d))[i]
        np.testing.assert_array_equal(E, pr["E"])


def full_batch(Ls, seeds, chi, precision, p):
    from paper_2409_06538_amd import binding
    beta = binding.nishimori_beta(p)
    b = binding.Batch(Ls, [beta] * len(Ls), seeds, chi, precision, K=4)
    b.make_couplings(seeds, p)
    lnZ = host(b.build_env())
    st, words = b.status_check()
    assert st == 0, words
    return b, lnZ


@pytest.mark.parametrize("name", ["rbim256_p0.10_s0", "rbim256_p0.109_s77", "rbim256_p0.12_s11"])
def test_rbim256_chi48_bf16_batch_against_oracle(tnmc_gpu, name):
    """L = 256, chi = 48, BF16 environments: the 128-realization batch of one disorder strength."""
    g = load(name)
    w = synth.WORKLOADS["rbim256"]
    seeds = list(w["seeds"])
    b, lnZ = full_batch([g["L"]] * len(seeds), seeds, g["chi"], "bf16", g["p"])
    check_case(b, seeds.index(g["coupling_seed"]), g, 5e-3, 5e-3, lnZ)


def test_rbim256_chi48_fp32_against_oracle(tnmc_gpu):
    g = load("rbim256_p0.109_s77")
    seeds = list(range(64, 96))
    b, lnZ = full_batch([g["L"]] * len(seeds), seeds, g["chi"], "fp32", g["p"])
    check_case(b, seeds.index(g["coupling_seed"]), g, 1e-5, 1e-4, lnZ)


def test_mixed_batch_against_oracle(tnmc_gpu):
    """The 256-realization mixed-L batch (L = 32, 64, 128, 256; chi = 32; FP32) in one launch:
    realizations 14 (L = 128) and 19 (L = 256) against the oracle."""
    w = synth.WORKLOADS["mixed"]
    seeds = list(w["seeds"])
    Ls = [w["Ls"][i % 4] for i in range(len(seeds))]
    b, lnZ = full_batch(Ls, seeds, w["chi"], "fp32", w["p"])
    for name in ("mixed_L128_s14", "mixed_L256_s19"):
        g = load(name)
        i = g["coupling_seed"]
        assert Ls[i] == g["L"]
        check_case(b, i, g, 1e-5, 1e-4, lnZ)


@pytest.mark.parametrize("precision,tol", [
    pytest.param("fp32", 1e-5, marks=pytest.mark.skip(
        reason="the FP32 chi = 64 build of an L = 1024 lattice (FP64 Gram matrices) takes about "
               "four minutes; FP32 chi = 64 parity is checked at L <= 256 in test_gpu_chi64.py")),
    ("bf16", 5e-3)])
def test_rbim1024_chi64_first_rows_against_oracle(tnmc_gpu, precision, tol):
    """L = 1024, chi = 64, both realizations of the workload (BF16 environments, the benchmark's
    launch): the first rows built (from the bottom) against the oracle's slice, with the bond
    table bounding every stored site."""
    from oracle import energy as o_energy
    from oracle import instance as o_inst
    L = 1024
    b, lnZ = full_batch([L, L], [0, 1], 64, precision, 0.109)
    for i in (0, 1):
        check_case(b, i, load(f"rbim1024_s{i}_rows8"), tol, tol, lnZ)
        # the bond table bounds the stored sites of the rows compared
        bt = b.bond_table(i).cpu().numpy().astype(int)
        al = np.arange(64)
        for r in range(L - 9, L):
            e = b.env_tensor(i)[r].float().cpu().numpy()          # (L, 2, 64, 64)
            for c in range(L):
                outside = (al[:, None] >= bt[r, c]) | (al[None, :] >= bt[r, c + 1])
                assert not np.any(e[c][:, outside]), (r, c)
    # proposals in the benchmark's launch: exact energies and self-consistent log q
    spins, logq, E = b.propose(4, 0)
    np.testing.assert_array_equal(host(b.logq(spins)), host(logq))
    for i in (0, 1):
        Jh, Jv = o_inst.couplings(i, L, 0.109)
        sp = synth.unpack_rows(host(spins)[i].view(np.uint64), L)
        np.testing.assert_array_equal(host(E)[i], o_energy.energy(sp, Jh, Jv))
