"""Observables of Sec. III C through the C ABI: the disorder-average kernel against the oracle's
definitions, and the Nishimori-line identities through whole GPU chains (statistical).

On the Nishimori line, exp(-2 beta) = p / (1 - p) (Sec. III A), the disorder-averaged energy is
exactly [<E>] = -N_B tanh(beta) = -N_B (1 - 2p), and [<q^2>] = [<m^2>] (gauge symmetry).  The
Metropolis step makes the chains exact whatever the precision of the environments, so every
precision must reproduce both within the disorder-sample error: the "equal observable accuracy"
of the reduced-precision batched forms.
"""
import math

import numpy as np
import pytest

import synth
from oracle import observables as o_obs

pytestmark = pytest.mark.gpu


def test_disorder_average_kernel_matches_oracle(tnmc_gpu):
    import torch
    from paper_2409_06538_amd import binding
    rng = np.random.default_rng(3)
    n, L, beta, n_chain = 37, 24, 0.8, 2
    T = rng.integers(50, 200, size=n).astype(np.float64)
    acc = np.zeros((n, 9))
    acc[:, 0] = n_chain * T
    acc[:, 1] = -rng.uniform(500, 900, n) * acc[:, 0]
    acc[:, 2] = rng.uniform(3e5, 8e5, n) * acc[:, 0]
    acc[:, 3:6] = rng.uniform(0, 1, (n, 3)) * acc[:, :1]
    acc[:, 6] = rng.uniform(-0.2, 0.2, n) * T
    acc[:, 7:9] = rng.uniform(0, 1, (n, 2)) * T[:, None]
    b = binding.Batch([L] * n, [beta] * n, list(range(n)), 4, "fp64")
    got = b.disorder_average(torch.from_numpy(acc).to(b.device), n_chain).cpu().numpy()
    ref = o_obs.disorder_averages(acc, L, beta, n_chain)
    assert tuple(binding.AVG_NAMES) == tuple(o_obs.AVG_NAMES)
    np.testing.assert_allclose(got, ref, rtol=1e-12)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
def test_nishimori_identities_rbim64(tnmc_gpu, precision):
    """The L = 64, chi = 32 batch of 64 realizations (p = 0.109 on the Nishimori line), two chains
    of 128 steps each per realization."""
    import torch
    from paper_2409_06538_amd import binding
    w = synth.WORKLOADS["rbim64"]
    L, chi, p, seeds = w["L"], w["chi"], w["p"], list(w["seeds"])
    K, n_chain = 256, 2
    beta = binding.nishimori_beta(p)
    b = binding.Batch([L] * len(seeds), [beta] * len(seeds), seeds, chi, precision, K=K)
    b.make_couplings(seeds, p)
    b.build_env(want_lnZ=False)
    prop = b.propose(K, 21)
    chains = b.new_chains(n_chain)
    accum = torch.zeros((len(seeds), 9), dtype=torch.float64, device=b.device)
    acc, _ = b.accept(prop, chains, seed=22, accum=accum)
    st, words = b.status_check()
    assert st == 0, words
    avg = dict(zip(binding.AVG_NAMES, b.disorder_average(accum, n_chain).cpu().numpy()))
    a = accum.cpu().numpy()
    nb = 2 * L * (L - 1)
    e_i = a[:, 1] / a[:, 0]
    target = -nb * (1 - 2 * p)
    se = e_i.std(ddof=1) / math.sqrt(len(e_i))
    pa = acc.float().sum().item() / (len(seeds) * (K - n_chain))
    print(f"{precision}: [<E>] = {avg['E']:.2f} +- {se:.2f} (exact {target:.1f}), "
          f"[<q^2>] = {avg['q2']:.5f}, [<m^2>] = {avg['m2']:.5f}, p_a = {pa:.4f}", flush=True)
    assert abs(avg["E"] - e_i.mean()) < 1e-9 * abs(target)
    assert abs(avg["E"] - target) < 4 * se
    d = a[:, 7] / (a[:, 0] / n_chain) - a[:, 3] / a[:, 0]
    assert abs(d.mean()) < 4 * d.std(ddof=1) / math.sqrt(len(d)) + 1e-4
