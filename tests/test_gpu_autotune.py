"""The proposal kernel's launch-shape autotuner (tnmc_autotune_propose, tnmc_tune_set/get).

Every candidate shape (wavefronts per workgroup) must give bit-identical proposals, log q and
energies, sampled and teacher-forced: a proposal's arithmetic does not depend on how many
proposals share its workgroup.  The tuner must store one of the candidates for the batch shape.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("Ls,chi,precision,K", [([64] * 8, 32, "fp32", 100),
                                                ([24, 17, 24], 48, "bf16", 40),
                                                ([20, 20], 16, "fp64", 33),
                                                ([12, 9], 8, "fp32", 70)])
def test_every_shape_bit_identical_and_tuned(tnmc_gpu, Ls, chi, precision, K):
    import torch
    from paper_2409_06538_amd import binding
    p = 0.109
    seeds = list(range(3, 3 + len(Ls)))
    b = binding.Batch(Ls, [binding.nishimori_beta(p)] * len(Ls), seeds, chi, precision, K=K)
    b.make_couplings(seeds, p)
    b.build_env()
    cands = b.propose_candidates()
    assert cands == ([1, 2, 4, 8] if chi % 16 == 0 else [1])
    ref = None
    try:
        for w in cands:
            b.tune_set(K, w)
            assert b.tune_get(K) == w
            spins, logq, E = b.propose(K, 5, first_proposal=7)
            lq2 = b.logq(spins)
            got = [x.cpu().numpy() for x in (spins, logq, E, lq2)]
            if ref is None:
                ref = got
            for a, r in zip(got, ref):
                np.testing.assert_array_equal(a, r)
        best, ms = b.autotune_propose(K, seed=5, reps=1)
        assert best in cands and set(ms) == set(cands) and all(v > 0 for v in ms.values())
        assert b.tune_get(K) == best
        spins, logq, E = b.propose(K, 5, first_proposal=7)
        np.testing.assert_array_equal(spins.cpu().numpy(), ref[0])
        np.testing.assert_array_equal(logq.cpu().numpy(), ref[1])
    finally:
        b.tune_set(K, 0)
    torch.cuda.synchronize()
