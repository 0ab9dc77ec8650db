"""Numeric status words through the C ABI (tnmc_status_check, TNMC_ST_* bits).

The faults are injected as values only (a NaN written into an environment that the build filled,
a zeroed environment, a NaN log q handed to the accept kernel): every kernel still reads and writes
inside its buffers and exits normally.  Readings checked here: a non-finite conditional weight
is a fault (TNMC_ENUMERIC), while two vanishing weights are the p+ = 1/2 fallback of the
reading for truncation artefacts, counted but not a fault.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

P = 0.109


def make(Ls, seeds, chi, precision, K):
    from paper_2409_06538_amd import binding
    beta = binding.nishimori_beta(P)
    b = binding.Batch(Ls, [beta] * len(Ls), seeds, chi, precision, K=K)
    b.make_couplings(seeds, P)
    return b


@pytest.mark.parametrize("chi,precision", [(8, "fp32"), (32, "fp32"), (16, "bf16"), (16, "fp64")])
def test_clean_run_has_no_status_bits(tnmc_gpu, chi, precision):
    import torch
    from paper_2409_06538_amd import binding
    b = make([16, 12], [1, 2], chi, precision, K=32)
    b.build_env()
    prop = b.propose(32, 3)
    chains = b.new_chains(1)
    b.accept(prop, chains, seed=4)
    st, words = b.status_check()
    assert st == 0
    assert all(w & binding.ST_FAULTS == 0 for w in words), words
    torch.cuda.synchronize()


@pytest.mark.parametrize("chi,precision", [(8, "fp32"), (32, "fp32"), (16, "bf16")])
def test_nan_environment_is_enumeric(tnmc_gpu, chi, precision):
    """A NaN written into one stored site of realization 1 makes its conditional weights NaN:
    TNMC_ST_WEIGHT in its word, TNMC_ENUMERIC from tnmc_status_check, realization 0 untouched;
    the fallback p+ = 1/2 keeps every log q finite."""
    import torch
    from paper_2409_06538_amd import binding
    K = 32
    b = make([16, 16], [5, 6], chi, precision, K=K)
    b.build_env()
    torch.cuda.synchronize()
    assert b.status_check() == (0, [0, 0])
    env = b.env_tensor(1)                       # (L, L, 2, chi, chi)
    env[3, 5, 0, 0, 0] = float("nan")           # site (row 3, column 5), a nonzero entry
    fb = torch.zeros(2, dtype=torch.int32, device=b.device)
    spins, logq, E = b.propose(K, 7, fallbacks=fb)
    st, words = b.status_check()
    assert st == binding.ENUMERIC
    assert words[1] & binding.ST_WEIGHT and words[1] & binding.ST_FALLBACK, words
    assert words[0] == 0, words
    assert np.all(np.isfinite(logq.cpu().numpy()))
    assert fb[1].item() > 0 and fb[0].item() == 0
    # the teacher-forced log q sees the same fault
    b.clear_status()
    b.logq(spins)
    st, words = b.status_check()
    assert st == binding.ENUMERIC and words[1] & binding.ST_WEIGHT and words[0] == 0


@pytest.mark.parametrize("chi,precision", [(8, "fp32"), (32, "fp32"), (32, "bf16")])
def test_zeroed_environment_falls_back_to_one_half(tnmc_gpu, chi, precision):
    """All conditional weights vanish: p+ = 1/2 at every site, so log q = -N ln 2 exactly and every
    site counts one fallback; TNMC_ST_FALLBACK is set, which is not a fault."""
    import torch
    from paper_2409_06538_amd import binding
    L, K = 12, 24
    b = make([L], [3], chi, precision, K=K)
    b.build_env()
    b.env[0].zero_()
    fb = torch.zeros(1, dtype=torch.int32, device=b.device)
    spins, logq, E = b.propose(K, 2, fallbacks=fb)
    st, words = b.status_check()
    assert st == 0 and words[0] == binding.ST_FALLBACK, words
    assert fb.item() == K * L * L
    lq = logq.cpu().numpy()[0]
    np.testing.assert_allclose(lq, -L * L * math.log(2.0), rtol=1e-14)


def test_nan_logq_in_accept_sets_delta(tnmc_gpu):
    import torch
    from paper_2409_06538_amd import binding
    K = 16
    b = make([8, 8], [1, 2], 4, "fp64", K=K)
    b.build_env()
    spins, logq, E = b.propose(K, 1)
    logq[1, 5] = float("nan")
    chains = b.new_chains(1)
    acc, cur = b.accept((spins, logq, E), chains, seed=3)
    st, words = b.status_check()
    assert st == binding.ENUMERIC and words == [0, binding.ST_DELTA], words
    assert acc[1, 5].item() == 0                  # a NaN exponent is never accepted
    torch.cuda.synchronize()
