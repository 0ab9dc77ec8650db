"""tnmc_build_env_static: the allocation-free build (descriptor table and build scratch in the
library's fixed device array) against tnmc_build_env with a caller workspace, bit for bit, on
two calls in a row (the second with a smaller batch, so that it reuses the array that the first
call left filled)."""
import ctypes

import numpy as np
import pytest


def test_static_build_rejects_batches_beyond_the_array():
    """Host check before any HIP call: a batch whose scratch exceeds the array is refused."""
    from paper_2409_06538_amd import binding
    lib = binding.load()
    tab = (binding.Instance * 1)()
    tab[0].L, tab[0].beta = 1024, 1.0
    tab[0].d_Jh = tab[0].d_Jv = tab[0].d_env = tab[0].d_lognorm = 1 << 20
    # 1024 x (2 chi)^2 FP64 carried factors at chi = 48: 75.5 MB > 64 MiB
    assert lib.tnmc_build_env_static(tab, 1, 48, binding.FP32, None, None) == -2
    tab[0].L = 1
    assert lib.tnmc_build_env_static(tab, 1, 48, binding.FP32, None, None) == -1


def _both(Ls, seeds, chi, precision, p=0.109):
    import torch
    from paper_2409_06538_amd import binding
    beta = binding.nishimori_beta(p)
    b = binding.Batch(Ls, [beta] * len(Ls), seeds, chi, precision)
    b.make_couplings(seeds, p)
    lnZ_ws = b.build_env().cpu().numpy()
    lam_ws = [x.cpu().numpy().copy() for x in b.lognorm]
    env_ws = [x.view(torch.uint8).cpu().numpy().copy() for x in b.env]
    for x in b.env + b.lognorm:
        x.zero_()
    lnZ_st = b.build_env_static().cpu().numpy()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(lnZ_st, lnZ_ws)
    for i in range(len(Ls)):
        np.testing.assert_array_equal(b.lognorm[i].cpu().numpy(), lam_ws[i])
        got = b.env[i].view(torch.uint8).cpu().numpy()
        assert np.array_equal(got, env_ws[i]), i
    st, words = b.status_check()
    assert st == 0, words
    return lnZ_st


@pytest.mark.gpu
@pytest.mark.parametrize("chi,precision", [(16, "fp64"), (32, "fp32"), (48, "bf16")])
def test_static_build_matches_workspace_build(tnmc_gpu, chi, precision):
    big = _both([20, 33, 17], [4, 5, 6], chi, precision)
    small = _both([9], [7], chi, precision)
    assert np.all(np.isfinite(big)) and np.all(np.isfinite(small))
