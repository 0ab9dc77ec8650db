"""The bond table (tnmc_instance.d_bonds): written by the build, it bounds the nonzero block of
every stored site; proposals that load only the nonzero block of the narrow sites through it are
bit-identical to proposals that load whole sites."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L,chi,precision,form", [(40, 32, "fp32", 0), (40, 48, "bf16", 0),
                                                  (24, 16, "fp64", 0), (40, 64, "bf16", 0),
                                                  (30, 64, "fp32", 0), (40, 48, "bf16", 1)])
def test_bond_table_bounds_sites_and_proposals_identical(tnmc_gpu, L, chi, precision, form):
    import torch
    from paper_2409_06538_amd import binding
    p, seeds, K = 0.109, [3, 4], 48
    b = binding.Batch([L, L], [binding.nishimori_beta(p)] * 2, seeds, chi, precision, K=K)
    b.make_couplings(seeds, p)
    b.build_env_form(form)
    for i in range(2):
        bt = b.bond_table(i).cpu().numpy().astype(int)
        assert (bt[:, 0] == 1).all() and (bt[:, L] == 1).all() and (bt[L - 1] == 1).all()
        e = b.env_tensor(i).float().cpu().numpy()                 # (L, L, 2, chi, chi)
        al = np.arange(chi)
        for r in range(L):
            for c in range(L):
                outside = (al[:, None] >= bt[r, c]) | (al[None, :] >= bt[r, c + 1])
                assert not np.any(e[r, c][:, outside]), (r, c, bt[r, c], bt[r, c + 1])
        assert bt.max() <= chi
    with_table = [x.cpu().numpy() for x in b.propose(K, 6, first_proposal=3)]
    lq_table = b.logq(b.propose(K, 6, first_proposal=3)[0]).cpu().numpy()
    b.use_bonds(False)
    without = [x.cpu().numpy() for x in b.propose(K, 6, first_proposal=3)]
    lq = b.logq(b.propose(K, 6, first_proposal=3)[0]).cpu().numpy()
    for a, c in zip(with_table, without):
        np.testing.assert_array_equal(a, c)
    np.testing.assert_array_equal(lq_table, lq)
    torch.cuda.synchronize()
