"""One build launch over the realizations of several batches (binding.build_env_group, the
benchmark's grouped steps): every realization's environments, log-norms and bond table equal,
bit for bit, those of building each batch on its own (one workgroup per realization, so the
grouping changes no arithmetic)."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("chi,precision", [(64, "bf16"), (32, "fp32")])
def test_group_build_equals_separate_builds(tnmc_gpu, chi, precision):
    import torch
    from paper_2409_06538_amd import binding
    p = 0.109
    beta = binding.nishimori_beta(p)
    specs = [([24, 24], [3, 4]), ([24, 24], [5, 6]), ([20, 20], [7, 8])]
    batches = []
    for Ls, seeds in specs:
        b = binding.Batch(Ls, [beta] * len(Ls), seeds, chi, precision, K=4)
        b.make_couplings(seeds, p)
        batches.append(b)
    ref = []
    for b in batches:
        b.build_env(want_lnZ=False)
        torch.cuda.synchronize()
        ref.append([(b.env[i].clone(), b.lognorm[i].clone(), b.bonds[i].clone())
                    for i in range(b.n)])
        for i in range(b.n):
            b.env[i].zero_()
            b.lognorm[i].zero_()
            b.bonds[i].zero_()
    ws = torch.empty(binding.group_workspace_bytes(batches), dtype=torch.uint8,
                     device=batches[0].device)
    binding.build_env_group(batches, ws)
    torch.cuda.synchronize()
    for b, rb in zip(batches, ref):
        st, words = b.status_check()
        assert st == 0, words
        for i in range(b.n):
            env, lam, bd = rb[i]
            assert torch.equal(b.env[i], env)
            assert torch.equal(b.lognorm[i], lam)
            assert torch.equal(b.bonds[i], bd)


def test_group_build_rejects_mixed_chi(tnmc_gpu):
    from paper_2409_06538_amd import binding
    beta = binding.nishimori_beta(0.109)
    b1 = binding.Batch([16], [beta], [0], 32, "fp32", K=4)
    b2 = binding.Batch([16], [beta], [1], 16, "fp32", K=4)
    with pytest.raises(binding.TNMCError):
        binding.build_env_group([b1, b2], b1.workspace)
