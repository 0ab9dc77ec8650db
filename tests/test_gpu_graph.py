"""The whole step (couplings -> environments -> proposals -> accept) of a mixed-L batch captured
into one HIP graph and replayed.

Every replay must reproduce the eager step bit for bit (couplings, log-norms, environments,
spins, log q, energies, accept decisions, chain state, observable sums), with eager work that
overwrites every buffer and host synchronisations between the replays.  The eager step itself is
checked against the oracle in test_gpu_parity.py; here one realization is re-checked against the
oracle from the replayed buffers.
"""
import numpy as np
import pytest

import synth
from oracle import energy as o_energy
from oracle import envbuild as o_env
from oracle import instance as o_inst

pytestmark = pytest.mark.gpu


def _step(b, seeds, p, K, seed, out, chains, accum):
    b.make_couplings(seeds, p)
    b.build_env(want_lnZ=False)
    b.propose(K, seed, first_proposal=0, out=out)
    for t in (chains["spins"], chains["E"], chains["logq"], chains["init"], accum):
        t.zero_()                         # fill kernels (no memset nodes in the graph)
    acc, cur = b.accept(out, chains, seed=seed, accum=accum)
    return acc, cur


def _snapshot(b, out, chains, accum, acc, cur):
    import torch
    torch.cuda.synchronize()
    snap = [t.detach().clone() for t in (*out, acc, cur, accum, chains["spins"], chains["E"],
                                          chains["logq"], chains["init"])]
    snap += [t.detach().clone() for t in b.lognorm]
    snap += [t.detach().clone() for t in b.Jh + b.Jv]
    snap += [b.env[i].detach().clone() for i in range(0, b.n, max(1, b.n // 4))]
    return snap


def _same(a, b):
    import torch
    return len(a) == len(b) and all(torch.equal(x, y) for x, y in zip(a, b))


def _run(tnmc_gpu, Ls, seeds, chi, p, K, replays):
    import torch
    from paper_2409_06538_amd import binding
    beta = binding.nishimori_beta(p)
    b = binding.Batch(Ls, [beta] * len(Ls), seeds, chi, "fp32", K=K)
    out = (torch.empty(b.spins_shape(K), dtype=torch.int64, device=b.device),
           torch.empty((b.n, K), dtype=torch.float64, device=b.device),
           torch.empty((b.n, K), dtype=torch.int32, device=b.device))
    chains = b.new_chains(1)
    accum = torch.zeros((b.n, binding.OBS_COUNT), dtype=torch.float64, device=b.device)
    other = [s + 1000 for s in seeds]

    acc, cur = _step(b, seeds, p, K, 7, out, chains, accum)          # eager reference
    ref = _snapshot(b, out, chains, accum, acc, cur)

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gacc, gcur = _step(b, seeds, p, K, 7, out, chains, accum)
    for rep in range(replays):
        # eager work in between that overwrites every buffer the graph writes
        _step(b, other, p, K, 11 + rep, out, chains, accum)
        torch.cuda.synchronize()
        assert not _same(_snapshot(b, out, chains, accum, acc, cur), ref)
        g.replay()
        torch.cuda.synchronize()
        got = _snapshot(b, out, chains, accum, gacc, gcur)
        assert _same(got, ref), f"replay {rep} differs from the eager step"
    return b, out, gacc


def test_graph_mixed_small_replays(tnmc_gpu):
    Ls = [8, 16, 24, 32] * 4
    seeds = list(range(40, 40 + len(Ls)))
    p, K = 0.109, 64
    b, out, acc = _run(tnmc_gpu, Ls, seeds, 32, p, K, replays=3)
    # one realization from the replayed buffers against the oracle
    i, L = 1, Ls[1]
    beta = o_inst.nishimori_beta(p)
    Jh, Jv = o_inst.couplings(seeds[i], L, p)
    env = o_env.build_env(Jh, Jv, beta, 32)
    lam = b.lognorm[i].cpu().numpy()
    assert np.max(np.abs(lam - env["lognorm"]) / np.maximum(1.0, np.abs(env["lognorm"]))) < 1e-5
    words = out[0].cpu().numpy()[i].view(np.uint64)[:, :L, :]
    spins = synth.unpack_rows(words, L)
    E_ref = o_energy.energy(spins[:16], Jh, Jv)
    assert np.array_equal(out[2].cpu().numpy()[i][:16], E_ref)


def test_graph_mixed_full_size(tnmc_gpu):
    """256 realizations, L = (32, 64, 128, 256)[i % 4], seed i, chi = 32, FP32: one graph for the
    whole step, replayed twice."""
    w = synth.WORKLOADS["mixed"]
    seeds = list(w["seeds"])
    Ls = [w["Ls"][i % 4] for i in range(len(seeds))]
    _run(tnmc_gpu, Ls, seeds, w["chi"], w["p"], 16, replays=2)
