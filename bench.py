"""Benchmark of the TNMC hot path on one MI355X.

One step = one pass of the whole hot path over one batch: couplings (a1) -> environments (a2,
a3) -> K proposals per realization with log q and exact energies (a4, a5) -> independence
Metropolis over them (a6).  Default workload: 64 realizations of the 64 x 64 open +-J lattice at
p = 0.109 on the Nishimori line, chi = 32, 1000 proposals each, FP32 batched (one launch per
stage for the whole batch).

Consecutive steps overlap: the builds of steps t+1 and t+2 (one workgroup per realization each,
on CUs kept free of proposal work by a CU mask, one stream each) run during the proposals and
accepts of step t (on the other CUs); three sets of environments rotate.  The timed region starts
with an empty pipeline and ends when the last step's accepts are done.  Batches of more than 64
realizations run their two builds in flight without the CU mask.  `--workload rbim256` runs the
L = 256, chi = 48 BF16 workload at its three disorder strengths (one batch per p, consecutive
pipeline stages); `--workload mixed` the mixed-L batch.  `serial` reports the same steps one
after the other on one stream.  Also measured: the FP64 plain form (FP64 environments, one
realization per call, one proposal per call) on a bounded sample, and the CPU FP64 oracle on the
host (bounded sample, extrapolated; labelled).

Prints ONE JSON line.  Usage: python bench.py [--gpus 1] [--steps 50] [--warmup 1] [--serial]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "accepted spin-updates/s + acceptance rate, BF16/FP32 batched vs FP64 plain"
FP32_VECTOR_PEAK_TFLOPS = 157.3
FP64_VECTOR_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


def proposals_per_wg(precision, n, K, Lmax):
    """Proposals per workgroup of the matrix-core proposal kernel (16 per wavefront; the library
    picks 8 wavefronts for L <= 64 and at least 256 workgroups of 128 proposals, else 4)."""
    wide = Lmax <= 64 and n * ((K + 127) // 128) >= 256
    return 128 if wide else 64


# HBM bytes per launch of the dominant kernel from the FETCH_SIZE / WRITE_SIZE counters, each
# scaled by the same counter on a plain 1 GiB copy (profiles/rbim64_fp32_hbm_traffic.md).  Valid
# only for the kernel sources they were taken on: reported as null once those change.
COUNTED_TRAFFIC = {
    ("rbim64", "fp32", "env_build"): {
        "fetch_kib": 5936819.4, "fetch_factor": 1048576.0 / 524308.125,
        "write_kib": 10232238.3, "write_factor": 1.0,
        "sources_sha256": {
            "envbuild.hip": "6fc5dfae0fc8a49b502a914813092c0315ef4f41b71a8f94fa3504fd604a2c99",
            "common.hpp": "2bc982fcaf62715dab9d8874db2780a5211c7c295637a1e3d7cedcf3f832a587",
        },
    },
    ("rbim64", "fp32", "propose"): {
        "fetch_kib": 20744570.6, "fetch_factor": 1048576.0 / 524308.125,
        "write_kib": 36749974.3, "write_factor": 1.0,
        "sources_sha256": {
            "sampler.hip": "fc28505af48c47c184cb1a9bf4848e969c43fb5c6c03192785ad9cf606fb087d",
            "common.hpp": "2bc982fcaf62715dab9d8874db2780a5211c7c295637a1e3d7cedcf3f832a587",
        },
    },
}


def counted_traffic(workload, precision, kernel):
    import hashlib
    rec = COUNTED_TRAFFIC.get((workload, precision, kernel))
    if rec is None:
        return None
    csrc = os.path.join(ROOT, "paper_2409_06538_amd", "csrc")
    for name, digest in rec["sources_sha256"].items():
        with open(os.path.join(csrc, name), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    return 1024.0 * (rec["fetch_kib"] * rec["fetch_factor"] + rec["write_kib"] * rec["write_factor"])


def build_flops_per_site(chi):
    """Algorithmic work of one site of the canonical compression (QR of a 4chi x 2chi matrix
    with Q, SVD of a 2chi x 2chi matrix, the two contractions), ~270 chi^3."""
    return 270.0 * chi ** 3


def workload_sizes(w):
    """Lattice size of every realization of a workload (uniform L, or L cycling through Ls)."""
    seeds = list(w["seeds"])
    if "Ls" in w:
        return [w["Ls"][i % len(w["Ls"])] for i in range(len(seeds))], seeds
    return [w["L"]] * len(seeds), seeds


def add_rooflines(res, args, Ls):
    """Dominant-kernel rooflines from the HIP-event launch times in `res`."""
    chi, K, build_ms, prop_ms = res["chi"], res["K"], res["build_ms"], res["propose_ms"]
    flops = sum(build_flops_per_site(chi) * (L - 1) * L for L in Ls)
    peak = FP64_VECTOR_PEAK_TFLOPS if args.precision == "fp64" else FP32_VECTOR_PEAK_TFLOPS
    achieved = flops / (build_ms * 1e-3) / 1e12
    res["roofline"] = {"kernel": "env_build_kernel", "bound": "alu", "achieved": achieved,
                       "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                       "traffic": counted_traffic(args.workload, args.precision, "env_build"),
                       "launch_ms": build_ms,
                       "algorithmic_flops_per_launch": flops}
    # proposals: HBM-bound; algorithmic bytes = the per-row V store written and read back (2 x
    # 16 rows per proposal at a narrow site, 2 x chi elsewhere), plus each workgroup of
    # proposals_per_wg() proposals streaming its realization's environments once per sweep
    elem = 8 if args.precision == "fp64" else 4
    esize = {"fp64": 8, "fp32": 4, "bf16": 2}[args.precision]
    g = proposals_per_wg(args.precision, len(Ls), K, max(Ls))
    kpad = (K + g - 1) // g * g
    nf = res.get("narrow_fraction", 0.0)
    vrows = min(16, chi) * nf + chi * (1.0 - nf)
    vbytes = sum(2.0 * L * L * 2 * vrows * kpad * elem for L in Ls)
    ebytes = sum(2.0 * L * L * 2 * chi * chi * esize * (kpad // g) for L in Ls)
    pbytes = vbytes + ebytes
    pach = pbytes / (prop_ms * 1e-3) / 1e9
    res["roofline_propose"] = {"kernel": "propose_mfma_kernel" if chi % 16 == 0 else "propose_kernel",
                               "bound": "hbm", "achieved": pach, "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": pach / HBM_PEAK_GBS,
                               "traffic": counted_traffic(args.workload, args.precision, "propose"),
                               "launch_ms": prop_ms, "algorithmic_bytes_per_launch": pbytes,
                               "narrow_site_fraction": nf}
    return res


def narrow_fraction(batch):
    """Fraction of the environment sites whose entries all lie in the leading 16 x 16 block of
    both matrices (the proposal kernel then stores one 16-row tile of V per spin value)."""
    import torch
    tot = wide = 0
    for i, L in enumerate(batch.Ls):
        e = batch.env_tensor(i)
        if batch.chi <= 16:
            tot += L * L
            continue
        w = ((e[..., 16:, :] != 0).flatten(2).any(-1) | (e[..., :, 16:] != 0).flatten(2).any(-1))
        tot += L * L
        wide += int(w.sum().item())
    return 1.0 - wide / max(1, tot)


def disorder_strengths(w):
    """The p values of a workload: one, or several sharing the coupling seeds (common random
    numbers across p)."""
    return list(w["ps"]) if "ps" in w else [w["p"]]


def run_gpu(args, w=None):
    """Steps one after the other on one stream (or replayed from one HIP graph).  A workload with
    several disorder strengths runs every p in each step, one batch after the other, reusing
    the same buffers."""
    import torch
    from paper_2409_06538_amd import binding
    import synth

    w = synth.WORKLOADS[args.workload] if w is None else w
    Ls, seeds = workload_sizes(w)
    ps = disorder_strengths(w)
    chi, K = w["chi"], args.proposals or w["proposals"]
    n = len(seeds)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    b = binding.Batch(Ls, [binding.nishimori_beta(ps[0])] * n, seeds, chi, args.precision, K=K,
                      device=dev)
    out = (torch.empty(b.spins_shape(K), dtype=torch.int64, device=dev),
           torch.empty((n, K), dtype=torch.float64, device=dev),
           torch.empty((n, K), dtype=torch.int32, device=dev))
    accum = torch.zeros((n, binding.OBS_COUNT), dtype=torch.float64, device=dev)
    chains = b.new_chains(1)
    L2 = torch.tensor([L * L for L in Ls], dtype=torch.float64, device=dev)
    ev = []

    def step(events):
        """One pass over every p; returns per-p [accepted, accepted x L^2] (device tensors)."""
        sums = []
        for j, p in enumerate(ps):
            if len(ps) > 1:
                b.set_betas([binding.nishimori_beta(p)] * n)
            b.make_couplings(seeds, p)
            if events is not None:
                events[3 * j].record()
            b.build_env(want_lnZ=False)
            if events is not None:
                events[3 * j + 1].record()
            b.propose(K, args.seed, first_proposal=0, out=out)
            if events is not None:
                events[3 * j + 2].record()
            for t in (chains["spins"], chains["E"], chains["logq"], chains["init"]):
                t.zero_()
            acc, _ = b.accept(out, chains, seed=args.seed, accum=accum)
            per_real = acc.sum(dim=1, dtype=torch.float64)
            sums.append(torch.stack([per_real.sum(), (per_real * L2).sum()]))
        return torch.stack(sums)

    def new_events():
        return [torch.cuda.Event(enable_timing=True) for _ in range(3 * len(ps))]

    for _ in range(max(1, args.warmup) if args.graph else args.warmup):
        e = new_events()
        step(e)
        ev.append(e)          # graph mode: phase times come from the eager warm-up steps
    torch.cuda.synchronize()
    if not args.graph:
        ev = []
    graph = None
    if args.graph:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            gsums = step(None)
        torch.cuda.synchronize()
    accs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        if graph is not None:
            graph.replay()
            accs.append(gsums.clone())
        else:
            e = new_events()
            accs.append(step(e))
            ev.append(e)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per_p = torch.stack(accs).sum(dim=0).tolist()            # [len(ps)][2]
    accepted = int(sum(a for a, _ in per_p))
    updates = sum(u for _, u in per_p)
    attempted = args.steps * len(ps) * n * (K - 1)
    nb = len(ev) * len(ps)
    build_ms = sum(e[3 * j].elapsed_time(e[3 * j + 1]) for e in ev for j in range(len(ps))) / nb
    prop_ms = sum(e[3 * j + 1].elapsed_time(e[3 * j + 2]) for e in ev for j in range(len(ps))) / nb
    wall = t1 - t0
    res = {
        "Ls": sorted(set(Ls)), "chi": chi, "n": n, "K": K, "p": ps[0] if len(ps) == 1 else ps,
        "wall_s": wall, "ms_per_step": 1e3 * wall / args.steps,
        "value": updates / wall,
        "accepted": accepted, "attempted": attempted,
        "acceptance": accepted / attempted,
        "build_ms": build_ms, "propose_ms": prop_ms,
        "graph": bool(args.graph),
        "narrow_fraction": narrow_fraction(b),
    }
    if len(ps) > 1:
        res["acceptance_per_p"] = {str(p): per_p[j][0] / (args.steps * n * (K - 1))
                                   for j, p in enumerate(ps)}
        res["batches_per_step"] = len(ps)
    return add_rooflines(res, args, Ls)


def reserved_cu_bits(word, sets=1):
    """Bit positions cleared in 32-bit word `word` of the CU mask: 8 per set, one per residue mod 8
    and two per byte, rotated by the word index (and by two bytes for the second set).  Whether
    the mask enumerates CUs XCD by XCD (32 per XCD, shader engines by byte or interleaved mod 4)
    or interleaved across the 8 XCDs with shader engines by byte, every XCD then keeps 8 CUs per
    set free, spread evenly over its shader engines."""
    return [8 * ((x // 2 + word + 2 * k) % 4) + x for k in range(sets) for x in range(8)]


def cu_masked_stream(reserve):
    """A stream (default priority) whose kernels avoid 8 `reserve` CUs of every XCD, so that the
    64 workgroups of each of `reserve` concurrent builds always find free CUs.  Returns (stream,
    mask words), or (None, None) when no mask is asked for or the call fails."""
    import ctypes
    import torch
    if not reserve:
        return None, None
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    words = (n_cu + 31) // 32
    vals = []
    for w in range(words):
        v = 0xFFFFFFFF
        for bit in reserved_cu_bits(w, reserve):
            v &= ~(1 << bit)
        vals.append(v)
    mask = (ctypes.c_uint32 * words)(*vals)
    try:
        hip = ctypes.CDLL("libamdhip64.so")
    except OSError:
        return None, None
    stream = ctypes.c_void_p()
    err = hip.hipExtStreamCreateWithCUMask(ctypes.byref(stream), ctypes.c_uint32(words), mask)
    if err != 0 or not stream.value:
        return None, None
    ext = torch.cuda.ExternalStream(stream.value)
    ext.destroy = lambda: hip.hipStreamDestroy(stream)    # the library owns it, not torch
    return ext, [hex(v) for v in vals]


def run_gpu_pipelined(args):
    """Consecutive steps overlapped: the builds of the next `depth` batches (one workgroup per
    realization each, so a fraction of the CUs; one stream per build in flight) run while the
    proposals and accepts of the current batch use the rest of the chip (one stream, CU-masked).
    depth + 1 sets of environments and workspaces rotate, so a build never overwrites
    environments that proposals still read.  A workload with several disorder strengths runs
    its batches (one per p, the same coupling seeds) as consecutive pipeline stages."""
    import torch
    from paper_2409_06538_amd import binding
    import synth

    w = synth.WORKLOADS[args.workload]
    Ls, seeds = workload_sizes(w)
    ps = disorder_strengths(w)
    chi, K = w["chi"], args.proposals or w["proposals"]
    n = len(seeds)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # each build in flight keeps 8 CUs of every XCD (64 CUs) per 64 realizations free of
    # proposal work; at most two such sets are cleared.  Larger batches (whose builds in flight
    # would need more) run unmasked: their builds then fill the chip together and the proposals
    # take the CUs each build frees.
    per_build = (n + 63) // 64
    depth = args.builds_in_flight
    reserve = depth * per_build if args.reserve_cus and depth * per_build <= 2 else 0
    s_builds = [torch.cuda.Stream() for _ in range(depth)]
    s_prop, cu_mask = cu_masked_stream(reserve)
    if s_prop is None:
        s_prop = torch.cuda.Stream()
    sets = []
    for _ in range(depth + 1):
        b = binding.Batch(Ls, [binding.nishimori_beta(ps[0])] * n, seeds, chi, args.precision,
                          K=K, device=dev)
        out = (torch.empty(b.spins_shape(K), dtype=torch.int64, device=dev),
               torch.empty((n, K), dtype=torch.float64, device=dev),
               torch.empty((n, K), dtype=torch.int32, device=dev))
        sets.append({"b": b, "out": out, "chains": b.new_chains(1),
                     "accum": torch.zeros((n, binding.OBS_COUNT), dtype=torch.float64, device=dev),
                     "done": None})
    L2 = torch.tensor([L * L for L in Ls], dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    def run(steps):
        """`steps` passes over every p: one pipeline stage per (step, p)."""
        sums, ev = [], []
        for u in range(steps * len(ps)):
            p = ps[u % len(ps)]
            st = sets[u % (depth + 1)]
            b = st["b"]
            s_build = s_builds[u % depth]
            e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            with torch.cuda.stream(s_build):
                if st["done"] is not None:
                    s_build.wait_event(st["done"])     # proposals of stage u-depth-1 read this env
                b.set_betas([binding.nishimori_beta(p)] * n)
                b.make_couplings(seeds, p)
                e[0].record(s_build)
                b.build_env(want_lnZ=False)
                e[1].record(s_build)
            with torch.cuda.stream(s_prop):
                s_prop.wait_event(e[1])
                e[2].record(s_prop)
                b.propose(K, args.seed, first_proposal=0, out=st["out"])
                e[3].record(s_prop)
                ch = st["chains"]
                for x in (ch["spins"], ch["E"], ch["logq"], ch["init"]):
                    x.zero_()
                acc, _ = b.accept(st["out"], ch, seed=args.seed, accum=st["accum"])
                per_real = acc.sum(dim=1, dtype=torch.float64)
                sums.append(torch.stack([per_real.sum(), (per_real * L2).sum()]))
                done = torch.cuda.Event()
                done.record(s_prop)
                st["done"] = done
            ev.append(e)
        return sums, ev

    run(max(1, args.warmup))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sums, ev = run(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per_stage = torch.stack(sums).tolist()                   # [steps * len(ps)][2]
    accepted = int(sum(a for a, _ in per_stage))
    updates = sum(x for _, x in per_stage)
    attempted = args.steps * len(ps) * n * (K - 1)
    build_ms = sum(e[0].elapsed_time(e[1]) for e in ev) / len(ev)
    prop_ms = sum(e[2].elapsed_time(e[3]) for e in ev) / len(ev)
    wall = t1 - t0
    nfrac = narrow_fraction(sets[0]["b"])
    del sets, sums, ev
    torch.cuda.synchronize()
    if cu_mask is not None:
        s_prop.destroy()
    res = {"Ls": sorted(set(Ls)), "chi": chi, "n": n, "K": K, "p": ps[0] if len(ps) == 1 else ps,
           "wall_s": wall, "ms_per_step": 1e3 * wall / args.steps,
           "value": updates / wall, "accepted": accepted, "attempted": attempted,
           "acceptance": accepted / attempted, "build_ms": build_ms, "propose_ms": prop_ms,
           "graph": False, "pipelined": True, "builds_in_flight": depth,
           "narrow_fraction": nfrac,
           "propose_cu_mask": cu_mask}
    if len(ps) > 1:
        res["acceptance_per_p"] = {
            str(p): sum(per_stage[u][0] for u in range(j, len(per_stage), len(ps)))
            / (args.steps * n * (K - 1)) for j, p in enumerate(ps)}
        res["batches_per_step"] = len(ps)
    return add_rooflines(res, args, Ls)


def run_fp64_plain(args, L, chi, p, K_full, n_prop=20):
    """FP64 environments, one realization per call, one proposal per call (bounded sample)."""
    import torch
    from paper_2409_06538_amd import binding
    beta = binding.nishimori_beta(p)
    dev = torch.device("cuda:0")
    b = binding.Batch([L], [beta], [0], chi, "fp64", K=1, device=dev)
    b.make_couplings([0], p)
    b.build_env(want_lnZ=False)     # warm-up launch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.build_env(want_lnZ=False)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    chains = b.new_chains(1)
    accepted = 0
    t0 = time.perf_counter()
    for k in range(n_prop):
        prop = b.propose(1, args.seed, first_proposal=k)
        acc, _ = b.accept(prop, chains, seed=args.seed, first_step=k)
        accepted += int(acc.sum().item())
    torch.cuda.synchronize()
    t_prop = (time.perf_counter() - t0) / n_prop
    pa = accepted / max(1, n_prop - 1)
    t_real = t_build + K_full * t_prop
    return {"value": (K_full - 1) * pa * L * L / t_real, "unit": "spin-updates/s",
            "acceptance": pa, "build_s": t_build, "s_per_proposal": t_prop,
            "sample": f"1 realization (seed 0): FP64 build + {n_prop} single-proposal calls, "
                      f"extrapolated to {K_full} proposals"}


def run_cpu_baseline(L, chi, p, K_full, seed, n_real=6, n_prop=150):
    """The oracle on one host core: n_real realizations (coupling seeds 0..n_real-1), each a full
    build + n_prop proposals (vectorised) + the chain, extrapolated to K_full proposals per
    realization."""
    from threadpoolctl import threadpool_limits
    from oracle import accept, energy, envbuild, instance, sampler
    beta = instance.nishimori_beta(p)
    t_build = t_prop = 0.0
    acc = 0
    with threadpool_limits(limits=1):
        for i in range(n_real):
            Jh, Jv = instance.couplings(i, L, p)
            t0 = time.perf_counter()
            env = envbuild.build_env(Jh, Jv, beta, chi)
            t_build += time.perf_counter() - t0
            t0 = time.perf_counter()
            smp = sampler.run(env, Jh, Jv, beta, K=n_prop, seed=seed, realization=i)
            E = energy.energy(smp["spins"], Jh, Jv)
            ch = accept.chain(E, smp["logq"], beta, seed=seed, realization=i)
            t_prop += time.perf_counter() - t0
            acc += int(ch["accepted"].sum())
    pa = acc / (n_real * (n_prop - 1))
    t_b = t_build / n_real
    t_p = t_prop / (n_real * n_prop)
    t_real = t_b + K_full * t_p
    return {"value": (K_full - 1) * pa * L * L / t_real, "unit": "spin-updates/s", "cores": 1,
            "kind": "oracle", "acceptance": pa,
            "sample": f"{n_real} realizations (coupling seeds 0..{n_real - 1}), each a full FP64 "
                      f"environment build ({t_b:.2f} s) + {n_prop} proposals ({t_p * 1e3:.1f} ms "
                      f"each) + accepts; {t_build + t_prop:.1f} s of CPU work in all, "
                      f"extrapolated to {K_full} proposals per realization; single thread"}


def _cpu_worker(job):
    """One realization on one core: full FP64 build, n_prop proposals, the chain."""
    L, chi, p, seed, i, n_prop = job
    from threadpoolctl import threadpool_limits
    from oracle import accept, energy, envbuild, instance, sampler
    beta = instance.nishimori_beta(p)
    with threadpool_limits(limits=1):
        Jh, Jv = instance.couplings(i, L, p)
        t0 = time.perf_counter()
        env = envbuild.build_env(Jh, Jv, beta, chi)
        t_build = time.perf_counter() - t0
        t0 = time.perf_counter()
        smp = sampler.run(env, Jh, Jv, beta, K=n_prop, seed=seed, realization=i)
        E = energy.energy(smp["spins"], Jh, Jv)
        ch = accept.chain(E, smp["logq"], beta, seed=seed, realization=i)
        t_prop = time.perf_counter() - t0
    return t_build, t_prop, int(ch["accepted"].sum())


def run_cpu_all_cores(L, chi, p, K_full, seed, n_prop=150, max_workers=16):
    """The oracle on every host core the process may use (at most max_workers): one process per
    core, each a realization (coupling seeds 0..w-1) with a full build + n_prop proposals + the
    chain, extrapolated to K_full proposals; the realizations run side by side, so the batch takes
    the longest extrapolated time.  Runs before anything touches the GPU (forked workers)."""
    import multiprocessing as mp
    w = max(1, min(max_workers, len(os.sched_getaffinity(0))))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(w) as pool:
        out = pool.map(_cpu_worker, [(L, chi, p, seed, i, n_prop) for i in range(w)])
    wall = time.perf_counter() - t0
    t_real = max(tb + K_full * tp / n_prop for tb, tp, _ in out)
    updates = sum((K_full - 1) * (a / (n_prop - 1)) * L * L for _, _, a in out)
    return {"value": updates / t_real, "unit": "spin-updates/s", "cores": w, "kind": "oracle",
            "sample": f"{w} realizations (coupling seeds 0..{w - 1}), one process each, each a "
                      f"full FP64 build + {n_prop} proposals + accepts ({wall:.1f} s wall), "
                      f"extrapolated to {K_full} proposals per realization"}


def calib_copy(mib):
    """One device-to-device copy of `mib` MiB: reads and writes exactly mib MiB each."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


DEFAULT_STEPS = {"rbim16": 50, "rbim64": 50, "mixed": 4, "rbim256": 2, "rbim256_chi32": 2}

SWEEP_LS = (16, 32, 64, 128, 256)
SWEEP_CHIS = (8, 16, 32, 48)


def run_sweep(args):
    """Acceptance and cost against L and chi (the quantities of the paper's acceptance-ratio and
    cost figures, Sec. III B): for each (L, chi), 16 realizations at p = 0.109 on the Nishimori
    line, 256 proposals each, one serial step timed after one warm-up.  One JSON line per point:
    p_a, build and proposal times, the time per valid (accepted) sample per realization, and the
    accepted spin-updates/s of the batch."""
    import copy
    for chi in SWEEP_CHIS:
        for L in SWEEP_LS:
            w = dict(L=L, p=0.109, chi=chi, seeds=tuple(range(16)), proposals=256)
            a = copy.copy(args)
            a.steps, a.warmup, a.graph = 1, 1, False
            res = run_gpu(a, w)
            wall_per_real = res["wall_s"]          # the realizations run side by side
            print(json.dumps({
                "sweep": "acceptance_cost", "L": L, "chi": chi, "precision": args.precision,
                "realizations": res["n"], "proposals": res["K"], "acceptance": res["acceptance"],
                "build_ms": res["build_ms"], "propose_ms": res["propose_ms"],
                "ms_per_valid_sample": 1e3 * wall_per_real / max(1.0, res["acceptance"] * (res["K"] - 1)),
                "accepted_spin_updates_per_s": res["value"]}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=0,
                    help="timed steps (default: 50 for rbim64 and rbim16, whose steps take "
                         "milliseconds, so that the pipeline fill and drain inside the timed "
                         "region are amortised; 4 for mixed; 2 for rbim256)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rbim64")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "bf16"])
    ap.add_argument("--proposals", type=int, default=0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--serial", action="store_true",
                    help="run the steps one after the other on one stream (default: consecutive "
                         "steps overlap on two streams, the build of step t+1 during the "
                         "proposals of step t, with double-buffered environments)")
    ap.add_argument("--no-serial", action="store_true",
                    help="skip the serial comparison run")
    ap.add_argument("--reserve-cus", type=int, default=1, choices=[0, 1],
                    help="overlapped steps: keep 8 CUs of every XCD per build in flight free of "
                         "proposal work (0: no CU mask)")
    ap.add_argument("--builds-in-flight", type=int, default=2, choices=[1, 2],
                    help="overlapped steps: environment builds of later steps running at once")
    ap.add_argument("--sweep", action="store_true",
                    help="acceptance and cost against L and chi (one JSON line per point) instead "
                         "of the benchmark line")
    ap.add_argument("--graph", action="store_true",
                    help="capture the whole step in one HIP graph and time its replays (phase "
                         "times then come from the eager warm-up steps)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the run, copy one buffer of this many MiB once (a plain copy "
                         "kernel of known size, the reference for hardware byte counters)")
    args = ap.parse_args()
    if not args.steps:
        args.steps = DEFAULT_STEPS.get(args.workload, 20)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the realizations of a "
              "batch are independent, so N GPUs would each run their own share; this "
              "benchmark measures one GPU's share.", file=sys.stderr)
        sys.exit(2)
    if args.sweep:
        run_sweep(args)
        return
    import synth
    wl = synth.WORKLOADS[args.workload]
    multi_p = len(disorder_strengths(wl)) > 1
    # the oracle on all host cores first, while no process has touched the GPU (forked workers)
    cpu_all = None
    if not args.no_cpu and not multi_p and "L" in wl and not args.sweep:
        cpu_all = run_cpu_all_cores(wl["L"], wl["chi"], wl["p"], args.proposals or wl["proposals"],
                                    args.seed)
    serial = args.serial or args.graph
    res = run_gpu(args) if serial else run_gpu_pipelined(args)
    if not serial and not args.no_serial:
        # the same steps one after the other on one stream, for comparison
        import copy
        a2 = copy.copy(args)
        a2.steps, a2.warmup = (1, 0) if multi_p else (3, 1)
        r2 = run_gpu(a2)
        res["serial"] = {"value": r2["value"], "ms_per_step": r2["ms_per_step"], "steps": a2.steps,
                         "build_ms": r2["build_ms"], "propose_ms": r2["propose_ms"]}
    if args.calib_copy_mib:
        calib_copy(args.calib_copy_mib)
    uniform = len(res["Ls"]) == 1
    L0 = res["Ls"][0]
    p0 = res["p"][len(res["p"]) // 2] if multi_p else res["p"]
    # the FP64 plain form and the CPU oracle are measured on uniform-L workloads with one
    # disorder strength (the FP64 plain form where FP64 environments exist at this chi)
    from paper_2409_06538_amd import binding
    fp64_ok = bool(binding.load().tnmc_chi_supported(res["chi"], binding.PRECISIONS["fp64"]))
    plain = None if args.no_plain or not uniform or not fp64_ok else \
        run_fp64_plain(args, L0, res["chi"], p0, res["K"])
    cpu = None if args.no_cpu or not uniform or multi_p else \
        run_cpu_baseline(L0, res["chi"], p0, res["K"], args.seed)
    if cpu is not None:
        cpu["all_cores"] = cpu_all
    size = f"{L0}x{L0}" if uniform else "L x L (L in " + ", ".join(map(str, res["Ls"])) + ")"
    line = {
        "metric": METRIC,
        "value": res["value"],
        "unit": "spin-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {res['n']} realizations of the {size} open "
                               + (f"+-J lattice for each p in {tuple(res['p'])} (the same coupling "
                                  f"seeds, one batch per p), Nishimori beta, chi={res['chi']}, "
                                  if multi_p else
                                  f"+-J lattice, p={res['p']}, Nishimori beta, chi={res['chi']}, ")
                               + f"{res['K']} proposals each, {args.precision} batched"
                               + (", one HIP graph per step" if res["graph"] else "")
                               + (f", consecutive steps overlapped (builds of the next "
                                  f"{res.get('builds_in_flight')} step(s) during the proposals of "
                                  f"step t)" if res.get("pipelined") else ""),
                   "L": L0 if uniform else res["Ls"], "chi": res["chi"], "realizations": res["n"],
                   "proposals": res["K"], "p": res["p"], "precision": args.precision,
                   "graph": res["graph"], "pipelined": bool(res.get("pipelined")),
                   "builds_in_flight": res.get("builds_in_flight"),
                   "propose_cu_mask": res.get("propose_cu_mask")},
        "acceptance": res["acceptance"],
        "acceptance_per_p": res.get("acceptance_per_p"),
        "accepted": res["accepted"],
        "attempted": res["attempted"],
        "build_ms": res["build_ms"],
        "propose_ms": res["propose_ms"],
        "serial": res.get("serial"),
        "fp64_plain": plain,
        "roofline": res["roofline"],
        "roofline_propose": res["roofline_propose"],
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
