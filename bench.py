"""Benchmark of the TNMC hot path on one MI355X.

One step = one pass of the whole hot path over one batch: couplings (a1) -> environments (a2,
a3) -> K proposals per realization with log q and exact energies (a4, a5) -> independence
Metropolis over them (a6).  Default workload: the largest configuration built, 128 realizations
of the 256 x 256 open +-J lattice at each of p = 0.10, 0.109, 0.12 on the Nishimori line
(the same coupling seeds), chi = 48, BF16 environments, 1000 proposals each (one launch per
stage for each batch).  `--workload rbim64` runs the 64 realizations of the 64 x 64 lattice at
chi = 32 (FP32), `--workload mixed` the mixed-L batch, `--workload rbim16` the single 16 x 16
FP64 realization.

Consecutive stages overlap: the builds of the next one or two batches (one workgroup per
realization each, one stream each) run during the proposals and accepts of the current one (on
the other CUs; a CU mask keeps 8 CUs of every XCD per build free when a build has at most 64
workgroups); depth + 1 sets of environments rotate.  The timed region starts with an empty
pipeline and ends when the last stage's accepts are done.  Every stage draws new proposals
(first proposal id = stage index x K) and its chains continue from the previous stage of the
same batch (the same instance, so the same target distribution).  `serial` reports the same
steps one after the other on one stream.  Also measured: the FP64 plain form (FP64
environments, one realization per call, one proposal per call) on a bounded sample, the CPU
FP64 oracle on the host (bounded sample, extrapolated; labelled), and the error of the timed
run's environments and log q against stored oracle values (tests/golden).

Prints ONE JSON line.  Usage: python bench.py [--gpus 1] [--steps 2] [--warmup 1] [--serial]
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
# published dense peaks of MI355X per arithmetic type (matrix cores; FP32 and FP64 equal the
# vector rates)
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}
HBM_PEAK_GBS = 8000.0
DEFAULT_WORKLOAD = "rbim1024"
GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")
PARITY_BOUND = {"fp64": 1e-10, "fp32": 1e-4, "bf16": 5e-3}


def build_arithmetic(precision, chi):
    """Arithmetic type of env_build_kernel: FP64 for FP64 environments and for the Gram form
    (chi <= 32) of FP32 / BF16 environments; FP32 for the QR form at chi = 48."""
    return "f64" if precision == "fp64" or chi <= 32 else "f32"


def sampler_arithmetic(precision):
    return "f64" if precision == "fp64" else "f32"


def proposals_per_wg(precision, n, K, Lmax):
    """Proposals per workgroup of the matrix-core proposal kernel (16 per wavefront; the library
    picks 8 wavefronts for L <= 64 and at least 256 workgroups of 128 proposals, else 4)."""
    wide = Lmax <= 64 and n * ((K + 127) // 128) >= 256
    return 128 if wide else 64


# Counters per dispatch of the dominant kernels in the benchmark's launch shapes (rocprofv3 --pmc;
# the summaries and commands are in profiles/rbim1024_bf16_counters.md): FETCH_SIZE / WRITE_SIZE
# in KiB, each scaled by the same counter on a plain copy of known size, and the matrix-core
# counters (SQ_INSTS_VALU_MFMA_MOPS_* count 512 flops each; SQ_VALU_MFMA_BUSY_CYCLES and
# GRBM_GUI_ACTIVE as read).  The build's are those of a grouped launch (3 batches).  Valid only
# for the kernel sources they were taken on: reported as null once those change (SHA-256).
COUNTERS = {
    ('rbim1024', 'bf16', 'env_build'): {
        "fetch_kib": 19791756.125,
        "fetch_factor": 1.9999215633637493,
        "write_kib": 107822896.0625,
        "write_factor": 1.0,
        "mfma_mops": {
            "f64": 0.0,
            "f32": 1569153360.0,
            "bf16": 0.0
        },
        "mfma_busy_cycles": 12553226880.0,
        "gui_active_cycles": 327197643153.3333,
        "sources_sha256": {
            "envbuild_big.hip": "d6209715394e95d4116bd132216b20fc5332447b129ff980638cbc8edb6fe23a",
            "envbuild.hip": "d97c38100d1f5525e3885a57b0b45f8f9c3c24d3e100170ee22714174da530d1",
            "common.hpp": "373c1289408779effdb76fff0cb18b389447af9368a0c2b3675272823aa4c649",
            "internal.hpp": "3d0517399abdfb569676091d83432670ac9227b5acd41f4e53100848669d982a"
        }
    },
    ('rbim1024', 'bf16', 'propose'): {
        "fetch_kib": 205306683.9943182,
        "fetch_factor": 1.9999215633637493,
        "write_kib": 277552281.70454544,
        "write_factor": 1.0,
        "mfma_mops": {
            "f64": 0.0,
            "f32": 10007662592.0,
            "bf16": 0.0
        },
        "mfma_busy_cycles": 80061300736.0,
        "gui_active_cycles": 98373586976.45454,
        "sources_sha256": {
            "sampler.hip": "21f7e11f26a4a70d277c53c83d2085e292c1ca8e1f3769bf674d6adcdeb0eec1",
            "common.hpp": "373c1289408779effdb76fff0cb18b389447af9368a0c2b3675272823aa4c649",
            "internal.hpp": "3d0517399abdfb569676091d83432670ac9227b5acd41f4e53100848669d982a"
        }
    },
}

def counted(workload, precision, kernel):
    import hashlib
    rec = COUNTERS.get((workload, precision, kernel))
    if rec is None:
        return None
    csrc = os.path.join(ROOT, "paper_2409_06538_amd", "csrc")
    for name, digest in rec["sources_sha256"].items():
        with open(os.path.join(csrc, name), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    return rec


def counted_traffic(rec):
    if rec is None or "fetch_kib" not in rec:
        return None
    return 1024.0 * (rec["fetch_kib"] * rec["fetch_factor"] + rec["write_kib"] * rec["write_factor"])


def mfma_counters(rec, launch_ms, peak_tflops):
    """Executed matrix-core flops of one launch and their rate against the peak of the kernel's
    arithmetic type, and the matrix-core busy fraction."""
    if rec is None or "mfma_mops" not in rec:
        return None
    mops = rec["mfma_mops"]
    flops = {k: 512.0 * v for k, v in mops.items()}
    total = sum(flops.values())
    ach = total / (launch_ms * 1e-3) / 1e12
    return {"executed_flops_per_launch": flops, "executed_tflops": ach,
            "executed_frac_of_peak": ach / peak_tflops,
            "mfma_busy_cycles": rec.get("mfma_busy_cycles"),
            "grbm_gui_active_cycles": rec.get("gui_active_cycles")}


def build_flops_per_site(chi):
    """Algorithmic work of one site of the canonical compression (QR of a 4chi x 2chi matrix
    with Q, SVD of a 2chi x 2chi matrix, the two contractions), ~270 chi^3."""
    return 270.0 * chi ** 3


def build_bytes_per_site(chi, env_bytes, carry_bytes):
    """Algorithmic HBM bytes of one site: the site of E_r read twice (4 chi^2 elements), the site
    of E_{r-1} written (2 chi^2), the carried factor (2chi x 2chi) written and read back."""
    return 6.0 * chi * chi * env_bytes + 2.0 * (2 * chi) ** 2 * carry_bytes


ENV_BYTES = {"fp64": 8, "fp32": 4, "bf16": 2}


def workload_sizes(w):
    """Lattice size of every realization of a workload (uniform L, or L cycling through Ls)."""
    seeds = list(w["seeds"])
    if "Ls" in w:
        return [w["Ls"][i % len(w["Ls"])] for i in range(len(seeds))], seeds
    return [w["L"]] * len(seeds), seeds


def add_rooflines(res, args, Ls):
    """Dominant-kernel rooflines from the HIP-event launch times in `res`.

    Build: 270 chi^3 flops per site (the canonical compression), against the dense peak of the
    build's own arithmetic type.  Proposals: per realization the environments are streamed once
    per pass, 2 passes x 2 chi^2 L^2 elements, and every proposal costs 8 chi^2 L^2 flops; the
    kernel is quoted against the matrix-core peak of its arithmetic when that intensity is past
    the ridge point, else against HBM."""
    chi, K, prop_ms = res["chi"], res["K"], res["propose_ms"]
    # one build launch may cover the batches of several stages (grouped steps)
    units = res.get("build_units_per_launch", 1)
    build_ms = res.get("build_launch_ms", res["build_ms"])
    prec = args.precision
    bar = build_arithmetic(prec, chi)
    flops = units * sum(build_flops_per_site(chi) * (L - 1) * L for L in Ls)
    carry = 8 if bar == "f64" else 4
    bbytes = units * sum(build_bytes_per_site(chi, ENV_BYTES[prec], carry) * (L - 1) * L
                         for L in Ls)
    peak = PEAK_TFLOPS[bar]
    achieved = flops / (build_ms * 1e-3) / 1e12
    rec = counted(args.workload, prec, "env_build")
    traffic = counted_traffic(rec)
    res["roofline"] = {"kernel": "env_build_kernel", "bound": "mfma", "arithmetic": bar,
                       "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                       "frac": achieved / peak, "traffic": traffic,
                       "traffic_over_algorithmic": None if traffic is None else traffic / bbytes,
                       "launch_ms": build_ms, "batches_per_launch": units,
                       "algorithmic_flops_per_launch": flops,
                       "algorithmic_bytes_per_launch": bbytes,
                       "mfma_counters": mfma_counters(rec, build_ms, peak)}
    sar = sampler_arithmetic(prec)
    pbytes = sum(2.0 * 2 * chi * chi * L * L * ENV_BYTES[prec] for L in Ls)
    pflops = sum(8.0 * chi * chi * L * L * K for L in Ls)
    ppeak = PEAK_TFLOPS[sar]
    ridge = ppeak * 1e12 / (HBM_PEAK_GBS * 1e9)
    t = prop_ms * 1e-3
    gbs = pbytes / t / 1e9
    prec_ = counted(args.workload, prec, "propose")
    ptraffic = counted_traffic(prec_)
    kern = "propose_mfma_kernel" if chi % 16 == 0 else "propose_kernel"
    if pflops / pbytes > ridge:
        ach = pflops / t / 1e12
        rp = {"bound": "mfma", "achieved": ach, "peak": ppeak, "unit": "TFLOP/s",
              "frac": ach / ppeak}
    else:
        rp = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
              "frac": gbs / HBM_PEAK_GBS}
    res["roofline_propose"] = dict(
        kernel=kern, arithmetic=sar, **rp, traffic=ptraffic,
        traffic_over_algorithmic=None if ptraffic is None else ptraffic / pbytes,
        launch_ms=prop_ms, algorithmic_bytes_per_launch=pbytes,
        algorithmic_flops_per_launch=pflops, intensity_flop_per_byte=pflops / pbytes,
        ridge_flop_per_byte=ridge, hbm_algorithmic_GBs=gbs,
        narrow_site_fraction=res.get("narrow_fraction"),
        mfma_counters=mfma_counters(prec_, prop_ms, ppeak))
    return res


def progress(msg):
    """A line on stderr as each part of the run completes (the JSON line goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def autotune(args, b, K):
    """The library's launch-shape autotuner on the built batch: every candidate shape of the
    proposal kernel timed once after an untimed launch; the fastest is kept in the library's
    tuning table and used by the timed steps."""
    if not args.autotune:
        return None
    t0 = time.perf_counter()
    best, ms = b.autotune_propose(K, seed=args.seed, reps=1)
    progress(f"autotune: {best} wavefronts per workgroup ({ms})")
    return {"kernel": "propose", "waves_per_workgroup": best, "proposals_per_workgroup":
            16 * best if b.chi % 16 == 0 else 64, "ms_per_candidate": ms,
            "search_s": time.perf_counter() - t0}


def load_goldens():
    """Stored FP64 oracle values (tests/golden/oracle_*.json, written by
    tests/golden/make_oracle_goldens.py, which calls only the oracle)."""
    import glob
    out = []
    for f in sorted(glob.glob(os.path.join(GOLDEN_DIR, "oracle_*.json"))):
        with open(f) as fh:
            g = json.load(fh)
        g["name"] = os.path.basename(f)[len("oracle_"):-len(".json")]
        out.append(g)
    return out


def error_vs_oracle(envs, args, w, Ls, seeds):
    """Error of the timed run's results against the stored oracle values of the realizations
    they cover: every environment log-norm lambda_r, the GPU's teacher-forced log q of the
    oracle's own proposals (relative and absolute), and their exact energies (bit for bit).
    `envs` lists (batch, p) of the environments still held after the timed steps."""
    import numpy as np
    import torch
    bound = PARITY_BOUND[args.precision]
    cases = []
    for g in load_goldens():
        if g["chi"] != w["chi"] or g["coupling_seed"] not in seeds:
            continue
        i = seeds.index(g["coupling_seed"])
        if Ls[i] != g["L"]:
            continue
        hit = [b for b, p in envs if abs(p - g["p"]) < 1e-12]
        if not hit:
            continue
        b = hit[0]
        torch.cuda.synchronize()
        lam = b.lognorm[i].cpu().numpy()
        ref = np.array([np.nan if x is None else x for x in g["lognorm"]])
        ok = ~np.isnan(ref)
        rl = np.abs(lam[ok] - ref[ok]) / np.abs(ref[ok])
        case = {"golden": g["name"], "realization": i, "rows_compared": int(ok.sum()),
                "lognorm_max_rel": float(rl.max()),
                "lognorm_max_abs": float(np.abs(lam[ok] - ref[ok]).max())}
        if "proposals" in g:
            pr = g["proposals"]
            K = len(pr["logq"])
            words = np.zeros((b.n, K, b.Lmax, b.Wmax), dtype=np.uint64)
            sp = np.array([[[int(x, 16) for x in row.split()] for row in conf]
                           for conf in pr["spins_hex"]], dtype=np.uint64)
            words[i, :, :g["L"], :sp.shape[2]] = sp
            d = torch.from_numpy(words.view(np.int64)).to(b.device)
            lq = b.logq(d)[i].cpu().numpy()
            E = b.energy(d)[i].cpu().numpy()
            ref_q = np.array(pr["logq"])
            case.update({"proposals": K,
                         "logq_max_rel": float((np.abs(lq - ref_q) / np.abs(ref_q)).max()),
                         "logq_max_abs": float(np.abs(lq - ref_q).max()),
                         "energy_bit_exact": bool(np.array_equal(E, pr["E"]))})
        cases.append(case)
    if not cases:
        return None
    lmax = max(c["lognorm_max_rel"] for c in cases)
    qs = [c["logq_max_rel"] for c in cases if "logq_max_rel" in c]
    return {"source": "tests/golden/oracle_*.json (FP64 oracle)", "bound_rel": bound,
            "lognorm_max_rel": lmax, "logq_max_rel": max(qs) if qs else None,
            "energy_bit_exact": all(c.get("energy_bit_exact", True) for c in cases),
            "within_bound": lmax < bound and (not qs or max(qs) < bound), "cases": cases}


def narrow_fraction(batch):
    """Fraction of the environment sites whose both bonds are at most 16 by the bond table the
    build wrote (their entries all lie in the leading 16 x 16 block of both matrices: the
    proposal kernel then stores one 16-row tile of V per spin value)."""
    tot = narrow = 0
    for i, L in enumerate(batch.Ls):
        bt = batch.bond_table(i)
        tot += L * L
        narrow += int(((bt[:, :L] <= 16) & (bt[:, 1:] <= 16)).sum().item())
    return narrow / max(1, tot)


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
    chains = [b.new_chains(1) for _ in ps]       # one chain per realization and disorder strength
    L2 = torch.tensor([L * L for L in Ls], dtype=torch.float64, device=dev)
    ev = []
    stage = [0] * len(ps)

    def step(events):
        """One pass over every p; returns per-p [accepted, accepted x L^2, attempted] (device
        tensors).  Eager steps draw new proposals (first proposal id = stage x K) and continue
        each p's chains; a captured step restarts its chains and replays the same proposals."""
        sums = []
        for j, p in enumerate(ps):
            ch = chains[j]
            if len(ps) > 1:
                b.set_betas([binding.nishimori_beta(p)] * n)
            b.make_couplings(seeds, p)
            if events is not None:
                events[3 * j].record()
            b.build_env(want_lnZ=False)
            if events is not None:
                events[3 * j + 1].record()
            first = 0 if args.graph else stage[j] * K
            b.propose(K, args.seed, first_proposal=first, out=out)
            if events is not None:
                events[3 * j + 2].record()
            if args.graph:
                for t in (ch["spins"], ch["E"], ch["logq"], ch["init"]):
                    t.zero_()
            fresh = (ch["init"] == 0).sum(dtype=torch.float64)
            acc, _ = b.accept(out, ch, seed=args.seed, first_step=first, accum=accum)
            per_real = acc.sum(dim=1, dtype=torch.float64)
            sums.append(torch.stack([per_real.sum(), (per_real * L2).sum(), n * K - fresh]))
            stage[j] += 1
        return torch.stack(sums)

    def new_events():
        return [torch.cuda.Event(enable_timing=True) for _ in range(3 * len(ps))]

    for _ in range(max(1, args.warmup) if args.graph else args.warmup):
        e = new_events()
        step(e)
        ev.append(e)          # graph mode: phase times come from the eager warm-up steps
    torch.cuda.synchronize()
    progress("warm-up steps done")
    tune = autotune(args, b, K)
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
    progress(f"timed steps done ({t1 - t0:.1f} s)")
    per_p = torch.stack(accs).sum(dim=0).tolist()            # [len(ps)][3]
    accepted = int(sum(a for a, _, _ in per_p))
    updates = sum(u for _, u, _ in per_p)
    attempted = int(sum(t for _, _, t in per_p))
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
        "error_vs_oracle": error_vs_oracle([(b, ps[-1])], args, w, Ls, seeds),
        "autotune": tune,
    }
    if len(ps) > 1:
        res["acceptance_per_p"] = {str(p): per_p[j][0] / per_p[j][2] for j, p in enumerate(ps)}
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


def run_gpu_grouped(args):
    """Consecutive steps overlapped in groups: the batches of `group` consecutive pipeline
    stages are built by one launch (one workgroup per realization, group x n of them) on one
    stream, while the proposal launches of the previous group run side by side, one stream each,
    and its accepts follow in stage order (the chains continue from stage to stage); two groups
    of batches alternate, so a build never overwrites environments that proposals still read.
    For workloads with few realizations (rbim1024: 2), whose build occupies a few CUs for seconds
    per launch while a proposal launch fills a few dozen."""
    import torch
    from paper_2409_06538_amd import binding
    import synth

    w = synth.WORKLOADS[args.workload]
    Ls, seeds = workload_sizes(w)
    ps = disorder_strengths(w)
    chi, K = w["chi"], args.proposals or w["proposals"]
    n = len(seeds)
    D = args.group_steps
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # one build stream; the proposal launches of a group run side by side, one stream each (a
    # launch of a few realizations fills a few dozen CUs), and the accepts follow on the first
    s_build = torch.cuda.Stream()
    s_props = [torch.cuda.Stream() for _ in range(D)]
    s_prop = s_props[0]
    groups = []
    for _ in range(2):
        members = []
        for _ in range(D):
            b = binding.Batch(Ls, [binding.nishimori_beta(ps[0])] * n, seeds, chi, args.precision,
                              K=K, device=dev)
            out = (torch.empty(b.spins_shape(K), dtype=torch.int64, device=dev),
                   torch.empty((n, K), dtype=torch.float64, device=dev),
                   torch.empty((n, K), dtype=torch.int32, device=dev))
            members.append({"b": b, "out": out, "p": None,
                            "accum": torch.zeros((n, binding.OBS_COUNT), dtype=torch.float64,
                                                 device=dev)})
        ws = torch.empty(binding.group_workspace_bytes([m["b"] for m in members]),
                         dtype=torch.uint8, device=dev)
        groups.append({"members": members, "ws": ws, "done": None})
    chains = [groups[0]["members"][0]["b"].new_chains(1) for _ in ps]
    stage = [0] * len(ps)
    L2 = torch.tensor([L * L for L in Ls], dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    def run(steps):
        """`steps` passes over every p; stages (step, p) in order, D per build launch."""
        sums, ev = [], []
        n_stage = steps * len(ps)
        for g0 in range(0, n_stage, D):
            grp = groups[(g0 // D) % 2]
            us = list(range(g0, min(g0 + D, n_stage)))
            mem = grp["members"][:len(us)]
            e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            with torch.cuda.stream(s_build):
                if grp["done"] is not None:
                    s_build.wait_event(grp["done"])   # proposals of the group before still read
                for u, m in zip(us, mem):
                    m["p"] = ps[u % len(ps)]
                    m["b"].set_betas([binding.nishimori_beta(m["p"])] * n)
                    m["b"].make_couplings(seeds, m["p"])
                e[0].record(s_build)
                binding.build_env_group([m["b"] for m in mem], grp["ws"])
                e[1].record(s_build)
            firsts, pdone = [], []
            for k, (u, m) in enumerate(zip(us, mem)):
                sp = s_props[k]
                with torch.cuda.stream(sp):
                    sp.wait_event(e[1])
                    jp = u % len(ps)
                    ep = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
                    ep[0].record(sp)
                    first = stage[jp] * K
                    stage[jp] += 1
                    firsts.append(first)
                    m["b"].propose(K, args.seed, first_proposal=first, out=m["out"])
                    ep[1].record(sp)
                    ev.append(("propose", ep))
                    pdone.append(ep[1])
            with torch.cuda.stream(s_prop):
                for d in pdone:
                    s_prop.wait_event(d)
                for u, m, first in zip(us, mem, firsts):   # the chains advance in stage order
                    jp = u % len(ps)
                    ch = chains[jp]
                    fresh = (ch["init"] == 0).sum(dtype=torch.float64)
                    acc, _ = m["b"].accept(m["out"], ch, seed=args.seed, first_step=first,
                                           accum=m["accum"])
                    per_real = acc.sum(dim=1, dtype=torch.float64)
                    sums.append(torch.stack([per_real.sum(), (per_real * L2).sum(), n * K - fresh]))
                done = torch.cuda.Event()
                done.record(s_prop)
                grp["done"] = done
            ev.append(("build", e, len(us)))
        return sums, ev

    run(max(1, args.warmup))
    torch.cuda.synchronize()
    progress("warm-up stages done")
    tune = autotune(args, groups[0]["members"][0]["b"], K)
    t0 = time.perf_counter()
    sums, ev = run(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    progress(f"timed steps done ({t1 - t0:.1f} s)")
    per_stage = torch.stack(sums).tolist()
    accepted = int(sum(a for a, _, _ in per_stage))
    updates = sum(x for _, x, _ in per_stage)
    attempted = int(sum(t for _, _, t in per_stage))
    builds = [x for x in ev if x[0] == "build"]
    props = [x for x in ev if x[0] == "propose"]
    build_launch_ms = sum(x[1][0].elapsed_time(x[1][1]) for x in builds) / len(builds)
    units = sum(x[2] for x in builds) / len(builds)
    build_ms = build_launch_ms / units     # per batch
    prop_ms = sum(x[1][0].elapsed_time(x[1][1]) for x in props) / len(props)
    wall = t1 - t0
    last = groups[((len(range(0, args.steps * len(ps), D)) - 1)) % 2]["members"]
    nfrac = narrow_fraction(last[0]["b"])
    envs = [(m["b"], m["p"]) for g in groups for m in g["members"] if m["p"] is not None]
    err = error_vs_oracle(envs, args, w, Ls, seeds)
    del envs, groups, sums, ev, last
    torch.cuda.synchronize()
    res = {"Ls": sorted(set(Ls)), "chi": chi, "n": n, "K": K, "p": ps[0] if len(ps) == 1 else ps,
           "wall_s": wall, "ms_per_step": 1e3 * wall / args.steps,
           "value": updates / wall, "accepted": accepted, "attempted": attempted,
           "acceptance": accepted / attempted, "build_ms": build_ms,
           "build_launch_ms": build_launch_ms, "build_units_per_launch": units,
           "propose_ms": prop_ms,
           "graph": False, "pipelined": True, "group_steps": D, "builds_in_flight": D,
           "narrow_fraction": nfrac, "propose_cu_mask": None, "error_vs_oracle": err,
           "autotune": tune}
    if len(ps) > 1:
        res["acceptance_per_p"] = {
            str(p): sum(per_stage[u][0] for u in range(j, len(per_stage), len(ps)))
            / sum(per_stage[u][2] for u in range(j, len(per_stage), len(ps)))
            for j, p in enumerate(ps)}
        res["batches_per_step"] = len(ps)
    return add_rooflines(res, args, Ls)


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
        sets.append({"b": b, "out": out,
                     "accum": torch.zeros((n, binding.OBS_COUNT), dtype=torch.float64, device=dev),
                     "done": None, "p": None})
    # one chain per realization and disorder strength, continued from stage to stage (all
    # accepts run in stage order on the proposal stream)
    chains = [sets[0]["b"].new_chains(1) for _ in ps]
    stage = [0] * len(ps)
    L2 = torch.tensor([L * L for L in Ls], dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    def run(steps):
        """`steps` passes over every p: one pipeline stage per (step, p)."""
        sums, ev = [], []
        for u in range(steps * len(ps)):
            jp = u % len(ps)
            p = ps[jp]
            st = sets[u % (depth + 1)]
            st["p"] = p
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
                first = stage[jp] * K
                stage[jp] += 1
                b.propose(K, args.seed, first_proposal=first, out=st["out"])
                e[3].record(s_prop)
                ch = chains[jp]
                fresh = (ch["init"] == 0).sum(dtype=torch.float64)
                acc, _ = b.accept(st["out"], ch, seed=args.seed, first_step=first,
                                  accum=st["accum"])
                per_real = acc.sum(dim=1, dtype=torch.float64)
                sums.append(torch.stack([per_real.sum(), (per_real * L2).sum(), n * K - fresh]))
                done = torch.cuda.Event()
                done.record(s_prop)
                st["done"] = done
            ev.append(e)
        return sums, ev

    run(max(1, args.warmup))
    torch.cuda.synchronize()
    progress("warm-up stages done")
    tune = autotune(args, sets[0]["b"], K)
    t0 = time.perf_counter()
    sums, ev = run(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    progress(f"timed steps done ({t1 - t0:.1f} s)")
    per_stage = torch.stack(sums).tolist()                   # [steps * len(ps)][3]
    accepted = int(sum(a for a, _, _ in per_stage))
    updates = sum(x for _, x, _ in per_stage)
    attempted = int(sum(t for _, _, t in per_stage))
    build_ms = sum(e[0].elapsed_time(e[1]) for e in ev) / len(ev)
    prop_ms = sum(e[2].elapsed_time(e[3]) for e in ev) / len(ev)
    wall = t1 - t0
    nfrac = narrow_fraction(sets[0]["b"])
    envs = [(st["b"], st["p"]) for st in sets if st["p"] is not None]
    err = error_vs_oracle(envs, args, w, Ls, seeds)
    del envs, sets, sums, ev
    torch.cuda.synchronize()
    if cu_mask is not None:
        s_prop.destroy()
    res = {"Ls": sorted(set(Ls)), "chi": chi, "n": n, "K": K, "p": ps[0] if len(ps) == 1 else ps,
           "wall_s": wall, "ms_per_step": 1e3 * wall / args.steps,
           "value": updates / wall, "accepted": accepted, "attempted": attempted,
           "acceptance": accepted / attempted, "build_ms": build_ms, "propose_ms": prop_ms,
           "graph": False, "pipelined": True, "builds_in_flight": depth,
           "narrow_fraction": nfrac,
           "propose_cu_mask": cu_mask, "error_vs_oracle": err, "autotune": tune}
    if len(ps) > 1:
        res["acceptance_per_p"] = {
            str(p): sum(per_stage[u][0] for u in range(j, len(per_stage), len(ps)))
            / sum(per_stage[u][2] for u in range(j, len(per_stage), len(ps)))
            for j, p in enumerate(ps)}
        res["batches_per_step"] = len(ps)
    return add_rooflines(res, args, Ls)


PLAIN_MAX_L = 128


def run_fp64_plain(args, L, chi, p, K_full, n_prop=None):
    """FP64 environments, one realization per call, one proposal per call (bounded sample).
    Lattices above PLAIN_MAX_L (whose FP64 build takes minutes: about 300 us per site) are
    measured on an L = PLAIN_MAX_L lattice and extrapolated by the site count, L^2, for both the
    build and the proposals; the acceptance is the smaller lattice's (an upper bound)."""
    L_run = min(L, PLAIN_MAX_L)
    out = _run_fp64_plain(args, L_run, chi, p, K_full, n_prop)
    if L_run == L:
        return out
    scale = (L / L_run) ** 2
    t_real = out["build_s"] * scale + K_full * out["s_per_proposal"] * scale
    out.update({"value": (K_full - 1) * out["acceptance"] * L * L / t_real,
                "measured_L": L_run,
                "sample": out["sample"] + f"; measured at L = {L_run} and extrapolated to L = {L} "
                          f"by the site count (x{scale:.0f}), acceptance of L = {L_run}"})
    return out


def _run_fp64_plain(args, L, chi, p, K_full, n_prop=None):
    import torch
    from paper_2409_06538_amd import binding
    n_prop = n_prop or (20 if L < 512 else 4)
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


def _oracle_realization(job):
    """The oracle on one realization, single-threaded.  Full mode: the whole FP64 build, n_prop
    proposals (vectorised) and the chain.  Sliced mode (lattices whose oracle build takes
    minutes): rows_a and rows_b rows of the build from the bottom, the cost per row taken from
    the difference (rows with saturated bonds), and n_prop proposals timed on environments whose
    unbuilt rows repeat the last built row (the same tensor shapes; timing only)."""
    L, chi, p, seed, i, n_prop, sliced = job
    from threadpoolctl import threadpool_limits
    from oracle import accept, energy, envbuild, instance, sampler
    beta = instance.nishimori_beta(p)
    with threadpool_limits(limits=1):
        Jh, Jv = instance.couplings(i, L, p)
        if not sliced:
            t0 = time.perf_counter()
            env = envbuild.build_env(Jh, Jv, beta, chi)
            t_build = time.perf_counter() - t0
            t0 = time.perf_counter()
            smp = sampler.run(env, Jh, Jv, beta, K=n_prop, seed=seed, realization=i)
            E = energy.energy(smp["spins"], Jh, Jv)
            ch = accept.chain(E, smp["logq"], beta, seed=seed, realization=i)
            t_prop = time.perf_counter() - t0
            return t_build, t_prop, int(ch["accepted"].sum()), t_build + t_prop
        rows_a, rows_b = sliced
        t0 = t_start = time.perf_counter()
        envbuild.build_env(Jh, Jv, beta, chi, rows=rows_a)
        t1 = time.perf_counter()
        env = envbuild.build_env(Jh, Jv, beta, chi, rows=rows_b)
        t2 = time.perf_counter()
        per_row = ((t2 - t1) - (t1 - t0)) / (rows_b - rows_a)
        t_build = (t2 - t1) + per_row * (L - 1 - rows_b)
        last = L - 1 - rows_b
        sites = [env["sites"][r] if env["sites"][r] is not None else env["sites"][last]
                 for r in range(L)]
        t0 = time.perf_counter()
        smp = sampler.run({"sites": sites}, Jh, Jv, beta, K=n_prop, seed=seed, realization=i)
        E = energy.energy(smp["spins"], Jh, Jv)
        t_prop = time.perf_counter() - t0
        return t_build, t_prop, None, time.perf_counter() - t_start


def cpu_sample_plan(L):
    """Full oracle realizations up to L = 64; beyond, the sliced sample (8 and 16 rows, 2
    proposals; 4 and 8 rows and one proposal from L = 512 on, where one oracle proposal takes
    seconds)."""
    if L <= 64:
        return None, 150
    return ((8, 16), 2) if L < 512 else ((4, 8), 1)


def _cpu_result(out, L, K_full, n_prop, sliced, cores):
    """Accepted spin-updates/s of realizations run side by side, extrapolated to K_full
    proposals each (the batch takes the longest extrapolated time)."""
    t_real = max(tb + K_full * tp / n_prop for tb, tp, _, _ in out)
    if sliced:
        pas = [1.0] * len(out)       # not measurable from a sample: 1 is an upper bound
    else:
        pas = [a / (n_prop - 1) for _, _, a, _ in out]
    updates = sum((K_full - 1) * pa * L * L for pa in pas)
    return updates / t_real, sum(pas) / len(pas), t_real


def run_cpu_baseline(L, chi, p, K_full, seed, n_real=None):
    """The oracle on one host core: a bounded sample of the workload's realizations (coupling
    seeds 0, 1, ...), extrapolated to K_full proposals per realization."""
    sliced, n_prop = cpu_sample_plan(L)
    n_real = n_real or (6 if not sliced else 1)
    out = [_oracle_realization((L, chi, p, seed, i, n_prop, sliced)) for i in range(n_real)]
    v, pa, t_real = _cpu_result(out, L, K_full, n_prop, sliced, 1)
    v = v / n_real                   # one core runs its realizations one after the other
    work = sum(o[3] for o in out)
    t_b = sum(o[0] for o in out) / n_real
    t_p = sum(o[1] for o in out) / (n_real * n_prop)
    if sliced:
        sample = (f"{n_real} realization (coupling seed 0): the first {sliced[0]} and "
                  f"{sliced[1]} environment rows built (build of all {L - 1} rows extrapolated "
                  f"from the difference: {t_b:.1f} s) + {n_prop} proposals ({t_p:.1f} s each) "
                  f"on environments whose unbuilt rows repeat the last built row (timing only); "
                  f"{work:.1f} s of CPU work in all, extrapolated to {K_full} proposals; "
                  f"acceptance taken as 1 (an upper bound); single thread")
    else:
        sample = (f"{n_real} realizations (coupling seeds 0..{n_real - 1}), each a full FP64 "
                  f"environment build ({t_b:.2f} s) + {n_prop} proposals ({t_p * 1e3:.1f} ms "
                  f"each) + accepts; {work:.1f} s of CPU work in all, extrapolated to {K_full} "
                  f"proposals per realization; single thread")
    return {"value": v, "unit": "spin-updates/s", "cores": 1, "kind": "oracle",
            "acceptance": pa, "sample": sample}


def run_cpu_all_cores(L, chi, p, K_full, seed, max_workers=16):
    """The oracle on every host core the process may use (at most max_workers): one process per
    core, each a realization (coupling seeds 0..w-1) with the bounded sample of
    _oracle_realization, extrapolated to K_full proposals; the realizations run side by side.
    Runs before anything touches the GPU (forked workers)."""
    import multiprocessing as mp
    sliced, n_prop = cpu_sample_plan(L)
    avail = len(os.sched_getaffinity(0))
    w = max(1, min(max_workers, avail))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(w) as pool:
        out = pool.map(_oracle_realization, [(L, chi, p, seed, i, n_prop, sliced)
                                             for i in range(w)])
    wall = time.perf_counter() - t0
    v, pa, _ = _cpu_result(out, L, K_full, n_prop, sliced, w)
    what = (f"the first {sliced[1]} environment rows + {n_prop} proposals (timing only)"
            if sliced else f"a full FP64 build + {n_prop} proposals + accepts")
    return {"value": v, "unit": "spin-updates/s", "cores": w, "cores_available": avail,
            "kind": "oracle", "acceptance": pa,
            "sample": f"{w} realizations (coupling seeds 0..{w - 1}), one process each on the "
                      f"{w} of {avail} cores this process may use (capped at {max_workers}), "
                      f"each {what} ({wall:.1f} s wall), extrapolated to {K_full} proposals per "
                      f"realization" + ("; acceptance taken as 1 (an upper bound)" if sliced else "")}


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


# stages built per launch in the overlapped mode (1: one build per stage, several in flight)
DEFAULT_GROUP_STEPS = {"rbim1024": 3}
DEFAULT_STEPS = {"rbim16": 50, "rbim64": 50, "mixed": 4, "rbim256": 2, "rbim256_chi32": 2,
                 "rbim1024": 9}

SWEEP_LS = (16, 32, 64, 128, 256)
SWEEP_CHIS = (8, 16, 32, 48)


SWEEP_NISHIMORI_PS = (0.05, 0.08, 0.10, 0.109, 0.12, 0.14)
SWEEP_NISHIMORI_LS = (64, 128, 256)
SWEEP_LARGE_LS = (512, 1024)


def sweep_point(args, L, chi, p, n_real, K, kind):
    import copy
    w = dict(L=L, p=p, chi=chi, seeds=tuple(range(n_real)), proposals=K)
    a = copy.copy(args)
    # lattices of 512 and more: no warm-up step (one build takes tens of seconds)
    a.steps, a.warmup, a.graph = 1, (1 if L < 512 else 0), False
    res = run_gpu(a, w)
    wall_per_real = res["wall_s"]          # the realizations run side by side
    print(json.dumps({
        "sweep": kind, "L": L, "chi": chi, "p": p, "T": 2.0 / math.log((1 - p) / p),
        "precision": args.precision, "realizations": res["n"], "proposals": res["K"],
        "acceptance": res["acceptance"], "build_ms": res["build_ms"],
        "propose_ms": res["propose_ms"],
        "ms_per_valid_sample": 1e3 * wall_per_real / max(1.0, res["acceptance"] * (res["K"] - 1)),
        "accepted_spin_updates_per_s": res["value"]}), flush=True)


SWEEP_OBS_LS = (8, 16, 32, 64)
# (L, chi, precision, realizations, proposals) of the forms sweep
SWEEP_FORMS = ((64, 16, "fp32", 64, 256), (256, 16, "fp32", 16, 256), (256, 32, "fp32", 16, 256),
               (256, 64, "bf16", 16, 256), (256, 64, "fp32", 4, 256), (512, 16, "fp32", 4, 128),
               (1024, 64, "bf16", 2, 256))


def sweep_forms_point(L, chi, precision, n_real, K, p=0.109, seed=0):
    """f3: the canonical compression (Gram form, matrices in the workspace) against the zip-up
    on the same batch: build time (HIP events on the launch stream), mean kept bond (bond
    table, interior cuts of every built row), ln Z difference, acceptance of one chain per
    realization over K proposals, accepted spin-updates/s of one serial step."""
    import torch
    from paper_2409_06538_amd import binding
    dev = torch.device("cuda:0")
    beta = binding.nishimori_beta(p)
    seeds = list(range(n_real))
    b = binding.Batch([L] * n_real, [beta] * n_real, seeds, chi, precision, K=K, device=dev)
    b.make_couplings(seeds, p)
    out, lnZs = {}, {}
    for name, form in (("canonical", binding.FORM_GRAM_L2), ("zipup", binding.FORM_ZIPUP)):
        progress(f"forms L={L} chi={chi} {precision}: {name} build")
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        t0 = time.perf_counter()
        e0.record()
        lnZ = b.build_env_form(form)
        e1.record()
        prop = b.propose(K, seed)
        chains = b.new_chains(1)
        acc, _ = b.accept(prop, chains, seed=seed)
        e2.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st, _ = b.status_check()
        bonds = torch.stack([b.bond_table(i)[:L - 1, 1:L].float().mean() for i in range(n_real)])
        accepted = acc.float().sum().item()
        lnZs[name] = lnZ.cpu()
        out[name] = {"build_ms": e0.elapsed_time(e1), "propose_accept_ms": e1.elapsed_time(e2),
                     "mean_bond": bonds.mean().item(), "acceptance": accepted / (n_real * (K - 1)),
                     "accepted_spin_updates_per_s": accepted * L * L / wall, "status": st}
    d = (lnZs["zipup"] - lnZs["canonical"]).abs() / lnZs["canonical"].abs()
    return {"sweep": "forms", "L": L, "chi": chi, "p": p, "precision": precision,
            "realizations": n_real, "proposals": K, **out,
            "lnZ_rel_diff_max": d.max().item(), "lnZ_rel_diff_mean": d.mean().item()}


# (torus side, chi, precision, tori, proposals per step, steps) of the periodic-lattice sweep
SWEEP_PBC = ((17, 16, "fp32", 64, 256, 40), (65, 32, "fp32", 64, 1000, 20),
             (129, 32, "fp32", 16, 256, 5), (257, 48, "bf16", 16, 256, 4))


def step_autocorrelation(E, kmax=5):
    """rho(k), k = 1..kmax, of a (steps, tori) array of per-step energies, pooled over tori
    (each torus's own mean removed), and tau_int = 1/2 + sum of rho(k) up to the first k whose
    rho is not positive."""
    import numpy as np
    x = E - E.mean(axis=0, keepdims=True)
    var = float((x * x).sum())
    rho = [float((x[:-k] * x[k:]).sum()) / var if var > 0 else 0.0
           for k in range(1, min(kmax, E.shape[0] - 1) + 1)]
    tau = 0.5
    for r in rho:
        if r <= 0:
            break
        tau += r
    return rho, tau


def sweep_pbc_point(L, chi, precision, n, K, steps, p=0.109, seed=0):
    """f4: periodic L x L lattices stepped by a frozen row and column per step (Sec. IV), one
    chain per torus: per step the block of (L-1)^2 spins is built, sampled and accepted against.
    Reports the step time (HIP events), the acceptance, accepted block spin-updates/s, the
    Nishimori-line check of the torus energy, [<E>] = -2 L^2 (1 - 2p), over the timed steps after
    the first, and the step-to-step autocorrelation of the torus energy."""
    import numpy as np
    import torch
    import synth
    from paper_2409_06538_amd import binding
    dev = torch.device("cuda:0")
    beta = binding.nishimori_beta(p)
    P = binding.PBC(L, n, [beta] * n, list(range(n)), chi, precision, K=K, device=dev)
    W = synth.words_per_row(L)
    init = synth.random_spins(seed + 77, n, L)
    for i in range(n):
        Jh_t, Jv_t = synth.torus_couplings(seed + i, L, p)
        P.set_torus(i, synth.pack_rows(Jh_t), synth.pack_rows(Jv_t), synth.pack_rows(init[i]))
    lines = [synth.frozen_lines(seed + 1000 + t, n, L) for t in range(steps + 2)]
    # two untimed steps start the chains from proposals (a random configuration can hold an
    # independence chain where q underrates it), covering all but the lines' crossings
    for t in range(2):
        progress(f"pbc L={L} chi={chi} {precision}: starting step {t}")
        P.step(lines[t], K, seed, first_proposal=K * t, first_step=K * t, init=True)
    ms, acc, Es = [], [], []
    for t in range(2, steps + 2):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        a, _ = P.step(lines[t], K, seed, first_proposal=K * t, first_step=K * t)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
        acc.append(a.float().sum().item())
        Es.append(P.E.cpu().numpy().astype(np.float64))
        progress(f"pbc L={L} step {t}: {ms[-1]:.1f} ms, accepted {acc[-1]:.0f}")
    st, _ = P.batch.status_check()
    E = np.array(Es[1:]).mean(axis=0)            # per-torus mean over the timed steps after the first
    # successive steps share the frozen lines' spins (and the rest of the previous state, when a
    # step's chain rejects everything): the correlation of the torus energy from step to step
    rho, tau = step_autocorrelation(np.array(Es[1:]))
    step_ms = float(np.mean(ms))
    return {"sweep": "pbc", "L": L, "block": L - 1, "chi": chi, "p": p, "precision": precision,
            "tori": n, "proposals": K, "steps": steps, "ms_per_step": step_ms,
            "acceptance": float(np.sum(acc)) / (n * K * steps),
            "accepted_spin_updates_per_s": float(np.mean(acc)) * (L - 1) ** 2 / (step_ms * 1e-3),
            "E_mean": float(E.mean()), "E_err": float(E.std(ddof=1) / np.sqrt(n)),
            "E_nishimori": -2 * L * L * (1 - 2 * p),
            "E_step_autocorrelation": rho, "E_tau_int_steps": tau, "status": st}


def run_observables(args, L, chi, p, n_real, K, n_chain=2):
    """f1: the sampled quantities of Sec. III C through the GPU chains, disorder-averaged on the
    GPU (Q_q, chi_q, chi_edge), with the Nishimori-line check [<E>] = -N_B (1 - 2p)."""
    import numpy as np
    import torch
    from paper_2409_06538_amd import binding
    dev = torch.device("cuda:0")
    beta = binding.nishimori_beta(p)
    seeds = list(range(n_real))
    b = binding.Batch([L] * n_real, [beta] * n_real, seeds, chi, args.precision, K=K, device=dev)
    b.make_couplings(seeds, p)
    t0 = time.perf_counter()
    b.build_env(want_lnZ=False)
    prop = b.propose(K, args.seed)
    chains = b.new_chains(n_chain)
    accum = torch.zeros((n_real, binding.OBS_COUNT), dtype=torch.float64, device=dev)
    acc, _ = b.accept(prop, chains, seed=args.seed, accum=accum)
    avg = dict(zip(binding.AVG_NAMES, b.disorder_average(accum, n_chain).cpu().numpy().tolist()))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    a = accum.cpu().numpy()
    e_i = a[:, 1] / a[:, 0]
    nb = 2 * L * (L - 1)
    return {"sweep": "observables", "L": L, "chi": chi, "p": p, "T": 1.0 / beta,
            "precision": args.precision, "realizations": n_real, "chains": n_chain,
            "proposals": K, "acceptance": acc.float().sum().item() / (n_real * (K - n_chain)),
            **avg, "E_err": float(e_i.std(ddof=1) / np.sqrt(n_real)),
            "E_nishimori": -nb * (1 - 2 * p), "wall_s": wall}


def run_sweep(args):
    """Acceptance and cost (the quantities of the paper's acceptance-ratio and cost figures,
    Sec. III B), one serial step per point after one warm-up, one JSON line per point: p_a,
    build and proposal times, the time per valid (accepted) sample per realization, and the
    accepted spin-updates/s of the batch.
      acceptance_cost  L in 16..256 and chi in 8..48; 16 realizations at p = 0.109, 256 proposals
      nishimori        p_a against the temperature along the Nishimori line (p and beta_N(p)),
                       L in 64..256, chi = 16 and 32; 16 realizations, 256 proposals
      large_L          L = 512 and 1024 at chi = 16 and 32; 4 realizations, 64 proposals
      observables      Q_q, chi_q, chi_edge (Sec. III C) at the multicritical point p = 0.10926,
                       L = 8 .. 64, chi = 32, 128 realizations, two chains of 256 steps
      forms            canonical compression against the zip-up on the same batches (Sec. II B
                       variants): build time, kept bonds, ln Z, acceptance
      pbc              periodic lattices by a frozen line pair per step (Sec. IV): step time,
                       acceptance, accepted spin-updates/s and the Nishimori check of the torus
                       energy"""
    if args.sweep == "acceptance_cost":
        for chi in SWEEP_CHIS:
            for L in SWEEP_LS:
                sweep_point(args, L, chi, 0.109, 16, 256, args.sweep)
    elif args.sweep == "nishimori":
        for chi in (16, 32):
            for L in SWEEP_NISHIMORI_LS:
                for p in SWEEP_NISHIMORI_PS:
                    sweep_point(args, L, chi, p, 16, 256, args.sweep)
    elif args.sweep == "large_L":
        for chi in (16, 32):
            for L in SWEEP_LARGE_LS:
                sweep_point(args, L, chi, 0.109, 4, 64, args.sweep)
    elif args.sweep == "observables":
        for L in SWEEP_OBS_LS:
            print(json.dumps(run_observables(args, L, 32, 0.10926, 128, 512)), flush=True)
    elif args.sweep == "forms":
        for L, chi, prec, n_real, K in SWEEP_FORMS:
            print(json.dumps(sweep_forms_point(L, chi, prec, n_real, K, seed=args.seed)),
                  flush=True)
    elif args.sweep == "pbc":
        for L, chi, prec, n, K, steps in SWEEP_PBC:
            print(json.dumps(sweep_pbc_point(L, chi, prec, n, K, steps, seed=args.seed)),
                  flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=0,
                    help="timed steps (default: 2 for rbim256, whose steps take seconds; 50 for "
                         "rbim64 and rbim16, whose steps take milliseconds, so that the pipeline "
                         "fill and drain inside the timed region are amortised; 4 for mixed; 9 "
                         "(three build groups) for rbim1024)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--precision", default=None, choices=["fp32", "fp64", "bf16"],
                    help="environment precision (default: the workload's)")
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
    ap.add_argument("--group-steps", type=int, default=0,
                    help="overlapped steps: build the batches of this many consecutive stages in "
                         "one launch while the proposals of the previous group run (default: 3 "
                         "for rbim1024, whose two realizations leave the chip idle during a "
                         "build; 1 elsewhere: one build per stage with --builds-in-flight)")
    ap.add_argument("--builds-in-flight", type=int, default=2, choices=[1, 2],
                    help="overlapped steps: environment builds of later steps running at once")
    ap.add_argument("--sweep", default=None,
                    choices=["acceptance_cost", "nishimori", "large_L", "observables", "forms",
                             "pbc"],
                    help="one JSON line per point instead of the benchmark line: acceptance and "
                         "cost against L and chi; against the temperature along the Nishimori "
                         "line; at L = 512 and 1024; or the disorder-averaged Binder ratio and "
                         "susceptibilities at the multicritical point")
    ap.add_argument("--graph", action="store_true",
                    help="capture the whole step in one HIP graph and time its replays (phase "
                         "times then come from the eager warm-up steps)")
    ap.add_argument("--autotune", type=int, default=1, choices=[0, 1],
                    help="time every launch shape of the proposal kernel on the built batch "
                         "before the timed steps and keep the fastest (0: library default)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the run, copy one buffer of this many MiB once (a plain copy "
                         "kernel of known size, the reference for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the realizations of a "
              "batch are independent, so N GPUs would each run their own share; this "
              "benchmark measures one GPU's share.", file=sys.stderr)
        sys.exit(2)
    import synth
    wl = synth.WORKLOADS[args.workload]
    if args.precision is None:
        args.precision = wl.get("precision", "fp32")
    if not args.steps:
        args.steps = DEFAULT_STEPS.get(args.workload, 20)
    if args.sweep:
        run_sweep(args)
        return
    multi_p = len(disorder_strengths(wl)) > 1
    ps = disorder_strengths(wl)
    p_cpu = ps[len(ps) // 2]
    K_full = args.proposals or wl["proposals"]
    # the oracle on all host cores first, while no process has touched the GPU (forked workers)
    cpu_all = None
    if not args.no_cpu and "L" in wl:
        cpu_all = run_cpu_all_cores(wl["L"], wl["chi"], p_cpu, K_full, args.seed)
        progress("oracle on all host cores done")
    serial = args.serial or args.graph
    if not args.group_steps:
        args.group_steps = DEFAULT_GROUP_STEPS.get(args.workload, 1)
    res = run_gpu(args) if serial else (run_gpu_grouped(args) if args.group_steps > 1
                                        else run_gpu_pipelined(args))
    if not serial and not args.no_serial:
        # the same steps one after the other on one stream, for comparison
        import copy
        a2 = copy.copy(args)
        a2.steps, a2.warmup = (1, 0) if (multi_p or max(workload_sizes(wl)[0]) > 256) else (3, 1)
        a2.autotune = 0          # the tuning table already holds this batch shape
        r2 = run_gpu(a2)
        progress("serial comparison done")
        res["serial"] = {"value": r2["value"], "ms_per_step": r2["ms_per_step"], "steps": a2.steps,
                         "build_ms": r2["build_ms"], "propose_ms": r2["propose_ms"],
                         "acceptance": r2["acceptance"]}
    if args.calib_copy_mib:
        calib_copy(args.calib_copy_mib)
    uniform = len(res["Ls"]) == 1
    L0 = res["Ls"][0]
    # the FP64 plain form and the CPU oracle are measured on uniform-L workloads (the FP64 plain
    # form at the largest chi that FP64 environments are built for, up to the workload's)
    from paper_2409_06538_amd import binding
    chi_plain = max(c for c in (2, 4, 8, 16, 32, 48, 64)
                    if c <= res["chi"] and binding.load().tnmc_chi_supported(c, binding.FP64))
    plain = None if args.no_plain or not uniform else \
        run_fp64_plain(args, L0, chi_plain, p_cpu, res["K"])
    if plain is not None:
        progress("FP64 plain form done")
    if plain is not None and chi_plain != res["chi"]:
        plain["chi"] = chi_plain
        plain["note"] = (f"FP64 environments are built up to chi = {chi_plain}: the FP64 plain form "
                         f"runs the same lattice at chi = {chi_plain}")
    cpu = None if args.no_cpu or not uniform else \
        run_cpu_baseline(L0, res["chi"], p_cpu, res["K"], args.seed)
    if cpu is not None:
        cpu["all_cores"] = cpu_all
        cpu["cores_available"] = len(os.sched_getaffinity(0))
    size = f"{L0}x{L0}" if uniform else "L x L (L in " + ", ".join(map(str, res["Ls"])) + ")"
    bar = build_arithmetic(args.precision, res["chi"])
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
        "dtype": sampler_arithmetic(args.precision),
        "arithmetic": {"storage": {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}[args.precision],
                       "build": bar, "sampler": sampler_arithmetic(args.precision),
                       "lognorm_logq_delta": "f64", "energy": "int"},
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {res['n']} realizations of the {size} open "
                               + (f"+-J lattice for each p in {tuple(res['p'])} (the same coupling "
                                  f"seeds, one batch per p), Nishimori beta, chi={res['chi']}, "
                                  if multi_p else
                                  f"+-J lattice, p={res['p']}, Nishimori beta, chi={res['chi']}, ")
                               + f"{res['K']} proposals each per step, {args.precision} "
                               "environments, batched"
                               + (", one HIP graph per step (its replays repeat one batch of "
                                  "proposals from restarted chains)" if res["graph"] else
                                  "; every step draws new proposals and continues the chains")
                               + ((f", consecutive steps overlapped (the batches of "
                                   f"{res['group_steps']} consecutive steps built by one launch "
                                   f"while the proposals of the previous group run)"
                                   if res.get("group_steps") else
                                   f", consecutive steps overlapped (builds of the next "
                                   f"{res.get('builds_in_flight')} stage(s) during the proposals "
                                   f"of the current one)") if res.get("pipelined") else ""),
                   "L": L0 if uniform else res["Ls"], "chi": res["chi"], "realizations": res["n"],
                   "proposals": res["K"], "p": res["p"], "precision": args.precision,
                   "graph": res["graph"], "pipelined": bool(res.get("pipelined")),
                   "builds_in_flight": res.get("builds_in_flight"),
                   "group_steps": res.get("group_steps"),
                   "propose_cu_mask": res.get("propose_cu_mask")},
        "acceptance": res["acceptance"],
        "acceptance_per_p": res.get("acceptance_per_p"),
        "accepted": res["accepted"],
        "attempted": res["attempted"],
        "build_ms": res["build_ms"],
        "propose_ms": res["propose_ms"],
        "serial": res.get("serial"),
        "autotune": res.get("autotune"),
        "fp64_plain": plain,
        "error_vs_oracle": res.get("error_vs_oracle"),
        "roofline": res["roofline"],
        "roofline_propose": res["roofline_propose"],
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
