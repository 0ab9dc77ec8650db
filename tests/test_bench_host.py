"""Host logic of bench.py: workload sizes and the CU mask that keeps CUs free for the build."""
from collections import Counter

import bench
import synth


def test_reserved_cu_bits_spread_under_each_layout():
    words = 8                                  # 256 CUs
    bits = [32 * w + b for w in range(words) for b in bench.reserved_cu_bits(w)]
    assert len(bits) == len(set(bits)) == 64
    # CUs enumerated XCD by XCD (32 each), shader engines by byte or interleaved mod 4
    assert Counter(i // 32 for i in bits) == Counter({x: 8 for x in range(8)})
    assert set(Counter((i // 32, (i % 32) // 8) for i in bits).values()) == {2}
    assert set(Counter((i // 32, (i % 32) % 4) for i in bits).values()) == {2}
    # CUs interleaved across the 8 XCDs, shader engines by byte of the per-XCD index
    assert Counter(i % 8 for i in bits) == Counter({x: 8 for x in range(8)})
    assert set(Counter((i % 8, (i // 8) % 4) for i in bits).values()) == {2}


def test_workload_sizes():
    Ls, seeds = bench.workload_sizes(synth.WORKLOADS["mixed"])
    assert len(Ls) == len(seeds) == 256
    assert Ls[:5] == [32, 64, 128, 256, 32]
    Ls, seeds = bench.workload_sizes(synth.WORKLOADS["rbim64"])
    assert Ls == [64] * 64 and seeds == list(range(64))


def test_reserved_cu_bits_two_sets():
    """With two builds in flight, 16 CUs of every XCD are kept free, 4 in each shader engine."""
    bits = [32 * w + b for w in range(8) for b in bench.reserved_cu_bits(w, 2)]
    assert len(bits) == len(set(bits)) == 128
    assert Counter(i // 32 for i in bits) == Counter({x: 16 for x in range(8)})
    assert set(Counter((i // 32, (i % 32) // 8) for i in bits).values()) == {4}
    assert set(Counter((i // 32, (i % 32) % 4) for i in bits).values()) == {4}
    assert Counter(i % 8 for i in bits) == Counter({x: 16 for x in range(8)})
    assert set(Counter((i % 8, (i // 8) % 4) for i in bits).values()) == {4}


def test_rooflines_from_launch_times():
    """The bench line's roofline objects from launch times alone (no GPU)."""
    import argparse
    args = argparse.Namespace(precision="fp32", workload="rbim64")
    res = {"chi": 32, "K": 1000, "build_ms": 100.0, "propose_ms": 50.0, "narrow_fraction": 0.5}
    out = bench.add_rooflines(res, args, [64] * 64)
    r = out["roofline"]
    # the chi = 32 build of FP32 environments computes in FP64 (Gram form): FP64 peak
    assert r["bound"] == "mfma" and r["arithmetic"] == "f64" and r["peak"] == 78.6
    assert abs(r["achieved"] - 270 * 32 ** 3 * 63 * 64 * 64 / 0.1 / 1e12) < 1e-9
    p = out["roofline_propose"]
    # 2 passes x 2 chi^2 L^2 x 4 bytes per realization; 8 chi^2 L^2 flops per proposal: 500
    # flop/byte, past the FP32 ridge (157.3 / 8 = 19.7), so quoted against the FP32 peak
    assert abs(p["algorithmic_bytes_per_launch"] - 2 * 2 * 32 * 32 * 64 * 64 * 4 * 64) < 1.0
    assert abs(p["algorithmic_flops_per_launch"] - 8 * 32 * 32 * 64 * 64 * 1000 * 64) < 1.0
    assert p["bound"] == "mfma" and p["peak"] == 157.3 and p["unit"] == "TFLOP/s"
    assert abs(p["intensity_flop_per_byte"] - 500.0) < 1e-9
    # chi = 48 builds in FP32 (QR form); FP64 environments in FP64
    args48 = argparse.Namespace(precision="bf16", workload="rbim256")
    r48 = bench.add_rooflines(dict(res, chi=48), args48, [256] * 4)["roofline"]
    assert r48["arithmetic"] == "f32" and r48["peak"] == 157.3
    assert bench.build_arithmetic("fp64", 16) == "f64"
    # a single proposal per realization is HBM-bound
    r1 = bench.add_rooflines(dict(res, K=1), args, [64] * 64)["roofline_propose"]
    assert r1["bound"] == "hbm" and r1["peak"] == bench.HBM_PEAK_GBS
    assert bench.proposals_per_wg("fp32", 64, 1000, 64) == 128
    assert bench.proposals_per_wg("fp32", 256, 1000, 256) == 64


def test_disorder_strengths():
    """The L = 256 workload runs three disorder strengths on the same coupling seeds; the others
    one."""
    assert bench.disorder_strengths(synth.WORKLOADS["rbim256"]) == [0.10, 0.109, 0.12]
    assert bench.disorder_strengths(synth.WORKLOADS["rbim64"]) == [0.109]
    Ls, seeds = bench.workload_sizes(synth.WORKLOADS["rbim256"])
    assert Ls == [256] * 128 and seeds == list(range(128))


def test_cpu_all_cores_baseline_shape():
    """The all-core oracle baseline: one forked process per core, a bounded sample each."""
    r = bench.run_cpu_all_cores(8, 4, 0.109, 100, 0, max_workers=2)
    assert r["kind"] == "oracle" and r["unit"] == "spin-updates/s"
    assert 1 <= r["cores"] <= 2 and r["value"] > 0
    assert r["cores_available"] >= r["cores"]


def test_cpu_sliced_sample_shape():
    """The bounded oracle sample for lattices whose full oracle build takes minutes: a few rows
    of the build, proposals timed on environments that repeat the last built row."""
    out = bench._oracle_realization((24, 4, 0.109, 0, 0, 2, (2, 4)))
    t_build, t_prop, acc, work = out
    assert t_build > 0 and t_prop > 0 and acc is None and work > 0
    assert bench.cpu_sample_plan(64)[0] is None and bench.cpu_sample_plan(256)[0] == (8, 16)
