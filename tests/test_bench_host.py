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
    assert r["bound"] == "alu" and r["peak"] == bench.FP32_VECTOR_PEAK_TFLOPS
    assert abs(r["achieved"] - 270 * 32 ** 3 * 63 * 64 * 64 / 0.1 / 1e12) < 1e-9
    p = out["roofline_propose"]
    assert p["bound"] == "hbm" and p["peak"] == bench.HBM_PEAK_GBS
    # V round trip at 16 rows (narrow half) and 32 rows, plus 8 workgroups streaming the sites twice
    v = 2.0 * 64 * 64 * 2 * (16 * 0.5 + 32 * 0.5) * 1024 * 4 * 64
    e = 2.0 * 64 * 64 * 2 * 32 * 32 * 4 * 8 * 64
    assert abs(p["algorithmic_bytes_per_launch"] - (v + e)) < 1.0
    assert bench.proposals_per_wg("fp32", 64, 1000, 64) == 128
    assert bench.proposals_per_wg("bf16", 64, 1000, 64) == 128
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
    r = bench.run_cpu_all_cores(8, 4, 0.109, 100, 0, n_prop=10, max_workers=2)
    assert r["kind"] == "oracle" and r["unit"] == "spin-updates/s"
    assert 1 <= r["cores"] <= 2 and r["value"] > 0
