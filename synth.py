"""Seeded synthetic inputs and the workload table, shared by the tests and the benchmark.

This module holds none of the method's arithmetic: only sizes, seeds, seeded random arrays drawn
with numpy's default generator, and the bit-packing layout of spin configurations.  Couplings and
every random draw of the method itself come from Philox on each side independently (the oracle
in Python, the HIP path on the device), keyed by the seeds listed here.

The paper's own workload is synthetic (i.i.d. +-J instances, Sec. III A): there is no external
dataset.  Workloads (open L x L lattices, beta on the Nishimori line):
  rbim16    L=16,  p=0.109, chi=16, 1 realization (coupling seed 0), 200 proposals, FP64
  rbim64    L=64,  p=0.109, chi=32, 64 realizations (seeds 0..63), 1000 proposals each
  rbim256   L=256, p in {0.10, 0.109, 0.12}, chi=48, 128 realizations, 1000 proposals, BF16
  mixed     256 realizations with L = (32, 64, 128, 256)[i mod 4], seed i, p=0.109, chi=32, FP32
  rbim1024  L=1024, p=0.109, chi=64, 2 realizations (seeds 0, 1), FP32 and BF16
Periodic lattices (the frozen-line-pair steps) take their couplings and the lines of each step
from torus_couplings and frozen_lines.
"""
import numpy as np

WORKLOADS = {
    "rbim16": dict(L=16, p=0.109, chi=16, seeds=(0,), proposals=200, philox_seed=0,
                   precision="fp64"),
    "rbim64": dict(L=64, p=0.109, chi=32, seeds=tuple(range(64)), proposals=1000, philox_seed=0,
                   precision="fp32"),
    "rbim256": dict(L=256, ps=(0.10, 0.109, 0.12), chi=48, seeds=tuple(range(128)),
                    proposals=1000, philox_seed=0, precision="bf16"),
    # the same lattices and disorder at chi = 32 (FP32 environments): the bond / precision trade-off
    "rbim256_chi32": dict(L=256, ps=(0.10, 0.109, 0.12), chi=32, seeds=tuple(range(128)),
                          proposals=1000, philox_seed=0, precision="fp32"),
    "mixed": dict(Ls=(32, 64, 128, 256), p=0.109, chi=32, seeds=tuple(range(256)),
                  proposals=1000, philox_seed=0, precision="fp32"),
    "rbim1024": dict(L=1024, p=0.109, chi=64, seeds=(0, 1), proposals=1000, philox_seed=0,
                     precision="bf16"),
}


def random_spins(seed, K, Lr, Lc=None):
    """K random +-1 configurations (int8, shape (K, Lr, Lc)) from numpy's default generator."""
    Lc = Lr if Lc is None else Lc
    rng = np.random.default_rng(seed)
    return (1 - 2 * rng.integers(0, 2, size=(K, Lr, Lc))).astype(np.int8)


def random_pm1(seed, shape):
    """Random +-1 int8 array of the given shape."""
    rng = np.random.default_rng(seed)
    return (1 - 2 * rng.integers(0, 2, size=shape)).astype(np.int8)


def torus_couplings(seed, L, p):
    """+-1 couplings of an L x L torus with P(J = -1) = p, from numpy's default generator:
    (Jh_t, Jv_t), int8 (L, L); Jh_t[r, c] is the bond (r, c)-(r, (c+1) mod L), Jv_t[r, c] the bond
    (r, c)-((r+1) mod L, c)."""
    rng = np.random.default_rng(seed)
    Jh = np.where(rng.random((L, L)) < p, -1, 1).astype(np.int8)
    Jv = np.where(rng.random((L, L)) < p, -1, 1).astype(np.int8)
    return Jh, Jv


def frozen_lines(seed, steps, L):
    """(steps, 2) int32 array of (row, column) pairs, uniform on [0, L), one pair per step."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, L, size=(steps, 2)).astype(np.int32)


def words_per_row(L):
    return (L + 63) // 64


def pack_rows(pm1):
    """Bit-pack +-1 values along the last axis: bit j of word j//64 is 1 iff the value is -1.

    (..., n) int8 -> (..., ceil(n/64)) uint64, padding bits 0.
    """
    pm1 = np.asarray(pm1)
    n = pm1.shape[-1]
    W = words_per_row(n)
    bits = np.zeros(pm1.shape[:-1] + (W * 64,), dtype=np.uint64)
    bits[..., :n] = (pm1 < 0).astype(np.uint64)
    bits = bits.reshape(pm1.shape[:-1] + (W, 64))
    shifts = np.arange(64, dtype=np.uint64)
    return np.bitwise_or.reduce(bits << shifts, axis=-1)


def unpack_rows(words, n):
    """Inverse of pack_rows: (..., W) uint64 -> (..., n) int8 of +-1."""
    words = np.asarray(words, dtype=np.uint64)
    shifts = np.arange(64, dtype=np.uint64)
    bits = (words[..., None] >> shifts) & np.uint64(1)
    bits = bits.reshape(words.shape[:-1] + (-1,))[..., :n]
    return (1 - 2 * bits.astype(np.int64)).astype(np.int8)
