"""The C-ABI library loads and exports every entry point include/tnmc.h declares; host-side size
queries and argument validation work without a GPU (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tnmc.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tnmc_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2409_06538_amd import binding
    return binding.load()


def test_header_declares_the_hot_path():
    names = declared_symbols()
    for required in ("tnmc_build_env", "tnmc_propose", "tnmc_accept", "tnmc_observables"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2409_06538_amd import binding
    names = declared_symbols()
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(binding.exported_symbols()) == names


def test_size_queries(lib):
    from paper_2409_06538_amd import binding
    assert lib.tnmc_env_bytes(64, 32, binding.FP32) == 64 * 64 * 2 * 32 * 32 * 4
    assert lib.tnmc_env_bytes(16, 16, binding.FP64) == 16 * 16 * 2 * 16 * 16 * 8
    assert lib.tnmc_env_bytes(1, 16, binding.FP64) == 0
    assert lib.tnmc_env_bytes(16, 12, binding.FP64) == 0
    assert lib.tnmc_chi_supported(32, binding.FP32) == 1
    assert lib.tnmc_chi_supported(33, binding.FP32) == 0
    tab = (binding.Instance * 2)()
    for i, L in enumerate((16, 64)):
        tab[i].L, tab[i].beta = L, 1.0
    ws = lib.tnmc_workspace_bytes(tab, 2, 16, 100, binding.FP64)
    assert ws >= 64 * 4 * 16 * 2 * 16 * 8          # Q scratch of the L=64 build
    assert ws >= 64 * 2 * 16 * 100 * 8              # proposal scratch
    tab[1].L = 2000
    assert lib.tnmc_workspace_bytes(tab, 2, 16, 100, binding.FP64) == 0


def test_host_validation_rejects_bad_arguments(lib):
    from paper_2409_06538_amd import binding
    tab = (binding.Instance * 1)()
    tab[0].L, tab[0].beta = 16, 1.0
    # null device pointers / workspace: rejected on the host before any HIP call
    st = lib.tnmc_build_env(tab, 1, 16, binding.FP64, None, 0, None, None)
    assert lib.tnmc_status_string(st).decode() == "invalid argument"
    tab[0].L = 1
    assert lib.tnmc_energy(tab, 1, 4, None, None, None, 0, None) == -1
    tab[0].L, tab[0].beta = 8, -1.0
    assert lib.tnmc_propose(tab, 1, 8, binding.FP32, 4, 0, 0, None, 0, None, None, None, None,
                            None) == -1
    tab[0].beta = 1.0
    # K not a multiple of the number of chains
    dummy = ctypes.c_void_p(16)
    assert lib.tnmc_accept(tab, 1, 3, 4, dummy, dummy, dummy, 0, 0, dummy, dummy, dummy, dummy,
                           dummy, dummy, None, dummy, 1 << 20, None) == -1
    assert lib.tnmc_status_string(-2).decode() == "workspace too small"
