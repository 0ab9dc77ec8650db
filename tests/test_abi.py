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


def test_short_workspace_is_enomem_on_every_entry_point(lib):
    """Every entry point that takes the workspace checks its size on the host and returns
    TNMC_ENOMEM before anything is enqueued (the pointers here are never dereferenced)."""
    from paper_2409_06538_amd import binding
    tab = (binding.Instance * 2)()
    fake = ctypes.c_void_p(1 << 20)
    for i, L in enumerate((16, 40)):
        tab[i].L, tab[i].beta, tab[i].id = L, 0.9, i
        tab[i].d_Jh = tab[i].d_Jv = tab[i].d_env = tab[i].d_lognorm = 1 << 20
    seeds = (ctypes.c_uint64 * 2)(0, 1)
    tori, btab = _tori(binding, (17, 41))
    short = 8
    enomem = -2
    calls = {
        "tnmc_make_couplings": lambda: lib.tnmc_make_couplings(
            tab, 2, ctypes.cast(seeds, ctypes.c_void_p), 0.1, fake, short, None),
        "tnmc_build_env": lambda: lib.tnmc_build_env(tab, 2, 16, binding.FP32, fake, short, None,
                                                     None),
        "tnmc_build_env_form": lambda: lib.tnmc_build_env_form(tab, 2, 16, binding.FP32, 1, fake,
                                                               short, None, None),
        "tnmc_propose": lambda: lib.tnmc_propose(tab, 2, 16, binding.FP32, 8, 0, 0, fake, short,
                                                 fake, fake, fake, None, None),
        "tnmc_logq": lambda: lib.tnmc_logq(tab, 2, 16, binding.FP32, 8, fake, fake, short, fake,
                                           None),
        "tnmc_autotune_propose": lambda: lib.tnmc_autotune_propose(
            tab, 2, 16, binding.FP32, 8, 0, fake, short, fake, fake, fake, 1, None, None, None),
        "tnmc_energy": lambda: lib.tnmc_energy(tab, 2, 8, fake, fake, fake, short, None),
        "tnmc_accept": lambda: lib.tnmc_accept(tab, 2, 1, 8, fake, fake, fake, 0, 0, fake, fake,
                                               fake, fake, fake, fake, None, fake, short, None),
        "tnmc_observables": lambda: lib.tnmc_observables(tab, 2, 1, fake, fake, fake, fake, short,
                                                         None),
        "tnmc_pbc_block": lambda: lib.tnmc_pbc_block(tori, btab, 2, fake, fake, short, None),
        "tnmc_pbc_merge": lambda: lib.tnmc_pbc_merge(tori, btab, 2, fake, None, fake, short, None),
    }
    takes_workspace = [n for n in declared_symbols()
                       if "workspace_bytes" in header_signature(n) and n != "tnmc_workspace_bytes"]
    assert sorted(calls) == sorted(takes_workspace)
    for name, call in calls.items():
        assert call() == enomem, name


def _tori(binding, Ls):
    """Torus descriptors and their block instances with placeholder device pointers (never
    dereferenced: every call below returns before anything is enqueued)."""
    tori = (binding.TorusDesc * len(Ls))()
    btab = (binding.Instance * len(Ls))()
    for i, L in enumerate(Ls):
        tori[i].L, tori[i].r0, tori[i].c0 = L, i, L - 1
        tori[i].d_Jh = tori[i].d_Jv = tori[i].d_spins = 1 << 20
        btab[i].L, btab[i].beta, btab[i].id = L - 1, 0.9, i
        btab[i].d_Jh = btab[i].d_Jv = btab[i].d_field = 1 << 20
    return tori, btab


def test_pbc_arguments_host_side(lib):
    """tnmc_pbc_block / tnmc_pbc_merge reject, on the host, a block whose side is not L - 1,
    frozen lines outside the torus, L < 3 and a block without a field buffer."""
    from paper_2409_06538_amd import binding
    fake = ctypes.c_void_p(1 << 20)
    nb = lib.tnmc_pbc_workspace_bytes(2)
    assert nb > 0 and lib.tnmc_pbc_workspace_bytes(0) == 0
    cases = []
    tori, btab = _tori(binding, (9, 12))
    btab[1].L = 12
    cases.append((tori, btab))
    tori, btab = _tori(binding, (9, 12))
    tori[0].r0 = 9
    cases.append((tori, btab))
    tori, btab = _tori(binding, (9, 12))
    tori[1].c0 = -1
    cases.append((tori, btab))
    tori, btab = _tori(binding, (2, 12))
    cases.append((tori, btab))
    for tori, btab in cases:
        assert lib.tnmc_pbc_block(tori, btab, 2, fake, fake, nb, None) == -1
        assert lib.tnmc_pbc_merge(tori, btab, 2, fake, None, fake, nb, None) == -1
    tori, btab = _tori(binding, (9, 12))
    btab[0].d_field = None
    assert lib.tnmc_pbc_block(tori, btab, 2, fake, fake, nb, None) == -1


def header_signature(name):
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    m = re.search(r"\b" + name + r"\s*\((.*?)\);", text, flags=re.S)
    return m.group(1) if m else ""


def test_status_bits_match_header():
    from paper_2409_06538_amd import binding
    text = open(HEADER).read()
    bits = dict(re.findall(r"#define (TNMC_ST_[A-Z]+) (0x[0-9a-f]+)u", text))
    assert int(bits["TNMC_ST_LOGNORM"], 16) == binding.ST_LOGNORM
    assert int(bits["TNMC_ST_WEIGHT"], 16) == binding.ST_WEIGHT
    assert int(bits["TNMC_ST_LOGQ"], 16) == binding.ST_LOGQ
    assert int(bits["TNMC_ST_DELTA"], 16) == binding.ST_DELTA
    assert int(bits["TNMC_ST_FALLBACK"], 16) == binding.ST_FALLBACK
    assert "tnmc_status_check" in declared_symbols()


def test_tuning_table_host_side(lib):
    """The proposal kernel's launch-shape table: candidates per chi, set / get / erase (host
    only)."""
    from paper_2409_06538_amd import binding
    buf = (ctypes.c_int32 * 4)()
    assert lib.tnmc_propose_candidates(32, ctypes.cast(buf, ctypes.c_void_p)) == 4
    assert list(buf) == [1, 2, 4, 8]
    assert lib.tnmc_propose_candidates(8, ctypes.cast(buf, ctypes.c_void_p)) == 1
    assert lib.tnmc_tune_get(32, binding.FP32, 64, 64, 1000) == 8      # default: 8 for L <= 64
    assert lib.tnmc_tune_get(48, binding.BF16, 256, 128, 1000) == 4
    assert lib.tnmc_tune_set(32, binding.FP32, 64, 64, 1000, 2) == 0
    assert lib.tnmc_tune_get(32, binding.FP32, 64, 64, 1000) == 2
    assert lib.tnmc_tune_set(32, binding.FP32, 64, 64, 1000, 3) == -1  # not a candidate
    assert lib.tnmc_tune_set(8, binding.FP32, 64, 64, 1000, 2) == -1   # one thread per proposal
    assert lib.tnmc_tune_set(32, binding.FP32, 64, 64, 1000, 0) == 0   # erase
    assert lib.tnmc_tune_get(32, binding.FP32, 64, 64, 1000) == 8


def test_build_forms_host_side(lib):
    """The build forms of the header match the binding; a form that does not exist, or one not
    built for the precision, is TNMC_EINVAL before anything is enqueued."""
    from paper_2409_06538_amd import binding
    text = open(HEADER).read()
    forms = dict(re.findall(r"#define (TNMC_FORM_[A-Z0-9_]+) (\d+)", text))
    assert int(forms["TNMC_FORM_DEFAULT"]) == binding.FORM_DEFAULT
    assert int(forms["TNMC_FORM_GRAM_L2"]) == binding.FORM_GRAM_L2
    assert int(forms["TNMC_FORM_ZIPUP"]) == binding.FORM_ZIPUP
    tab = (binding.Instance * 1)()
    tab[0].L, tab[0].beta, tab[0].id = 16, 0.9, 0
    tab[0].d_Jh = tab[0].d_Jv = tab[0].d_env = tab[0].d_lognorm = 1 << 20
    fake = ctypes.c_void_p(1 << 20)
    big = 1 << 40
    for form, prec, chi in ((3, binding.FP32, 16), (-1, binding.FP32, 16),
                            (binding.FORM_ZIPUP, binding.FP64, 16),
                            (binding.FORM_GRAM_L2, binding.FP64, 16),
                            (binding.FORM_ZIPUP, binding.FP32, 4)):
        assert lib.tnmc_build_env_form(tab, 1, chi, prec, form, fake, big, None, None) == -1, \
            (form, prec, chi)
