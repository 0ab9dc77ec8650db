"""Thin Python binding of the C ABI in include/tnmc.h (ctypes; argument marshalling only).

Every step of the hot path runs in the HIP kernels of ``libtnmc.so``; torch only allocates
device memory and supplies the stream.  There is no CPU fallback: ``load()`` raises if the
library has not been built (``python -m paper_2409_06538_amd.build``) or no GPU is visible.

Names follow the C entry points: ``make_couplings``, ``build_env``, ``propose``, ``logq``,
``energy``, ``accept``, ``observables``.
"""
import ctypes
import math
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtnmc.so")

FP64, FP32, BF16 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": BF16}
# storage dtype of the environments per precision
ENV_DTYPES = {FP64: torch.float64, FP32: torch.float32, BF16: torch.bfloat16}
OBS_COUNT = 9
OBS_NAMES = ("count", "E", "E2", "m2", "m4", "medge2", "q", "q2", "q4")
# status word bits (include/tnmc.h)
ST_LOGNORM, ST_WEIGHT, ST_LOGQ, ST_DELTA, ST_FALLBACK = 0x1, 0x2, 0x4, 0x8, 0x10
ST_FAULTS = ST_LOGNORM | ST_WEIGHT | ST_LOGQ | ST_DELTA
ENUMERIC = -4
FORM_DEFAULT, FORM_GRAM_L2, FORM_ZIPUP = 0, 1, 2
AVG_COUNT = 12
AVG_NAMES = ("E", "E2", "m2", "m4", "medge2", "q", "q2", "q4", "q2sq", "Q_q", "chi_q", "chi_edge")

_lib = None


class Instance(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("pad_", ctypes.c_int32), ("beta", ctypes.c_double),
                ("id", ctypes.c_uint64), ("d_Jh", ctypes.c_void_p), ("d_Jv", ctypes.c_void_p),
                ("d_env", ctypes.c_void_p), ("d_lognorm", ctypes.c_void_p),
                ("d_status", ctypes.c_void_p), ("d_bonds", ctypes.c_void_p),
                ("d_field", ctypes.c_void_p)]


class TorusDesc(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("r0", ctypes.c_int32), ("c0", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("d_Jh", ctypes.c_void_p), ("d_Jv", ctypes.c_void_p),
                ("d_spins", ctypes.c_void_p)]


class TNMCError(RuntimeError):
    pass


def load():
    """Load libtnmc.so (once) and declare its signatures; raise if unavailable."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise TNMCError(f"{LIB_PATH} is missing: build it with "
                        "`python -m paper_2409_06538_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(Instance)
    vp, i32, u64, sz, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_size_t, ctypes.c_double
    sigs = {
        "tnmc_chi_supported": (ctypes.c_int, [i32, ctypes.c_int]),
        "tnmc_env_bytes": (sz, [i32, i32, ctypes.c_int]),
        "tnmc_workspace_bytes": (sz, [P, i32, i32, i32, ctypes.c_int]),
        "tnmc_make_couplings": (ctypes.c_int, [P, i32, vp, dbl, vp, sz, vp]),
        "tnmc_build_env": (ctypes.c_int, [P, i32, i32, ctypes.c_int, vp, sz, vp, vp]),
        "tnmc_build_env_static": (ctypes.c_int, [P, i32, i32, ctypes.c_int, vp, vp]),
        "tnmc_build_env_form": (ctypes.c_int, [P, i32, i32, ctypes.c_int, i32, vp, sz, vp, vp]),
        "tnmc_propose": (ctypes.c_int, [P, i32, i32, ctypes.c_int, i32, u64, u64, vp, sz, vp, vp,
                                        vp, vp, vp]),
        "tnmc_logq": (ctypes.c_int, [P, i32, i32, ctypes.c_int, i32, vp, vp, sz, vp, vp]),
        "tnmc_propose_candidates": (i32, [i32, vp]),
        "tnmc_tune_set": (ctypes.c_int, [i32, ctypes.c_int, i32, i32, i32, i32]),
        "tnmc_tune_get": (i32, [i32, ctypes.c_int, i32, i32, i32]),
        "tnmc_autotune_propose": (ctypes.c_int, [P, i32, i32, ctypes.c_int, i32, u64, vp, sz, vp,
                                                 vp, vp, i32, vp, vp, vp]),
        "tnmc_energy": (ctypes.c_int, [P, i32, i32, vp, vp, vp, sz, vp]),
        "tnmc_accept": (ctypes.c_int, [P, i32, i32, i32, vp, vp, vp, u64, u64, vp, vp, vp, vp, vp,
                                       vp, vp, vp, sz, vp]),
        "tnmc_observables": (ctypes.c_int, [P, i32, i32, vp, vp, vp, vp, sz, vp]),
        "tnmc_disorder_average": (ctypes.c_int, [vp, i32, i32, dbl, i32, vp, vp]),
        "tnmc_status_check": (ctypes.c_int, [P, i32, vp, vp]),
        "tnmc_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "tnmc_pbc_workspace_bytes": (sz, [i32]),
        "tnmc_pbc_block": (ctypes.c_int, [ctypes.POINTER(TorusDesc), P, i32, vp, vp, sz, vp]),
        "tnmc_pbc_merge": (ctypes.c_int, [ctypes.POINTER(TorusDesc), P, i32, vp, vp, vp, sz, vp]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    """Names of the C entry points this binding declares."""
    return ["tnmc_chi_supported", "tnmc_env_bytes", "tnmc_workspace_bytes", "tnmc_make_couplings",
            "tnmc_build_env", "tnmc_build_env_form", "tnmc_build_env_static", "tnmc_propose", "tnmc_propose_candidates", "tnmc_tune_set", "tnmc_tune_get",
            "tnmc_autotune_propose", "tnmc_logq", "tnmc_energy", "tnmc_accept",
            "tnmc_observables", "tnmc_disorder_average", "tnmc_status_check",
            "tnmc_status_string", "tnmc_pbc_workspace_bytes", "tnmc_pbc_block", "tnmc_pbc_merge"]


def _check(status, what):
    if status != 0:
        msg = _lib.tnmc_status_string(status).decode()
        raise TNMCError(f"{what} failed: {msg} ({status})")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def words_per_row(L):
    return (L + 63) // 64


def nishimori_beta(p):
    """Inverse temperature on the Nishimori line exp(-2 beta) = p / (1 - p) (J = 1)."""
    return 0.5 * math.log((1.0 - p) / p)


def group_table(batches):
    """One instance table over the realizations of several batches (same chi and precision),
    in order: the device buffers stay the batches' own."""
    tab = (Instance * sum(b.n for b in batches))()
    k = 0
    for b in batches:
        for i in range(b.n):
            tab[k] = b.table[i]
            k += 1
    return tab


def group_workspace_bytes(batches):
    """Workspace for tnmc_build_env over the realizations of several batches in one call."""
    b0 = batches[0]
    tab = group_table(batches)
    return int(load().tnmc_workspace_bytes(tab, len(tab), b0.chi, 1, b0.prec))


def build_env_group(batches, workspace):
    """tnmc_build_env over the realizations of several batches in one launch (each batch's
    environments, log-norms, bond tables and status words are written in place); `workspace` is
    a uint8 tensor of at least group_workspace_bytes(batches)."""
    b0 = batches[0]
    if any(b.chi != b0.chi or b.prec != b0.prec for b in batches):
        raise TNMCError("build_env_group: batches differ in chi or precision")
    tab = group_table(batches)
    _check(load().tnmc_build_env(tab, len(tab), b0.chi, b0.prec,
                                 ctypes.c_void_p(workspace.data_ptr()),
                                 ctypes.c_size_t(workspace.numel()), None, _stream()),
           "tnmc_build_env")


class Batch:
    """Device buffers for a batch of realizations plus the host instance table."""

    def __init__(self, Ls, betas, ids, chi, precision="fp32", K=1, device="cuda:0",
                 fields=False):
        lib = load()
        self.n = len(Ls)
        self.Ls = [int(L) for L in Ls]
        self.Lmax = max(self.Ls)
        self.Wmax = words_per_row(self.Lmax)
        self.chi = int(chi)
        self.prec = PRECISIONS[precision]
        self.precision = precision
        self.dtype = ENV_DTYPES[self.prec]
        self.device = torch.device(device)
        if not lib.tnmc_chi_supported(self.chi, self.prec):
            raise TNMCError(f"chi={chi} not supported for {precision}")
        self.Jh, self.Jv, self.env, self.lognorm, self.bonds = [], [], [], [], []
        self.field = []   # per-realization L x L int8 site fields (fields=True)
        self.table = (Instance * self.n)()
        # one numeric status word per realization (TNMC_ST_* bits)
        self.status = torch.zeros(self.n, dtype=torch.int32, device=self.device)
        for i, L in enumerate(self.Ls):
            W = words_per_row(L)
            jh = torch.zeros(L * W, dtype=torch.int64, device=self.device)
            jv = torch.zeros((L - 1) * W, dtype=torch.int64, device=self.device)
            nbytes = lib.tnmc_env_bytes(L, self.chi, self.prec)
            env = torch.zeros(nbytes // self.dtype.itemsize, dtype=self.dtype, device=self.device)
            lam = torch.zeros(L, dtype=torch.float64, device=self.device)
            self.Jh.append(jh)
            self.Jv.append(jv)
            self.env.append(env)
            self.lognorm.append(lam)
            bd = torch.zeros(L * (L + 1), dtype=torch.uint8, device=self.device)
            self.bonds.append(bd)
            t = self.table[i]
            t.L, t.pad_, t.beta, t.id = L, 0, float(betas[i]), int(ids[i])
            t.d_Jh, t.d_Jv = jh.data_ptr(), jv.data_ptr()
            t.d_env, t.d_lognorm = env.data_ptr(), lam.data_ptr()
            t.d_status = self.status.data_ptr() + 4 * i
            t.d_bonds = bd.data_ptr()
            if fields:
                fl = torch.zeros(L * L, dtype=torch.int8, device=self.device)
                self.field.append(fl)
                t.d_field = fl.data_ptr()
        self.K = 0
        self.workspace = None
        self.ensure_workspace(K)

    def set_field(self, i, h):
        """Copy an (L, L) integer field array (host) into realization i (fields=True)."""
        L = self.Ls[i]
        self.field[i].copy_(torch.as_tensor(h, dtype=torch.int8).reshape(L * L))

    def use_bonds(self, on=True):
        """Pass (or not) each realization's bond table: written by the build, read by the
        proposals to load only the nonzero block of each site."""
        for i in range(self.n):
            self.table[i].d_bonds = self.bonds[i].data_ptr() if on else None

    def bond_table(self, i):
        """Bond table of realization i as (L, L + 1)."""
        L = self.Ls[i]
        return self.bonds[i].view(L, L + 1)

    def set_betas(self, betas):
        """Change the inverse temperature of every realization (the table is passed by value
        on each call, so this takes effect from the next call on)."""
        for i in range(self.n):
            self.table[i].beta = float(betas[i])

    # -- workspace -------------------------------------------------------------------------
    def ensure_workspace(self, K):
        if K <= self.K and self.workspace is not None:
            return
        nbytes = load().tnmc_workspace_bytes(self.table, self.n, self.chi, int(K), self.prec)
        if nbytes == 0:
            raise TNMCError("tnmc_workspace_bytes rejected the batch")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.K = int(K)

    def _ws(self):
        return ctypes.c_void_p(self.workspace.data_ptr()), ctypes.c_size_t(self.workspace.numel())

    # -- entry points ----------------------------------------------------------------------
    def make_couplings(self, seeds, p):
        """tnmc_make_couplings: i.i.d. +-1 couplings with P(J=-1) = p from Philox."""
        seeds = (ctypes.c_uint64 * self.n)(*[int(s) for s in seeds])
        ws, nb = self._ws()
        _check(load().tnmc_make_couplings(self.table, self.n, ctypes.cast(seeds, ctypes.c_void_p),
                                          float(p), ws, nb, _stream()), "tnmc_make_couplings")

    def set_couplings(self, i, jh_words, jv_words):
        """Copy caller-packed coupling words (int64/uint64 arrays) into realization i."""
        self.Jh[i].copy_(torch.as_tensor(jh_words.view("int64")).reshape(-1))
        self.Jv[i].copy_(torch.as_tensor(jv_words.view("int64")).reshape(-1))

    def build_env(self, want_lnZ=True):
        """tnmc_build_env: environments, log-norms and (optionally) ln Z_TN per realization."""
        lnZ = torch.zeros(self.n, dtype=torch.float64, device=self.device) if want_lnZ else None
        ws, nb = self._ws()
        _check(load().tnmc_build_env(self.table, self.n, self.chi, self.prec, ws, nb, _ptr(lnZ),
                                     _stream()), "tnmc_build_env")
        return lnZ

    def build_env_form(self, form, want_lnZ=True):
        """tnmc_build_env_form: the environments by a chosen form of the build (0 = default,
        1 = the Gram form with the per-site matrices in the workspace)."""
        lnZ = torch.zeros(self.n, dtype=torch.float64, device=self.device) if want_lnZ else None
        ws, nb = self._ws()
        _check(load().tnmc_build_env_form(self.table, self.n, self.chi, self.prec, int(form), ws,
                                          nb, _ptr(lnZ), _stream()), "tnmc_build_env_form")
        return lnZ

    def build_env_static(self, want_lnZ=True):
        """tnmc_build_env_static: the same as build_env, with the library's fixed scratch array
        instead of the workspace (nothing allocated by the call)."""
        lnZ = torch.zeros(self.n, dtype=torch.float64, device=self.device) if want_lnZ else None
        _check(load().tnmc_build_env_static(self.table, self.n, self.chi, self.prec, _ptr(lnZ),
                                            _stream()), "tnmc_build_env_static")
        return lnZ

    def spins_shape(self, K):
        return (self.n, K, self.Lmax, self.Wmax)

    def propose(self, K, seed, first_proposal=0, out=None, fallbacks=None):
        """tnmc_propose: K proposals per realization -> (spins words, logq, E)."""
        self.ensure_workspace(K)
        if out is None:
            spins = torch.empty(self.spins_shape(K), dtype=torch.int64, device=self.device)
            logq = torch.empty((self.n, K), dtype=torch.float64, device=self.device)
            E = torch.empty((self.n, K), dtype=torch.int32, device=self.device)
        else:
            spins, logq, E = out
        ws, nb = self._ws()
        _check(load().tnmc_propose(self.table, self.n, self.chi, self.prec, int(K), int(seed),
                                   int(first_proposal), ws, nb, _ptr(spins), _ptr(logq), _ptr(E),
                                   _ptr(fallbacks), _stream()), "tnmc_propose")
        return spins, logq, E

    # -- launch-shape tuning of the proposal kernel ------------------------------------------
    def propose_candidates(self):
        """Wavefronts per workgroup the proposal kernel can use at this chi."""
        buf = (ctypes.c_int32 * 4)()
        m = load().tnmc_propose_candidates(self.chi, ctypes.cast(buf, ctypes.c_void_p))
        return list(buf[:m])

    def tune_set(self, K, waves):
        """Force (waves > 0) or clear (0) the launch shape of this batch shape."""
        _check(load().tnmc_tune_set(self.chi, self.prec, self.Lmax, self.n, int(K), int(waves)),
               "tnmc_tune_set")

    def tune_get(self, K):
        return int(load().tnmc_tune_get(self.chi, self.prec, self.Lmax, self.n, int(K)))

    def autotune_propose(self, K, seed=0, reps=2):
        """tnmc_autotune_propose: time every candidate shape on this batch, keep the fastest.
        Returns (best waves, {waves: ms per launch})."""
        self.ensure_workspace(K)
        spins = torch.empty(self.spins_shape(K), dtype=torch.int64, device=self.device)
        logq = torch.empty((self.n, K), dtype=torch.float64, device=self.device)
        E = torch.empty((self.n, K), dtype=torch.int32, device=self.device)
        cands = self.propose_candidates()
        ms = (ctypes.c_float * 4)()
        best = ctypes.c_int32(0)
        ws, nb = self._ws()
        _check(load().tnmc_autotune_propose(self.table, self.n, self.chi, self.prec, int(K),
                                            int(seed), ws, nb, _ptr(spins), _ptr(logq), _ptr(E),
                                            int(reps), ctypes.byref(best),
                                            ctypes.cast(ms, ctypes.c_void_p), _stream()),
               "tnmc_autotune_propose")
        return best.value, {c: ms[j] for j, c in enumerate(cands)}

    def logq(self, spins, workspace=None):
        """tnmc_logq: log q of given configurations (spins words [n][K][Lmax][Wmax]); workspace:
        an optional uint8 tensor of tnmc_workspace_bytes for K instead of the batch's own (for a
        call on another stream)."""
        K = spins.shape[1]
        out = torch.empty((self.n, K), dtype=torch.float64, device=self.device)
        if workspace is None:
            self.ensure_workspace(K)
            ws, nb = self._ws()
        else:
            ws, nb = ctypes.c_void_p(workspace.data_ptr()), ctypes.c_size_t(workspace.numel())
        _check(load().tnmc_logq(self.table, self.n, self.chi, self.prec, int(K), _ptr(spins), ws,
                                nb, _ptr(out), _stream()), "tnmc_logq")
        return out

    def energy(self, spins, workspace=None):
        """tnmc_energy: exact integer energies of given configurations (workspace as for logq)."""
        K = spins.shape[1]
        E = torch.empty((self.n, K), dtype=torch.int32, device=self.device)
        if workspace is None:
            ws, nb = self._ws()
        else:
            ws, nb = ctypes.c_void_p(workspace.data_ptr()), ctypes.c_size_t(workspace.numel())
        _check(load().tnmc_energy(self.table, self.n, int(K), _ptr(spins), _ptr(E), ws, nb,
                                  _stream()), "tnmc_energy")
        return E

    def new_chains(self, n_chain):
        """Zeroed chain state for n_chain chains per realization."""
        return {
            "spins": torch.zeros((self.n, n_chain, self.Lmax, self.Wmax), dtype=torch.int64,
                                 device=self.device),
            "E": torch.zeros((self.n, n_chain), dtype=torch.int32, device=self.device),
            "logq": torch.zeros((self.n, n_chain), dtype=torch.float64, device=self.device),
            "init": torch.zeros((self.n, n_chain), dtype=torch.uint8, device=self.device),
            "n_chain": n_chain,
        }

    def accept(self, proposals, chains, seed, first_step=0, accum=None):
        """tnmc_accept: independence Metropolis over the proposals; updates `chains` in place."""
        spins, logq, E = proposals
        K = spins.shape[1]
        self.ensure_workspace(K)
        n_chain = chains["n_chain"]
        accepted = torch.empty((self.n, K), dtype=torch.uint8, device=self.device)
        current = torch.empty((self.n, K), dtype=torch.int32, device=self.device)
        ws, nb = self._ws()
        _check(load().tnmc_accept(self.table, self.n, n_chain, int(K), _ptr(spins), _ptr(logq),
                                  _ptr(E), int(seed), int(first_step), _ptr(chains["spins"]),
                                  _ptr(chains["E"]), _ptr(chains["logq"]), _ptr(chains["init"]),
                                  _ptr(accepted), _ptr(current), _ptr(accum), ws, nb, _stream()),
               "tnmc_accept")
        return accepted, current

    def observables(self, chains, accum):
        """tnmc_observables: add one sample per chain (current states) to accum [n][9]."""
        ws, nb = self._ws()
        _check(load().tnmc_observables(self.table, self.n, chains["n_chain"], _ptr(chains["spins"]),
                                       _ptr(chains["E"]), _ptr(accum), ws, nb, _stream()),
               "tnmc_observables")

    def disorder_average(self, accum, n_chain, rows=None):
        """tnmc_disorder_average over the realizations `rows` (default: all; they must share one L
        and one beta) of accum [n][9] -> tensor of AVG_COUNT values (AVG_NAMES order)."""
        rows = list(range(self.n)) if rows is None else list(rows)
        Ls = {self.Ls[i] for i in rows}
        betas = {self.table[i].beta for i in rows}
        if len(Ls) != 1 or len(betas) != 1:
            raise TNMCError("disorder_average needs rows of one L and one beta")
        sub = accum[rows].contiguous()
        out = torch.empty(AVG_COUNT, dtype=torch.float64, device=self.device)
        _check(load().tnmc_disorder_average(_ptr(sub), len(rows), Ls.pop(), betas.pop(),
                                            int(n_chain), _ptr(out), _stream()),
               "tnmc_disorder_average")
        return out

    def status_check(self):
        """tnmc_status_check: wait for the stream, return (status code, status words as a list);
        the code is 0 (ok) or ENUMERIC (a fault bit is set in some realization's word)."""
        words = (ctypes.c_uint32 * self.n)()
        st = load().tnmc_status_check(self.table, self.n, ctypes.cast(words, ctypes.c_void_p),
                                      _stream())
        if st not in (0, ENUMERIC):
            _check(st, "tnmc_status_check")
        return st, list(words)

    def clear_status(self):
        """Zero every realization's status word (a device fill on the current stream)."""
        self.status.zero_()

    def env_tensor(self, i):
        """Environments of realization i as (L, L, 2, chi, chi)."""
        L = self.Ls[i]
        return self.env[i].view(L, L, 2, self.chi, self.chi)


class PBC:
    """Periodic L x L lattices (one chain per torus) stepped by a frozen row and column per step
    (Sec. IV): torus couplings and configurations on the device, the open (L-1) x (L-1) blocks in
    a Batch with fields.  Every step runs tnmc_pbc_block, the block's build, proposals, the
    current state's log q and energy, tnmc_accept and tnmc_pbc_merge; nothing is computed here."""

    def __init__(self, L, n, betas, ids, chi, precision="fp32", K=1, device="cuda:0"):
        if L < 3:
            raise TNMCError("PBC: L >= 3")
        self.L, self.n = int(L), int(n)
        self.W = words_per_row(self.L)
        self.device = torch.device(device)
        self.Jh = torch.zeros((self.n, self.L * self.W), dtype=torch.int64, device=self.device)
        self.Jv = torch.zeros_like(self.Jh)
        self.spins = torch.zeros_like(self.Jh)
        self.E = torch.zeros(self.n, dtype=torch.int32, device=self.device)
        self.batch = Batch([self.L - 1] * self.n, betas, ids, chi, precision, K=K, device=device,
                           fields=True)
        self.chains = self.batch.new_chains(1)
        self.desc = (TorusDesc * self.n)()
        for i in range(self.n):
            d = self.desc[i]
            d.L, d.r0, d.c0, d.pad_ = self.L, 0, 0, 0
            d.d_Jh, d.d_Jv = self.Jh[i].data_ptr(), self.Jv[i].data_ptr()
            d.d_spins = self.spins[i].data_ptr()
        nb = int(load().tnmc_pbc_workspace_bytes(self.n))
        self.pws = torch.empty(nb, dtype=torch.uint8, device=self.device)
        # the current states' log q and energy run on a second stream beside the proposals,
        # with a workspace of their own
        nb = int(load().tnmc_workspace_bytes(self.batch.table, self.n, self.batch.chi, 1,
                                             self.batch.prec))
        self.ws_side = torch.empty(nb, dtype=torch.uint8, device=self.device)
        self.side = torch.cuda.Stream(device=self.device)

    def set_torus(self, i, jh_words, jv_words, spin_words):
        """Copy caller-packed torus couplings and configuration (L x W words each) into torus i."""
        self.Jh[i].copy_(torch.as_tensor(jh_words.view("int64")).reshape(-1))
        self.Jv[i].copy_(torch.as_tensor(jv_words.view("int64")).reshape(-1))
        self.spins[i].copy_(torch.as_tensor(spin_words.view("int64")).reshape(-1))

    def _pws(self):
        return ctypes.c_void_p(self.pws.data_ptr()), ctypes.c_size_t(self.pws.numel())

    def set_lines(self, lines):
        """Frozen (row, column) of each torus for the next block / merge."""
        for i, (r0, c0) in enumerate(lines):
            self.desc[i].r0, self.desc[i].c0 = int(r0), int(c0)

    def block(self):
        ws, nb = self._pws()
        _check(load().tnmc_pbc_block(self.desc, self.batch.table, self.n,
                                     _ptr(self.chains["spins"]), ws, nb, _stream()),
               "tnmc_pbc_block")

    def merge(self, want_energy=True):
        ws, nb = self._pws()
        _check(load().tnmc_pbc_merge(self.desc, self.batch.table, self.n,
                                     _ptr(self.chains["spins"]),
                                     _ptr(self.E) if want_energy else None, ws, nb, _stream()),
               "tnmc_pbc_merge")

    def step(self, lines, K, seed, first_proposal=0, first_step=0, init=False):
        """One step on every torus with the given lines: returns (accepted [n][K], proposals).
        init=True starts every chain afresh from the step's first proposal (taken
        unconditionally); otherwise the current block states' log q and energy under the step's
        environments are evaluated on a second stream while the proposals are drawn."""
        b, ch = self.batch, self.chains
        self.set_lines(lines)
        self.block()
        b.build_env(want_lnZ=False)
        cur = torch.cuda.current_stream(self.device)
        if init:
            ch["init"].fill_(0)
        else:
            self.side.wait_stream(cur)
            with torch.cuda.stream(self.side):
                ch["logq"].copy_(b.logq(ch["spins"], workspace=self.ws_side))
                ch["E"].copy_(b.energy(ch["spins"], workspace=self.ws_side))
                ch["init"].fill_(1)
        props = b.propose(K, seed, first_proposal)
        if not init:
            cur.wait_stream(self.side)
        accepted, _ = b.accept(props, ch, seed, first_step)
        self.merge()
        return accepted, props
