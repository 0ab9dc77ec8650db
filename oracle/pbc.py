"""Periodic boundaries by a frozen line pair, and partial-block proposals (Sec. IV; Sec. I).

The method proposes configurations of a chosen block of spins, which may be the whole system or
a part of it (Sec. I).  Sec. IV extends it to periodic boundaries: at each step one row r0 and
one column c0 of the L x L torus are picked and their 2L - 1 spins are held fixed for the step;
they act as external fields on their neighbours, and the rest of the torus is an open block.

Block.  The block has (L-1) x (L-1) sites; its site (a, b) is torus site (R(a), C(b)) with
R(a) = (r0 + 1 + a) mod L and C(b) = (c0 + 1 + b) mod L.  Every torus bond with both ends in the
block is a block bond (rows and columns keep their order, so the block is an ordinary open
lattice); a bond from block site i to a frozen spin f adds J_if s_f to the integer field h_i of
that site; the bonds with both ends frozen are a constant of the step.  Therefore, for every
configuration s that agrees with the frozen spins,

    E_torus(s) = E_block(s_b) + E_frozen,   E_block = - sum_block bonds J s s - sum_i h_i s_i,

and the target of the step, P(s_b | frozen) ~ exp(-beta E_block(s_b)), is the Boltzmann weight
of the open block in the fields h, which ``envbuild`` / ``sampler`` contract and sample like any
open lattice (with field=h).

Step (one chain on one torus).  Build the block environments in the fields h, draw K proposals
of the block, evaluate log q of the current block configuration under the same environments
(teacher forcing), run the independence Metropolis chain (``accept``) over the K proposals
starting from the current block state, and write the final block state back into the torus.
Each step's chain targets P(s_b | frozen), so the torus Boltzmann distribution is stationary for
every choice of lines; picking the lines at random makes every spin movable.

Readings where the paper is silent: the lines (r0, c0) of each step are inputs (the caller draws
them); a chain may start afresh at a step (init), taking that step's first proposal
unconditionally, which is how a chain is started from a configuration the proposals consider
typical (a random start can hold a chain for many steps where q underrates it); the torus couplings are inputs, Jh_t[r, c] on the bond (r, c)-(r, (c+1) mod L) and Jv_t[r,
c] on (r, c)-((r+1) mod L, c); L >= 3, so that the block has at least 2 x 2 sites.

This is test infrastructure (see the package docstring).
"""
import numpy as np

from . import accept, energy, envbuild, sampler


def torus_energy(s, Jh_t, Jv_t):
    """E(s) = -sum over the 2 L^2 torus bonds of J s s (integer), batched over s[..., L, L]."""
    s = np.asarray(s, dtype=np.int64)
    L = s.shape[-1]
    E = np.zeros(s.shape[:-2], dtype=np.int64)
    for r in range(L):
        for c in range(L):
            E -= int(Jh_t[r, c]) * s[..., r, c] * s[..., r, (c + 1) % L]
            E -= int(Jv_t[r, c]) * s[..., r, c] * s[..., (r + 1) % L, c]
    return E


def block(Jh_t, Jv_t, s_t, r0, c0):
    """The open block of the torus configuration s_t with row r0 and column c0 frozen.

    Returns (Jh, Jv, h, s_b): block couplings (Lb, Lb-1) and (Lb-1, Lb), integer fields (Lb, Lb)
    and the block's part of s_t (Lb, Lb), Lb = L - 1.
    """
    L = s_t.shape[-1]
    Lb = L - 1
    R = [(r0 + 1 + a) % L for a in range(Lb)]
    C = [(c0 + 1 + b) % L for b in range(Lb)]
    Jh = np.zeros((Lb, Lb - 1), dtype=np.int8)
    Jv = np.zeros((Lb - 1, Lb), dtype=np.int8)
    h = np.zeros((Lb, Lb), dtype=np.int8)
    s_b = np.zeros((Lb, Lb), dtype=np.int8)
    for a in range(Lb):
        for b in range(Lb):
            s_b[a, b] = s_t[R[a], C[b]]
            if b + 1 < Lb:
                Jh[a, b] = Jh_t[R[a], C[b]]
            if a + 1 < Lb:
                Jv[a, b] = Jv_t[R[a], C[b]]
    # fields: the four neighbours of each block site, those on the frozen lines
    for a in range(Lb):
        for b in range(Lb):
            r, c = R[a], C[b]
            nbrs = [((r - 1) % L, c, Jv_t[(r - 1) % L, c]),      # above
                    ((r + 1) % L, c, Jv_t[r, c]),                # below
                    (r, (c - 1) % L, Jh_t[r, (c - 1) % L]),      # left
                    (r, (c + 1) % L, Jh_t[r, c])]                # right
            for rr, cc, J in nbrs:
                if rr == r0 or cc == c0:
                    h[a, b] += int(J) * int(s_t[rr, cc])
    return Jh, Jv, h, s_b


def merge(s_t, s_b, r0, c0):
    """The torus configuration s_t with its block replaced by s_b (the frozen lines kept)."""
    L = s_t.shape[-1]
    out = np.array(s_t, dtype=np.int8, copy=True)
    for a in range(L - 1):
        for b in range(L - 1):
            out[(r0 + 1 + a) % L, (c0 + 1 + b) % L] = s_b[a, b]
    return out


def step(Jh_t, Jv_t, s_t, beta, chi, r0, c0, K, seed=0, realization=0, first_proposal=0,
         first_step=0, init=False):
    """One TNMC step on the torus with lines (r0, c0) frozen; returns (new s_t, info dict).
    init=True starts the chain afresh: the step's first proposal is taken unconditionally (as
    ``accept`` does for a new chain) instead of the current block configuration."""
    Jh, Jv, h, s_b = block(Jh_t, Jv_t, s_t, r0, c0)
    env = envbuild.build_env(Jh, Jv, beta, chi, field=h)
    smp = sampler.run(env, Jh, Jv, beta, K=K, seed=seed, realization=realization,
                      first_proposal=first_proposal, field=h)
    E_prop = energy.energy(smp["spins"], Jh, Jv, field=h)
    if init:
        state, E_cur, logq_cur = None, None, None
    else:
        cur = sampler.run(env, Jh, Jv, beta, teacher=s_b[None], field=h)
        E_cur = int(energy.energy(s_b[None], Jh, Jv, field=h)[0])
        logq_cur = float(cur["logq"][0])
        state = {"idx": -1, "E": E_cur, "logq": logq_cur}
    out = accept.chain(E_prop, smp["logq"], beta, seed=seed, realization=realization,
                       chain_index=0, first_step=first_step, state=state)
    final = int(out["current"][-1])
    s_new = s_b if final < 0 else smp["spins"][final]
    info = {"block": (Jh, Jv, h, s_b), "env": env, "proposals": smp, "E_prop": E_prop,
            "E_cur": E_cur, "logq_cur": logq_cur, "chain": out}
    return merge(s_t, s_new, r0, c0), info
