"""Energy of the +-J random-bond Ising model with open boundaries (Sec. III A, Eq. (10)).

E(s) = - sum over nearest-neighbour bonds (ij) of J_ij s_i s_j, plus - sum_i h_i s_i when the
lattice is a block of a larger system whose other spins are held fixed: h_i = sum of J s_f over
the fixed neighbours f of site i (the fields of Sec. II B's sampling step, here on the boundary of
the block; see ``pbc``).  Written as the plain double loop over bonds and sites; the batch of
configurations is the only vectorised axis.

This is test infrastructure (see the package docstring).
"""
import numpy as np


def energy(s, Jh, Jv, field=None):
    """Integer energy of each configuration.

    s     : (..., Lr, Lc) array of +1/-1 spins
    Jh    : (Lr, Lc-1) couplings of horizontal bonds (r, c)-(r, c+1)
    Jv    : (Lr-1, Lc) couplings of vertical bonds (r, c)-(r+1, c)
    field : optional (Lr, Lc) integer fields h (units of the coupling)
    returns an int64 array of shape s.shape[:-2]
    """
    s = np.asarray(s, dtype=np.int64)
    Lr, Lc = s.shape[-2], s.shape[-1]
    E = np.zeros(s.shape[:-2], dtype=np.int64)
    for r in range(Lr):
        for c in range(Lc - 1):
            E -= int(Jh[r, c]) * s[..., r, c] * s[..., r, c + 1]
    for r in range(Lr - 1):
        for c in range(Lc):
            E -= int(Jv[r, c]) * s[..., r, c] * s[..., r + 1, c]
    if field is not None:
        for r in range(Lr):
            for c in range(Lc):
                E -= int(field[r, c]) * s[..., r, c]
    return E
