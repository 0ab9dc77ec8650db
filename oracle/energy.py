"""Energy of the +-J random-bond Ising model with open boundaries (Sec. III A, Eq. (10)).

E(s) = - sum over nearest-neighbour bonds (ij) of J_ij s_i s_j.  Written as the plain double
loop over bonds; the batch of configurations is the only vectorised axis.

This is test infrastructure (see the package docstring).
"""
import numpy as np


def energy(s, Jh, Jv):
    """Integer energy of each configuration.

    s  : (..., Lr, Lc) array of +1/-1 spins
    Jh : (Lr, Lc-1) couplings of horizontal bonds (r, c)-(r, c+1)
    Jv : (Lr-1, Lc) couplings of vertical bonds (r, c)-(r+1, c)
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
    return E
