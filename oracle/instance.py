"""Problem instances: +-J couplings on an open Lr x Lc square lattice and the Nishimori line.

Sec. III A: J_ij = +1 with probability 1-p and -1 (antiferromagnetic) with probability p,
independently per nearest-neighbour bond (the disorder law of Eq. (11)); free boundaries
in both directions (Sec. II).  Sec. III A also gives the Nishimori line, exp(-2/T) = p/(1-p)
for J = 1, i.e. beta_N = (1/2) ln((1-p)/p).

Layout (both sides): rows r = 0..Lr-1 top to bottom, columns c = 0..Lc-1 left to right.
``Jh[r, c]`` joins (r, c)-(r, c+1), shape (Lr, Lc-1); ``Jv[r, c]`` joins (r, c)-(r+1, c),
shape (Lr-1, Lc).  Values are +1/-1 (int8).

Draw order: bond k takes Philox draw k of the stream with key (seed, STREAM_COUPLINGS) and
counter words (c1, c2, c3) = (0, 0, 0); the Jh bonds come first in row-major order
(k = r*(Lc-1) + c), then the Jv bonds in row-major order (k = Lr*(Lc-1) + r*Lc + c).
A bond is antiferromagnetic iff its uniform u < p.

This is test infrastructure (see the package docstring).
"""
import math

import numpy as np

from . import philox


def nishimori_beta(p):
    """Inverse temperature on the Nishimori line for J = 1: beta = ln((1-p)/p) / 2."""
    return 0.5 * math.log((1.0 - p) / p)


def couplings(seed, L, p, Lc=None):
    """+-1 couplings (Jh, Jv) for an L x Lc lattice (Lc defaults to L), i.i.d. with P(J=-1)=p."""
    Lr = L
    Lc = L if Lc is None else Lc
    nh = Lr * (Lc - 1)
    nv = (Lr - 1) * Lc
    u = philox.uniforms((seed, philox.STREAM_COUPLINGS), np.arange(nh + nv, dtype=np.uint64))
    J = np.where(u < p, -1, 1).astype(np.int8)
    Jh = J[:nh].reshape(Lr, Lc - 1)
    Jv = J[nh:].reshape(Lr - 1, Lc)
    return Jh, Jv


def bond_count(Lr, Lc=None):
    """Number of nearest-neighbour bonds with open boundaries: Lr(Lc-1) + (Lr-1)Lc."""
    Lc = Lr if Lc is None else Lc
    return Lr * (Lc - 1) + (Lr - 1) * Lc
