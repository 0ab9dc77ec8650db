"""Exact references that do not use the tensor-network code: enumeration and transfer matrices.

* Brute force (Eqs. (1)-(2)): enumerate all 2^N configurations of a small lattice, giving Z,
  log P(s) = -beta E(s) - ln Z, and exact expectation values.
* Exact row transfer matrix: the same sum organised row by row over 2^Lc row states, giving
  ln Z and the exact bottom environments E_r(x) = sum over rows below r (the exact objects the
  boundary MPS approximates, Sec. II B) for lattices up to Lc of about 18.

Configuration index convention (brute force): bit j of the index, j = r*Lc + c (the zig-zag /
row-major order of Sec. II A), is 1 iff s[r, c] = -1.  Row-state convention (transfer matrix):
bit c of the row index is 1 iff the spin in column c is -1.

This is test infrastructure (see the package docstring).
"""
import numpy as np

from .energy import energy


def all_configs(Lr, Lc):
    """All 2^(Lr*Lc) configurations as an int8 array (2^N, Lr, Lc) in index order."""
    N = Lr * Lc
    idx = np.arange(2 ** N, dtype=np.int64)
    bits = (idx[:, None] >> np.arange(N)[None, :]) & 1
    return (1 - 2 * bits).astype(np.int8).reshape(-1, Lr, Lc)


def _logsumexp(a):
    m = np.max(a)
    return float(m + np.log(np.sum(np.exp(a - m))))


def brute_force(Jh, Jv, beta, field=None):
    """Exact enumeration. Returns dict with configs, E, lnZ and logP for every configuration
    (field: optional (Lr, Lc) site fields, see energy)."""
    Lr, Lc = Jh.shape[0], Jv.shape[1]
    s = all_configs(Lr, Lc)
    E = energy(s, Jh, Jv, field)
    lw = -beta * E.astype(np.float64)
    lnZ = _logsumexp(lw)
    return {"configs": s, "E": E, "lnZ": lnZ, "logP": lw - lnZ}


def _row_spins(Lc):
    """(2^Lc, Lc) spins of every row state."""
    idx = np.arange(2 ** Lc, dtype=np.int64)
    return 1 - 2 * ((idx[:, None] >> np.arange(Lc)[None, :]) & 1)


def _row_weight(Jh_row, beta, ys):
    """H_r(y) = prod_c exp(beta Jh[r,c] y_c y_{c+1}) for every row state (log form)."""
    lw = np.zeros(ys.shape[0])
    for c in range(ys.shape[1] - 1):
        lw += beta * Jh_row[c] * ys[:, c] * ys[:, c + 1]
    return lw


def _apply_vertical(psi, Jv_row, beta, Lc):
    """(V psi)(x) = sum_y prod_c exp(beta Jv[c] x_c y_c) psi(y), one column (bit) at a time."""
    out = psi
    for c in range(Lc):
        a = np.exp(beta * Jv_row[c])
        b = np.exp(-beta * Jv_row[c])
        v = out.reshape(-1, 2, 2 ** c)          # axis 1 is bit c
        up, dn = v[:, 0, :], v[:, 1, :]
        new = np.empty_like(v)
        new[:, 0, :] = a * up + b * dn          # x_c = +1: sum over y_c
        new[:, 1, :] = b * up + a * dn          # x_c = -1
        out = new.reshape(-1)
    return out


def transfer_matrix(Jh, Jv, beta):
    """Exact ln Z and exact bottom environments by the row transfer matrix.

    E_{Lr-1}(x) = 1;  E_{r-1}(x) = sum_y V_{r-1}(x, y) H_r(y) E_r(y);  Z = sum_x H_0(x) E_0(x).
    Returns dict with lnZ, envs (list of (scale, vector) with E_r = exp(scale) * vector) and
    lognorm[r] = ln ||E_r||_2.
    """
    Lr, Lc = Jh.shape[0], Jv.shape[1]
    ys = _row_spins(Lc)
    envs = [None] * Lr
    vec = np.ones(2 ** Lc)
    scale = 0.0
    envs[Lr - 1] = (scale, vec.copy())
    for r in range(Lr - 1, 0, -1):
        f = np.exp(_row_weight(Jh[r], beta, ys)) * vec
        vec = _apply_vertical(f, Jv[r - 1], beta, Lc)
        m = np.max(np.abs(vec))
        vec = vec / m
        scale += np.log(m)
        envs[r - 1] = (scale, vec.copy())
    top = np.exp(_row_weight(Jh[0], beta, ys)) * vec
    lnZ = scale + float(np.log(np.sum(top)))
    lognorm = np.array([sc + 0.5 * np.log(np.sum(v * v)) for sc, v in envs])
    return {"lnZ": lnZ, "envs": envs, "lognorm": lognorm}


def log_prob(s, Jh, Jv, beta, lnZ):
    """Exact log P(s) = -beta E(s) - ln Z (Eq. (1))."""
    return -beta * energy(s, Jh, Jv).astype(np.float64) - lnZ
