"""Whole-lattice proposals s ~ q(s) from the cached environments, with log q(s) (Sec. II A-B).

Eq. (4) factorises P(s) into conditionals in the zig-zag (row-major) order; Eq. (5) writes each
conditional as a ratio of conditional partition functions; with truncated contractions these
become the approximate conditionals q(s_i | s_<i) whose product is the proposal q(s), Eq. (6).
Sampling runs in the reverse order of the contraction (Sec. II B): spins already fixed become
reduced copy tensors, and their Boltzmann matrices towards the next row act as external fields.

With the row environments E_r of ``envbuild`` the conditional of row r given the rows above is
the row chain

    f_r(y) = prod_c phi_c(y_c) prod_c w_c(y_c, y_{c+1}) E_r(y),
    phi_c(y) = exp(beta Jv[r-1,c] s[r-1,c] y)   (1 on row 0),   w_c(y, y') = exp(beta Jh[r,c] y y'),

(with site fields h, phi_c(y) also carries exp(beta h[r,c] y), on row 0 too),

which is summed exactly column by column:

  right partial sums  R_{Lc-1}(y) = [1],
                      R_c(y) = sum_{y'} w_c(y, y') phi_{c+1}(y') A^{(c+1)}[y'] R_{c+1}(y');
  left running vector l = [1]; at column c, for y = +-1
                      Z_c(y) = [w_{c-1}(s_{c-1}, y) if c > 0] phi_c(y) l A^{(c)}[y] R_c(y),
                      p+ = Z_c(+) / (Z_c(+) + Z_c(-)),
  draw s_c, then      l <- l A^{(c)}[s_c] [w_{c-1}(s_{c-1}, s_c)] phi_c(s_c).

Every R_c and l may be rescaled by a positive constant (they cancel in p+).  Readings where the
paper is silent: negative Z_c(y) (possible after truncation) are set to 0; if both vanish or the
sum is not finite, p+ = 1/2 and a fallback is counted; p+ is clamped to [1e-12, 1 - 1e-12] so
that q(s) > 0 wherever P(s) > 0; the spin is +1 iff u < p+ (strict), with u the 53-bit Philox
uniform number c of the stream keyed (seed, STREAM_PROPOSAL) with counter words
(r, proposal, realization); log q accumulates ln p+ or ln(1 - p+) with p- = 1 - p+ in FP64.

This is test infrastructure (see the package docstring).
"""
import numpy as np

from . import philox

P_CLAMP = 1e-12
_SGN = np.array([1.0, -1.0])


def _bond_matrix(beta, J):
    return np.exp(beta * J * np.outer(_SGN, _SGN))


def _rescale(x):
    """Divide each batch entry (axis 0) by its largest magnitude (if positive and finite)."""
    m = np.max(np.abs(x.reshape(x.shape[0], -1)), axis=1)
    m = np.where((m > 0) & np.isfinite(m), m, 1.0)
    return x / m.reshape((-1,) + (1,) * (x.ndim - 1))


def proposal_uniforms(seed, realization, proposals, r, Lc):
    """u[k, c] for the given proposal ids (array) at row r: draw c, counter words (r, k, id)."""
    k = np.asarray(proposals, dtype=np.uint64)[:, None]
    c = np.arange(Lc, dtype=np.uint64)[None, :]
    return philox.uniforms((seed, philox.STREAM_PROPOSAL), c, c1=r, c2=k, c3=realization)


def run(env, Jh, Jv, beta, K=None, seed=0, realization=0, first_proposal=0, teacher=None,
        field=None):
    """Sample K proposals (teacher=None) or evaluate log q of given configurations.

    env     : dict from envbuild.build_env (built with the same field)
    teacher : optional (K, Lr, Lc) array of +1/-1 spins to evaluate instead of sampling
    field   : optional (Lr, Lc) integer site fields
    returns dict with spins (K, Lr, Lc) int8, logq (K,) float64, fallbacks (int),
    pplus (K, Lr, Lc) float64: the p+ used at every site (after the clamp)
    """
    sites = env["sites"]
    Lr, Lc = Jh.shape[0], Jh.shape[1] + 1
    if teacher is not None:
        teacher = np.asarray(teacher, dtype=np.int8)
        K = teacher.shape[0]
    ids = first_proposal + np.arange(K, dtype=np.uint64)
    s = np.zeros((K, Lr, Lc), dtype=np.int8)
    logq = np.zeros(K)
    pplus = np.zeros((K, Lr, Lc))
    fallbacks = 0
    for r in range(Lr):
        A = sites[r]
        if r > 0:
            phi = np.exp(beta * Jv[r - 1][None, :, None] * s[:, r - 1, :, None].astype(np.float64)
                         * _SGN[None, None, :])                       # (K, Lc, 2)
        else:
            phi = np.ones((K, Lc, 2))
        if field is not None:
            phi = phi * np.exp(beta * np.asarray(field[r], dtype=np.float64)[None, :, None]
                               * _SGN[None, None, :])
        w = [_bond_matrix(beta, Jh[r, c]) for c in range(Lc - 1)]
        # right partial sums R[c][k, y, beta], beta = right bond of site c
        R = [None] * Lc
        R[Lc - 1] = np.ones((K, 2, 1))
        for c in range(Lc - 2, -1, -1):
            v = np.einsum("asb,ksb->ksa", A[c + 1], R[c + 1])          # A^{(c+1)}[y'] R_{c+1}(y')
            R[c] = _rescale(np.einsum("st,kt,kta->ksa", w[c], phi[:, c + 1, :], v))
        u = None if teacher is not None else proposal_uniforms(seed, realization, ids, r, Lc)
        ell = np.ones((K, 1))
        for c in range(Lc):
            t = np.einsum("ka,asb->ksb", ell, A[c])                    # l A^{(c)}[y]
            pre = phi[:, c, :].copy()
            if c > 0:
                prev = (s[:, r, c - 1] < 0).astype(np.int64)          # 0 <-> +1, 1 <-> -1
                pre *= w[c - 1][prev, :]
            Z = pre * np.einsum("ksb,ksb->ks", t, R[c])
            Zp = np.maximum(Z[:, 0], 0.0)
            Zm = np.maximum(Z[:, 1], 0.0)
            tot = Zp + Zm
            bad = ~np.isfinite(tot) | (tot <= 0)
            fallbacks += int(np.count_nonzero(bad))
            pp = np.where(bad, 0.5, Zp / np.where(bad, 1.0, tot))
            pp = np.clip(pp, P_CLAMP, 1.0 - P_CLAMP)
            if teacher is None:
                up = u[:, c] < pp
            else:
                up = teacher[:, r, c] > 0
            s[:, r, c] = np.where(up, 1, -1)
            pplus[:, r, c] = pp
            logq += np.where(up, np.log(pp), np.log(1.0 - pp))
            idx = np.where(up, 0, 1)
            ell = _rescale(t[np.arange(K), idx, :] * pre[np.arange(K), idx][:, None])
    return {"spins": s, "logq": logq, "fallbacks": fallbacks, "pplus": pplus}
