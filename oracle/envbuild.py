"""Boundary-MPS environments of the 2D open-lattice Ising tensor network (Sec. II B).

The partition function of Eq. (2) is a network of copy tensors (delta) and Boltzmann matrices W
(Eq. (10) for W; the T tensor of Sec. II B absorbs the W on the right and bottom bonds of each
site).  It is contracted from the last site upward, storing the process tensors for later
sampling, with bond dimensions truncated by SVD to a fixed maximum D = chi (Sec. II B).

Contraction scheme (a reading: the paper absorbs one T tensor at a time and defers the
truncation details to its references).  A whole row is absorbed at once: the bottom
environment of row r is the function of the row configuration x

    E_{Lr-1}(x) = 1,
    E_{r-1}(x)  = sum_y V_{r-1}(x, y) H_r(y) E_r(y),       r = Lr-1, ..., 1,
    Z           = sum_x H_0(x) E_0(x),

with H_r(y) = prod_c exp(beta Jh[r,c] y_c y_{c+1}) and V_{r-1}(x, y) = prod_c exp(beta
Jv[r-1,c] x_c y_c).  A lattice that is a block of a larger system with its other spins held
fixed (see ``pbc``) carries integer site fields h; their weight F_r(y) = prod_c exp(beta h[r,c]
y_c) enters with the row's own bonds, H_r(y) -> H_r(y) F_r(y), in the recursion and in Z.  Each E_r is kept as a matrix-product state (MPS) along the row.  Applying
the row operator to an MPS of bond chi gives an MPS of bond 2*chi whose site tensor carries the
spin y_c on its right bond:

    At[c][(a, alpha), x, (b, alpha')] = exp(beta Jh[r,c-1] a b) exp(beta Jv[r-1,c] x b) A[c][alpha, b, alpha']

(times exp(beta h[r,c] b) with fields)

(no a at c = 0; b summed at c = Lc-1).  It is compressed back to chi by the canonical SVD
compression: a QR sweep left to right (left-orthonormal sites), then an SVD sweep right to left
keeping k = min(chi, rows, cols) singular values at every bond (LAPACK order).  The result has
right-orthonormal sites 1..Lc-1; the norm is taken out of site 0, so the stored MPS has unit
2-norm and lognorm[r] = ln ||E_r||_2 (gauge invariant, the quantity compared across
implementations).  For range only, the factor carried to the next site (R after each QR step, U S after each
SVD step) is divided by its Frobenius norm and the log of that norm is accumulated; positive
factors leave the compressed, normalised state unchanged.

Tensor convention: A[c] has shape (chi_left, 2, chi_right); physical index 0 <-> spin +1,
1 <-> spin -1.

This is test infrastructure (see the package docstring).
"""
import math

import numpy as np

_SGN = np.array([1.0, -1.0])


def _bond_matrix(beta, J):
    """exp(beta J s s') for s, s' in (+1, -1): the Boltzmann matrix W of Eq. (10)."""
    return np.exp(beta * J * np.outer(_SGN, _SGN))


def apply_row_mpo(mps, Jh_row, Jv_row, beta, field_row=None):
    """Site tensors of (V H F f) for the MPS f: Jh_row = Jh[r], Jv_row = Jv[r-1], field_row =
    h[r] (None: no field)."""
    Lc = len(mps)
    out = []
    for c, A in enumerate(mps):
        dl, _, dr = A.shape
        if field_row is not None:
            A = A * np.exp(beta * field_row[c] * _SGN)[None, :, None]
        wv = _bond_matrix(beta, Jv_row[c])                    # (x, b)
        if Lc == 1:
            T = np.einsum("xb,ubv->uxv", wv, A)
        elif c == 0:
            T = np.einsum("xb,ubv->uxbv", wv, A).reshape(dl, 2, 2 * dr)
        else:
            wh = _bond_matrix(beta, Jh_row[c - 1])            # (a, b)
            if c == Lc - 1:
                T = np.einsum("ab,xb,ubv->auxv", wh, wv, A).reshape(2 * dl, 2, dr)
            else:
                T = np.einsum("ab,xb,ubv->auxbv", wh, wv, A).reshape(2 * dl, 2, 2 * dr)
        out.append(T)
    return out


def compress(mps, chi):
    """Canonical SVD compression to bond dimension chi.

    Returns (sites, log_norm, cuts): the normalised right-canonical MPS, the log of the norm
    taken out, and per truncated bond c a pair (s_k / s_1, (s_k - s_{k+1}) / s_k) describing the
    cut (s = singular values at that bond, k kept).  Rounding of size eps * s_1 rotates the kept
    subspace by about eps * s_1 / (s_k - s_{k+1}), which changes the normalised state by about
    min(eps / relgap, s_k / s_1): see ``sensitivity``.
    """
    T = [t.copy() for t in mps]
    Lc = len(T)
    log_carried = 0.0
    for c in range(Lc - 1):                                   # QR sweep, left to right
        dl, d, dr = T[c].shape
        Q, R = np.linalg.qr(T[c].reshape(dl * d, dr))
        nR = float(np.linalg.norm(R))
        log_carried += math.log(nR)
        T[c] = Q.reshape(dl, d, Q.shape[1])
        T[c + 1] = np.tensordot(R / nR, T[c + 1], axes=(1, 0))
    cuts = {}
    for c in range(Lc - 1, 0, -1):                            # SVD sweep, right to left
        dl, d, dr = T[c].shape
        U, S, Vt = np.linalg.svd(T[c].reshape(dl, d * dr), full_matrices=False)
        k = min(chi, S.shape[0])
        if k < S.shape[0] and S[k - 1] > 0:
            cuts[c] = (S[k - 1] / S[0], (S[k - 1] - S[k]) / S[k - 1])
        nS = float(np.linalg.norm(S[:k]))
        log_carried += math.log(nS)
        T[c] = Vt[:k].reshape(k, d, dr)
        T[c - 1] = np.tensordot(T[c - 1], U[:, :k] * (S[:k] / nS), axes=(2, 0))
    n = float(np.linalg.norm(T[0]))
    T[0] = T[0] / n
    return T, log_carried + math.log(n), cuts


def compress_zipup(mps, chi, direction):
    """Zip-up compression (Stoudenmire and White, New J. Phys. 12, 055026 (2010)): one sweep of
    SVD truncations over the row-operator-applied MPS, without the orthonormalising sweep of
    the canonical compression.  Applying the operator exactly and then truncating site by site
    is the same arithmetic as contracting each operator site into the carried factor during the
    sweep.  The sweep must run away from the input's orthogonality centre: direction "rl"
    (right to left, for an input whose norm sits in the last site, leaving sites 1..Lc-1 right-
    orthonormal) or "lr" (left to right, for an input whose norm sits in site 0, leaving sites
    0..Lc-2 left-orthonormal).  The truncation at a cut keeps the k = min(chi, rows, cols)
    largest singular values of the partly swept object; unlike the canonical compression it is
    not the optimal truncation of the whole state, because the not yet swept part is not
    orthonormal once the operator is applied.  Returns (sites, log_norm, cuts) as compress."""
    T = [t.copy() for t in mps]
    Lc = len(T)
    log_carried = 0.0
    cuts = {}
    if direction == "rl":
        for c in range(Lc - 1, 0, -1):
            dl, d, dr = T[c].shape
            U, S, Vt = np.linalg.svd(T[c].reshape(dl, d * dr), full_matrices=False)
            k = min(chi, S.shape[0])
            if k < S.shape[0] and S[k - 1] > 0:
                cuts[c] = (S[k - 1] / S[0], (S[k - 1] - S[k]) / S[k - 1])
            nS = float(np.linalg.norm(S[:k]))
            log_carried += math.log(nS)
            T[c] = Vt[:k].reshape(k, d, dr)
            T[c - 1] = np.tensordot(T[c - 1], U[:, :k] * (S[:k] / nS), axes=(2, 0))
        n = float(np.linalg.norm(T[0]))
        T[0] = T[0] / n
    elif direction == "lr":
        for c in range(Lc - 1):
            dl, d, dr = T[c].shape
            U, S, Vt = np.linalg.svd(T[c].reshape(dl * d, dr), full_matrices=False)
            k = min(chi, S.shape[0])
            if k < S.shape[0] and S[k - 1] > 0:
                cuts[c + 1] = (S[k - 1] / S[0], (S[k - 1] - S[k]) / S[k - 1])
            nS = float(np.linalg.norm(S[:k]))
            log_carried += math.log(nS)
            T[c] = U[:, :k].reshape(dl, d, k)
            T[c + 1] = np.tensordot((S[:k] / nS)[:, None] * Vt[:k], T[c + 1], axes=(1, 0))
        n = float(np.linalg.norm(T[Lc - 1]))
        T[Lc - 1] = T[Lc - 1] / n
    else:
        raise ValueError(direction)
    return T, log_carried + math.log(n), cuts


def zipup_direction(Lr, r):
    """Sweep direction of the zip-up that builds E_{r-1} from E_r: right to left for the first
    row applied (E_{Lr-1} is a product state, so its centre may be taken at the last site), then
    alternating, so that every sweep runs away from the centre the previous one left."""
    return "rl" if (Lr - 1 - r) % 2 == 0 else "lr"


def sensitivity(env, eps):
    """Largest estimated relative change of any built E_r under rounding of relative size eps:
    max over truncated cuts of min(eps / relgap, s_k / s_1).  Parity with another correct
    implementation is expected to about this level times a modest factor."""
    worst = 0.0
    for cuts in env["cuts"]:
        for sk, rel in cuts.values():
            worst = max(worst, min(eps / rel if rel > 0 else math.inf, sk))
    return worst


def top_row_sum(mps, Jh_row, beta, field_row=None):
    """ln sum_x H_0(x) F_0(x) E(x) for the MPS E, with a running rescale (log kept separately);
    F_0 = 1 without fields."""
    Lc = len(mps)
    g = [np.ones(2) if field_row is None else np.exp(beta * field_row[c] * _SGN) for c in range(Lc)]
    v = mps[0][0] * g[0][:, None]                             # v[sigma] = A0[0, sigma, :] -> (2, dr)
    logscale = 0.0
    for c in range(1, Lc):
        wh = _bond_matrix(beta, Jh_row[c - 1])               # (sigma, sigma')
        A = mps[c] * g[c][None, :, None]                     # (dl, 2, dr)
        v = np.einsum("st,sa,atb->tb", wh, v, A)
        m = float(np.max(np.abs(v)))
        v = v / m
        logscale += math.log(m)
    total = float(np.sum(v))
    return logscale + math.log(total) if total > 0 else float("nan")


def build_env(Jh, Jv, beta, chi, rows=None, method="canonical", field=None):
    """Environments E_{Lr-1}, ..., E_0 by repeated row-MPO application and compression
    (method "canonical": compress, the canonical SVD compression; "zipup": compress_zipup in the
    direction of zipup_direction).  field: optional (Lr, Lc) integer site fields.

    Returns dict with
      sites[r][c] : (chi_l, 2, chi_r) tensors of the normalised MPS of E_r
      lognorm[r]  : ln ||E_r||_2
      lnZ         : lambda_0 + ln sum_x H_0(x) E_0(x) / ||E_0||   (the TN estimate of ln Z)
      cuts[r]     : {bond c: (s_k / s_1, relative gap)} of the truncations that produced E_r
    ``rows`` (optional) stops after building that many rows below the bottom one (for slices of
    large lattices); lnZ is then omitted.
    """
    Lr, Lc = Jh.shape[0], Jh.shape[1] + 1
    # E_{Lr-1} = 1: each site 1/sqrt(2) (right-orthonormal), norm 2^(Lc/2).
    mps = [np.full((1, 2, 1), 1.0 / math.sqrt(2.0)) for _ in range(Lc)]
    sites = [None] * Lr
    lognorm = np.full(Lr, np.nan)
    cuts = [dict() for _ in range(Lr)]
    sites[Lr - 1] = mps
    lognorm[Lr - 1] = 0.5 * Lc * math.log(2.0)
    last = 1 if rows is None else max(1, Lr - rows)
    for r in range(Lr - 1, last - 1, -1):
        big = apply_row_mpo(mps, Jh[r], Jv[r - 1], beta, None if field is None else field[r])
        if method == "canonical":
            mps, ln_n, cuts[r - 1] = compress(big, chi)
        elif method == "zipup":
            mps, ln_n, cuts[r - 1] = compress_zipup(big, chi, zipup_direction(Lr, r))
        else:
            raise ValueError(method)
        sites[r - 1] = mps
        lognorm[r - 1] = lognorm[r] + ln_n
    out = {"sites": sites, "lognorm": lognorm, "cuts": cuts, "chi": chi, "method": method}
    if rows is None:
        out["lnZ"] = lognorm[0] + top_row_sum(sites[0], Jh[0], beta,
                                              None if field is None else field[0])
    return out

