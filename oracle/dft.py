"""The Fourier transform on the pattern P(M), float64 (Section 2.2, eq.
Fouriermatrix).

TEST INFRASTRUCTURE ONLY (see the package docstring).

    F(M) = m^{-1/2} ( exp(-2 pi i h^T M^{-1} g) )_{h in G(M^T), g in G(M)}

with m = |det M|.  Inputs are indexed by the natural box of M (samples g),
outputs by the natural box of M^T (frequencies h); see ``oracle.lattice``.
The inverse is the conjugate transpose (F(M) is unitary).

Two independent algorithms:
  * ``lattice_dft_direct`` is the definition written out: an O(m^2) sum with
    exact integer phase residues.  Pins: diagonal M equals numpy's fftn with
    orthonormal scaling (Section 4.1, Kronecker form with the identity
    permutations); d_M = 1 equals a 1-D DFT; impulse and plane-wave inputs;
    Parseval.
  * ``lattice_dft_hnf`` is a row/column FFT on the Hermite form H = M U,
    with exact twiddle residues between the axes (a Mersereau-style twisted
    decomposition, the approach the paper contrasts itself with in
    Section 1).  It never uses the Smith form, so it shares no structure with
    the GPU path.  Pinned against ``lattice_dft_direct`` for m up to 2^14 and
    against sampled direct bins (``direct_bins``) at any size.
"""
import os

import numpy as np
import scipy.fft

from . import lattice as L


def _natural_keys(H):
    """(m, d) int64 array of the natural box points of H, C order."""
    shape = L.box_shape(H)
    grids = np.meshgrid(*[np.arange(n, dtype=np.int64) for n in shape], indexing="ij")
    return np.stack([g.reshape(-1) for g in grids], axis=1)


def natural_keys(M, which="samples"):
    """Natural keys: samples g in box(HNF(M)) or frequencies h in box(HNF(M^T))."""
    M = L.as_matrix(M)
    H, _ = L.hnf(M if which == "samples" else L.transpose(M))
    return _natural_keys(H)


def _check_size(m):
    # every residue product below is (x mod m) * (y mod m) < 2^62
    if m >= (1 << 31):
        raise ValueError("oracle supports m < 2^31")


def _modmatvec(W, keys, m):
    """((W @ key) mod m) for every row key of keys (int64), exactly.

    Each product (W_ij mod m) * key_j is below m * m < 2^62 and is reduced
    before the next addition, so int64 never overflows.
    """
    out = np.zeros((keys.shape[0], len(W)), dtype=np.int64)
    for i in range(len(W)):
        acc = np.zeros(keys.shape[0], dtype=np.int64)
        for j in range(keys.shape[1]):
            c = int(W[i][j]) % m
            acc = (acc + (c * (keys[:, j] % m)) % m) % m
        out[:, i] = acc
    return out


def reduce_box_np(H, V):
    """Vectorised ``lattice.reduce_box`` for an (n, d) int64 array."""
    V = np.array(V, dtype=np.int64, copy=True)
    d = len(H)
    for i in range(d - 1, -1, -1):
        q = np.floor_divide(V[:, i], H[i][i])
        for r in range(i + 1):
            V[:, r] -= q * H[r][i]
    return V


def box_index_np(H, V):
    idx = np.zeros(V.shape[0], dtype=np.int64)
    for i in range(len(H)):
        idx = idx * H[i][i] + V[:, i]
    return idx


def _weights(M):
    """Integer matrix W = sgn(det M) adj(M) (so h^T M^{-1} g = h^T W g / m)."""
    D = L.det(M)
    A = L.adjugate(M)
    s = L.sign(D)
    return [[s * x for x in row] for row in A], abs(D)


def _residues(hk, wg, m):
    """(hk @ wg.T) mod m with every partial product reduced (no overflow)."""
    r = np.zeros((hk.shape[0], wg.shape[0]), dtype=np.int64)
    for i in range(hk.shape[1]):
        r = (r + (np.outer(hk[:, i] % m, wg[:, i]) % m)) % m
    return r


def lattice_dft_direct(M, a, inverse=False):
    """Direct O(m^2) sum of the definition (eq. Fouriermatrix).

    a: complex array of shape (..., m) in natural sample order of M (forward)
    or natural frequency order of M^T (inverse).  Returns complex128.
    Phases use the exact residue r = (h^T sgn(det M) adj(M) g) mod m and a
    float64 table exp(-2 pi i r / m).
    """
    M = L.as_matrix(M)
    W, m = _weights(M)
    g = natural_keys(M, "samples")
    h = natural_keys(M, "freqs")
    a = np.asarray(a, dtype=np.complex128)
    assert a.shape[-1] == m
    _check_size(m)
    wg = _modmatvec(W, g, m)                         # (W g) mod m for every g
    table = np.exp(-2j * np.pi * np.arange(m, dtype=np.float64) / m)
    out = np.zeros(a.shape, dtype=np.complex128)
    blk = max(1, (1 << 22) // m)
    src = a if not inverse else a
    for s in range(0, m, blk):
        e = min(m, s + blk)
        if not inverse:
            # rows h[s:e], columns g
            r = _residues(h[s:e], wg, m)                # (blk, m) residues
            F = table[r]
            out[..., s:e] = src @ F.T
        else:
            # inverse: a_g = m^{-1/2} sum_h ahat_h exp(+2 pi i h^T M^{-1} g)
            r = _residues(h, wg[s:e], m)                # (m_h, blk)
            F = np.conj(table[r])
            out[..., s:e] = src @ F
    return out / np.sqrt(m)


def direct_bins(M, a, hs):
    """Exact-residue O(m) sum for selected frequencies hs (list of int vectors).

    Used to spot-check any transform at sizes where the full O(m^2) sum is
    infeasible.  a: (m,) complex in natural sample order.
    """
    M = L.as_matrix(M)
    W, m = _weights(M)
    _check_size(m)
    g = natural_keys(M, "samples")
    a = np.asarray(a, dtype=np.complex128)
    res = []
    for hv in hs:
        # c_j = (sum_i h_i W_ij) mod m (Python ints), then r(g) = (c . g) mod m
        c = [sum(int(hv[i]) * W[i][j] for i in range(len(M))) % m for j in range(len(M))]
        r = _modmatvec([c], g, m)[:, 0]
        ph = np.exp(-2j * np.pi * r.astype(np.float64) / m)
        res.append(np.sum(a * ph) / np.sqrt(m))
    return np.array(res)


def _hnf_forward(M, a, workers):
    """Row/column FFT on the Hermite form (forward, sign -).

    With H = M U: h^T M^{-1} g = (U^T h)^T H^{-1} g.  Write T = H^{-1} =
    adj(H)/m (H upper triangular, det H = m).  For ht = U^T h reduced into the
    box of the lower-triangular lattice H^T Z^d, the exponent is
    sum_{i <= j} ht_i T_ij g_j, which is evaluated one axis j at a time:
    multiply by exp(-2 pi i (sum_{i<j} ht_i adj(H)_ij) g_j / m), an exact
    residue, then an FFT of length H_jj along g_j.
    Output is reordered to the natural frequency box of M^T.
    """
    M = L.as_matrix(M)
    d = len(M)
    H, U = L.hnf(M)
    m = abs(L.det(M))
    _check_size(m)
    shape = L.box_shape(H)
    a = np.asarray(a, dtype=np.complex128)
    batch = a.shape[:-1]
    X = a.reshape(batch + shape)
    adjH = L.adjugate(H)            # upper triangular, adj(H) = m H^{-1}
    nb = len(batch)
    for j in range(d):
        if j > 0:
            # twiddle exp(-2 pi i (sum_{i<j} ht_i adjH_ij) g_j / m)
            idx = [np.arange(shape[i], dtype=np.int64) for i in range(j + 1)]
            res = np.zeros(tuple(shape[:j]) + (1,), dtype=np.int64)
            for i in range(j):
                coef = adjH[i][j] % m
                v = (idx[i] * coef) % m
                res = (res + v.reshape([-1 if k == i else 1 for k in range(j + 1)])) % m
            gj = idx[j].reshape([1] * j + [-1])
            r = (res * gj) % m
            tw = np.exp(-2j * np.pi * r.astype(np.float64) / m)
            tw = tw.reshape(tw.shape + (1,) * (d - j - 1))
            X = X * tw
        X = scipy.fft.fft(X, axis=nb + j, workers=workers)
    # X is indexed by ht in prod [0, H_jj); map to natural h of M^T
    HT, _ = L.hnf(L.transpose(M))
    Uinv = L.inverse(U)             # integer (unimodular)
    UinvT = L.transpose(tuple(tuple(int(x) for x in row) for row in Uinv))
    ht = _natural_keys(H)           # the same box, enumerated in C order
    if max(abs(x) for row in UinvT for x in row) * m * d >= (1 << 62):
        raise ValueError("unimodular factor too large for int64")
    hv = ht @ np.array(UinvT, dtype=np.int64).T
    nat = box_index_np(HT, reduce_box_np(HT, hv))
    perm = np.empty(m, dtype=np.int64)
    perm[nat] = np.arange(m, dtype=np.int64)
    Y = X.reshape(batch + (m,))
    return Y[..., perm] / np.sqrt(m)


def lattice_dft_hnf(M, a, inverse=False, workers=None):
    """Hermite-form row/column FFT in float64 (independent of the Smith form).

    Forward as in ``_hnf_forward``.  The inverse uses F(M)^{-1} = F(M)^H and
    F(M)^T = F(M^T) (rows g in G(M), columns h in G(M^T)):
    F(M)^{-1} a = conj( F(M^T) conj(a) ).
    """
    if workers is None:
        workers = os.cpu_count() or 1
    M = L.as_matrix(M)
    if not inverse:
        return _hnf_forward(M, a, workers)
    a = np.asarray(a, dtype=np.complex128)
    return np.conj(_hnf_forward(L.transpose(M), np.conj(a), workers))
