"""Wavelet split for dilations with q = |det J| >= 2 channels, float64
(Section 5.3, steps 3-5 for general |det J|; Section 6.2 Dirichlet kernel).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings (each is listed in the design notes):
  * Fibers.  G(J^T) is enumerated in the natural order of the Hermite box of
    J^T, g_0 = 0.  For k in G(N^T) (natural box of N^T) the fiber positions
    are h_l = k + N^T g_l reduced into G(M^T), l = 0 .. q-1; every class of
    G(M^T) lies in exactly one fiber, at exactly one label l.
  * Scaling mask.  The quotient of the Dirichlet kernels' Fourier
    coefficients, c_k(phi_N) / c_k(phi_M) (Section 6.2 definition of the
    kernel), is sqrt(q) 2^{(r_M - r_N)/2} inside the closed N-box and 0
    outside; for q = 2 this is the printed mask.  It is evaluated on the
    symmetric representative of each class, as for q = 2.
  * Wavelet channels for q > 2.  The paper gives the Dirichlet wavelet only
    for q = 2.  Per fiber let u = (a(h_l) / sqrt q)_l (a unit vector by the
    QMF identity), sigma = 1 if u_0 >= 0 else -1, v = u + sigma e_0 (so
    v^T v >= 1) and H = I - 2 v v^T / (v^T v), the reflection that maps e_0
    to -sigma u.  The fiber matrix S has first row u and rows 1 .. q-1 those
    of H, so it is orthogonal.  Channel 0 is the scaling channel (symbol a);
    channel j >= 1 has the unnormalised symbol b_j(h_l) = sqrt(q) S[j, l].
    For q = 2 and u_0 >= 0 row 1 of S is -(u_1, -u_0): the printed wavelet
    channel is -phi times this one (the same wavelet translated by y0, with
    the opposite sign).
  * Step 4 with conjugated symbols (analysis is the adjoint of synthesis):
    dhat_j(k) = q^{-1/2} sum_l conj(b_j(h_l)) ahat(h_l); synthesis is the
    adjoint, ahat(h_l) = q^{-1/2} sum_j b_j(h_l) dhat_j(k).
  * Pyramid: channel 0 of a level is the input of the next (M_{l+1} = N_l);
    the coefficients of a level are its channels 1 .. q-1 back to back, each
    in natural sample order of N_l, and the last block is channel 0 of the
    last level:  [lvl 1: ch 1 | ... | ch q-1] ... [lvl L: ch 1 | ... ] [ch 0].

Pins: the time-domain definition d_{j,x} = <gamma, T(x) g_j> with
orthonormal translates (``split_direct_q``, O(m^2)); the Dirichlet kernel
relation c_k(phi_N) = a(h) c_k(phi_M) checked coefficient by coefficient
from the kernels' definitions; the QMF identity; Parseval and perfect
reconstruction; the q = 2 split of ``oracle.wavelet`` (an independent
implementation pinned to its own time-domain definition), which must equal
this split up to the per-fiber factor -phi; the one-dimensional closed form
of the mask.
"""
import numpy as np

from . import dft
from . import lattice as L
from . import wavelet as W


def classes(J):
    """Representatives g_0 = 0, ..., g_{q-1} of G(J^T) (int64, (q, d)), in
    the natural order of the Hermite box of J^T."""
    return dft.natural_keys(J, "freqs")


def fiber_maps(M, J):
    """(N, idx, m): idx[l, k] is the natural index in G(M^T) of
    h_l = k + N^T g_l for every natural k in G(N^T)."""
    M = L.as_matrix(M)
    N = W.quotient(J, M)
    NT = np.array(L.transpose(N), dtype=np.int64)
    g = classes(J)
    HMT, _ = L.hnf(L.transpose(M))
    k = dft.natural_keys(N, "freqs")
    q = g.shape[0]
    idx = np.zeros((q, k.shape[0]), dtype=np.int64)
    for l in range(q):
        h = dft.reduce_box_np(HMT, k + (NT @ g[l]))
        idx[l] = dft.box_index_np(HMT, h)
    return N, idx, abs(L.det(M))


def dirichlet_mask(M, N):
    """Dirichlet scaling mask on natural G(M^T) for M = J N, any q = m / n:
    sqrt(q) 2^{(r_M - r_N)/2} inside the closed N-box, 0 outside."""
    M = L.as_matrix(M)
    N = L.as_matrix(N)
    q = abs(L.det(M)) // abs(L.det(N))
    d = len(M)
    hk = dft.natural_keys(M, "freqs")
    t, m = W._sym_t(M, hk)
    rM = np.sum(2 * t == -m, axis=1)
    MT = L.transpose(M)
    hs = np.zeros_like(t)
    for i in range(d):
        acc = np.zeros(t.shape[0], dtype=np.int64)
        for j in range(d):
            acc += MT[i][j] * t[:, j]
        assert np.all(acc % m == 0)
        hs[:, i] = acc // m
    DN = L.det(N)
    n = abs(DN)
    AN = L.adjugate(N)
    sN = L.sign(DN)
    w = np.zeros_like(hs)
    for j in range(d):
        acc = np.zeros(hs.shape[0], dtype=np.int64)
        for k in range(d):
            acc += sN * AN[k][j] * hs[:, k]
        w[:, j] = acc
    inside = np.all(np.abs(2 * w) <= n, axis=1)
    rN = np.sum(np.abs(2 * w) == n, axis=1)
    return np.where(inside, np.sqrt(float(q)) * 2.0 ** ((rM - rN) / 2.0), 0.0)


def default_masks(M, J, levels):
    return [dirichlet_mask(Ml, Nl) for (Ml, Nl) in W.level_matrices(M, J, levels)]


def householder(u):
    """Per-fiber matrices S (q, q, n): row 0 is u, rows j >= 1 those of
    H = I - 2 v v^T / (v^T v), v = u + sigma e_0, sigma = sign(u_0) (+1 at 0)."""
    u = np.asarray(u, dtype=np.float64)
    q, n = u.shape
    sigma = np.where(u[0] >= 0, 1.0, -1.0)
    v = u.copy()
    v[0] += sigma
    vv = np.sum(v * v, axis=0)
    S = np.zeros((q, q, n), dtype=np.float64)
    for j in range(q):
        for l in range(q):
            S[j, l] = (1.0 if j == l else 0.0) - 2.0 * v[j] * v[l] / vv
    S[0] = u
    return S


def symbols(M, J, mask):
    """Unnormalised channel symbols b_j on natural G(M^T), (q, m) complex:
    b_0 = a and b_j(h_l) = sqrt(q) S[j, l] on every fiber."""
    N, idx, m = fiber_maps(M, J)
    q = idx.shape[0]
    mask = np.asarray(mask, dtype=np.float64)
    S = householder(mask[idx] / np.sqrt(q))
    b = np.zeros((q, m), dtype=np.complex128)
    for j in range(q):
        for l in range(q):
            b[j, idx[l]] = np.sqrt(q) * S[j, l]
    return b


def split(M, J, ahat, mask):
    """One level: ahat (..., m) on natural G(M^T) -> dhat (..., q, m/q), each
    channel in natural G(N^T) order (Section 5.3 step 4)."""
    N, idx, m = fiber_maps(M, J)
    q = idx.shape[0]
    b = symbols(M, J, mask)
    ahat = np.asarray(ahat, dtype=np.complex128)
    out = np.zeros(ahat.shape[:-1] + (q, idx.shape[1]), dtype=np.complex128)
    for j in range(q):
        for l in range(q):
            out[..., j, :] += np.conj(b[j, idx[l]]) * ahat[..., idx[l]]
    return out / np.sqrt(q)


def unsplit(M, J, dhat, mask):
    """Synthesis (adjoint of ``split``): (..., q, m/q) -> (..., m)."""
    N, idx, m = fiber_maps(M, J)
    q = idx.shape[0]
    b = symbols(M, J, mask)
    dhat = np.asarray(dhat, dtype=np.complex128)
    out = np.zeros(dhat.shape[:-2] + (m,), dtype=np.complex128)
    for l in range(q):
        acc = np.zeros(dhat.shape[:-2] + (idx.shape[1],), dtype=np.complex128)
        for j in range(q):
            acc += b[j, idx[l]] * dhat[..., j, :]
        out[..., idx[l]] = acc / np.sqrt(q)
    return out


def _fft(M, x, inverse, direct):
    if direct:
        return dft.lattice_dft_direct(M, x, inverse=inverse)
    return dft.lattice_dft_hnf(M, x, inverse=inverse)


def coeff_layout(M, J, levels):
    """[(level, channel, offset, size)] of the coefficient blocks."""
    mats = W.level_matrices(M, J, levels)
    q = abs(L.det(L.as_matrix(J)))
    out, off = [], 0
    for lvl, (_, Nl) in enumerate(mats):
        n = abs(L.det(Nl))
        for j in range(1, q):
            out.append((lvl, j, off, n))
            off += n
    n = abs(L.det(mats[-1][1]))
    out.append((levels - 1, 0, off, n))
    return out


def decompose(x, M, J, levels, masks=None, direct=False):
    """Multi-level q-channel pyramid; x (..., m) natural samples of P(M)."""
    mats = W.level_matrices(M, J, levels)
    if masks is None:
        masks = [dirichlet_mask(Ml, Nl) for (Ml, Nl) in mats]
    ahat = _fft(mats[0][0], x, False, direct)
    blocks = []
    for (Ml, Nl), mk in zip(mats, masks):
        dh = split(Ml, J, ahat, mk)
        for j in range(1, dh.shape[-2]):
            blocks.append(_fft(Nl, dh[..., j, :], True, direct))
        ahat = dh[..., 0, :]
    blocks.append(_fft(mats[-1][1], ahat, True, direct))
    return np.concatenate(blocks, axis=-1)


def reconstruct(coeffs, M, J, levels, masks=None, direct=False):
    """Inverse of ``decompose``."""
    mats = W.level_matrices(M, J, levels)
    if masks is None:
        masks = [dirichlet_mask(Ml, Nl) for (Ml, Nl) in mats]
    coeffs = np.asarray(coeffs, dtype=np.complex128)
    q = abs(L.det(L.as_matrix(J)))
    lay = coeff_layout(M, J, levels)
    _, _, off, n = lay[-1]
    ahat = _fft(mats[-1][1], coeffs[..., off:off + n], False, direct)
    for lvl in range(levels - 1, -1, -1):
        Ml, Nl = mats[lvl]
        n = abs(L.det(Nl))
        dh = np.zeros(coeffs.shape[:-1] + (q, n), dtype=np.complex128)
        dh[..., 0, :] = ahat
        for (lv, j, off, size) in lay:
            if lv == lvl and j > 0:
                dh[..., j, :] = _fft(Nl, coeffs[..., off:off + size], False, direct)
        ahat = unsplit(Ml, J, dh, masks[lvl])
    return _fft(mats[0][0], ahat, True, direct)


def split_direct_q(M, J, a, mask):
    """Time-domain definition the split must equal (O(m^2)): with the
    filters b_{j,y} = m^{-1} sum_h b_j(h) exp(+2 pi i h^T y) of the channel
    symbols, d_{j,x} = sum_{y in P(M)} a_y conj(b_{j, y - x}) for x in P(N).
    Returns (q, n) in natural sample order of N."""
    M = L.as_matrix(M)
    N = W.quotient(J, M)
    m = abs(L.det(M))
    HM, _ = L.hnf(M)
    b = symbols(M, J, mask)
    q = b.shape[0]
    filt = np.stack([dft.lattice_dft_direct(M, b[j], inverse=True) / np.sqrt(m) for j in range(q)])
    g = dft.natural_keys(M, "samples")
    k = dft.natural_keys(N, "samples")
    Jm = np.array(L.as_matrix(J), dtype=np.int64)
    xk = k @ Jm.T                              # keys J k in G(M)
    a = np.asarray(a, dtype=np.complex128)
    d = np.zeros((q, k.shape[0]), dtype=np.complex128)
    for p in range(k.shape[0]):
        diff = dft.box_index_np(HM, dft.reduce_box_np(HM, g - xk[p]))
        d[:, p] = np.sum(a[None, :] * np.conj(filt[:, diff]), axis=1)
    return d
