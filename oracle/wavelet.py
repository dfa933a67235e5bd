"""Fast lattice wavelet decomposition, float64 (Sections 5.1-5.3 and 6.2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings of the paper used here (each is listed in the design notes):
  * The dilation J has |det J| = 2, M = J N with N integral (Section 5.3).
  * Masks are unnormalised symbols (eq. subspaces-coeffs): the low-pass
    symbol a(h) on G(M^T) satisfies the QMF identity
    sum_{l in G(J^T)} |a(h + N^T l)|^2 = |det J|, and the signal transform
    ahat = F(M) x is unitary.
  * Step 4 of Section 5.3 is read with the filter symbols conjugated
    (analysis is the adjoint of synthesis); for the real scaling mask this
    changes nothing, for the complex wavelet symbol it is required.
  * Wavelet symbol (Section 6.2, Dirichlet wavelet): with g0 the non-zero
    class of G(J^T), s = N^T g0, and y0 the non-zero point of P(J) taken in
    [-1/2, 1/2)^d, b2(h) = conj(a(h + s)) * phi(h), phi(h) = exp(-2 pi i
    h^T N^{-1} y0) = exp(-2 pi i h^T M^{-1} v), v = J y0.
  * Dirichlet mask (Section 6.2): evaluated on the symmetric representative
    h* of each class, with the closed N-box test |N^{-T} h*|_j <= 1/2.

Per fiber {h0, h0 + s} over k in G(N^T), with a0 = a(h0), a1 = a(h0 + s),
phi0 = phi(h0) (and phi(h0 + s) = -phi0):
    d1hat(k) = (a0 ahat(h0) + a1 ahat(h0+s)) / sqrt 2
    d2hat(k) = conj(phi0) (a1 ahat(h0) - a0 ahat(h0+s)) / sqrt 2
and the inverse (the 2x2 matrix is unitary when a0^2 + a1^2 = 2):
    ahat(h0)   = (a0 d1hat + a1 phi0 d2hat) / sqrt 2
    ahat(h0+s) = (a1 d1hat - a0 phi0 d2hat) / sqrt 2

Pins: ``split_direct`` (the time-domain inner products the split must
equal: d_{j,x} = <gamma, T(x) g_j> with orthonormal translates), Parseval
sum_j ||d_j||^2 = ||a||^2, perfect reconstruction, the QMF identity of the
mask, and the 1-D closed form of the Dirichlet mask for diagonal M.
"""
import numpy as np

from . import dft
from . import lattice as L


def quotient(J, M):
    """N = J^{-1} M exactly; raises ValueError if it is not integral."""
    Jinv = L.inverse(J)
    N = L.matmul(Jinv, L.as_matrix(M))
    if any(x.denominator != 1 for row in N for x in row):
        raise ValueError("J^{-1} M is not integral")
    return tuple(tuple(int(x) for x in row) for row in N)


def level_matrices(M, J, levels):
    """[(M_1, N_1), ..., (M_L, N_L)] with M_1 = M, N_l = J^{-1} M_l,
    M_{l+1} = N_l (Section 5.3: later steps split the low-pass space)."""
    out = []
    Ml = L.as_matrix(M)
    for _ in range(levels):
        Nl = quotient(J, Ml)
        out.append((Ml, Nl))
        Ml = Nl
    return out


def dilation_data(J):
    """(g0, y0, v) for |det J| = 2.

    g0: an integer vector whose class is the non-zero element of G(J^T).
    y0: the non-zero element of P(J) in [-1/2, 1/2)^d (as Fractions).
    v = J y0 (integer).
    """
    J = L.as_matrix(J)
    d = len(J)
    if abs(L.det(J)) != 2:
        raise ValueError("only |det J| = 2 is supported")
    JT = L.transpose(J)
    JTinv = L.inverse(JT)
    Jinv = L.inverse(J)
    g0 = None
    for i in range(d):
        e = [int(k == i) for k in range(d)]
        if any(x.denominator != 1 for x in L.matvec(JTinv, e)):
            g0 = tuple(e)
            break
    y0 = None
    for i in range(d):
        e = [int(k == i) for k in range(d)]
        y = L.matvec(Jinv, e)
        if any(x.denominator != 1 for x in y):
            # reduce into [-1/2, 1/2)
            y0 = tuple(x - ((x + L.Fraction(1, 2)) // 1) for x in y)
            break
    assert g0 is not None and y0 is not None
    v = L.matvec(J, y0)
    assert all(x.denominator == 1 for x in v)
    v = tuple(int(x) for x in v)
    return g0, y0, v


def _sym_t(M, hk):
    """t with M^{-T} h = t/m, reduced into [-m/2, m/2) (vectorised, exact)."""
    D = L.det(M)
    m = abs(D)
    A = L.adjugate(M)
    s = L.sign(D)
    d = len(M)
    # row j of (s adj(M)^T) is s * column j of adj(M)
    W = [[s * A[k][j] for k in range(d)] for j in range(d)]
    t = dft._modmatvec(W, hk, m)
    half = m // 2
    return ((t + half) % m) - half, m


def dirichlet_mask(M, N):
    """Dirichlet scaling mask a(h) on natural G(M^T) (Section 6.2), float64.

    For each class h: h* is its symmetric representative, r_M the number of
    coordinates of M^{-T} h* equal to -1/2, w/n = N^{-T} h*.  If
    |w_j/n| <= 1/2 for all j the value is 2^{(1 + r_M - r_N)/2} with r_N the
    number of coordinates where |w_j/n| = 1/2, otherwise 0.
    """
    M = L.as_matrix(M)
    N = L.as_matrix(N)
    d = len(M)
    hk = dft.natural_keys(M, "freqs")
    t, m = _sym_t(M, hk)
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
    val = np.where(inside, 2.0 ** ((1 + rM - rN) / 2.0), 0.0)
    return val


def _fiber_maps(M, J):
    """Natural-index maps of the fibers and the wavelet phase residues.

    Returns (N, i0, i1, rho, m) where, for every natural k in G(N^T),
    i0[k] is the natural index in G(M^T) of k, i1[k] that of k + s, and
    rho[k] the residue with phi(h0) = exp(-2 pi i rho/m).
    """
    M = L.as_matrix(M)
    N = quotient(J, M)
    g0, y0, v = dilation_data(J)
    NT = L.transpose(N)
    s = L.matvec(NT, g0)
    HMT, _ = L.hnf(L.transpose(M))
    k = dft.natural_keys(N, "freqs")
    h0 = dft.reduce_box_np(HMT, k)
    h1 = dft.reduce_box_np(HMT, k + np.array(s, dtype=np.int64))
    i0 = dft.box_index_np(HMT, h0)
    i1 = dft.box_index_np(HMT, h1)
    W, m = dft._weights(M)
    c = [sum(W[i][j] * v[j] for j in range(len(M))) % m for i in range(len(M))]
    rho = dft._modmatvec([c], h0, m)[:, 0]
    return N, i0, i1, rho, m


def split(M, J, ahat, mask):
    """One decomposition level in the Fourier domain (Section 5.3, step 4).

    ahat: (..., m) natural G(M^T) order; mask: (m,) real.  Returns
    (d1hat, d2hat), each (..., m/2) in natural G(N^T) order.
    """
    N, i0, i1, rho, m = _fiber_maps(M, J)
    ahat = np.asarray(ahat, dtype=np.complex128)
    a0 = np.asarray(mask, dtype=np.float64)[i0]
    a1 = np.asarray(mask, dtype=np.float64)[i1]
    x0 = ahat[..., i0]
    x1 = ahat[..., i1]
    phi = np.exp(-2j * np.pi * rho.astype(np.float64) / m)
    r2 = np.sqrt(2.0)
    d1 = (a0 * x0 + a1 * x1) / r2
    d2 = np.conj(phi) * (a1 * x0 - a0 * x1) / r2
    return d1, d2


def unsplit(M, J, d1hat, d2hat, mask):
    """Inverse of ``split`` (synthesis): returns ahat in natural G(M^T) order."""
    N, i0, i1, rho, m = _fiber_maps(M, J)
    d1 = np.asarray(d1hat, dtype=np.complex128)
    d2 = np.asarray(d2hat, dtype=np.complex128)
    a0 = np.asarray(mask, dtype=np.float64)[i0]
    a1 = np.asarray(mask, dtype=np.float64)[i1]
    phi = np.exp(-2j * np.pi * rho.astype(np.float64) / m)
    r2 = np.sqrt(2.0)
    out = np.zeros(d1.shape[:-1] + (m,), dtype=np.complex128)
    out[..., i0] = (a0 * d1 + a1 * phi * d2) / r2
    out[..., i1] = (a1 * d1 - a0 * phi * d2) / r2
    return out


def _fft(M, x, inverse, direct):
    if direct:
        return dft.lattice_dft_direct(M, x, inverse=inverse)
    return dft.lattice_dft_hnf(M, x, inverse=inverse)


def default_masks(M, J, levels):
    return [dirichlet_mask(Ml, Nl) for (Ml, Nl) in level_matrices(M, J, levels)]


def decompose(x, M, J, levels, masks=None, direct=False):
    """Multi-level pyramid (Section 5.3: one FFT, then steps 2-4 on d1hat).

    x: (..., m) natural samples of P(M).  Returns (..., m) coefficients laid
    out as [d2^(1) | d2^(2) | ... | d2^(L) | d1^(L)], each block in natural
    sample order of its N_l.
    """
    mats = level_matrices(M, J, levels)
    if masks is None:
        masks = [dirichlet_mask(Ml, Nl) for (Ml, Nl) in mats]
    ahat = _fft(mats[0][0], x, False, direct)
    blocks = []
    for (Ml, Nl), mk in zip(mats, masks):
        d1, d2 = split(Ml, J, ahat, mk)
        blocks.append(_fft(Nl, d2, True, direct))
        ahat = d1
    blocks.append(_fft(mats[-1][1], ahat, True, direct))
    return np.concatenate(blocks, axis=-1)


def reconstruct(coeffs, M, J, levels, masks=None, direct=False):
    """Inverse of ``decompose`` (synthesis: gamma = sum_j sum_y d_{j,y} T(y) g_j)."""
    mats = level_matrices(M, J, levels)
    if masks is None:
        masks = [dirichlet_mask(Ml, Nl) for (Ml, Nl) in mats]
    coeffs = np.asarray(coeffs, dtype=np.complex128)
    sizes = [abs(L.det(Nl)) for (_, Nl) in mats]
    offs = np.cumsum([0] + sizes)
    d1 = coeffs[..., offs[-1]:offs[-1] + sizes[-1]]
    ahat = _fft(mats[-1][1], d1, False, direct)
    for lvl in range(levels - 1, -1, -1):
        Ml, Nl = mats[lvl]
        d2 = _fft(Nl, coeffs[..., offs[lvl]:offs[lvl] + sizes[lvl]], False, direct)
        ahat = unsplit(Ml, J, ahat, d2, masks[lvl])
    return _fft(mats[0][0], ahat, True, direct)


def filters_time_domain(M, J, mask):
    """Time-domain filters b_j on natural G(M) for the two channels.

    b_j[g] = m^{-1} sum_h bhat_j(h) exp(+2 pi i h^T M^{-1} g) with the
    unnormalised symbols bhat_1 = a, bhat_2(h) = conj(a(h+s)) phi(h).
    """
    M = L.as_matrix(M)
    m = abs(L.det(M))
    N = quotient(J, M)
    g0, y0, v = dilation_data(J)
    s = L.matvec(L.transpose(N), g0)
    HMT, _ = L.hnf(L.transpose(M))
    h = dft.natural_keys(M, "freqs")
    partner = dft.box_index_np(HMT, dft.reduce_box_np(HMT, h + np.array(s)))
    W, _ = dft._weights(M)
    c = [sum(W[i][j] * v[j] for j in range(len(M))) % m for i in range(len(M))]
    rho = dft._modmatvec([c], h, m)[:, 0]
    phi = np.exp(-2j * np.pi * rho.astype(np.float64) / m)
    mask = np.asarray(mask, dtype=np.float64)
    b1hat = mask.astype(np.complex128)
    b2hat = np.conj(mask[partner]) * phi
    # inverse unnormalised transform: b = m^{-1/2} F(M)^{-1} bhat
    b1 = dft.lattice_dft_direct(M, b1hat, inverse=True) / np.sqrt(m)
    b2 = dft.lattice_dft_direct(M, b2hat, inverse=True) / np.sqrt(m)
    return b1, b2


def split_direct(M, J, a, mask):
    """The plain definition the split must equal (time domain, O(m^2)).

    With orthonormal translates T(y) f (Section 6.2), g_j = sum_y b_{j,y}
    T(y) f and gamma = sum_y a_y T(y) f:
        d_{j,x} = <gamma, T(x) g_j> = sum_{y in P(M)} a_y conj(b_{j, y - x})
    for x in P(N).  A point x = N^{-1} k of P(N) has key J k in G(M).
    Returns (d1, d2) in natural sample order of N.
    """
    M = L.as_matrix(M)
    N = quotient(J, M)
    HM, _ = L.hnf(M)
    b1, b2 = filters_time_domain(M, J, mask)
    g = dft.natural_keys(M, "samples")
    k = dft.natural_keys(N, "samples")
    Jm = np.array(L.as_matrix(J), dtype=np.int64)
    xk = k @ Jm.T                              # keys J k in G(M)
    a = np.asarray(a, dtype=np.complex128)
    d1 = np.zeros(k.shape[0], dtype=np.complex128)
    d2 = np.zeros(k.shape[0], dtype=np.complex128)
    for p in range(k.shape[0]):
        diff = dft.box_index_np(HM, dft.reduce_box_np(HM, g - xk[p]))
        d1[p] = np.sum(a * np.conj(b1[diff]))
        d2[p] = np.sum(a * np.conj(b2[diff]))
    return d1, d2
