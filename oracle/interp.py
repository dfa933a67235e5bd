"""Change of basis between point values and orthonormal-translate
coefficients of V_M^phi (Section 6.2: the samples of a function are turned
into coefficients in the basis of the translates T(y) phi_M before the
wavelet decomposition; Section 5.1, eq. subspaces-coeffs, for the spaces of
translates).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Reading (the corollary the paper cites is not in the text; this is derived
from the relations the paper states).  A function g = sum_y a_y T(y) phi of
V_M^phi, sampled at the points 2 pi x, x in P(M), gives

    s_x = sum_y a_y phi(2 pi (x - y)),

a cyclic convolution over P(M).  On the pattern, exp(i k^T 2 pi z) depends
only on the class h of k in G(M^T), so phi(2 pi z) = sum_h theta_h
exp(2 pi i h^T z) with the bracket sum theta_h = sum_{k = h mod M^T Z^d}
c_k(phi).  With the unitary F(M) of eq. Fouriermatrix this is the pointwise
relation

    (F(M) s)_h = m theta_h (F(M) a)_h,

so a = F(M)^{-1} [ (F(M) s) / (m theta) ] whenever no theta_h vanishes.  For
the Dirichlet kernel phi_M the coefficients m^{-1/2} 2^{-r(k)/2} on the
closed cube M^{-T} k in [-1/2, 1/2]^d give theta_h = m^{-1/2} 2^{r(h)/2}
(each class on r boundary hyperplanes has 2^r members in the closed cube),
so m theta_h = sqrt(m) 2^{r(h)/2}.

Pins: the interpolation property (the coefficients, put back into the
translates of phi_M whose samples come from its Fourier series summed
directly over the closed cube, reproduce the samples exactly), the
orthonormality of those translates (Gram matrix by Parseval), the bracket sum
counted member by member with exact rationals, and the closed form for odd m
(no boundary classes: a = s / sqrt(m)).
"""
from fractions import Fraction
from itertools import product

import numpy as np

from . import dft
from . import lattice as L
from . import wavelet as W


def dirichlet_r(M):
    """r_M(h) for every class h of G(M^T) in natural order: the number of
    coordinates of M^{-T} h (symmetric representative, [-1/2, 1/2)) equal to
    -1/2 (Section 6.2)."""
    M = L.as_matrix(M)
    t, m = W._sym_t(M, dft.natural_keys(M, "freqs"))
    return np.sum(2 * t == -m, axis=1).astype(np.int64)


def dirichlet_bracket_factor(M):
    """m theta_h = sqrt(m) 2^{r(h)/2} for the Dirichlet kernel phi_M, every
    class h in natural G(M^T) order (float64)."""
    m = abs(L.det(L.as_matrix(M)))
    return np.sqrt(float(m)) * 2.0 ** (dirichlet_r(M) / 2.0)


def samples_to_coeffs(M, s, fourier=False):
    """Coefficients in the orthonormal translates of phi_M of the function of
    V_M^phi with point values s (natural P(M) order, shape (..., m)).
    fourier=True returns F(M) a in natural G(M^T) order instead of a."""
    s = np.asarray(s, dtype=np.complex128)
    ahat = _fft(M, s, False) / dirichlet_bracket_factor(M)
    return ahat if fourier else _fft(M, ahat, True)


def coeffs_to_samples(M, a, fourier=False):
    """Inverse of samples_to_coeffs: point values of sum_y a_y T(y) phi_M
    (fourier=True: the input is F(M) a)."""
    a = np.asarray(a, dtype=np.complex128)
    ahat = a if fourier else _fft(M, a, False)
    return _fft(M, ahat * dirichlet_bracket_factor(M), True)


def _fft(M, x, inverse):
    m = abs(L.det(L.as_matrix(M)))
    if m <= 4096:
        return dft.lattice_dft_direct(M, x, inverse=inverse)
    return dft.lattice_dft_hnf(M, x, inverse=inverse)


# ---------------------------------------------------------------------------
# Brute-force pieces used only by the pins

def dirichlet_coefficients(M):
    """{k: c_k(phi_M)} over the integer points k of the closed cube
    M^{-T} k in [-1/2, 1/2]^d, exact: m^{-1/2} 2^{-r(k)/2} is returned as the
    pair (r(k), m) so callers can stay exact where they need to."""
    M = L.as_matrix(M)
    d = len(M)
    m = abs(L.det(M))
    MT = L.transpose(M)
    MTinv = L.inverse(MT)
    # bounding box of M^T [-1/2, 1/2]^d
    lo = [0] * d
    hi = [0] * d
    for corner in product((Fraction(-1, 2), Fraction(1, 2)), repeat=d):
        img = L.matvec(MT, corner)
        for i in range(d):
            lo[i] = min(lo[i], int(np.floor(float(img[i]))) - 1)
            hi[i] = max(hi[i], int(np.ceil(float(img[i]))) + 1)
    out = {}
    for k in product(*[range(lo[i], hi[i] + 1) for i in range(d)]):
        u = L.matvec(MTinv, k)
        if all(abs(c) <= Fraction(1, 2) for c in u):
            out[k] = (sum(1 for c in u if abs(c) == Fraction(1, 2)), m)
    return out


def kernel_samples(M):
    """phi_M(2 pi z) for every sample z of P(M) in natural order, summed
    directly from its Fourier series (the coefficients of
    dirichlet_coefficients)."""
    M = L.as_matrix(M)
    m = abs(L.det(M))
    coeffs = dirichlet_coefficients(M)
    gk = dft.natural_keys(M, "samples")
    Minv = L.inverse(M)
    out = np.zeros(m, dtype=np.complex128)
    for i, g in enumerate(gk):
        z = L.matvec(Minv, tuple(int(v) for v in g))
        acc = 0j
        for k, (r, _) in coeffs.items():
            ph = sum(Fraction(kk) * zz for kk, zz in zip(k, z))
            acc += np.exp(2j * np.pi * float(ph - (ph.numerator // ph.denominator))) * 2.0 ** (-r / 2)
        out[i] = acc / np.sqrt(m)
    return out


def interpolant_values(M, a):
    """sum_y a_y phi_M(2 pi (x - y)) at every sample x of P(M), O(m^2), with
    phi_M's samples from kernel_samples (differences reduced into the box)."""
    M = L.as_matrix(M)
    H, _ = L.hnf(M)
    gk = [tuple(int(v) for v in g) for g in dft.natural_keys(M, "samples")]
    phi = kernel_samples(M)
    a = np.asarray(a, dtype=np.complex128)
    out = np.zeros(a.shape, dtype=np.complex128)
    for ix, x in enumerate(gk):
        for iy, y in enumerate(gk):
            j = L.natural_index(H, tuple(p - q for p, q in zip(x, y)))
            out[..., ix] += a[..., iy] * phi[j]
    return out


def translates_gram(M):
    """Gram matrix <T(y) phi_M, T(y') phi_M> over P(M) by Parseval:
    sum_k |c_k|^2 exp(-2 pi i k^T (y - y'))."""
    M = L.as_matrix(M)
    m = abs(L.det(M))
    coeffs = dirichlet_coefficients(M)
    gk = [tuple(int(v) for v in g) for g in dft.natural_keys(M, "samples")]
    Minv = L.inverse(M)
    ys = [L.matvec(Minv, g) for g in gk]
    G = np.zeros((m, m), dtype=np.complex128)
    for i, y in enumerate(ys):
        for j, yp in enumerate(ys):
            acc = 0j
            for k, (r, _) in coeffs.items():
                ph = sum(Fraction(kk) * (p - q) for kk, p, q in zip(k, y, yp))
                acc += np.exp(-2j * np.pi * float(ph - (ph.numerator // ph.denominator))) * 2.0 ** (-r)
            G[i, j] = acc / m
    return G
