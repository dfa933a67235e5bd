"""Pins of the oracle's lattice DFT (eq. Fouriermatrix) against library routines,
closed forms and invariants."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import dft, lattice as L
import workloads


def _rand(seed, n, batch=()):
    return workloads.complex_normal(seed, tuple(batch) + (n,), np.complex128)


@pytest.mark.parametrize("shape", [(8,), (4, 6), (5, 3), (2, 3, 4)])
def test_diagonal_equals_fftn(shape):
    """Diagonal M: F(M) is the tensor-product DFT with unitary scaling
    (Kronecker form of Section 4.1 with identity permutations)."""
    d = len(shape)
    if d == 1:
        M = ((shape[0],),)
    else:
        M = tuple(tuple(shape[i] if i == j else 0 for j in range(d)) for i in range(d))
    m = int(np.prod(shape))
    a = _rand(1, m)
    ref = np.fft.fftn(a.reshape(shape), norm="ortho").reshape(-1)
    np.testing.assert_allclose(dft.lattice_dft_direct(M, a), ref, atol=1e-12)
    np.testing.assert_allclose(dft.lattice_dft_hnf(M, a), ref, atol=1e-12)
    np.testing.assert_allclose(dft.lattice_dft_direct(M, ref, inverse=True), a, atol=1e-12)


def test_block_diagonal_is_kronecker():
    """M = diag(A, B): F(M) = F(A) (x) F(B) on the product of natural boxes."""
    A = ((3, 1), (1, 2))            # det 5
    M = ((3, 1, 0), (1, 2, 0), (0, 0, 4))
    a = _rand(2, 20)
    out = dft.lattice_dft_direct(M, a)
    HA, _ = L.hnf(A)
    # natural box of M = box(A) x [0,4) because H_M = diag(H_A, 4)
    HM, _ = L.hnf(M)
    assert HM == ((HA[0][0], HA[0][1], 0), (0, HA[1][1], 0), (0, 0, 4))
    HMT, _ = L.hnf(L.transpose(M))
    HAT, _ = L.hnf(L.transpose(A))
    assert HMT == ((HAT[0][0], HAT[0][1], 0), (0, HAT[1][1], 0), (0, 0, 4))
    X = a.reshape(5, 4)
    Y = np.stack([dft.lattice_dft_direct(A, X[:, j]) for j in range(4)], axis=1)
    Y = np.fft.fft(Y, axis=1, norm="ortho")
    np.testing.assert_allclose(out, Y.reshape(-1), atol=1e-12)


MATS = [((32, 8), (-8, 32)), ((4, -3), (4, 5)), ((5, 2), (1, 3)), ((12, 4), (0, 6)),
        ((3, 1, 0), (0, 3, 1), (1, 0, 3)), ((-7, 2), (3, 5)), ((16, 8), (0, 16))]


@pytest.mark.parametrize("M", MATS)
def test_plane_wave_is_delta(M):
    """a_g = exp(+2 pi i h0^T M^{-1} g) transforms to sqrt(m) at h0 and 0
    elsewhere.  Phases here are computed with exact rational arithmetic from
    M^{-1}, not with the residue code under test."""
    m = abs(L.det(M))
    Minv = L.inverse(M)
    g = dft.natural_keys(M, "samples")
    h = dft.natural_keys(M, "freqs")
    for p in (0, 1, m // 2, m - 1):
        h0 = tuple(int(x) for x in h[p])
        ph = []
        for gv in g:
            r = sum(h0[i] * Minv[i][j] * int(gv[j]) for i in range(len(M)) for j in range(len(M)))
            r = r - (r.numerator // r.denominator)
            ph.append(np.exp(2j * np.pi * float(r)))
        out = dft.lattice_dft_direct(M, np.array(ph))
        ref = np.zeros(m, complex)
        ref[p] = np.sqrt(m)
        np.testing.assert_allclose(out, ref, atol=1e-10)


@pytest.mark.parametrize("M", MATS)
def test_impulse_parseval_inverse(M):
    m = abs(L.det(M))
    e = np.zeros(m, complex)
    e[0] = 1
    np.testing.assert_allclose(dft.lattice_dft_direct(M, e), np.full(m, 1 / np.sqrt(m)), atol=1e-14)
    a = _rand(3, m, (2,))
    A = dft.lattice_dft_direct(M, a)
    np.testing.assert_allclose(np.linalg.norm(A, axis=-1), np.linalg.norm(a, axis=-1), rtol=1e-13)
    np.testing.assert_allclose(dft.lattice_dft_direct(M, A, inverse=True), a, atol=1e-12)


@pytest.mark.parametrize("M", MATS)
def test_hnf_fft_equals_direct(M):
    """Two independent algorithms agree (Hermite row/column FFT vs the sum)."""
    m = abs(L.det(M))
    a = _rand(4, m, (3,))
    A = dft.lattice_dft_direct(M, a)
    np.testing.assert_allclose(dft.lattice_dft_hnf(M, a), A, atol=1e-12)
    np.testing.assert_allclose(dft.lattice_dft_hnf(M, A, inverse=True), a, atol=1e-12)


@pytest.mark.parametrize("seed", range(10))
def test_hnf_fft_equals_direct_random(seed):
    rng = np.random.default_rng(500 + seed)
    d = 2 + seed % 2
    M = workloads.random_regular_matrix(rng, d, max_det=2000)
    m = abs(L.det(M))
    a = _rand(seed, m)
    np.testing.assert_allclose(dft.lattice_dft_hnf(M, a), dft.lattice_dft_direct(M, a), atol=1e-11)


def test_hnf_fft_equals_direct_2_14():
    M = ((128, 32), (0, 128))
    a = _rand(5, 1 << 14)
    np.testing.assert_allclose(dft.lattice_dft_hnf(M, a), dft.lattice_dft_direct(M, a), atol=1e-11)


def test_direct_bins_large():
    """Sampled exact bins against the Hermite FFT at m = 2^20."""
    M = ((1024, 256), (0, 1024))
    a = _rand(6, 1 << 20)
    A = dft.lattice_dft_hnf(M, a)
    HT, _ = L.hnf(L.transpose(M))
    hs = [(0, 0), (1, 0), (4095, 255), (1234, 77)]
    bins = dft.direct_bins(M, a, hs)
    np.testing.assert_allclose(bins, A[[L.natural_index(HT, h) for h in hs]], atol=1e-10)
