"""Pins of the oracle's q-channel split (Section 5.3, step 4 for |det J| = q)
and the Dirichlet mask for any q (Section 6.2 kernel definitions): the
time-domain definition, the kernels' coefficient relation, QMF, Parseval,
perfect reconstruction, the independent q = 2 oracle and closed forms."""
from fractions import Fraction
from itertools import product

import numpy as np
import pytest

from oracle import dft, lattice as L, wavelet as W, wavelet_q as Q
import workloads

J2 = ((2, 0), (0, 2))
J21 = ((2, 1), (0, 2))
J3 = ((3, 0), (0, 1))
JR = ((0, -2), (2, 0))                     # J_d squared: rotation by 90 degrees, scale 2
J2_3D = ((2, 0, 0), (0, 2, 0), (0, 0, 2))

PAIRS = [
    (((8, 0), (0, 8)), J2),
    (((12, 4), (-4, 8)), J2),
    (((7, 6), (2, 8)), J21),               # J21 @ ((3, 1), (1, 4))
    (((9, 0), (0, 4)), J3),
    (((9, 3), (-2, 5)), J3),               # J3 @ ((3, 1), (-2, 5))
    (((0, -8), (8, 0)), JR),
    (((4, 0, 0), (0, 4, 2), (0, 0, 4)), J2_3D),
    (((16,),), ((4,),)),
    (((9,),), ((3,),)),
]


def _q(J):
    return abs(L.det(L.as_matrix(J)))


@pytest.mark.parametrize("M,J", PAIRS)
def test_fibers_by_brute_force(M, J):
    """Every class of G(M^T) sits in exactly one fiber at one label; the
    label is the class of N^{-T}(h - k) in G(J^T), solved exactly."""
    N, idx, m = Q.fiber_maps(M, J)
    q = _q(J)
    assert idx.shape == (q, m // q)
    assert np.array_equal(np.sort(idx.ravel()), np.arange(m))
    HMT, _ = L.hnf(L.transpose(L.as_matrix(M)))
    HNT, _ = L.hnf(L.transpose(N))
    HJT, _ = L.hnf(L.transpose(L.as_matrix(J)))
    NTinv = L.inverse(L.transpose(N))
    g = [tuple(int(x) for x in row) for row in Q.classes(J)]
    assert g[0] == (0,) * len(g[0])
    hs = L.box_points(HMT)
    for k_i, k in enumerate(L.box_points(HNT)):
        for l in range(q):
            h = hs[idx[l, k_i]]
            assert L.reduce_box(HNT, h) == k
            z = L.matvec(NTinv, [h[i] - k[i] for i in range(len(h))])
            assert all(x.denominator == 1 for x in z)
            assert L.reduce_box(HJT, [int(x) for x in z]) == L.reduce_box(HJT, g[l])


def _c_dirichlet(M, k):
    """c_k(phi_M) * sqrt(m) from the kernel's definition (Section 6.2):
    2^{-r/2} if M^{-T} k lies in the closed cube [-1/2, 1/2]^d, r the number
    of its coordinates of modulus 1/2; else 0."""
    x = L.matvec(L.inverse(L.transpose(L.as_matrix(M))), k)
    if any(abs(c) > Fraction(1, 2) for c in x):
        return 0.0
    r = sum(1 for c in x if abs(c) == Fraction(1, 2))
    return 2.0 ** (-r / 2.0)


@pytest.mark.parametrize("M,J", PAIRS)
def test_mask_is_the_dirichlet_kernel_quotient(M, J):
    """c_k(phi_N) = a(h) c_k(phi_M) for every k in Z^d (phi_N lies in V_M):
    checked over a box that holds the closed M^T-cube."""
    M = L.as_matrix(M)
    N = W.quotient(J, M)
    m, n = abs(L.det(M)), abs(L.det(N))
    mask = Q.dirichlet_mask(M, N)
    HMT, _ = L.hnf(L.transpose(M))
    d = len(M)
    reach = [sum(abs(M[j][i]) for j in range(d)) // 2 + 1 for i in range(d)]
    hit = 0
    for k in product(*[range(-r, r + 1) for r in reach]):
        cM = _c_dirichlet(M, k) / np.sqrt(m)
        cN = _c_dirichlet(N, k) / np.sqrt(n)
        a = mask[L.natural_index(HMT, k)]
        assert abs(cN - a * cM) < 1e-14, (k, cN, a, cM)
        hit += cN != 0
    assert hit >= n          # the closed N-cube holds at least n points


@pytest.mark.parametrize("M,J", PAIRS)
def test_mask_qmf(M, J):
    N = W.quotient(J, M)
    mask = Q.dirichlet_mask(M, N)
    _, idx, _ = Q.fiber_maps(M, J)
    np.testing.assert_allclose(np.sum(mask[idx] ** 2, axis=0), _q(J), rtol=1e-14)


def test_mask_one_dimensional_closed_form():
    """M = 16, J = 4: a = 2 for |h*| < 2, sqrt 2 at |h*| = 2, 0 otherwise;
    M = 9, J = 3: a = sqrt 3 for |h*| <= 1, else 0 (h* in [-m/2, m/2))."""
    h = np.arange(16)
    hs = ((h + 8) % 16) - 8
    ref = np.where(np.abs(hs) < 2, 2.0, np.where(np.abs(hs) == 2, np.sqrt(2.0), 0.0))
    np.testing.assert_allclose(Q.dirichlet_mask(((16,),), ((4,),)), ref, atol=1e-15)
    h = np.arange(9)
    hs = ((h + 4) % 9) - 4
    ref = np.where(np.abs(hs) <= 1, np.sqrt(3.0), 0.0)
    np.testing.assert_allclose(Q.dirichlet_mask(((9,),), ((3,),)), ref, atol=1e-15)


def test_mask_q2_equals_printed_mask():
    for M, J in [(((32, 8), (-8, 32)), workloads.J_QUINCUNX), (((12, 4), (0, 6)), workloads.J_X)]:
        N = W.quotient(J, M)
        np.testing.assert_allclose(Q.dirichlet_mask(M, N), W.dirichlet_mask(M, N), rtol=1e-15)


def test_householder_rows():
    rng = np.random.default_rng(3)
    for q in (2, 3, 4, 8):
        u = rng.standard_normal((q, 50))
        u /= np.linalg.norm(u, axis=0)
        u[:, 0] = 0.0
        u[0, 0] = 1.0                          # v = 0: identity
        u[:, 1] = 0.0
        u[q - 1, 1] = 1.0                      # one-hot off the first label: a signed swap
        S = Q.householder(u)
        for f in range(u.shape[1]):
            np.testing.assert_allclose(S[:, :, f] @ S[:, :, f].T, np.eye(q), atol=1e-14)
            np.testing.assert_allclose(S[0, :, f], u[:, f], atol=1e-15)
        np.testing.assert_array_equal(S[:, :, 0], np.eye(q))
        swap = np.eye(q)
        swap[[0, q - 1]] = swap[[q - 1, 0]]
        swap[q - 1] *= -1.0
        np.testing.assert_allclose(S[:, :, 1], swap, atol=1e-15)
        # no cancellation near u = e_0: orthogonal to rounding
        t = np.full((q, 1), 1e-9)
        t[0] = np.sqrt(1.0 - (q - 1) * 1e-18)
        St = Q.householder(t)[:, :, 0]
        np.testing.assert_allclose(St @ St.T, np.eye(q), atol=1e-15)


def _random_qmf_mask(seed, M, J):
    """A real mask with the QMF identity: positive random values normalised
    per fiber to sum of squares q."""
    _, idx, m = Q.fiber_maps(M, J)
    q = idx.shape[0]
    r = np.random.default_rng(seed).random(idx.shape) + 0.05
    r *= np.sqrt(q) / np.linalg.norm(r, axis=0)
    mask = np.zeros(m)
    mask[idx] = r
    return mask


@pytest.mark.parametrize("M,J", PAIRS)
@pytest.mark.parametrize("kind", ["dirichlet", "random"])
def test_split_equals_time_domain_definition(M, J, kind):
    m = abs(L.det(L.as_matrix(M)))
    N = W.quotient(J, M)
    mask = Q.dirichlet_mask(M, N) if kind == "dirichlet" else _random_qmf_mask(5, M, J)
    a = workloads.complex_normal(11, m, np.complex128)
    ah = dft.lattice_dft_direct(M, a)
    dh = Q.split(M, J, ah, mask)
    d = np.stack([dft.lattice_dft_direct(N, dh[j], inverse=True) for j in range(dh.shape[0])])
    np.testing.assert_allclose(d, Q.split_direct_q(M, J, a, mask), atol=1e-12)
    # orthonormal channels: Parseval, and the synthesis inverts the analysis
    np.testing.assert_allclose(np.sum(np.abs(dh) ** 2), np.sum(np.abs(a) ** 2), rtol=1e-12)
    np.testing.assert_allclose(Q.unsplit(M, J, dh, mask), ah, atol=1e-12)


@pytest.mark.parametrize("M", [((32, 8), (-8, 32)), ((16, 8), (0, 16)), ((8, 0), (0, 8))])
def test_q2_matches_the_printed_wavelet_up_to_its_phase(M):
    """For q = 2 the completion's wavelet row is -(u1, -u0) (u0 >= 0): the
    printed wavelet channel equals it times -conj(phi(h0)) (``oracle.wavelet``)."""
    for J in (workloads.J_QUINCUNX, workloads.J_X, workloads.J_D):
        N = W.quotient(J, M)
        mask = W.dirichlet_mask(M, N)
        m = abs(L.det(M))
        ah = workloads.complex_normal(2, (3, m), np.complex128)
        d1, d2 = W.split(M, J, ah, mask)
        _, i0, i1, rho, _ = W._fiber_maps(M, J)
        _, idx, _ = Q.fiber_maps(M, J)
        np.testing.assert_array_equal(idx[0], i0)
        np.testing.assert_array_equal(idx[1], i1)
        dh = Q.split(M, J, ah, mask)
        phi = np.exp(-2j * np.pi * rho / m)
        np.testing.assert_allclose(dh[:, 0], d1, atol=1e-13)
        np.testing.assert_allclose(-np.conj(phi) * dh[:, 1], d2, atol=1e-13)


@pytest.mark.parametrize("M,J,levels", [
    (((16, 0), (0, 16)), J2, 3),
    (((18, 6), (-6, 12)), J3, 1),
    (((0, -16), (16, 0)), JR, 2),
    (((8, 0, 0), (0, 8, 4), (0, 0, 8)), J2_3D, 2),
    (((64,),), ((4,),), 3),
])
def test_multilevel_pyramid(M, J, levels):
    m = abs(L.det(L.as_matrix(M)))
    x = workloads.complex_normal(13, (2, m), np.complex128)
    c = Q.decompose(x, M, J, levels)
    assert c.shape == x.shape
    np.testing.assert_allclose(np.sum(np.abs(c) ** 2, axis=-1), np.sum(np.abs(x) ** 2, axis=-1),
                               rtol=1e-12)
    np.testing.assert_allclose(Q.reconstruct(c, M, J, levels), x, atol=1e-12)
    # the HNF FFT path equals the direct transforms
    np.testing.assert_allclose(Q.decompose(x, M, J, levels, direct=True), c, atol=1e-11)
    # the layout accounts for every coefficient once
    lay = Q.coeff_layout(M, J, levels)
    assert sum(s for (_, _, _, s) in lay) == m
    assert [o for (_, _, o, _) in lay] == list(np.cumsum([0] + [s for (_, _, _, s) in lay])[:-1])
