"""Pins of the oracle's wavelet split (Section 5.3) and Dirichlet mask
(Section 6.2) against the time-domain definition, closed forms and invariants."""
import numpy as np
import pytest

from oracle import dft, lattice as L, wavelet as W
import workloads

PAIRS = [
    (((32, 8), (-8, 32)), workloads.J_QUINCUNX),
    (((8, 0), (0, 8)), workloads.J_X),
    (((8, 0), (0, 8)), workloads.J_Y),
    (((8, 0), (0, 8)), workloads.J_D),
    (((12, 4), (0, 6)), workloads.J_X),
    (((16, 8), (0, 16)), workloads.J_QUINCUNX),
    (((4, -3), (4, 5)), workloads.J_D),          # Example 1: M = J_d N
    (((6, 2, 0), (0, 4, 2), (0, 0, 6)), ((2, 0, 0), (0, 1, 0), (0, 0, 1))),
]


@pytest.mark.parametrize("M,J", PAIRS)
def test_mask_qmf_and_values(M, J):
    N = W.quotient(J, M)
    mask = W.dirichlet_mask(M, N)
    _, i0, i1, _, _ = W._fiber_maps(M, J)
    np.testing.assert_allclose(mask[i0] ** 2 + mask[i1] ** 2, 2.0, rtol=1e-15)
    vals = set(np.round(mask, 12))
    assert vals <= {0.0, 1.0, round(np.sqrt(2.0), 12)}
    # every class is in exactly one fiber
    assert np.array_equal(np.sort(np.concatenate([i0, i1])), np.arange(abs(L.det(M))))


@pytest.mark.parametrize("n", [4, 6, 8, 16])
def test_mask_one_dimensional_closed_form(n):
    """M = diag(2n, 1), J = diag(2, 1): the lattice reduces to the 1-D torus,
    where the Dirichlet two-scale symbol is sqrt 2 for |k| < n/2, 1 for
    |k| = n/2 and 0 otherwise (k the symmetric representative mod 2n)."""
    M = ((2 * n, 0), (0, 1))
    N = W.quotient(workloads.J_X, M)
    mask = W.dirichlet_mask(M, N)
    k = np.arange(2 * n)
    ks = ((k + n) % (2 * n)) - n
    ref = np.where(np.abs(ks) < n / 2, np.sqrt(2), np.where(np.abs(ks) == n / 2, 1.0, 0.0))
    np.testing.assert_allclose(mask, ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("M,J", PAIRS)
def test_split_equals_time_domain_definition(M, J):
    m = abs(L.det(M))
    N = W.quotient(J, M)
    mask = W.dirichlet_mask(M, N)
    a = workloads.complex_normal(7, m, np.complex128)
    ah = dft.lattice_dft_direct(M, a)
    d1h, d2h = W.split(M, J, ah, mask)
    d1 = dft.lattice_dft_direct(N, d1h, inverse=True)
    d2 = dft.lattice_dft_direct(N, d2h, inverse=True)
    e1, e2 = W.split_direct(M, J, a, mask)
    np.testing.assert_allclose(d1, e1, atol=1e-12)
    np.testing.assert_allclose(d2, e2, atol=1e-12)
    # Parseval: orthonormal decomposition
    np.testing.assert_allclose(np.linalg.norm(d1) ** 2 + np.linalg.norm(d2) ** 2,
                               np.linalg.norm(a) ** 2, rtol=1e-12)
    # perfect reconstruction in the Fourier domain
    np.testing.assert_allclose(W.unsplit(M, J, d1h, d2h, mask), ah, atol=1e-12)


def test_split_without_conjugate_is_wrong():
    """The conjugate on the filter symbol in step 4 matters (reading of
    Section 5.3): dropping it breaks agreement with the definition."""
    M, J = PAIRS[0]
    m = abs(L.det(M))
    N = W.quotient(J, M)
    mask = W.dirichlet_mask(M, N)
    a = workloads.complex_normal(8, m, np.complex128)
    ah = dft.lattice_dft_direct(M, a)
    _, i0, i1, rho, _ = W._fiber_maps(M, J)
    phi = np.exp(-2j * np.pi * rho / m)
    wrong = phi * (mask[i1] * ah[i0] - mask[i0] * ah[i1]) / np.sqrt(2)
    _, e2 = W.split_direct(M, J, a, mask)
    d2 = dft.lattice_dft_direct(N, wrong, inverse=True)
    assert np.linalg.norm(d2 - e2) / np.linalg.norm(e2) > 0.5


@pytest.mark.parametrize("M,J,levels", [(((32, 8), (-8, 32)), workloads.J_QUINCUNX, 1),
                                         (((16, 8), (0, 16)), workloads.J_QUINCUNX, 4),
                                         (((64, 16), (0, 64)), workloads.J_QUINCUNX, 5)])
def test_multilevel_pyramid(M, J, levels):
    m = abs(L.det(M))
    x = workloads.complex_normal(9, (2, m), np.complex128)
    c_direct = W.decompose(x, M, J, levels, direct=True)
    c_fast = W.decompose(x, M, J, levels, direct=False)
    np.testing.assert_allclose(c_fast, c_direct, atol=1e-11)
    np.testing.assert_allclose(np.linalg.norm(c_fast, axis=-1), np.linalg.norm(x, axis=-1), rtol=1e-12)
    np.testing.assert_allclose(W.reconstruct(c_fast, M, J, levels), x, atol=1e-11)
    # level 1 of the pyramid equals the time-domain definition
    mask = W.dirichlet_mask(M, W.quotient(J, M))
    e1, e2 = W.split_direct(M, J, x[0], mask)
    np.testing.assert_allclose(c_direct[0, : m // 2], e2, atol=1e-11)


def test_large_level_chain_shapes():
    """The 8 quincunx levels of M = [[4096, 2048], [0, 4096]]: every level is
    integral and |det| halves; Theorem 3 case 2 keeps d = 2."""
    mats = W.level_matrices(((4096, 2048), (0, 4096)), workloads.J_QUINCUNX, 8)
    dets = [abs(L.det(Nl)) for (_, Nl) in mats]
    assert dets == [1 << (24 - l) for l in range(1, 9)]
    eps = [L.elementary_divisors(Nl) for (_, Nl) in mats]
    assert eps == [(1024, 8192), (1024, 4096), (512, 4096), (512, 2048),
                   (256, 2048), (256, 1024), (128, 1024), (128, 512)]
