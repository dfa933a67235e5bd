"""Pins of the samples <-> orthonormal-translate coefficients basis change
(oracle.interp): interpolation property, orthonormal translates, the bracket
sum counted member by member, and the odd-m closed form."""
import numpy as np
import pytest

from oracle import dft, interp as IP, lattice as L
import workloads

SMALL = [((4, 0), (0, 4)), ((4, -3), (4, 5)), ((6, 2), (0, 4)), ((5, 2), (1, 3)),
         ((2, 1, 0), (0, 2, 1), (1, 0, 2)), ((8,),), ((3, 1), (-2, 4))]


@pytest.mark.parametrize("M", SMALL)
def test_interpolation_property(M):
    """The coefficients put back into the translates of phi_M (samples of
    phi_M from its Fourier series, summed directly) reproduce the samples."""
    m = abs(L.det(M))
    s = workloads.complex_normal(3, (2, m), np.complex128)
    a = IP.samples_to_coeffs(M, s)
    np.testing.assert_allclose(IP.interpolant_values(M, a), s, atol=1e-12)
    np.testing.assert_allclose(IP.coeffs_to_samples(M, a), s, atol=1e-12)
    ahat = IP.samples_to_coeffs(M, s, fourier=True)
    np.testing.assert_allclose(ahat, dft.lattice_dft_direct(M, a), atol=1e-12)
    np.testing.assert_allclose(IP.coeffs_to_samples(M, ahat, fourier=True), s, atol=1e-12)


@pytest.mark.parametrize("M", SMALL)
def test_translates_orthonormal(M):
    m = abs(L.det(M))
    np.testing.assert_allclose(IP.translates_gram(M), np.eye(m), atol=1e-12)


@pytest.mark.parametrize("M", SMALL)
def test_bracket_sum_member_by_member(M):
    """m theta_h from the closed-cube coefficients grouped by class."""
    M_ = L.as_matrix(M)
    m = abs(L.det(M_))
    HT, _ = L.hnf(L.transpose(M_))
    theta = np.zeros(m)
    for k, (r, _) in IP.dirichlet_coefficients(M_).items():
        theta[L.natural_index(HT, k)] += 2.0 ** (-r / 2) / np.sqrt(m)
    np.testing.assert_allclose(m * theta, IP.dirichlet_bracket_factor(M), rtol=1e-14)


@pytest.mark.parametrize("M", [((5, 2), (1, 3)), ((3, 0), (0, 5)), ((7,),), ((3, 1, 0), (0, 3, 1), (0, 0, 3))])
def test_odd_m_closed_form(M):
    """Odd m: no class lies on the cube's boundary, phi_M(2 pi z) = sqrt(m)
    delta_z, so the coefficients are the samples over sqrt(m)."""
    m = abs(L.det(M))
    assert m % 2 == 1
    s = workloads.complex_normal(4, m, np.complex128)
    np.testing.assert_allclose(IP.samples_to_coeffs(M, s), s / np.sqrt(m), atol=1e-12)
    phi = IP.kernel_samples(M)
    np.testing.assert_allclose(phi, np.sqrt(m) * (np.arange(m) == 0), atol=1e-12)
