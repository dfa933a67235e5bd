"""GPU parity of the change of basis between point values and
orthonormal-translate coefficients of the Dirichlet kernel (lfft_basis_change)
and of the pyramid on point values (LWT_SAMPLES), against the FP64 oracle."""
import numpy as np
import pytest

from oracle import interp as IP, lattice as L, wavelet as W, wavelet_q as WQ
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


CASES = [((32, 8), (-8, 32)), ((4, -3), (4, 5)), ((64, 16), (0, 64)), ((512, 0), (0, 512)),
         ((6, 2, 0), (0, 4, 2), (0, 0, 6)), ((5, 2), (1, 3)), ((1 << 12,),), ((4096, 2048), (0, 4096))]


@pytest.mark.parametrize("M", CASES)
def test_basis_change_both_directions(M):
    from paper_1107_5415_amd import lfft
    m = abs(L.det(M))
    B = 1 if m > (1 << 20) else 2
    print("case basis", M, B, flush=True)
    s = workloads.complex_normal(70, (B, m))
    p = lfft.LatticePlan(M, batch=B)
    sd = _dev(s)
    a = p.basis_change(sd).cpu().numpy()
    ahat = p.basis_change(sd, fourier=True).cpu().numpy()
    s64 = s.astype(np.complex128)
    assert rel_l2(a, IP.samples_to_coeffs(M, s64)) < TOL
    assert rel_l2(ahat, IP.samples_to_coeffs(M, s64, fourier=True)) < TOL
    back = p.basis_change(_dev(a.astype(np.complex64)), lfft.LFFT_COEFFS_TO_SAMPLES).cpu().numpy()
    assert rel_l2(back, IP.coeffs_to_samples(M, a.astype(np.complex64).astype(np.complex128))) < TOL
    back2 = p.basis_change(_dev(ahat), lfft.LFFT_COEFFS_TO_SAMPLES, fourier=True).cpu().numpy()
    assert rel_l2(back2, s) < 2 * TOL


@pytest.mark.parametrize("M,J,levels,B", [
    (((32, 8), (-8, 32)), workloads.J_QUINCUNX, 1, 1),
    (((64, 16), (0, 64)), workloads.J_QUINCUNX, 5, 2),
    (((16, 0), (0, 16)), workloads.J_2I, 2, 2),
    (((4096, 2048), (0, 4096)), workloads.J_QUINCUNX, 8, 1),
])
def test_pyramid_on_samples(M, J, levels, B):
    """LWT_SAMPLES: the decomposition of point values equals the
    decomposition of their orthonormal-translate coefficients, and the
    reconstruction returns point values."""
    from paper_1107_5415_amd import lfft
    m = abs(L.det(M))
    q = abs(L.det(L.as_matrix(J)))
    print("case pyramid samples", M, J, levels, flush=True)
    s = workloads.complex_normal(71, (B, m))
    w = lfft.WaveletPlan(M, J, levels, batch=B, samples=True)
    masks = w.dirichlet_masks("cuda")
    c = w.decompose(_dev(s), masks)
    a = IP.samples_to_coeffs(M, s.astype(np.complex128))
    Wm = W if q == 2 else WQ
    ref = Wm.decompose(a, M, J, levels)
    assert rel_l2(c.cpu().numpy(), ref) < TOL
    cz = workloads.complex_normal(72, (B, m))
    xr = w.reconstruct(_dev(cz), masks).cpu().numpy()
    assert rel_l2(xr, IP.coeffs_to_samples(M, Wm.reconstruct(cz.astype(np.complex128), M, J, levels))) < TOL
    assert rel_l2(w.reconstruct(c, masks).cpu().numpy(), s) < 2 * TOL


def test_pyramid_on_samples_adjoints():
    """<D_s v, u> = <v, D_s^H u> for the decomposition of point values, and
    the same for its reconstruction (q = 2 with mask gradients' saved path
    and q = 4)."""
    from paper_1107_5415_amd import lfft
    for M, J, levels, B in ((((64, 16), (0, 64)), workloads.J_QUINCUNX, 3, 2),
                            (((16, 0), (0, 16)), workloads.J_2I, 2, 1)):
        m = abs(L.det(M))
        w = lfft.WaveletPlan(M, J, levels, batch=B, samples=True)
        masks = w.dirichlet_masks("cuda")
        v = _dev(workloads.complex_normal(73, (B, m)))
        u = _dev(workloads.complex_normal(74, (B, m)))
        for fwd, bwd in ((w.decompose, w.decompose_backward), (w.reconstruct, w.reconstruct_backward)):
            Av = fwd(v, masks)
            AHu = bwd(u, None, masks)
            lhs = torch.vdot(Av.flatten().to(torch.complex128), u.flatten().to(torch.complex128)).item()
            rhs = torch.vdot(v.flatten().to(torch.complex128), AHu.flatten().to(torch.complex128)).item()
            assert abs(lhs - rhs) / abs(lhs) < 1e-5


def test_basis_change_autograd():
    """The basis change is self-adjoint: its autograd backward equals the
    oracle's gradient of a quadratic loss."""
    from paper_1107_5415_amd import autograd as AG
    M = ((64, 16), (0, 64))
    m = 4096
    s = workloads.complex_normal(75, (2, m))
    sd = _dev(s).requires_grad_(True)
    a = AG.samples_to_coeffs(sd, M)
    t = _dev(workloads.complex_normal(76, (2, m)))
    loss = torch.sum((a - t).real ** 2 + (a - t).imag ** 2)
    loss.backward()
    # d/ds ||B s - t||^2 = 2 B^H (B s - t) = 2 B (B s - t)
    a64 = IP.samples_to_coeffs(M, s.astype(np.complex128))
    ref = 2 * IP.samples_to_coeffs(M, a64 - workloads.complex_normal(76, (2, m)).astype(np.complex128))
    assert rel_l2(sd.grad.cpu().numpy(), ref) < TOL
