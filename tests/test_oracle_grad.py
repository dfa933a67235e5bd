"""Pins of the FP64 torch gradient oracle: forward values equal the numpy
oracle, Parseval's closed-form gradient, and central finite differences."""
import numpy as np
import pytest
import torch

from oracle import dft, grad as G, lattice as L, wavelet as W, wavelet_q as WQ
import workloads


@pytest.mark.parametrize("M", [((32, 8), (-8, 32)), ((5, 2), (1, 3)), ((3, 1, 0), (0, 3, 1), (1, 0, 3)),
                               ((16, 8), (0, 16))])
def test_torch_fft_matches_oracle(M):
    m = abs(L.det(M))
    x = workloads.complex_normal(1, (2, m), np.complex128)
    p = G.TorchPair(M)
    X = p.forward(torch.from_numpy(x)).numpy()
    np.testing.assert_allclose(X, dft.lattice_dft_direct(M, x), atol=1e-12)
    np.testing.assert_allclose(p.inverse(torch.from_numpy(X)).numpy(), x, atol=1e-12)


def test_parseval_gradient_closed_form():
    """grad_x ||F(M) x||^2 = 2 x (F unitary)."""
    M = ((12, 4), (0, 6))
    x = torch.from_numpy(workloads.complex_normal(2, (1, 72), np.complex128)).requires_grad_(True)
    y = G.TorchPair(M).forward(x)
    torch.sum(y.real ** 2 + y.imag ** 2).backward()
    np.testing.assert_allclose(x.grad.numpy(), 2 * x.detach().numpy(), atol=1e-12)


CASES = [(((16, 8), (0, 16)), workloads.J_QUINCUNX, 3), (((12, 4), (0, 6)), workloads.J_X, 1),
         (((32, 8), (-8, 32)), workloads.J_QUINCUNX, 1)]


@pytest.mark.parametrize("M,J,levels", CASES)
def test_pyramid_forward_matches_oracle(M, J, levels):
    m = abs(L.det(M))
    x = workloads.complex_normal(3, (2, m), np.complex128)
    masks = W.default_masks(M, J, levels)
    pyr = G.TorchPyramid(M, J, levels)
    mt = [torch.from_numpy(mk) for mk in masks]
    c = pyr.decompose(torch.from_numpy(x), mt).numpy()
    np.testing.assert_allclose(c, W.decompose(x, M, J, levels), atol=1e-12)
    np.testing.assert_allclose(pyr.reconstruct(torch.from_numpy(c), mt).numpy(),
                               W.reconstruct(c, M, J, levels), atol=1e-12)


# q = |det J| > 2: four channels (J = 2I), three (J = diag(3, 1)), eight in 3-D
QCASES = [(((16, 8), (0, 16)), workloads.J_2I, 2), (((27, 9), (0, 9)), ((3, 0), (0, 1)), 2),
          (((8, 4, 0), (0, 8, 4), (0, 0, 8)), ((2, 0, 0), (0, 2, 0), (0, 0, 2)), 1)]


@pytest.mark.parametrize("M,J,levels", QCASES)
def test_pyramid_q_forward_matches_oracle(M, J, levels):
    """The torch q-channel pyramid equals oracle.wavelet_q, with the Dirichlet
    masks and with perturbed (non-QMF) masks."""
    m = abs(L.det(M))
    rng = np.random.default_rng(11)
    x = workloads.complex_normal(12, (2, m), np.complex128)
    pyr = G.TorchPyramidQ(M, J, levels)
    for masks in (WQ.default_masks(M, J, levels),
                  [mk + 0.2 * rng.standard_normal(mk.shape) for mk in WQ.default_masks(M, J, levels)]):
        mt = [torch.from_numpy(mk) for mk in masks]
        c = pyr.decompose(torch.from_numpy(x), mt).numpy()
        np.testing.assert_allclose(c, WQ.decompose(x, M, J, levels, masks=masks), atol=1e-12)
        np.testing.assert_allclose(pyr.reconstruct(torch.from_numpy(c), mt).numpy(),
                                   WQ.reconstruct(c, M, J, levels, masks=masks), atol=1e-12)


@pytest.mark.parametrize("M,J,levels", QCASES)
def test_pyramid_q_parseval_gradient(M, J, levels):
    """With the Dirichlet masks the q-channel pyramid is unitary, so
    grad_x ||D x||^2 = 2 x."""
    m = abs(L.det(M))
    x = torch.from_numpy(workloads.complex_normal(13, (1, m), np.complex128)).requires_grad_(True)
    pyr = G.TorchPyramidQ(M, J, levels)
    c = pyr.decompose(x, [torch.from_numpy(mk) for mk in WQ.default_masks(M, J, levels)])
    torch.sum(c.real ** 2 + c.imag ** 2).backward()
    np.testing.assert_allclose(x.grad.numpy(), 2 * x.detach().numpy(), atol=1e-11)


@pytest.mark.parametrize("M,J,levels", CASES + QCASES)
def test_gradients_finite_differences(M, J, levels):
    """Central differences in FP64 along random directions of the samples and
    of the (non-QMF, perturbed) masks."""
    m = abs(L.det(M))
    rng = np.random.default_rng(4)
    x = workloads.complex_normal(5, (2, m), np.complex128)
    target = workloads.complex_normal(6, (2, m), np.complex128)
    q = abs(L.det(L.as_matrix(J)))
    base = W.default_masks(M, J, levels) if q == 2 else WQ.default_masks(M, J, levels)
    masks = [mk + 0.1 * rng.standard_normal(mk.shape) for mk in base]
    weights = [1.0 + 0.5 * l for l in range(levels)]
    loss, gx, gm = G.loss_and_grads(M, J, levels, x, masks, target, weights)
    pyr = G.make_pyramid(M, J, levels)

    def Lf(xx, mm):
        with torch.no_grad():
            return float(G.pyramid_loss(pyr, torch.from_numpy(xx), [torch.from_numpy(a) for a in mm],
                                        torch.from_numpy(target), weights))
    v = workloads.complex_normal(7, (2, m), np.complex128)
    h = 1e-3   # the loss is quadratic in x: central differences are exact up to rounding
    fd = (Lf(x + h * v, masks) - Lf(x - h * v, masks)) / (2 * h)
    an = float(np.sum((np.conj(gx) * v).real))
    assert abs(fd - an) <= 1e-9 * max(1.0, abs(an))
    u = [rng.standard_normal(mk.shape) for mk in masks]
    # quadratic in each mask for q = 2; through the reflection for q > 2 the
    # loss is smooth but not quadratic, and the O(h^2) term stays far below
    # the tolerance at this step
    h = 1e-5
    fd = (Lf(x, [a + h * b for a, b in zip(masks, u)]) - Lf(x, [a - h * b for a, b in zip(masks, u)])) / (2 * h)
    an = float(sum(np.sum(g * b) for g, b in zip(gm, u)))
    assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))


def test_gradient_parts_finite_differences():
    """The decomposition's and the reconstruction's contributions to the mask
    gradient, each pinned by central differences that perturb only the masks
    of that half; their sum is the whole mask gradient."""
    M, J, levels = ((16, 8), (0, 16)), workloads.J_QUINCUNX, 2
    m = abs(L.det(M))
    rng = np.random.default_rng(8)
    x = workloads.complex_normal(9, (2, m), np.complex128)
    target = workloads.complex_normal(10, (2, m), np.complex128)
    masks = [mk + 0.1 * rng.standard_normal(mk.shape) for mk in W.default_masks(M, J, levels)]
    weights = [1.0] * levels
    _, _, gd, gs = G.loss_and_grads(M, J, levels, x, masks, target, weights, parts=True)
    _, _, gm = G.loss_and_grads(M, J, levels, x, masks, target, weights)
    for a, b, c in zip(gd, gs, gm):
        np.testing.assert_allclose(a + b, c, atol=1e-9 * np.abs(c).max())
    pyr = G.TorchPyramid(M, J, levels)

    def Lf(md, ms):
        with torch.no_grad():
            return float(G.pyramid_loss(pyr, torch.from_numpy(x), [torch.from_numpy(a) for a in md],
                                        torch.from_numpy(target), weights,
                                        masks_rec=[torch.from_numpy(a) for a in ms]))
    u = [rng.standard_normal(mk.shape) for mk in masks]
    h = 1e-5
    plus = [a + h * b for a, b in zip(masks, u)]
    minus = [a - h * b for a, b in zip(masks, u)]
    fd_d = (Lf(plus, masks) - Lf(minus, masks)) / (2 * h)
    fd_s = (Lf(masks, plus) - Lf(masks, minus)) / (2 * h)
    an_d = float(sum(np.sum(g * b) for g, b in zip(gd, u)))
    an_s = float(sum(np.sum(g * b) for g, b in zip(gs, u)))
    assert abs(fd_d - an_d) <= 1e-6 * max(1.0, abs(an_d))
    assert abs(fd_s - an_s) <= 1e-6 * max(1.0, abs(an_s))
