"""The functional forms of the binding (lfft.forward / inverse / decompose /
reconstruct on [..., m] tensors, plans cached per matrix and batch) against
the FP64 oracle."""
import numpy as np
import pytest

from oracle import dft, wavelet as W
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_functional_fft_and_pyramid():
    from paper_1107_5415_amd import lfft
    M, J, levels = ((64, 16), (0, 64)), workloads.J_QUINCUNX, 3
    m = 4096
    xh = workloads.complex_normal(81, (2, 3, m))
    x = torch.from_numpy(xh).cuda()
    print("functional fft", flush=True)
    X = lfft.forward(x, M)
    assert X.shape == x.shape
    ref = dft.lattice_dft_hnf(M, xh.reshape(-1, m).astype(np.complex128)).reshape(xh.shape)
    assert rel_l2(X.cpu().numpy(), ref) < TOL
    assert rel_l2(lfft.inverse(X, M).cpu().numpy(), xh) < TOL
    # the same plan is reused for the same matrix and batch
    assert lfft.get_plan(M, 6) is lfft.get_plan(M, 6)
    print("functional pyramid", flush=True)
    c = lfft.decompose(x, M, J, levels)
    assert c.shape == x.shape
    cref = W.decompose(xh.reshape(-1, m).astype(np.complex128), M, J, levels).reshape(xh.shape)
    assert rel_l2(c.cpu().numpy(), cref) < TOL
    r = lfft.reconstruct(c, M, J, levels)
    assert rel_l2(r.cpu().numpy(), xh) < 2 * TOL
    assert lfft.get_wavelet_plan(M, J, levels, 6) is lfft.get_wavelet_plan(M, J, levels, 6)
    # explicit masks give the same result as the default Dirichlet masks
    plan = lfft.get_wavelet_plan(M, J, levels, 6)
    c2 = lfft.decompose(x, M, J, levels, masks=plan.dirichlet_masks(x.device))
    assert torch.equal(c, c2)
