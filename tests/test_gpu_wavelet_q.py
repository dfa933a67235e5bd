"""GPU parity of the q-channel pyramid (|det J| = q > 2, Section 5.3 step 4
for general q) against the FP64 oracle."""
import numpy as np
import pytest

from oracle import lattice as L, wavelet as W, wavelet_q as Q
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5

J2 = ((2, 0), (0, 2))
J21 = ((2, 1), (0, 2))
J3 = ((3, 0), (0, 1))
JR = ((0, -2), (2, 0))
J2_3D = ((2, 0, 0), (0, 2, 0), (0, 0, 2))


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


CASES = [
    ("j2_3", ((16, 0), (0, 16)), J2, 3, 2),
    ("j2_sheared", ((12, 4), (-4, 8)), J2, 1, 1),
    ("j21", ((7, 6), (2, 8)), J21, 1, 3),
    ("j3", ((18, 6), (-6, 12)), J3, 1, 2),
    ("rot_2", ((0, -16), (16, 0)), JR, 2, 1),
    ("d3_q8", ((8, 0, 0), (0, 8, 4), (0, 0, 8)), J2_3D, 2, 2),
    ("d1_q4", ((256,),), ((4,),), 3, 1),
    ("q5", ((25, 0), (0, 5)), ((5, 0), (0, 1)), 2, 1),
    ("two_pass_levels", ((512, 128), (-128, 512)), J2, 3, 1),
]


@pytest.mark.parametrize("name,M,J,levels,batch", CASES, ids=[c[0] for c in CASES])
def test_decompose_reconstruct(name, M, J, levels, batch):
    from paper_1107_5415_amd import lfft
    m = abs(L.det(L.as_matrix(M)))
    print("case", name, flush=True)
    x = workloads.complex_normal(41, (batch, m))
    w = lfft.WaveletPlan(M, J, levels, batch=batch)
    masks = w.dirichlet_masks("cuda")
    c = w.decompose(_dev(x), masks).cpu().numpy()
    ref = Q.decompose(x.astype(np.complex128), M, J, levels)
    assert rel_l2(c, ref) < TOL
    cz = workloads.complex_normal(42, (batch, m))
    xr = w.reconstruct(_dev(cz), masks).cpu().numpy()
    assert rel_l2(xr, Q.reconstruct(cz.astype(np.complex128), M, J, levels)) < TOL


def _random_qmf_masks(seed, M, J, levels):
    """Real masks with the QMF identity (random positive values normalised
    per fiber), one per level."""
    out = []
    for i, (Ml, _) in enumerate(W.level_matrices(M, J, levels)):
        _, idx, ml = Q.fiber_maps(Ml, J)
        q = idx.shape[0]
        r = np.random.default_rng(seed + i).random(idx.shape) + 0.05
        r *= np.sqrt(q) / np.linalg.norm(r, axis=0)
        mk = np.zeros(ml)
        mk[idx] = r
        out.append(mk.astype(np.float32))
    return out


@pytest.mark.parametrize("M,J,levels", [
    (((32, 0), (0, 32)), J2, 2),
    (((9, 3), (-2, 5)), J3, 1),
    (((8, 0, 0), (0, 8, 4), (0, 0, 8)), J2_3D, 1),
])
def test_random_qmf_masks(M, J, levels):
    """Masks whose fibers hold several non-zero values exercise every term
    of the channel matrix (the Dirichlet masks are mostly one-hot)."""
    from paper_1107_5415_amd import lfft
    m = abs(L.det(L.as_matrix(M)))
    masks = _random_qmf_masks(7, M, J, levels)
    x = workloads.complex_normal(43, (2, m))
    w = lfft.WaveletPlan(M, J, levels, batch=2)
    dm = [_dev(mk) for mk in masks]
    c = w.decompose(_dev(x), dm)
    ref = Q.decompose(x.astype(np.complex128), M, J, levels, masks=[mk.astype(np.float64) for mk in masks])
    assert rel_l2(c.cpu().numpy(), ref) < TOL
    xr = w.reconstruct(c, dm).cpu().numpy()
    assert rel_l2(xr, x) < 2e-5


def test_full_size_four_channels():
    """M = [[4096, 2048], [0, 4096]] (m = 2^24), J = 2 I (four channels),
    four levels: the benchmark's q = 4 workload."""
    from paper_1107_5415_amd import lfft
    cfg = workloads.CONFIGS["q4"]
    M, J, levels = cfg["M"], cfg["J"], cfg["levels"]
    x = workloads.complex_normal(cfg["seed"], 1 << 24)
    w = lfft.WaveletPlan(M, J, levels)
    masks = w.dirichlet_masks("cuda")
    c = w.decompose(_dev(x), masks)
    ref = Q.decompose(x.astype(np.complex128), M, J, levels)
    assert rel_l2(c.cpu().numpy(), ref) < TOL
    del ref
    xr = w.reconstruct(c, masks).cpu().numpy()
    assert rel_l2(xr, x) < 2e-5


@pytest.mark.parametrize("M,J,levels", [
    (((16, 0), (0, 16)), J2, 2),
    (((8, 0, 0), (0, 8, 4), (0, 0, 8)), J2_3D, 1),
])
def test_adjoint_dot_products(M, J, levels):
    """<D v, u> = <v, D^H u> and <S v, u> = <v, S^H u> with masks that do not
    satisfy the QMF identity (so the adjoint is not the inverse)."""
    from paper_1107_5415_amd import lfft
    m = abs(L.det(L.as_matrix(M)))
    rng = np.random.default_rng(46)
    w = lfft.WaveletPlan(M, J, levels, batch=2)
    masks = [_dev((rng.random(ml) * 1.5).astype(np.float32)) for ml in w.level_m]
    v = _dev(workloads.complex_normal(47, (2, m)))
    u = _dev(workloads.complex_normal(48, (2, m)))
    Dv = w.decompose(v, masks)
    DHu = w.decompose_backward(u, None, masks)
    lhs = torch.vdot(u.reshape(-1), Dv.reshape(-1)).item()
    rhs = torch.vdot(DHu.reshape(-1), v.reshape(-1)).item()
    assert abs(lhs - rhs) < 1e-4 * abs(lhs)
    Sv = w.reconstruct(v, masks)
    SHu = w.reconstruct_backward(u, None, masks)
    lhs = torch.vdot(u.reshape(-1), Sv.reshape(-1)).item()
    rhs = torch.vdot(SHu.reshape(-1), v.reshape(-1)).item()
    assert abs(lhs - rhs) < 1e-4 * abs(lhs)
    # the oracle's analysis agrees with the GPU on these masks too
    ref = Q.decompose(workloads.complex_normal(47, (2, m)).astype(np.complex128), M, J, levels,
                      masks=[mk.cpu().numpy().astype(np.float64) for mk in masks])
    assert rel_l2(Dv.cpu().numpy(), ref) < TOL


def test_sample_gradients_through_autograd():
    """loss = ||D(x)||^2 with QMF masks: D is orthogonal, so grad = 2 x."""
    from paper_1107_5415_amd import lfft
    from paper_1107_5415_amd import autograd as AG
    w = lfft.WaveletPlan(((32, 0), (0, 32)), J2, 2)
    masks = w.dirichlet_masks("cuda")
    x = _dev(workloads.complex_normal(49, 1024)).requires_grad_(True)
    c = AG.wavelet_decompose(x, w, masks)
    loss = torch.sum(c.real ** 2 + c.imag ** 2)
    loss.backward()
    assert rel_l2(x.grad.cpu().numpy(), 2 * x.detach().cpu().numpy()) < 1e-5


def test_mask_gradients_need_saved():
    """Mask gradients of the q-channel adjoints read the forward call's saved
    inputs: asking for them without `saved` is an argument error."""
    from paper_1107_5415_amd import lfft
    w = lfft.WaveletPlan(((16, 0), (0, 16)), J2, 1)
    masks = w.dirichlet_masks("cuda")
    x = _dev(workloads.complex_normal(45, 256))
    for fn in (w.decompose_backward, w.reconstruct_backward):
        with pytest.raises(lfft.LfftError) as e:
            fn(x, None, masks, grad_masks=[torch.empty_like(mk) for mk in masks])
        assert e.value.code == -1
    # with `saved` the decomposition keeps its Fourier inputs and gives the
    # same coefficients as without
    saved = w.new_saved(x.device)
    assert saved.numel() == 256
    assert torch.allclose(w.decompose(x, masks, saved=saved), w.decompose(x, masks), rtol=0,
                          atol=1e-6)
