"""GPU gradients of the differentiation workload through the hand-written
adjoints (autograd Functions), against the FP64 torch oracle and finite
differences."""
import numpy as np
import pytest

from oracle import grad as G, lattice as L, wavelet as W
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def gpu_loss(plan, x, masks, target, weights):
    from paper_1107_5415_amd import autograd as AG
    c = AG.wavelet_decompose(x, plan, masks)
    loss = torch.zeros((), dtype=torch.float64, device=x.device)
    for (off, n), w in zip(AG.channel_blocks(plan)[:-1], weights):
        blk = c[:, off:off + n]
        loss = loss + w * torch.sum(blk.real.double() ** 2 + blk.imag.double() ** 2)
    r = AG.wavelet_reconstruct(c, plan, masks) - target
    return loss + torch.sum(r.real.double() ** 2 + r.imag.double() ** 2)


def run_case(M, J, levels, B, perturb, seed=5):
    from paper_1107_5415_amd import lfft
    m = abs(L.det(M))
    x = workloads.complex_normal(seed, (B, m))
    target = workloads.complex_normal(seed + 1, (B, m))
    rng = np.random.default_rng(seed)
    masks = [(mk + perturb * rng.standard_normal(mk.shape)).astype(np.float32)
             for mk in W.default_masks(M, J, levels)]
    weights = [1.0] * levels
    plan = lfft.WaveletPlan(M, J, levels, batch=B)
    xd = torch.from_numpy(x).cuda().requires_grad_(True)
    md = [torch.from_numpy(mk).cuda().requires_grad_(True) for mk in masks]
    td = torch.from_numpy(target).cuda()
    loss = gpu_loss(plan, xd, md, td, weights)
    loss.backward()
    ref_loss, gx, gm = G.loss_and_grads(M, J, levels, x.astype(np.complex128),
                                        [mk.astype(np.float64) for mk in masks],
                                        target.astype(np.complex128), weights)
    return plan, (xd, md, td, weights), loss.item(), ref_loss, xd.grad, [g.grad for g in md], gx, gm


@pytest.mark.parametrize("M,J,levels,B,perturb", [
    (((16, 8), (0, 16)), workloads.J_QUINCUNX, 3, 2, 0.1),
    (((32, 8), (-8, 32)), workloads.J_QUINCUNX, 1, 3, 0.0),
    (((12, 4), (0, 6)), workloads.J_X, 1, 2, 0.2),
    (((256, 64), (0, 256)), workloads.J_QUINCUNX, 4, 2, 0.05),
])
def test_gradients_vs_oracle(M, J, levels, B, perturb):
    print("case", M, levels, B, flush=True)
    _, _, loss, ref_loss, gx, gms, rgx, rgm = run_case(M, J, levels, B, perturb)
    assert abs(loss - ref_loss) / abs(ref_loss) < 1e-5
    assert rel_l2(gx.cpu().numpy(), rgx) < 1e-5
    for g, r in zip(gms, rgm):
        assert rel_l2(g.cpu().numpy(), r) < 1e-4


def test_gradients_differentiation_workload():
    """M = [[1024, 256], [0, 1024]] (m = 2^20), batch 16, 4 quincunx levels,
    Dirichlet-initialised masks, target from seed 6."""
    cfg = workloads.CONFIGS["grad"]
    plan, args, loss, ref_loss, gx, gms, rgx, rgm = run_case(cfg["M"], cfg["J"], cfg["levels"],
                                                              cfg["batch"], 0.0, seed=cfg["seed"])
    assert abs(loss - ref_loss) / abs(ref_loss) < 1e-5
    assert rel_l2(gx.cpu().numpy(), rgx) < 1e-5
    for g, r in zip(gms, rgm):
        assert rel_l2(g.cpu().numpy(), r) < 1e-4
    # finite differences on the GPU along one random direction of the samples:
    # the loss is quadratic in x, so central differences are exact up to rounding
    xd, md, td, weights = args
    v = torch.from_numpy(workloads.complex_normal(99, tuple(xd.shape))).cuda()
    h = 0.05
    with torch.no_grad():
        lp = gpu_loss(plan, xd + h * v, md, td, weights).item()
        lm = gpu_loss(plan, xd - h * v, md, td, weights).item()
    fd = (lp - lm) / (2 * h)
    an = float(torch.sum((torch.conj(gx) * v).real.double()).item())
    assert abs(fd - an) / abs(an) < 2e-3
