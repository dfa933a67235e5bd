"""lfft_forward_noalloc (no workspace, no allocation) against lfft_forward on
the same inputs, through the C ABI, two calls in a row with the second on a
smaller lattice, and the size limit of its fixed scratch array."""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_forward_noalloc_matches_forward():
    from paper_1107_5415_amd import lfft
    cases = [(((4096, 2048), (0, 2048)), 1), (((256, 64), (0, 256)), 2), (((32, 8), (-8, 32)), 3)]
    for i, (M, B) in enumerate(cases):
        print("case noalloc", M, B, flush=True)
        plan = lfft.LatticePlan(M, batch=B)
        x = torch.from_numpy(workloads.complex_normal(60 + i, (B, plan.m))).cuda()
        ref = plan.forward(x)
        out = torch.empty_like(x)
        plan.forward_noalloc(x, out)
        torch.cuda.synchronize()
        # same kernels, same arithmetic, only the workspace differs: bit-equal
        assert torch.equal(out, ref)
        for layout in (lfft.LFFT_OUT_GRID, lfft.LFFT_IN_GRID | lfft.LFFT_OUT_GRID):
            assert torch.equal(plan.forward_noalloc(x, torch.empty_like(x), layout=layout),
                               plan.forward(x, layout=layout))


def test_forward_noalloc_limit():
    from paper_1107_5415_amd import lfft
    plan = lfft.LatticePlan(((4096, 2048), (0, 4096)))   # 128 MiB workspace > 64 MiB
    assert plan.workspace_bytes() > 64 << 20
    x = torch.zeros(plan.m, dtype=torch.complex64, device="cuda")
    with pytest.raises(lfft.LfftError) as e:
        plan.forward_noalloc(x, torch.empty_like(x))
    assert e.value.code == -5
