"""GPU parity of the batched lattice FFT (lfft_batch_*: per-lattice launches,
one persistent launch, and its captured graph) against the FP64 oracle:
relative L2 <= 1e-5 for every lattice of the batch."""
import numpy as np
import pytest

from oracle import dft, lattice as L
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


def oracle_fft(M, x, inverse=False):
    x = np.asarray(x, np.complex128)[None, :]
    if abs(L.det(M)) <= 1024:
        return dft.lattice_dft_direct(M, x, inverse=inverse)[0]
    return dft.lattice_dft_hnf(M, x, inverse=inverse)[0]


def check_all(plan, Ms, x, y, inverse=False, which=None):
    off = plan.offsets
    xs = x.cpu().numpy()
    ys = y.cpu().numpy()
    worst = 0.0
    for i in (range(len(Ms)) if which is None else which):
        ref = oracle_fft(Ms[i], xs[off[i]:off[i + 1]], inverse)
        got = ys[off[i]:off[i + 1]]
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        assert err <= TOL, (i, Ms[i], err)
        worst = max(worst, err)
    return worst


# edge cases of the batched workload's family plus lattices outside the
# fixed-tile schedule (non-power-of-two cycles, fewer than 32 points)
EDGE = [((1, 0), (0, 1 << 10)), ((1 << 10, 0), (0, 1)), ((32, 0), (0, 32)),
        ((32, 7), (0, 32)), ((2, 1), (0, 1 << 13)), ((4, 0), (0, 1 << 12)),
        ((1 << 9, 5), (0, 1 << 9)), ((1, 0), (0, 1 << 18)), ((1 << 9, 0), (0, 1 << 9)),
        ((64, 16), (0, 1 << 10)), ((32, 8), (-8, 32)), ((3, 0), (0, 5)), ((4, 1), (0, 4))]


def small_batch():
    return EDGE + workloads.batched_matrices(seed=11, count=40)


def make_input(plan, seed):
    return torch.from_numpy(workloads.complex_normal(seed, plan.total)).cuda()


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_batch_modes_forward_inverse(mode):
    from paper_1107_5415_amd import lfft
    Ms = small_batch()
    plan = lfft.BatchPlan(Ms)
    print("batch modes", mode, plan.config(), flush=True)
    x = make_input(plan, 21)
    y = plan.execute(x, mode=mode)
    check_all(plan, Ms, x, y)
    z = plan.execute(y, inverse=True, mode=mode)
    check_all(plan, Ms, y, z, inverse=True)
    torch.cuda.synchronize()
    assert float(torch.linalg.norm(z - x) / torch.linalg.norm(x)) < 2 * TOL


@pytest.mark.parametrize("tile_lg", [11, 12, 13])
@pytest.mark.parametrize("order", range(8))
def test_batch_configurations(tile_lg, order):
    from paper_1107_5415_amd import lfft
    Ms = small_batch()
    plan = lfft.BatchPlan(Ms)
    plan.configure(tile_lg, order)
    print("batch config", tile_lg, order, flush=True)
    x = make_input(plan, 22)
    y = plan.execute(x, mode=1)
    check_all(plan, Ms, x, y)
    z = plan.execute(y, inverse=True, mode=1)
    check_all(plan, Ms, y, z, inverse=True)


def test_batch_graph_replays():
    """The captured graph replayed on changing data, with eager work and
    synchronisation between replays: every replay matches the oracle."""
    from paper_1107_5415_amd import lfft
    Ms = small_batch()
    plan = lfft.BatchPlan(Ms)
    x = make_input(plan, 23)
    y = torch.empty_like(x)
    for r in range(4):
        print("graph replay", r, flush=True)
        plan.execute(x, mode=2, out=y)
        torch.cuda.synchronize()
        check_all(plan, Ms, x, y)
        x.mul_(complex(0.5, -1.25))
        x[::7] += 1.0
        torch.cuda.synchronize()


def test_batch_workload_tuned(tmp_path):
    """The batched workload (512 lattices [[2^a, c], [0, 2^b]], a + b in
    10..18): autotuned, graph mode, every lattice against the oracle, and
    the per-lattice launches agree."""
    from paper_1107_5415_amd import lfft
    Ms = workloads.batched_matrices(seed=workloads.CONFIGS["batched"]["seed"])
    plan = lfft.BatchPlan(Ms)
    x = make_input(plan, workloads.CONFIGS["batched"]["seed"])
    print("tune", flush=True)
    best = plan.tune(x, reps=2)
    cfg = plan.config()
    print("tuned", cfg, best, flush=True)
    assert cfg["eligible"] == len(Ms)
    y = plan.execute(x, mode=2)
    worst = check_all(plan, Ms, x, y)
    print("worst rel l2", worst, flush=True)
    y0 = plan.execute(x, mode=0)
    assert float(torch.linalg.norm(y0 - y) / torch.linalg.norm(y0)) < 2 * TOL
    z = plan.execute(y, inverse=True, mode=2)
    assert float(torch.linalg.norm(z - x) / torch.linalg.norm(x)) < 2 * TOL
    # the choice is remembered for the same matrices
    plan2 = lfft.BatchPlan(Ms)
    assert plan2.tune(x, reps=1) == -1.0
    assert plan2.config() == cfg
    # and survives the process through the cache file
    path = str(tmp_path / "tune.json")
    lfft.tune_save(path)
    assert lfft.tune_clear() >= 1
    assert lfft.tune_load(path) >= 1
    plan3 = lfft.BatchPlan(Ms)
    assert plan3.tune(x, reps=1) == -1.0
    assert plan3.config() == cfg
