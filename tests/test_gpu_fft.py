"""GPU parity of the lattice FFT (C ABI through the binding) against the FP64
oracle: element-wise relative L2 <= 1e-5 in FP32 (tolerance of the
plain-FP32 path), on seeded inputs."""
import numpy as np
import pytest

from oracle import dft, lattice as L
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


def _lfft():
    from paper_1107_5415_amd import lfft
    return lfft


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle_fft(M, x, inverse=False):
    m = abs(L.det(M))
    x = np.asarray(x, np.complex128)
    if m <= 2048:
        return dft.lattice_dft_direct(M, x, inverse=inverse)
    return dft.lattice_dft_hnf(M, x, inverse=inverse)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


CASES = [
    ("small_1088_radix17", ((32, 8), (-8, 32)), 3),
    ("example1_cyclic32", ((4, -3), (4, 5)), 2),
    ("odd_primes", ((3 * 5, 4), (0, 7 * 11)), 2),
    ("generic_prime_23", ((23, 5), (0, 46)), 1),
    ("negative_det", ((-7, 2), (3, 5)), 4),
    ("d3_small", ((3, 1, 0), (0, 3, 1), (1, 0, 3)), 2),
    ("d3_mixed", ((6, 0, 0), (0, 10, 0), (0, 0, 15)), 1),
    ("d4_small", ((2, 1, 0, 0), (0, 3, 1, 0), (1, 0, 4, 1), (0, 1, 0, 5)), 1),
    # four dimensions beyond one tile: several passes with 4-D natural maps
    ("d4_sheared_multi_pass", ((16, 4, 0, 0), (0, 16, 4, 0), (0, 0, 16, 4), (0, 0, 0, 32)), 1),
    ("d4_lower_mixed", ((12, 0, 0, 0), (3, 10, 0, 0), (0, 5, 14, 0), (1, 0, 7, 18)), 2),
    ("two_pass_2^14", ((128, 32), (0, 128)), 2),
    ("two_pass_odd", ((105, 0), (0, 1287)), 1),
    ("split_then_axis_d3", ((16, 0, 0), (0, 1024, 3), (0, 0, 1024)), 1),
    ("three_axes_three_pass", ((16, 0, 0), (0, 1024, 0), (0, 0, 1024)), 1),
    ("split_axis_2^18", ((1, 0), (0, 1 << 18)), 1),
    ("split_axis_plus_axis", ((2, 0), (0, 1 << 17)), 2),
    ("quincunx_level", ((2048, 3072), (2048, -1024)), 1),
    ("tile_ragged", ((7, 3), (0, 9)), 5),
    ("trivial_m1", ((1, 0), (0, 1)), 3),
    ("d1_prime_997", ((997,),), 2),
    ("d1_pow2_8192", ((8192,),), 3),
    ("d1_four_step_2^20", ((1 << 20,),), 1),
    ("d1_negative_mixed", ((-360,),), 2),
    ("d1_trivial", ((1,),), 2),
    # long power-of-two cycles split as 32 x (n / 32)
    ("d1_split_2^14", ((1 << 14,),), 2),
    ("d1_split_2^16", ((1 << 16,),), 1),
    ("split_2^15_plus_axis", ((4, 0), (0, 1 << 15)), 2),
    ("split_2^17_sheared", ((8, 4), (0, 1 << 17)), 1),
    # a short leading axis joined by the high digit of the next one
    ("short_axis_4x4096", ((4, 0), (0, 4096)), 3),
    ("short_axis_2x8192_sheared", ((2, 1), (0, 8192)), 2),
    ("short_axis_16x2048", ((16, 0), (0, 2048)), 1),
    ("short_axes_d3", ((2, 0, 0), (0, 4, 0), (0, 0, 4096)), 2),
    # the short axis's split axis followed by another axis (three passes)
    ("short_axis_split_then_axis", ((16, 0, 0), (0, 1024, 0), (0, 0, 1024)), 1),
    ("short_axis_split_then_axis_sheared", ((16, 16, 0), (0, 1024, 1024), (0, 0, 1024)), 1),
    # a prime factor beyond one pencil (8209 > 8192): the axis by chirp-z
    ("chirp_z_2x8209", ((1, 0), (0, 2 * 8209)), 2),
    ("chirp_z_d1", ((2 * 8209,),), 1),
    ("chirp_z_plus_axis_d3", ((2, 0, 0), (0, 2, 0), (0, 0, 8209)), 2),
    ("chirp_z_sheared", ((8209, 1), (0, 3)), 1),
    ("chirp_z_lower", ((8209, 0), (5, 8)), 1),
    # streaming passes over several signals with non-temporal row accesses:
    # loads on the forward's first pass and stores on the inverse's last
    # (forward-aligned), and the mirror order (inverse-aligned)
    ("streaming_batch3_upper_2^22", ((2048, 1024), (0, 2048)), 3),
    ("streaming_batch2_lower_2^22", ((2048, 0), (1024, 2048)), 2),
]


@pytest.mark.parametrize("name,M,batch", CASES, ids=[c[0] for c in CASES])
def test_forward_inverse_natural(name, M, batch):
    lfft = _lfft()
    m = abs(L.det(M))
    print("case", name, "m", m, "batch", batch, flush=True)
    x = workloads.complex_normal(11, (batch, m))
    plan = lfft.LatticePlan(M, batch=batch)
    X = plan.forward(_dev(x)).cpu().numpy()
    ref = oracle_fft(M, x)
    assert rel_l2(X, ref) < TOL
    z = workloads.complex_normal(12, (batch, m))
    Z = plan.inverse(_dev(z)).cpu().numpy()
    assert rel_l2(Z, oracle_fft(M, z, inverse=True)) < TOL


def _maps_from_oracle(M, q):
    """natural->grid maps recomputed from the plan's (Q, R) with exact ints."""
    d = len(M)
    eps = [int(e) for e in q["eps"]]
    nz = [j for j in range(d) if eps[j] > 1]
    Q = tuple(map(tuple, q["Q"].tolist()))
    R = tuple(map(tuple, q["R"].tolist()))
    Qinv = np.array(L.inverse(Q), dtype=object).astype(np.int64)
    RinvT = np.array(L.transpose(L.inverse(R)), dtype=object).astype(np.int64)
    g = dft.natural_keys(M, "samples")
    h = dft.natural_keys(M, "freqs")

    def lin(keys, A):
        v = keys @ A.T
        out = np.zeros(keys.shape[0], np.int64)
        for j in nz:
            out = out * eps[j] + np.mod(v[:, j], eps[j])
        return out
    return lin(g, Qinv), lin(h, RinvT)


@pytest.mark.parametrize("M", [((32, 8), (-8, 32)), ((128, 32), (0, 128)), ((2, 0), (0, 1 << 17)),
                               ((3, 1, 0), (0, 3, 1), (1, 0, 3)),
                               ((2, 0, 0), (0, 2, 0), (0, 0, 8209))])
def test_grid_layouts(M):
    """GRID order (Theorem 1, no rearrangement): every in/out layout pair."""
    lfft = _lfft()
    m = abs(L.det(M))
    plan = lfft.LatticePlan(M, batch=2)
    smap, fmap = _maps_from_oracle(M, plan.query())
    x = workloads.complex_normal(13, (2, m))
    ref = oracle_fft(M, x)
    xg = np.empty_like(x)
    xg[:, smap] = x
    refg = np.empty_like(ref)
    refg[:, fmap] = ref
    for lay, src, want in [(lfft.LFFT_IN_GRID, xg, ref), (lfft.LFFT_OUT_GRID, x, refg),
                           (lfft.LFFT_IN_GRID | lfft.LFFT_OUT_GRID, xg, refg)]:
        out = plan.forward(_dev(src), layout=lay).cpu().numpy()
        assert rel_l2(out, want) < TOL, lay
    # inverse in grid layouts
    z = workloads.complex_normal(14, (2, m))
    zref = oracle_fft(M, z, inverse=True)
    zg = np.empty_like(z)
    zg[:, fmap] = z
    zrefg = np.empty_like(zref)
    zrefg[:, smap] = zref
    for lay, src, want in [(lfft.LFFT_IN_GRID, zg, zref), (lfft.LFFT_OUT_GRID, z, zrefg),
                           (lfft.LFFT_IN_GRID | lfft.LFFT_OUT_GRID, zg, zrefg)]:
        out = plan.inverse(_dev(src), layout=lay).cpu().numpy()
        assert rel_l2(out, want) < TOL, lay


def test_large_forward_inverse_full_size():
    """d = 2, M = [[4096, 2048], [0, 4096]], m = 2^24 in the launch
    configuration the benchmark times; checked against the Hermite-form FP64
    FFT (an independent algorithm) and against exact direct bins."""
    lfft = _lfft()
    cfg = workloads.CONFIGS["large"]
    M = cfg["M"]
    m = 1 << 24
    x = workloads.complex_normal(cfg["seed"], m)
    plan = lfft.LatticePlan(M, batch=1)
    X = plan.forward(_dev(x)).cpu().numpy()
    ref = dft.lattice_dft_hnf(M, x)
    assert rel_l2(X, ref) < TOL
    HT, _ = L.hnf(L.transpose(M))
    rng = np.random.default_rng(0)
    idx = rng.integers(0, m, 16)
    hs = [tuple(int(v) for v in dft.natural_keys(M, "freqs")[i]) for i in idx[:4]]
    bins = dft.direct_bins(M, x, hs)
    np.testing.assert_allclose(X[idx[:4]], bins, rtol=0, atol=2e-5 * np.abs(bins).max() + 1e-4)
    z = workloads.complex_normal(cfg["seed"] + 100, m)
    Z = plan.inverse(_dev(z)).cpu().numpy()
    assert rel_l2(Z, dft.lattice_dft_hnf(M, z, inverse=True)) < TOL


@pytest.mark.parametrize("name,M", [
    ("d1_2^27", ((1 << 27,),)),
    ("d1_3x2^25", ((3 << 25,),)),
    ("d1_2^28", ((1 << 28,),)),
    ("sheared_cyclic_2^27", ((2, 1), (0, 1 << 26))),
])
def test_cycles_split_in_three(name, M):
    """Cycles longer than two on-chip pencils (above 2^26 points) run as
    three passes with two four-step twiddles; forward against the Hermite
    FP64 FFT and inverse round trip."""
    lfft = _lfft()
    m = abs(L.det(M))
    print("case", name, "m", m, flush=True)
    plan = lfft.LatticePlan(M)
    assert plan.query()["passes"] == 3
    x = workloads.complex_normal(61, m)
    xd = _dev(x)
    X = plan.forward(xd)
    assert rel_l2(X.cpu().numpy(), dft.lattice_dft_hnf(M, x)) < TOL
    back = plan.inverse(X).cpu().numpy()
    assert rel_l2(back, x) < 2 * TOL


def test_cycle_of_2_30_points():
    """The longest cycle the planner takes (three digits of 1024): exact bins
    of a sparse signal at sampled frequencies (its unitary DFT in closed form,
    phases reduced mod m in integers), Parseval and the round trip on a dense
    one."""
    lfft = _lfft()
    m = 1 << 30
    plan = lfft.LatticePlan(((m,),))
    assert plan.query()["passes"] == 3
    rng = np.random.default_rng(30)
    k = rng.choice(m, 8, replace=False).astype(np.int64)
    a = workloads.complex_normal(31, 8).astype(np.complex128)
    print("case 2^30 sparse", flush=True)
    xs = torch.zeros(m, dtype=torch.complex64, device="cuda")
    xs[torch.from_numpy(k).cuda()] = torch.from_numpy(a.astype(np.complex64)).cuda()
    X = plan.forward(xs)
    del xs
    h = np.concatenate([rng.integers(0, m, 4096), [0, 1, m - 1]]).astype(np.int64)
    got = X[torch.from_numpy(h).cuda()].cpu().numpy().astype(np.complex128)
    del X
    r = (h[:, None] * k[None, :]) % m
    want = (a[None, :] * np.exp(-2j * np.pi * r / m)).sum(1) / np.sqrt(m)
    assert rel_l2(got, want) < TOL
    print("case 2^30 dense", flush=True)
    g = torch.Generator(device="cuda").manual_seed(32)
    x = torch.randn(m, dtype=torch.complex64, device="cuda", generator=g)
    X = plan.forward(x)
    nx = torch.linalg.vector_norm(x.to(torch.complex128)).item()
    nX = torch.linalg.vector_norm(X.to(torch.complex128)).item()
    assert abs(nX / nx - 1) < 1e-5
    back = plan.inverse(X)
    del X
    err = torch.linalg.vector_norm((back - x).to(torch.complex128)).item() / nx
    assert err < 2 * TOL


def _random_lattice(seed):
    """Seeded random regular matrices: d = 2, 3, 4 in turn, entries and
    determinant bounds that give m from a few hundred to 2^18 points, every
    shape (Hermite form with any diagonal, Smith grids of one to four axes,
    either basis aligned or neither)."""
    rng = np.random.default_rng(1000 + seed)
    d = 2 + seed % 3
    if seed >= 36:
        # several elementary divisors: U1 diag(e) U2 with random unimodular
        # U1, U2 (products of integer row and column additions)
        while True:
            base = rng.choice([1, 2, 3, 4, 6, 8, 12, 16, 32, 64, 128], size=d)
            e = np.cumprod(base).astype(np.int64)   # e_1 | e_2 | ... | e_d
            if (1 << 12) <= int(np.prod(e)) <= (1 << 20):
                break
        A = np.diag(e[::-1])
        for _ in range(2 * d):
            i, j = rng.choice(d, 2, replace=False)
            A[i] += int(rng.integers(-2, 3)) * A[j]
            i, j = rng.choice(d, 2, replace=False)
            A[:, i] += int(rng.integers(-2, 3)) * A[:, j]
        return tuple(tuple(int(v) for v in row) for row in A)
    lo, hi, md = {2: (-600, 601, 1 << 18), 3: (-60, 61, 1 << 18), 4: (-12, 13, 1 << 17)}[d]
    while True:
        M = workloads.random_regular_matrix(rng, d, lo=lo, hi=hi, max_det=md)
        if abs(L.det(M)) >= 256:
            return M


@pytest.mark.parametrize("seed", range(48))
def test_random_lattices(seed):
    """Forward and inverse, natural order, batch 2, on random lattices."""
    lfft = _lfft()
    M = _random_lattice(seed)
    m = abs(L.det(M))
    print("case seed", seed, "M", M, "m", m, flush=True)
    plan = lfft.LatticePlan(M, batch=2)
    x = workloads.complex_normal(70 + seed, (2, m))
    X = plan.forward(_dev(x)).cpu().numpy()
    for b in range(2):
        assert rel_l2(X[b], oracle_fft(M, x[b])) < TOL
    Y = plan.inverse(_dev(x)).cpu().numpy()
    for b in range(2):
        assert rel_l2(Y[b], oracle_fft(M, x[b], inverse=True)) < TOL


def test_d3_full_size_forward():
    lfft = _lfft()
    cfg = workloads.CONFIGS["d3"]
    M = cfg["M"]
    x = workloads.complex_normal(cfg["seed"], 1 << 24)
    X = lfft.LatticePlan(M).forward(_dev(x)).cpu().numpy()
    assert rel_l2(X, dft.lattice_dft_hnf(M, x)) < TOL


def test_properties_at_any_size():
    """Unitarity and inverse(forward) = id on the large workload."""
    lfft = _lfft()
    M = workloads.CONFIGS["large"]["M"]
    x = _dev(workloads.complex_normal(21, 1 << 24))
    plan = lfft.LatticePlan(M)
    X = plan.forward(x)
    nx = torch.linalg.vector_norm(x.to(torch.complex128)).item()
    nX = torch.linalg.vector_norm(X.to(torch.complex128)).item()
    assert abs(nX / nx - 1) < 1e-5
    back = plan.inverse(X)
    err = torch.linalg.vector_norm((back - x).to(torch.complex128)).item() / nx
    assert err < 2e-5


def test_chirp_z_direct_bins():
    """Chirp-z axis: exact direct-sum bins of the natural output."""
    lfft = _lfft()
    M = ((2, 0, 0), (0, 2, 0), (0, 0, 8209))
    m = abs(L.det(M))
    x = workloads.complex_normal(13, m)
    X = lfft.LatticePlan(M).forward(_dev(x)).cpu().numpy()
    rng = np.random.default_rng(3)
    hk = dft.natural_keys(M, "freqs")
    idx = rng.choice(m, 24, replace=False)
    bins = dft.direct_bins(M, x.astype(np.complex128), [tuple(int(v) for v in hk[i]) for i in idx])
    assert rel_l2(X[idx], bins) < TOL


def test_chirp_z_in_batch():
    """A batch mixing power-of-two lattices with chirp-z ones: the chirp-z
    lattices run through their own plans in the shared extra workspace."""
    lfft = _lfft()
    Ms = [((1, 0), (0, 2 * 8209)), ((64, 16), (0, 256)), ((8209, 1), (0, 3)), ((32, 8), (-8, 32))]
    plan = lfft.BatchPlan(Ms)
    x = workloads.complex_normal(14, plan.total)
    for mode in (0, 1, 2):
        y = plan.execute(_dev(x), mode=mode).cpu().numpy()
        off = plan.offsets
        for i, M in enumerate(Ms):
            ref = oracle_fft(M, x[off[i]:off[i + 1]][None, :])[0]
            assert rel_l2(y[off[i]:off[i + 1]], ref) < TOL, (mode, i)
