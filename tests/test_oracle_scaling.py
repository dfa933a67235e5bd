"""Pins of the per-level scaling report (Section 5.2, Theorem 3)."""
import pytest

from oracle import lattice as L, scaling as S, wavelet as W
import workloads

CASES = [
    (((2, 0), (0, 2)), workloads.J_X),            # adds a cycle: (1,2) -> (2,2)
    (((6, 0), (0, 1)), workloads.J_X),            # grows: (1,3) -> (1,6)
    (((1, 4), (1, -4)), workloads.J_QUINCUNX),    # grows: (1,4) -> (1,8)
    (((32, 8), (-8, 32)), workloads.J_QUINCUNX),
    (((8, 0), (0, 8)), workloads.J_D),
    (((4, -3), (4, 5)), workloads.J_D),           # Example 1
    (((6, 2, 0), (0, 4, 2), (0, 0, 6)), ((2, 0, 0), (0, 1, 0), (0, 0, 1))),
    (((9, 0), (0, 4)), ((3, 0), (0, 1))),
    (((9, 3), (-2, 5)), ((3, 0), (0, 1))),
    (((12, 0), (0, 12)), ((2, 1), (0, 2))),       # q = 4, cyclic P(J)
]


@pytest.mark.parametrize("M,J", CASES)
def test_dimension_by_brute_force(M, J):
    N = W.quotient(J, M)
    assert S.p_rank_dimension(M) == L.pattern_dimension(M)
    assert S.p_rank_dimension(N) == L.pattern_dimension(N)


@pytest.mark.parametrize("M,J", CASES)
def test_theorem3_adds_or_grows_one_cycle(M, J):
    d_M, d_N, key = S.level_scaling(M, J)
    assert key is not None                          # every J here has a cyclic pattern
    assert d_M - d_N in (0, 1)
    # the direction is a point of P(M) of order exactly q modulo P(N)
    q = abs(L.det(L.as_matrix(J)))
    N = W.quotient(J, M)
    assert S.order_modulo_sublattice(M, N, key) == q


def test_cases_of_the_examples():
    assert S.level_scaling(((2, 0), (0, 2)), workloads.J_X)[:2] == (2, 1)
    assert S.level_scaling(((4, 0), (0, 2)), workloads.J_X)[:2] == (2, 2)
    assert S.level_scaling(((6, 0), (0, 1)), workloads.J_X)[:2] == (1, 1)
    assert S.level_scaling(((1, 4), (1, -4)), workloads.J_QUINCUNX)[:2] == (1, 1)


def test_quincunx_direction_is_the_wavelet_phase_point():
    """For |det J| = 2 the direction is the non-zero point of P(J) lifted;
    it is defined modulo P(N), so its key is congruent to v = J y0 of the
    wavelet phase modulo J Z^d (the same class of G(J))."""
    for M in (((32, 8), (-8, 32)), ((16, 8), (0, 16)), ((4096, 2048), (0, 4096))):
        for J in (workloads.J_QUINCUNX, workloads.J_X, workloads.J_Y, workloads.J_D):
            try:
                W.quotient(J, M)
            except ValueError:
                continue
            _, _, v = W.dilation_data(J)
            HJ, _ = L.hnf(L.as_matrix(J))
            key = S.level_scaling(M, J)[2]
            assert L.reduce_box(HJ, key) == L.reduce_box(HJ, v)
            assert key != tuple(0 for _ in key)


def test_non_cyclic_dilation_has_no_generator():
    assert S.generator_key(((2, 0), (0, 2))) is None
    assert S.generator_key(((2, 0, 0), (0, 2, 0), (0, 0, 2))) is None
    g = S.generator_key(((3, 0), (0, 1)))
    assert S.class_order(((3, 0), (0, 1)), g) == 3
