"""Pins of the oracle's exact integer algebra (Section 2.2) against the paper's
printed values, closed forms and brute force."""
import json
import os
from fractions import Fraction
from itertools import product

import numpy as np
import pytest

from oracle import lattice as L
import workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def test_table1_cycles():
    """Elementary divisors of the timing-table matrices (Section 6.1, Table 1)."""
    g = _gold("table1_cycles.json")
    for row in g["rows"]:
        M = workloads.table1_matrix(row["i"], g["k"], g["l"])
        eps = L.elementary_divisors(M)
        assert [e for e in eps if e > 1] == row["cycles"]
        assert eps[0] * eps[1] == g["k"] * g["l"]


def test_example1_invariants():
    """Example 1/2: eps = (1, 32), d_M = 1, M = J N (Section 2.2, Section 3)."""
    g = _gold("example1.json")
    M = tuple(map(tuple, g["M"]))
    assert L.elementary_divisors(M) == tuple(g["elementary_divisors"])
    assert L.pattern_dimension(M) == g["pattern_dimension"]
    assert L.matmul(g["J"], g["N"]) == M


def test_example2_printed_basis_on_consistent_matrix():
    """The printed Smith factors are a Smith form of [[3,-4],[5,4]]; the
    printed pattern basis y1 = R^{-1} e2 / 32 = (3/8, 1/32) lies in its
    lattice and the printed h1 = R^T e2 satisfies h1^T y1 = 1/32 (Lemma 1)."""
    g = _gold("example1.json")
    Q, E, R = (g["printed_snf"][k] for k in ("Q", "E", "R"))
    C = tuple(map(tuple, g["consistent_matrix"]))
    assert L.matmul(L.matmul(Q, E), R) == C
    assert L.matmul(L.matmul(Q, E), R) != tuple(map(tuple, g["M"]))
    assert abs(L.det(Q)) == 1 and abs(L.det(R)) == 1
    Rinv = L.inverse(R)
    y1 = tuple(x / 32 for x in L.matvec(Rinv, (0, 1)))
    assert y1 == tuple(Fraction(s) for s in g["y1"])
    assert all(x.denominator == 1 for x in L.matvec(C, y1))     # y1 in Lambda(C)
    h1 = L.matvec(L.transpose(R), (0, 1))
    assert list(h1) == g["h1"]
    assert sum(a * b for a, b in zip(h1, y1)) == Fraction(g["h1_dot_y1"])


@pytest.mark.parametrize("seed", range(12))
def test_det_adjugate_identity(seed):
    rng = np.random.default_rng(seed)
    d = 2 + seed % 3
    M = workloads.random_regular_matrix(rng, d)
    A = L.adjugate(M)
    D = L.det(M)
    assert L.matmul(M, A) == tuple(tuple(D * int(i == j) for j in range(d)) for i in range(d))
    assert abs(D) == abs(round(np.linalg.det(np.array(M, dtype=float))))


@pytest.mark.parametrize("seed", range(20))
def test_elementary_divisors_properties(seed):
    """eps_j | eps_{j+1}, product = |det M|, invariant under unimodular changes."""
    rng = np.random.default_rng(100 + seed)
    d = 2 + seed % 3
    M = workloads.random_regular_matrix(rng, d)
    eps = L.elementary_divisors(M)
    assert np.prod(eps) == abs(L.det(M))
    for a, b in zip(eps, eps[1:]):
        assert b % a == 0
    # left/right unimodular transformations leave the divisors unchanged
    U = ((1, 2) + (0,) * (d - 2),) + tuple(tuple(int(i == j) for j in range(d)) for i in range(1, d))
    V = tuple(tuple(int(i == j) + (3 if (i == d - 1 and j == 0) else 0) for j in range(d)) for i in range(d))
    assert L.elementary_divisors(L.matmul(L.matmul(U, M), V)) == eps


def test_elementary_divisors_diagonal():
    assert L.elementary_divisors(((4, 0), (0, 6))) == (2, 12)
    # p-parts: 2 -> (0,1,1), 3 -> (0,1,1), 5 -> (0,1,1)
    assert L.elementary_divisors(((6, 0, 0), (0, 10, 0), (0, 0, 15))) == (1, 30, 30)
    assert L.elementary_divisors(((4, 0, 0), (0, 9, 0), (0, 0, 25))) == (1, 1, 900)
    assert L.elementary_divisors(((8, 0), (0, 8))) == (8, 8)


@pytest.mark.parametrize("seed", range(16))
def test_hnf_box_is_complete_residue_system(seed):
    """The natural box of the Hermite form holds exactly one key per class of
    Z^d / M Z^d: brute force over the points of P(M) in [0,1)^d."""
    rng = np.random.default_rng(200 + seed)
    d = 2 + seed % 2
    M = workloads.random_regular_matrix(rng, d, max_det=300)
    H, U = L.hnf(M)
    m = abs(L.det(M))
    # shape properties
    for i in range(d):
        assert H[i][i] > 0
        for j in range(i):
            assert H[i][j] == 0
        for j in range(i + 1, d):
            assert 0 <= H[i][j] < H[i][i]
    assert L.matmul(M, U) == H and abs(L.det(U)) == 1
    pts = L.box_points(H)
    assert len(pts) == m
    brute = L.lattice_points_bruteforce(M)
    assert len(brute) == m
    Minv = L.inverse(M)
    reps = set()
    for g in pts:
        y = L.matvec(Minv, g)
        reps.add(tuple(x - (x.numerator // x.denominator) for x in y))
    assert reps == brute
    # reduce_box is idempotent and stays in the class
    for g in product(range(-7, 8), repeat=d):
        r = L.reduce_box(H, g)
        assert L.reduce_box(H, r) == r
        diff = L.matvec(Minv, [a - b for a, b in zip(g, r)])
        assert all(x.denominator == 1 for x in diff)


def test_hnf_of_upper_triangular_reduced_is_identity():
    """A matrix already in the normal form of Section 6.1 (eq.
    FFTexampleMatrix) is its own Hermite form."""
    for i in (0, 1, 5, 2047):
        M = workloads.table1_matrix(i)
        assert L.hnf(M)[0] == M


@pytest.mark.parametrize("seed", range(8))
def test_symmetric_representative(seed):
    rng = np.random.default_rng(300 + seed)
    M = workloads.random_regular_matrix(rng, 2, max_det=200)
    HT, _ = L.hnf(L.transpose(M))
    MTinv = L.inverse(L.transpose(M))
    for h in L.box_points(HT):
        hs, t, m = L.symmetric_rep_T(M, h)
        z = L.matvec(MTinv, [a - b for a, b in zip(h, hs)])
        assert all(x.denominator == 1 for x in z)           # same class
        y = L.matvec(MTinv, hs)
        assert all(Fraction(-1, 2) <= c < Fraction(1, 2) for c in y)


@pytest.mark.parametrize("seed", range(6))
def test_scaling_property_dimension(seed):
    """Theorem 3 (d_J = 1): d_M = d_N or d_M = d_N + 1 for M = J N."""
    rng = np.random.default_rng(400 + seed)
    for J in (workloads.J_X, workloads.J_Y, workloads.J_D, workloads.J_QUINCUNX):
        N = workloads.random_regular_matrix(rng, 2, max_det=500)
        M = L.matmul(J, N)
        dM, dN = L.pattern_dimension(M), L.pattern_dimension(N)
        assert dM in (dN, dN + 1)


@pytest.mark.parametrize("M", [((4, -3), (4, 5)), ((3, 1), (-2, 4)), ((2, 0), (0, 4)),
                               ((3, 1, 0), (0, 2, 1), (1, 0, 3)), ((5,),), ((6,),)])
def test_symmetric_representatives_bruteforce(M):
    """The symmetric representatives of the samples and of the frequencies are
    the points of P(M) (resp. P(M^T)) moved into [-1/2, 1/2)^d, enumerated by
    brute force (coordinates >= 1/2 shifted by -1), one per class."""
    M = L.as_matrix(M)
    for side, fn in (("samples", L.symmetric_rep), ("freqs", None)):
        A = M if side == "samples" else L.transpose(M)
        brute = set()
        for y in L.lattice_points_bruteforce(A):
            brute.add(tuple(c - 1 if c >= Fraction(1, 2) else c for c in y))
        H, _ = L.hnf(A)
        got = set()
        Ainv = L.inverse(A)
        for key in L.box_points(H):
            if fn is not None:
                t, m = fn(M, key)
            else:
                _, t, m = L.symmetric_rep_T(M, key)
            pt = tuple(Fraction(x, m) for x in t)
            assert all(Fraction(-1, 2) <= c < Fraction(1, 2) for c in pt)
            y = L.matvec(Ainv, key)
            assert all((a - b).denominator == 1 for a, b in zip(pt, y))
            got.add(pt)
        assert got == brute
