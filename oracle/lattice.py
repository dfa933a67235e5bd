"""Exact integer lattice algebra for the oracle (Section 2.2 of the paper).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Everything here works on Python integers (arbitrary precision), so no result
can overflow.  Matrices are tuples of row tuples.

Conventions (the paper leaves the order of a pattern open: any complete set
of congruence-class representatives, Section 2.2):
  * A sample of P(M) is addressed by its integer key g = M y in G(M) = Z^d/MZ^d
    (Section 2.2, generating group).
  * The *natural* order of G(M) is the box  prod_i [0, H_ii)  of the column
    Hermite normal form H = M U (U unimodular, H upper triangular with H_ii > 0
    and 0 <= H_ij < H_ii for j > i), enumerated in C order (last coordinate
    fastest).  It is a complete residue system because H is triangular.
  * Frequencies h in G(M^T) = Z^d/M^T Z^d use the same convention with M^T.
"""
from fractions import Fraction
from itertools import combinations, product
from math import gcd


def as_matrix(M):
    """Return M as a tuple of tuples of Python ints (square)."""
    rows = tuple(tuple(int(x) for x in row) for row in M)
    d = len(rows)
    if d == 0 or any(len(r) != d for r in rows):
        raise ValueError("square integer matrix expected")
    return rows


def transpose(M):
    M = as_matrix(M)
    d = len(M)
    return tuple(tuple(M[j][i] for j in range(d)) for i in range(d))


def matmul(A, B):
    """Exact product of two integer (or Fraction) matrices."""
    n, k, p = len(A), len(B), len(B[0])
    return tuple(tuple(sum(A[i][t] * B[t][j] for t in range(k)) for j in range(p))
                 for i in range(n))


def matvec(A, v):
    return tuple(sum(A[i][t] * v[t] for t in range(len(v))) for i in range(len(A)))


def det(M):
    """Determinant by exact Gaussian elimination over the rationals."""
    A = [[Fraction(x) for x in row] for row in as_matrix(M)]
    d = len(A)
    result = Fraction(1)
    for c in range(d):
        piv = next((r for r in range(c, d) if A[r][c] != 0), None)
        if piv is None:
            return 0
        if piv != c:
            A[c], A[piv] = A[piv], A[c]
            result = -result
        result *= A[c][c]
        for r in range(c + 1, d):
            f = A[r][c] / A[c][c]
            if f:
                A[r] = [A[r][j] - f * A[c][j] for j in range(d)]
    assert result.denominator == 1
    return int(result)


def minor(M, rows, cols):
    return det(tuple(tuple(M[r][c] for c in cols) for r in rows))


def adjugate(M):
    """Classical adjoint adj(M) = det(M) M^{-1}, from cofactors."""
    M = as_matrix(M)
    d = len(M)
    if d == 1:
        return ((1,),)
    adj = [[0] * d for _ in range(d)]
    for i in range(d):
        for j in range(d):
            rows = [r for r in range(d) if r != j]
            cols = [c for c in range(d) if c != i]
            adj[i][j] = (-1) ** (i + j) * minor(M, rows, cols)
    return tuple(tuple(r) for r in adj)


def inverse(M):
    """Exact rational inverse M^{-1} = adj(M)/det(M)."""
    D = det(M)
    if D == 0:
        raise ValueError("singular matrix")
    return tuple(tuple(Fraction(x, D) for x in row) for row in adjugate(M))


def elementary_divisors(M):
    """Elementary divisors eps_1 | eps_2 | ... | eps_d of eq. (SNF).

    Closed form, independent of any elimination: eps_k = D_k / D_{k-1}, where
    D_k is the gcd of all k x k minors of M (determinantal divisors).  The
    divisors are unique, so this pins the Smith form of Section 2.2.
    """
    M = as_matrix(M)
    d = len(M)
    if det(M) == 0:
        raise ValueError("singular matrix")
    D = [1]
    for k in range(1, d + 1):
        g = 0
        for rows in combinations(range(d), k):
            for cols in combinations(range(d), k):
                g = gcd(g, minor(M, rows, cols))
        D.append(abs(g))
    return tuple(D[k] // D[k - 1] for k in range(1, d + 1))


def pattern_dimension(M):
    """d_M = number of elementary divisors greater than one (Section 2.2)."""
    return sum(1 for e in elementary_divisors(M) if e > 1)


def hnf(M):
    """Column Hermite normal form H = M U, U unimodular.

    H is upper triangular, H_ii > 0 and 0 <= H_ij < H_ii for j > i.  Only
    column operations are used, so H Z^d = M Z^d (the same lattice).
    Returns (H, U) with H = M U exactly.
    """
    M = as_matrix(M)
    d = len(M)
    if det(M) == 0:
        raise ValueError("singular matrix")
    H = [list(r) for r in M]
    U = [[int(i == j) for j in range(d)] for i in range(d)]

    def colop(dst, src, f):          # col_dst -= f * col_src
        for r in range(d):
            H[r][dst] -= f * H[r][src]
            U[r][dst] -= f * U[r][src]

    def colswap(a, b):
        for r in range(d):
            H[r][a], H[r][b] = H[r][b], H[r][a]
            U[r][a], U[r][b] = U[r][b], U[r][a]

    def colneg(a):
        for r in range(d):
            H[r][a] = -H[r][a]
            U[r][a] = -U[r][a]

    for i in range(d - 1, -1, -1):
        # gather gcd of row i over columns 0..i into column i (Euclid)
        while True:
            nz = [c for c in range(i + 1) if H[i][c] != 0]
            if len(nz) <= 1:
                break
            p = min(nz, key=lambda c: abs(H[i][c]))
            for c in nz:
                if c != p:
                    colop(c, p, H[i][c] // H[i][p])
        nz = [c for c in range(i + 1) if H[i][c] != 0]
        assert len(nz) == 1
        if nz[0] != i:
            colswap(nz[0], i)
        if H[i][i] < 0:
            colneg(i)
    # reduce the entries right of each diagonal element, bottom row first
    for i in range(d - 1, -1, -1):
        for j in range(i + 1, d):
            colop(j, i, H[i][j] // H[i][i])
    Ht = tuple(tuple(r) for r in H)
    Ut = tuple(tuple(r) for r in U)
    assert matmul(as_matrix(M), Ut) == Ht
    assert abs(det(Ut)) == 1
    return Ht, Ut


def box_shape(H):
    return tuple(H[i][i] for i in range(len(H)))


def reduce_box(H, v):
    """Representative of v + H Z^d inside prod_i [0, H_ii) (H from hnf)."""
    d = len(H)
    v = list(int(x) for x in v)
    for i in range(d - 1, -1, -1):
        q = v[i] // H[i][i]
        if q:
            for r in range(i + 1):
                v[r] -= q * H[r][i]
    return tuple(v)


def box_points(H):
    """All points of the natural box of H in C order (last axis fastest)."""
    return [tuple(p) for p in product(*[range(H[i][i]) for i in range(len(H))])]


def box_index(H, v):
    """C-order linear index of a reduced point v of the box of H."""
    idx = 0
    for i in range(len(H)):
        assert 0 <= v[i] < H[i][i]
        idx = idx * H[i][i] + v[i]
    return idx


def natural_index(H, v):
    """Linear index of the class of an arbitrary integer vector v."""
    return box_index(H, reduce_box(H, v))


def sign(x):
    return (x > 0) - (x < 0)


def phase_residue(M, h, g):
    """Integer r with h^T M^{-1} g = r/m (mod 1), m = |det M|.

    Exact: M^{-1} = adj(M)/det(M), so h^T M^{-1} g = sgn(det M) h^T adj(M) g / m.
    (Fourier matrix of Section 2.2.)
    """
    D = det(M)
    m = abs(D)
    A = adjugate(M)
    return (sign(D) * sum(h[i] * A[i][j] * g[j]
                          for i in range(len(h)) for j in range(len(g)))) % m


def symmetric_rep_T(M, h):
    """Symmetric representative h* of h + M^T Z^d.

    h* = M^T t/m with t/m = M^{-T} h reduced into [-1/2, 1/2)^d, i.e. the
    representative with M^{-T} h* in the half-open symmetric unit cube
    (the choice of representatives used in Section 6.2).  Returns (h*, t, m).
    """
    M = as_matrix(M)
    D = det(M)
    m = abs(D)
    A = adjugate(M)
    d = len(M)
    half = m // 2
    # M^{-T} h = adj(M)^T h / det(M) = sgn * adj(M)^T h / m
    t = [sign(D) * sum(A[k][j] * h[k] for k in range(d)) for j in range(d)]
    t = [((x + half) % m) - half for x in t]
    # for odd m, (x + half) % m - half lies in [-(m-1)/2, (m-1)/2]; the cube
    # [-1/2,1/2) then contains exactly these values, as required.
    MT = transpose(M)
    hs = [sum(MT[i][j] * t[j] for j in range(d)) for i in range(d)]
    assert all(x % m == 0 for x in hs)
    return tuple(x // m for x in hs), tuple(t), m


def symmetric_rep(M, g):
    """Symmetric representative of the sample point y = M^{-1} g of P(M).

    The representative of y + Z^d in [-1/2, 1/2)^d (Section 6.2's symmetric
    pattern), returned as the integer vector t with that point = t/m,
    m = |det M|: M^{-1} g = sgn(det M) adj(M) g / m, reduced coordinatewise
    into [-m/2, m/2).  Returns (t, m).
    """
    M = as_matrix(M)
    D = det(M)
    m = abs(D)
    A = adjugate(M)
    d = len(M)
    half = m // 2
    t = [sign(D) * sum(A[j][k] * g[k] for k in range(d)) for j in range(d)]
    return tuple(((x + half) % m) - half for x in t), m


def lattice_points_bruteforce(M):
    """Brute-force enumeration of P(M) = M^{-1} Z^d cap [0,1)^d (tiny m only).

    Returns the set of sample points as tuples of Fractions.  Independent of
    the Hermite form: scans the integer vectors g in the bounding box of
    M [0,1)^d and keeps those whose point y = M^{-1} g lies in [0,1)^d.
    """
    M = as_matrix(M)
    d = len(M)
    Minv = inverse(M)
    lo = [0] * d
    hi = [0] * d
    for corner in product((0, 1), repeat=d):
        img = matvec(M, corner)
        for i in range(d):
            lo[i] = min(lo[i], img[i])
            hi[i] = max(hi[i], img[i])
    pts = set()
    for g in product(*[range(lo[i], hi[i] + 1) for i in range(d)]):
        y = matvec(Minv, g)
        if all(0 <= c < 1 for c in y):
            pts.add(tuple(y))
    return pts
