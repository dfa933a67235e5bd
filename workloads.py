"""Seeded synthetic workloads shared by the tests, the smoke check and the
benchmark.

This module holds inputs only: matrices, seeds, shapes and random samples.
It contains none of the method's arithmetic (no determinants, normal forms,
index maps or transforms), so both the oracle and the GPU path may read it
without sharing any computation.

Sample data follow the paper's timing experiment (Section 6.1: randomly
generated data values): complex samples whose real and imaginary parts are
i.i.d. N(0, 1), drawn in float64 from numpy's PCG64 ``default_rng(seed)``.
GPU inputs are those values rounded to complex64; the oracle is fed the same
rounded values upcast to complex128, so reported errors measure the kernels.
"""
import numpy as np

# quincunx dilation J = [[1, 1], [1, -1]] (|det J| = 2)
J_QUINCUNX = ((1, 1), (1, -1))
# the dilation set of Section 6.2
J_X = ((2, 0), (0, 1))
J_Y = ((1, 0), (0, 2))
J_D = ((1, -1), (1, 1))
# |det J| = 4: four channels per level
J_2I = ((2, 0), (0, 2))

CONFIGS = {
    # d = 2 plain method: m = 1088, one quincunx level
    "small": dict(M=((32, 8), (-8, 32)), J=J_QUINCUNX, levels=1, batch=1, seed=1),
    # d = 2 large: m = 2^24, forward/inverse FFT and 8 quincunx levels
    "large": dict(M=((4096, 2048), (0, 4096)), J=J_QUINCUNX, levels=8, batch=1, seed=2),
    # d = 3 precision case: m = 2^24
    "d3": dict(M=((256, 64, 0), (0, 256, 64), (0, 0, 256)), J=None, levels=0, batch=1, seed=3),
    # batched: 512 instances of 2 x 2 upper-triangular M (see batched_matrices)
    "batched": dict(M=None, J=None, levels=0, batch=512, seed=4),
    # differentiation: m = 2^20, batch 16, 4 quincunx levels
    "grad": dict(M=((1024, 256), (0, 1024)), J=J_QUINCUNX, levels=4, batch=16, seed=5,
                 target_seed=6),
    # four channels per level: the large M with J = 2 I, 4 levels (the same
    # final resolution m_L = 2^16 as 8 quincunx levels)
    "q4": dict(M=((4096, 2048), (0, 4096)), J=J_2I, levels=4, batch=1, seed=7),
    # the timing table of Section 6.1: M = [[2048, i], [0, 2048]], m = 2^22,
    # for every divisor i of 2048 and i = 0 (see table1_matrix)
    "table1": dict(M=None, J=None, levels=0, batch=1, seed=8,
                   i=(1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 0)),
    # the wavelet experiment of Section 6.2 without its box splines: point
    # values on M = diag(512, 512), one level for each dilation of J_x, J_y, J_d
    "dirichlet_1level": dict(M=((512, 0), (0, 512)), J=(J_X, J_Y, J_D), levels=1, batch=1,
                             seed=9),
}


def complex_normal(seed, shape, dtype=np.complex64):
    """i.i.d. complex N(0,1) samples (real and imaginary parts each N(0,1))."""
    rng = np.random.default_rng(seed)
    shape = tuple(shape) if not isinstance(shape, int) else (shape,)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    z = (re + 1j * im)
    return z.astype(dtype)


def batched_matrices(seed=4, count=512):
    """Upper-triangular instances M = [[2^a, c], [0, 2^b]] of the pattern
    normal form (Section 6.1, eq. FFTexampleMatrix), with a + b = s drawn
    uniformly from 10..18, a uniform in 0..s and c uniform in [0, 2^a)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        s = int(rng.integers(10, 19))
        a = int(rng.integers(0, s + 1))
        b = s - a
        c = int(rng.integers(0, 1 << a))
        out.append(((1 << a, c), (0, 1 << b)))
    return out


def table1_matrix(i, k=2048, l=2048):
    """The matrices of the timing table of Section 6.1: [[l, i], [0, k]]."""
    return ((l, i), (0, k))


def random_regular_matrix(rng, d, lo=-6, hi=7, max_det=4096):
    """A random regular integer d x d matrix with 0 < |det| <= max_det.

    The determinant test uses a plain float estimate only to reject samples;
    exact values are computed by whoever consumes the matrix.
    """
    while True:
        M = rng.integers(lo, hi, size=(d, d))
        dv = abs(round(float(np.linalg.det(M.astype(np.float64)))))
        if 0 < dv <= max_det:
            return tuple(tuple(int(x) for x in row) for row in M)
