"""Float64 torch re-implementation of the oracle for gradient checks.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The lattice FFT is the Hermite-form row/column FFT of ``oracle.dft`` written
with torch operations (``torch.fft.fft`` along each axis, exact-residue
twiddles, a final gather to natural frequency order); the split and unsplit of
``oracle.wavelet`` are written with gathers.  Everything runs on the CPU in
complex128, so torch autograd gives an independent FP64 reference for the
gradients of any loss built from decompose/reconstruct with respect to the
samples and the real scaling masks.

The q-channel pyramid (q = |det J| > 2) is ``oracle.wavelet_q`` written the
same way: per fiber the matrix with first row u = a / sqrt q and the other
rows those of the reflection I - 2 v v^T / (v^T v), v = u + sigma e_0,
sigma = sign(u_0) (a constant of the fiber: its derivative is zero wherever it
exists), so autograd differentiates through the reflection.

Pins: central finite differences of the loss along random directions
(complex samples and real masks); Parseval's closed form
grad ||F x||^2 = 2 x, and grad ||D x||^2 = 2 x for a pyramid D that is
unitary (Dirichlet masks); the forward values equal ``oracle.wavelet`` and
``oracle.wavelet_q``.
"""
import numpy as np
import torch

from . import dft
from . import lattice as L
from . import wavelet as W
from . import wavelet_q as WQ


class TorchLattice:
    """Differentiable FP64 lattice DFT on natural orders (forward, sign -)."""

    def __init__(self, M):
        M = L.as_matrix(M)
        self.M = M
        d = len(M)
        H, U = L.hnf(M)
        m = abs(L.det(M))
        self.m = m
        self.shape = L.box_shape(H)
        adjH = L.adjugate(H)
        self.tw = []
        for j in range(d):
            if j == 0:
                self.tw.append(None)
                continue
            idx = [np.arange(self.shape[i], dtype=np.int64) for i in range(j + 1)]
            res = np.zeros(tuple(self.shape[:j]) + (1,), dtype=np.int64)
            for i in range(j):
                coef = adjH[i][j] % m
                v = (idx[i] * coef) % m
                res = (res + v.reshape([-1 if k == i else 1 for k in range(j + 1)])) % m
            r = (res * idx[j].reshape([1] * j + [-1])) % m
            t = np.exp(-2j * np.pi * r.astype(np.float64) / m)
            t = t.reshape(t.shape + (1,) * (d - j - 1))
            self.tw.append(torch.from_numpy(t))
        HT, _ = L.hnf(L.transpose(M))
        Uinv = L.inverse(U)
        UinvT = np.array(L.transpose(tuple(tuple(int(x) for x in row) for row in Uinv)), dtype=np.int64)
        ht = dft._natural_keys(H)
        nat = dft.box_index_np(HT, dft.reduce_box_np(HT, ht @ UinvT.T))
        perm = np.empty(m, dtype=np.int64)
        perm[nat] = np.arange(m, dtype=np.int64)
        self.perm = torch.from_numpy(perm)

    def __call__(self, x):
        B = x.shape[0]
        X = x.reshape((B,) + tuple(self.shape))
        for j, t in enumerate(self.tw):
            if t is not None:
                X = X * t
            X = torch.fft.fft(X, dim=1 + j)
        return X.reshape(B, self.m)[:, self.perm] / np.sqrt(self.m)


class TorchPair:
    """Forward transform on M and its inverse (via the transform on M^T)."""

    def __init__(self, M):
        self.f = TorchLattice(M)
        self.ft = TorchLattice(L.transpose(L.as_matrix(M)))

    def forward(self, x):
        return self.f(x)

    def inverse(self, y):
        return torch.conj(self.ft(torch.conj(y))).resolve_conj()


class TorchPyramid:
    """FP64 pyramid: decompose / reconstruct, masks as real tensors."""

    def __init__(self, M, J, levels):
        self.mats = W.level_matrices(M, J, levels)
        self.J = J
        self.top = TorchPair(self.mats[0][0])
        self.lv = []
        for (Ml, Nl) in self.mats:
            _, i0, i1, rho, ml = W._fiber_maps(Ml, J)
            phi = torch.from_numpy(np.exp(-2j * np.pi * rho.astype(np.float64) / ml))
            inv = np.argsort(np.concatenate([i0, i1]))
            self.lv.append(dict(i0=torch.from_numpy(i0), i1=torch.from_numpy(i1), phi=phi,
                                inv=torch.from_numpy(inv), fftN=TorchPair(Nl), ml=ml))
        # (level, channel, offset, size) of the coefficient blocks: each
        # level's wavelet channel, then the last level's low-pass channel
        offs = np.cumsum([0] + [v["ml"] // 2 for v in self.lv])
        self.blocks = [(l, 1, int(offs[l]), v["ml"] // 2) for l, v in enumerate(self.lv)]
        self.blocks.append((levels - 1, 0, int(offs[-1]), self.lv[-1]["ml"] // 2))

    def _split(self, l, ah, mask):
        v = self.lv[l]
        a0 = mask[v["i0"]].to(torch.complex128)
        a1 = mask[v["i1"]].to(torch.complex128)
        x0 = ah[:, v["i0"]]
        x1 = ah[:, v["i1"]]
        r2 = np.sqrt(2.0)
        d1 = (a0 * x0 + a1 * x1) / r2
        d2 = torch.conj(v["phi"]) * (a1 * x0 - a0 * x1) / r2
        return d1, d2

    def _unsplit(self, l, d1, d2, mask):
        v = self.lv[l]
        a0 = mask[v["i0"]].to(torch.complex128)
        a1 = mask[v["i1"]].to(torch.complex128)
        r2 = np.sqrt(2.0)
        y2 = v["phi"] * d2
        h0 = (a0 * d1 + a1 * y2) / r2
        h1 = (a1 * d1 - a0 * y2) / r2
        return torch.cat([h0, h1], dim=1)[:, v["inv"]]

    def decompose(self, x, masks):
        ah = self.top.forward(x)
        blocks = []
        for l, mk in enumerate(masks):
            d1, d2 = self._split(l, ah, mk)
            blocks.append(self.lv[l]["fftN"].inverse(d2))
            ah = d1
        blocks.append(self.lv[-1]["fftN"].inverse(ah))
        return torch.cat(blocks, dim=1)

    def reconstruct(self, c, masks):
        sizes = [v["ml"] // 2 for v in self.lv]
        offs = np.cumsum([0] + sizes)
        ah = self.lv[-1]["fftN"].forward(c[:, offs[-1]:offs[-1] + sizes[-1]])
        for l in range(len(self.lv) - 1, -1, -1):
            d2 = self.lv[l]["fftN"].forward(c[:, offs[l]:offs[l] + sizes[l]])
            ah = self._unsplit(l, ah, d2, masks[l])
        return self.top.inverse(ah)


class TorchPyramidQ:
    """FP64 q-channel pyramid (q = |det J| > 2), masks as real tensors, with
    the fibers, channel matrices and coefficient layout of oracle.wavelet_q."""

    def __init__(self, M, J, levels):
        self.mats = W.level_matrices(M, J, levels)
        self.q = abs(L.det(L.as_matrix(J)))
        self.top = TorchPair(self.mats[0][0])
        self.lv = []
        for (Ml, Nl) in self.mats:
            _, idx, ml = WQ.fiber_maps(Ml, J)
            # natural position h <- (member l, fiber k) for the synthesis
            inv = np.argsort(idx.reshape(-1))
            self.lv.append(dict(idx=torch.from_numpy(idx), inv=torch.from_numpy(inv),
                                fftN=TorchPair(Nl), ml=ml))
        self.blocks = WQ.coeff_layout(M, J, levels)

    def _matrix(self, l, mask):
        """S (q, q, n) of every fiber: row 0 is u, rows j >= 1 those of the
        reflection I - 2 v v^T / (v^T v)."""
        q = self.q
        u = mask[self.lv[l]["idx"]] / np.sqrt(q)
        sigma = torch.where(u[0].detach() >= 0, 1.0, -1.0).to(u.dtype)
        v = torch.cat([(u[0] + sigma)[None], u[1:]], dim=0)
        vv = torch.sum(v * v, dim=0)
        eye = torch.eye(q, dtype=u.dtype)[:, :, None]
        H = eye - 2.0 * v[:, None, :] * v[None, :, :] / vv
        return torch.cat([u[None], H[1:]], dim=0)

    def _split(self, l, ah, mask):
        S = self._matrix(l, mask).to(torch.complex128)
        x = ah[:, self.lv[l]["idx"]]                      # (B, q, n)
        return torch.einsum("jln,bln->bjn", S, x)         # dhat_j = sum_l S[j, l] x_l

    def _unsplit(self, l, dh, mask):
        S = self._matrix(l, mask).to(torch.complex128)
        x = torch.einsum("jln,bjn->bln", S, dh)           # x_l = sum_j S[j, l] dhat_j
        return x.reshape(x.shape[0], -1)[:, self.lv[l]["inv"]]

    def decompose(self, x, masks):
        ah = self.top.forward(x)
        blocks = []
        for l, mk in enumerate(masks):
            dh = self._split(l, ah, mk)
            for j in range(1, self.q):
                blocks.append(self.lv[l]["fftN"].inverse(dh[:, j]))
            ah = dh[:, 0]
        blocks.append(self.lv[-1]["fftN"].inverse(ah))
        return torch.cat(blocks, dim=1)

    def reconstruct(self, c, masks):
        _, _, off, n = self.blocks[-1]
        ah = self.lv[-1]["fftN"].forward(c[:, off:off + n])
        for l in range(len(self.lv) - 1, -1, -1):
            chans = [ah] + [self.lv[l]["fftN"].forward(c[:, o:o + n])
                            for (lv, j, o, n) in self.blocks if lv == l and j > 0]
            ah = self._unsplit(l, torch.stack(chans, dim=1), masks[l])
        return self.top.inverse(ah)


def make_pyramid(M, J, levels):
    """TorchPyramid for |det J| = 2, TorchPyramidQ otherwise."""
    q = abs(L.det(L.as_matrix(J)))
    return TorchPyramid(M, J, levels) if q == 2 else TorchPyramidQ(M, J, levels)


def pyramid_loss(pyr, x, masks, target, weights, masks_rec=None):
    """sum_l w_l ||wavelet channels of level l||^2 +
    ||reconstruct(decompose(x)) - target||^2 (the differentiation workload's
    loss; channels in the time domain).  masks_rec: the masks the
    reconstruction uses (default: the same tensors), so the two contributions
    to a mask gradient can be taken apart."""
    c = pyr.decompose(x, masks)
    loss = 0.0
    for (lvl, ch, off, n) in pyr.blocks:
        if ch == 0:
            continue
        blk = c[:, off:off + n]
        loss = loss + weights[lvl] * torch.sum(blk.real ** 2 + blk.imag ** 2)
    r = pyr.reconstruct(c, masks if masks_rec is None else masks_rec) - target
    return loss + torch.sum(r.real ** 2 + r.imag ** 2)


def loss_and_grads(M, J, levels, x, masks, target, weights, parts=False):
    """FP64 loss and autograd gradients w.r.t. x (complex) and the masks.

    parts=True: the mask gradients are returned as two lists, the
    contribution through the decomposition and the one through the
    reconstruction (their sum is the mask gradient)."""
    pyr = make_pyramid(M, J, levels)
    xt = torch.tensor(np.asarray(x), dtype=torch.complex128, requires_grad=True)
    mt = [torch.tensor(np.asarray(mk), dtype=torch.float64, requires_grad=True) for mk in masks]
    ms = ([torch.tensor(np.asarray(mk), dtype=torch.float64, requires_grad=True) for mk in masks]
          if parts else None)
    tt = torch.tensor(np.asarray(target), dtype=torch.complex128)
    loss = pyramid_loss(pyr, xt, mt, tt, weights, masks_rec=ms)
    loss.backward()
    if parts:
        return (float(loss.detach()), xt.grad.numpy(), [m.grad.numpy() for m in mt],
                [m.grad.numpy() for m in ms])
    return float(loss.detach()), xt.grad.numpy(), [m.grad.numpy() for m in mt]
