"""torch.autograd.Function wrappers over the library's hand-written adjoints.

Gradients follow PyTorch's convention for complex tensors (for a real loss L,
grad_z = dL/dRe z + i dL/dIm z), so a linear map A has backward A^H:
  * lattice FFT: F(M) is unitary, its adjoint is the inverse transform;
  * wavelet decomposition D: the backward is lwt_decompose_backward (the
    synthesis with the same masks), plus d loss / d mask per level;
  * reconstruction S: the backward is lwt_reconstruct_backward (the analysis
    with the same masks), plus d loss / d mask per level.
Every step runs in the HIP kernels; this module only wires buffers.
"""
import torch

from .lfft import LatticePlan, WaveletPlan, get_plan


class LatticeFFT(torch.autograd.Function):
    """y = F(M) x (natural orders), x: complex64 [batch, m] on the GPU."""

    @staticmethod
    def forward(ctx, x, plan):
        ctx.plan = plan
        return plan.forward(x.contiguous())

    @staticmethod
    def backward(ctx, g):
        return ctx.plan.inverse(g.contiguous()), None


class LatticeIFFT(torch.autograd.Function):
    """x = F(M)^{-1} y."""

    @staticmethod
    def forward(ctx, y, plan):
        ctx.plan = plan
        return plan.inverse(y.contiguous())

    @staticmethod
    def backward(ctx, g):
        return ctx.plan.forward(g.contiguous()), None


class BasisChange(torch.autograd.Function):
    """a = B s: point values on P(M) -> coefficients in the orthonormal
    translates of the Dirichlet kernel (lfft_basis_change).  B = F^H W F with
    a real diagonal W, so B is self-adjoint and its backward is B itself."""

    @staticmethod
    def forward(ctx, s, plan):
        ctx.plan = plan
        return plan.basis_change(s.contiguous())

    @staticmethod
    def backward(ctx, g):
        return ctx.plan.basis_change(g.contiguous()), None


class WaveletDecompose(torch.autograd.Function):
    """coeffs = D(x; masks) with the pyramid layout of lwt_decompose."""

    @staticmethod
    def forward(ctx, x, plan, *masks):
        # the saved Fourier inputs are needed for mask gradients (and, for
        # q = 2, the saved path is the one-launch-per-level schedule)
        keep = plan.q == 2 or any(ctx.needs_input_grad[2:])
        saved = plan.new_saved(x.device) if keep else None
        c = plan.decompose(x.contiguous(), list(masks), saved=saved)
        ctx.plan = plan
        ctx.save_for_backward(saved, *masks)
        return c

    @staticmethod
    def backward(ctx, g):
        saved, *masks = ctx.saved_tensors
        plan = ctx.plan
        need_m = any(ctx.needs_input_grad[2:])
        gm = [torch.empty_like(m) for m in masks] if need_m else None
        gx = plan.decompose_backward(g.contiguous(), saved, masks, grad_masks=gm)
        return (gx, None) + (tuple(gm) if need_m else (None,) * len(masks))


class WaveletReconstruct(torch.autograd.Function):
    """x = S(coeffs; masks), the inverse pyramid."""

    @staticmethod
    def forward(ctx, c, plan, *masks):
        keep = plan.q == 2 or any(ctx.needs_input_grad[2:])
        saved = plan.new_saved(c.device) if keep else None
        x = plan.reconstruct(c.contiguous(), list(masks), saved=saved)
        ctx.plan = plan
        ctx.save_for_backward(saved, *masks)
        return x

    @staticmethod
    def backward(ctx, g):
        saved, *masks = ctx.saved_tensors
        plan = ctx.plan
        need_m = any(ctx.needs_input_grad[2:])
        gm = [torch.empty_like(m) for m in masks] if need_m else None
        gc = plan.reconstruct_backward(g.contiguous(), saved, masks, grad_masks=gm)
        return (gc, None) + (tuple(gm) if need_m else (None,) * len(masks))


def lattice_fft(x, M):
    return LatticeFFT.apply(x, get_plan(M, x.numel() // x.shape[-1]))


def lattice_ifft(y, M):
    return LatticeIFFT.apply(y, get_plan(M, y.numel() // y.shape[-1]))


def samples_to_coeffs(s, M):
    return BasisChange.apply(s, get_plan(M, s.numel() // s.shape[-1]))


def wavelet_decompose(x, plan, masks):
    return WaveletDecompose.apply(x, plan, *masks)


def wavelet_reconstruct(c, plan, masks):
    return WaveletReconstruct.apply(c, plan, *masks)


def channel_blocks(plan):
    """(offset, length) of every coefficient block of one signal, in the
    library's layout (lwt_coeff_layout): the wavelet channels of every level,
    then the final low-pass block."""
    return [(off, n) for (_, _, off, n) in plan.coeff_blocks()]
