"""Differentiable full convolution and a sigma-parameterised Gaussian PSF.

ConvFull.apply(x, h) computes Y = X (x) H with conv_full_nd.  Its backward
is hand-written: for an upstream gradient G (extent m+2p),
  dX = (A^h)^T G = conv_adjoint_nd(G, H)            (Property 2)
  dH[j] = sum_k X[k] G[k+j] = conv_dH_nd(X, G)       (Property 1 with X as
                                                      the template)
Both run in the library's kernels.  GaussianPSF builds a normalised
separable Gaussian from log-sigmas with ordinary torch ops, so autograd
carries dH on to the sigmas (blind PSF refinement).  JointRefiner
alternates projected steps on X with optimizer steps on the sigmas, both
from one backward pass of the loss 1/2 ||X (x) H(sigma) - Y||^2.
"""
import torch

from . import conv_adjoint_nd, conv_dH_nd, conv_full_nd


class ConvFull(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, h, precision="native"):
        x = x.contiguous()
        h = h.contiguous()
        ctx.save_for_backward(x, h)
        ctx.precision = precision
        return conv_full_nd(x, h, precision=precision)

    @staticmethod
    def backward(ctx, gy):
        x, h = ctx.saved_tensors
        gy = gy.contiguous()
        dx = conv_adjoint_nd(gy, h, precision=ctx.precision) if ctx.needs_input_grad[0] else None
        dh = conv_dH_nd(x, gy, tuple(h.shape)) if ctx.needs_input_grad[1] else None
        return dx, dh, None


def conv_full_ad(x, h, precision="native"):
    """Differentiable Y = X (x) H."""
    return ConvFull.apply(x, h, precision)


class GaussianPSF(torch.nn.Module):
    """h(t) proportional to exp(-sum_i t_i^2 / (2 sigma_i^2)) on t_i in
    [-p_i, p_i], normalised to sum 1, with sigma_i = exp(log_sigma_i)."""

    def __init__(self, shape, sigmas, dtype=torch.float32, device="cuda"):
        super().__init__()
        for e in shape:
            if e % 2 != 1:
                raise ValueError("PSF extents must be odd")
        self.shape = tuple(int(e) for e in shape)
        self.log_sigma = torch.nn.Parameter(torch.log(torch.tensor(sigmas, dtype=torch.float64, device=device)))
        self.dtype = dtype

    def sigmas(self):
        return torch.exp(self.log_sigma)

    def forward(self):
        s = self.sigmas()
        h = None
        for ax, e in enumerate(self.shape):
            p = (e - 1) // 2
            t = torch.arange(-p, p + 1, dtype=torch.float64, device=s.device)
            f = torch.exp(-(t * t) / (2.0 * s[ax] * s[ax]))
            f = f / f.sum()
            h = f if h is None else h[..., None] * f
        return h.to(self.dtype).contiguous()


class JointRefiner:
    """Joint refinement of X and the PSF widths on 1/2 ||X (x) H(sigma) - Y||^2.

    One step is one forward (ConvFull) and its hand-written backward, which
    gives dX (the transpose) and dH (the PSF-gradient kernel; autograd carries
    it on to log sigma through GaussianPSF).  Then X takes the projected
    gradient step of the paper's method, X <- max(X - delta dX, 0) with
    delta = 1/||H||_1^2 (at most 1/L, so the X step alone never increases the
    loss), and the sigmas take one step of `opt`.

    With X unknown the loss alone does not pin sigma down from below: for
    any narrower Gaussian the true object blurred by the missing width is a
    non-negative X with the same noise-free fit, and a narrower PSF lets X
    follow more of the noise."""

    def __init__(self, y, x0, psf_model, lr=0.05):
        self.y = y
        self.x = x0.detach().clone().contiguous()
        self.psf = psf_model
        self.opt = torch.optim.Adam(psf_model.parameters(), lr=lr)

    def step(self):
        self.opt.zero_grad()
        x = self.x.requires_grad_(True)
        h = self.psf()
        loss = 0.5 * ((ConvFull.apply(x, h) - self.y) ** 2).sum()
        loss.backward()
        with torch.no_grad():  # delta stays on the device: no host wait per step
            delta = (1.0 / h.detach().abs().sum(dtype=torch.float64) ** 2).to(x.dtype)
            self.x = torch.clamp(x.detach() - delta * x.grad, min=0).contiguous()
        self.opt.step()
        return loss.detach()
