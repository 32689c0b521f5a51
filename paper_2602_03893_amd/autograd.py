"""torch.autograd.Function over the HIP operators.

Forward: y = A(x; sigma) (gpair_forward).  Backward: the hand-written adjoint
(gpair_adjoint) gives dL/dA and dL/dsigma from dL/dy; the taps are recomputed
in the backward, so only A and sigma are saved (no per-tap intermediates and
no copy of y).  The adjoint is the transpose of the forward (arXiv 2602.03893,
Methods, "Adjoint Operator" subsection) and the sigma-gradient the derivative
of Eq. (single_forward) with respect to sigma.
"""
import torch


def _checked(plan, call, what):
    """Run `call` and raise if it met widths the operators had to clamp (or
    covariances they had to replace): the result and its backward would then
    belong to another function than the one the caller's parameters define.
    Reads the plan's violation counter before and after (two stream syncs)."""
    before = plan.sigma_violations()
    out = call()
    met = plan.sigma_violations() - before
    if met:
        raise ValueError(f"{what}: {met} kernel(s) outside the admitted range (sigma in "
                         f"(0, sigma_max], covariances positive definite with largest "
                         f"eigenvalue <= sigma_max^2); project the parameters first, or "
                         f"pass check=False to accept the clamped operator")
    return out


class GpairForward(torch.autograd.Function):
    """y = A(x; sigma) (gpair_forward); `check` (default True) raises
    ValueError when a sigma_k lies outside (0, sigma_max], which the operator
    would otherwise clamp, giving the gradient of the clamped function."""

    @staticmethod
    def forward(ctx, A, sigma, plan, check=True):
        A = A.contiguous()
        sigma = sigma.contiguous()
        ctx.plan = plan
        ctx.save_for_backward(A, sigma)
        if check:
            return _checked(plan, lambda: plan.forward(A, sigma), "gpair_forward")
        return plan.forward(A, sigma)

    @staticmethod
    def backward(ctx, grad_y):
        A, sigma = ctx.saved_tensors
        want_a = ctx.needs_input_grad[0]
        want_s = ctx.needs_input_grad[1]
        if not (want_a or want_s):
            return None, None, None, None
        gA, gS = ctx.plan.adjoint(A, sigma, grad_y.contiguous(), want_sigma=want_s)
        return (gA if want_a else None), (gS if want_s else None), None, None


def gpair_forward(A, sigma, plan, check=True):
    """Differentiable y = A(x; sigma) for the given bound Plan (see
    GpairForward for `check`)."""
    return GpairForward.apply(A, sigma, plan, check)


class AssaForward(torch.autograd.Function):
    """y = S(h * P_up(x)) with one shared sigma (the ASSA operators); the
    backward is the hand-written transpose (gpair_assa_adjoint).  sigma is a
    Python float: the ASSA kernel h is not differentiated."""

    @staticmethod
    def forward(ctx, x, sigma, plan):
        ctx.plan = plan
        ctx.sigma = float(sigma)
        return plan.assa_forward(x.contiguous(), ctx.sigma)

    @staticmethod
    def backward(ctx, grad_y):
        if not ctx.needs_input_grad[0]:
            return None, None, None
        return ctx.plan.assa_adjoint(ctx.sigma, grad_y.contiguous()), None, None


def assa_forward(x, sigma, plan):
    """Differentiable ASSA forward y = S(h * P_up(x)) for a bound Plan."""
    return AssaForward.apply(x, sigma, plan)


class AnisoForward(torch.autograd.Function):
    """y = A(x; Sigma) for anisotropic kernels (gpair_forward_aniso); the
    backward is the hand-written adjoint (gpair_adjoint_aniso): dL/dA and
    dL/dSigma for the six covariance parameters (xx, yy, zz, xy, xz, yz) at
    fixed windows, taps recomputed.  sigma6 is (6, M).  `check` (default
    True) raises ValueError when a covariance lies outside the admitted set,
    which the operator would otherwise replace by sigma_max^2 I."""

    @staticmethod
    def forward(ctx, A, sigma6, plan, check=True):
        A = A.contiguous()
        sigma6 = sigma6.contiguous()
        ctx.plan = plan
        ctx.save_for_backward(A, sigma6)
        if check:
            return _checked(plan, lambda: plan.forward_aniso(A, sigma6), "gpair_forward_aniso")
        return plan.forward_aniso(A, sigma6)

    @staticmethod
    def backward(ctx, grad_y):
        A, sigma6 = ctx.saved_tensors
        want_a = ctx.needs_input_grad[0]
        want_s = ctx.needs_input_grad[1]
        if not (want_a or want_s):
            return None, None, None, None
        gA, gS = ctx.plan.adjoint_aniso(A, sigma6, grad_y.contiguous(), want_sigma=want_s)
        return (gA if want_a else None), (gS if want_s else None), None, None


def aniso_forward(A, sigma6, plan, check=True):
    """Differentiable y = A(x; Sigma) of anisotropic kernels for a bound Plan
    (see AnisoForward for `check`)."""
    return AnisoForward.apply(A, sigma6, plan, check)
