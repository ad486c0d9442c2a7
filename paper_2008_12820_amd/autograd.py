"""Differentiable forms of the transport map and the regulariser.

TransportMap: (m0, v) -> m(1), the semi-Lagrangian solution of the
constraint of eq. "problem" (d_t m + v . grad m = 0, m(0) = m0) with N_t RK2
steps and cubic Lagrange interpolation.  Its backward is the hand-written
adjoint transport of eq. "adj-transport" run by liblddmm (final value
dL/dm(1)), which gives dL/dm0 = lam(0) and dL/dv = -int_0^1 lam grad m dt
(the discretise-after-optimise adjoint of the paper; it agrees with finite
differences of the discrete map to discretisation error).  The forward pass
keeps m_j for every time step as the checkpoints the backward reads.

RegEnergy: v -> 1/2 sum_x (A v) . v (plain sum), backward A v, so that
beta * RegEnergy(v) is the beta/2 reg(v) term of eq. "problem" in plain sums.
"""
import torch

from .plan import Plan


class _Transport(torch.autograd.Function):
    @staticmethod
    def forward(ctx, m0, v, plan):
        ckpt = torch.empty((plan.nt + 1,) + plan.shape, device=plan.device, dtype=torch.float32)
        m1 = plan.transport_forward(m0.detach(), v.detach(), ckpt)
        ctx.save_for_backward(ckpt, v.detach())
        ctx.plan = plan
        return m1

    @staticmethod
    def backward(ctx, grad_m1):
        ckpt, v = ctx.saved_tensors
        want_m0, want_v = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (want_m0 or want_v):
            return None, None, None
        gm0, gv = ctx.plan.transport_vjp(ckpt, v, grad_m1.contiguous().to(torch.float32),
                                         want_m0=want_m0, want_v=want_v)
        return gm0, gv, None


class _RegEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v, plan):
        e, Av = plan.reg_energy(v.detach(), want_Av=True)
        ctx.save_for_backward(Av)
        return torch.tensor(e, device=v.device, dtype=torch.float32)

    @staticmethod
    def backward(ctx, grad_e):
        (Av,) = ctx.saved_tensors
        return grad_e * Av, None


class TransportMap(torch.nn.Module):
    """m1 = TransportMap(shape, nt)(m0, v); owns a transport-only plan."""

    def __init__(self, shape, nt, reg=2, beta=1e-4, device=None):
        super().__init__()
        self.plan = Plan(shape, nt, reg=reg, beta=beta, device=device, transport_only=True)

    def forward(self, m0, v):
        return _Transport.apply(m0, v, self.plan)

    def reg_energy(self, v):
        return _RegEnergy.apply(v, self.plan)


def transport(m0, v, plan):
    return _Transport.apply(m0, v, plan)


def reg_energy(v, plan):
    return _RegEnergy.apply(v, plan)
