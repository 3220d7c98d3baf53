"""Differentiable terminal potential A(T) of the linearised space-time system.

``terminal_potential(problem, a0, f)`` solves J x = b(a0, f) on the GPU and
returns x_A at the last slab.  The right-hand side is

    b = b_fixed + e_{A,1} (M_A / dt) a0 + e_u f

(the initial potential enters the induction row of the first slab, the forcing
the momentum rows of every slab; paper, recurrence eq. (recurrence)).  The
backward pass solves the adjoint system J^T lam = e_{A,Nt} grad with
``st_adjoint_solve`` (block upper-bidiagonal, backward in time) and returns

    dL/da0 = (M_A / dt) lam_A^1,     dL/df = lam_u.

Checkpointing: the forward pass keeps no space-time vector, only the host-side
linearisation state needed to rebuild the operator.  With ``checkpoint=True``
(or ``"auto"`` when the workspace would exceed half of the free device memory)
the device system is released after the forward solve and rebuilt from that
state for the backward solve: setup time traded for memory.
"""
from __future__ import annotations

import torch

from . import binding


class SpaceTimeProblem:
    """A linearised space-time system whose operator can be dropped and rebuilt."""

    def __init__(self, n, nt, dt, mu, eta, mu0, ubar, abar, b_fixed=None, precision="fp64", rtol=1e-12,
                 checkpoint="auto", device="cuda:0", **plan_kw):
        self.args = (n, nt, dt, mu, eta, mu0, ubar, abar)
        self.plan_kw = dict(plan_kw, precision=precision, adjoint=True)
        self.device = torch.device(device)
        self.rtol = rtol
        self.checkpoint = checkpoint
        self._sys = None
        self.rebuilds = 0
        sysg = self.system()
        self.N, self.ns, self.nt = sysg.N, sysg.ns, nt
        self.offsets = sysg.offsets
        self.b_fixed = (torch.zeros(self.N, dtype=torch.float64, device=self.device) if b_fixed is None
                        else b_fixed.to(self.device, torch.float64).contiguous())

    def system(self):
        if self._sys is None:
            plan = binding.Plan(*self.args, **self.plan_kw)
            self._sys = binding.System(plan, self.device)
            self._ws_bytes = plan.workspace_bytes
            plan.close()
            self.rebuilds += 1
        return self._sys

    def release(self):
        """Drop the device system (its workspace returns to the torch allocator)."""
        if self._sys is not None:
            self._sys.close()
            self._sys = None

    def should_release(self):
        if self.checkpoint is True:
            return True
        if self.checkpoint == "auto":
            free, _ = torch.cuda.mem_get_info(self.device)
            return self._ws_bytes > 0.5 * free
        return False

    def rhs(self, a0, f):
        o = self.offsets
        b = self.b_fixed.clone().view(self.nt, self.ns)
        b[0, o[4]:o[5]] += self.system().initial_coupling(a0.contiguous())
        b[:, o[0]:o[2]] += f.view(self.nt, o[2] - o[0])
        return b.view(-1)


class _TerminalPotential(torch.autograd.Function):
    @staticmethod
    def forward(ctx, problem, a0, f):
        b = problem.rhs(a0.detach().to(torch.float64), f.detach().to(torch.float64))
        x, info, rc, _ = problem.system().solve(b, rtol=problem.rtol)
        if rc != 0:
            raise RuntimeError(f"forward solve did not converge (residual {info.true_rel_residual:.2e})")
        o = problem.offsets
        out = x.view(problem.nt, problem.ns)[-1, o[4]:o[5]].clone()
        del x
        ctx.problem = problem
        if problem.should_release():
            problem.release()
        return out

    @staticmethod
    def backward(ctx, grad):
        problem = ctx.problem
        sysg = problem.system()
        o = problem.offsets
        g = torch.zeros(problem.N, dtype=torch.float64, device=problem.device)
        g.view(problem.nt, problem.ns)[-1, o[4]:o[5]] = grad.to(torch.float64)
        lam, info, rc, _ = sysg.solve(g, rtol=problem.rtol, adjoint=True)
        if rc != 0:
            raise RuntimeError(f"adjoint solve did not converge (residual {info.true_rel_residual:.2e})")
        L = lam.view(problem.nt, problem.ns)
        grad_a0 = sysg.initial_coupling(L[0, o[4]:o[5]].contiguous())
        grad_f = L[:, o[0]:o[2]].contiguous().view(-1)
        return None, grad_a0, grad_f


def terminal_potential(problem: SpaceTimeProblem, a0: torch.Tensor, f: torch.Tensor) -> torch.Tensor:
    """x_A at the last slab of J^{-1} b(a0, f); differentiable in a0 and f."""
    return _TerminalPotential.apply(problem, a0, f)
