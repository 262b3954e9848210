"""Host-side checks of DGRollout's bookkeeping with a stand-in solver on the
CPU (no library calls): the reverse sweep must never write into the gradient
tensor the caller passes in, and the number of reverse steps and their order
must match the forward steps."""

import torch

from paper_2605_26388_amd.rollout import DGRollout


class DoublingSolver:
    """U_{n+1} = 2 U_n per step (stages U1 = U, U2 = U as stand-ins); the
    adjoint of a step is lam_prev = 2 lam, so after n steps the gradient of
    sum(U_n) with respect to U_0 is 2^n."""

    dtype = torch.float64

    def __init__(self, shape):
        self.shape = shape
        self.adjoint_calls = 0

    def empty(self):
        return torch.empty(self.shape, dtype=self.dtype)

    def ssprk3_step(self, U, dt, U1, U2):
        U1.copy_(U)
        U2.copy_(U)
        U.mul_(2.0)
        return U

    def rk_stage(self, U0, Uk, out, a, b, c_dt):
        out.copy_(Uk)
        return out

    def ssprk3_step_adjoint(self, states, dt, lam, lam_prev, acc, mu2, mu1):
        self.adjoint_calls += 1
        lam_prev.copy_(2.0 * lam)
        return lam_prev


def _run(nsteps, checkpoint):
    s = DoublingSolver((1, 5, 2, 8))
    U0 = torch.rand(s.shape, dtype=torch.float64, requires_grad=True)
    UN = DGRollout.apply(U0, s, 0.1, nsteps, checkpoint)
    g = torch.ones_like(UN)
    g_before = g.clone()
    (gU0,) = torch.autograd.grad(UN, U0, grad_outputs=g)
    return s, g, g_before, gU0


def test_backward_leaves_grad_output_untouched():
    for nsteps in (1, 2, 3, 4):
        for cp in ("stages", "steps"):
            s, g, g_before, gU0 = _run(nsteps, cp)
            assert torch.equal(g, g_before), (nsteps, cp)
            assert torch.allclose(gU0, torch.full_like(gU0, 2.0 ** nsteps)), (nsteps, cp)
            assert s.adjoint_calls == nsteps


def test_forward_leaves_input_untouched():
    s = DoublingSolver((1, 5, 2, 8))
    U0 = torch.rand(s.shape, dtype=torch.float64)
    keep = U0.clone()
    UN = DGRollout.apply(U0, s, 0.1, 3, "stages")
    assert torch.equal(U0, keep)
    assert torch.allclose(UN, 8.0 * keep)
