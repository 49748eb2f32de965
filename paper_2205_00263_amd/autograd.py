"""torch.autograd interface to the library's hand-written adjoint of back-substitution.

`SetBound.apply(alpha, beta, gamma, problem, sid, set_idx)` evaluates one
parameter set of one subproblem: its rows (the spec rows for set 0, the
lower / upper rows of one ReLU layer otherwise) are back-substituted through
Eq. 2 and the ReLU rule of Eq. 5 and concretised over the input box (Eq. 6).
It returns the set's objective (the sum of its rows' lower bounds, the
quantity the projected gradient ascent of Section 3.1 maximises) and the rows'
lower bounds (not differentiable).  The backward pass is the library's
adjoint: x* pushed forward through every row's linearised network, which
gives d lb / d(alpha, beta, gamma) with the intermediate bounds l, u held
constant, summed over the set's rows.  Both passes run in the HIP library on
device memory (mnb_set_params_device / mnb_bound_grad_device); this module only
hands over tensor pointers.
"""
from __future__ import annotations

import torch

__all__ = ["SetBound", "set_bound", "optimize_set"]


def _dev(t):
    """A contiguous float32 CUDA tensor for t (None stays None)."""
    if t is None or t.numel() == 0:
        return None
    if not t.is_cuda:
        raise ValueError("SetBound needs CUDA tensors (device memory is handed to the library)")
    return t.detach().to(torch.float32).contiguous()


class SetBound(torch.autograd.Function):
    @staticmethod
    def forward(ctx, alpha, beta, gamma, problem, sid, set_idx):
        a, b, g = _dev(alpha), _dev(beta), _dev(gamma)
        # the library runs on its own stream unless torch's was installed: order torch's writes first
        torch.cuda.current_stream(alpha.device).synchronize()
        problem.set_params_device(sid, set_idx, a.data_ptr() if a is not None else 0,
                                  b.data_ptr() if b is not None else 0, g.data_ptr() if g is not None else 0)
        dev = alpha.device
        td = problem.total_d
        cap = problem.S if set_idx == 0 else max(problem.net.relu_sizes)
        lb = torch.empty(cap, dtype=torch.float32, device=dev)
        ga = torch.empty(td, dtype=torch.float32, device=dev)
        gb = torch.empty(td, dtype=torch.float32, device=dev)
        ng = problem.net.n_relu * problem.max_mnc
        gg = torch.empty(max(ng, 1), dtype=torch.float32, device=dev)
        rows = problem.bound_grad_device(sid, set_idx, lb.data_ptr(), ga.data_ptr(), gb.data_ptr(),
                                         gg.data_ptr() if ng else 0)
        lbt = lb[:rows]
        ctx.save_for_backward(ga, gb, gg[:ng])
        ctx.gamma_shape = gamma.shape
        obj = lbt.double().sum().float()
        ctx.mark_non_differentiable(lbt)
        return obj, lbt

    @staticmethod
    def backward(ctx, g_obj, g_lb):
        ga, gb, gg = ctx.saved_tensors
        g_gamma = (gg * g_obj).reshape(ctx.gamma_shape) if gg.numel() else torch.zeros(ctx.gamma_shape,
                                                                                      device=ga.device)
        return ga * g_obj, gb * g_obj, g_gamma, None, None, None


def set_bound(problem, sid, set_idx, alpha, beta, gamma=None):
    """(objective, row lower bounds) of one parameter set at the given parameters."""
    if gamma is None:
        gamma = torch.zeros(0, device=alpha.device)
    return SetBound.apply(alpha, beta, gamma, problem, sid, set_idx)


def optimize_set(problem, sid, set_idx, steps=20, lr=0.1, device="cuda"):
    """Projected Adam ascent (PyTorch's optimiser, the library's adjoint) on one set.

    Starts from the subproblem's stored parameters; keeps the best lower bound
    per row over the steps + 1 evaluations and writes the final parameters back.
    Returns the best row bounds (a CUDA tensor)."""
    a0, b0, g0 = problem.get_params(sid, set_idx)
    alpha = torch.tensor(a0, device=device, requires_grad=True)
    beta = torch.tensor(b0, device=device, requires_grad=True)
    gamma = torch.tensor(g0, device=device, requires_grad=True)
    opt = torch.optim.Adam([alpha, beta, gamma], lr=lr, maximize=True)
    best = None
    for t in range(steps + 1):
        obj, lb = set_bound(problem, sid, set_idx, alpha, beta, gamma)
        best = lb.clone() if best is None else torch.maximum(best, lb)
        if t == steps:
            break
        opt.zero_grad()
        obj.backward()
        opt.step()
        with torch.no_grad():
            alpha.clamp_(0.0, 1.0)
            beta.clamp_(min=0.0)
            gamma.clamp_(min=0.0)
    torch.cuda.current_stream(alpha.device).synchronize()
    g = _dev(gamma)
    problem.set_params_device(sid, set_idx, _dev(alpha).data_ptr(), _dev(beta).data_ptr(),
                              g.data_ptr() if g is not None else 0)
    return best
