"""Reverse-mode differentiation of several SDC steps as a torch.autograd.Function.

Forward: n steps of the library from (v0, w0) at the given coefficients,
keeping the step-start state every `ckpt_every` steps.  Backward: for each
checkpoint segment, last first, the segment's steps are recomputed once from
the checkpoint with every sweep recorded (sdc_adjoint_record, one recording
slot per step), then reversed step by step, last first (sdc_adjoint_reverse,
active sets held fixed).
All arithmetic runs in the HIP library; this module only sequences calls.
"""
import numpy as np
import torch


class SDCRun(torch.autograd.Function):
    """v_T, w_T = SDCRun.apply(sigma, a, v0, w0, solver, n_steps, t0, ckpt_every)

    sigma: [N] nodal conductivity multipliers, a: [n_inst] Aliev-Panfilov
    parameter a (both float64; the solver is reassembled with them), v0, w0:
    [N] initial state on the solver's device.  Gradients flow to sigma, a,
    v0 and w0.
    """

    @staticmethod
    def forward(ctx, sigma, a, v0, w0, solver, n_steps, t0, ckpt_every):
        if not 1 <= ckpt_every <= solver.max_recordings:
            raise ValueError(f"ckpt_every must be in 1..{solver.max_recordings}")
        sig = sigma.detach().cpu().numpy()
        ionic = solver.ionic.copy()
        ionic[:, 1] = a.detach().cpu().numpy()
        # reassemble only when the coefficients differ from the solver's
        solver.set_coefficients(None if np.array_equal(sig, solver.node_sigma) else sig,
                                None if np.array_equal(ionic, solver.ionic) else ionic)
        v = v0.detach().clone()
        w = w0.detach().clone()
        ckpts = []
        for n in range(n_steps):
            if n % ckpt_every == 0:
                ckpts.append((n, v.clone(), w.clone()))
            solver.step(v, w, t0 + n * solver.dt)
        ctx.solver, ctx.n_steps, ctx.t0, ctx.ckpt_every, ctx.ckpts = solver, n_steps, t0, ckpt_every, ckpts
        ctx.sigma_shape, ctx.a_shape = sigma.shape, a.shape
        return v, w

    @staticmethod
    def backward(ctx, gv, gw):
        s = ctx.solver
        dev = s.device
        lam_v = (gv if gv is not None else torch.zeros(s.N, dtype=torch.float64, device=dev)).detach().clone()
        lam_w = (gw if gw is not None else torch.zeros(s.N, dtype=torch.float64, device=dev)).detach().clone()
        g_sigma = torch.zeros(s.N, dtype=torch.float64, device=dev)
        g_a = torch.zeros(s.n_inst, dtype=torch.float64, device=dev)
        bounds = [c[0] for c in ctx.ckpts] + [ctx.n_steps]
        for q in range(len(ctx.ckpts) - 1, -1, -1):
            n0, v, w = ctx.ckpts[q]
            n1 = bounds[q + 1]
            v, w = v.clone(), w.clone()
            for n in range(n0, n1):
                s.adjoint_record(n - n0, v, w, ctx.t0 + n * s.dt)
            for n in range(n1 - 1, n0 - 1, -1):
                s.adjoint_reverse(n - n0, lam_v, lam_w, g_sigma, g_a)
        return g_sigma.to(dev), g_a.reshape(ctx.a_shape), lam_v, lam_w, None, None, None, None
