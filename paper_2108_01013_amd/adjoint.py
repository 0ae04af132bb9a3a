"""Stress objective of a simulated run as a differentiable torch function.

StressObjective.apply(x0, u0, w0, mu, F_ER, radius, params, n_steps, stress_every, ckpt_every,
weight) runs n_steps time steps of the HIP library from the initial state (x0, u0, w0) with
an empty contact history, and returns J = sum_ab weight_ab mean_samples(Sigma_ab).  Its
backward pass is the library's discrete adjoint (dss_adjoint): gradients with respect to
x0, u0, w0 (by particle id), mu and F_ER, with the run's pair set, contact states and
Coulomb-cap states held fixed.  Tensors may live on the host or on the GPU (float64); the
forward pass computes the gradients together with J when any input requires them.
"""
from __future__ import annotations

import numpy as np
import torch

from .dss import DSS_FP64, Simulation


class StressObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, u0, w0, mu, fer, radius, params, n_steps, stress_every, ckpt_every, weight,
                precision=DSS_FP64):
        p = dict(params, mu=float(mu), F_ER=float(fer))
        ctx.theta_dev = tuple(t.device if torch.is_tensor(t) else None for t in (mu, fer))
        dev = x0.device
        if dev.type == "cuda":
            # device tensors go to the library as device pointers, on torch's current stream
            sim = Simulation(p, precision=precision, stream=torch.cuda.current_stream(dev).cuda_stream)
            inputs = tuple(t.detach().to(dev, torch.float64).contiguous() for t in (x0, radius, u0, w0))
        else:
            sim = Simulation(p, precision=precision)
            inputs = tuple(t.detach().to("cpu", torch.float64).contiguous().numpy() for t in (x0, radius, u0, w0))
        try:
            sim.set_particles(*inputs)
            wt = np.asarray(weight, np.float64).reshape(3, 3)
            if any(ctx.needs_input_grad[:5]):
                if dev.type == "cuda":
                    gx = torch.empty_like(x0, dtype=torch.float64).contiguous()
                    gu = torch.empty_like(gx)
                    gw = torch.empty_like(gx)
                    torch.cuda.synchronize(dev)
                    J, dmu, dfer = sim.adjoint_into(n_steps, stress_every, ckpt_every, wt, gx, gu, gw)
                else:
                    r = sim.adjoint(n_steps, stress_every, ckpt_every, wt)
                    J, dmu, dfer = r["J"], r["dmu"], r["dF_ER"]
                    gx, gu, gw = (torch.from_numpy(r[k]) for k in ("dx", "du", "dw"))
                ctx.save_for_backward(gx, gu, gw)
                ctx.dtheta = (dmu, dfer)
            else:
                sim.step(n_steps, stress_every=stress_every)
                _, mean, _ = sim.read_stress()
                J = float(np.sum(wt * mean))
        finally:
            sim.close()
        return torch.tensor(J, dtype=torch.float64, device=x0.device)

    @staticmethod
    def backward(ctx, gJ):
        gx, gu, gw = ctx.saved_tensors
        dmu, dfer = ctx.dtheta
        g = gJ.to(gx.device)
        th = []
        for val, dev in zip((dmu, dfer), ctx.theta_dev):
            th.append(None if dev is None else gJ.to(dev) * torch.tensor(val, dtype=torch.float64, device=dev))
        return g * gx, g * gu, g * gw, th[0], th[1], None, None, None, None, None, None, None


def stress_objective(x0, u0, w0, mu, fer, radius, params, n_steps, stress_every, ckpt_every=20, weight=None,
                     precision=DSS_FP64):
    """Functional form of StressObjective (weight defaults to the shear stress Sigma_xy)."""
    if weight is None:
        weight = np.zeros((3, 3))
        weight[0, 1] = 1.0
    return StressObjective.apply(x0, u0, w0, mu, fer, radius, params, n_steps, stress_every, ckpt_every, weight,
                                 precision)
