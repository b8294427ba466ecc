"""kappa_eff as a differentiable function of the relaxation times of the frequency bins.

The gradient comes from the sensitivity replay; the default estimator is the local pathwise form
(each flight's own flux differentiated through its length, what follows it by its likelihood ratio),
"score" and "pathwise" are the alternatives (see mcbte_adjoint in include/mcbte.h).

The forward pass traces the problem with the rows of bin i given relaxation time tau[i] (the
relaxation time depends on the frequency only, so the rows of the branches that share a bin share
it) and returns kappa_eff; it also runs the sensitivity replay of the same particles, and the
backward pass returns grad_out * dkappa/dtau_i = grad_out * (dkappa/dln tau_i) / tau_i.  Both
numbers are Monte Carlo estimates from one set of particles: the gradient is an unbiased estimate
of the gradient of the expected kappa, not the derivative of the returned sample.
"""
from __future__ import annotations

import copy

import numpy as np
import torch

from .mcbte import sensitivities


def tau_bins(w: dict) -> np.ndarray:
    """Per-bin relaxation times of a workload (every row of a bin must carry the same tau)."""
    m = w["modes"]
    nb = int(m["bin"].max()) + 1
    out = np.zeros(nb)
    seen = np.zeros(nb, dtype=bool)
    for b, t in zip(m["bin"], m["tau"]):
        if seen[b] and out[b] != t:
            raise ValueError(f"bin {b} holds rows with different relaxation times")
        out[b], seen[b] = t, True
    return out


def with_tau_bins(w: dict, tau) -> dict:
    """Copy of workload w whose rows take tau[bin] as relaxation time."""
    tau = np.asarray(tau, dtype=np.float64)
    w2 = copy.deepcopy(w)
    m = w2["modes"]
    if tau.shape != (int(m["bin"].max()) + 1,):
        raise ValueError("tau must hold one value per frequency bin")
    m["tau"] = tau[m["bin"]]
    return w2


class KappaOfTau(torch.autograd.Function):
    """kappa = KappaOfTau.apply(tau, w, n, precision, estimator, device): tau is a 1-D float64
    tensor of per-bin relaxation times (any device); the result is a 0-d float64 tensor on
    tau's device."""

    @staticmethod
    def forward(ctx, tau, w, n=None, precision=32, estimator="local", device=0):
        t = tau.detach().to("cpu", torch.float64).numpy()
        out = sensitivities(with_tau_bins(w, t), n, precision=precision, device=device, estimator=estimator)
        grad = np.where(t > 0.0, out["dkappa_dlntau"] / np.where(t > 0.0, t, 1.0), 0.0)
        ctx.save_for_backward(torch.from_numpy(grad).to(tau.device))
        ctx.kappa_sigma = out.get("kappa_sigma")
        return torch.tensor(out["kappa"], dtype=torch.float64, device=tau.device)

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return g * grad, None, None, None, None, None


def kappa_of_tau(tau: torch.Tensor, w: dict, n: int | None = None, precision: int = 32,
                 estimator: str = "local", device: int = 0) -> torch.Tensor:
    return KappaOfTau.apply(tau, w, n, precision, estimator, device)
