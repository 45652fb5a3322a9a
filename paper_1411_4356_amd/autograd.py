"""Steady-state observables as a differentiable function of the model
parameters, with the adjoint method as the backward pass.

forward:  theta = (Delta, g0, E, kappa, Gamma_m) -> (<a^dag a>, <b^dag b>, F)
          by the method of Sec. II-IV (assembly, RCM, ILUT, right-preconditioned
          GMRES on the trace-constrained system);
backward: for each objective f = Re o_f^T x, solve A^H lambda_f = conj(o_f)
          with the same factors (their conjugate transposes), and
          df/dtheta = -Re lambda_f^H P0 (dL/dtheta) x, P0 removing the trace row
          (its derivative is irrelevant because Tr x = 1 holds for every theta).

Every solve and contraction runs in libomss; this module only chains the
calls and applies the vector-Jacobian product of the 3 x 5 Jacobian.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import api

THETA_NAMES = ("delta", "g0", "E", "kappa", "gamma_m")


@dataclass
class SolveConfig:
    """Fixed (non-differentiable) part of the problem and the solver knobs."""
    nc: int
    nm: int
    omega_m: float = 1.0
    n_th: float = 0.0
    drop_tol: float = 1e-6
    fill_factor: float = 60.0
    m: int = 50
    tol: float = 1e-12
    maxiter: int = 1000
    nth0_fix: bool = True


def _solve(theta: np.ndarray, cfg: SolveConfig):
    n_th = cfg.n_th
    if cfg.nth0_fix and n_th == 0.0:
        n_th = 1e-15   # Sec. V: keeps the incomplete factorisation stable, same rho to 1e-12
    p = dict(nc=cfg.nc, nm=cfg.nm, omega_m=cfg.omega_m, n_th=n_th,
             **{k: float(v) for k, v in zip(THETA_NAMES, theta)})
    A, w = api.liouvillian_build(p)
    B, perm, _ = api.rcm_permute(A)
    M = api.ilu_factor(B, cfg.drop_tol, cfg.fill_factor, adjoint=True)
    # right-hand side w e_0 of the constrained system, in the RCM ordering
    pos0 = int(np.flatnonzero(perm == 0)[0])
    b = torch.zeros((1, B.n), dtype=torch.complex128, device="cuda")
    b[0, pos0] = complex(w[0])
    x, info = api.gmres_solve(B, M, b, m=cfg.m, tol=cfg.tol, maxiter=cfg.maxiter)
    return B, M, x, info


class SteadyStateObs(torch.autograd.Function):
    """SteadyStateObs.apply(theta, cfg) -> float64[3] = (<a^dag a>, <b^dag b>, F).

    theta: float64 tensor [5] = (Delta, g0, E, kappa, Gamma_m) (any device);
    cfg: SolveConfig.  The backward pass costs three adjoint GMRES solves that
    reuse the forward factorisation."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, cfg: SolveConfig):
        th = theta.detach().to("cpu", torch.float64).numpy()
        B, M, x, info = _solve(th, cfg)
        obs = api.observables(B, x)[0]
        ctx.state = (B, M, x, cfg)
        ctx.info = info
        return torch.tensor(obs, dtype=torch.float64, device=theta.device)

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        B, M, x, cfg = ctx.state
        g = api.objective_vectors(B, x)                      # [3, 1, n]
        lam = torch.empty_like(g)
        for f in range(3):
            lam[f], _ = api.gmres_solve(B, M, g[f].contiguous(), adjoint=True, m=cfg.m, tol=cfg.tol,
                                        maxiter=cfg.maxiter)
        jac = api.param_gradient(B, x, lam)[0]             # [3, 5]: d obs_f / d theta_t
        go = grad_out.detach().to("cpu", torch.float64).numpy()
        vjp = go @ jac
        return torch.tensor(vjp, dtype=torch.float64, device=grad_out.device), None
