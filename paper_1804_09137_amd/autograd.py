"""torch.autograd wrapper and a host-side maximum-likelihood driver.

Both only drive the library: every likelihood and score evaluation is one
``tlr_loglik_grad`` call on the GPU.  The optimiser itself is host logic on
two scalars (the paper maximises Eq. (1) over theta, Section III; it uses a
derivative-free NLopt search, Section VI; with the score available, L-BFGS is
the natural choice).
"""
from __future__ import annotations

import math

import torch

from . import Handle


class TLRLogLik(torch.autograd.Function):
    """l(theta) for theta = (sigma^2, beta) at fixed smoothness nu.

    forward(theta, handle, x, y, z, nu) -> 0-d float64 tensor l; backward
    returns g * dl/d(sigma^2, beta) from the same library call (the TLR
    approximation of the exact score).
    """

    @staticmethod
    def forward(ctx, theta, handle: Handle, x, y, z, nu: float):
        th = [float(v) for v in theta.detach().cpu().tolist()]
        ll, (gs, gb) = handle.loglik_grad(x, y, z, (th[0], th[1], float(nu)))
        ctx.save_for_backward(torch.tensor([gs, gb], dtype=torch.float64, device=theta.device))
        return torch.tensor(ll, dtype=torch.float64, device=theta.device)

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return g * grad, None, None, None, None, None


def fit(handle: Handle, x, y, z, theta0, nu: float | None = None, method: str = "L-BFGS-B", tol: float = 1e-6,
        maxiter: int = 200) -> dict:
    """Maximise l over (sigma^2, beta) > 0 from theta0 = (sigma^2, beta) at
    fixed smoothness nu, or over (sigma^2, beta, nu) from a three-entry theta0
    (nu None): the paper estimates all three (Section VIII-D).

    The search runs on log(theta) so that the bounds are implicit; the score
    maps through d l / d log(theta_i) = theta_i * d l / d theta_i.
    method: "L-BFGS-B" (uses the score) or "Nelder-Mead" (values only, the
    derivative-free baseline).  tol: relative change of the parameters at
    convergence.  Returns theta, l, the score at the optimum and the number of
    likelihood evaluations.
    """
    import numpy as np
    from scipy.optimize import minimize

    evals = {"n": 0}
    free_nu = len(theta0) == 3
    if free_nu == (nu is not None):
        raise ValueError("give nu for a two-entry theta0, or a three-entry theta0 without nu")

    def evaluate(th):
        if free_nu:
            return handle.loglik_grad3(x, y, z, tuple(float(t) for t in th))
        return handle.loglik_grad(x, y, z, (float(th[0]), float(th[1]), float(nu)))

    def negll(phi):
        th = np.exp(phi)
        ll, g = evaluate(th)
        evals["n"] += 1
        if not math.isfinite(ll):
            return 1e300, np.zeros(len(phi))
        return -ll, -np.array(g) * th

    phi0 = np.log(np.asarray(theta0, dtype=np.float64))
    if method == "L-BFGS-B":
        res = minimize(negll, phi0, jac=True, method="L-BFGS-B",
                       options={"maxiter": maxiter, "ftol": 1e-15, "gtol": tol})
    elif method == "Nelder-Mead":
        res = minimize(lambda p: negll(p)[0], phi0, method="Nelder-Mead",
                       options={"maxiter": 20 * maxiter, "xatol": tol, "fatol": 1e-10})
    else:
        raise ValueError(f"unknown method {method!r}")
    th = np.exp(res.x)
    ll, g = evaluate(th)
    return {"theta": tuple(float(t) for t in th), "ll": ll, "grad": g, "evals": evals["n"] + 1,
            "converged": bool(res.success), "message": str(res.message)}
