"""Maximum-likelihood fit through the library (the workflow the score is for):
L-BFGS on the GPU likelihood + score reaches the same optimum as the same
optimiser run on the CPU oracle's dense likelihood and gradient, and the
autograd wrapper returns the library's score."""
import numpy as np
import pytest

from oracle import dense as D

from gpu_util import field, log, to_dev

pytestmark = pytest.mark.gpu


def _oracle_fit(x, y, z, th0, nu):
    from scipy.optimize import minimize

    def f(phi):
        th = np.exp(phi)
        r = D.gradient(x, y, z, (th[0], th[1], nu))
        return -r["ll"], -np.array([r["dsigma2"] * th[0], r["dbeta"] * th[1]])
    res = minimize(f, np.log(th0), jac=True, method="L-BFGS-B", options={"ftol": 1e-15, "gtol": 1e-9})
    return np.exp(res.x)


@pytest.mark.parametrize("mode", ["dense", "tlr"])
def test_lbfgs_matches_oracle_optimum(mode):
    import paper_1804_09137_amd as P
    from paper_1804_09137_amd.autograd import fit
    n, nb, nu = 900, 128, 0.5
    x, y, z = field(n, 5, (1.0, 0.1, nu))
    ref = _oracle_fit(x, y, z, (0.5, 0.05), nu)
    h = P.Handle(n, nb, mode=mode, tol=1e-10, maxrank=nb, want_grad=True)
    xd, yd, zd = to_dev(x, y, z)
    r = fit(h, xd, yd, zd, (0.5, 0.05), nu, tol=1e-9)
    log(f"{mode}: theta {r['theta']} vs oracle {tuple(ref)}; {r['evals']} evals; score {r['grad']}")
    assert r["converged"]
    np.testing.assert_allclose(r["theta"], ref, rtol=1e-5)


def test_nelder_mead_agrees_with_lbfgs():
    import paper_1804_09137_amd as P
    from paper_1804_09137_amd.autograd import fit
    n, nb, nu = 700, 128, 0.5
    x, y, z = field(n, 6, (1.0, 0.1, nu))
    h = P.Handle(n, nb, mode="dense", want_grad=True)
    xd, yd, zd = to_dev(x, y, z)
    a = fit(h, xd, yd, zd, (0.5, 0.05), nu, tol=1e-9)
    b = fit(h, xd, yd, zd, (0.5, 0.05), nu, method="Nelder-Mead", tol=1e-9)
    log(f"L-BFGS {a['theta']} in {a['evals']} evals; Nelder-Mead {b['theta']} in {b['evals']} evals")
    np.testing.assert_allclose(a["theta"], b["theta"], rtol=1e-4)
    assert a["evals"] < b["evals"]


def test_autograd_wrapper_returns_library_score():
    import torch
    import paper_1804_09137_amd as P
    n, nb, nu = 600, 128, 1.0
    x, y, z = field(n, 7, (1.0, 0.1, nu))
    h = P.Handle(n, nb, mode="dense", want_grad=True)
    xd, yd, zd = to_dev(x, y, z)
    th = torch.tensor([0.8, 0.07], dtype=torch.float64, requires_grad=True)
    ll = P.TLRLogLik.apply(th, h, xd, yd, zd, nu)
    (2.0 * ll).backward()
    ll2, (gs, gb) = h.loglik_grad(xd, yd, zd, (0.8, 0.07, nu))
    assert float(ll) == ll2
    np.testing.assert_array_equal(th.grad.numpy(), 2.0 * np.array([gs, gb]))
