"""The autotuner on the GPU: it times every candidate through the library and
returns the fastest, and that configuration meets the oracle."""
import pytest

from oracle import dense as D

from gpu_util import field, log, to_dev

pytestmark = pytest.mark.gpu


def test_tune_picks_fastest_valid_configuration():
    import paper_1804_09137_amd as P
    from paper_1804_09137_amd.tune import tune
    n, eps = 6400, 1e-8
    th = (1.0, 0.1, 0.5)
    x, y, z = field(n, 0, th)
    xd, yd, zd = to_dev(x, y, z)
    r = tune(xd, yd, zd, th, eps, cands=[(400, 100), (800, 200), (640, 160)], reps=1, log=log)
    assert (r["nb"], r["maxrank"]) == min(r["ms"], key=r["ms"].get)
    h = P.Handle(n, r["nb"], tol=eps, maxrank=r["maxrank"], want_grad=True)
    ll, _ = h.loglik_grad(xd, yd, zd, th)
    ref = D.loglik(x, y, z, th)["ll"]
    assert abs(ll - ref) <= 10 * eps * abs(ref)
