"""Repeated evaluations on one handle: the sketch widths of an evaluation come
from the previous one's ranks.  The result must stay within the compression
accuracy of the oracle whatever the history (same theta, a nearby theta, and
a far one whose ranks differ)."""
import pytest

from oracle import dense as D

from gpu_util import field, log, to_dev

pytestmark = pytest.mark.gpu


def test_rank_history_keeps_accuracy():
    import paper_1804_09137_amd as P
    n, nb, eps = 2500, 256, 1e-8
    x, y, z = field(n, 2, (1.0, 0.1, 0.5))
    h = P.Handle(n, nb, tol=eps, maxrank=200, want_grad=True)
    xd, yd, zd = to_dev(x, y, z)
    for th in [(1.0, 0.1, 0.5), (1.0, 0.1, 0.5), (1.02, 0.105, 0.5), (0.7, 0.03, 0.5), (1.0, 0.3, 0.5)]:
        ref = D.loglik(x, y, z, th)["ll"]
        ll, _ = h.loglik_grad(xd, yd, zd, th)
        log(f"theta {th}: rel {abs(ll - ref) / abs(ref):.2e} max rank {h.ranks().max()}")
        assert abs(ll - ref) <= 10 * eps * abs(ref)
