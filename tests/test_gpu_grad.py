"""GPU parity of the score dl/d(sigma^2, beta) (tlr_loglik_grad) against the
oracle's textbook formula (explicit Sigma^{-1}) and against finite
differences of the oracle's dense log-likelihood.

Tolerances:
  * dense: the tangent propagation and the oracle's explicit inverse are two
    exact algorithms; FP64 rounding on matrices of condition <= 1e5 keeps the
    difference below 1e-8 of the score's two terms.
  * TLR: the trace term is propagated through compressed tangent tiles; the
    error is bounded by 100 eps times the magnitude of the score's terms.
"""
import numpy as np
import pytest

from oracle import dense as D

from gpu_util import field, log, to_dev

pytestmark = pytest.mark.gpu


def _handle(n, nb, **kw):
    import paper_1804_09137_amd as P
    return P.Handle(n, nb, want_grad=True, **kw)


@pytest.mark.parametrize("n,nb,th", [(1000, 160, (1.0, 0.1, 0.5)), (700, 128, (0.7, 0.05, 1.0)),
                                     (1600, 320, (1.2, 0.2, 1.5))])
def test_dense_gradient_matches_oracle(n, nb, th):
    x, y, z = field(n, 0, th)
    log(f"dense grad n={n} nb={nb} th={th}")
    ref = D.gradient(x, y, z, th)
    h = _handle(n, nb, mode="dense")
    xd, yd, zd = to_dev(x, y, z)
    ll, (gs, gb) = h.loglik_grad(xd, yd, zd, th)
    scale = 0.5 * (abs(ref["tr_beta"]) + abs(ref["qf_beta"]))
    log(f"  ll {ll} vs {ref['ll']}; dsigma2 {gs} vs {ref['dsigma2']}; dbeta {gb} vs {ref['dbeta']} (scale {scale:.3e})")
    assert abs(ll - ref["ll"]) <= 1e-9 * abs(ref["ll"])
    assert abs(gs - ref["dsigma2"]) <= 1e-8 * max(1.0, abs(ref["dsigma2"]))
    assert abs(gb - ref["dbeta"]) <= 1e-8 * scale


def test_dense_gradient_central_difference():
    n, nb = 900, 128
    th = (1.0, 0.1, 0.5)
    x, y, z = field(n, 3, th)
    h = _handle(n, nb, mode="dense")
    xd, yd, zd = to_dev(x, y, z)
    _, (gs, gb) = h.loglik_grad(xd, yd, zd, th)
    hb = 1e-5 * th[1]
    fd = (D.loglik(x, y, z, (th[0], th[1] + hb, th[2]))["ll"] -
          D.loglik(x, y, z, (th[0], th[1] - hb, th[2]))["ll"]) / (2 * hb)
    hs = 1e-5
    fds = (D.loglik(x, y, z, (th[0] + hs, th[1], th[2]))["ll"] -
           D.loglik(x, y, z, (th[0] - hs, th[1], th[2]))["ll"]) / (2 * hs)
    assert abs(gb - fd) <= 1e-6 * max(1.0, abs(fd))
    assert abs(gs - fds) <= 1e-6 * max(1.0, abs(fds))


# (4321, 800): the column-update kernel's tiles of 256 columns plus the 32
# beyond 768, a ragged last tile (321 rows: update workgroups past M), and the
# tangent columns folded into their compression
@pytest.mark.parametrize("n,nb,th,eps", [(1600, 320, (1.0, 0.1, 0.5), 1e-9), (2000, 256, (1.0, 0.1, 1.0), 1e-7),
                                         (1234, 160, (0.8, 0.05, 1.5), 1e-9), (4321, 800, (1.0, 0.1, 0.5), 1e-7)])
def test_tlr_gradient_matches_oracle(n, nb, th, eps):
    x, y, z = field(n, 1, th)
    ref = D.gradient(x, y, z, th)
    h = _handle(n, nb, tol=eps, maxrank=nb)
    xd, yd, zd = to_dev(x, y, z)
    ll, (gs, gb) = h.loglik_grad(xd, yd, zd, th)
    scale = 0.5 * (abs(ref["tr_beta"]) + abs(ref["qf_beta"]))
    log(f"tlr grad n={n} eps={eps}: ll rel {abs(ll - ref['ll']) / abs(ref['ll']):.2e}; "
        f"dbeta {gb} vs {ref['dbeta']} (rel to scale {abs(gb - ref['dbeta']) / scale:.2e}); "
        f"dsigma2 {gs} vs {ref['dsigma2']}")
    assert abs(ll - ref["ll"]) <= 10 * eps * abs(ref["ll"])
    assert abs(gb - ref["dbeta"]) <= 100 * eps * scale
    assert abs(gs - ref["dsigma2"]) <= 100 * eps * (n / (2 * th[0]))


def test_tlr_loglik_grad_value_equals_potrf_path():
    n, nb, eps = 1500, 256, 1e-8
    th = (1.0, 0.1, 0.5)
    x, y, z = field(n, 0, th)
    h = _handle(n, nb, tol=eps, maxrank=200)
    xd, yd, zd = to_dev(x, y, z)
    ll_g, _ = h.loglik_grad(xd, yd, zd, th)
    h.generate(xd, yd, th)
    h.potrf()
    ll, _, _ = h.loglik(zd)
    # the second factorisation may sketch some tiles wider (its widths come
    # from the first one's ranks), so the two agree to the compression accuracy
    assert abs(ll - ll_g) <= 10 * eps * abs(ll)


def test_tlr_gradient_with_dense_tiles():
    n, nb, eps = 1600, 320, 1e-9
    th = (1.0, 0.1, 0.5)
    x, y, z = field(n, 0, th)
    ref = D.gradient(x, y, z, th)
    h = _handle(n, nb, tol=eps, maxrank=40)
    xd, yd, zd = to_dev(x, y, z)
    ll, (gs, gb) = h.loglik_grad(xd, yd, zd, th)
    scale = 0.5 * (abs(ref["tr_beta"]) + abs(ref["qf_beta"]))
    log(f"grad with {h.info().dense_tiles} dense tiles: dbeta rel {abs(gb - ref['dbeta']) / scale:.2e}")
    assert h.info().dense_tiles > 0
    assert abs(ll - ref["ll"]) <= 10 * eps * abs(ref["ll"])
    assert abs(gb - ref["dbeta"]) <= 100 * eps * scale


def test_tlr_gradient_folded_term_fallbacks(monkeypatch):
    # The primal column's last update term is folded into the compression of
    # the tiles below its diagonal tile.  When the per-tile products of that
    # term do not fit their buffer (forced here by a zero capacity) the term is
    # applied to the tiles instead; tiles that end dense take it before they
    # are copied.  The last tile's points are spread over the whole domain, so
    # its tiles are dense while the columns above stay low rank and fold.  z
    # need not be a sample of the field for the formula to hold.
    n, nb, eps = 1600, 320, 1e-9
    th = (1.0, 0.1, 0.5)
    x, y, z = field(n, 0, th)
    rng = np.random.default_rng(7)
    x, y = x.copy(), y.copy()
    x[-nb:] = rng.uniform(x.min(), x.max(), nb)
    y[-nb:] = rng.uniform(y.min(), y.max(), nb)
    ref = D.gradient(x, y, z, th)
    scale = 0.5 * (abs(ref["tr_beta"]) + abs(ref["qf_beta"]))
    xd, yd, zd = to_dev(x, y, z)
    for cap in (None, "0"):
        if cap is None:
            monkeypatch.delenv("TLR_FOLD_GBUF", raising=False)
        else:
            monkeypatch.setenv("TLR_FOLD_GBUF", cap)
        h = _handle(n, nb, tol=eps, maxrank=160)
        ll, (gs, gb) = h.loglik_grad(xd, yd, zd, th)
        info = h.info()
        log(f"fold cap {cap}: {info.dense_tiles} dense tiles, rank_max {info.rank_max}, "
            f"ll rel {abs(ll - ref['ll']) / abs(ref['ll']):.2e}, dbeta rel {abs(gb - ref['dbeta']) / scale:.2e}")
        assert 0 < info.dense_tiles and info.rank_max > 0   # dense and low-rank tiles in the same columns
        assert abs(ll - ref["ll"]) <= 10 * eps * abs(ref["ll"])
        assert abs(gb - ref["dbeta"]) <= 100 * eps * scale
        assert abs(gs - ref["dsigma2"]) <= 100 * eps * (n / (2 * th[0]))
