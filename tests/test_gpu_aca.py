"""ACA compression fused with generation (tlr_compress with TLR_FLAG_ACA):
every tile of Sigma within eps of the generated tile in the spectral norm,
ranks near the SVD's (ACA's cross terms overshoot a little), the stored
factors equal to what the tiles' entries say, and the likelihood of the
compressed Sigma (dense Cholesky of the TLR approximation) within 10 eps."""
import numpy as np
import pytest

from oracle import dense as D
from oracle import matern as M

from gpu_util import field, log, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,nb,eps,nu", [(1600, 320, 1e-7, 0.5), (2000, 256, 1e-9, 1.0), (1234, 160, 1e-5, 1.5)])
def test_aca_compress_meets_threshold(n, nb, eps, nu):
    import paper_1804_09137_amd as P
    th = (1.0, 0.1, nu)
    x, y, z = field(n, 0, th)
    h = P.Handle(n, nb, tol=eps, maxrank=nb // 2, aca=True)
    xd, yd = to_dev(x, y)
    h.generate(xd, yd, th)
    h.compress()
    R = h.ranks()
    nt = R.shape[0]
    errs, over = [], []
    S = np.zeros((n, n))
    for i in range(nt):
        si = slice(i * nb, min(n, (i + 1) * nb))
        S[si, si] = M.covariance(x, y, th, si, si)
        for j in range(i):
            sj = slice(j * nb, min(n, (j + 1) * nb))
            A = M.covariance(x, y, th, si, sj)
            T = h.tile(i, j).cpu().numpy()
            errs.append(np.linalg.norm(A - T, 2))
            k_svd = int(np.sum(np.linalg.svd(A, compute_uv=False) > eps))
            over.append(int(R[i, j]) - k_svd)
            S[si, sj] = T
            S[sj, si] = T.T
    log(f"n={n} nb={nb} eps={eps} nu={nu}: max tile error {max(errs):.2e} ({max(errs) / eps:.2f} eps); "
        f"rank excess over SVD min {min(over)} max {max(over)} mean {np.mean(over):.1f}; dense {h.info().dense_tiles}")
    assert max(errs) <= eps
    assert min(over) >= -1
    ref = D.loglik(x, y, z, th)["ll"]
    L = D.cholesky_lower(S)
    w = np.linalg.solve(L, z)
    ll = -0.5 * n * np.log(2 * np.pi) - np.sum(np.log(np.diag(L))) - 0.5 * w @ w
    log(f"  l of the ACA-compressed Sigma {ll:.10g} vs dense {ref:.10g}: rel {abs(ll - ref) / abs(ref):.2e}")
    assert abs(ll - ref) <= 10 * eps * abs(ref)


def test_aca_strict_rank_and_dense_tiles():
    import paper_1804_09137_amd as P
    n, nb, eps = 1500, 256, 1e-10
    th = (1.0, 0.3, 1.5)
    x, y, _ = field(n, 1, th, with_z=False)
    xd, yd = to_dev(x, y)
    h = P.Handle(n, nb, tol=eps, maxrank=16, aca=True)
    h.generate(xd, yd, th)
    h.compress()
    i = h.info()
    log(f"maxrank 16: dense tiles {i.dense_tiles}, rank max {i.rank_max}")
    assert i.dense_tiles > 0 and i.rank_max <= 16
    # a dense tile is the generated tile itself
    R = h.ranks()
    ii, jj = [(a, b) for a in range(R.shape[0]) for b in range(a) if R[a, b] == nb][0]
    T = h.tile(ii, jj).cpu().numpy()
    np.testing.assert_allclose(T, M.covariance(x, y, th, slice(ii * nb, (ii + 1) * nb), slice(jj * nb, (jj + 1) * nb)),
                               rtol=2e-13, atol=0)
    hs = P.Handle(n, nb, tol=eps, maxrank=16, aca=True, strict_rank=True)
    hs.generate(xd, yd, th)
    with pytest.raises(P.RankError):
        hs.compress()
