"""tlr_loglik_grad_batched: several independent fields (different sizes,
theta and smoothness) evaluated concurrently give what one-at-a-time calls
give on fresh handles (the same computation, bit for bit), each within the
compression accuracy of the oracle; a failing field reports its own error
and leaves the other handles usable."""
import numpy as np
import pytest

import synth
from oracle import dense as D
from oracle import ordering as O

from gpu_util import log, to_dev

pytestmark = pytest.mark.gpu

FIELDS = [(900, 128, (1.0, 0.1, 0.5)), (1500, 160, (0.6, 0.05, 1.5)), (2100, 256, (1.7, 0.2, 0.5)),
          (1200, 128, (1.2, 0.03, 1.5)), (1800, 192, (0.8, 0.3, 0.5)), (640, 64, (2.0, 0.12, 1.5))]
EPS = 1e-8


def _field(n, seed, th):
    x, y = synth.jittered_subset(n, seed)
    p = O.morton_order(x, y)
    x, y = x[p], y[p]
    z = D.sample_z(x, y, th, synth.standard_normal(n, seed + 1))
    return x, y, z


def _handles(streams=True, single_stream=False):
    import torch
    import paper_1804_09137_amd as P
    return [P.Handle(n, nb, tol=EPS, maxrank=nb, want_grad=True, stream=torch.cuda.Stream() if streams else None,
                     single_stream=single_stream)
            for n, nb, _ in FIELDS]


@pytest.mark.parametrize("single_stream", [False, True])
def test_batched_equals_sequential_and_oracle(single_stream):
    import torch
    import paper_1804_09137_amd as P
    data = [_field(n, 10 + f, th) for f, (n, nb, th) in enumerate(FIELDS)]
    dev = [to_dev(*d) for d in data]
    thetas = [th for _, _, th in FIELDS]
    torch.cuda.synchronize()
    ll_b, g_b = P.loglik_grad_batched(_handles(single_stream=single_stream), [d[0] for d in dev],
                                      [d[1] for d in dev], [d[2] for d in dev], thetas, nthreads=4)
    for f, ((n, nb, th), (x, y, z), (xd, yd, zd)) in enumerate(zip(FIELDS, data, dev)):
        h = P.Handle(n, nb, tol=EPS, maxrank=nb, want_grad=True, single_stream=single_stream)
        ll, g = h.loglik_grad(xd, yd, zd, th)
        assert ll == ll_b[f] and g[0] == g_b[f, 0] and g[1] == g_b[f, 1], f
        ref = D.gradient(x, y, z, th)
        scale = 0.5 * (abs(ref["tr_beta"]) + abs(ref["qf_beta"]))
        log(f"field {f} n={n}: ll rel {abs(ll - ref['ll']) / abs(ref['ll']):.2e}, "
            f"dbeta rel {abs(g[1] - ref['dbeta']) / scale:.2e}")
        assert abs(ll - ref["ll"]) <= 10 * EPS * abs(ref["ll"])
        assert abs(g[1] - ref["dbeta"]) <= 100 * EPS * scale


def test_batched_reports_the_failing_field():
    import torch
    import paper_1804_09137_amd as P
    data = [_field(n, 20 + f, th) for f, (n, nb, th) in enumerate(FIELDS[:3])]
    dev = [to_dev(*d) for d in data]
    xs, ys, zs = ([d[k] for d in dev] for k in range(3))
    hs = _handles()[:3]
    torch.cuda.synchronize()
    # sigma^2 < 0 is a valid parameter whose Sigma = sigma^2 C is negative
    # definite: field 1 fails at its first pivot
    thetas = [th for _, _, th in FIELDS[:3]]
    thetas[1] = (-1.0, 0.1, 0.5)
    with pytest.raises(P.NotSPDError) as e:
        P.loglik_grad_batched(hs, xs, ys, zs, thetas)
    assert "field 1" in str(e.value) and e.value.info == 1
    # beta = 0 is rejected by field 2's parameter check
    thetas = [th for _, _, th in FIELDS[:3]]
    thetas[2] = (1.0, 0.0, 0.5)
    with pytest.raises(P.TLRError) as e:
        P.loglik_grad_batched(hs, xs, ys, zs, thetas)
    assert "field 2" in str(e.value) and e.value.status == -1
    # the handles stay usable
    ll, g = P.loglik_grad_batched(hs, xs, ys, zs, [th for _, _, th in FIELDS[:3]])
    assert np.all(np.isfinite(ll)) and np.all(np.isfinite(g))


def test_batched_rejects_a_repeated_handle():
    import paper_1804_09137_amd as P
    hs = _handles()[:2]
    d = to_dev(*_field(FIELDS[0][0], 1, FIELDS[0][2]))
    with pytest.raises(P.TLRError):
        P.loglik_grad_batched([hs[0], hs[0]], [d[0]] * 2, [d[1]] * 2, [d[2]] * 2, [FIELDS[0][2]] * 2)


def test_single_stream_handle_matches_the_default_one():
    # TLR_FLAG_SINGLE_STREAM: the same factorisation issued on one stream (no
    # look-ahead, the update of a column in one pass): equal up to the
    # summation order of the split updates and what it does to the ranks
    import paper_1804_09137_amd as P
    n, nb, eps = 4000, 400, 1e-7
    th = (1.0, 0.1, 0.5)
    x, y, z = _field(n, 5, th)
    xd, yd, zd = to_dev(x, y, z)
    out = []
    for single in (False, True):
        h = P.Handle(n, nb, tol=eps, maxrank=nb // 2, want_grad=True, single_stream=single)
        out.append(h.loglik_grad(xd, yd, zd, th))
        log(f"single_stream={single}: ll {out[-1][0]!r} grad {out[-1][1]}")
    # each is within about 3e-9 (l) and 6e-7 (score) of the exact values at
    # this eps; rounding may move a rank decision at the threshold
    assert abs(out[0][0] - out[1][0]) <= 1e-8 * abs(out[0][0])
    for i in range(2):
        assert abs(out[0][1][i] - out[1][1][i]) <= 5e-6 * abs(out[0][1][i])
