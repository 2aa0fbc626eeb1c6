"""bench.py's extrapolation of the CPU oracle's time to the full problem size.

With n2 = 2 n1 the two-term fit t(n) = a n^2 + b n^3 has a >= 0 and b > 0 exactly
when 4 < t2 / t1 <= 8; outside that range the power-law fallback applies, its
exponent clamped to 2 (ratio below 4) or 3 (ratio above 8)."""
import math
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from bench import fit_cpu_time  # noqa: E402

N1, N2, NT = 3000, 6000, 102400


@pytest.mark.parametrize("a,b", [(1e-9, 2e-13), (0.0, 5e-12), (4e-8, 1e-15)])
def test_two_term_law_is_recovered(a, b):
    meds = {N2: a * N2 ** 2 + b * N2 ** 3, N1: a * N1 ** 2 + b * N1 ** 3}
    t, law, fa, fb = fit_cpu_time(meds, NT)
    assert fa == pytest.approx(a, rel=1e-9, abs=1e-20)
    assert fb == pytest.approx(b, rel=1e-9)
    assert t == pytest.approx(a * NT ** 2 + b * NT ** 3, rel=1e-9)
    assert "n^2" in law and "n^3" in law


@pytest.mark.parametrize("ratio", [4.5, 6.0, 8.0])
def test_two_term_extrapolation_lies_between_the_pure_laws(ratio):
    t1 = 2.0
    t, _, fa, fb = fit_cpu_time({N1: t1, N2: ratio * t1}, NT)
    assert fa is not None and fb is not None and fa >= 0.0 and fb > 0.0
    t2 = ratio * t1
    assert t2 * (NT / N2) ** 2 <= t * (1 + 1e-12)
    assert t <= t2 * (NT / N2) ** 3 * (1 + 1e-12)


@pytest.mark.parametrize("ratio,power", [(3.0, 2.0), (1.0, 2.0), (0.9, 2.0), (9.0, 3.0), (20.0, 3.0)])
def test_noisy_medians_fall_back_to_a_clamped_power_law(ratio, power):
    t1 = 1.5
    t2 = ratio * t1
    t, law, fa, fb = fit_cpu_time({N1: t1, N2: t2}, NT)
    assert fa is None and fb is None
    assert t == pytest.approx(t2 * (NT / N2) ** power, rel=1e-12)
    assert f"^{power:.3f}" in law


@pytest.mark.parametrize("n1,n2", [(3000, 6000), (2000, 6000), (5000, 7000)])
def test_extrapolation_is_continuous_across_the_regimes(n1, n2):
    # b > 0 exactly when the measured exponent log(t2/t1)/log(n2/n1) exceeds 2,
    # and a >= 0 exactly when it is at most 3, so the fallback only ever runs
    # with the exponent clamped to a bound, and meets the two-term law there.
    r = n2 / n1
    for p in (2.0, 3.0):
        lo = fit_cpu_time({n1: 1.0, n2: r ** p * (1 - 1e-9)}, NT)
        hi = fit_cpu_time({n1: 1.0, n2: r ** p * (1 + 1e-9)}, NT)
        assert (lo[2] is None) == (p == 2.0) and (hi[2] is None) == (p == 3.0)
        assert lo[0] == pytest.approx(hi[0], rel=1e-6)
        assert lo[0] == pytest.approx(r ** p * (NT / n2) ** p, rel=1e-6)


def test_key_order_does_not_matter():
    m = {N1: 1.0, N2: 6.0}
    r = {N2: 6.0, N1: 1.0}
    assert fit_cpu_time(m, NT) == fit_cpu_time(r, NT)
    assert math.isfinite(fit_cpu_time(m, NT)[0])
