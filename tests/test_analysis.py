"""The delta_eff(rho) analysis of paper Sec. 5.3 on curves with known answers
(no GPU): exact power laws, the corrections-to-scaling form the paper assumes,
and the densities assembled from recorded counts."""
import numpy as np
import pytest

from paper_1301_6082_amd import analysis as an
from paper_1301_6082_amd import workloads

TIMES = np.asarray(workloads.log_times(10**6), float)


@pytest.mark.parametrize("delta,span", [(0.2, 1), (0.37, 4), (0.5, 9)])
def test_power_law_has_constant_delta_eff(delta, span):
    t, r, d = an.delta_eff(TIMES, 0.7 * TIMES ** -delta, span)
    assert len(d) == len(TIMES) - span
    np.testing.assert_allclose(d, delta, rtol=0, atol=1e-12)
    np.testing.assert_allclose(r, 0.7 * t ** -delta, rtol=1e-12)


def test_corrections_to_scaling_extrapolate_to_delta():
    """rho = c1 t^-delta + c2 t^-2delta: with x = t^-delta, delta_eff =
    delta (c1 + 2 c2 x) / (c1 + c2 x) and rho = c1 x + c2 x^2, so delta_eff is
    a straight line in rho near rho = 0 with intercept delta and slope
    delta c2 / c1^2 (the paper's extrapolation)."""
    delta, c1, c2 = 0.2, 0.5, 0.8
    t = np.exp(np.linspace(np.log(10.0), np.log(1e18), 600))
    rho = c1 * t ** -delta + c2 * t ** (-2 * delta)
    tm, rm, d = an.delta_eff(t, rho)
    x = tm ** -delta
    exact = delta * (c1 + 2 * c2 * x) / (c1 + c2 * x)
    np.testing.assert_allclose(d, exact, rtol=2e-4)
    est, slope = an.extrapolate(rm, d, rho_max=0.02)
    assert abs(est - delta) < 2e-3
    # the slope at rho = 0, from the points closest to it
    est0, slope0 = an.extrapolate(rm, d, rho_max=0.002)
    assert abs(est0 - delta) < 1e-4
    assert abs(slope0 - delta * c2 / c1 ** 2) < 0.05 * delta * c2 / c1 ** 2


def test_extinct_records_are_dropped_and_short_curves_are_empty():
    r = 0.5 * TIMES ** -0.3
    r[-5:] = 0.0
    t, rm, d = an.delta_eff(TIMES, r)
    assert len(d) == len(TIMES) - 6 and np.all(np.abs(d - 0.3) < 1e-12)
    assert len(an.delta_eff([1.0, 2.0], [0.5, 0.0])[2]) == 0
    assert np.isnan(an.extrapolate([0.1], [0.2], 1.0)[0])


def test_curves_from_counts():
    times = [1, 10, 100]
    L, planes, runs = 128, 2, 3
    c = np.zeros((3, runs, planes, 3), dtype=np.uint64)
    c[:, :, :, 0] = np.array([8192, 4096, 1024], dtype=np.uint64)[:, None, None]
    c[:, :, :, 1] = np.array([8192, 1024, 64], dtype=np.uint64)[:, None, None]
    cv = an.curves_from_counts(times, c, L, planes)
    np.testing.assert_allclose(cv.rho, [1.0, 0.5, 0.125])
    np.testing.assert_allclose(cv.rho_pair, [1.0, 0.125, 1 / 128])
    assert cv.runs == runs
    t, r, d = cv.particle()
    np.testing.assert_allclose(d, [np.log(2) / np.log(10), np.log(4) / np.log(10)])


def test_deviation_statistic_is_the_largest_standardized_mean_difference():
    """_deviations: per key, the largest over records of |mean_k - mean_ref| /
    sqrt(var_k / R + var_ref / R) with sample variances over the R runs; the
    reference itself deviates by 0."""
    rng = np.random.default_rng(5)
    R = 8
    ref = rng.normal(1.0, 0.1, size=(3, R))
    other = ref + np.array([[0.0], [0.05], [0.02]])     # shift records 1 and 2 only
    dev = an._deviations({"a": other, "b": ref}, "b", R)
    assert dev["b"] == 0.0
    sd = np.sqrt(ref.var(axis=1, ddof=1) / R * 2)        # same spread in both (a shifted copy)
    want = max(0.05 / sd[1], 0.02 / sd[2])
    assert dev["a"] == pytest.approx(want, rel=1e-12)
