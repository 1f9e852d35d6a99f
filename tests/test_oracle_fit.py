"""Pins of the oracle's peak-width fit (Sec. V.F, Eq. asymmetricLorentzian).

The model is pinned by its special cases (c = 0 is a Cauchy density times
pi (a + b/2); a steep step c -> +inf leaves a on the right of eps and a + b on the
left; the integral with b = 0 is pi a; c -> -c is (a, b) -> (a + b, -b)), the fit by
recovering the parameters of noise-free data and by being a minimum of the
squared error on noisy data.
"""
import numpy as np
import pytest
from scipy import integrate, stats

from oracle import fit

P_TRUE = np.array([0.30, 0.25, 6.0, 0.22, 1.35])  # a, b, c, gamma, eps


def test_model_special_cases():
    w = np.linspace(-2.0, 4.0, 301)
    a, b, c, g, e = 0.7, -0.3, 0.0, 0.4, 1.1
    ref = np.pi * (a + b / 2) * stats.cauchy.pdf(w, loc=e, scale=g)
    assert np.abs(fit.model((a, b, c, g, e), w) - ref).max() <= 1e-14 * np.abs(ref).max()
    # a steep step: a alone for w > eps, a + b for w < eps
    lor = np.pi * stats.cauchy.pdf(w, loc=e, scale=g)
    right, left = w > e + 0.5, w < e - 0.5
    s = fit.model((a, b, 200.0, g, e), w)
    assert np.allclose(s[right], a * lor[right], rtol=1e-12, atol=0)
    assert np.allclose(s[left], (a + b) * lor[left], rtol=1e-12, atol=0)
    # the value at the peak centre
    assert fit.model((a, b, 5.0, g, e), np.array([e]))[0] == pytest.approx((a + b / 2) / g, rel=1e-15)
    # c -> -c swaps the sides
    assert np.allclose(fit.model((a, b, -3.0, g, e), w), fit.model((a + b, -b, 3.0, g, e), w), rtol=1e-13, atol=0)
    # integral over the real line with b = 0 is pi a
    val, _ = integrate.quad(lambda x: fit.model((a, 0.0, 2.0, g, e), np.array([x]))[0], -np.inf, np.inf,
                            epsabs=1e-13, epsrel=1e-12)
    assert val == pytest.approx(np.pi * a, rel=1e-9)


@pytest.mark.parametrize("start", ["data", "given"])
def test_fit_recovers_noise_free_parameters(start):
    w = np.linspace(0.0, 3.0, 601)
    y = fit.model(P_TRUE, w)
    init = None if start == "data" else P_TRUE * np.array([1.3, 0.6, 0.5, 1.4, 1.05])
    p, cost, ratio = fit.fit_asymmetric_lorentzian(w, y, 1.0, 2.0, init)
    assert np.abs(p - P_TRUE).max() <= 1e-8 * np.abs(P_TRUE).max()
    assert cost <= 1e-20 and ratio == pytest.approx(P_TRUE[3] / P_TRUE[4], rel=1e-8)


def test_fit_is_a_minimum_on_noisy_data():
    rng = np.random.default_rng(5)
    w = np.linspace(0.0, 3.0, 601)
    y = fit.model(P_TRUE, w) * (1 + 0.03 * rng.normal(size=w.size))
    p, cost, _ = fit.fit_asymmetric_lorentzian(w, y, 1.0, 2.0)
    ww, yy = fit.window(w, y, 1.0, 2.0)

    def f(q):
        r = fit.model(q, ww) - yy
        return 0.5 * float(r @ r)

    assert cost == pytest.approx(f(p), rel=1e-14)
    # stationary: central differences of the cost vanish relative to its curvature scale
    for j in range(5):
        h = 1e-6 * max(abs(p[j]), 1e-3)
        dp = np.zeros(5)
        dp[j] = h
        grad = (f(p + dp) - f(p - dp)) / (2 * h)
        curv = (f(p + dp) - 2 * f(p) + f(p - dp)) / (h * h)
        assert abs(grad) <= 1e-4 * abs(curv) * max(abs(p[j]), 1e-3)
    # no random nearby point is lower
    for _ in range(200):
        q = p * (1 + 1e-3 * rng.normal(size=5))
        assert f(q) >= cost
    assert np.abs(p - P_TRUE).max() <= 0.2 * np.abs(P_TRUE).max()


def test_fit_reports_positive_gamma_and_needs_points():
    w = np.linspace(0.0, 3.0, 301)
    y = fit.model(P_TRUE, w)
    p, _, _ = fit.fit_asymmetric_lorentzian(w, y, 1.0, 2.0, init=P_TRUE * np.array([-1, -1, 1, -1, 1]))
    assert p[3] > 0 and np.abs(p - P_TRUE).max() <= 1e-8
    with pytest.raises(ValueError):
        fit.fit_asymmetric_lorentzian(w, y, 1.0, 1.03)
