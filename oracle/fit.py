"""Peak-width extraction from a produced spectrum -- oracle side.

Test infrastructure only (see ``oracle/__init__``).

Sec. V.F (Eq. asymmetricLorentzian): the high-energy peak of S(Q, omega) is fitted
by an asymmetric Lorentzian

    s(w) = gamma / (gamma^2 + (w - eps)^2) * (a + b / (1 + exp(c (w - eps)))),

with free a, b, c, gamma, eps, on an energy window [lo, hi] that leaves out the
low-energy tail; gamma / eps then measures the width of the peak.  The paper
states neither the loss nor the start; we take ordinary least squares
sum_i (s(w_i) - y_i)^2 over the grid points inside the window (inclusive) and the
start of ``initial_guess``.  The minimisation itself is a library routine
(MINPACK's Levenberg-Marquardt through scipy).  gamma and -gamma give the same
curve with (a, b) negated, so the result is reported with gamma > 0.
"""
import numpy as np
from scipy.optimize import least_squares


def model(p, w):
    """s(w) for p = (a, b, c, gamma, eps), written as the equation reads."""
    a, b, c, g, e = p
    x = np.asarray(w, dtype=np.float64) - e
    t = np.clip(c * x, -700.0, 700.0)
    return g / (g * g + x * x) * (a + b / (1.0 + np.exp(t)))


def window(w, y, lo, hi):
    w = np.asarray(w, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    sel = (w >= lo) & (w <= hi)
    return w[sel], y[sel]


def initial_guess(w, y):
    """Start of the fit from the windowed data: eps at the largest value y_max,
    gamma the half width at half maximum (mean of the distances from the peak to
    the nearest points on either side below y_max / 2, the one side found if only
    one is, a quarter of the window if none), a + b/2 = y_max gamma (the value at
    the peak with c = 0) split as a = 0.75 y_max gamma, b = 0.5 y_max gamma, c = 0."""
    k = int(np.argmax(y))
    ym, e = float(y[k]), float(w[k])
    half = []
    for rng_ in (range(k - 1, -1, -1), range(k + 1, len(y))):
        for i in rng_:
            if y[i] < 0.5 * ym:
                half.append(abs(float(w[i]) - e))
                break
    g = float(np.mean(half)) if half else 0.25 * float(w[-1] - w[0])
    return np.array([0.75 * ym * g, 0.5 * ym * g, 0.0, g, e])


def fit_asymmetric_lorentzian(w, y, lo, hi, init=None):
    """Least-squares parameters (a, b, c, gamma, eps) on [lo, hi], their cost
    0.5 sum r^2 and gamma / eps."""
    ww, yy = window(w, y, lo, hi)
    if len(ww) < 5:
        raise ValueError("fewer than 5 points in the window")
    p0 = initial_guess(ww, yy) if init is None else np.asarray(init, dtype=np.float64)
    res = least_squares(lambda p: model(p, ww) - yy, p0, method="lm", xtol=1e-15, ftol=1e-15, gtol=1e-15,
                        max_nfev=20000)
    p = res.x.copy()
    if p[3] < 0:
        p[0], p[1], p[3] = -p[0], -p[1], -p[3]
    r = model(p, ww) - yy
    return p, 0.5 * float(r @ r), p[3] / p[4]
