"""Canonical typical pure state phi_beta = e^{-beta H/2} phi_0 (Eq. tau) -- oracle side.

Test infrastructure only (see ``oracle/__init__``).

Appendix A: with h = H/N,
    e^{N beta l/2} phi_beta = e^{N beta (l - h)/2} phi_0 = sum_k (N beta/2)^k (l - h)^k phi_0 / k!,
split into M_d factors e^{(N beta / 2 M_d)(l - h)}, each summed as a Taylor series.
The k-th term of one factor is bounded by X^k/k! with X = (N beta / 2 M_d)(l + |e_0|);
its largest value is about e^X / sqrt(2 pi X), and M_d is chosen so that this is
the preset Lambda.  X solves e^X / sqrt(2 pi X) = Lambda through the recurrence
X_{k+1} = ln Lambda + (1/2) ln(2 pi X_k), X_0 = Lambda.

Readings where the appendix is silent or garbled:
  * l and e_0 are taken as the upper and lower bounds of the spectrum of h,
    l = B_H/N and e_0 = -B_H/N with B_H = sum over bonds of the largest |bond
    eigenvalue|, so (l - h) >= 0 and every series term is a positive combination.
  * The printed equation e^X/(2 pi X)^{-1/2} = Lambda disagrees with the recurrence
    and with the asymptotic maximum just above it; the recurrence (e^X/(2 pi X)^{1/2}) is used.
  * Lambda = 1e8; M_d = ceil(N beta (l + |e_0|) / (2 X)), at least 1 when beta > 0.
  * The series of one factor stops at the first k > X with X^k/k! < 1e-18 (the
    factor is >= 1 on every eigenvector, so this bounds the relative truncation).
  * After every factor the vector is renormalised and log of the norm accumulated,
    so e^{-beta H/2} phi_0 = exp(log_norm) * phi_beta_hat never overflows.
Per element, one term is t' = fma(a, t, b (H t)) with a = s l, b = -(s/N),
s = c/k, c = N beta/(2 M_d); the sum accumulates acc = acc + t'.
"""
import math

import numpy as np

from . import _native
from ._native import ptr
from .hamiltonian import normalize

LAMBDA = 1e8


def x_of_lambda(lam=LAMBDA, iters=200):
    x = lam
    for _ in range(iters):
        x = math.log(lam) + 0.5 * math.log(2.0 * math.pi * x)
    return x


def split_plan(N, beta, norm_bound, lam=LAMBDA):
    """(M_d, c, K, ell): number of factors, per-factor time, terms per factor, shift l."""
    ell = norm_bound / N
    width = 2.0 * norm_bound / N  # l + |e_0|
    if beta == 0.0:
        return 0, 0.0, 0, ell
    X = x_of_lambda(lam)
    Md = max(1, int(math.ceil(N * beta * width / (2.0 * X))))
    c = N * beta / (2.0 * Md)
    Xs = c * width
    tau = 1.0
    k = 0
    while True:
        k += 1
        tau = tau * Xs / k
        if (k > Xs and tau < 1e-18) or k >= 400:
            break
    return Md, c, k, ell


def canonical_state(H, phi0, beta, lam=LAMBDA):
    """Normalised phi_beta and log ||e^{-beta H/2} phi0|| (phi0 normalised on input)."""
    N = H.N
    Md, c, K, ell = split_plan(N, beta, H.norm_bound, lam)
    phi = np.array(phi0, dtype=np.float64, copy=True)
    log_norm = 0.0
    lib = _native.lib()
    for _ in range(Md):
        t = phi.copy()
        acc = phi.copy()
        tn = np.empty_like(phi)
        for k in range(1, K + 1):
            s = c / k
            a = s * ell
            b = -(s / N)
            lib.orc_taylor_term(*H._args(), ptr(t), ptr(tn), ptr(acc), a, b)
            t, tn = tn, t
        phi, nrm = normalize(acc)
        log_norm += math.log(nrm)
    # the factors computed e^{N beta l / 2} e^{-beta H / 2} phi0
    log_norm -= N * beta * ell / 2.0
    return phi, log_norm
