"""Reweighting of shell data into canonical S(Q, omega, T') (Sec. III.D) -- oracle side.

Test infrastructure only (see ``oracle/__init__``).

Eq. (FRW1): <O>_{beta'} = sum_m e^{(beta - beta') E_m} <phi^m|O|phi^m>
                          / sum_l e^{(beta - beta') E_l} <phi^l|phi^l>.
Eq. (limGAB) averages numerator and denominator over random vectors separately
(E[<phi_beta|phi_beta> G~] / E[<phi_beta|phi_beta>]), so the sample average is a
ratio of sums.  Each sample's shell data are stored for the normalised phi_beta
together with log ||e^{-beta H/2} phi_0||, so sample s carries the factor
exp(2 log_norm_s).  Readings:
  * the FRW1 denominator sum_l n_l is used for every beta' (including beta' = beta);
  * each T' uses the anchor with the largest beta_a <= beta' (the hottest anchor
    if none is that cold), as the paper reweights from the nearest anchor above;
  * exponents are shifted by their maximum before exponentiation;
  * the standard error comes from binning (Sec. V.D): the samples are split into
    B contiguous bins, the ratio is formed per bin, and
    sigma_E = std_{ddof=1}(bin values) / sqrt(B).
Output: S(Q, omega, T') = -(1/pi) Im [sum over alpha of the reweighted g].
"""
import math

import numpy as np


def pick_anchor(betas, beta_t):
    """Index of the anchor with the largest beta_a <= beta_t (else the smallest beta_a)."""
    best = None
    for a, b in enumerate(betas):
        if b <= beta_t and (best is None or b > betas[best]):
            best = a
    if best is None:
        best = int(np.argmin(betas))
    return best


def _ratio(logw, g, n):
    """-(1/pi) Im(sum W g) / sum W n with W = exp(logw - max)."""
    mx = np.max(logw)
    w = np.exp(logw - mx)
    num = np.tensordot(w, g, axes=(list(range(w.ndim)), list(range(w.ndim))))
    den = float(np.sum(w * n))
    return -(num.imag) / (math.pi * den)


def reweight(betas, E_m, eps, log_norm, n_m, g, temps, n_bins=8):
    """betas [A]; E_m [A, L]; eps [A]; log_norm [S, A]; n_m [S, A, L];
    g [S, A, L, Q, W] complex (already summed over alpha); temps [T'].

    Returns S [Q, T', W], stderr [Q, T', W] (NaN when fewer than 2 bins) and
    P [T', L] (Eq. FRW2 on the grid of the anchor used)."""
    betas = np.asarray(betas, dtype=np.float64)
    S_n, A = log_norm.shape
    _, _, L, nQ, nW = g.shape
    nT = len(temps)
    out = np.zeros((nQ, nT, nW))
    err = np.full((nQ, nT, nW), np.nan)
    P = np.zeros((nT, L))
    B = min(n_bins, S_n)
    for it, T in enumerate(temps):
        bt = 1.0 / T
        a = pick_anchor(betas, bt)
        logw = 2.0 * log_norm[:, a][:, None] + (betas[a] - bt) * E_m[a][None, :]  # [S, L]
        valid = n_m[:, a, :] > 0
        logw = np.where(valid, logw, -np.inf)
        out[:, it, :] = _ratio(logw, g[:, a], n_m[:, a])
        w = np.exp(logw - np.max(logw))
        wn = (w * n_m[:, a]).sum(axis=0)
        P[it] = wn / (2.0 * eps[a] * wn.sum())
        if B >= 2:
            vals = []
            for b in range(B):
                sel = slice(b * S_n // B, (b + 1) * S_n // B)
                vals.append(_ratio(logw[sel], g[sel, a], n_m[sel, a]))
            vals = np.array(vals)
            err[:, it, :] = vals.std(axis=0, ddof=1) / math.sqrt(B)
    return out, err, P


def reweight_observable(betas, E_m, log_norm, n_m, O, temps, n_bins=8):
    """Eq. (FRW1) for real static observables: O [S, A, L, K] holds <phi^m|O_k|phi^m>
    per sample, anchor and shell (e.g. ||S^alpha_Q phi^m||^2 for the static structure
    factor).  Returns out [K, T'] = sum W O / sum W n and its binned error (NaN below 2
    bins), with the anchors, weights and sample average of reweight()."""
    betas = np.asarray(betas, dtype=np.float64)
    O = np.asarray(O, dtype=np.float64)
    S_n, A = log_norm.shape
    K = O.shape[3]
    nT = len(temps)
    out = np.zeros((K, nT))
    err = np.full((K, nT), np.nan)
    B = min(n_bins, S_n)

    def ratio(logw, o, n):
        w = np.exp(logw - np.max(logw))
        return np.tensordot(w, o, axes=([0, 1], [0, 1])) / float(np.sum(w * n))

    for it, T in enumerate(temps):
        bt = 1.0 / T
        a = pick_anchor(betas, bt)
        logw = 2.0 * log_norm[:, a][:, None] + (betas[a] - bt) * E_m[a][None, :]
        logw = np.where(n_m[:, a, :] > 0, logw, -np.inf)
        out[:, it] = ratio(logw, O[:, a], n_m[:, a])
        if B >= 2:
            vals = np.array([ratio(logw[b * S_n // B:(b + 1) * S_n // B], O[b * S_n // B:(b + 1) * S_n // B, a],
                                   n_m[b * S_n // B:(b + 1) * S_n // B, a]) for b in range(B)])
            err[:, it] = vals.std(axis=0, ddof=1) / math.sqrt(B)
    return out, err


def reweight_cross(betas, E_m, eps, log_norm, n_m, gab, gba, temps, n_bins=8):
    """Complex spectral density of operator pairs, Eq. (FRW1) applied to
    S_AB,m(w) = -(1/(2 pi i)) (G_AB,m(w) - conj(G_BA,m(w))): gab, gba [S, A, L, P, W].
    With X = (G_AB - conj(G_BA)) / 2, Re S_AB is what reweight() makes of X and Im S_AB
    minus what it makes of i X.  Returns S [P, T', W] complex and its binned errors
    (real and imaginary parts, NaN below 2 bins)."""
    X = 0.5 * (np.asarray(gab) - np.conj(gba))
    sr, er, _ = reweight(betas, E_m, eps, log_norm, n_m, X, temps, n_bins)
    si, ei, _ = reweight(betas, E_m, eps, log_norm, n_m, 1j * X, temps, n_bins)
    return sr - 1j * si, er + 1j * ei
