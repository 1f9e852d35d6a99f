"""Thermodynamics from the shell data of the filtered typical states -- oracle side.

Test infrastructure only (see ``oracle/__init__``).

Sec. II.A: Z(beta) = N_F E[<phi_0|e^{-beta H}|phi_0>], so the anchor's own
partition function is N_F times the sample mean of ||phi_beta||^2 =
exp(2 log_norm_s).  Eq. (FRW1) with O = H and O = H^2 gives the reweighted
moments from the per-shell values h1_m = <phi^m|H|phi^m> and
h2_m = <H phi^m|H phi^m> (phi^m built from the normalised phi_beta):
    W_sm   = exp(2 log_norm_s + (beta_a - beta') E_m),
    <H>    = sum W h1 / sum W n,     <H^2> = sum W h2 / sum W n,
    C      = beta'^2 (<H^2> - <H>^2)                      (k_B = 1),
    ln Z(beta') = ln N_F + ln mean_s exp(2 log_norm_s)
                  + ln( sum W n / sum W(beta' = beta_a) n ),
    S      = beta' <H> + ln Z(beta')        (F = <H> - T S = -T ln Z).
The shell sums enter Z only as a ratio to the anchor's own sum, so the
partition-of-unity defect of sum_m f_m^2 cancels at beta' = beta_a.  When h1,
h2 are not given, E_m n_m and E_m^2 n_m stand in (their error is O(eps)).
Anchors, sample averaging (ratio of sums), exponent shifts and binning follow
reweight.py.
"""
import math

import numpy as np

from .reweight import pick_anchor


def _logsumexp(x):
    mx = np.max(x)
    return mx + math.log(float(np.sum(np.exp(x - mx))))


def _one(beta_a, bt, E_m, ln, n, h1, h2, N):
    """(E, C, S, lnZ) of one anchor from samples ln [S], n/h1/h2 [S, L]."""
    e1, e2, lnZ = _moments(beta_a, bt, E_m, ln, n, h1, h2, N)
    C = bt * bt * (e2 - e1 * e1)
    S = bt * e1 + lnZ
    return e1, C, S, lnZ


def _moments(beta_a, bt, E_m, ln, n, h1, h2, N):
    """(<H>, <H^2>, lnZ) of one anchor reweighted to bt."""
    valid = n > 0
    logw = np.where(valid, 2.0 * ln[:, None] + (beta_a - bt) * E_m[None, :], -np.inf)
    log0 = np.where(valid, 2.0 * ln[:, None] + 0.0 * E_m[None, :], -np.inf)
    mx = np.max(logw)
    w = np.exp(logw - mx)
    den = float(np.sum(w * n))
    e1 = float(np.sum(w * h1)) / den
    e2 = float(np.sum(w * h2)) / den
    lnZ = (N * math.log(2.0) + _logsumexp(2.0 * ln) - math.log(len(ln))
           + (math.log(den) + mx) - _logsumexp(np.log(np.where(valid, n, 1.0)) + log0))
    return e1, e2, lnZ


def thermodynamics(betas, E_m, log_norm, n_m, h1, h2, n_sites, temps, n_bins=8):
    """betas [A]; E_m [A, L]; log_norm [S, A]; n_m, h1, h2 [S, A, L] (h1/h2 may be None).

    Returns dict of arrays over temps: E, C, S, lnZ and their binned standard errors
    E_err, C_err, S_err, lnZ_err (NaN below 2 bins)."""
    betas = np.asarray(betas, dtype=np.float64)
    E_m = np.asarray(E_m, dtype=np.float64)
    n_m = np.asarray(n_m, dtype=np.float64)
    if h1 is None:
        h1 = E_m[None, :, :] * n_m
    if h2 is None:
        h2 = E_m[None, :, :] ** 2 * n_m
    S_n = log_norm.shape[0]
    B = min(n_bins, S_n)
    nT = len(temps)
    out = {k: np.zeros(nT) for k in ("E", "C", "S", "lnZ")}
    out.update({k + "_err": np.full(nT, np.nan) for k in ("E", "C", "S", "lnZ")})
    for it, T in enumerate(temps):
        bt = 1.0 / T
        a = pick_anchor(betas, bt)
        vals = _one(betas[a], bt, E_m[a], log_norm[:, a], n_m[:, a], h1[:, a], h2[:, a], n_sites)
        for k, v in zip(("E", "C", "S", "lnZ"), vals):
            out[k][it] = v
        if B >= 2:
            bins = []
            for b in range(B):
                sel = slice(b * S_n // B, (b + 1) * S_n // B)
                bins.append(_one(betas[a], bt, E_m[a], log_norm[sel, a], n_m[sel, a], h1[sel, a], h2[sel, a],
                                 n_sites))
            bins = np.array(bins)
            for j, k in enumerate(("E", "C", "S", "lnZ")):
                out[k + "_err"][it] = bins[:, j].std(ddof=1) / math.sqrt(B)
    return out


def diagnostics(betas, E_m, log_norm, n_m, h1, h2, n_sites, inv_temps, n_bins=8):
    """Per inverse temperature b (b >= 0): the energy variance <H^2> - <H>^2 (the squared
    width C/b^2 of the energy distribution, Sec. III.D) and ln[Z(2b)/Z(b)^2] (Sec. III.C and V.B:
    equal to -S(b*) for some b* in [b, 2b]; its square root sets the sample scatter),
    each quantity from the anchors thermodynamics() picks for b and for 2b on the same
    samples.  Returns dict var, log_typ and their binned errors (NaN below 2 bins)."""
    betas = np.asarray(betas, dtype=np.float64)
    E_m = np.asarray(E_m, dtype=np.float64)
    n_m = np.asarray(n_m, dtype=np.float64)
    if h1 is None:
        h1 = E_m[None, :, :] * n_m
    if h2 is None:
        h2 = E_m[None, :, :] ** 2 * n_m
    S_n = log_norm.shape[0]
    B = min(n_bins, S_n)

    def vals(b, sel):
        a = pick_anchor(betas, b)
        e1, e2, lz1 = _moments(betas[a], b, E_m[a], log_norm[sel, a], n_m[sel, a], h1[sel, a], h2[sel, a], n_sites)
        a2 = pick_anchor(betas, 2.0 * b)
        _, _, lz2 = _moments(betas[a2], 2.0 * b, E_m[a2], log_norm[sel, a2], n_m[sel, a2], h1[sel, a2],
                             h2[sel, a2], n_sites)
        return e2 - e1 * e1, lz2 - 2.0 * lz1

    nT = len(inv_temps)
    out = {"var": np.zeros(nT), "log_typ": np.zeros(nT),
           "var_err": np.full(nT, np.nan), "log_typ_err": np.full(nT, np.nan)}
    for it, b in enumerate(inv_temps):
        out["var"][it], out["log_typ"][it] = vals(b, slice(0, S_n))
        if B >= 2:
            bins = np.array([vals(b, slice(k * S_n // B, (k + 1) * S_n // B)) for k in range(B)])
            out["var_err"][it], out["log_typ_err"][it] = bins.std(axis=0, ddof=1) / math.sqrt(B)
    return out


def overlap_ratio(E1, var1, E2, var2):
    """r of Sec. III.D: |<H>_1 - <H>_2| / (sigma_1 + sigma_2), sigma^2 = C/(k_B beta^2)."""
    return abs(E1 - E2) / (math.sqrt(var1) + math.sqrt(var2))


def choose_anchors(beta_grid, E, var, r_max, max_anchors):
    """Anchor ladder down an ascending grid of inverse temperatures (Sec. III.D: the
    reweighting works while the energy distributions at the anchor and at the target
    overlap, r small).  A target is reweighted from the hottest anchor at or above its
    temperature (reweight() picks the largest beta_a <= beta'), so the first anchor is
    beta_grid[0] and each next anchor is the first grid point whose r with the current
    anchor exceeds r_max; every target then has r <= r_max unless max_anchors runs out.
    E, var: <H> and <H^2> - <H>^2 on the grid.  Returns the anchor indices."""
    n = len(beta_grid)
    anchors = [0]
    i = 0
    while len(anchors) < max_anchors:
        j = i + 1
        while j < n and overlap_ratio(E[i], var[i], E[j], var[j]) <= r_max:
            j += 1
        if j >= n:
            break
        anchors.append(j)
        i = j
    return anchors
