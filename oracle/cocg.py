"""Shifted COCG with seed switching -- oracle side.

Test infrastructure only (see ``oracle/__init__``).

Sec. II.B solves (zeta - H) chi(zeta) = rho for a whole set of shifts with shifted
BiCG and an arbitrary shadow vector.  In the S^z basis H is real symmetric, so every
zeta - H is complex symmetric; with the shadow vector taken as the complex conjugate
of the right-hand side, BiCG becomes COCG (conjugate-orthogonal CG: the bilinear form
x^T y replaces <x|y>), and its residuals for all shifts are collinear, so one seed
recurrence serves every shift through scalar factors pi (the shifted methods the paper
cites).  Appendix C tracks the largest residual 2-norm over the shifts by seed
switching: when the seed system has converged, the unconverged shift with the
largest residual becomes the seed.

Two forms live here.

``shifted_cocg`` is the textbook algorithm with vectors: the seed's x, r, p and, for
every shift, x^j and p^j, so that the pins can check (zeta_j - H) x^j = rho directly.

``lanczos_bilinear`` + ``cocg_from_bilinear`` is the form the device follows (its
arithmetic twin): the complex-symmetric Lanczos basis q_k with q_j^T q_k = delta_jk
(unnormalised residuals with a carried complex scale, exact-sum bilinear products),
then per shift the shifted COCG scalar recurrences with seed switching driven by the
basis coefficients a_k, b_k and the projections c_k = <lam|q_k>.  The seed's CG
coefficients are the pivots of (z_s - T_n) = L D L^T: 1/alpha_k = z_s - a_k -
b_k^2 alpha_{k-1}, beta_k = b_{k+1}^2 alpha_k^2, and its residual is r_k = delta_k q_k
with delta_{k+1} = alpha_k b_{k+1} delta_k (delta_0 = sqrt(rho^T rho)).
"""
import ctypes
import math

import numpy as np

from . import _native
from ._native import ptr


def _c(v):
    return np.ascontiguousarray(v, dtype=np.float64).view(np.complex128)


def shifted_cocg(H, rho, z, n, lam=None, seed=0, seed_tol=1e-12):
    """Textbook shifted COCG with seed switching for (z_j - H) x_j = rho, n steps.

    rho, lam: interleaved float64 vectors (lam defaults to rho).  Returns (G, X, resid,
    seeds): G[j] = <lam|x_j>, X[j] = x_j (complex rows), resid[j] = ||rho - (z_j - H) x_j||
    as the recurrence tracks it, and the seed index used at every step."""
    z = np.asarray(z, dtype=np.complex128)
    b = _c(rho).copy()
    lv = b if lam is None else _c(lam)
    nz, dim = len(z), b.shape[0]
    s = int(seed)
    r = b.copy()
    x = np.zeros_like(b)
    p = np.zeros_like(b)
    X = np.zeros((nz, dim), dtype=np.complex128)
    Pj = np.zeros((nz, dim), dtype=np.complex128)
    pi = np.ones(nz, dtype=np.complex128)
    pi_old = np.ones(nz, dtype=np.complex128)
    alpha_old, beta_old = 1.0 + 0j, 0j
    rho_k = np.dot(r, r)  # bilinear
    nrm_b = np.linalg.norm(b)
    seeds = []

    def apply_A(zs, v):
        hv = _c(H.apply(np.ascontiguousarray(v).view(np.float64)))
        return zs * v - hv

    for k in range(n):
        seeds.append(s)
        zs = z[s]
        p = r + beta_old * p
        w = apply_A(zs, p)
        alpha = rho_k / np.dot(p, w)
        # shifted systems: collinear residuals r_j = r / pi_j
        sigma = z - zs
        pi_new = (1.0 + alpha * sigma) * pi + (alpha * beta_old / alpha_old) * (pi - pi_old)
        beta_j = (pi_old / pi) ** 2 * beta_old
        alpha_j = (pi / pi_new) * alpha
        Pj = r[None, :] / pi[:, None] + beta_j[:, None] * Pj
        X = X + alpha_j[:, None] * Pj
        x = x + alpha * p
        r = r - alpha * w
        rho_new = np.dot(r, r)
        beta = rho_new / rho_k
        pi_old, pi = pi, pi_new
        alpha_old, beta_old, rho_k = alpha, beta, rho_new
        res = np.linalg.norm(r) / np.abs(pi)
        # seed switching: the seed has converged and another shift has not
        if res[s] <= seed_tol * nrm_b and res.max() > seed_tol * nrm_b:
            t = int(np.argmax(res))
            # the new seed's residual, search direction and CG coefficients
            r = r / pi[t]
            p = Pj[t].copy()
            alpha_old = alpha_old * pi_old[t] / pi[t]
            beta_old = beta_old * (pi_old[t] / pi[t]) ** 2
            rho_k = np.dot(r, r)
            pi_old = pi_old / pi_old[t]
            pi = pi / pi[t]
            s = t
    G = np.array([np.vdot(lv, X[j]) for j in range(nz)])
    resid = np.linalg.norm(r) / np.abs(pi)
    return G, X, resid, seeds


def lanczos_bilinear(H, start, n, lam=None):
    """Complex-symmetric Lanczos in the device's arithmetic (ftk_oracle.c:orc_lanczos_bilinear).

    Returns (a, b, c, hn, delta0, steps): a[k] = q_k^T H q_k, b[k] = b_{k+1} (complex;
    principal square roots), c[k] = <lam|q_k>, hn[k] = ||q_k||^2 (Hermitian norm of the
    bilinear-normalised vector, k = 0..steps), delta0 = sqrt(rho^T rho)."""
    start = np.ascontiguousarray(start, dtype=np.float64)
    lamv = start if lam is None else np.ascontiguousarray(lam, dtype=np.float64)
    a = np.zeros(2 * n)
    b = np.zeros(2 * n)
    c = np.zeros(2 * (n + 1))
    hn = np.zeros(n + 1)
    d0 = np.zeros(2)
    steps = _native.lib().orc_lanczos_bilinear(*H._args(), ptr(start), ptr(lamv), n, H.breakdown_tol(), ptr(a),
                                               ptr(b), ptr(c), ptr(hn), ptr(d0))
    cv = lambda v: v.view(np.complex128)
    return cv(a)[:steps], cv(b)[:steps], cv(c)[: steps + 1], hn[: steps + 1], complex(d0[0], d0[1]), steps


# complex scalar arithmetic on (re, im) float pairs, spelled out so that the device's
# per-shift kernel can follow the same IEEE operations
def cmul(ar, ai, br, bi):
    return ar * br - ai * bi, ar * bi + ai * br


def cdiv(ar, ai, br, bi):
    """(ar + i ai) / (br + i bi) by Smith's algorithm (R. L. Smith, CACM 5, 435, 1962),
    elementwise on scalars or arrays: no squares of the divisor, so no overflow."""
    ar, ai, br, bi = (np.asarray(x, dtype=np.float64) for x in (ar, ai, br, bi))
    big = np.abs(br) >= np.abs(bi)
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = bi / br
        d1 = br + bi * t1
        r1, i1 = (ar + ai * t1) / d1, (ai - ar * t1) / d1
        t2 = br / bi
        d2 = br * t2 + bi
        r2, i2 = (ar * t2 + ai) / d2, (ai * t2 - ar) / d2
    re, im = np.where(big, r1, r2), np.where(big, i1, i2)
    if re.ndim == 0:
        return float(re), float(im)
    return re, im


def cocg_from_bilinear(a, b, c, hn, delta0, z, seed=0, seed_tol=1e-12, rtol=0.0):
    """Per-shift shifted COCG with seed switching from the complex-symmetric Lanczos
    coefficients: G[j] = <lam|x_j>, the residual 2-norm of every shift and the seed of
    every step followed by the final seed (so len(seeds) - 1 steps were taken).
    Vectorised over the shifts, the same scalar operations as the device kernel.

    A shift other than the seed whose residual has fallen to seed_tol ||rho|| is
    converged: it is no longer updated (its x_j is final; continuing would only drive
    pi_j towards overflow once the Krylov space is exhausted).  The run ends after n =
    len(a) steps, once every shift is converged to seed_tol ||rho||, or with rtol > 0
    once the largest residual is at most rtol ||rho|| (the truncation of Appendix C)."""
    z = np.asarray(z, dtype=np.complex128)
    zr, zi = z.real.copy(), z.imag.copy()
    nz = len(z)
    n = len(a)
    s = int(seed)
    # seed CG state: alpha_{k-1}, beta_{k-1}, delta_k
    alr, ali = 1.0, 0.0
    ber, bei = 0.0, 0.0
    dr, di = delta0.real, delta0.imag
    nrm_b = math.sqrt(hn[0]) * math.sqrt(delta0.real * delta0.real + delta0.imag * delta0.imag)  # ||rho||
    # per shift: pi_k, pi_{k-1}, P_{k-1}, g
    pr, pim = np.ones(nz), np.zeros(nz)
    por, poi = np.ones(nz), np.zeros(nz)
    Pr, Pi = np.zeros(nz), np.zeros(nz)
    gr, gi = np.zeros(nz), np.zeros(nz)
    res = np.full(nz, np.inf)
    thr = seed_tol * nrm_b
    idx = np.arange(nz)
    seeds = []
    for k in range(n):
        seeds.append(s)
        live = (idx == s) | ~(res <= thr)
        ak, bk = a[k], (b[k - 1] if k > 0 else 0j)
        # seed pivot: 1/alpha_k = z_s - a_k - b_k^2 alpha_{k-1}
        b2r, b2i = cmul(bk.real, bk.imag, bk.real, bk.imag)
        tr, ti = cmul(b2r, b2i, alr, ali)
        dvr = (zr[s] - ak.real) - tr
        dvi = (zi[s] - ak.imag) - ti
        anr, ani = cdiv(1.0, 0.0, dvr, dvi)
        # shifted factors
        sgr, sgi = zr - zr[s], zi - zi[s]
        t1r, t1i = cmul(anr, ani, sgr, sgi)
        fr, fi = cmul(anr, ani, ber, bei)
        fr, fi = cdiv(fr, fi, alr, ali)  # alpha_k beta_{k-1} / alpha_{k-1}
        d1r, d1i = pr - por, pim - poi
        u1r, u1i = cmul(1.0 + t1r, t1i, pr, pim)
        u2r, u2i = cmul(fr, fi, d1r, d1i)
        pnr, pni = u1r + u2r, u1i + u2i
        # beta^j_{k-1} = beta_{k-1} (pi_{k-1}/pi_k)^2, alpha^j_k = alpha_k pi_k / pi_{k+1}
        qr, qi = cdiv(por, poi, pr, pim)
        q2r, q2i = cmul(qr, qi, qr, qi)
        bjr, bji = cmul(ber, bei, q2r, q2i)
        xr, xi = cdiv(pr, pim, pnr, pni)
        ajr, aji = cmul(anr, ani, xr, xi)
        # P^j_k = delta_k c_k / pi_k + beta^j_{k-1} P^j_{k-1};  g += alpha^j_k P^j_k
        ck = c[k]
        er, ei = cmul(dr, di, ck.real, ck.imag)
        hr, hi = cdiv(er, ei, pr, pim)
        mr, mi = cmul(bjr, bji, Pr, Pi)
        Pnr, Pni = hr + mr, hi + mi
        vr, vi = cmul(ajr, aji, Pnr, Pni)
        # converged shifts keep their values
        Pr, Pi = np.where(live, Pnr, Pr), np.where(live, Pni, Pi)
        gr, gi = np.where(live, gr + vr, gr), np.where(live, gi + vi, gi)
        pnr, pni = np.where(live, pnr, pr), np.where(live, pni, pim)
        por_n, poi_n = np.where(live, pr, por), np.where(live, pim, poi)
        # seed coefficients for the next step and the new residual scale
        bn = b[k]
        bnr, bni = cmul(bn.real, bn.imag, bn.real, bn.imag)
        a2r, a2i = cmul(anr, ani, anr, ani)
        ber, bei = cmul(bnr, bni, a2r, a2i)  # beta_k = b_{k+1}^2 alpha_k^2
        wr, wi = cmul(anr, ani, bn.real, bn.imag)
        dr, di = cmul(wr, wi, dr, di)        # delta_{k+1} = alpha_k b_{k+1} delta_k
        alr, ali = anr, ani
        por, poi, pr, pim = por_n, poi_n, pnr, pni
        # residual 2-norms: |delta_{k+1}| ||q_{k+1}|| / |pi_{k+1}|
        rs = math.sqrt(dr * dr + di * di) * math.sqrt(hn[k + 1])
        res = np.where(live, rs / np.sqrt(pr * pr + pim * pim), res)
        if rtol > 0.0 and res.max() <= rtol * nrm_b:
            break
        if res[s] <= thr and not res.max() > thr:
            break  # every shift converged
        if res[s] <= thr:
            t = int(np.argmax(res))
            # alpha_k, beta_k, delta_{k+1} of the new seed; all pi rebased on it
            xr, xi = cdiv(por[t], poi[t], pr[t], pim[t])
            alr, ali = cmul(alr, ali, xr, xi)
            x2r, x2i = cmul(xr, xi, xr, xi)
            ber, bei = cmul(ber, bei, x2r, x2i)
            dr, di = cdiv(dr, di, pr[t], pim[t])
            o_r, o_i = por[t], poi[t]
            n_r, n_i = pr[t], pim[t]
            rb = res > thr  # the shifts still running
            xr, xi = cdiv(por, poi, o_r, o_i)
            por, poi = np.where(rb, xr, por), np.where(rb, xi, poi)
            xr, xi = cdiv(pr, pim, n_r, n_i)
            pr, pim = np.where(rb, xr, pr), np.where(rb, xi, pim)
            s = t
    seeds.append(s)
    return gr + 1j * gi, res, seeds
