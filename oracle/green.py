"""Equi-energy Green's functions and the spectrum estimator (Sec. III.C, Sec. V) -- oracle side.

Test infrastructure only (see ``oracle/__init__``).

For each shell m, spin component alpha and momentum Q (Eq. SQomega_TPS):
    g_m(omega) = <phi^m| S^alpha_{-Q} (omega + i eta + E_m - H)^{-1} S^alpha_{+Q} |phi^m>.
With chi = S^alpha_{+Q} phi^m and S^alpha_{-Q} = (S^alpha_{+Q})^dagger this is
<chi|(z - H)^{-1}|chi>, and the n-step Galerkin value (lanczos.py) is
    g_m(omega) = ||chi||^2 [(z - T_n)^{-1}]_{00},   z = omega + i eta + E_m.
The vectors phi^m are kept unnormalised; the per-sample normalisation of
Eq. (GAB_TPS) cancels in the reweighted ratio (reweight.py).

General operators A != B (Sec. III.B, Eq. GAB_TPS): with lam = A phi^m and
rho = B phi^m, G_AB(z) = <lam|(z - H)^{-1}|rho>.  Reading: the sesquilinear form is
split by the polarization identity into four quadratic forms,
    G_AB = (g[lam+rho] - g[lam-rho] - i g[lam+i rho] + i g[lam-i rho]) / 4,
    G_BA = (g[lam+rho] - g[lam-rho] + i g[lam+i rho] - i g[lam-i rho]) / 4,
each an ordinary Galerkin value ||s||^2 [(z - T_n)^{-1}]_{00} of the Lanczos sequence
from s, so the same four sequences give both orders (the paper solves the same
systems with shifted BiCG and the shadow vector lam; both converge to the same
resolvent).  The spectral density of the pair is
    S_AB(w) = -(1/(2 pi i)) (G_AB(w + i eta) - G_AB(w - i eta)),
and G_AB(w - i eta) = conj(G_BA(w + i eta)) because H is real symmetric.
"""
import math

import numpy as np

from .hamiltonian import apply_sq, apply_spin_op, dot_re
from .lanczos import galerkin_residual, lanczos, lanczos_plain, resolvent_00, truncation_step


def green_sequence(H, chi, n, omega, eta, E_m, tol=0.0):
    """(g(omega), max residual, alpha, beta) for one start vector chi.  tol > 0 truncates
    the sequence at the first step whose residuals over all shifts are <= tol (per unit
    right-hand side)."""
    omega = np.asarray(omega, dtype=np.float64)
    nrm = math.sqrt(dot_re(chi, chi))
    if nrm == 0.0:
        return np.zeros(len(omega), dtype=np.complex128), 0.0, np.zeros(0), np.zeros(0)
    alpha, beta, _, nrm = lanczos(H, chi, n)
    z = omega + E_m + 1j * eta
    if tol > 0:
        k = truncation_step(alpha, beta, z, tol)
        alpha, beta = alpha[:k], beta[:k]
    g = (nrm * nrm) * resolvent_00(alpha, beta, z)
    res = nrm * galerkin_residual(alpha, beta, z)
    return g, float(res.max()), alpha, beta


def green_sequence_plain(H, chi, n, omega, eta, E_m):
    """g(omega) and the Galerkin residual of every shift from the plain-form Lanczos
    recurrence (lanczos.lanczos_plain): g = ||chi||^2 [(z - T_n)^{-1}]_{00} at
    z = omega + i eta + E_m.  Returns (g, residual per shift, alpha, beta)."""
    omega = np.asarray(omega, dtype=np.float64)
    alpha, beta, _, nrm = lanczos_plain(H, chi, n)
    z = omega + E_m + 1j * eta
    g = (nrm * nrm) * resolvent_00(alpha, beta, z)
    return g, nrm * galerkin_residual(alpha, beta, z), alpha, beta


def green_sequence_cocg(H, chi, n, omega, eta, E_m, seed=0, seed_tol=1e-12, rtol=0.0):
    """g(omega) = <chi|x_n(z)> from up to n steps of shifted COCG with seed switching at
    z = omega + i eta + E_m, in the device's form (cocg.lanczos_bilinear +
    cocg.cocg_from_bilinear).  Returns (g, residual per shift, a, b, c, seeds), the
    coefficients cut to the steps taken (len(seeds) - 1)."""
    from . import cocg
    omega = np.asarray(omega, dtype=np.float64)
    a, b, c, hn, d0, _ = cocg.lanczos_bilinear(H, chi, n)
    z = (omega + E_m) + 1j * eta
    g, res, seeds = cocg.cocg_from_bilinear(a, b, c, hn, d0, z, seed, seed_tol, rtol)
    k = len(seeds) - 1
    return g, res, a[:k], b[:k], c[: k + 1], seeds


def cross_green_cocg(H, lam, rho, n, omega, eta, E_m, seed=0, seed_tol=1e-12):
    """G_AB and G_BA by shifted COCG (the paper's shifted BiCG with the shadow vector
    conj(rho), Sec. II.B): G_AB = <lam|x(z)> from the run on rho, G_BA = <rho|y(z)> from
    the run on lam, z = omega + i eta + E_m; <lam|rho>; the largest residual of the two
    runs and the two runs' (a, b, c), cut to the steps each run took."""
    from . import cocg
    omega = np.asarray(omega, dtype=np.float64)
    z = (omega + E_m) + 1j * eta
    out = []
    for rhs, proj in ((rho, lam), (lam, rho)):
        a, b, c, hn, d0, _ = cocg.lanczos_bilinear(H, rhs, n, lam=proj)
        g, res, seeds = cocg.cocg_from_bilinear(a, b, c, hn, d0, z, seed, seed_tol)
        k = len(seeds) - 1
        out.append((g, res, a[:k], b[:k], c[: k + 1], d0))
    (gab, rab, a0, b0, c0, d0), (gba, rba, a1, b1, c1, _) = out
    ov = complex(c0[0].real * d0.real - c0[0].imag * d0.imag, c0[0].real * d0.imag + c0[0].imag * d0.real)
    return gab, gba, ov, max(rab.max(), rba.max()), ((a0, b0, c0), (a1, b1, c1))


def shell_spectra(H, Phi, E_m, qs, alphas, n, omega, eta, tol=0.0, norms=False):
    """g[m, a, q, w] for the filtered states Phi[m] (interleaved float64 rows).

    qs: list of (qx, qy); alphas: subset of (0, 1, 2) for x, y, z.  With norms, also
    ||chi||^2 = <phi^m|S^alpha_{-Q} S^alpha_{+Q}|phi^m> [m, a, q] (static structure factor)."""
    L = Phi.shape[0]
    out = np.zeros((L, len(alphas), len(qs), len(omega)), dtype=np.complex128)
    resid = np.zeros((L, len(alphas), len(qs)))
    chi2 = np.zeros((L, len(alphas), len(qs)))
    for m in range(L):
        for ia, a in enumerate(alphas):
            for iq, (qx, qy) in enumerate(qs):
                chi = apply_sq(H.cluster, a, qx, qy, Phi[m])
                g, r, _, _ = green_sequence(H, chi, n, omega, eta, E_m[m], tol)
                out[m, ia, iq] = g
                resid[m, ia, iq] = r
                chi2[m, ia, iq] = dot_re(chi, chi)
    if norms:
        return out, resid, chi2
    return out, resid


def polarized_starts(lam, rho):
    """lam + rho, lam - rho, lam + i rho, lam - i rho (interleaved float64 rows)."""
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    lr, li = lam[0::2], lam[1::2]
    rr, ri = rho[0::2], rho[1::2]
    out = np.empty((4, lam.shape[0]))
    out[0] = lam + rho
    out[1] = lam - rho
    out[2, 0::2] = lr - ri
    out[2, 1::2] = li + rr
    out[3, 0::2] = lr + ri
    out[3, 1::2] = li - rr
    return out


def combine_polarized(g):
    """(G_AB, G_BA) from the four quadratic forms g [4, ...] (complex)."""
    g = np.asarray(g, dtype=np.complex128)
    d_re = g[0].real - g[1].real
    d_im = g[0].imag - g[1].imag
    e_re = g[2].imag - g[3].imag  # real part of -i (g2 - g3)
    e_im = g[2].real - g[3].real  # minus the imaginary part of -i (g2 - g3)
    gab = 0.25 * (d_re + e_re) + 1j * (0.25 * (d_im - e_im))
    gba = 0.25 * (d_re - e_re) + 1j * (0.25 * (d_im + e_im))
    return gab, gba


def overlap_polarized(n2):
    """<lam|rho> from the four squared norms ||s_k||^2."""
    return complex(0.25 * (n2[0] - n2[1]), 0.25 * (n2[3] - n2[2]))


def cross_green(H, lam, rho, n, omega, eta, E_m, tol=0.0):
    """G_AB(omega), G_BA(omega) at z = omega + i eta + E_m, <lam|rho>, the largest residual
    of the four sequences and their (alpha, beta)."""
    S = polarized_starts(lam, rho)
    gs, res, coefs, n2 = [], [], [], []
    for k in range(4):
        g, r, al, be = green_sequence(H, S[k], n, omega, eta, E_m, tol)
        gs.append(g)
        res.append(r)
        coefs.append((al, be))
        n2.append(dot_re(S[k], S[k]))
    gab, gba = combine_polarized(gs)
    return gab, gba, overlap_polarized(n2), max(res), coefs


def spectral_density(gab, gba):
    """S_AB(w) = -(1/(2 pi i)) (G_AB(w + i eta) - conj(G_BA(w + i eta)))."""
    return -(np.asarray(gab) - np.conj(gba)) / (2j * math.pi)


def shell_cross(H, Phi, E_m, pairs, n, omega, eta, tol=0.0):
    """gab, gba [L, P, W] and <lam|rho> [L, P] for operator pairs (coef_A, coef_B)."""
    L = Phi.shape[0]
    N = H.cluster.n_sites
    gab = np.zeros((L, len(pairs), len(omega)), dtype=np.complex128)
    gba = np.zeros_like(gab)
    lr = np.zeros((L, len(pairs)), dtype=np.complex128)
    for m in range(L):
        for ip, (ca, cb) in enumerate(pairs):
            lam = apply_spin_op(N, ca, Phi[m])
            rho = apply_spin_op(N, cb, Phi[m])
            gab[m, ip], gba[m, ip], lr[m, ip], _, _ = cross_green(H, lam, rho, n, omega, eta, E_m[m], tol)
    return gab, gba, lr
