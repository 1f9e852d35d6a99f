"""Equi-energy Green's functions and the spectrum estimator (Sec. III.C, Sec. V) -- oracle side.

Test infrastructure only (see ``oracle/__init__``).

For each shell m, spin component alpha and momentum Q (Eq. SQomega_TPS):
    g_m(omega) = <phi^m| S^alpha_{-Q} (omega + i eta + E_m - H)^{-1} S^alpha_{+Q} |phi^m>.
With chi = S^alpha_{+Q} phi^m and S^alpha_{-Q} = (S^alpha_{+Q})^dagger this is
<chi|(z - H)^{-1}|chi>, and the n-step Galerkin value (lanczos.py) is
    g_m(omega) = ||chi||^2 [(z - T_n)^{-1}]_{00},   z = omega + i eta + E_m.
The vectors phi^m are kept unnormalised; the per-sample normalisation of
Eq. (GAB_TPS) cancels in the reweighted ratio (reweight.py).
"""
import math

import numpy as np

from .hamiltonian import apply_sq, dot_re
from .lanczos import galerkin_residual, lanczos, resolvent_00, truncation_step


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
