"""Lanczos basis and shifted Galerkin solves -- oracle side.

Test infrastructure only (see ``oracle/__init__``).

Sec. II.B solves (zeta - H) chi(zeta) = rho by shifted BiCG for many zeta at once,
relying on the shift invariance K_n(zeta - H, rho) = K_n(zeta' - H, rho).  For a
Hermitian H with the shadow vector taken equal to rho, the BiCG residuals are
proportional to the Hermitian Lanczos vectors, so the n-step iterate for every
shift is the Galerkin solution
    chi_n(zeta) = ||rho|| V_n (zeta - T_n)^{-1} e_1,
with T_n = tridiag(alpha_0..alpha_{n-1}; beta_1..beta_{n-1}).  The oracle builds
V_n and T_n by the plain Lanczos recurrence and evaluates (zeta - T_n)^{-1}
through the eigendecomposition of T_n (a library eigensolver); the GPU path uses a
different route (a per-shift continued-fraction recurrence), so agreement is a
real check.
"""
import ctypes

import numpy as np
import scipy.linalg

from . import _native
from ._native import ptr


def _cplx(v):
    """Interleaved float64 (re, im) -> complex128 view/copy."""
    return np.ascontiguousarray(v, dtype=np.float64).view(np.complex128)


def lanczos_plain(H, start, n, store=False, tol=None):
    """The Hermitian Lanczos recurrence behind the shifted solves of Sec. II.B, in the
    plain form of the textbook, with explicitly normalised basis vectors:

        v_0 = rho / ||rho||,  beta_0 = 0,  v_{-1} = 0
        w = H v_k - beta_k v_{k-1}
        alpha_k = Re <v_k|w>
        w = w - alpha_k v_k
        beta_{k+1} = ||w||,   v_{k+1} = w / beta_{k+1}

    Vector operations are NumPy complex128 arithmetic and H v is the oracle's matrix-free
    product; inner products are NumPy's (np.vdot).  Nothing here follows the device's
    arithmetic order, so after the Ritz values converge its coefficients drift away from
    any other implementation's; only converged quantities are comparable.

    Returns (alpha, beta, V, norm): alpha[k] = alpha_k, beta[k] = beta_{k+1}, norm =
    ||rho|| and, with store=True, V[k] = v_k (complex128 rows, k < steps).  The run stops
    early, after step k, when beta_{k+1} <= tol (default: the oracle Hamiltonian's
    breakdown threshold), i.e. when the Krylov space is invariant."""
    if tol is None:
        tol = H.breakdown_tol()
    rho = _cplx(start).copy()
    nrm = float(np.sqrt(np.vdot(rho, rho).real))
    v = rho / nrm
    v_prev = np.zeros_like(v)
    b = 0.0
    alpha, beta, V = [], [], []
    for _ in range(n):
        if store:
            V.append(v.copy())
        w = _cplx(H.apply(v.view(np.float64))) - b * v_prev
        a = float(np.vdot(v, w).real)
        w = w - a * v
        b_next = float(np.sqrt(np.vdot(w, w).real))
        alpha.append(a)
        beta.append(b_next)
        if b_next <= tol:
            break
        v_prev, v, b = v, w / b_next, b_next
    return np.array(alpha), np.array(beta), (np.array(V) if store else None), nrm


def lanczos(H, start, n, store=False):
    """n Lanczos steps from the start vector (normalised inside: v_0 = start/||start||),
    in the arithmetic-contract form shared with the device (the twin of
    ``lanczos_plain``: the same recurrence with the scale of v_k carried as a scalar).

    Returns (alpha, beta, W, norm) with alpha[k] = alpha_k, beta[k] = beta_{k+1}
    (beta[-1] is the residual coupling beta_n), norm = ||start|| and, when
    store=True, W[k] = w_{k-1}: the unnormalised vector with v_k = W[k] / ||W[k]||
    (W[0] = start, W[k] = beta_k v_k).  Fewer than n steps are returned if the
    Krylov space became invariant.  See ftk_oracle.c:orc_lanczos for the exact
    arithmetic.
    """
    start = np.ascontiguousarray(start, dtype=np.float64)
    alpha = np.zeros(n)
    beta = np.zeros(n)
    W = np.zeros((n, start.shape[0])) if store else None
    nrm = ctypes.c_double()
    steps = _native.lib().orc_lanczos(
        *H._args(), ptr(start), n, H.breakdown_tol(), ptr(alpha), ptr(beta), ptr(W) if store else None,
        ctypes.byref(nrm))
    alpha, beta = alpha[:steps], beta[:steps]
    if store:
        W = W[:steps]
    return alpha, beta, W, nrm.value


def lanczos_combine(H, start, n, D):
    """The twin of ``lanczos`` run again from start, adding each residual vector into the
    rows of D as it is formed: Phi[m] = sum_k D[m, k] W[k] (D [nm, n] complex, the
    scale inv_k folded in), with the operations of ftk_oracle.c:orc_combine, without
    storing the W[k].  Returns (Phi [nm, 2 dim], alpha, beta, norm)."""
    start = np.ascontiguousarray(start, dtype=np.float64)
    D = np.ascontiguousarray(D, dtype=np.complex128)
    nm = D.shape[0]
    assert D.shape[1] == n
    alpha, beta = np.zeros(n), np.zeros(n)
    Phi = np.zeros((nm, start.shape[0]))
    nrm = ctypes.c_double()
    steps = _native.lib().orc_lanczos_combine(
        *H._args(), ptr(start), n, H.breakdown_tol(), ptr(alpha), ptr(beta), ctypes.byref(nrm), nm,
        ptr(D.view(np.float64)), ptr(Phi))
    return Phi, alpha[:steps], beta[:steps], nrm.value


def inverse_norms(nrm, beta):
    """inv_k = 1/beta_k with beta_0 = ||start||: the scale of W[k] in v_k = W[k] * inv_k."""
    inv = np.empty(len(beta))
    inv[0] = 1.0 / nrm
    for k in range(1, len(beta)):
        inv[k] = 1.0 / beta[k - 1]
    return inv


def tridiag(alpha, beta):
    """Dense T_n from alpha_0..alpha_{n-1} and beta_1..beta_{n-1}."""
    n = len(alpha)
    T = np.diag(alpha).astype(np.float64)
    if n > 1:
        T += np.diag(beta[: n - 1], 1) + np.diag(beta[: n - 1], -1)
    return T


def ritz(alpha, beta):
    """Ritz values theta_k and first-row weights Q_{0k}, last-row Q_{n-1,k} of T_n."""
    n = len(alpha)
    if n == 1:
        return np.array(alpha, dtype=np.float64), np.ones(1), np.ones(1)
    theta, Q = scipy.linalg.eigh_tridiagonal(np.asarray(alpha), np.asarray(beta[: n - 1]), lapack_driver="stev")
    return theta, Q[0].copy(), Q[-1].copy()


def resolvent_00(alpha, beta, z):
    """[(z - T_n)^{-1}]_{00} for every z, via the Ritz decomposition."""
    theta, q0, _ = ritz(alpha, beta)
    z = np.asarray(z, dtype=np.complex128)
    return ((q0 * q0)[None, :] / (z[:, None] - theta[None, :])).sum(axis=1)


def galerkin_residual(alpha, beta, z):
    """||r_n(z)|| / ||rho|| = beta_n |[(z - T_n)^{-1}]_{n-1,0}| for the Galerkin solution."""
    theta, q0, ql = ritz(alpha, beta)
    z = np.asarray(z, dtype=np.complex128)
    e = ((q0 * ql)[None, :] / (z[:, None] - theta[None, :])).sum(axis=1)
    return beta[-1] * np.abs(e)


def truncation_step(alpha, beta, z, tol):
    """Smallest k in 1..n for which every shift z has Galerkin residual <= tol per unit
    right-hand side (the largest residual 2-norm over the shifts decides, Sec. V); n if
    none.  Evaluated from the Ritz decomposition of each T_k."""
    n = len(alpha)
    for k in range(1, n + 1):
        if galerkin_residual(alpha[:k], beta[:k], z).max() <= tol:
            return k
    return n


def residual_history(alpha, beta, z):
    """max over the shifts z of ||r_k(z)|| / ||rho|| for k = 1..n: the CG-step dependence of
    the largest residual 2-norm (Sec. V).  The shifted BiCG iterate with the shadow
    vector equal to the right-hand side is the Galerkin solution of K_k(H, rho), so its
    residuals are these."""
    n = len(alpha)
    return np.array([galerkin_residual(alpha[:k], beta[:k], z).max() for k in range(1, n + 1)])
