"""The FTKw method end to end, step by step in the paper's order -- oracle side.

Test infrastructure only (see ``oracle/__init__``).

Eq. (tau) -> Eq. (filtered) -> Eqs. (GAB_TPS)/(SQomega_TPS) -> Eq. (FRW1):
  1. phi_0: normalised complex Gaussian vector (Sec. II.A);
  2. phi_beta = e^{-beta H/2} phi_0 with its log-norm (Appendix A, taylor.py);
  3. Lanczos basis of phi_beta, shell coefficients, phi^m = V_n c^m and
     n_m = <phi^m|phi^m> (Sec. III.B, filters.py);
  4. g_m^{alpha,Q}(omega) for every shell (Sec. III.C, green.py);
  5. reweighting to every target temperature (Sec. III.D, reweight.py).
"""
from dataclasses import dataclass

import numpy as np

from . import filters, green, rng, taylor
from ._native import ptr, lib as _lib
from .hamiltonian import Hamiltonian, normalize
from .lanczos import inverse_norms, lanczos, lanczos_combine, lanczos_plain, truncation_step


@dataclass
class States:
    """Shell data of one (sample, anchor): normalised-phi_beta quantities."""
    log_norm: float  # log ||e^{-beta H/2} phi_0||
    nrm: float  # norm of the stored phi_beta (1 up to rounding)
    alpha: np.ndarray
    beta: np.ndarray
    coef: np.ndarray  # [L, n] complex c^m_k (coefficients of the normalised v_k)
    Phi: np.ndarray  # [L, 2 dim] interleaved phi^m
    n_m: np.ndarray  # [L]
    E_m: np.ndarray  # [L]
    h1: np.ndarray = None  # [L] <phi^m|H|phi^m> (when asked for)
    h2: np.ndarray = None  # [L] <H phi^m|H phi^m>


def start_vector(N, seed, sample, gaussian=None):
    """phi_0 = g / ||g||; g from the counter-based generator unless given."""
    if gaussian is None:
        gaussian = rng.gaussian(seed, sample, N)
    v, _ = normalize(np.ascontiguousarray(gaussian, dtype=np.float64))
    return v


def typical_state(H, phi0, beta, E_b, eps, L, M, n_steps, margin=None, tol=0.0, moments=False):
    """Steps 2-3 for one start vector and one anchor beta.  With E_b = eps = None the
    window comes from this vector's own Ritz extremes (filters.auto_window).  tol > 0
    truncates each filter operator separately, as the paper solves each filter's M
    contour shifts on its own (Sec. V): shell m takes T_{k_m} for the first k_m at
    which all of its M shifts have converged, and the sequence runs to max k_m."""
    phib, log_norm = taylor.canonical_state(H, phi0, beta)
    alpha, bet, W, nrm = lanczos(H, phib, n_steps, store=True)
    if E_b is None:
        E_b, eps = filters.auto_window(alpha, bet, L, margin)
    if tol > 0:
        wr, wi = filters.contour_nodes(eps, M)
        Em = filters.energy_grid(E_b, eps, L)
        k_m = np.array([truncation_step(alpha, bet, Em[m] + wr + 1j * wi, tol) for m in range(L)])
        k = int(k_m.max())
        alpha, bet, W = alpha[:k], bet[:k], W[:k]
        coef = filters.shell_coefficients_per_shell(alpha, bet, nrm, E_b, eps, L, M, k_m)
    else:
        coef = filters.shell_coefficients(alpha, bet, nrm, E_b, eps, L, M)
    n = len(alpha)
    # phi^m = sum_k c^m_k v_k = sum_k (c^m_k inv_k) W[k]
    inv = inverse_norms(nrm, bet)
    d = np.empty((L, n), dtype=np.complex128)
    d.real = coef.real * inv[None, :]
    d.imag = coef.imag * inv[None, :]
    Phi = np.zeros((L, W.shape[1]))
    cf = np.ascontiguousarray(d).view(np.float64)  # [L, 2n]
    _lib().orc_combine(H.N, n, L, ptr(np.ascontiguousarray(W)), ptr(cf), ptr(Phi))
    from .hamiltonian import dot_re
    n_m = np.array([dot_re(Phi[m], Phi[m]) for m in range(L)])
    E_m = filters.energy_grid(E_b, eps, L)
    h1 = h2 = None
    if moments:  # <phi^m|H|phi^m> and ||H phi^m||^2, for the thermodynamics
        HP = [H.apply(Phi[m]) for m in range(L)]
        h1 = np.array([dot_re(Phi[m], HP[m]) for m in range(L)])
        h2 = np.array([dot_re(HP[m], HP[m]) for m in range(L)])
    return States(log_norm, nrm, alpha, bet, coef, Phi, n_m, E_m, h1, h2)


def filter_pass1(H, phi0, beta, n_steps):
    """The canonical state and pass 1 of the filter: (log_norm, phi_beta, alpha, beta,
    norm) with T_n of phi_beta."""
    phib, log_norm = taylor.canonical_state(H, phi0, beta)
    alpha, bet, _, nrm = lanczos(H, phib, n_steps)
    return log_norm, phib, alpha, bet, nrm


def regenerate_shells(H, phib, alpha, bet, nrm, coef, shells):
    """Pass 2 for the listed shells only: the Lanczos twin run again from phi_beta, each
    regenerated vector added into those shells as it is formed (Sec. III.B).  Returns
    (Phi [len(shells), 2 dim], n_m of those shells)."""
    from .hamiltonian import dot_re
    inv = inverse_norms(nrm, bet)
    d = np.empty((len(shells), len(alpha)), dtype=np.complex128)
    d.real = coef[list(shells)].real * inv[None, :]
    d.imag = coef[list(shells)].imag * inv[None, :]
    Phi, a2, b2, _ = lanczos_combine(H, phib, len(alpha), d)
    assert np.array_equal(a2, alpha) and np.array_equal(b2, bet)  # pass 2 regenerates pass 1 exactly
    return Phi, np.array([dot_re(Phi[i], Phi[i]) for i in range(len(shells))])


def typical_shells(H, phi0, beta, E_b, eps, L, M, n_steps, shells):
    """typical_state for the listed shells only, in memory for a few vectors: pass 1 of
    the filter gives T_n, the shell coefficients of all L shells follow from it, and
    pass 2 regenerates the Lanczos vectors into the listed shells.  Returns (log_norm,
    alpha, beta, norm, coef [L, n], Phi [len(shells), 2 dim], n_m of the listed
    shells, E_m [L])."""
    log_norm, phib, alpha, bet, nrm = filter_pass1(H, phi0, beta, n_steps)
    coef = filters.shell_coefficients(alpha, bet, nrm, E_b, eps, L, M)
    Phi, n_m = regenerate_shells(H, phib, alpha, bet, nrm, coef, shells)
    return log_norm, alpha, bet, nrm, coef, Phi, n_m, filters.energy_grid(E_b, eps, L)


def typical_state_plain(H, phi0, beta, E_b, eps, L, M, n_steps):
    """Steps 2-3 with the plain-form Lanczos recurrence (lanczos.lanczos_plain): the
    normalised basis vectors v_k are kept and phi^m = sum_k c^m_k v_k is one NumPy matrix
    product.  Returns (Phi [L, dim] complex, n_m [L], alpha, beta, norm of phi_beta)."""
    phib, _ = taylor.canonical_state(H, phi0, beta)
    alpha, bet, V, nrm = lanczos_plain(H, phib, n_steps, store=True)
    coef = filters.shell_coefficients(alpha, bet, nrm, E_b, eps, L, M)
    Phi = coef @ V
    n_m = np.einsum("mx,mx->m", Phi.conj(), Phi).real
    return Phi, n_m, alpha, bet, nrm


def run(cluster, K, J, *, seed, n_samples, betas, E_b, eps, L, M, n_filter, n_green,
        qs, alphas, omega, eta, temps, gaussians=None, n_bins=8, margin=0.1, first_sample=0, filter_tol=0.0,
        green_tol=0.0):
    """Full method.  gaussians[s] (optional) replaces the generator's draw for sample s.
    E_b = eps = None: each anchor's window is taken from sample 0's Ritz extremes
    (filters.auto_window with the given margin) and shared by all samples.

    Returns dict with S [Q, T', W], stderr, P, and the raw per-(s, a) data."""
    H = Hamiltonian(cluster, K, J)
    A = len(betas)
    if E_b is None:
        phi0 = start_vector(H.N, seed, first_sample, None if gaussians is None else gaussians[0])
        E_b, eps = np.zeros(A), np.zeros(A)
        for a, b in enumerate(betas):
            phib, _ = taylor.canonical_state(H, phi0, float(b))
            al, be, _, _ = lanczos(H, phib, n_filter)
            E_b[a], eps[a] = filters.auto_window(al, be, L, margin)
    E_b = np.broadcast_to(np.asarray(E_b, dtype=np.float64), (A,))
    eps = np.broadcast_to(np.asarray(eps, dtype=np.float64), (A,))
    W = len(omega)
    log_norm = np.zeros((n_samples, A))
    n_m = np.zeros((n_samples, A, L))
    E_m = np.zeros((A, L))
    graw = np.zeros((n_samples, A, L, len(alphas), len(qs), W), dtype=np.complex128)
    resid = np.zeros((n_samples, A, L, len(alphas), len(qs)))
    for s in range(n_samples):
        phi0 = start_vector(H.N, seed, first_sample + s, None if gaussians is None else gaussians[s])
        for a, b in enumerate(betas):
            st = typical_state(H, phi0, float(b), float(E_b[a]), float(eps[a]), L, M, n_filter, tol=filter_tol)
            log_norm[s, a] = st.log_norm
            n_m[s, a] = st.n_m
            E_m[a] = st.E_m
            g, r = green.shell_spectra(H, st.Phi, st.E_m, qs, alphas, n_green, omega, eta, green_tol)
            graw[s, a] = g
            resid[s, a] = r
    from . import reweight
    S, err, P = reweight.reweight(betas, E_m, eps, log_norm, n_m, graw.sum(axis=3), temps, n_bins)
    return dict(S=S, stderr=err, P=P, log_norm=log_norm, n_m=n_m, E_m=E_m, eps=np.array(eps), g=graw,
                resid=resid)
