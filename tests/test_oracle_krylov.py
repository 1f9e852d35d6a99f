"""Pins of the oracle's Krylov pieces against exact diagonalisation and closed forms.

Sec. II.B (shifted Krylov), Sec. III.B (Eq. dfilterP, Eq. filtered), Appendix A (Eq. tau).
"""
import math

import numpy as np
import pytest

from oracle import cluster, ed, filters, hamiltonian, lanczos, pipeline, rng, taylor
from seeded_inputs import SUPERCELLS

N = 8


@pytest.fixture(scope="module")
def sys8():
    cl = cluster.honeycomb(*SUPERCELLS[N])
    return cl, hamiltonian.Hamiltonian(cl, -1.0, 0.1), ed.ED(cl, -1.0, 0.1)


def _start(seed=11):
    v, _ = hamiltonian.normalize(rng.gaussian(seed, 0, N))
    return v


def test_resolvent_converges_to_ed(sys8):
    """T4: <v|(z - H)^{-1}|v> from n Lanczos steps approaches the ED value as n grows."""
    cl, H, E = sys8
    v = _start()
    z = np.linspace(-3, 3, 61) + 0.05j
    c = E.U.T @ v.view(np.complex128)
    exact = (np.abs(c) ** 2 / (z[:, None] - E.E[None, :])).sum(axis=1)
    errs = []
    for n in (32, 96, 400):
        a, b, _, _ = lanczos.lanczos(H, v, n)
        errs.append(np.abs(lanczos.resolvent_00(a, b, z) - exact).max() / np.abs(exact).max())
    assert errs[0] > errs[1] > 0 and errs[2] < 1e-10


def test_galerkin_residual_identity(sys8):
    """||(z - H) x_n - v|| equals beta_n |[(z - T_n)^{-1}]_{n-1,0}| for x_n = V_n (z - T_n)^{-1} e_1."""
    cl, H, E = sys8
    v = _start(3)
    n = 30
    a, b, W, nrm = lanczos.lanczos(H, v, n, store=True)
    V = W * lanczos.inverse_norms(nrm, b)[:, None]  # v_k = W[k] / beta_k
    Vc = V.view(np.complex128)  # [n, dim]
    assert np.abs(Vc.conj() @ Vc.T - np.eye(n)).max() < 1e-8  # orthonormal before ghosts appear
    T = lanczos.tridiag(a, b)
    Hd = E.H
    for z in (0.3 + 0.1j, -1.2 + 0.02j):
        y = np.linalg.solve(z * np.eye(n) - T, np.eye(n)[:, 0])
        x = Vc.T @ y
        r = z * x - Hd @ x - v.view(np.complex128)
        assert abs(np.linalg.norm(r) - lanczos.galerkin_residual(a, b, [z])[0]) < 1e-10


def test_breakdown_on_eigenvector():
    """At K = 0 the fully polarised state is an eigenvector: the sequence stops after one
    step and the resolvent is exactly 1/(z - E)."""
    cl = cluster.honeycomb(*SUPERCELLS[N])
    H = hamiltonian.Hamiltonian(cl, 0.0, 1.0)
    v = np.zeros(2 << N)
    v[0] = 1.0
    a, b, _, _ = lanczos.lanczos(H, v, 20)
    assert len(a) == 1 and b[0] == 0.0
    Eferro = 3 * N / 2 * 0.25
    assert a[0] == Eferro
    z = np.array([0.1 + 0.2j])
    assert abs(lanczos.resolvent_00(a, b, z)[0] - 1 / (z[0] - Eferro)) < 1e-15


@pytest.mark.parametrize("M", [2, 4, 16, 64])
def test_filter_closed_form(M):
    """The M-point contour sum of Eq. (dfilterP) on an eigenvalue equals 1/(1 + x^M)."""
    E = np.linspace(-4, 4, 2001)
    lit = filters.filter_literal(E, 0.37, 0.05, M)
    cf = filters.filter_closed_form(E, 0.37, 0.05, M)
    assert np.abs(lit.imag).max() < 1e-12
    assert np.abs(lit.real - cf).max() < 1e-12
    if M == 2:  # Lorentzian rho^2 / (rho^2 + (gamma - E)^2)
        assert np.abs(cf - 0.05**2 / (0.05**2 + (0.37 - E) ** 2)).max() < 1e-14


def test_odd_M_rejected():
    with pytest.raises(ValueError):
        filters.contour_nodes(0.1, 15)


def test_shell_coefficients_solve_tridiagonal(sys8):
    """The elimination solves (z_mj - T_n) y = e_1: compare c^m with dense solves."""
    cl, H, E = sys8
    a, b, _, _ = lanczos.lanczos(H, _start(4), 40)
    E_b, eps, L, M = -3.0, 0.1, 30, 8
    c = filters.shell_coefficients(a, b, 1.0, E_b, eps, L, M)
    T = lanczos.tridiag(a, b)
    n = len(a)
    Em = filters.energy_grid(E_b, eps, L)
    for m in (0, 7, 29):
        ref = np.zeros(n, dtype=complex)
        for j in range(1, M + 1):
            w = eps * np.exp(1j * 2 * math.pi * (j - 0.5) / M)
            ref += w * np.linalg.solve((Em[m] + w) * np.eye(n) - T, np.eye(n)[:, 0])
        ref /= M
        assert np.abs(c[m] - ref).max() < 1e-12 * max(1, np.abs(ref).max())


def test_filtered_states_match_ed(sys8):
    """T5: phi^m = V_n c^m approaches f_m(H) phi_beta (ED, closed-form filter)."""
    cl, H, E = sys8
    phi0 = _start(5)
    E_b, eps, L, M = -3.3, 0.15, 22, 8
    st = pipeline.typical_state(H, phi0, 0.0, E_b, eps, L, M, 500)
    d = E.U.T @ phi0.view(np.complex128)
    for m in range(L):
        f = filters.filter_closed_form(E.E, st.E_m[m], eps, M)
        ref = E.U @ (f * d)
        got = st.Phi[m].view(np.complex128)
        assert np.abs(got - ref).max() < 1e-9
        assert abs(st.n_m[m] - np.sum(np.abs(f * d) ** 2)) < 1e-9


def test_regenerated_shells_match_ed_and_stored(sys8):
    """Pass 2 by regeneration (pipeline.typical_shells: the twin run again, each vector
    added into the chosen shells as it is formed) gives f_m(H) phi_beta (ED, closed-form
    filter) for those shells, the same filter coefficients, and bit for bit the shells of
    the stored-vector route."""
    cl, H, E = sys8
    phi0 = _start(6)
    E_b, eps, L, M, beta = -3.3, 0.15, 22, 8, 1.0
    shells = [2, 11, 21]
    ln, al, be, nrm, coef, Phi, n_m, E_m = pipeline.typical_shells(H, phi0, beta, E_b, eps, L, M, 500, shells)
    st = pipeline.typical_state(H, phi0, beta, E_b, eps, L, M, 500)
    assert np.array_equal(al, st.alpha) and np.array_equal(coef, st.coef) and ln == st.log_norm
    ex = E.expm_half(beta, phi0.view(np.complex128) / np.linalg.norm(phi0))
    d = E.U.T @ (ex / np.linalg.norm(ex))
    for i, m in enumerate(shells):
        assert np.array_equal(Phi[i], st.Phi[m]) and n_m[i] == st.n_m[m]
        f = filters.filter_closed_form(E.E, E_m[m], eps, M)
        assert np.abs(Phi[i].view(np.complex128) - E.U @ (f * d)).max() < 1e-9


@pytest.mark.parametrize("beta", [0.5, 10.0, 100.0])
def test_taylor_matches_ed(sys8, beta):
    """Eq. (tau) via Appendix A: exp(log_norm) phi_beta_hat = e^{-beta H/2} phi_0."""
    cl, H, E = sys8
    phi0 = _start(6)
    phib, log_norm = taylor.canonical_state(H, phi0, beta)
    ex = E.expm_half(beta, phi0.view(np.complex128))
    lex = math.log(np.linalg.norm(ex))
    assert abs(log_norm - lex) < 1e-12 * max(1.0, abs(lex))
    assert np.abs(phib.view(np.complex128) - ex / np.linalg.norm(ex)).max() < 1e-12


def test_taylor_split_plan():
    """M_d from e^X / sqrt(2 pi X) = Lambda; beta = 0 needs no factors."""
    X = taylor.x_of_lambda()
    assert abs(math.exp(X) / math.sqrt(2 * math.pi * X) - taylor.LAMBDA) < 1e-6 * taylor.LAMBDA
    assert taylor.split_plan(8, 0.0, 3.3)[0] == 0
    Md, c, K, ell = taylor.split_plan(8, 100.0, 3.3)
    assert Md == math.ceil(100.0 * 3.3 / X) and K > c * 2 * 3.3 / 8


def test_auto_window_from_ritz_extremes(sys8):
    """The automatic shell window spans the extreme eigenvalues of H (ED) plus the margin
    once the Lanczos run has converged its extreme Ritz values; with few steps the Ritz
    extremes lie inside the spectrum (Cauchy interlacing)."""
    cl, H, E = sys8
    v = _start(8)
    a, b, _, _ = lanczos.lanczos(H, v, 120)
    E_b, eps = filters.auto_window(a, b, 16, 0.1)
    assert abs(E_b - (E.E[0] - 0.1)) < 1e-10
    assert abs(E_b + 2 * 16 * eps - (E.E[-1] + 0.1)) < 1e-10
    a, b, _, _ = lanczos.lanczos(H, v, 5)
    E_b5, eps5 = filters.auto_window(a, b, 16, 0.0)
    assert E_b5 > E.E[0] and E_b5 + 32 * eps5 < E.E[-1]


@pytest.mark.parametrize("tol", [1e-2, 1e-4, 1e-7])
def test_green_truncation_bound(sys8, tol):
    """Residual-controlled truncation: k is the first step whose residuals are all <= tol,
    and the truncated Green's function is within ||chi||^2 tol / eta of the exact resolvent
    (|<chi|(z-H)^{-1} r>| <= ||chi|| ||r|| / Im z)."""
    from oracle import green
    cl, H, E = sys8
    chi = rng.gaussian(21, 0, N) * 0.3
    c = E.U.T @ chi.view(np.complex128)
    nrm2 = float(np.sum(np.abs(c) ** 2))
    omega, eta = np.linspace(-3, 3, 41), 0.1
    a, b, _, _ = lanczos.lanczos(H, chi, 200)
    z = omega + 1j * eta
    k = lanczos.truncation_step(a, b, z, tol)
    assert lanczos.galerkin_residual(a[:k], b[:k], z).max() <= tol
    assert k == 1 or lanczos.galerkin_residual(a[: k - 1], b[: k - 1], z).max() > tol
    g, _, at, _ = green.green_sequence(H, chi, 200, omega, eta, 0.0, tol)
    assert len(at) == k
    exact = (np.abs(c) ** 2 / (z[:, None] - E.E[None, :])).sum(axis=1)
    assert np.abs(g - exact).max() <= nrm2 * tol / eta * (1 + 1e-9)


def test_filter_truncation_bound(sys8):
    """Filter truncation, each filter operator on its own (Sec. V): all M contour shifts of
    shell m converged at its step k_m, so each filtered state is within tol / sin(pi/M)
    of f_m(H) phi (|Im z_mj| >= eps sin(pi/M))."""
    cl, H, E = sys8
    phi0 = _start(9)
    E_b, eps, L, M, tol = -3.3, 0.15, 22, 8, 1e-5
    full = pipeline.typical_state(H, phi0, 0.0, E_b, eps, L, M, 400)
    st = pipeline.typical_state(H, phi0, 0.0, E_b, eps, L, M, 400, tol=tol)
    assert 1 < len(st.alpha) < len(full.alpha)
    # each filter stops on its own: outer shells need fewer steps than the sequence ran
    wr, wi = filters.contour_nodes(eps, M)
    k_m = [lanczos.truncation_step(full.alpha, full.beta, st.E_m[m] + wr + 1j * wi, tol) for m in range(L)]
    assert max(k_m) == len(st.alpha) and min(k_m) < max(k_m)
    for m in range(L):
        assert np.all(st.coef[m, k_m[m]:] == 0) and st.coef[m, k_m[m] - 1] != 0
    d = E.U.T @ phi0.view(np.complex128)
    for m in range(L):
        ref = E.U @ (filters.filter_closed_form(E.E, st.E_m[m], eps, M) * d)
        assert np.linalg.norm(st.Phi[m].view(np.complex128) - ref) <= tol / math.sin(math.pi / M) + 1e-12


def _bicg(Hd, b, z, n):
    """Plain BiCG on (z - H) x = b with the shadow residual started at b (textbook
    recurrences, dense H): the iterates x_1..x_n."""
    A = z * np.eye(Hd.shape[0]) - Hd
    x = np.zeros_like(b)
    r, rt = b.copy(), b.copy()
    p, pt = r.copy(), rt.copy()
    out = []
    for _ in range(n):
        Ap = A @ p
        rho = np.vdot(rt, r)
        alpha = rho / np.vdot(pt, Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        rt = rt - np.conj(alpha) * (A.conj().T @ pt)
        beta = np.vdot(rt, r) / rho
        p = r + beta * p
        pt = rt + np.conj(beta) * pt
        out.append(x.copy())
    return out


def test_bicg_with_rhs_shadow_is_lanczos_galerkin(sys8):
    """Sec. II.B / reading of the filter and Green's solver: BiCG on (z - H) x = b with the
    shadow vector b (H Hermitian) produces, step by step, the Lanczos-Galerkin iterate
    ||b|| V_k (z - T_k)^{-1} e_1, so the shifted BiCG of the paper and one Lanczos
    sequence give the same approximations for every shift."""
    cl, H, E = sys8
    b = _start(5)
    n = 20
    a, be, W, nrm = lanczos.lanczos(H, b, n, store=True)
    V = (W * lanczos.inverse_norms(nrm, be)[:, None]).view(np.complex128)
    bc = b.view(np.complex128)
    for z in (0.4 + 0.15j, -2.0 + 0.05j):
        xs = _bicg(E.H, bc, z, n)
        for k in (1, 5, 12, 20):
            T = lanczos.tridiag(a[:k], be[:k])
            y = np.linalg.solve(z * np.eye(k) - T, np.eye(k)[:, 0]) * nrm
            xg = V[:k].T @ y
            assert np.linalg.norm(xs[k - 1] - xg) <= 1e-9 * np.linalg.norm(xg), (z, k)


def test_cg_step_dependence_of_filter_residuals():
    """Sec. V (CG-step study): the largest residual 2-norm over a filter's M contour shifts
    falls with the step count, and reaching 1e-4 takes more steps when the contour comes
    closer to the real axis (larger M, smaller eps: min |Im z| = eps sin(pi/M))."""
    N12 = 12
    cl = cluster.honeycomb(*SUPERCELLS[N12])
    H = hamiltonian.Hamiltonian(cl, -1.0, 0.1)
    v, _ = hamiltonian.normalize(rng.gaussian(8, 0, N12))
    a, b, _, _ = lanczos.lanczos(H, v, 200)
    Em = -1.0

    def steps(eps, M):
        wr, wi = filters.contour_nodes(eps, M)
        hist = lanczos.residual_history(a, b, Em + wr + 1j * wi)
        assert hist[-1] < 1e-4 and hist[9] > 10 * hist[-1]
        return int(np.argmax(hist <= 1e-4)) + 1

    k4 = steps(0.5, 4)
    assert k4 < steps(0.5, 8) < steps(0.3, 8)
    # the history is the per-step maximum the truncation rule scans
    wr, wi = filters.contour_nodes(0.5, 4)
    z = Em + wr + 1j * wi
    assert lanczos.truncation_step(a, b, z, 1e-4) == k4
