"""Pins of the plain-form Lanczos recurrence (Sec. II.B as the textbook writes it:
v_{k+1} = w / beta_{k+1}) and of its agreement with the arithmetic-contract twin
(the carried-scale form the device follows).

The plain form shares nothing with the twin but the matrix-free H v, so these pins
check the twin's recurrence against an independent restatement, and both against
exact diagonalisation.
"""
import numpy as np
import pytest

from oracle import cluster, ed, filters, green, hamiltonian, lanczos, pipeline, rng
from seeded_inputs import SUPERCELLS

N = 8


@pytest.fixture(scope="module")
def sys8():
    cl = cluster.honeycomb(*SUPERCELLS[N])
    return cl, hamiltonian.Hamiltonian(cl, -1.0, 0.1), ed.ED(cl, -1.0, 0.1)


def _start(seed):
    v, _ = hamiltonian.normalize(rng.gaussian(seed, 0, N))
    return v


def test_lanczos_relation_and_orthonormality(sys8):
    """H V_n = V_n T_n + beta_n v_n e_{n-1}^T with V_n orthonormal, checked with the dense
    Hamiltonian (an independent assembly): a dropped term, a wrong sign or an index shift
    in the recurrence breaks the relation."""
    cl, H, E = sys8
    n = 24
    a, b, V, nrm = lanczos.lanczos_plain(H, _start(21), n + 1, store=True)
    Vn = V[:n].T  # [dim, n] columns v_0..v_{n-1}
    assert np.abs(Vn.conj().T @ Vn - np.eye(n)).max() < 1e-12
    T = lanczos.tridiag(a[:n], b[:n])
    R = E.H @ Vn - Vn @ T
    R[:, n - 1] -= b[n - 1] * V[n]
    assert np.abs(R).max() < 1e-12
    assert abs(nrm - 1.0) < 1e-14


def test_first_coefficients_are_moments(sys8):
    """alpha_0 = <v_0|H|v_0> and beta_1^2 = ||H v_0||^2 - alpha_0^2 (closed forms of the
    first two moments, dense H)."""
    cl, H, E = sys8
    v = _start(22).view(np.complex128)
    a, b, _, _ = lanczos.lanczos_plain(H, v.view(np.float64), 3)
    hv = E.H @ v
    m1 = np.vdot(v, hv).real
    m2 = np.vdot(hv, hv).real
    assert abs(a[0] - m1) < 1e-13
    assert abs(b[0] ** 2 - (m2 - m1 * m1)) < 1e-12


def test_invariant_subspace_of_three_eigenvectors(sys8):
    """A start vector in the span of three eigenvectors: the recurrence stops after exactly
    three steps and T_3 has exactly those three eigenvalues."""
    cl, H, E = sys8
    idx = [0, 57, 200]
    v = (E.U[:, idx] @ np.array([0.6, 0.3 - 0.5j, 0.55j])).astype(np.complex128)
    a, b, _, _ = lanczos.lanczos_plain(H, v.view(np.float64).copy(), 10)
    assert len(a) == 3
    th = np.linalg.eigvalsh(lanczos.tridiag(a, b))
    assert np.abs(np.sort(th) - np.sort(E.E[idx])).max() < 1e-12


def test_breakdown_on_eigenvector_plain():
    """At K = 0 the fully polarised state is an eigenvector: one step, alpha_0 = 3N/8."""
    cl = cluster.honeycomb(*SUPERCELLS[N])
    H = hamiltonian.Hamiltonian(cl, 0.0, 1.0)
    v = np.zeros(2 << N)
    v[0] = 1.0
    a, b, _, _ = lanczos.lanczos_plain(H, v, 20)
    assert len(a) == 1 and b[0] == 0.0 and a[0] == 3 * N / 8


def test_plain_matches_twin_before_loss_of_orthogonality(sys8):
    """The twin (carried scale, contract arithmetic) and the plain form agree to 1e-13
    relative over the first steps, where no Ritz value has converged yet."""
    cl, H, E = sys8
    v = _start(23)
    a1, b1, _, n1 = lanczos.lanczos_plain(H, v, 16)
    a2, b2, _, n2 = lanczos.lanczos(H, v, 16)
    assert abs(n1 - n2) <= 1e-15
    scale = np.abs(a1).max()
    assert np.abs(a1 - a2).max() <= 1e-13 * scale
    assert np.abs(b1 - b2).max() <= 1e-13 * np.abs(b1).max()


def test_plain_resolvent_converges_to_ed(sys8):
    """<chi|(z - H)^{-1}|chi> from the plain form reaches the ED value (1e-10 at n = 400),
    as does the twin; on converged shifts the two agree to 1e-10."""
    cl, H, E = sys8
    chi = (1.7 * _start(24)).copy()
    omega = np.linspace(-3, 3, 61)
    eta = 0.05
    c = E.U.T @ chi.view(np.complex128)
    z = omega + 1j * eta
    exact = (np.abs(c) ** 2 / (z[:, None] - E.E[None, :])).sum(axis=1)
    gp, rp, _, _ = green.green_sequence_plain(H, chi, 400, omega, eta, 0.0)
    gt, _, _, _ = green.green_sequence(H, chi, 400, omega, eta, 0.0)
    scale = np.abs(exact).max()
    assert np.abs(gp - exact).max() <= 1e-10 * scale
    assert np.abs(gt - exact).max() <= 1e-10 * scale
    assert rp.max() < 1e-10


def test_plain_filtered_states_match_ed(sys8):
    """phi^m = V_n c^m from the plain form approaches f_m(H) phi (ED, closed-form filter)."""
    cl, H, E = sys8
    phi0 = _start(25)
    E_b, eps, L, M = -3.3, 0.15, 22, 8
    Phi, n_m, _, _, _ = pipeline.typical_state_plain(H, phi0, 0.0, E_b, eps, L, M, 500)
    d = E.U.T @ phi0.view(np.complex128)
    Em = filters.energy_grid(E_b, eps, L)
    for m in range(L):
        f = filters.filter_closed_form(E.E, Em[m], eps, M)
        assert np.abs(Phi[m] - E.U @ (f * d)).max() < 1e-9
        assert abs(n_m[m] - np.sum(np.abs(f * d) ** 2)) < 1e-9
