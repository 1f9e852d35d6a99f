"""Pins of the oracle's shifted COCG (Sec. II.B with the shadow vector conj(rho); seed
switching of Appendix C): the textbook algorithm with vectors against exact
diagonalisation and its own residuals, and the device-form twin (complex-symmetric
Lanczos + per-shift scalar recurrences) against the textbook form and against the
Hermitian Lanczos twin in the case where the two coincide (a real start vector)."""
import numpy as np
import pytest

from oracle import cluster, cocg, ed, green, hamiltonian, lanczos, rng
from seeded_inputs import SUPERCELLS

N = 8


@pytest.fixture(scope="module")
def sys8():
    cl = cluster.honeycomb(*SUPERCELLS[N])
    return cl, hamiltonian.Hamiltonian(cl, -1.0, 0.1), ed.ED(cl, -1.0, 0.1)


def _exact(E, rho, lam, z):
    cr = E.U.T @ rho.view(np.complex128)
    cl_ = E.U.T @ lam.view(np.complex128)
    return ((np.conj(cl_) * cr)[None, :] / (z[:, None] - E.E[None, :])).sum(axis=1)


def test_textbook_cocg_solves_every_shift(sys8):
    """At convergence every x_j solves (z_j - H) x_j = rho (dense H) and <lam|x_j> is the
    ED resolvent; the seed was switched on the way."""
    cl, H, E = sys8
    rho = rng.gaussian(31, 0, N)
    lam = rng.gaussian(32, 0, N)
    z = np.linspace(-3, 3, 13) + 0.1j
    G, X, res, seeds = cocg.shifted_cocg(H, rho, z, 400, lam=lam)
    b = rho.view(np.complex128)
    for j in range(len(z)):
        assert np.linalg.norm(z[j] * X[j] - E.H @ X[j] - b) <= 1e-10 * np.linalg.norm(b)
    ex = _exact(E, rho, lam, z)
    assert np.abs(G - ex).max() <= 1e-10 * np.abs(ex).max()
    assert res.max() <= 1e-10 * np.linalg.norm(b)
    assert len(set(seeds)) >= 2


def test_textbook_tracked_residual_is_the_true_residual(sys8):
    """Before convergence the residual the recurrence tracks (||r_seed|| / |pi_j|) equals
    ||rho - (z_j - H) x_j|| computed with the dense H."""
    cl, H, E = sys8
    rho = rng.gaussian(33, 0, N)
    z = np.linspace(-3, 3, 7) + 0.2j
    G, X, res, _ = cocg.shifted_cocg(H, rho, z, 12)
    b = rho.view(np.complex128)
    true = np.array([np.linalg.norm(b - (z[j] * X[j] - E.H @ X[j])) for j in range(len(z))])
    assert np.all(np.abs(res - true) <= 1e-8 * true + 1e-12 * np.linalg.norm(b))
    assert true.max() > 1.0  # far from converged at some shifts


def test_real_rhs_cocg_is_lanczos_galerkin(sys8):
    """For a real right-hand side the bilinear form is the inner product: shifted COCG
    gives the Lanczos-Galerkin values, and the complex-symmetric Lanczos twin reproduces
    the Hermitian twin's coefficients bit for bit."""
    cl, H, E = sys8
    rho = np.zeros(2 << N)
    rho[0::2] = rng.gaussian(34, 0, N)[: 1 << N]
    z = np.linspace(-3, 3, 11) + 0.1j
    G, _, _, _ = cocg.shifted_cocg(H, rho, z, 20)
    g, _, al, be = green.green_sequence(H, rho, 20, z.real, 0.1, 0.0)
    assert np.abs(G - g).max() <= 1e-9 * np.abs(g).max()
    a, b, c, hn, d0, steps = cocg.lanczos_bilinear(H, rho, 20)
    assert steps == 20
    assert np.array_equal(a.real, al) and not a.imag.any()
    assert np.array_equal(b.real, be) and not b.imag.any()


def test_complex_rhs_cocg_differs_at_finite_n_and_converges(sys8):
    """For a complex right-hand side COCG and Lanczos-Galerkin are different
    approximations at finite n (both valid) and meet at the ED resolvent."""
    cl, H, E = sys8
    rho = rng.gaussian(35, 0, N)
    z = np.linspace(-3, 3, 11) + 0.1j
    ex = _exact(E, rho, rho, z)
    Gc, _, _, _ = cocg.shifted_cocg(H, rho, z, 15)
    gl, _, _, _ = green.green_sequence(H, rho, 15, z.real, 0.1, 0.0)
    assert np.abs(Gc - gl).max() > 1e-4 * np.abs(ex).max()
    Gc, _, _, _ = cocg.shifted_cocg(H, rho, z, 400)
    gl, _, _, _ = green.green_sequence(H, rho, 400, z.real, 0.1, 0.0)
    assert np.abs(Gc - ex).max() <= 1e-10 * np.abs(ex).max()
    assert np.abs(gl - ex).max() <= 1e-10 * np.abs(ex).max()


def test_seed_choice_does_not_change_the_converged_result(sys8):
    cl, H, E = sys8
    rho = rng.gaussian(36, 0, N)
    z = np.linspace(-3, 3, 9) + 0.05j
    G0, _, _, _ = cocg.shifted_cocg(H, rho, z, 500, seed=0)
    G8, _, _, s8 = cocg.shifted_cocg(H, rho, z, 500, seed=8)
    assert s8[0] == 8
    assert np.abs(G0 - G8).max() <= 1e-10 * np.abs(G0).max()


@pytest.mark.parametrize("n", [6, 14, 400])
def test_device_form_matches_textbook(sys8, n):
    """The twin the device follows (complex-symmetric Lanczos basis, per-shift scalar
    recurrences, seed switching on scalars) against the textbook vectors: values and
    residual 2-norms, before convergence and converged (then also the ED resolvent)."""
    cl, H, E = sys8
    rho = rng.gaussian(37, 0, N)
    lam = rng.gaussian(38, 0, N)
    z = np.linspace(-3, 3, 13) + 0.1j
    G, _, res, seeds = cocg.shifted_cocg(H, rho, z, n, lam=lam)
    a, b, c, hn, d0, steps = cocg.lanczos_bilinear(H, rho, n, lam=lam)
    g2, res2, seeds2 = cocg.cocg_from_bilinear(a, b, c, hn, d0, z)
    assert steps == n
    assert np.abs(g2 - G).max() <= 1e-9 * np.abs(G).max()
    if n < 100:
        assert np.abs(res2 - res).max() <= 1e-8 * res.max()
        assert seeds2[:-1] == seeds
    else:
        ex = _exact(E, rho, lam, z)
        assert np.abs(g2 - ex).max() <= 1e-10 * np.abs(ex).max()
        assert res2.max() <= 1e-10 * np.linalg.norm(rho)


def test_bilinear_breakdown_on_eigenvector():
    """K = 0, fully polarised start: one step, a_0 = 3N/8, b_1 = 0."""
    cl = cluster.honeycomb(*SUPERCELLS[N])
    H = hamiltonian.Hamiltonian(cl, 0.0, 1.0)
    v = np.zeros(2 << N)
    v[0], v[1] = 0.6, 0.8
    a, b, c, hn, d0, steps = cocg.lanczos_bilinear(H, v, 10)
    assert steps == 1 and abs(a[0] - 3 * N / 8) <= 1e-14 and abs(b[0]) <= 1e-14


def test_pair_cocg_matches_ed(sys8):
    """G_AB and G_BA by two shifted COCG runs (each projected on the other operator's
    vector) equal the exact <lam|(z - H)^{-1}|rho> and <rho|(z - H)^{-1}|lam> at
    convergence; <lam|rho> = c_0 delta_0."""
    cl, H, E = sys8
    lam = rng.gaussian(41, 0, N)
    rho = rng.gaussian(42, 0, N)
    omega = np.linspace(-3, 3, 25)
    gab, gba, ov, res, _ = green.cross_green_cocg(H, lam, rho, 400, omega, 0.1, 0.3)
    z = omega + 0.3 + 0.1j
    ab = _exact(E, rho, lam, z)
    ba = _exact(E, lam, rho, z)
    assert np.abs(gab - ab).max() <= 1e-10 * np.abs(ab).max()
    assert np.abs(gba - ba).max() <= 1e-10 * np.abs(ba).max()
    assert abs(ov - np.vdot(lam.view(np.complex128), rho.view(np.complex128))) <= 1e-12 * np.linalg.norm(lam) * np.linalg.norm(rho)
    assert res <= 1e-10 * max(np.linalg.norm(lam), np.linalg.norm(rho))


def test_converged_shifts_stop_and_tiny_rhs(sys8):
    """Past convergence the twin stops updating a shift (its residual is at most seed_tol
    ||rho||) and ends once every shift is converged, so 400 steps on a 256-state space
    stay finite: G equals the ED resolvent, and scaling lam and rho by 2^-64 (a shell of
    weight ~1e-38) scales G by exactly 2^-128 and changes no step."""
    cl, H, E = sys8
    lam = rng.gaussian(43, 0, N)
    rho = rng.gaussian(44, 0, N)
    omega = np.linspace(-3, 3, 25)
    z = omega + 0.3 + 0.1j
    s = 2.0 ** -64
    with np.errstate(all="raise"):
        gab, gba, ov, res, coefs = green.cross_green_cocg(H, lam, rho, 400, omega, 0.1, 0.3)
        gab_s, gba_s, ov_s, res_s, coefs_s = green.cross_green_cocg(H, lam * s, rho * s, 400, omega, 0.1, 0.3)
    assert len(coefs[0][0]) < 400 and len(coefs[1][0]) < 400  # ended on convergence
    ab = _exact(E, rho, lam, z)
    assert np.abs(gab - ab).max() <= 1e-10 * np.abs(ab).max()
    assert np.array_equal(gab_s, gab * s * s) and np.array_equal(gba_s, gba * s * s)
    assert ov_s == ov * s * s and res_s == res * s
    for k in range(2):
        assert len(coefs_s[k][0]) == len(coefs[k][0])
        assert np.array_equal(coefs_s[k][0], coefs[k][0]) and np.array_equal(coefs_s[k][2], coefs[k][2] * s)
