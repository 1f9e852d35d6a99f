"""Pins of the oracle's Green's functions for general operator pairs A != B.

Sec. III.B (G^AB of a resolvent between A|0> and B|0>), Eq. GAB_TPS (the same with
filtered typical states), Eq. chiAB (the canonical pair correlation), Eq. FRW1
(reweighting).  The oracle splits <lam|(z - H)^{-1}|rho> into four Lanczos-Galerkin
quadratic forms by the polarization identity; these tests pin it against dense Pauli
matrices, the exact resolvent from exact diagonalisation, the diagonal case and the
exact expectation of the estimator.
"""
import math

import numpy as np
import pytest

from oracle import cluster, ed, filters, green, hamiltonian, pipeline, reweight, rng
from seeded_inputs import SUPERCELLS

N = 8


@pytest.fixture(scope="module")
def sys8():
    cl = cluster.honeycomb(*SUPERCELLS[N])
    return cl, hamiltonian.Hamiltonian(cl, -1.0, 0.1), ed.ED(cl, -1.0, 0.1)


def _coef(seed, n):
    r = np.random.default_rng(seed)
    return r.normal(size=(n, 3)) + 1j * r.normal(size=(n, 3))


def _local_pair(n):
    """A = S^z_0 + 0.5 S^x_1, B = S^z_1 + (0.3 + 0.4i) S^x_0 + 0.2i S^z_0.  The pi rotations
    about the spin axes are symmetries of H, so correlations of different components
    vanish in the ensemble; the complex coefficients on equal components make the
    pair's spectral density complex."""
    a = np.zeros((n, 3), dtype=np.complex128)
    b = np.zeros((n, 3), dtype=np.complex128)
    a[0, 2], a[1, 0] = 1.0, 0.5
    b[1, 2], b[0, 0], b[0, 2] = 1.0, 0.3 + 0.4j, 0.2j
    return a, b


def test_spin_op_matches_pauli_matrices():
    """A v for random complex coefficients equals the dense operator built from Pauli
    matrices (bit 0 = up, S = sigma/2); a one-component column reproduces S^alpha_{+Q}."""
    n = 6
    cl = cluster.honeycomb(*SUPERCELLS[n])
    v = rng.gaussian(3, 0, n)
    vc = v.view(np.complex128)
    for seed in (1, 2):
        c = _coef(seed, n)
        w = hamiltonian.apply_spin_op(n, c, v).view(np.complex128)
        assert np.abs(w - ed.dense_spin_op(n, c) @ vc).max() <= 1e-14 * np.abs(vc).max() * np.abs(c).sum()
    for alpha in range(3):
        for _, qx, qy in cluster.allowed_momenta(cl)[:3]:
            c = hamiltonian.spin_op_q(cl, alpha, qx, qy)
            w = hamiltonian.apply_spin_op(n, c, v)
            ref = hamiltonian.apply_sq(cl, alpha, qx, qy, v)
            assert np.abs(w - ref).max() <= 1e-15 * np.abs(ref).max()


@pytest.mark.parametrize("pair", ["momentum", "local"])
def test_cross_green_matches_exact_resolvent(sys8, pair):
    """Run to exhaustion (256 steps on a 256-state space), the four polarized sequences
    give <lam|(z - H)^{-1}|rho> and <rho|(z - H)^{-1}|lam> of the exact eigen-decomposition,
    and <lam|rho> from the four norms."""
    cl, H, E = sys8
    phi, _ = hamiltonian.normalize(rng.gaussian(11, 0, N))
    if pair == "momentum":
        _, qx, qy = cluster.allowed_momenta(cl)[1]
        ca, cb = hamiltonian.spin_op_q(cl, 0, qx, qy), hamiltonian.spin_op_q(cl, 1, qx, qy)
    else:
        ca, cb = _local_pair(N)
    lam = hamiltonian.apply_spin_op(N, ca, phi)
    rho = hamiltonian.apply_spin_op(N, cb, phi)
    omega = np.linspace(-3, 3, 61)
    eta, Em = 0.1, 0.3
    gab, gba, lr, _, _ = green.cross_green(H, lam, rho, 1 << N, omega, eta, Em)
    z = omega + 1j * eta + Em
    lc, rc = lam.view(np.complex128), rho.view(np.complex128)
    ex_ab = E.resolvent_pair(lc, rc, z)
    ex_ba = E.resolvent_pair(rc, lc, z)
    scale = np.abs(ex_ab).max() + np.abs(ex_ba).max()
    assert np.abs(gab - ex_ab).max() <= 1e-10 * scale
    assert np.abs(gba - ex_ba).max() <= 1e-10 * scale
    assert abs(lr - np.vdot(lc, rc)) <= 1e-14 * (np.linalg.norm(lc) * np.linalg.norm(rc))
    # a planted mistake in the combination (the sign of the i-terms swapped) is caught
    assert np.abs(gba - ex_ab).max() > 1e-3 * scale


def test_cross_reduces_to_diagonal(sys8):
    """A = B: lam + i lam and lam - i lam are the same vector up to the exact factor -i and
    lam + lam is 2 lam, so G_AB = G_BA = the ordinary g of green_sequence, bit for bit."""
    cl, H, E = sys8
    phi, _ = hamiltonian.normalize(rng.gaussian(12, 0, N))
    _, qx, qy = cluster.allowed_momenta(cl)[2]
    c = hamiltonian.spin_op_q(cl, 2, qx, qy)
    lam = hamiltonian.apply_spin_op(N, c, phi)
    omega = np.linspace(-3, 3, 31)
    gab, gba, lr, _, coefs = green.cross_green(H, lam, lam, 40, omega, 0.05, -0.2)
    g, _, al, be = green.green_sequence(H, lam, 40, omega, 0.05, -0.2)
    assert np.array_equal(gab, g) and np.array_equal(gba, g)
    assert np.array_equal(coefs[2][0], coefs[3][0]) and np.array_equal(coefs[0][0], al)
    assert lr == hamiltonian.dot_re(lam, lam)


def test_cross_spectrum_hermitian_pairs(sys8):
    """S_BA = conj(S_AB) for every pair, S_AA is real and non-negative (finite n)."""
    cl, H, E = sys8
    phi, _ = hamiltonian.normalize(rng.gaussian(13, 0, N))
    ca, cb = _local_pair(N)
    lam = hamiltonian.apply_spin_op(N, ca, phi)
    rho = hamiltonian.apply_spin_op(N, cb, phi)
    omega = np.linspace(-3, 3, 31)
    gab, gba, _, _, _ = green.cross_green(H, lam, rho, 30, omega, 0.05, 0.0)
    s_ab = green.spectral_density(gab, gba)
    s_ba = green.spectral_density(gba, gab)
    assert np.abs(s_ba - np.conj(s_ab)).max() <= 1e-15 * np.abs(s_ab).max()
    gaa, _, _, _, _ = green.cross_green(H, lam, lam, 30, omega, 0.05, 0.0)
    s_aa = green.spectral_density(gaa, gaa)
    assert np.abs(s_aa.imag).max() == 0.0 and (s_aa.real >= -1e-15).all()


def test_cross_pipeline_exact_mean(sys8):
    """Eq. GAB_TPS / FRW1 for a general pair: the reweighted ratio-of-sums estimator over
    32 samples lies within its binning error of the estimator's exact expectation (ED),
    and that expectation approaches the canonical pair spectrum (Eq. chiAB) as M grows
    and eps shrinks."""
    cl, H, E = sys8
    ca, cb = _local_pair(N)
    omega = np.linspace(-2.5, 2.5, 11)
    eta = 0.15
    E_b, eps, L, M = -3.45, 0.15, 23, 8
    betas = [0.0, 1.0]
    n_s, nf, ng = 32, 300, 100
    Em = filters.energy_grid(E_b, eps, L)
    log_norm = np.zeros((n_s, 2))
    n_m = np.zeros((n_s, 2, L))
    gab = np.zeros((n_s, 2, L, 1, len(omega)), dtype=np.complex128)
    gba = np.zeros_like(gab)
    for s in range(n_s):
        phi0 = pipeline.start_vector(N, 77, s)
        for a, b in enumerate(betas):
            st = pipeline.typical_state(H, phi0, b, E_b, eps, L, M, nf)
            log_norm[s, a], n_m[s, a] = st.log_norm, st.n_m
            x, y, _ = green.shell_cross(H, st.Phi, st.E_m, [(ca, cb)], ng, omega, eta)
            gab[s, a], gba[s, a] = x, y
    S, err = reweight.reweight_cross(betas, np.stack([Em, Em]), [eps, eps], log_norm, n_m, gab, gba,
                                     [1.0, 1.5], n_bins=8)
    Aeig, Beig = E.op_eig(ca), E.op_eig(cb)
    for it, (ba, bt) in enumerate([(1.0, 1.0), (0.0, 1.0 / 1.5)]):
        exact = E.estimator_mean_cross(Aeig, Beig, ba, Em, eps, M, omega, eta, beta_t=bt)
        for part in ("real", "imag"):
            dev = np.abs(getattr(S[0, it], part) - getattr(exact, part)) / getattr(err[0, it], part)
            assert np.median(dev) < 2.0 and dev.max() < 5.0, (it, part)
        assert np.abs(exact.imag).max() > 0.05 * np.abs(exact).max()  # a genuinely complex pair
    can = E.canonical_cross(Aeig, Beig, omega, eta, 1.0)
    errs = []
    for eps_, M_ in ((0.2, 8), (0.003125, 512)):
        L_ = int(round(6.8 / (2 * eps_)))
        Em_ = filters.energy_grid(-3.41237, eps_, L_)
        errs.append(np.abs(E.estimator_mean_cross(Aeig, Beig, 1.0, Em_, eps_, M_, omega, eta) - can).max())
    assert errs[0] > 0.05 * np.abs(can).max() and errs[1] < 0.01 * np.abs(can).max()
