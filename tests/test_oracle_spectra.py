"""Pins of the oracle's spectrum estimator, reweighting and random vectors.

Sec. II.A (random vectors, Eq. variance_HDR), Sec. III (Eqs. chiAB, GAB_TPS, limGAB,
FRW1, FRW2), Sec. V (Eq. SQomega_TPS, binning).
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


def _start(seed):
    v, _ = hamiltonian.normalize(rng.gaussian(seed, 0, N))
    return v


@pytest.mark.parametrize("beta", [0.0, 2.0])
def test_per_sample_estimator_matches_ed(sys8, beta):
    """T6: for one fixed phi_0, g_m(w) and n_m from the Krylov path equal the same
    estimator evaluated in the ED eigenbasis (only Krylov truncation separates them)."""
    cl, H, E = sys8
    phi0 = _start(21)
    E_b, eps, L, M = -3.3, 0.15, 22, 8
    omega = np.linspace(-3, 3, 41)
    eta = 0.1
    st = pipeline.typical_state(H, phi0, beta, E_b, eps, L, M, 500)
    qx, qy = cluster.allowed_momenta(cl)[1][1:]
    g, res = green.shell_spectra(H, st.Phi, st.E_m, [(qx, qy)], [0, 2], 500, omega, eta)
    phib = E.expm_half(beta, phi0.view(np.complex128))
    phib /= np.linalg.norm(phib)
    for ia, a in enumerate([0, 2]):
        Se = E.sq_eig(a, qx, qy)
        gx, nx = E.estimator_exact(Se, phib, st.E_m, eps, M, omega, eta)
        assert np.abs(st.n_m - nx).max() < 1e-9
        assert np.abs(g[:, ia, 0, :] - gx).max() < 1e-7 * max(1.0, np.abs(gx).max())
    # -(1/pi) Im g >= 0: the Galerkin Ritz weights are non-negative
    assert (-g.imag >= -1e-15).all()


def test_sequence_sum_rule(sys8):
    """T8 (one sequence): the spectral weight of -(1/pi) Im g integrates to ||chi||^2."""
    cl, H, E = sys8
    chi = _start(7) * 1.7
    omega = np.linspace(-60, 60, 240001)
    g, _, _, _ = green.green_sequence(H, chi, 64, omega, 0.05, 0.0)
    integral = np.trapezoid(-g.imag / math.pi, omega)
    # Lorentzian tails beyond +-60: 2 * eta / (pi * 60) of the weight
    tail = 2 * 0.05 / (math.pi * 60) * 1.7**2
    assert abs(integral + tail - 1.7**2) < 2e-4


def test_infinite_temperature_sum_rule():
    """T8 (ensemble): E[sum_a <phi0|S^a_{-Q} S^a_Q|phi0>] = Tr(...)/N_F = 3/4 for every Q;
    sample scatter bounded by the Hams-De Raedt variance."""
    cl = cluster.honeycomb(*SUPERCELLS[N])
    for _, qx, qy in cluster.allowed_momenta(cl)[:2]:
        vals = []
        for s in range(400):
            v, _ = hamiltonian.normalize(rng.gaussian(99, s, N))
            tot = 0.0
            for a in range(3):
                chi = hamiltonian.apply_sq(cl, a, qx, qy, v)
                tot += hamiltonian.dot_re(chi, chi)
            vals.append(tot)
        vals = np.array(vals)
        O = sum(ed.dense_sq(cl, a, qx, qy).conj().T @ ed.dense_sq(cl, a, qx, qy) for a in range(3))
        NF = 1 << N
        assert abs(np.trace(O).real / NF - 0.75) < 1e-12
        var = (np.trace(O @ O).real / NF - (np.trace(O).real / NF) ** 2) / (NF + 1)
        assert abs(vals.mean() - 0.75) < 5 * math.sqrt(var / len(vals))
        assert 0.5 < vals.var() / var < 1.6


def test_rng_moments_and_hdr_variance(sys8):
    """T12: Gaussian draws have unit variance per component; <phi0|H|phi0> has mean
    Tr H / N_F = 0 and the Hams-De Raedt variance (Tr H^2/N_F) / (N_F + 1)."""
    cl, H, E = sys8
    g = rng.gaussian(1, 0, 16)
    assert abs(g.mean()) < 5 / math.sqrt(g.size) and abs(g.var() - 1) < 0.01
    NF = 1 << N
    vals = []
    for s in range(1000):
        v, _ = hamiltonian.normalize(rng.gaussian(2, s, N))
        vals.append(hamiltonian.dot_re(v, H.apply(v)))
    vals = np.array(vals)
    var_hdr = (np.trace(E.H @ E.H) / NF) / (NF + 1)
    assert abs(vals.mean()) < 5 * math.sqrt(var_hdr / len(vals))
    assert 0.85 < vals.var() / var_hdr < 1.15


def test_rng_splitmix64_reference_outputs():
    """The generator is SplitMix64 as published (Steele, Lea and Flood, OOPSLA 2014, and
    its reference C implementation): seeded with 0, its first three outputs are
    e220a8397b1dcdaf, 6e789e6aa1b965f4 and 06c45d188009454f.  The draws use its streams as
    documented: the key of sample s is output s + 1 of the seed's stream, and entry 0 of a
    vector takes outputs 1 and 2 of the key's stream through Box-Muller (u1 in (0, 1])."""
    assert [rng.splitmix64(0, k) for k in (1, 2, 3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                                         0x06C45D188009454F]
    for seed, sample in ((0, 0), (180202854, 3)):
        key = rng.splitmix64(seed, sample + 1)
        u1, u2 = rng.splitmix64(key, 1), rng.splitmix64(key, 2)
        r = math.sqrt(-2.0 * math.log(((u1 >> 11) + 1) * 2.0 ** -53))
        th = 2.0 * math.pi * ((u2 >> 11) * 2.0 ** -53)
        g = rng.gaussian(seed, sample, 2)
        assert abs(g[0] - r * math.cos(th)) <= 1e-15 * r and abs(g[1] - r * math.sin(th)) <= 1e-15 * r


def test_su2_lorentzian_at_k0():
    """T9: at K = 0, S^a_Gamma commutes with H, so the canonical spectrum is a Lorentzian
    of weight <S_tot(S_tot+1)>_beta / N, and the three components are equal."""
    cl = cluster.honeycomb(*SUPERCELLS[N])
    E = ed.ED(cl, 0.0, 1.0)
    omega = np.linspace(-1, 1, 21)
    eta, beta = 0.05, 2.0
    S = [E.canonical_dsf([a], 0.0, 0.0, omega, eta, beta) for a in range(3)]
    assert np.abs(S[0] - S[1]).max() < 1e-12 and np.abs(S[0] - S[2]).max() < 1e-12
    w = np.exp(-beta * (E.E - E.E[0]))
    w /= w.sum()
    Stot2 = sum(ed.dense_sq(cl, a, 0.0, 0.0).conj().T @ ed.dense_sq(cl, a, 0.0, 0.0) for a in range(3)) * N
    ss1 = float(np.real(np.einsum("n,mn,mk,kn->", w, E.U.conj(), Stot2, E.U)))
    lor = (eta / math.pi) / (omega**2 + eta**2) * ss1 / N
    assert np.abs(S[0] + S[1] + S[2] - lor).max() < 1e-10


def test_kitaev_nearest_neighbour_correlations():
    """T10: at J = 0, <S^a_i S^b_j>_beta = 0 unless i = j (a = b) or ij is an a-bond (a = b).
    Checked on the 12-site cluster where no plaquette wraps onto itself."""
    cl = cluster.honeycomb(*SUPERCELLS[12])
    E = ed.ED(cl, 1.0, 0.0)
    beta = 1.5
    w = np.exp(-beta * (E.E - E.E[0]))
    w /= w.sum()
    rho = (E.U * w[None, :]) @ E.U.conj().T
    Nc = cl.n_sites
    bond_type = {}
    for i, j, g in cl.bonds:
        bond_type[(i, j)] = bond_type[(j, i)] = g
    ops = [[ed.site_op(Nc, l, ed.PAULI[a]) for a in range(3)] for l in range(Nc)]
    for i in (0, 1, 5):
        for j in range(Nc):
            for a in range(3):
                for b in range(3):
                    c = np.real(np.sum((ops[i][a] @ ops[j][b]).multiply(rho.T)))
                    allowed = (i == j and a == b) or (a == b and bond_type.get((i, j)) == a)
                    if not allowed:
                        assert abs(c) < 1e-10, (i, j, a, b, c)
                    elif i != j:
                        assert abs(c) > 1e-3


def test_canonical_dsf_sum_rule():
    """The ED checker itself: the canonical spectrum integrates to <S_{-Q}S_Q>_beta, which is
    3/4 at beta = 0.  Each Lorentzian pole integrates in closed form over [-W, W]."""
    cl = cluster.honeycomb(*SUPERCELLS[N])
    E = ed.ED(cl, -1.0, 0.1)
    omega = np.linspace(-3, 3, 61)
    eta, W = 0.05, 40.0
    S = E.canonical_dsf([0, 1, 2], 0.0, 0.0, omega, eta, 0.0)
    total = 0.0
    integ = 0.0
    for a in range(3):
        M2 = np.abs(E.sq_eig(a, 0.0, 0.0)) ** 2 / (1 << N)
        total += M2.sum()
        dE = E.E[None, :] - E.E[:, None]  # pole at omega = E_mu - E_nu = -dE
        integ += (M2 * (np.arctan((W + dE) / eta) + np.arctan((W - dE) / eta)) / math.pi).sum()
    assert abs(total - 0.75) < 1e-12
    assert abs(integ + 2 * eta / (math.pi * W) * 0.75 - 0.75) < 1e-5
    assert (S >= -1e-15).all()


def test_reweight_identity_and_exact_mean(sys8):
    """T11: at beta' = beta_a the reweighted value is the plain ratio; with many samples
    the ratio-of-sums estimator approaches the estimator's exact mean (ED) within its
    binning standard error, and the exact mean approaches the canonical spectrum."""
    cl, H, E = sys8
    omega = np.linspace(-2.5, 2.5, 11)
    eta = 0.1
    E_b, eps, L, M = -3.45, 0.15, 23, 8
    betas = [0.0, 1.0]
    n_s = 48
    res = pipeline.run(cl, -1.0, 0.1, seed=5, n_samples=n_s, betas=betas, E_b=E_b, eps=eps, L=L, M=M,
                       n_filter=400, n_green=120, qs=[(0.0, 0.0)], alphas=[0, 1, 2], omega=omega,
                       eta=eta, temps=[1.0, 1.5], n_bins=8)
    # identity: T' = 1 uses anchor beta = 1 with unit reweighting factors
    g = res["g"].sum(axis=3)
    lw = 2 * res["log_norm"][:, 1][:, None] + 0 * res["E_m"][1][None, :]
    wts = np.exp(lw - lw.max())
    num = np.einsum("sl,slqw->qw", wts, g[:, 1])
    den = float((wts * res["n_m"][:, 1]).sum())
    assert np.abs(res["S"][:, 0, :] - (-num.imag / (math.pi * den))).max() < 1e-13
    # statistics: estimator vs its exact expectation at T' = 1 and reweighted T' = 1/1.5
    Sl = [E.sq_eig(a, 0.0, 0.0) for a in range(3)]
    Em = filters.energy_grid(E_b, eps, L)
    # T' = 1 comes from the beta = 1 anchor; T' = 1.5 is reweighted from the beta = 0 anchor
    for it, (ba, bt) in enumerate([(1.0, 1.0), (0.0, 1.0 / 1.5)]):
        exact = E.estimator_mean(Sl, ba, Em, eps, M, omega, eta, beta_t=bt)
        dev = np.abs(res["S"][0, it] - exact) / res["stderr"][0, it]
        assert np.median(dev) < 2.0 and dev.max() < 5.0
    # discretisation: the exact mean approaches the canonical spectrum when M grows and
    # then eps shrinks (Eq. limGAB).  Levels that sit within ~eps/M of a shell edge keep
    # only half their weight (sum_m f_m^2 = 1/2 there), so convergence is checked at a
    # coarse and a fine discretisation with an irrational grid offset.
    can = E.canonical_dsf([0, 1, 2], 0.0, 0.0, omega, eta, 1.0)
    errs = []
    for eps_, M_ in ((0.2, 8), (0.003125, 512)):
        L_ = int(round(6.8 / (2 * eps_)))
        Em_ = filters.energy_grid(-3.41237, eps_, L_)
        errs.append(np.abs(E.estimator_mean(Sl, 1.0, Em_, eps_, M_, omega, eta) - can).max())
    assert errs[0] > 0.1 * np.abs(can).max() and errs[1] < 0.01 * np.abs(can).max()
