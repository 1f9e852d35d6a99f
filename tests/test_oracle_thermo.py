"""Pins of the oracle's thermodynamics from shell data (Sec. II.A partition function,
Eq. FRW1 with O = H, H^2) against exact diagonalisation."""
import math

import numpy as np
import pytest

from oracle import cluster, ed, hamiltonian, pipeline, rng, thermo
from seeded_inputs import SUPERCELLS

N = 8


@pytest.fixture(scope="module")
def sys8():
    cl = cluster.honeycomb(*SUPERCELLS[N])
    return cl, hamiltonian.Hamiltonian(cl, -1.0, 0.1), ed.ED(cl, -1.0, 0.1)


def _samples(H, betas, n_s, E_b, eps, L, M, n, seed):
    A = len(betas)
    ln = np.zeros((n_s, A))
    nm, h1, h2 = (np.zeros((n_s, A, L)) for _ in range(3))
    Em = np.zeros((A, L))
    for s in range(n_s):
        phi0, _ = hamiltonian.normalize(rng.gaussian(seed, s, N))
        for a, b in enumerate(betas):
            st = pipeline.typical_state(H, phi0, b, E_b, eps, L, M, n, moments=True)
            ln[s, a], nm[s, a], h1[s, a], h2[s, a], Em[a] = st.log_norm, st.n_m, st.h1, st.h2, st.E_m
    return ln, nm, h1, h2, Em


def test_shell_moments_match_ed(sys8):
    """h1_m = <phi^m|H|phi^m> and h2_m = ||H phi^m||^2 against f_m(H) phi in the eigenbasis."""
    from oracle import filters
    cl, H, E = sys8
    phi0, _ = hamiltonian.normalize(rng.gaussian(3, 0, N))
    E_b, eps, L, M = -3.3, 0.15, 22, 8
    st = pipeline.typical_state(H, phi0, 0.0, E_b, eps, L, M, 300, moments=True)
    d = E.U.T @ phi0.view(np.complex128)
    for m in range(L):
        w = np.abs(filters.filter_closed_form(E.E, st.E_m[m], eps, M) * d) ** 2
        assert abs(st.h1[m] - float((w * E.E).sum())) <= 1e-10
        assert abs(st.h2[m] - float((w * E.E ** 2).sum())) <= 1e-10


def test_single_sample_at_anchor(sys8):
    """beta' = beta_a, one sample: <H> = sum h1 / sum n and ln Z = ln N_F + 2 log_norm."""
    cl, H, E = sys8
    ln, nm, h1, h2, Em = _samples(H, [0.5], 1, -3.3, 0.15, 22, 8, 200, 4)
    out = thermo.thermodynamics([0.5], Em, ln, nm, h1, h2, N, [2.0], n_bins=1)
    assert abs(out["E"][0] - h1.sum() / nm.sum()) <= 1e-14 * abs(h1.sum() / nm.sum())
    assert abs(out["lnZ"][0] - (N * math.log(2) + 2 * ln[0, 0])) <= 1e-12
    assert math.isnan(out["E_err"][0])


@pytest.fixture(scope="module")
def samples48(sys8):
    """48 random vectors at anchors T = inf and T = 1 (E_b -3.3, eps 0.15, L 22, M 8)."""
    cl, H, E = sys8
    return _samples(H, [0.0, 1.0], 48, -3.3, 0.15, 22, 8, 200, 11)


def test_estimator_converges_to_exact_mean(sys8, samples48):
    """48 random vectors at anchors T = inf and T = 1: E, C, S, ln Z at several T' agree with
    the exact expectation of the estimator (ED) within 5 binned standard errors."""
    cl, H, E = sys8
    betas = [0.0, 1.0]
    E_b, eps, L, M = -3.3, 0.15, 22, 8
    ln, nm, h1, h2, Em = samples48
    temps = [0.8, 1.0, 1.5, 4.0]
    out = thermo.thermodynamics(betas, Em, ln, nm, h1, h2, N, temps, n_bins=8)
    for it, T in enumerate(temps):
        a = 1 if T <= 1.0 else 0
        ref = E.thermo_estimator_mean(betas[a], Em[a], eps, M, 1.0 / T)
        for j, k in enumerate(("E", "C", "S", "lnZ")):
            assert abs(out[k][it] - ref[j]) <= 5 * out[k + "_err"][it] + 1e-9, (T, k, out[k][it], ref[j])


def test_exact_mean_tends_to_canonical(sys8):
    """Narrow, sharp shells (eps -> 0, M -> infinity): the estimator's exact mean approaches
    the canonical E, C, S, ln Z.  For a discrete spectrum both limits are needed: a level
    within a few 1/M of a shell edge carries sum_m f_m^2 down to 1/2 whatever eps is.  The
    grid is offset by an irrational amount (many levels of this model are round numbers)."""
    cl, H, E = sys8
    E_b = -3.3 - 1e-3 * math.sqrt(2.0)
    for T in (0.7, 1.0, 3.0):
        can = np.array(E.thermo_canonical(1.0 / T))
        errs = []
        for eps, L, M in ((0.1, 33, 16), (0.003, 1100, 4096)):
            Em = E_b + (2 * np.arange(L) + 1) * eps
            with np.errstate(over="ignore"):
                errs.append(np.abs(np.array(E.thermo_estimator_mean(0.0, Em, eps, M, 1.0 / T)) - can).max())
        assert errs[1] < errs[0] / 5 and errs[1] < 1e-3, (T, errs)


def _static_exact_mean(E, S, beta_a, E_m, eps, M, beta_t):
    """Exact expectation of the FRW1 estimator of <S^dag S> (S in the eigenbasis)."""
    from oracle import filters
    d = (np.abs(S) ** 2).sum(axis=0)  # (S^dag S)_{nu nu}
    bw = np.exp(-beta_a * (E.E - E.E[0]))
    num = den = 0.0
    for m in range(len(E_m)):
        with np.errstate(over="ignore"):
            f2 = filters.filter_closed_form(E.E, E_m[m], eps, M) ** 2
        rw = math.exp((beta_a - beta_t) * (E_m[m] - E_m[0]))
        num += rw * float((bw * f2 * d).sum())
        den += rw * float((bw * f2).sum())
    return num / den


def test_static_structure_factor(sys8):
    """Static S^{alpha alpha}(Q) = <S_{-Q} S_{+Q}> reweighted by Eq. FRW1 from ||S_Q phi^m||^2:
    48 vectors against the exact expectation of the estimator (ED) within 5 binned errors,
    and that exact mean against the canonical value for narrow, sharp shells."""
    from oracle import reweight
    cl, H, E = sys8
    q = cluster.allowed_momenta(cl)[1][1:]
    Smats = [E.sq_eig(a, *q) for a in range(3)]
    E_b, eps, L, M, n_s = -3.3, 0.15, 22, 8, 48
    O = np.zeros((n_s, 1, L, 3))
    ln, nm, Em = np.zeros((n_s, 1)), np.zeros((n_s, 1, L)), None
    for s in range(n_s):
        phi0, _ = hamiltonian.normalize(rng.gaussian(71, s, N))
        st = pipeline.typical_state(H, phi0, 0.0, E_b, eps, L, M, 200)
        ln[s, 0], nm[s, 0], Em = st.log_norm, st.n_m, st.E_m
        for m in range(L):
            for a in range(3):
                chi = hamiltonian.apply_sq(cl, a, *q, st.Phi[m])
                O[s, 0, m, a] = hamiltonian.dot_re(chi, chi)
    temps = [0.7, 2.0]
    out, err = reweight.reweight_observable([0.0], Em[None], ln, nm, O, temps, n_bins=8)
    for it, T in enumerate(temps):
        for a in range(3):
            ref = _static_exact_mean(E, Smats[a], 0.0, Em, eps, M, 1.0 / T)
            assert abs(out[a, it] - ref) <= 5 * err[a, it] + 1e-12, (T, a, out[a, it], ref)
    # canonical limit
    E_b2, eps2, L2, M2 = -3.3 - 1e-3 * math.sqrt(2.0), 0.003, 1100, 4096
    Em2 = E_b2 + (2 * np.arange(L2) + 1) * eps2
    for T in (0.7, 2.0):
        w = np.exp(-(E.E - E.E[0]) / T)
        for a in range(3):
            can = float((w * (np.abs(Smats[a]) ** 2).sum(axis=0)).sum() / w.sum())
            assert abs(_static_exact_mean(E, Smats[a], 0.0, Em2, eps2, M2, 1.0 / T) - can) <= 2e-3 * can


def test_diagnostics_match_exact_mean(sys8, samples48):
    """Energy variance and ln[Z(2b)/Z(b)^2] from the 48 vectors agree with the exact
    expectation of the estimator (ED) within 5 binned errors (2b may use another anchor)."""
    cl, H, E = sys8
    betas = [0.0, 1.0]
    eps, M = 0.15, 8
    ln, nm, h1, h2, Em = samples48
    bts = [0.25, 0.6, 1.0, 1.25]
    out = thermo.diagnostics(betas, Em, ln, nm, h1, h2, N, bts, n_bins=8)
    for it, b in enumerate(bts):
        a1 = 1 if b >= 1.0 else 0
        a2 = 1 if 2 * b >= 1.0 else 0
        e1, C1, _, lz1 = E.thermo_estimator_mean(betas[a1], Em[a1], eps, M, b)
        lz2 = E.thermo_estimator_mean(betas[a2], Em[a2], eps, M, 2 * b)[3]
        assert abs(out["var"][it] - C1 / b**2) <= 5 * out["var_err"][it] + 1e-9, b
        assert abs(out["log_typ"][it] - (lz2 - 2 * lz1)) <= 5 * out["log_typ_err"][it] + 1e-9, b


def test_typicality_factor_limits(sys8, samples48):
    """Sec. III.C, V.B and Appendix B: Z(2b)/Z(b)^2 -> 1/N_F as b -> 0 (estimator and ED), lies between 1/N_F and
    1/D (D = ground-state degeneracy) and equals e^{-S(b*)} with S(2b) <= S(b*) <= S(b)
    (canonical ED); the estimator's exact mean tends to the canonical value for narrow,
    sharp shells."""
    cl, H, E = sys8
    ln, nm, h1, h2, Em = samples48
    out = thermo.diagnostics([0.0, 1.0], Em, ln, nm, h1, h2, N, [1e-9], n_bins=1)
    assert abs(out["log_typ"][0] + N * math.log(2)) < 1e-6
    D = int(np.sum(E.E - E.E[0] < 1e-9))
    for b in (1e-6, 0.3, 1.0, 3.0, 30.0):
        lz1, lz2 = E.thermo_canonical(b)[3], E.thermo_canonical(2 * b)[3]
        lt = lz2 - 2 * lz1
        assert -N * math.log(2) - 1e-9 <= lt <= -math.log(D) + 1e-9
        assert E.thermo_canonical(2 * b)[2] - 1e-9 <= -lt <= E.thermo_canonical(b)[2] + 1e-9
    assert abs(E.thermo_canonical(1e-6)[3] * 2 - E.thermo_canonical(2e-6)[3] - N * math.log(2)) < 1e-4
    E_b = -3.3 - 1e-3 * math.sqrt(2.0)
    eps, L, M = 0.003, 1100, 4096
    Em2 = E_b + (2 * np.arange(L) + 1) * eps
    for b in (0.5, 1.0):
        with np.errstate(over="ignore"):
            lt = (E.thermo_estimator_mean(0.0, Em2, eps, M, 2 * b)[3]
                  - 2 * E.thermo_estimator_mean(0.0, Em2, eps, M, b)[3])
        can = E.thermo_canonical(2 * b)[3] - 2 * E.thermo_canonical(b)[3]
        assert abs(lt - can) < 2e-3, (b, lt, can)


def test_choose_anchors_covers_grid(sys8):
    """The anchor ladder on canonical E, var (ED): every grid temperature is reweighted from
    an anchor with r <= r_max, each new anchor is the first point beyond reach of the
    previous one, and max_anchors caps the ladder."""
    cl, H, E = sys8
    grid = np.linspace(0.0, 6.0, 61)
    Ev, var = [], []
    for b in grid:
        e1, C, _, _ = E.thermo_canonical(b)
        w = np.exp(-b * (E.E - E.E[0]))
        Ev.append(e1)
        var.append(float((w * (E.E - e1) ** 2).sum() / w.sum()))
    for r_max in (0.3, 0.6, 1.5):
        anc = thermo.choose_anchors(grid, Ev, var, r_max, 100)
        assert anc[0] == 0 and anc == sorted(anc)
        for j in range(len(grid)):
            a = max(k for k in anc if k <= j)
            assert thermo.overlap_ratio(Ev[a], var[a], Ev[j], var[j]) <= r_max or j == a
        for p, k in zip(anc, anc[1:]):
            assert thermo.overlap_ratio(Ev[p], var[p], Ev[k], var[k]) > r_max
    assert len(thermo.choose_anchors(grid, Ev, var, 0.3, 2)) == 2
    assert len(thermo.choose_anchors(grid, Ev, var, 0.3, 100)) > len(thermo.choose_anchors(grid, Ev, var, 1.5, 100))
