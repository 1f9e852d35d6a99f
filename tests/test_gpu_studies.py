"""The convergence studies of Appendix C on the GPU path.

E10, CG-step dependence (18 sites, antiferromagnetic Kitaev model K = 1, J = 0, at
T = 0.1, Table I's 18-site discretisation E_b = -4, eps = 1.953125e-3, M = 64, sixteen
shells of its grid around the peak of the energy distribution): the GPU's filter
Lanczos coefficients bit for bit against the oracle, the largest residual 2-norm over
each shell's M contour points as a function of the step (library host routine on the
GPU's coefficients against the oracle's Ritz route on its own), the steps to reach
the paper's bound 1e-4, which grow when L and M are doubled (smaller min Im z), and
the residual-truncated filter run (resid_tol = 1e-4) against the full run.  Dense
exact diagonalisation is out of reach at 2^18 states, so the ED comparisons below run
at 12 sites.

E10 against ED (12 sites): truncated filtered states of the GPU within the bound the
truncation guarantees of f_m(H) phi_beta (ED eigenbasis, closed-form filter).

E11, dependence on the discretisation delta (12 sites, K = -1, J = 0.1, T = 1, eta
0.05, delta = (E_b, eps, M) = (-3, 0.15, 8) and (-3, 0.1, 8), both converged in 700
filter and 500 Green's steps): for the two discretisations the GPU's per-sample estimator g_m(omega), n_m and the
reweighted S(Q, omega) equal the same estimator evaluated exactly in the ED
eigenbasis for that delta, so the delta-dependence the GPU reports is the method's own.
"""
import math

import numpy as np
import pytest

from seeded_inputs import SUPERCELLS, gaussian_vector

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1802_02854_amd as ftk
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return ftk, torch, ftk.Context(0)


def _states(ftk, torch, h, N, seed, betas, E_b, eps, L, M, n, **kw):
    g0 = gaussian_vector(seed, 0, N)
    G = torch.from_numpy(g0.view(np.complex128)).to("cuda").reshape(1, -1)
    st = ftk.TypicalStates(h, seed=seed, n_vectors=1, betas=betas, E_b=E_b, eps=eps, L=L, M=M, n_steps=n, gaussians=G,
                           **kw)
    return st, g0


def test_cg_step_study_n18(env):
    ftk, torch, ctx = env
    from oracle import cluster, filters, hamiltonian, lanczos, pipeline, taylor
    print("E10 N=18", flush=True)
    N, K, J, beta = 18, 1.0, 0.0, 10.0
    eps, M, m0, L, n = 1.953125e-3, 64, 148, 16, 320
    E_b = -4.0 + 2.0 * eps * m0  # shells 148..163 of Table I's 18-site grid
    cl = ftk.honeycomb_cluster(*SUPERCELLS[N])
    h = ftk.Hamiltonian(ctx, cl, K, J)
    oh = hamiltonian.Hamiltonian(cluster.honeycomb(*SUPERCELLS[N]), K, J)
    st, g0 = _states(ftk, torch, h, N, 5, [beta], E_b, eps, L, M, n)
    al, be = st.lanczos(0, 0)
    phib, _ = taylor.canonical_state(oh, pipeline.start_vector(N, 5, 0, g0), beta)
    ao, bo, _, _ = lanczos.lanczos(oh, phib, n)
    assert np.array_equal(al, ao) and np.array_equal(be, bo)
    ln, nm, Em, _ = st.scalars()
    peak = int(np.argmax(nm[0, 0]))
    steps = {}
    for (e2, M2) in ((eps, M), (eps / 2, 2 * M)):
        wr, wi = filters.contour_nodes(e2, M2)
        z = Em[0][peak] + wr + 1j * wi
        hist = ftk.residual_history(al, be, z)  # library host routine on the GPU's coefficients
        ref = lanczos.residual_history(ao, bo, z)  # oracle: Ritz decomposition of every T_k
        big = ref > 1e-12
        assert np.abs(hist[big] - ref[big]).max() <= 1e-7 * ref[big].max()
        assert hist[-1] < 1e-4  # decays below the paper's bound within n steps
        steps[M2] = int(np.argmax(hist <= 1e-4)) + 1
    # four times smaller min Im z takes more steps (the paper: about ten percent more)
    assert steps[M] <= steps[2 * M] <= 1.5 * steps[M]
    # the truncated run (each filter on its own contour points, bound 1e-4) against the full run
    st_t, _ = _states(ftk, torch, h, N, 5, [beta], E_b, eps, L, M, n, resid_tol=1e-4)
    _, nm_t, _, _ = st_t.scalars()
    k_t = len(st_t.lanczos(0, 0)[0])
    assert k_t < n
    assert np.abs(nm_t - nm).max() <= 1e-4 / math.sin(math.pi / M) * 2.0 * math.sqrt(nm.max())


@pytest.fixture(scope="module")
def ed12():
    from oracle import cluster, ed
    cl = cluster.honeycomb(*SUPERCELLS[12])
    return cl, ed.ED(cl, -1.0, 0.1)


def test_truncated_filters_against_ed_n12(env, ed12):
    """GPU filter runs truncated at the paper's bound (each shell on its own contour
    points) give states within tol / sin(pi/M) of f_m(H) phi_beta (ED)."""
    ftk, torch, ctx = env
    from oracle import filters
    print("E10 N=12 vs ED", flush=True)
    ocl, E = ed12
    N, beta, E_b, eps, L, M, tol = 12, 1.0, -2.4, 0.1, 16, 8, 1e-4
    h = ftk.Hamiltonian(ctx, ftk.honeycomb_cluster(*SUPERCELLS[N]), -1.0, 0.1)
    st, g0 = _states(ftk, torch, h, N, 9, [beta], E_b, eps, L, M, 600, resid_tol=tol)
    assert len(st.lanczos(0, 0)[0]) < 600
    phi0 = g0.view(np.complex128) / np.linalg.norm(g0)
    ex = E.expm_half(beta, phi0)
    phib = ex / np.linalg.norm(ex)
    d = E.U.T @ phib
    Em = filters.energy_grid(E_b, eps, L)
    bound = tol / math.sin(math.pi / M)
    for m in range(L):
        f = filters.filter_closed_form(E.E, Em[m], eps, M)
        ref = E.U @ (f * d)
        got = st.shell(0, 0, m).cpu().numpy()
        assert np.linalg.norm(got - ref) <= bound, m


def _ed_estimator(E, cl, phib, Em, eps, M, omega, eta, alphas, q):
    """Per-sample g_m(omega) summed over alphas, and n_m, exactly in the ED eigenbasis:
    phi^m = f_m(H) phi_beta, chi = S^alpha_Q phi^m, g = sum_mu |<mu|chi>|^2 / (z - E_mu)."""
    from oracle import filters, hamiltonian
    d = E.U.T @ phib
    g = np.zeros((len(Em), len(omega)), dtype=np.complex128)
    nm = np.zeros(len(Em))
    for m in range(len(Em)):
        f = filters.filter_closed_form(E.E, Em[m], eps, M)
        phim = E.U @ (f * d)
        nm[m] = float(np.sum(np.abs(f * d) ** 2))
        for a in alphas:
            chi = hamiltonian.apply_sq(cl, a, q[0], q[1], np.ascontiguousarray(phim).view(np.float64))
            c = E.U.T @ chi.view(np.complex128)
            z = omega[:, None] + 1j * eta + Em[m] - E.E[None, :]
            g[m] += (np.abs(c) ** 2 / z).sum(axis=1)
    return g, nm


def test_delta_dependence_n12(env, ed12):
    ftk, torch, ctx = env
    from oracle import filters
    print("E11 N=12 vs ED", flush=True)
    ocl, E = ed12
    N, beta, eta = 12, 1.0, 0.05
    omega = np.linspace(-3, 3, 121)
    h = ftk.Hamiltonian(ctx, ftk.honeycomb_cluster(*SUPERCELLS[N]), -1.0, 0.1)
    q = ftk.honeycomb_momenta(*SUPERCELLS[N])[1]
    Ss = []
    for (E_b, eps, L, M) in ((-3.0, 0.15, 20, 8), (-3.0, 0.1, 30, 8)):
        st, g0 = _states(ftk, torch, h, N, 11, [beta], E_b, eps, L, M, 700)
        sp = ftk.Spectrum(h, st, q_xy=[tuple(q)], omega=omega, eta=eta, n_steps=500)
        g, res = sp.raw()
        ln, nm, Em, ep = st.scalars()
        phi0 = g0.view(np.complex128) / np.linalg.norm(g0)
        ex = E.expm_half(beta, phi0)
        phib = ex / np.linalg.norm(ex)
        ge, ne = _ed_estimator(E, ocl, phib, Em[0], eps, M, omega, eta, (0, 1, 2), q)
        gs = g[0, 0, :, :, 0].sum(axis=1)
        assert np.abs(nm[0, 0] - ne).max() <= 1e-9 * ne.max()
        assert np.abs(gs - ge).max() <= 5e-7 * np.abs(ge).max()
        S, _, _ = ftk.reweight([beta], Em, ep, ln, nm, g.sum(axis=3), [1.0], n_bins=1)
        num = -(ge.sum(axis=0)).imag / math.pi
        assert np.abs(S[0, 0] - num / ne.sum()).max() <= 5e-7 * np.abs(num / ne.sum()).max()
        Ss.append(S[0, 0])
    # the two discretisations give different finite-delta estimates of the same spectrum
    assert np.abs(Ss[0] - Ss[1]).max() > 1e-6 * np.abs(Ss[1]).max()
