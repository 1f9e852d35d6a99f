"""CPU checks of the library: exported symbols, and the host-side steps of the path
(cluster, momenta, shell coefficients, Taylor plan, reweighting) against the oracle."""
import ctypes
import math
import re
import subprocess

import numpy as np
import pytest

import paper_1802_02854_amd as ftk
from oracle import cluster, filters, hamiltonian, lanczos, reweight, rng, taylor
from seeded_inputs import SUPERCELLS


def _declared():
    import os
    hdr = open(os.path.join(os.path.dirname(ftk.LIB_PATH), "..", "include", "ftkw.h")).read()
    return sorted(set(re.findall(r"\b(ftk_[a-z_0-9]+)\s*\(", hdr)))


def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", ftk.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r" T (ftk_[a-z_0-9]+)", out))
    declared = _declared()
    assert len(declared) >= 25
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    L = ctypes.CDLL(ftk.LIB_PATH)
    for s in declared:
        getattr(L, s)


@pytest.mark.parametrize("N", sorted(SUPERCELLS))
def test_cluster_and_momenta_match_oracle(N):
    T = SUPERCELLS[N]
    c = ftk.honeycomb_cluster(*T)
    o = cluster.honeycomb(*T)
    assert c.bonds == o.bonds
    assert np.array_equal(c.site_xy, o.site_xy)
    q = ftk.honeycomb_momenta(*T)
    qo = np.array([[a, b] for _, a, b in cluster.allowed_momenta(o)])
    assert np.array_equal(q, qo)


def test_named_momenta_match_oracle():
    for n in ("Gamma", "M", "K", "M'"):
        assert np.array_equal(ftk.named_momentum(n), np.array(cluster.named_momentum(n)))
    with pytest.raises(ftk.FTKError, match="EINVAL"):
        ftk.named_momentum("X")


def test_cluster_rejects_small_supercell():
    with pytest.raises(ftk.FTKError, match="EINVAL"):
        ftk.honeycomb_cluster((1, 0), (0, 1))
    with pytest.raises(ftk.FTKError, match="EINVAL"):
        ftk.honeycomb_cluster((2, 0), (4, 0))


@pytest.mark.parametrize("n,L,M", [(64, 64, 16), (17, 5, 2), (1, 3, 4)])
def test_filter_coefficients_bitwise(n, L, M):
    cl = cluster.honeycomb(*SUPERCELLS[8])
    H = hamiltonian.Hamiltonian(cl, -1.0, 0.1)
    v, nrm = hamiltonian.normalize(rng.gaussian(3, 1, 8))
    a, b, _, _ = lanczos.lanczos(H, v, n)
    c = ftk.filter_coefficients(a, b, 1.0000000000000002, -3.0, 3 / 64, L, M)
    co = filters.shell_coefficients(a, b, 1.0000000000000002, -3.0, 3 / 64, L, M)
    assert np.array_equal(c.view(np.float64), co.view(np.float64))
    with pytest.raises(ftk.FTKError, match="EINVAL"):
        ftk.filter_coefficients(a, b, 1.0, -3.0, 3 / 64, L, 3)


@pytest.mark.parametrize("N,beta", [(8, 0.0), (8, 0.7), (8, 100.0), (16, 5.0), (24, 5.0), (24, 1.0)])
def test_taylor_plan_matches_oracle(N, beta):
    cl = cluster.honeycomb(*SUPERCELLS[N])
    H = hamiltonian.Hamiltonian(cl, -1.0, 0.1)
    Md, c, K, ell = taylor.split_plan(N, beta, H.norm_bound)
    assert (Md, K, c, ell) == ftk.taylor_plan(N, beta, H.norm_bound)


def test_reweight_matches_oracle():
    rs = np.random.default_rng(3)
    nv, na, L, nq, nw = 6, 3, 10, 2, 7
    betas = np.array([0.0, 1.0, 5.0])
    E_m = np.stack([np.linspace(-3, 3, L) + 0.01 * a for a in range(na)])
    eps = np.array([0.3, 0.3, 0.2])
    log_norm = rs.normal(size=(nv, na)) * 10
    n_m = rs.uniform(0, 1, size=(nv, na, L))
    n_m[0, 1, 3] = 0.0
    g = rs.normal(size=(nv, na, L, nq, nw)) + 1j * rs.normal(size=(nv, na, L, nq, nw))
    temps = np.geomspace(0.1, 10, 9)
    S, err, P = ftk.reweight(betas, E_m, eps, log_norm, n_m, g, temps, n_bins=3)
    So, erro, Po = reweight.reweight(betas, E_m, eps, log_norm, n_m, g, temps, n_bins=3)
    assert np.abs(S - So).max() <= 1e-12 * np.abs(So).max()
    assert np.abs(err - erro).max() <= 1e-10 * np.abs(erro).max()
    assert np.abs(P - Po).max() <= 1e-12 * np.abs(Po).max()
    with pytest.raises(ftk.FTKError, match="EINVAL"):
        ftk.reweight(betas, E_m, eps, log_norm, n_m, g, [-1.0], n_bins=3)


@pytest.mark.parametrize("n", [1, 2, 7, 60])
def test_shell_window_matches_oracle(n):
    """The library's Sturm bisection finds the same extreme Ritz values as the oracle's
    dense eigensolver, so the automatic window agrees to rounding."""
    from oracle import filters, hamiltonian, lanczos, rng
    cl = cluster.honeycomb(*SUPERCELLS[8])
    H = hamiltonian.Hamiltonian(cl, -1.0, 0.3)
    v, _ = hamiltonian.normalize(rng.gaussian(17, 0, 8))
    a, b, _, _ = lanczos.lanczos(H, v, n)
    ref = filters.auto_window(a, b, 16, 0.1)
    got = ftk.shell_window(a, b, 16, 0.1)
    assert abs(got[0] - ref[0]) < 1e-13 and abs(got[1] - ref[1]) < 1e-14


def test_request_footprint():
    """The server's reservation: the shells of one vector plus its work vectors, the
    buffered Lanczos vectors and a batch of Green's sequences, each 16 2^N bytes, with
    a 2 % margin and 64 MiB for allocation granularity."""
    from paper_1802_02854_amd.api import Request
    cl = ftk.honeycomb_cluster(*SUPERCELLS[16])

    def req(N, B, betas=(0.0,), L=16, block_steps=16):
        c = ftk.honeycomb_cluster(*SUPERCELLS[N]) if N != 16 else cl
        return Request(c, -1.0, 0.1, seed=1, n_vectors=8, betas=betas, L=L, M=16, n_filter=300,
                       q_xy=[(0.0, 0.0)], omega=np.linspace(-4, 4, 1000), eta=0.02, n_green=300,
                       temps=[1.0, 2.0], rhs_block=B, block_steps=block_steps)

    for N in (16, 20, 24, 28):
        V = 16 * 2**N
        f = req(N, 1).footprint()
        assert 1.02 * (5 + 16 + 16) * V < f < 1.02 * (5 + 16 + 16) * V + 80 * 2**20
        assert req(N, 1, betas=(0.0, 1.0)).footprint() >= (7 + 16 + 32) * V  # Taylor buffers, 2 anchors
        assert req(N, 16).footprint() >= (16 + 48) * V
    # an N=28 request fits one MI355X (288 GB) at B = 1, but not at B = 16
    assert req(28, 1).footprint() < 200e9 < req(28, 16).footprint()


@pytest.mark.parametrize("N", [16, 20, 24, 28])
def test_plan_layout(N):
    """The planner's relabelling is a permutation of sites and bonds that keeps the
    cluster's bond set and needs no more passes than the natural numbering."""
    cl = ftk.honeycomb_cluster(*SUPERCELLS[N])
    rc, P, perm, order = ftk.plan_layout(cl)
    assert sorted(perm) == list(range(N)) and sorted(order) == list(range(cl.n_bonds))
    assert 1 <= P <= ftk.hv_plan(cl)[0]
    n, core, ends = ftk.hv_plan(rc)
    assert n == P and ends[-1] == cl.n_bonds
    old = {(min(perm[i], perm[j]), max(perm[i], perm[j]), g) for i, j, g in cl.bonds}
    assert old == {(min(i, j), max(i, j), g) for i, j, g in rc.bonds}
    oc = cluster.relabel(cluster.honeycomb(*SUPERCELLS[N]), perm, order)
    assert oc.bonds == rc.bonds and np.array_equal(oc.site_xy, rc.site_xy)
    if N == 24:
        assert P == 3 and core == 6


def _gf2_rank(vectors):
    """Rank over GF(2) of bit vectors given as Python ints (Gaussian elimination)."""
    basis = {}
    for v in vectors:
        while v:
            top = v.bit_length() - 1
            if top not in basis:
                basis[top] = v
                break
            v ^= basis[top]
    return len(basis)


@pytest.mark.parametrize("N", [18, 20, 24, 26, 28, 30])
def test_pass_count_against_rank_bound(N):
    """A pass's tile must be closed under the bond flips of its segment and under single
    flips of the c core sites, so it holds a coset of W_p = span(flip masks of the
    segment's bonds, unit vectors of the core) over GF(2), and 4096-element tiles need
    dim W_p <= 12.  Modulo the core the W_p together span GF(2)^N (a connected cluster),
    so sum_p (dim W_p - c) >= N - c and P >= ceil((N - c) / (12 - c)).  The planner's
    plans keep every W_p inside its tile and reach that minimum up to 28 sites; at 30
    sites it needs 5 passes against a bound of 4."""
    rc = ftk.plan_layout(ftk.honeycomb_cluster(*SUPERCELLS[N]))[0]
    P, c, ends = ftk.hv_plan(rc)
    core = [1 << s for s in range(c)]
    starts = [0] + list(ends[:-1])
    dims = []
    for b0, b1 in zip(starts, ends):
        masks = [(1 << i) | (1 << j) for i, j, _ in rc.bonds[b0:b1]]
        dims.append(_gf2_rank(masks + core))
    assert max(dims) <= 12
    assert _gf2_rank([(1 << i) | (1 << j) for i, j, _ in rc.bonds] + core) == N
    assert sum(d - c for d in dims) >= N - c
    bound = -(-(N - c) // (12 - c))
    assert P >= bound
    assert P == (bound if N <= 28 else bound + 1)


def test_two_pass_separator_at_20_sites():
    """At 20 sites (natural labels) the six sites {2, 6, 9, 12, 16, 19} cut the cluster
    into two 7-site halves, so two passes whose tiles are those six sites plus one half
    (13 sites, 8192-element tiles) carry every bond: the two-pass plan that the rank
    bound allows at 20 sites with 13-site tiles and a 6-site core."""
    cl = cluster.honeycomb(*SUPERCELLS[20])
    core = {2, 6, 9, 12, 16, 19}
    adj = {i: set() for i in range(20)}
    for i, j, _ in cl.bonds:
        adj[int(i)].add(int(j))
        adj[int(j)].add(int(i))
    halves, seen = [], set(core)
    for s0 in range(20):
        if s0 in seen:
            continue
        comp, stack = set(), [s0]
        while stack:
            v = stack.pop()
            if v not in comp:
                comp.add(v)
                stack += [w for w in adj[v] if w not in core and w not in comp]
        seen |= comp
        halves.append(comp)
    assert sorted(len(h) for h in halves) == [7, 7]
    tiles = [core | h for h in halves]
    assert all(any({int(i), int(j)} <= t for t in tiles) for i, j, _ in cl.bonds)
    core_units = [1 << s for s in core]
    for t in tiles:
        masks = [(1 << int(i)) | (1 << int(j)) for i, j, _ in cl.bonds if {int(i), int(j)} <= t]
        assert _gf2_rank(masks + core_units) == 13


@pytest.mark.parametrize("tol", [1e-3, 1e-6, 1e-9])
def test_truncation_steps_match_oracle(tol):
    """The library's recurrence and the oracle's Ritz residuals pick the same step."""
    from oracle import filters
    cl = cluster.honeycomb(*SUPERCELLS[8])
    H = hamiltonian.Hamiltonian(cl, -1.0, 0.2)
    v, _ = hamiltonian.normalize(rng.gaussian(5, 1, 8))
    a, b, _, _ = lanczos.lanczos(H, v, 150)
    wr, wi = filters.contour_nodes(0.2, 8)
    for z in (np.linspace(-3, 3, 61) + 0.05j,
              (filters.energy_grid(-3.0, 0.2, 15)[:, None] + (wr + 1j * wi)[None, :]).reshape(-1)):
        k = lanczos.truncation_step(a, b, z, tol)
        assert ftk.truncation_steps(a, b, z, tol) == k


@pytest.mark.parametrize("moments", [True, False])
def test_thermodynamics_matches_oracle(moments):
    """Library thermodynamics against the oracle's on synthetic shell data (two anchors,
    zero shells, binning)."""
    from oracle import thermo
    r = np.random.default_rng(4)
    nv, na, L = 6, 2, 9
    betas = np.array([0.0, 2.0])
    E_m = np.stack([np.linspace(-3, 3, L), np.linspace(-2.5, 1.0, L)])
    log_norm = r.normal(0.0, 3.0, (nv, na))
    n_m = r.uniform(0.0, 1.0, (nv, na, L))
    n_m[0, 0, 3] = 0.0
    h1 = (E_m[None] + r.normal(0, 0.05, (nv, na, L))) * n_m if moments else None
    h2 = (E_m[None] ** 2 + r.uniform(0, 0.1, (nv, na, L))) * n_m if moments else None
    temps = [0.3, 0.5, 1.0, 5.0]
    got = ftk.thermodynamics(betas, E_m, log_norm, n_m, h1, h2, 24, temps, n_bins=3)
    ref = thermo.thermodynamics(betas, E_m, log_norm, n_m, h1, h2, 24, temps, n_bins=3)
    for k in ("E", "C", "S", "lnZ", "E_err", "C_err", "S_err", "lnZ_err"):
        assert np.allclose(got[k], ref[k], rtol=1e-11, atol=1e-12), k


def test_reweight_observable_matches_oracle():
    """Eq. FRW1 for real observables: library against oracle, with an empty shell and bins."""
    r = np.random.default_rng(8)
    nv, na, L, K = 5, 2, 7, 3
    betas = np.array([0.0, 1.5])
    E_m = np.stack([np.linspace(-3, 3, L), np.linspace(-2, 1, L)])
    log_norm = r.normal(0, 2, (nv, na))
    n_m = r.uniform(0, 1, (nv, na, L))
    n_m[1, 1, 2] = 0.0
    O = r.uniform(0, 1, (nv, na, L, K)) * n_m[..., None]
    temps = [0.4, 0.8, 3.0]
    got, gerr = ftk.reweight_observable(betas, E_m, log_norm, n_m, O, temps, n_bins=2)
    ref, rerr = reweight.reweight_observable(betas, E_m, log_norm, n_m, O, temps, n_bins=2)
    assert np.allclose(got, ref, rtol=1e-12, atol=0) and np.allclose(gerr, rerr, rtol=1e-10, atol=1e-14)


def test_reweight_pair_matches_oracle():
    """Eq. FRW1 for operator pairs (complex spectral density and its binned errors):
    library against oracle, with an empty shell."""
    rs = np.random.default_rng(9)
    nv, na, L, npair, nw = 5, 2, 8, 2, 6
    betas = np.array([0.0, 2.0])
    E_m = np.stack([np.linspace(-3, 3, L), np.linspace(-2.5, 1, L)])
    eps = np.array([0.3, 0.2])
    log_norm = rs.normal(size=(nv, na)) * 5
    n_m = rs.uniform(0, 1, size=(nv, na, L))
    n_m[2, 0, 4] = 0.0
    shape = (nv, na, L, npair, nw)
    gab = rs.normal(size=shape) + 1j * rs.normal(size=shape)
    gba = rs.normal(size=shape) + 1j * rs.normal(size=shape)
    temps = [0.3, 0.7, 4.0]
    S, err = ftk.reweight_pair(betas, E_m, eps, log_norm, n_m, gab, gba, temps, n_bins=2)
    So, erro = reweight.reweight_cross(betas, E_m, eps, log_norm, n_m, gab, gba, temps, n_bins=2)
    assert np.abs(S - So).max() <= 1e-12 * np.abs(So).max()
    assert np.abs(err.real - erro.real).max() <= 1e-10 * np.abs(erro.real).max()
    assert np.abs(err.imag - erro.imag).max() <= 1e-10 * np.abs(erro.imag).max()
    # a Hermitian pair (G_BA = G_AB) has a real density equal to the plain reweighting
    Sh, _ = ftk.reweight_pair(betas, E_m, eps, log_norm, n_m, gab, gab, temps, n_bins=2)
    Sp, _, _ = ftk.reweight(betas, E_m, eps, log_norm, n_m, gab, temps, n_bins=2)
    assert np.abs(Sh.imag).max() == 0.0 and np.abs(Sh.real - Sp).max() <= 1e-15 * np.abs(Sp).max()


@pytest.mark.parametrize("N", [8, 24])
def test_momentum_operator_matches_oracle(N):
    """The coefficients of S^alpha_{+Q} as a general spin operator equal the oracle's
    bit for bit, for every allowed momentum."""
    cl = ftk.honeycomb_cluster(*SUPERCELLS[N])
    ocl = cluster.honeycomb(*SUPERCELLS[N])
    for q in ftk.honeycomb_momenta(*SUPERCELLS[N])[:4]:
        for alpha in range(3):
            got = ftk.momentum_operator(cl, alpha, q)
            assert np.array_equal(got, hamiltonian.spin_op_q(ocl, alpha, q[0], q[1]))


@pytest.mark.parametrize("moments", [False, True])
def test_thermo_diagnostics_match_oracle(moments):
    """Energy variance and ln Z(2b)/Z(b)^2 (b and 2b on different anchors too) against the
    oracle on synthetic shell data, with binning."""
    from oracle import thermo
    r = np.random.default_rng(5)
    nv, na, L = 6, 2, 9
    betas = np.array([0.0, 1.0])
    E_m = np.stack([np.linspace(-3, 3, L), np.linspace(-2.5, 1.0, L)])
    log_norm = r.normal(0.0, 2.0, (nv, na))
    n_m = r.uniform(0.0, 1.0, (nv, na, L))
    n_m[1, 1, 0] = 0.0
    h1 = (E_m[None] + r.normal(0, 0.05, (nv, na, L))) * n_m if moments else None
    h2 = (E_m[None] ** 2 + r.uniform(0, 0.1, (nv, na, L))) * n_m if moments else None
    bts = [0.0, 0.3, 0.7, 1.0, 3.0]
    got = ftk.thermo_diagnostics(betas, E_m, log_norm, n_m, h1, h2, 24, bts, n_bins=3)
    ref = thermo.diagnostics(betas, E_m, log_norm, n_m, h1, h2, 24, bts, n_bins=3)
    for k in ("var", "log_typ", "var_err", "log_typ_err"):
        assert np.allclose(got[k], ref[k], rtol=1e-11, atol=1e-12), k


def test_choose_anchors_matches_oracle():
    """The library's anchor ladder picks the oracle's grid points; bad grids are rejected."""
    from oracle import thermo
    grid = np.linspace(0.0, 5.0, 41)
    E = -2.0 * np.tanh(grid)  # a smooth, decreasing energy and a shrinking width
    var = 0.8 / np.cosh(grid) ** 2 + 1e-3
    for r_max, cap in ((0.3, 100), (0.6, 100), (0.6, 3), (5.0, 10)):
        assert ftk.choose_anchors(grid, E, var, r_max, cap) == thermo.choose_anchors(grid, E, var, r_max, cap)
    with pytest.raises(ftk.FTKError, match="EINVAL"):
        ftk.choose_anchors(grid[::-1].copy(), E, var, 0.6, 8)


def test_residual_history_matches_oracle():
    """The CG-step dependence of the largest residual over a filter contour: library
    recurrence against the oracle's Ritz evaluation."""
    from oracle import filters
    cl = cluster.honeycomb(*SUPERCELLS[8])
    H = hamiltonian.Hamiltonian(cl, -1.0, 0.1)
    v, _ = hamiltonian.normalize(rng.gaussian(6, 0, 8))
    a, b, _, _ = lanczos.lanczos(H, v, 80)
    wr, wi = filters.contour_nodes(0.2, 16)
    z = -1.0 + wr + 1j * wi
    got = ftk.residual_history(a, b, z)
    ref = lanczos.residual_history(a, b, z)
    assert np.allclose(got, ref, rtol=1e-8, atol=1e-14)
    assert ftk.truncation_steps(a, b, z, 1e-6) == int(np.argmax(got <= 1e-6)) + 1


def test_asymmetric_lorentzian_fit_matches_oracle():
    """Peak-width fit (Sec. V.F): the library's Levenberg-Marquardt lands on the oracle's
    least-squares minimum for noise-free, noisy and exact-diagonalisation spectra."""
    from oracle import ed, fit
    p_true = np.array([0.30, 0.25, 6.0, 0.22, 1.35])
    w = np.linspace(0.0, 3.0, 601)
    cases = [(w, fit.model(p_true, w), 1.0, 2.0)]
    for seed in (1, 2, 3):
        noise = np.random.default_rng(seed).normal(size=w.size)
        cases.append((w, fit.model(p_true, w) * (1 + 0.03 * noise), 1.0, 2.0))
    cl = cluster.honeycomb(*SUPERCELLS[8])
    omega = np.linspace(-3.0, 3.0, 601)
    _, qx, qy = cluster.allowed_momenta(cl)[0]
    S = np.asarray(ed.ED(cl, -1.0, 0.1).canonical_dsf([0, 1, 2], qx, qy, omega, 0.1, 2.0)).real
    k = int(np.argmax(np.where(omega >= 0.2, S, -np.inf)))
    cases.append((omega, S, omega[k] - 0.5, omega[k] + 0.5))
    for i, (x, y, lo, hi) in enumerate(cases):
        p, cost, ratio = fit.fit_asymmetric_lorentzian(x, y, lo, hi)
        got = ftk.fit_asymmetric_lorentzian(x, y, lo, hi)
        q = np.array([got[k_] for k_ in ("a", "b", "c", "gamma", "eps")])
        assert np.abs(q - p).max() <= 1e-6 * np.abs(p).max(), i
        assert got["cost"] == pytest.approx(cost, rel=1e-9, abs=1e-24), i
        assert got["width_ratio"] == pytest.approx(ratio, rel=1e-6) and got["gamma"] > 0, i
    assert np.abs(q - p_true).max() > 0  # the last case is not the synthetic curve
    got = ftk.fit_asymmetric_lorentzian(w, fit.model(p_true, w), 1.0, 2.0, init=p_true * np.array([-1, -1, 1, -1, 1]))
    assert got["gamma"] == pytest.approx(p_true[3], rel=1e-8) and got["a"] == pytest.approx(p_true[0], rel=1e-8)
    y = fit.model(p_true, w)
    bad = y.copy()
    bad[400] = np.nan
    for args, kw in (((w, y, 1.0, 1.005), {}), ((w, bad, 1.0, 2.0), {}), ((w[::-1].copy(), y[::-1].copy(), 1.0, 2.0), {}),
                     ((w, y, 2.0, 1.0), {}), ((w, y, 1.0, 2.0), {"init": [1, 1, 1, 0, 1]}),
                     ((w, -np.abs(y), 1.0, 2.0), {})):
        with pytest.raises(ftk.FTKError, match="EINVAL"):
            ftk.fit_asymmetric_lorentzian(*args, **kw)


def test_missing_library_is_an_import_error(tmp_path):
    """Without the built library the package has nothing to fall back to: lib() raises
    ImportError (checked on a copy of the package without libftkw.so)."""
    import os
    import shutil
    import sys
    src = os.path.dirname(ftk.LIB_PATH)
    dst = tmp_path / "paper_1802_02854_amd"
    shutil.copytree(src, dst, ignore=shutil.ignore_patterns("*.so", "__pycache__", "csrc"))
    code = ("import paper_1802_02854_amd as f\n"
            "try:\n    f.lib()\nexcept ImportError as e:\n    print('ImportError', e)\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=tmp_path, capture_output=True, text=True, timeout=120,
                         env={**os.environ, "PYTHONPATH": str(tmp_path)})
    assert out.returncode == 0 and out.stdout.startswith("ImportError"), out.stdout + out.stderr


def test_product_does_not_use_the_oracle():
    """The package and its native sources name no oracle module: the oracle is test
    infrastructure, and the product computes everything itself."""
    import os
    pkg = os.path.dirname(ftk.LIB_PATH)
    for root, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(root, f)).read()
                assert not re.search(r"\boracle\b", text), os.path.join(root, f)
