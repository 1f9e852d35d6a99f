"""Pins of the oracle's cluster, Hamiltonian and S_Q against independent constructions.

Sec. V.A (KH Hamiltonian), Fig. 2 caption (bond directions), Sec. V (S^alpha_Q).
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import cluster, ed, hamiltonian
from seeded_inputs import SUPERCELLS, real_vector

D = {0: (-0.5, math.sqrt(3) / 2), 1: (-0.5, -math.sqrt(3) / 2), 2: (1.0, 0.0)}


@pytest.mark.parametrize("N", sorted(SUPERCELLS))
def test_cluster_geometry(N):
    cl = cluster.honeycomb(*SUPERCELLS[N])
    assert cl.n_sites == N and cl.n_bonds == 3 * N // 2
    deg = np.zeros(N, int)
    per_type = np.zeros((N, 3), int)
    h = math.sqrt(3) / 2
    a1, a2 = np.array([1.5, -h]), np.array([1.5, h])
    T = [cl.T1[0] * a1 + cl.T1[1] * a2, cl.T2[0] * a1 + cl.T2[1] * a2]
    for i, j, g in cl.bonds:
        deg[i] += 1
        deg[j] += 1
        per_type[i, g] += 1
        per_type[j, g] += 1
        assert i % 2 == 0 and j % 2 == 1  # bonds join the two sublattices
        # B - A equals d_gamma up to a supercell translation
        d = cl.site_xy[j] - cl.site_xy[i] - np.array(D[g])
        coeff = np.linalg.solve(np.array(T).T, d)
        assert np.allclose(coeff, np.round(coeff), atol=1e-9)
    assert (deg == 3).all() and (per_type == 1).all()


def test_cluster_too_small_rejected():
    with pytest.raises(ValueError):
        cluster.honeycomb((1, 0), (0, 1))


@pytest.mark.parametrize("N", [8, 16, 24])
def test_momenta(N):
    cl = cluster.honeycomb(*SUPERCELLS[N])
    ms = cluster.allowed_momenta(cl)
    assert len(ms) == cl.n_cells
    for _, qx, qy in ms:
        assert cluster.is_allowed(cl, qx, qy)
    assert ms[0][1] == 0.0 and ms[0][2] == 0.0
    if N == 24:  # the 24-site hexagonal cluster holds Gamma, M and K
        for name in ("Gamma", "M", "K"):
            assert cluster.is_allowed(cl, *cluster.named_momentum(name))


@pytest.mark.parametrize("N,K,J", [(6, -1.0, 0.1), (8, -1.0, 0.1), (8, 0.7, -0.3), (10, 0.0, 1.0)])
def test_hv_equals_dense_kronecker(N, K, J):
    """T1: matrix-free H v (bond table) against H assembled from Pauli matrices."""
    cl = cluster.honeycomb(*SUPERCELLS[N])
    H = hamiltonian.Hamiltonian(cl, K, J)
    Hd = ed.dense_hamiltonian(cl, K, J)
    v = real_vector(N, 2 << N)
    w = H.apply(v).view(np.complex128)
    wd = Hd @ v.view(np.complex128)
    assert np.abs(w - wd).max() <= 1e-14 * max(1.0, np.abs(wd).max())
    # H is real symmetric, ||H|| <= B_H
    assert np.abs(Hd - Hd.T).max() == 0.0
    assert np.abs(np.linalg.eigvalsh(Hd)).max() <= H.norm_bound + 1e-12


@pytest.mark.parametrize("K,J", [(-1.0, 0.1), (1.0, 0.0), (0.3, 0.8)])
def test_trace_closed_forms(K, J):
    """T2: Tr H = 0 and Tr H^2 / N_F = (3N/2)((J+K)^2 + 2 J^2)/16."""
    N = 8
    cl = cluster.honeycomb(*SUPERCELLS[N])
    H = hamiltonian.Hamiltonian(cl, K, J)
    dim = 1 << N
    tr = 0.0
    tr2 = 0.0
    for x in range(dim):
        e = np.zeros(2 * dim)
        e[2 * x] = 1.0
        w = H.apply(e)
        tr += w[2 * x]
        tr2 += float(w @ w)
    assert abs(tr) < 1e-12
    assert abs(tr2 / dim - (3 * N / 2) * ((J + K) ** 2 + 2 * J**2) / 16) < 1e-12


def _flip_all(N, alpha):
    """prod_l sigma^alpha_l as a dense matrix."""
    P = ed.PAULI[alpha]
    M = np.array([[1.0]])
    for _ in range(N):
        M = np.kron(P, M)
    return M


def test_symmetries():
    """T3: Z2 x Z2 parities always; SU(2) at K = 0; plaquette fluxes at J = 0."""
    N = 8
    cl = cluster.honeycomb(*SUPERCELLS[N])
    Hd = ed.dense_hamiltonian(cl, -1.0, 0.1)
    for a in range(3):
        P = _flip_all(N, a)
        assert np.abs(P @ Hd - Hd @ P).max() < 1e-12
    H0 = ed.dense_hamiltonian(cl, 0.0, 1.0)
    for a in range(3):
        S = sum(ed.site_op(N, l, ed.PAULI[a]) for l in range(N)).toarray()
        assert np.abs(S @ H0 - H0 @ S).max() < 1e-12
    # J = 0: every hexagon operator W_p (on each site of the hexagon the Pauli
    # matrix of the bond that leaves the hexagon) commutes with H.
    for n_sites in (8, 12):
        clk = cluster.honeycomb(*SUPERCELLS[n_sites])
        Hk = ed.dense_hamiltonian(clk, 1.0, 0.0)
        Wlist = _plaquettes(clk)
        assert len(Wlist) == n_sites // 2
        for W in Wlist:
            assert np.abs(W @ Hk - (W.T @ Hk.T).T).max() < 1e-12
        # ... and not with the Heisenberg part
        Hh = ed.dense_hamiltonian(clk, 0.0, 1.0)
        assert max(np.abs(W @ Hh - (W.T @ Hh.T).T).max() for W in Wlist) > 0.1


def _plaquettes(cl):
    """W_p for every hexagon: on each site the Pauli matrix of the bond leaving the hexagon."""
    N = cl.n_sites
    nbr = {l: {} for l in range(N)}
    for i, j, g in cl.bonds:
        nbr[i][g] = j
        nbr[j][g] = i
    out = []
    seen = set()
    # hexagon through A site a: a -x- b1 -y- a2 -z- b2 -x- a3 -y- b3 -z- a
    for a in range(0, N, 2):
        path = [a]
        cur = a
        for g in (0, 1, 2, 0, 1, 2):
            cur = nbr[cur][g]
            path.append(cur)
        if path[-1] != a or len(set(path[:-1])) != 6:
            continue
        key = frozenset(path[:-1])
        if key in seen:
            continue
        seen.add(key)
        W = sp.identity(1 << N, dtype=complex, format="csr")
        ring = path[:-1]
        for k, l in enumerate(ring):
            gin = (0, 1, 2, 0, 1, 2)[k]
            gprev = (0, 1, 2, 0, 1, 2)[k - 1]
            outer = ({0, 1, 2} - {gin, gprev}).pop()
            W = ed.site_op(N, l, ed.PAULI[outer]) @ W
        out.append(W.tocsr())
    assert out
    return out


@pytest.mark.parametrize("alpha", [0, 1, 2])
def test_sq_equals_dense(alpha):
    """S^alpha_{+Q} v against the Kronecker construction, at a non-trivial Q."""
    N = 8
    cl = cluster.honeycomb(*SUPERCELLS[N])
    _, qx, qy = cluster.allowed_momenta(cl)[1]
    v = real_vector(3, 2 << N)
    w = hamiltonian.apply_sq(cl, alpha, qx, qy, v).view(np.complex128)
    wd = ed.dense_sq(cl, alpha, qx, qy) @ v.view(np.complex128)
    assert np.abs(w - wd).max() < 1e-14


def test_dot_is_correctly_rounded():
    """Re<a|b> equals math.fsum of the exact products (rounded once)."""
    from fractions import Fraction
    rng = np.random.default_rng(5)
    for trial in range(20):
        n = 1 << 10
        a = rng.standard_normal(2 * n) * np.exp(rng.uniform(-20, 20, 2 * n))
        b = rng.standard_normal(2 * n)
        exact = sum(Fraction(x) * Fraction(y) for x, y in zip(a, b))
        assert hamiltonian.dot_re(a, b) == float(exact)


def test_relabel_is_a_basis_permutation():
    """A relabelled cluster is the same system: H' = Pi H Pi^T with Pi the bit permutation,
    so the spectrum and S^alpha_Q matrix elements are unchanged."""
    from oracle import ed, hamiltonian
    cl = cluster.honeycomb(*SUPERCELLS[8])
    rng = np.random.default_rng(3)
    perm = rng.permutation(8)
    order = rng.permutation(cl.n_bonds)
    rc = cluster.relabel(cl, perm, order)
    E0 = ed.ED(cl, -1.0, 0.2).E
    E1 = ed.ED(rc, -1.0, 0.2).E
    assert np.abs(E0 - E1).max() < 1e-12
    # Pi: x -> x' with bit perm[l] of x' = bit l of x
    x = np.arange(256)
    xp = np.zeros(256, dtype=np.int64)
    for l in range(8):
        xp |= ((x >> l) & 1) << int(perm[l])
    v = rng.standard_normal(512)
    vc = v.view(np.complex128)
    vp = np.zeros(256, dtype=np.complex128)
    vp[xp] = vc
    H0, H1 = hamiltonian.Hamiltonian(cl, -1.0, 0.2), hamiltonian.Hamiltonian(rc, -1.0, 0.2)
    w0 = H0.apply(v).view(np.complex128)
    w1 = H1.apply(vp.view(np.float64).copy()).view(np.complex128)
    assert np.abs(w1[xp] - w0).max() < 1e-13
    q = cluster.allowed_momenta(cl)[1][1:]
    for a in range(3):
        s0 = hamiltonian.apply_sq(cl, a, *q, v).view(np.complex128)
        s1 = hamiltonian.apply_sq(rc, a, *q, vp.view(np.float64).copy()).view(np.complex128)
        assert np.abs(s1[xp] - s0).max() < 1e-14
    with pytest.raises(ValueError):
        cluster.relabel(cl, [0] * 8, order)
