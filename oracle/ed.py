"""Exact-diagonalisation checker for small clusters -- oracle side.

Test infrastructure only (see ``oracle/__init__``).

Built independently of hamiltonian.py: H is assembled from Pauli matrices with
Kronecker products (no bond-coefficient table), S^alpha_Q likewise.  Used to pin
the oracle:
  * canonical_dsf: the Lehmann form of Eq. (chiAB) with A = B = S^alpha_{+Q},
    S_c(Q, w) = -(1/pi) Im sum_alpha sum_{nu,mu} e^{-beta E_nu}/Z
                |<mu|S^alpha_Q|nu>|^2 / (w + i eta + E_nu - E_mu);
  * estimator_exact: the per-sample FTKw quantities evaluated in the eigenbasis,
    g_m = sum_mu |sum_nu <mu|S|nu> f_m(E_nu) d_nu|^2 / (w + i eta + E_m - E_mu),
    n_m = sum_nu f_m(E_nu)^2 |d_nu|^2, with d_nu = <nu|phi_beta> and f_m the
    discretised filter acting on an eigenvalue;
  * estimator_mean: the expectation of the ratio-of-sums estimator over uniform
    random phi_0 (E[c_x^* c_y] = delta_xy / N_F, Sec. II.A);
  * the same three for a pair of general linear spin operators A, B (Eq. chiAB):
    canonical_cross, resolvent_pair (one start vector) and estimator_mean_cross.
"""
import math

import numpy as np
import scipy.sparse as sp

SX = np.array([[0.0, 1.0], [1.0, 0.0]])
SY = np.array([[0.0, -1.0j], [1.0j, 0.0]])
SZ = np.array([[1.0, 0.0], [0.0, -1.0]])  # basis (up, down) = bit (0, 1)
PAULI = (SX, SY, SZ)


def site_op(N, l, op):
    """op acting on site l (bit l of the basis index)."""
    return sp.kron(sp.kron(sp.identity(1 << (N - 1 - l), format="csr"), sp.csr_matrix(op)),
                   sp.identity(1 << l, format="csr"), format="csr")


def dense_hamiltonian(cluster, K, J):
    N = cluster.n_sites
    ops = [[site_op(N, l, P) for P in PAULI] for l in range(N)]
    H = sp.csr_matrix((1 << N, 1 << N), dtype=np.complex128)
    for i, j, g in cluster.bonds:
        for a in range(3):
            c = J + (K if a == g else 0.0)
            H = H + (c / 4.0) * (ops[i][a] @ ops[j][a])
    H = H.toarray()
    assert np.abs(H.imag).max() < 1e-14
    return H.real.copy()


def dense_sq(cluster, alpha, qx, qy):
    N = cluster.n_sites
    S = sp.csr_matrix((1 << N, 1 << N), dtype=np.complex128)
    for l in range(N):
        rx, ry = cluster.site_xy[l]
        S = S + np.exp(1j * (qx * rx + qy * ry)) * site_op(N, l, PAULI[alpha] / 2.0)
    return (S / math.sqrt(N)).toarray()


def dense_spin_op(N, coef):
    """A = sum_l sum_alpha c_{l alpha} S^alpha_l from Pauli matrices (coef complex [N, 3])."""
    A = sp.csr_matrix((1 << N, 1 << N), dtype=np.complex128)
    for l in range(N):
        for a in range(3):
            if coef[l, a] != 0:
                A = A + coef[l, a] * site_op(N, l, PAULI[a] / 2.0)
    return A.toarray()


class ED:
    def __init__(self, cluster, K, J):
        self.cluster = cluster
        self.H = dense_hamiltonian(cluster, K, J)
        self.E, self.U = np.linalg.eigh(self.H)

    def sq_eig(self, alpha, qx, qy):
        """<mu|S^alpha_{+Q}|nu> in the eigenbasis."""
        S = dense_sq(self.cluster, alpha, qx, qy)
        return self.U.conj().T @ S @ self.U

    def expm_half(self, beta, v):
        """e^{-beta H/2} v."""
        c = self.U.T @ v
        return self.U @ (np.exp(-0.5 * beta * (self.E - self.E[0])) * c) * math.exp(-0.5 * beta * self.E[0])

    def canonical_dsf(self, alphas, qx, qy, omega, eta, beta):
        E = self.E
        w = np.exp(-beta * (E - E[0]))
        w /= w.sum()
        omega = np.asarray(omega)
        out = np.zeros(len(omega))
        for a in alphas:
            M2 = np.abs(self.sq_eig(a, qx, qy)) ** 2  # [mu, nu]
            wts = (M2 * w[None, :]).ravel()
            dE = (E[None, :] - E[:, None]).ravel()  # E_nu - E_mu
            keep = wts > 1e-300
            wts, dE = wts[keep], dE[keep]
            for k in range(len(omega)):
                out[k] += (wts / (omega[k] + 1j * eta + dE)).sum().imag
        return -out / math.pi

    def estimator_exact(self, Smat_eig, phi_beta, E_m, eps, M, omega, eta):
        """Per-sample (g_m(w), n_m) for every shell, exact in the eigenbasis."""
        from .filters import filter_closed_form
        d = self.U.conj().T @ phi_beta
        L = len(E_m)
        g = np.zeros((L, len(omega)), dtype=np.complex128)
        n = np.zeros(L)
        for m in range(L):
            f = filter_closed_form(self.E, E_m[m], eps, M)
            fd = f * d
            n[m] = float(np.sum(np.abs(fd) ** 2))
            amp2 = np.abs(Smat_eig @ fd) ** 2  # over mu
            z = np.asarray(omega)[:, None] + 1j * eta + E_m[m] - self.E[None, :]
            g[m] = (amp2[None, :] / z).sum(axis=1)
        return g, n

    def estimator_mean(self, Smat_eig_list, beta, E_m, eps, M, omega, eta, beta_t=None):
        """Expectation of the ratio-of-sums estimator reweighted to beta_t (default beta),
        summed over the given S matrices (spin components).  Returns S(w)."""
        from .filters import filter_closed_form
        if beta_t is None:
            beta_t = beta
        E = self.E
        bw = np.exp(-beta * (E - E[0]))
        num = np.zeros(len(omega), dtype=np.complex128)
        den = 0.0
        for m in range(len(E_m)):
            f = filter_closed_form(E, E_m[m], eps, M)
            rw = math.exp((beta - beta_t) * (E_m[m] - E_m[0]))
            wnu = rw * bw * f * f  # [nu]
            den += float(wnu.sum())
            z = np.asarray(omega)[:, None] + 1j * eta + E_m[m] - E[None, :]
            for S in Smat_eig_list:
                amp = (np.abs(S) ** 2 * wnu[None, :]).sum(axis=1)  # over nu -> [mu]
                num += (amp[None, :] / z).sum(axis=1)
        return -(num.imag) / (math.pi * den)

    def thermo_canonical(self, beta):
        """Canonical (E, C, S, ln Z) at inverse temperature beta (k_B = 1)."""
        E = self.E
        w = np.exp(-beta * (E - E[0]))
        z = float(w.sum())
        e1 = float((w * E).sum()) / z
        e2 = float((w * E * E).sum()) / z
        lnZ = math.log(z) - beta * E[0]
        return e1, beta * beta * (e2 - e1 * e1), beta * e1 + lnZ, lnZ

    def thermo_estimator_mean(self, beta_a, E_m, eps, M, beta_t):
        """(E, C, S, ln Z) that the shell estimator (thermo.py, exact h1/h2) converges to
        with many random vectors: numerator and denominator sums replaced by their
        expectations E[<phi0|A|phi0>] = Tr A / N_F, A = e^{-beta_a H} f_m(H)^2 H^p."""
        from .filters import filter_closed_form
        E = self.E
        bw = np.exp(-beta_a * (E - E[0]))
        s0 = s1 = s2 = d0 = 0.0
        for m in range(len(E_m)):
            f2 = filter_closed_form(E, E_m[m], eps, M) ** 2
            rw = math.exp((beta_a - beta_t) * (E_m[m] - E_m[0]))
            s0 += rw * float((bw * f2).sum())
            s1 += rw * float((bw * f2 * E).sum())
            s2 += rw * float((bw * f2 * E * E).sum())
            d0 += float((bw * f2).sum())
        e1, e2 = s1 / s0, s2 / s0
        lnZa = math.log(float(bw.sum())) - beta_a * E[0]
        lnZ = lnZa + math.log(s0 / d0) + (beta_a - beta_t) * E_m[0]
        return e1, beta_t * beta_t * (e2 - e1 * e1), beta_t * e1 + lnZ, lnZ

    def op_eig(self, coef):
        """<mu|A|nu> of a linear spin operator in the eigenbasis."""
        return self.U.conj().T @ dense_spin_op(self.cluster.n_sites, coef) @ self.U

    def resolvent_pair(self, lam, rho, z):
        """<lam|(z - H)^{-1}|rho> for complex vectors lam, rho at every z."""
        a = self.U.T @ lam  # U is real
        b = self.U.T @ rho
        w = np.conj(a) * b
        z = np.asarray(z)
        return (w[None, :] / (z[:, None] - self.E[None, :])).sum(axis=1)

    def canonical_cross(self, Aeig, Beig, omega, eta, beta):
        """S_AB(w) = -(1/(2 pi i)) [G_AB(w + i eta) - G_AB(w - i eta)] of the canonical
        ensemble, G_AB(z) = sum_{nu, mu} p_nu <nu|A^dag|mu><mu|B|nu> / (z + E_nu - E_mu)."""
        E = self.E
        p = np.exp(-beta * (E - E[0]))
        p /= p.sum()
        W = np.conj(Aeig) * Beig * p[None, :]  # [mu, nu]
        dE = E[None, :] - E[:, None]            # E_nu - E_mu
        omega = np.asarray(omega)
        out = np.zeros(len(omega), dtype=np.complex128)
        for k, w in enumerate(omega):
            gp = (W / (w + 1j * eta + dE)).sum()
            gm = (W / (w - 1j * eta + dE)).sum()
            out[k] = -(gp - gm) / (2j * math.pi)
        return out

    def estimator_mean_cross(self, Aeig, Beig, beta, E_m, eps, M, omega, eta, beta_t=None):
        """Expectation of the ratio-of-sums estimator of S_AB (reweight_cross), reweighted
        to beta_t (default beta): numerator and denominator sums replaced by their
        expectations over uniform random phi_0."""
        from .filters import filter_closed_form
        if beta_t is None:
            beta_t = beta
        E = self.E
        bw = np.exp(-beta * (E - E[0]))
        num = np.zeros(len(omega), dtype=np.complex128)
        den = 0.0
        omega = np.asarray(omega)
        for m in range(len(E_m)):
            f = filter_closed_form(E, E_m[m], eps, M)
            rw = math.exp((beta - beta_t) * (E_m[m] - E_m[0]))
            wnu = rw * bw * f * f
            den += float(wnu.sum())
            amp = (np.conj(Aeig) * Beig * wnu[None, :]).sum(axis=1)  # over nu -> [mu]
            zp = omega[:, None] + 1j * eta + E_m[m] - E[None, :]
            zm = omega[:, None] - 1j * eta + E_m[m] - E[None, :]
            num += -((amp[None, :] / zp).sum(axis=1) - (amp[None, :] / zm).sum(axis=1)) / (2j * math.pi)
        return num / den
