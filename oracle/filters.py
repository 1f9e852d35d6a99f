"""Filter operators and equi-energy shells (Sec. III.B) -- oracle side.

Test infrastructure only (see ``oracle/__init__``).

Eq. (dfilterP): P_{g,r,M} = (1/M) sum_{j=1..M} r e^{i th_j} / (r e^{i th_j} + g - H),
th_j = 2 pi (j - 1/2) / M.  Energy grid E_m = E_b + (2m + 1) eps, m = 0..L-1, and
the filtered state of Eq. (filtered) is phi^m = P_{E_m, eps, M} phi_beta.

In the Krylov basis of phi_beta (lanczos.py), every resolvent applied to phi_beta
is the Galerkin solution ||phi_beta|| V_n (z - T_n)^{-1} e_1, so
    phi^m = V_n c^m,  c^m = (||phi_beta|| / M) sum_j eps e^{i th_j} y_{mj},
    (z_{mj} - T_n) y_{mj} = e_1,  z_{mj} = E_m + eps e^{i th_j}.
Each tridiagonal system is solved by Gaussian elimination without pivoting
(|pivot| >= |Im z| > 0 for even M, so it cannot break down).  This routine, the
node table and the combination below are the arithmetic contract the GPU path
reproduces bit for bit (the downstream Lanczos runs amplify any difference):
complex products (a+ib)(c+id) = (ac - bd) + i(ad + bc), reciprocals
1/(a+ib) = (a/(a a + b b), -b/(a a + b b)), no fused operations.
"""
import math

import numpy as np


def energy_grid(E_b, eps, L):
    """E_m = E_b + (2m+1) eps."""
    return np.array([E_b + (2 * m + 1) * eps for m in range(L)])


def auto_window(alpha, beta, L, margin):
    """Shell window from the spectrum seen by a Lanczos run: (E_b, eps) such that the L
    shells of width 2 eps tile [theta_min - margin, theta_max + margin], with theta the
    extreme Ritz values of T_n (eigenvalues of the dense tridiagonal matrix)."""
    from .lanczos import tridiag
    theta = np.linalg.eigvalsh(tridiag(alpha, beta))
    lo, hi = float(theta[0]), float(theta[-1])
    E_b = lo - margin
    eps = ((hi + margin) - E_b) / (2.0 * L)
    return E_b, eps


def contour_nodes(eps, M):
    """(w_j, th_j): w_j = eps e^{i th_j}, th_j = 2 pi (j - 1/2)/M, j = 1..M."""
    if M < 2 or M % 2:
        raise ValueError("M must be even and >= 2 (odd M puts a node on the real axis)")
    wr = np.zeros(M)
    wi = np.zeros(M)
    for j in range(1, M + 1):
        th = 2.0 * math.pi * (j - 0.5) / M
        wr[j - 1] = eps * math.cos(th)
        wi[j - 1] = eps * math.sin(th)
    return wr, wi


def filter_closed_form(E, Em, eps, M):
    """The discretised filter acting on an eigenvalue E, summed in closed form:
    (1/M) sum_j 1/(1 - x e^{-i th_j}) = 1/(1 + x^M) with x = (E - Em)/eps."""
    x = (np.asarray(E, dtype=np.float64) - Em) / eps
    with np.errstate(over="ignore"):
        return 1.0 / (1.0 + x**M)


def filter_literal(E, Em, eps, M):
    """Eq. (dfilterP) evaluated literally on an eigenvalue E (complex result)."""
    E = np.asarray(E, dtype=np.float64)
    out = np.zeros(E.shape, dtype=np.complex128)
    for j in range(1, M + 1):
        w = eps * np.exp(1j * 2.0 * math.pi * (j - 0.5) / M)
        out += w / (w + Em - E)
    return out / M


def shell_coefficients(alpha, beta, nrm, E_b, eps, L, M):
    """c^m_k for m = 0..L-1, k = 0..n-1 (complex, shape [L, n]) as described above."""
    n = len(alpha)
    Em = energy_grid(E_b, eps, L)
    wr, wi = contour_nodes(eps, M)
    # shifts z_{mj}, arrays of shape [L, M]
    zr = Em[:, None] + wr[None, :]
    zi = np.broadcast_to(wi[None, :], (L, M)).copy()
    # forward elimination; ip[k] = 1/pivot_k, f[k] = forward-substituted e_1
    ipr = np.zeros((n, L, M))
    ipi = np.zeros((n, L, M))
    fr = np.zeros((n, L, M))
    fi = np.zeros((n, L, M))
    pr = zr - alpha[0]
    pi = zi.copy()
    den = pr * pr + pi * pi
    ipr[0] = pr / den
    ipi[0] = -pi / den
    fr[0] = 1.0
    fi[0] = 0.0
    for k in range(1, n):
        b = beta[k - 1]  # beta_k couples k-1 and k
        lr = b * ipr[k - 1]
        li = b * ipi[k - 1]
        pr = (zr - alpha[k]) - b * lr
        pi = zi - b * li
        den = pr * pr + pi * pi
        ipr[k] = pr / den
        ipi[k] = -pi / den
        fr[k] = lr * fr[k - 1] - li * fi[k - 1]
        fi[k] = lr * fi[k - 1] + li * fr[k - 1]
    # back substitution: y_{n-1} = f_{n-1}/p_{n-1}; y_k = (f_k + beta_{k+1} y_{k+1}) / p_k
    yr = np.zeros((n, L, M))
    yi = np.zeros((n, L, M))
    yr[n - 1] = fr[n - 1] * ipr[n - 1] - fi[n - 1] * ipi[n - 1]
    yi[n - 1] = fr[n - 1] * ipi[n - 1] + fi[n - 1] * ipr[n - 1]
    for k in range(n - 2, -1, -1):
        b = beta[k]  # beta_{k+1}
        tr = fr[k] + b * yr[k + 1]
        ti = fi[k] + b * yi[k + 1]
        yr[k] = tr * ipr[k] - ti * ipi[k]
        yi[k] = tr * ipi[k] + ti * ipr[k]
    # contour sum over j in order, then the factor ||phi|| / M
    accr = np.zeros((n, L))
    acci = np.zeros((n, L))
    for j in range(M):
        tr = wr[j] * yr[:, :, j] - wi[j] * yi[:, :, j]
        ti = wr[j] * yi[:, :, j] + wi[j] * yr[:, :, j]
        accr = accr + tr
        acci = acci + ti
    s = nrm / M
    c = np.empty((L, n), dtype=np.complex128)
    c.real = (accr * s).T
    c.imag = (acci * s).T
    return c


def shell_coefficients_per_shell(alpha, beta, nrm, E_b, eps, L, M, k_m):
    """c^m_k [L, max k_m] with shell m taken from T_{k_m} (its own truncation step) and
    zero beyond k_m: row m of shell_coefficients on alpha[:k_m], beta[:k_m]."""
    k_m = np.asarray(k_m, dtype=int)
    c = np.zeros((L, int(k_m.max())), dtype=np.complex128)
    for k in np.unique(k_m):
        rows = np.nonzero(k_m == k)[0]
        ck = shell_coefficients(alpha[:k], beta[:k], nrm, E_b, eps, L, M)
        c[rows, :k] = ck[rows]
    return c


def probability(n_m, nrm, eps):
    """P(E_m) = <phi^m|phi^m> / (2 eps <phi_beta|phi_beta>)  (Sec. III.B)."""
    return np.asarray(n_m) / (2.0 * eps * nrm * nrm)
