"""Kitaev-Heisenberg Hamiltonian and S^alpha_Q on the bit-string basis -- oracle side.

Test infrastructure only (see ``oracle/__init__``).

H = sum_gamma sum_{<ij> in gamma} [J S_i.S_j + K S_i^gamma S_j^gamma]   (Sec. V.A, Eq. H_ij)
with S = sigma/2 and the basis of Sec. II.A (bit l = 0: spin up on site l).

Per bond, write h_b = sum_a c_a S_i^a S_j^a with c_a = J + K [a == gamma].  In the
S^z basis: the diagonal is +c_z/4 for parallel spins and -c_z/4 otherwise, so the
whole diagonal is D(x) = (J/4) S_all(x) + (K/4) S_z(x) with S_all (S_z) the sum of
s_b = +-1 over all (z) bonds, evaluated as fma(K/4, S_z, (J/4) S_all);
S^x S^x flips both spins with amplitude 1/4; S^y S^y flips both with amplitude
-1/4 for a parallel pair and +1/4 for an antiparallel pair.  Hence the two-spin
flip amplitude is (c_x - c_y)/4 (parallel) or (c_x + c_y)/4 (antiparallel).
All matrix elements are real, so H is real symmetric.
"""
import math

import numpy as np

from . import _native
from ._native import ptr


def bond_coefficients(gammas, K, J):
    """Per-bond flip amplitudes (a_par, a_anti) with c_a = J for a != gamma and
    J + K for a == gamma: a_par = (c_x - c_y)/4, a_anti = (c_x + c_y)/4."""
    nb = len(gammas)
    ap = np.zeros(nb)
    aa = np.zeros(nb)
    for b, g in enumerate(gammas):
        c = [J, J, J]
        c[g] = J + K
        ap[b] = (c[0] - c[1]) / 4.0
        aa[b] = (c[0] + c[1]) / 4.0
    return ap, aa


def bond_norm(K, J, gamma):
    """Largest |eigenvalue| of one bond term: the eigenvalues are
    (c_z + c_x - c_y)/4, (c_z - c_x + c_y)/4, (-c_z + c_x + c_y)/4 (each once,
    triplet-like) and (-c_z - c_x - c_y)/4 (singlet-like)."""
    c = [J, J, J]
    c[gamma] = J + K
    cx, cy, cz = c
    ev = [(cz + cx - cy) / 4, (cz - cx + cy) / 4, (-cz + cx + cy) / 4, (-cz - cx - cy) / 4]
    return max(abs(e) for e in ev)


class Hamiltonian:
    """Matrix-free H on a honeycomb cluster (bond-list order = accumulation order)."""

    def __init__(self, cluster, K, J):
        self.cluster = cluster
        self.K = float(K)
        self.J = float(J)
        self.N = cluster.n_sites
        self.dim = 1 << self.N
        self.bi = np.array([b[0] for b in cluster.bonds], dtype=np.int32)
        self.bj = np.array([b[1] for b in cluster.bonds], dtype=np.int32)
        self.gamma = [b[2] for b in cluster.bonds]
        self.isz = np.array([1 if g == 2 else 0 for g in self.gamma], dtype=np.int32)
        self.jq = self.J / 4.0
        self.kq = self.K / 4.0
        self.ap, self.aa = bond_coefficients(self.gamma, self.K, self.J)
        # ||H|| <= B_H = sum over bonds of the largest |bond eigenvalue|
        bound = 0.0
        for g in self.gamma:
            bound = bound + bond_norm(self.K, self.J, g)
        self.norm_bound = bound

    def _args(self):
        return (self.N, len(self.bi), ptr(self.bi), ptr(self.bj), ptr(self.isz), self.jq, self.kq,
                ptr(self.ap), ptr(self.aa))

    def apply(self, v):
        """w = H v for an interleaved float64 vector of length 2^(N+1)."""
        v = np.ascontiguousarray(v, dtype=np.float64)
        assert v.shape == (2 * self.dim,)
        w = np.empty_like(v)
        _native.lib().orc_hv(*self._args(), ptr(v), ptr(w))
        return w

    def apply_at(self, v, idx):
        """(H v)[x] for x in idx only; returns complex128."""
        v = np.ascontiguousarray(v, dtype=np.float64)
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        out = np.empty(2 * len(idx))
        _native.lib().orc_hv_at(*self._args(), ptr(v), len(idx), ptr(idx), ptr(out))
        return out.view(np.complex128)

    def breakdown_tol(self):
        """Lanczos stops when beta_{k+1} <= 1e-12 * B_H (an invariant subspace)."""
        return 1e-12 * self.norm_bound


def sq_coefficients(cluster, qx, qy):
    """h_l = e^{i Q.R_l} (1/2) N^{-1/2}: the per-site factor of S^alpha_{+Q} (Sec. V).
    The phase argument is qx*rx + qy*ry."""
    N = cluster.n_sites
    s = 0.5 / math.sqrt(N)
    h = np.zeros(2 * N)
    for l in range(N):
        rx, ry = cluster.site_xy[l]
        th = qx * rx + qy * ry
        h[2 * l] = math.cos(th) * s
        h[2 * l + 1] = math.sin(th) * s
    return h


def apply_sq(cluster, alpha, qx, qy, v):
    """chi = S^alpha_{+Q} v with S^alpha_{+Q} = N^{-1/2} sum_l e^{iQ.R_l} S^alpha_l (Sec. V)."""
    h = sq_coefficients(cluster, qx, qy)
    v = np.ascontiguousarray(v, dtype=np.float64)
    w = np.empty_like(v)
    _native.lib().orc_apply_sq(cluster.n_sites, int(alpha), ptr(h), ptr(v), ptr(w))
    return w


def spin_op_q(cluster, alpha, qx, qy):
    """Coefficients c [N, 3] (complex) of S^alpha_{+Q} = N^{-1/2} sum_l e^{iQ.R_l} S^alpha_l
    (Sec. V) as a general linear spin operator (apply_spin_op)."""
    N = cluster.n_sites
    c = np.zeros((N, 3), dtype=np.complex128)
    s = 1.0 / math.sqrt(N)
    for l in range(N):
        rx, ry = cluster.site_xy[l]
        th = qx * rx + qy * ry
        c[l, alpha] = complex(math.cos(th) * s, math.sin(th) * s)
    return c


def apply_spin_op(n_sites, coef, v):
    """chi = A v for a linear spin operator A = sum_l sum_alpha c_{l alpha} S^alpha_l (the
    operators A, B of Eq. GAB_TPS; c complex [N, 3] for alpha = x, y, z).  Each component
    is applied as apply_sq applies S^alpha_{+Q}, with per-site factors h_l = c_{l alpha}/2
    (S = sigma/2), and the three parts are added per element in the order (x + y) + z."""
    coef = np.asarray(coef, dtype=np.complex128)
    assert coef.shape == (n_sites, 3)
    v = np.ascontiguousarray(v, dtype=np.float64)
    parts = []
    for a in range(3):
        h = np.empty(2 * n_sites)
        h[0::2] = 0.5 * coef[:, a].real
        h[1::2] = 0.5 * coef[:, a].imag
        w = np.empty_like(v)
        _native.lib().orc_apply_sq(n_sites, a, ptr(h), ptr(v), ptr(w))
        parts.append(w)
    return (parts[0] + parts[1]) + parts[2]


def dot_re(a, b):
    """Re <a|b>, the double nearest the exact sum."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    assert a.shape == b.shape
    return _native.lib().orc_dot_re(a.shape[0] // 2, ptr(a), ptr(b))


def normalize(v):
    """(v / ||v||, ||v||) with the contract's arithmetic: v * (1/sqrt(<v|v>))."""
    nrm = math.sqrt(dot_re(v, v))
    out = np.array(v, dtype=np.float64, copy=True)
    if nrm > 0.0:
        _native.lib().orc_scale(out.shape[0], ptr(out), 1.0 / nrm)
    return out, nrm
