"""Periodic honeycomb clusters (Sec. V, Fig. 2 caption) -- oracle side.

Test infrastructure only (see ``oracle/__init__``).

Geometry (the figure with the cluster shapes is missing, so this is a reading):
z bonds are horizontal, x and y bonds lie on the -60 and +60 degree lines.  An A
site at R has its three B neighbours at R + d_g with
    d_z = (1, 0),  d_x = (-1/2, sqrt3/2),  d_y = (-1/2, -sqrt3/2).
Bravais vectors a1 = d_z - d_x, a2 = d_z - d_y; the supercell is spanned by
T1 = t11 a1 + t12 a2 and T2 = t21 a1 + t22 a2 and holds |det T| cells.

Canonical numbering: cells are the representatives (c1, c2) with 0 <= c1 < p,
0 <= c2 < q of Z^2 modulo the supercell lattice, where p = gcd(t11, t21) and
q = |det| / p; cell index c = c1 + p c2; site 2c is the A site, 2c + 1 the B
site.  Bonds are listed cell by cell as (A, B, gamma) with gamma order x, y, z;
the bond-list order is also the order in which H v accumulates bond terms.
R_l is the site's own position (the B offset included), as the definition of
S_Q after Eq. (SQomega_TPS) requires.
"""
import math
from dataclasses import dataclass, field

import numpy as np

GAMMA_NAMES = ("x", "y", "z")


def _egcd(a, b):
    """Return (g, x, y) with a x + b y = g = gcd(a, b) >= 0."""
    x0, y0, x1, y1 = 1, 0, 0, 1
    while b != 0:
        k = a // b
        a, b = b, a - k * b
        x0, x1 = x1, x0 - k * x1
        y0, y1 = y1, y0 - k * y1
    if a < 0:
        a, x0, y0 = -a, -x0, -y0
    return a, x0, y0


@dataclass
class Cluster:
    T1: tuple
    T2: tuple
    n_cells: int
    p: int
    q: int
    s: int
    bonds: list = field(default_factory=list)  # (i, j, gamma)
    site_xy: np.ndarray = None  # [N, 2]

    @property
    def n_sites(self):
        return 2 * self.n_cells

    @property
    def n_bonds(self):
        return len(self.bonds)

    def reduce(self, c1, c2):
        k = c1 // self.p
        c1 -= k * self.p
        c2 -= k * self.s
        return c1, c2 % self.q

    def cell_index(self, c1, c2):
        c1, c2 = self.reduce(c1, c2)
        return c1 + self.p * c2


def honeycomb(T1, T2):
    t11, t12 = T1
    t21, t22 = T2
    det = t11 * t22 - t12 * t21
    if det == 0:
        raise ValueError("degenerate supercell")
    n_cells = abs(det)
    p, m, n = _egcd(t11, t21)
    if p == 0:
        raise ValueError("degenerate supercell")
    q = n_cells // p
    s = (m * t12 + n * t22) % q
    cl = Cluster(tuple(T1), tuple(T2), n_cells, p, q, s)
    h = math.sqrt(3.0) / 2.0
    xy = np.zeros((2 * n_cells, 2))
    bonds = []
    for c in range(n_cells):
        c1, c2 = c % p, c // p
        xa = 1.5 * c1 + 1.5 * c2
        ya = h * (c2 - c1)
        xy[2 * c] = (xa, ya)
        xy[2 * c + 1] = (xa + 1.0, ya)
        A = 2 * c
        bonds.append((A, 2 * cl.cell_index(c1 - 1, c2) + 1, 0))  # x: B of cell c - e1
        bonds.append((A, 2 * cl.cell_index(c1, c2 - 1) + 1, 1))  # y: B of cell c - e2
        bonds.append((A, 2 * c + 1, 2))  # z: B of the same cell
    seen = set()
    for i, j, g in bonds:
        key = (min(i, j), max(i, j))
        if key in seen:
            raise ValueError(f"supercell {T1},{T2} too small: duplicate bond {key}")
        seen.add(key)
    cl.bonds = bonds
    cl.site_xy = xy
    return cl


# Reciprocal vectors: b_i . a_j = 2 pi delta_ij, b1 = (2pi/3, -2pi/sqrt3), b2 = (2pi/3, 2pi/sqrt3).
def relabel(cl, site_perm, bond_order):
    """The same cluster with site l renamed site_perm[l] and the bonds listed in the order
    bond_order (a basis permutation: x -> sum_l bit_l(x) 2^site_perm[l])."""
    import dataclasses
    perm = [int(p) for p in site_perm]
    if sorted(perm) != list(range(cl.n_sites)) or sorted(int(b) for b in bond_order) != list(range(cl.n_bonds)):
        raise ValueError("site_perm and bond_order must be permutations")
    bonds = [(perm[cl.bonds[b][0]], perm[cl.bonds[b][1]], cl.bonds[b][2]) for b in bond_order]
    xy = np.empty_like(cl.site_xy)
    xy[perm] = cl.site_xy
    return dataclasses.replace(cl, bonds=bonds, site_xy=xy)


def momentum_xy(f1num, f2num, den):
    """Cartesian Q = (f1 b1 + f2 b2) for integer numerators over a common denominator."""
    tp3 = 2.0 * math.pi / 3.0
    tps = 2.0 * math.pi / math.sqrt(3.0)
    return (tp3 * ((f1num + f2num) / den), tps * ((f2num - f1num) / den))


def allowed_momenta(cl):
    """All Q with e^{i Q.T1} = e^{i Q.T2} = 1, folded into the first Brillouin zone
    (the inner hexagon), in canonical order; returns [(label, qx, qy)]."""
    (t11, t12), (t21, t22) = cl.T1, cl.T2
    det = abs(t11 * t22 - t12 * t21)
    out = []
    for a in range(det):
        for b in range(det):
            if (t11 * a + t12 * b) % det or (t21 * a + t22 * b) % det:
                continue
            best = None
            for i in (0, -1, 1, -2, 2):
                for j in (0, -1, 1, -2, 2):
                    f1, f2 = a - i * det, b - j * det
                    # |f1 b1 + f2 b2|^2 is proportional to f1^2 + f2^2 - f1 f2 (b1, b2 are 120 degrees apart)
                    r2 = f1 * f1 + f2 * f2 - f1 * f2
                    if best is None or r2 < best[0]:
                        best = (r2, f1, f2)
            _, f1, f2 = best
            qx, qy = momentum_xy(f1, f2, det)
            out.append(((f1, f2, det), qx, qy))
    assert len(out) == det
    return out


def named_momentum(name):
    """Gamma, M = (b1 + b2)/2 (mid-edge of the first zone) and K = (2 b1 + b2)/3 (corner)."""
    if name == "Gamma":
        return momentum_xy(0, 0, 1)
    if name == "M":
        return momentum_xy(1, 1, 2)
    if name == "K":
        return momentum_xy(2, 1, 3)
    if name == "M'":
        return momentum_xy(1, 0, 2)
    raise KeyError(name)


def is_allowed(cl, qx, qy, tol=1e-9):
    """e^{i Q.T} = 1 for both supercell vectors."""
    h = math.sqrt(3.0) / 2.0
    a1 = (1.5, -h)
    a2 = (1.5, h)
    for t1, t2 in (cl.T1, cl.T2):
        Tx = t1 * a1[0] + t2 * a2[0]
        Ty = t1 * a1[1] + t2 * a2[1]
        ph = (qx * Tx + qy * Ty) / (2 * math.pi)
        if abs(ph - round(ph)) > tol:
            return False
    return True
