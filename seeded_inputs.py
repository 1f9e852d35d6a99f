"""Seeded synthetic inputs shared by the tests, smoke() and bench.py.

This module holds none of the method's arithmetic: it only draws random numbers
and names workload sizes.  Both the GPU path and the CPU oracle receive the same
draws from here, so a parity run does not depend on either side's random
generator or math library.

Workloads (the paper's clusters, couplings, temperatures and discretisation,
Sec. V and Table I; no dataset is involved):
  plain-N8   N=8  (2x2 supercell), K=-1, J=0.1, 4 vectors, 64 Krylov steps,
             200 frequencies in [-3, 3], eta 0.05, Q = Gamma, 20 T' in [0.01, 1]
  plain-N16  N=16, K=-1, J=0.1 (plain-N16-J0: the pure Kitaev point J=0), 32 vectors,
             300 steps, 1000 frequencies, eta 0.02, 6 momenta, 50 T' in [0.1, 10]
  plain-N24  N=24 (hexagonal 24-site supercell), K=-1, J=0.1, 8 vectors, 500 steps,
             2000 frequencies in [-4, 4], eta 0.01, Q in {Gamma, M, K}, 100 T'
  serve      a stream of independent requests: N drawn from a size mix, K=-1,
             J ~ U[0, 0.3], n_vectors ~ U{lo..hi}, anchor T = inf, L=16 shells
             on the automatic window (margin 0.1), M=16, 300 steps, 1000
             frequencies in [-4, 4], eta 0.02, Q = Gamma, 20 T' in [1, 10];
             Poisson arrivals
"""
import numpy as np

BASE_SEED = 180202854

# default supercells (t11, t12), (t21, t22) in the (a1, a2) basis, per site count
SUPERCELLS = {
    6: ((1, 1), (-1, 2)),
    8: ((2, 0), (0, 2)),
    10: ((2, 1), (-1, 2)),
    12: ((2, 1), (-2, 2)),
    14: ((2, 1), (-1, 3)),
    16: ((2, 2), (-2, 2)),
    18: ((3, 0), (0, 3)),
    20: ((2, 2), (-3, 2)),
    24: ((2, 2), (-2, 4)),
    26: ((3, 1), (-1, 4)),
    28: ((3, 1), (-2, 4)),
    # 30 sites admit no hexagonal supercell; among the |det| = 15 lattices this one has the
    # longest shortest periodic image (6.245 nearest-neighbour distances); Gamma only
    30: ((3, 3), (-4, 1)),
}


def gaussian_vector(seed, sample, n_sites):
    """Un-normalised complex Gaussian amplitudes c_x (interleaved float64, length 2^(N+1))."""
    rng = np.random.default_rng([int(seed) & 0xFFFFFFFF, int(seed) >> 32, int(sample)])
    return rng.standard_normal(2 << n_sites)


def real_vector(seed, n, scale=1.0):
    """Generic seeded float64 test vector."""
    rng = np.random.default_rng([int(seed) & 0xFFFFFFFF, 7])
    return scale * rng.standard_normal(n)


def omega_grid(lo, hi, n):
    """Inclusive linear frequency grid."""
    return np.linspace(lo, hi, n)


def temperature_grid(lo, hi, n):
    """Inclusive geometric temperature grid."""
    return np.geomspace(lo, hi, n)


# Table I (24-site rows) and the configurations built on it.
def eps_table1_24(T):
    """Contour radius of Table I for the 24-site cluster at temperature T (inf allowed)."""
    if T == 0.2:
        return 14.0 * np.log(10.0) * 0.2 / 128.0 / 2.0
    if T == 0.1:
        return 1.5625e-2
    return 3.90625e-2


WORKLOADS = {
    "plain-N8": dict(N=8, K=-1.0, J=0.1, n_vectors=4, temps_anchor=(1.0, 0.1, 0.01), E_b=-3.0,
                     L=64, eps=3.0 / 64.0, M=16, n_filter=64, n_green=64, omega=(-3.0, 3.0, 200),
                     eta=0.05, q=("Gamma",), temps=(0.01, 1.0, 20)),
    "plain-N16": dict(N=16, K=-1.0, J=0.1, n_vectors=32, temps_anchor=(np.inf, 1.0, 0.5, 0.2),
                      E_b=-4.0, L=200, eps=0.02, M=16, n_filter=300, n_green=300,
                      omega=(-4.0, 4.0, 1000), eta=0.02, q=6, temps=(0.1, 10.0, 50)),
    "plain-N16-J0": dict(N=16, K=-1.0, J=0.0, n_vectors=32, temps_anchor=(np.inf, 1.0, 0.5, 0.2),
                         E_b=-4.0, L=200, eps=0.02, M=16, n_filter=300, n_green=300,
                         omega=(-4.0, 4.0, 1000), eta=0.02, q=6, temps=(0.1, 10.0, 50)),
    "plain-N24": dict(N=24, K=-1.0, J=0.1, n_vectors=8, temps_anchor=(np.inf, 1.0, 0.5, 0.2),
                      E_b=-5.0, L=128, eps="table1", M=16, n_filter=500, n_green=500,
                      omega=(-4.0, 4.0, 2000), eta=0.01, q=("Gamma", "M", "K"),
                      temps=(0.1, 10.0, 100)),

    "serve": dict(sizes=(16, 20, 24, 26, 28), weights=(0.4, 0.3, 0.2, 0.07, 0.03), K=-1.0, J=(0.0, 0.3),
                  n_vectors=(8, 32), temps_anchor=(np.inf,), L=16, margin=0.1, M=16, n_filter=300,
                  n_green=300, omega=(-4.0, 4.0, 1000), eta=0.02, q=("Gamma",), temps=(1.0, 10.0, 20)),
}


def serve_stream(seed, n, sizes, weights, J_range, nv_range):
    """n request draws (N, J, n_vectors, seed) for the serving workload."""
    rng = np.random.default_rng([int(seed) & 0xFFFFFFFF, 5])
    p = np.asarray(weights, dtype=np.float64)
    Ns = rng.choice(np.asarray(sizes), size=n, p=p / p.sum())
    Js = rng.uniform(J_range[0], J_range[1], size=n)
    nvs = rng.integers(nv_range[0], nv_range[1] + 1, size=n)
    return [dict(N=int(Ns[i]), J=float(Js[i]), n_vectors=int(nvs[i]), seed=int(seed) + 1000 * i)
            for i in range(n)]


def poisson_arrivals(seed, rate, n):
    """Arrival times (s) of a Poisson process of the given rate."""
    rng = np.random.default_rng([int(seed) & 0xFFFFFFFF, 6])
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
