"""Random start vectors (Sec. II.A) -- oracle side.

Test infrastructure only (see ``oracle/__init__``).

phi_0 = sum_x c_x |x> with c_x i.i.d. complex Gaussian and then normalised, which
makes {c_x} uniform on the unit sphere of R^{2 N_F}.  The draws use the
counter form of SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) and Box-Muller;
the C implementation is ftk_oracle.c:orc_gaussian.
"""
import numpy as np

from . import _native
from ._native import ptr


def gaussian(seed, sample, N):
    """Un-normalised complex Gaussian draw for (seed, sample), interleaved float64."""
    g = np.empty(2 << N)
    _native.lib().orc_gaussian(seed & 0xFFFFFFFFFFFFFFFF, sample, N, ptr(g))
    return g


def splitmix64(seed, k):
    """The k-th output (k >= 1) of SplitMix64 seeded with seed; the key of sample s is
    output s + 1 of the seed's stream, and element x draws outputs 2x + 1 and 2x + 2 of
    the key's stream."""
    return int(_native.lib().orc_splitmix64(seed & 0xFFFFFFFFFFFFFFFF, k))
