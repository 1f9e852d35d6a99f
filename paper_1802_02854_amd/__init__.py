"""MI355X-native FTKw hot path: finite-temperature spin structure factors of the
Kitaev-Heisenberg honeycomb model from filtered typical pure states and shifted
Krylov solves (Yamaji, Suzuki, Kawamura, arXiv:1802.02854).

The work happens in libftkw.so (HIP for gfx950 plus host-side scalar code,
C-ABI in include/ftkw.h); this package only marshals arguments.
"""
from ._lib import FTKError, LIB_PATH, lib
from .api import (Cluster, Context, GreenSequence, Hamiltonian, PairSpectrum, Request, Server, Spectrum, TypicalStates,
                  choose_anchors, filter_coefficients, fit_asymmetric_lorentzian, honeycomb_cluster,
                  honeycomb_momenta, hv_plan, momentum_operator, named_momentum, plan_layout, random_vector,
                  residual_history, reweight, reweight_observable, reweight_pair, set_tuning, shell_window,
                  taylor_plan, thermo_diagnostics, thermodynamics, truncation_steps)

__all__ = ["FTKError", "LIB_PATH", "lib", "Cluster", "Context", "GreenSequence", "Hamiltonian", "PairSpectrum", "Request", "Server",
           "Spectrum", "TypicalStates", "choose_anchors", "filter_coefficients", "fit_asymmetric_lorentzian",
           "honeycomb_cluster", "honeycomb_momenta", "hv_plan", "momentum_operator", "named_momentum", "plan_layout",
           "random_vector", "residual_history", "reweight", "reweight_observable", "reweight_pair", "set_tuning",
           "shell_window", "taylor_plan", "thermo_diagnostics", "thermodynamics", "truncation_steps"]
