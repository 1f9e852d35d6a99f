"""CPU oracle for the FTKw hot path (Yamaji, Suzuki, Kawamura, arXiv:1802.02854).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call, link or run anything in
this package.  The product package ``paper_1802_02854_amd`` never imports it,
and the two share no code: the only common module is ``seeded_inputs`` (seeded
random draws, none of the method's arithmetic).

The oracle is plain and slow on purpose.  Vector arithmetic lives in
``ftk_oracle.c`` (plain loops, FP64, explicit fma where the arithmetic contract
puts one); everything else is NumPy in FP64.  Each function cites the passage
of the paper it follows.

Parity status of each part (how it is pinned, tests in ``tests/test_oracle_*``):
  cluster      - 3-regularity, bond directions, no duplicate bonds, momenta.
  hamiltonian  - dense Pauli/Kronecker construction, Tr H, Tr H^2, symmetries.
  spin (S_Q)   - dense Kronecker construction, T=inf sum rule 3/4.
  lanczos      - ED resolvent; exact for n = dim.
  filters      - closed form 1/(1+x^M) of the contour sum; ED f_m(H) phi.
  taylor       - ED exp(-beta H / 2) phi0.
  green        - ED per-sample estimator; SU(2) Lorentzian at K=0; operator pairs
                 against the exact ED resolvent.
  reweight     - identity at beta' = beta; ED canonical S(Q,w,T) within error bars.
  thermo       - ED moments, exact expectation of the estimator, canonical limit,
                 the bounds of ln Z(2 beta)/Z(beta)^2.
  ed           - (the checker) dense spectra, sum rules, SU(2) and Kitaev limits.
  fit          - special cases of the asymmetric Lorentzian; recovery of
                 noise-free parameters; a least-squares minimum on noisy data.
  rng          - moments and the Hams-De Raedt variance of <phi0|O|phi0>.
No part is "parity unpinned".
"""
